// Fused red-black SOR sweep on the cube (k = 1): one launch updates the red
// and then the black volume-interior nodes of every macro tetrahedron, so u
// and b are read once and u written once per sweep instead of twice.
//
// A black node's stencil reads red neighbours in its own plane k and in the
// planes k - 1 and k + 1 (index offsets (0, -1, +1) and (0, +1, -1)), and a
// red node's stencil reads only black values that the sweep has not changed
// yet.  A workgroup therefore marches through the planes of a tile (i0 ..
// i0 + 63, rows j0 .. j0 + TJ - 1, planes k0 .. k0 + TK - 1): at plane p it
// computes the red nodes of plane p (from old black values) and then the
// black nodes of plane p - 1 (from the new red values of planes p - 2, p - 1
// and p).  The red values of one node, one row and one plane beyond the tile
// are recomputed by each workgroup that needs them, which is race free
// because the sweep reads the old iterate from one buffer and writes the new
// one to another (the two alternate within a pair of sweeps).  The moving
// window of old black planes (4) and new red planes (3) is kept in LDS, and
// the global loads of the next plane are issued before the current plane is
// computed, so their latency hides behind the LDS work.
//
// Interface masters (faces, edges, vertices) are updated by two small
// launches around this one: the red masters first (their ghost copies in
// the destination buffer are read here as the new red boundary values),
// the black masters after (they read the new red values).
//
// Slot of closure node (i, j, k) of colour c = (i + k) & 1 (colour-split
// layout, plane k, row j, i):
//   (c ? black0 : 0) + ps[c][k] + F(X) - F(X - j) + (i >> 1),
//   X = m + 2 - k - ((c + k) & 1),  F(n) = floor(n^2 / 4),
// where ps[c][k] is the first slot of plane k's colour-c nodes; F(X) - F(X - j)
// counts the colour-c nodes of the rows before j in plane k (a row of n nodes
// holds floor((n + 1 - i0) / 2) of them, i0 = (c + k) & 1).
#include <hip/hip_runtime.h>

#include "kernels.hpp"

// dynamic LDS of k_sweep_fused (size from fused_lds_bytes)
extern __shared__ unsigned char fused_lds[];

namespace hhgr {

namespace {

__device__ __forceinline__ unsigned fused_xcd_remap(unsigned f, unsigned total) {
    const unsigned per = total >> 3, rem = total & 7u, x = f & 7u, loc = f >> 3;
    return x < rem ? x * (per + 1) + loc : rem * (per + 1) + (x - rem) * per + loc;
}

// i values per tile (a host build for checking the tile seams may set a
// smaller even value)
#ifndef HHGR_FUSED_TI
#define HHGR_FUSED_TI 64
#endif
// workgroup size and elements per thread and plane (their product bounds the
// LDS rows of a tile: (TJ + 4) (Ti / 2 + 4) <= E BS, checked on the host)
#ifndef HHGR_FUSED_BS
#define HHGR_FUSED_BS 384
#endif
#ifndef HHGR_FUSED_E
#define HHGR_FUSED_E 3
#endif
constexpr int kFusedBS = HHGR_FUSED_BS;
constexpr int kFusedTi = HHGR_FUSED_TI;
constexpr int kFusedWt = kFusedTi / 2 + 4;    // LDS row: slots of one colour, with the halo
constexpr int kFusedE = HHGR_FUSED_E;

// SOR update of one node with the 7-point stencil of k = 1 (diagonal 6h,
// off-diagonal -h), the same expression as the colour-pass kernels
template <typename T>
__device__ __forceinline__ T sor7(T uo, T acc, T bb, T h, T om_d, T &rr) {
    rr = bb - h * (T(6) * uo - acc);
    return uo + om_d * rr;
}

// one tile's work: rows j0 .. j0 + TJ - 1, i0 .. i0 + Ti - 1 of black planes
// k0 .. k1 - 1 (and the red planes k0 - 1 .. k1 around them).  LDS holds the
// old black values of 4 planes (rows j0 - 2 .. j0 + TJ + 1) and the new red
// values of 3 planes (rows j0 - 1 .. j0 + TJ), each row the slots t of one
// colour from tw0 = i0 / 2 - 1 on (node i of colour c in plane k: t = i >> 1).
// The loads of plane p + 1 are issued before plane p is computed.
template <typename T, bool ZERO, bool RES>
__global__ void __launch_bounds__(kFusedBS) k_sweep_fused(FusedGeom g, const T *__restrict__ us, T *__restrict__ ud,
                                                          const T *__restrict__ b, T h, T om_d, T omega,
                                                          T *__restrict__ rout) {
    const int TJ = g.TJ, m = g.m, Wt = kFusedWt;
    const int LB = (TJ + 4) * Wt, LR = (TJ + 2) * Wt, LC = TJ * Wt;
    T *lb = reinterpret_cast<T *>(fused_lds);
    T *lr = lb + 4 * LB;
    // the plane starts in LDS: global loads of them would be repeated after
    // every store of the sweep (the compiler cannot rule out aliasing)
    int *ps = reinterpret_cast<int *>(lr + 3 * LR);
    for (int q = (int)threadIdx.x; q < 2 * (m + 2); q += kFusedBS) ps[q] = g.ps[q];
    const unsigned blk = g.remap ? fused_xcd_remap(blockIdx.x, gridDim.x) : blockIdx.x;
    const int tet = (int)(blk / (unsigned)g.ntiles), tile = (int)(blk % (unsigned)g.ntiles);
    const int4 tl = g.tiles[tile];
    const int i0 = tl.x, j0 = tl.y, k0 = tl.z;
    const int k1 = min(k0 + g.TK, m - 2);  // black planes k0 .. k1 - 1
    const int tw0 = (i0 >> 1) - 1;
    const long long vec = g.vd[tet].vec;
    const T *S = us + vec;
    T *D = ud + vec;
    const T *B = b + vec;
    T *R = RES ? rout + vec : nullptr;
    const int b0 = (int)g.black0;
    const int tid = (int)threadIdx.x;
    __syncthreads();

    // closure slot of node (i, j, k) of colour c (red without, black with b0)
    auto slot = [&](int c, int i, int j, int k) -> int {
        const int X = m + 2 - k - ((c + k) & 1);
        return (c ? b0 : 0) + ps[c * (m + 2) + k] + ((X * X) >> 2) - (((X - j) * (X - j)) >> 2) + (i >> 1);
    };
    auto in_closure = [&](int i, int j, int k) { return i >= 0 && j >= 0 && k >= 0 && i + j + k <= m; };
    auto interior = [&](int i, int j, int k) { return i >= 1 && j >= 1 && k >= 1 && i + j + k <= m - 1; };
    auto lbs = [&](int q, int jr, int i) -> T { return lb[(q & 3) * LB + (jr - (j0 - 2)) * Wt + ((i >> 1) - tw0)]; };
    auto lrs = [&](int q, int jr, int i) -> T { return lr[(q % 3) * LR + (jr - (j0 - 1)) * Wt + ((i >> 1) - tw0)]; };

    // black plane q, rows j0 - 2 .. j0 + TJ + 1: old values (zero outside the closure)
    auto load_black = [&](int q, T (&v)[kFusedE]) {
#pragma unroll
        for (int a = 0; a < kFusedE; a++) {
            const int e = tid + a * kFusedBS;
            v[a] = T(0);
            if (ZERO || e >= LB) continue;
            const int jr = j0 - 2 + e / Wt, i = 2 * (tw0 + e % Wt) + ((q + 1) & 1);
            if (q >= 0 && in_closure(i, jr, q)) v[a] = S[slot(1, i, jr, q)];
        }
    };
    auto store_black = [&](int q, const T (&v)[kFusedE]) {
#pragma unroll
        for (int a = 0; a < kFusedE; a++) {
            const int e = tid + a * kFusedBS;
            if (e < LB) lb[(q & 3) * LB + e] = v[a];
        }
    };
    // red plane p, rows j0 - 1 .. j0 + TJ, i0 - 1 <= i <= i0 + Ti: old value and
    // b of interior nodes, the new value of boundary nodes (from ud)
    auto load_red = [&](int p, T (&vu)[kFusedE], T (&vb)[kFusedE]) {
#pragma unroll
        for (int a = 0; a < kFusedE; a++) {
            const int e = tid + a * kFusedBS;
            vu[a] = T(0);
            vb[a] = T(0);
            if (e >= LR) continue;
            const int j = j0 - 1 + e / Wt, i = 2 * (tw0 + e % Wt) + (p & 1);
            if (i < i0 - 1 || i > i0 + kFusedTi || !in_closure(i, j, p)) continue;
            const int sl = slot(0, i, j, p);
            if (interior(i, j, p)) {
                if (!ZERO) vu[a] = S[sl];
                vb[a] = B[sl];
            } else {
                vu[a] = D[sl];
            }
        }
    };
    // b of the black nodes of plane k in the tile
    auto load_bb = [&](int k, T (&v)[kFusedE]) {
#pragma unroll
        for (int a = 0; a < kFusedE; a++) {
            const int e = tid + a * kFusedBS;
            v[a] = T(0);
            if (k < k0 || e >= LC) continue;
            const int j = j0 + e / Wt, i = 2 * (tw0 + e % Wt) + ((k + 1) & 1);
            if (i >= i0 && i < i0 + kFusedTi && interior(i, j, k)) v[a] = B[slot(1, i, j, k)];
        }
    };
    auto prefetch = [&](int p, T (&vb)[kFusedE], T (&vu)[kFusedE], T (&vr)[kFusedE], T (&vc)[kFusedE]) {
        load_black(p + 1, vb);
        load_red(p, vu, vr);
        load_bb(p - 1, vc);
    };
    // one plane step: red nodes of plane p, then black nodes of plane p - 1
    auto step = [&](int p, const T (&vb)[kFusedE], const T (&vu)[kFusedE], const T (&vr)[kFusedE],
                    const T (&vc)[kFusedE], T (&nb)[kFusedE], T (&nu)[kFusedE], T (&nr)[kFusedE],
                    T (&nc)[kFusedE]) {
        if (!ZERO) store_black(p + 1, vb);
        __syncthreads();
        if (p + 1 <= k1) prefetch(p + 1, nb, nu, nr, nc);
        // red nodes of plane p
#pragma unroll
        for (int a = 0; a < kFusedE; a++) {
            const int e = tid + a * kFusedBS;
            if (e >= LR) continue;
            const int j = j0 - 1 + e / Wt, i = 2 * (tw0 + e % Wt) + (p & 1);
            if (i < i0 - 1 || i > i0 + kFusedTi || !in_closure(i, j, p)) continue;
            T nv = vu[a];
            if (interior(i, j, p)) {
                T acc = T(0);
                if (!ZERO) {
                    const T ap = lbs(p, j, i + 1), am = lbs(p, j, i - 1);
                    const T bp = lbs(p, j + 1, i - 1), bm = lbs(p, j - 1, i + 1);
                    const T cp = lbs(p + 1, j - 1, i), cm = lbs(p - 1, j + 1, i);
                    acc = ((ap + am) + (bp + bm)) + (cp + cm);
                }
                T rr;
                nv = sor7<T>(vu[a], acc, vr[a], h, om_d, rr);
                if (p >= k0 && p < k1 && j >= j0 && j < j0 + TJ && i >= i0 && i < i0 + kFusedTi)
                    D[slot(0, i, j, p)] = nv;
            }
            lr[(p % 3) * LR + e] = nv;
        }
        __syncthreads();
        // black nodes of plane p - 1
        const int k = p - 1;
        if (k >= k0) {
#pragma unroll
            for (int a = 0; a < kFusedE; a++) {
                const int e = tid + a * kFusedBS;
                if (e >= LC) continue;
                const int j = j0 + e / Wt, i = 2 * (tw0 + e % Wt) + ((k + 1) & 1);
                if (i < i0 || i >= i0 + kFusedTi || !interior(i, j, k)) continue;
                const T uo = ZERO ? T(0) : lbs(k, j, i);
                const T ap = lrs(k, j, i + 1), am = lrs(k, j, i - 1);
                const T bp = lrs(k, j + 1, i - 1), bm = lrs(k, j - 1, i + 1);
                const T cp = lrs(k + 1, j - 1, i), cm = lrs(k - 1, j + 1, i);
                const T acc = ((ap + am) + (bp + bm)) + (cp + cm);
                T rr;
                const T nv = sor7<T>(uo, acc, vc[a], h, om_d, rr);
                const int sl = slot(1, i, j, k);
                D[sl] = nv;
                if (RES) R[sl] = (T(1) - omega) * rr;
            }
        }
    };

    T b0v[kFusedE], u0v[kFusedE], r0v[kFusedE], c0v[kFusedE];
    T b1v[kFusedE], u1v[kFusedE], r1v[kFusedE], c1v[kFusedE];
    if (!ZERO) {
        load_black(k0 - 2, b0v);
        store_black(k0 - 2, b0v);
        load_black(k0 - 1, b0v);
        store_black(k0 - 1, b0v);
    }
    prefetch(k0 - 1, b0v, u0v, r0v, c0v);
    for (int p = k0 - 1; p <= k1; p += 2) {
        step(p, b0v, u0v, r0v, c0v, b1v, u1v, r1v, c1v);
        if (p + 1 <= k1) step(p + 1, b1v, u1v, r1v, c1v, b0v, u0v, r0v, c0v);
    }
}

// SOR update of the interface masters [i0, i1) of one colour: own value
// from us (zero with OWN0), the 6 axis neighbours from un (zero with NB0),
// new value to ud at the master and at its ghost copies; RES also writes the
// residual after the update, (1 - omega) r, to rout.  The same expression as
// the interface part of the colour-pass kernels.
template <typename T, bool OWN0, bool NB0, bool RES>
__global__ void __launch_bounds__(256) k_ifc_sor(IfcGeom ig, const T *__restrict__ us, const T *__restrict__ un,
                                                 T *__restrict__ ud, const T *__restrict__ b, T h, T omega,
                                                 T *__restrict__ rout) {
    const int t = ig.i0 + (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (t >= ig.i1) return;
    const long long sl = ig.base + t;
    const T uo = OWN0 ? T(0) : us[sl];
    T acc = T(0);
    const T diag = T(6) * h;
    if (!NB0) {
#pragma unroll
        for (int e = 0; e < 6; e++) acc += un[ig.nbr[(long long)e * ig.stride + t]];
        acc *= h;
    }
    const T rr = b[sl] - (diag * uo - acc);
    const T nv = uo + omega * rr / diag;
    ud[sl] = nv;
    for (int q = ig.gptr[t]; q < ig.gptr[t + 1]; q++) ud[ig.gidx[q]] = nv;
    if (RES) rout[sl] = (T(1) - omega) * rr;
}

}  // namespace

size_t fused_lds_bytes(const FusedGeom &g, size_t word) {
    return (size_t)(4 * (g.TJ + 4) + 3 * (g.TJ + 2)) * (size_t)kFusedWt * word + 2 * (size_t)(g.m + 2) * sizeof(int);
}

int fused_tile_i() { return kFusedTi; }

bool fused_shape_ok(const FusedGeom &g) {
    return g.TJ >= 1 && g.TK >= 1 && (g.TJ + 4) * kFusedWt <= kFusedE * kFusedBS && g.m >= 8;
}

template <typename T>
void launch_ifc_sor(hipStream_t s, const IfcGeom &ig, const T *us, const T *un, T *ud, const T *b, double h,
                    double omega, bool own0, bool nb0, T *rout) {
    if (ig.i1 <= ig.i0) return;
    const T th = (T)h, to = (T)omega;
    const unsigned nb = (unsigned)((ig.i1 - ig.i0 + 255) / 256);
#define HHGR_IFC(O0, N0, RS)                                                                                 \
    hipLaunchKernelGGL((k_ifc_sor<T, O0, N0, RS>), dim3(nb), dim3(256), 0, s, ig, us, un, ud, b, th, to, rout)
    if (own0 && nb0) {
        if (rout) HHGR_IFC(true, true, true);
        else HHGR_IFC(true, true, false);
    } else if (own0) {
        if (rout) HHGR_IFC(true, false, true);
        else HHGR_IFC(true, false, false);
    } else {
        if (rout) HHGR_IFC(false, false, true);
        else HHGR_IFC(false, false, false);
    }
#undef HHGR_IFC
}

template <typename T>
void launch_sweep_fused_vol(hipStream_t s, const FusedGeom &g, const T *us, T *ud, const T *b, double h, double omega,
                            bool zero, T *rout) {
    const T th = (T)h, to = (T)omega, tod = (T)(omega / (6.0 * h));
    const unsigned grid = (unsigned)(g.nvol * g.ntiles);
    if (grid == 0) return;
    const size_t lds = fused_lds_bytes(g, sizeof(T));
#define HHGR_FUSED(Z, RS)                                                                                     \
    hipLaunchKernelGGL((k_sweep_fused<T, Z, RS>), dim3(grid), dim3(kFusedBS), lds, s, g, us, ud, b, th, tod, to, rout)
    if (zero) {
        if (rout) HHGR_FUSED(true, true);
        else HHGR_FUSED(true, false);
    } else {
        if (rout) HHGR_FUSED(false, true);
        else HHGR_FUSED(false, false);
    }
#undef HHGR_FUSED
}

template void launch_ifc_sor<double>(hipStream_t, const IfcGeom &, const double *, const double *, double *,
                                     const double *, double, double, bool, bool, double *);
template void launch_ifc_sor<float>(hipStream_t, const IfcGeom &, const float *, const float *, float *,
                                    const float *, double, double, bool, bool, float *);
template void launch_sweep_fused_vol<double>(hipStream_t, const FusedGeom &, const double *, double *, const double *,
                                             double, double, bool, double *);
template void launch_sweep_fused_vol<float>(hipStream_t, const FusedGeom &, const float *, float *, const float *,
                                            double, double, bool, float *);

}  // namespace hhgr
