// HIP kernels (gfx950) of the HHG multigrid engine.
//
// Volume containers are processed as structured arrays.  A closure stores its
// red nodes first and its black nodes after them (colour-split layout, plane
// by plane, row by row), so the nodes of one colour are contiguous: a colour
// pass streams whole cache lines of its own colour of u and b and of the
// other colour of u.  A launch walks a packed (i,j,k) node list that is the
// same for every tetrahedron; per-row tables give the slot of a node and of
// its neighbours, so consecutive threads touch consecutive slots.  Interface
// (face, edge, vertex) nodes are few and are handled through precomputed slot
// tables by the first workgroups of the same launch.  Block ids of the volume
// part are remapped so that each of the 8 XCDs walks a contiguous run of
// volumes, which keeps the neighbouring planes of a block in that XCD's L2.
//
// Operator (Sec. 2.1, eq. (2)): P1 stiffness on the Kuhn meshes couples each
// node to its 6 grid-axis neighbours only.  k = 1: diagonal 6h, off-diagonal
// -h.  Per-element k: edge (x, x+e) has weight (h/6) * (sum of k over the 6
// tetrahedra having that edge on their axis path), off-diagonal = -weight,
// diagonal = sum of the 6 incident weights.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace hhgr {

namespace {

__device__ __forceinline__ int row_of(int M, int j, int k) { return k * M - ((k * (k - 1)) >> 1) + j; }

// slot (within its closure) of node (i,j,k) from the row table of its level
__device__ __forceinline__ int lslot(const int2 *__restrict__ rowC, int M, int i, int j, int k) {
    const int2 r = rowC[row_of(M, j, k)];
    return (((i + k) & 1) ? r.y : r.x) + (i >> 1);
}

// Workgroups are dispatched to the 8 XCDs round-robin; map so that each XCD
// receives a contiguous range of logical block ids.
__device__ __forceinline__ unsigned xcd_remap(unsigned f, unsigned total) {
    const unsigned per = total >> 3, rem = total & 7u, x = f & 7u, loc = f >> 3;
    return x < rem ? x * (per + 1) + loc : rem * (per + 1) + (x - rem) * per + loc;
}
__device__ __forceinline__ unsigned block_order(unsigned f, unsigned total, int remap) {
    return remap ? xcd_remap(f, total) : f;
}

// thread -> node of a volume container
struct LNode {
    int v, i, j, k, r;
};

template <int CPB>
__device__ __forceinline__ unsigned list_blocks_per_vol(const VolGeom &g) {
    const unsigned per = (unsigned)(g.bs * CPB);
    return ((unsigned)g.nlist + per - 1) / per;
}

template <int CPB>
__device__ __forceinline__ bool list_node(const VolGeom &g, unsigned blk, unsigned per_vol, int q, LNode &n) {
    n.v = (int)(blk / per_vol);
    const int e = (int)(blk % per_vol) * g.bs * CPB + q * g.bs + (int)threadIdx.x;
    if (e >= g.nlist) return false;
    const unsigned w = g.list[e];
    n.i = (int)(w & 1023u);
    n.j = (int)((w >> 10) & 1023u);
    n.k = (int)(w >> 20);
    n.r = row_of(g.M, n.j, n.k);
    return true;
}

// closure slots of an interior node and of its 6 axis neighbours
// (local directions a, b, c; see topology.hpp for the index offsets)
struct Nb7 {
    int c0, ap, am, bp, bm, cp, cm;
};
__device__ __forceinline__ Nb7 nb7(const VolGeom &g, const LNode &n) {
    const int c = (n.i + n.k) & 1;
    const int4 *e = g.rowN + 2 * ((long long)c * g.nrows + n.r);
    const int4 A = e[0], B = e[1];
    const int t = n.i >> 1;
    Nb7 s;
    s.c0 = A.x + t;
    s.ap = A.y + t;
    s.am = A.y + t - 1;
    s.bp = A.z + t;
    s.bm = A.w + t;
    s.cp = B.x + t;
    s.cm = B.y + t;
    return s;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// sum over a wavefront with DPP moves instead of LDS permutes: prefix sums
// within each 16-lane row (shifts 1, 2, 4, 8), then the row totals carried
// into rows 1 and 3 (lane 15 broadcast) and rows 2 and 3 (lane 31
// broadcast); lane 63 ends with the total, which is returned to every lane.
// Out-of-row sources and masked rows contribute +0.  Fixed order.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_move(double v) {
    const unsigned long long x = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)x, CTRL, ROW_MASK, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(x >> 32), CTRL, ROW_MASK, 0xf, true);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double wave_sum_dpp(double v) {
    v += dpp_move<0x111, 0xf>(v);  // row_shr:1
    v += dpp_move<0x112, 0xf>(v);  // row_shr:2
    v += dpp_move<0x114, 0xf>(v);  // row_shr:4
    v += dpp_move<0x118, 0xf>(v);  // row_shr:8
    v += dpp_move<0x142, 0xa>(v);  // row_bcast:15
    v += dpp_move<0x143, 0xc>(v);  // row_bcast:31
    const unsigned long long x = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)x, 63);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(x >> 32), 63);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// sum over the block, result valid in every thread (fixed order)
__device__ __forceinline__ double block_sum_all(double v, double *sh) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = (blockDim.x + 63) >> 6;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int q = 0; q < nw; q++) s += sh[q];
    return s;
}

__device__ __forceinline__ void block_sum2_all(double &a, double &b, double *sh) {
    a = wave_sum(a);
    b = wave_sum(b);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = (blockDim.x + 63) >> 6;
    __syncthreads();
    if (lane == 0) {
        sh[w] = a;
        sh[32 + w] = b;
    }
    __syncthreads();
    a = 0.0;
    b = 0.0;
    for (int q = 0; q < nw; q++) {
        a += sh[q];
        b += sh[32 + q];
    }
}

inline int ifc_blocks(const IfcGeom &ig, int bs) {
    const int n = ig.i1 - ig.i0;
    if (n <= 0) return 0;
    const int b = (n + bs - 1) / bs;
    return (b + 7) & ~7;  // multiple of 8 keeps the XCD phase of the volume part
}

// ---------------------------------------------------------------------------
// linear interpolation of the coarse-grid correction (P e_c)
// ---------------------------------------------------------------------------
// (P e_c) at fine interior node n of a closure whose coarse closure holds ev:
// the coarse value where the node coincides with a coarse node, else the mean
// of the end points of the coarse edge it bisects
template <typename T>
__device__ __forceinline__ T coarse_corr(const T *__restrict__ ev, const int2 *__restrict__ cC, int Mc, const LNode &n) {
    // index direction (di, dj, dk) of that edge from the parity bits of
    // (i, j, k), one of the 7 edge directions of the index space:
    //   (i,j,k) mod 2: 000 001 010 011 100 101 110 111  (k j i)
    //   (di,dj,dk):    0    (1,0,0) (0,1,0) (-1,1,0) (0,0,1) (-1,0,1) (0,-1,1) (1,-1,1)
    // computed, not looked up, so the coarse loads depend on the node list
    // entry only
    const int pi = n.i & 1, pj = n.j & 1, pk = n.k & 1;
    const int dk = pk;
    const int dj = pk ? -pj : pj;
    const int di = (pj ^ pk) ? -pi : pi;
    // coarse end points of the bisected edge (the same node twice at even (i, j, k))
    const T e1 = ev[lslot(cC, Mc, (n.i - di) >> 1, (n.j - dj) >> 1, (n.k - dk) >> 1)];
    const T e2 = ev[lslot(cC, Mc, (n.i + di) >> 1, (n.j + dj) >> 1, (n.k + dk) >> 1)];
    return (pi | pj | pk) == 0 ? e1 : T(0.5) * (e1 + e2);
}

// (P e_c) at interface master t from its two coarse slots (equal where the
// master coincides with a coarse node)
template <typename T>
__device__ __forceinline__ T coarse_corr_ifc(const T *__restrict__ ec, const int *__restrict__ prl, int stride, int t) {
    return T(0.5) * (ec[prl[t]] + ec[prl[(long long)stride + t]]);
}

// ---------------------------------------------------------------------------
// red-black SOR colour pass
// ---------------------------------------------------------------------------
// PR: each node first receives its coarse-grid correction (the pass then
// runs on u + P e_c at its own colour; the other colour already holds it).
// TAIL: with r = b - A u of a node before its update, (1 - omega) r is the
// node's residual after the pass (its neighbours, all of the other colour,
// do not change in it).  kTailNorm: per-block partial sums of its square;
// kTailRes: it is written to rout at the node's slot.
constexpr int kTailNone = 0, kTailNorm = 1, kTailRes = 2;
template <typename T, bool VK, bool OWN0, bool NB0, bool PR, int TAIL, int CPB>
__global__ void __launch_bounds__(512) k_colour(VolGeom vg, IfcGeom ig, int nib, T *__restrict__ u,
                                                const T *__restrict__ b, Weights<T> w, T h, T omega, T om_d,
                                                Prol<T> p, double *__restrict__ partial, T *__restrict__ rout) {
    __shared__ double sh[64];
    const unsigned f = blockIdx.x;
    double r2 = 0.0;
    if (f < (unsigned)nib) {
        const int t = ig.i0 + (int)(f * blockDim.x + threadIdx.x);
        if (t < ig.i1 && !(ig.frozen && ig.frozen[t])) {
            const long long sl = ig.base + t;
            const T uo = OWN0 ? T(0) : PR ? u[sl] + coarse_corr_ifc(p.ec, p.prl, ig.stride, t) : u[sl];
            T acc = T(0), diag;
            // interface weights: variable k, or the intact-side stencils of a
            // Dirichlet-Neumann recovery (given also when k = 1)
            if (VK || w.wi) {
                diag = T(0);
#pragma unroll
                for (int e = 0; e < 6; e++) {
                    const T we = w.wi[(long long)e * ig.stride + t];
                    diag += we;
                    // edges of weight zero (outside an intact side) are not read
                    if (!NB0 && we != T(0)) acc += we * u[ig.nbr[(long long)e * ig.stride + t]];
                }
            } else {
                diag = T(6) * h;
                if (!NB0) {
#pragma unroll
                    for (int e = 0; e < 6; e++) acc += u[ig.nbr[(long long)e * ig.stride + t]];
                    acc *= h;
                }
            }
            const T rr = b[sl] - (diag * uo - acc);
            const T un = uo + omega * rr / diag;
            u[sl] = un;
            if (ig.gptr)
                for (int g = ig.gptr[t]; g < ig.gptr[t + 1]; g++) u[ig.gidx[g]] = un;
            if (TAIL == kTailNorm) {
                const double e = (1.0 - (double)omega) * (double)rr;
                r2 = e * e;
            }
            if (TAIL == kTailRes) rout[sl] = (T(1) - omega) * rr;
        }
    } else {
        // list holds only nodes of this colour
        const unsigned per_vol = list_blocks_per_vol<CPB>(vg);
        const unsigned blk = block_order(f - nib, gridDim.x - nib, vg.remap);
        T nv[CPB], rv[CPB];
        long long dst[CPB];
        bool ok[CPB];
#pragma unroll
        for (int q = 0; q < CPB; q++) {
            ok[q] = false;
            nv[q] = T(0);
            rv[q] = T(0);
            dst[q] = 0;
            LNode n;
            if (!list_node<CPB>(vg, blk, per_vol, q, n)) continue;
            const VolDesc d = vg.vd[n.v];
            const T *uv = u + d.vec;
            const Nb7 nb = nb7(vg, n);
            const int c0 = nb.c0;
            const T uo = OWN0 ? T(0) : PR ? uv[c0] + coarse_corr(p.ec + p.vdc[n.v].vec, p.cC, p.Mc, n) : uv[c0];
            T rr, res;
            if (VK) {
                const T *w0 = w.w0 + d.w, *w1 = w.w1 + d.w, *w2 = w.w2 + d.w;
                const T wap = w0[c0], wam = w0[nb.am], wbp = w1[c0], wbm = w1[nb.bm], wcp = w2[c0], wcm = w2[nb.cm];
                const T diag = ((wap + wam) + (wbp + wbm)) + (wcp + wcm);
                const T acc = NB0 ? T(0)
                                  : wap * uv[nb.ap] + wam * uv[nb.am] + wbp * uv[nb.bp] + wbm * uv[nb.bm] +
                                        wcp * uv[nb.cp] + wcm * uv[nb.cm];
                rr = (b + d.vec)[c0] - (diag * uo - acc);
                res = omega * rr / diag;
            } else {
                const T acc =
                    NB0 ? T(0) : (((uv[nb.ap] + uv[nb.am]) + (uv[nb.bp] + uv[nb.bm])) + (uv[nb.cp] + uv[nb.cm]));
                // diag = 6h, off-diagonal -h; om_d = omega / (6h)
                rr = (b + d.vec)[c0] - h * (T(6) * uo - acc);
                res = om_d * rr;
            }
            if (TAIL == kTailNorm) {
                const double e = (1.0 - (double)omega) * (double)rr;
                r2 += e * e;
            }
            if (TAIL == kTailRes) rv[q] = (T(1) - omega) * rr;
            nv[q] = uo + res;
            dst[q] = d.vec + c0;
            ok[q] = true;
        }
#pragma unroll
        for (int q = 0; q < CPB; q++)
            if (ok[q]) {
                u[dst[q]] = nv[q];
                if (TAIL == kTailRes) rout[dst[q]] = rv[q];
            }
    }
    if (TAIL == kTailNorm) {
        const double sum = block_sum_all(r2, sh);
        if (threadIdx.x == 0) partial[blockIdx.x] = sum;
    }
}

// ---------------------------------------------------------------------------
// residual r = b - A u (+ block partial sums of r^2)
// ---------------------------------------------------------------------------
template <typename T, typename TO, bool VK, bool WRITE, bool NORM, int CPB>
__global__ void __launch_bounds__(512) k_residual(VolGeom vg, IfcGeom ig, int nib, const T *__restrict__ u,
                                                  const T *__restrict__ b, Weights<T> w, T h, TO *__restrict__ r,
                                                  double *__restrict__ partial) {
    __shared__ double sh[64];
    const unsigned f = blockIdx.x;
    double acc2 = 0.0;
    if (f < (unsigned)nib) {
        const int t = ig.i0 + (int)(f * blockDim.x + threadIdx.x);
        if (t < ig.i1 && !(ig.frozen && ig.frozen[t])) {
            const long long sl = ig.base + t;
            const T uo = u[sl];
            T acc = T(0), diag;
            if (VK || w.wi) {
                diag = T(0);
#pragma unroll
                for (int e = 0; e < 6; e++) {
                    const T we = w.wi[(long long)e * ig.stride + t];
                    diag += we;
                    if (we != T(0)) acc += we * u[ig.nbr[(long long)e * ig.stride + t]];
                }
            } else {
                diag = T(6) * h;
#pragma unroll
                for (int e = 0; e < 6; e++) acc += u[ig.nbr[(long long)e * ig.stride + t]];
                acc *= h;
            }
            const T res = b[sl] - (diag * uo - acc);
            if (WRITE) r[sl] = (TO)res;
            acc2 = (double)res * (double)res;
        }
    } else {
        const unsigned per_vol = list_blocks_per_vol<CPB>(vg);
        const unsigned blk = block_order(f - nib, gridDim.x - nib, vg.remap);
        T res[CPB];
        long long dst[CPB];
        bool ok[CPB];
#pragma unroll
        for (int q = 0; q < CPB; q++) {
            ok[q] = false;
            res[q] = T(0);
            dst[q] = 0;
            LNode n;
            if (!list_node<CPB>(vg, blk, per_vol, q, n)) continue;
            const VolDesc d = vg.vd[n.v];
            const T *uv = u + d.vec;
            const Nb7 nb = nb7(vg, n);
            const int c0 = nb.c0;
            const T uo = uv[c0];
            T diag, acc;
            if (VK) {
                const T *w0 = w.w0 + d.w, *w1 = w.w1 + d.w, *w2 = w.w2 + d.w;
                const T wap = w0[c0], wam = w0[nb.am], wbp = w1[c0], wbm = w1[nb.bm], wcp = w2[c0], wcm = w2[nb.cm];
                diag = ((wap + wam) + (wbp + wbm)) + (wcp + wcm);
                acc = wap * uv[nb.ap] + wam * uv[nb.am] + wbp * uv[nb.bp] + wbm * uv[nb.bm] + wcp * uv[nb.cp] +
                      wcm * uv[nb.cm];
            } else {
                diag = T(6) * h;
                acc = h * (((uv[nb.ap] + uv[nb.am]) + (uv[nb.bp] + uv[nb.bm])) + (uv[nb.cp] + uv[nb.cm]));
            }
            res[q] = (b + d.vec)[c0] - (diag * uo - acc);
            dst[q] = d.vec + c0;
            ok[q] = true;
        }
#pragma unroll
        for (int q = 0; q < CPB; q++) {
            if (!ok[q]) continue;
            if (WRITE) r[dst[q]] = (TO)res[q];
            acc2 += (double)res[q] * (double)res[q];
        }
    }
    if (NORM) {
        const double s = block_sum_all(acc2, sh);
        if (threadIdx.x == 0) partial[blockIdx.x] = s;
    }
}

// ---------------------------------------------------------------------------
// restriction b_c = P^T r (weights 1 at the coinciding node, 1/2 at the 14
// Freudenthal neighbours, which are the midpoints of the coarse edges)
// ---------------------------------------------------------------------------
template <typename T, int CPB>
__global__ void __launch_bounds__(512) k_restrict(VolGeom vc, const VolDesc *__restrict__ vdf,
                                                  const int2 *__restrict__ fC, IfcGeom ig, int nib,
                                                  const int *__restrict__ rst, const T *__restrict__ rf,
                                                  T *__restrict__ bc) {
    const unsigned f = blockIdx.x;
    if (f < (unsigned)nib) {
        const int t = ig.i0 + (int)(f * blockDim.x + threadIdx.x);
        if (t >= ig.i1) return;
        if (ig.frozen && ig.frozen[t]) return;
        T s = T(0);
#pragma unroll
        for (int e = 1; e < 15; e++) s += rf[rst[(long long)e * ig.stride + t]];
        for (int e = 15; e < ig.w; e++) s += rf[rst[(long long)e * ig.stride + t]];
        bc[ig.base + t] = rf[rst[t]] + T(0.5) * s;
        return;
    }
    const unsigned per_vol = list_blocks_per_vol<CPB>(vc);
    const unsigned blk = block_order(f - nib, gridDim.x - nib, vc.remap);
    const int Mf = 2 * vc.M - 1;
    T nv[CPB];
    long long dst[CPB];
    bool ok[CPB];
#pragma unroll
    for (int q = 0; q < CPB; q++) {
        ok[q] = false;
        nv[q] = T(0);
        dst[q] = 0;
        LNode n;
        if (!list_node<CPB>(vc, blk, per_vol, q, n)) continue;
        const T *rv = rf + vdf[n.v].vec;
        // fine node (I,J,K) = (2i,2j,2k) (red) and its 14 Freudenthal neighbours,
        // grouped by fine row; a fine node (I',J',K') has colour (I'+K')&1
        const int I = 2 * n.i, J = 2 * n.j, K = 2 * n.k;
        const int t0 = I >> 1;  // half index of I (and of I+1)
        const int2 r0 = fC[row_of(Mf, J, K)];          // (I,J,K) red, (I+-1,J,K) black
        const int2 rjp = fC[row_of(Mf, J + 1, K)];     // (I-1,J+1,K) black, (I,J+1,K) red
        const int2 rjm = fC[row_of(Mf, J - 1, K)];     // (I+1,J-1,K) black, (I,J-1,K) red
        const int2 rcp = fC[row_of(Mf, J - 1, K + 1)]; // (I,J-1,K+1) black, (I+1,J-1,K+1) red
        const int2 rcm = fC[row_of(Mf, J + 1, K - 1)]; // (I,J+1,K-1) black, (I-1,J+1,K-1) red
        const int2 rkp = fC[row_of(Mf, J, K + 1)];     // (I-1,J,K+1) red, (I,J,K+1) black
        const int2 rkm = fC[row_of(Mf, J, K - 1)];     // (I+1,J,K-1) red, (I,J,K-1) black
        // axis neighbours
        const T s1 = ((rv[r0.y + t0] + rv[r0.y + t0 - 1]) + (rv[rjp.y + t0 - 1] + rv[rjm.y + t0])) +
                     (rv[rcp.y + t0] + rv[rcm.y + t0]);
        // face diagonals (0,+-1,0), (-+1,0,+-1), (+-1,-+1,+-1)
        const T s2 = ((rv[rjp.x + t0] + rv[rjm.x + t0]) + (rv[rkp.x + t0 - 1] + rv[rkm.x + t0])) +
                     (rv[rcp.x + t0] + rv[rcm.x + t0 - 1]);
        // body diagonal (0,0,+-1)
        const T s3 = rv[rkp.y + t0] + rv[rkm.y + t0];
        nv[q] = rv[r0.x + t0] + T(0.5) * ((s1 + s2) + s3);
        dst[q] = vc.vd[n.v].vec + lslot(vc.rowC, vc.M, n.i, n.j, n.k);
        ok[q] = true;
    }
#pragma unroll
    for (int q = 0; q < CPB; q++)
        if (ok[q]) bc[dst[q]] = nv[q];
}

// ---------------------------------------------------------------------------
// prolongation u_f += P e_c (linear interpolation)
// ---------------------------------------------------------------------------
template <typename T, int CPB>
__global__ void __launch_bounds__(512) k_prolong(VolGeom vf, const VolDesc *__restrict__ vdc, const int2 *__restrict__ cC,
                                                 int Mc, IfcGeom ig, int nib, const int *__restrict__ prl,
                                                 const T *__restrict__ ec, T *__restrict__ uf) {
    const unsigned f = blockIdx.x;
    if (f < (unsigned)nib) {
        const int t = ig.i0 + (int)(f * blockDim.x + threadIdx.x);
        if (t >= ig.i1) return;
        if (ig.frozen && ig.frozen[t]) return;
        const long long sl = ig.base + t;
        const T v = uf[sl] + coarse_corr_ifc(ec, prl, ig.stride, t);
        uf[sl] = v;
        if (ig.gptr)
            for (int g = ig.gptr[t]; g < ig.gptr[t + 1]; g++) uf[ig.gidx[g]] = v;
        return;
    }
    const unsigned per_vol = list_blocks_per_vol<CPB>(vf);
    const unsigned blk = block_order(f - nib, gridDim.x - nib, vf.remap);
    T nv[CPB];
    long long dst[CPB];
    bool ok[CPB];
#pragma unroll
    for (int q = 0; q < CPB; q++) {
        ok[q] = false;
        nv[q] = T(0);
        dst[q] = 0;
        LNode n;
        if (!list_node<CPB>(vf, blk, per_vol, q, n)) continue;
        const long long sl = vf.vd[n.v].vec + lslot(vf.rowC, vf.M, n.i, n.j, n.k);
        nv[q] = uf[sl] + coarse_corr(ec + vdc[n.v].vec, cC, Mc, n);
        dst[q] = sl;
        ok[q] = true;
    }
#pragma unroll
    for (int q = 0; q < CPB; q++)
        if (ok[q]) uf[dst[q]] = nv[q];
}

// ---------------------------------------------------------------------------
// general macro meshes: 15-point stencils (see Gen15)
// ---------------------------------------------------------------------------
// stencil tables in the value type of the pass
template <typename T>
__device__ __forceinline__ const T *gsel(const double *d, const float *f);
template <>
__device__ __forceinline__ const double *gsel<double>(const double *d, const float *) {
    return d;
}
template <>
__device__ __forceinline__ const float *gsel<float>(const double *, const float *f) {
    return f;
}

// A u at interface master t (diag: its diagonal entry); VK: the master's own
// 15 entries (per-element k, or the intact side of a Dirichlet-Neumann
// recovery), else its primitive's stencil
template <typename T, bool VK>
__device__ __forceinline__ T master_Au(const IfcGeom &ig, const Gen15 &g, const T *__restrict__ u, int t, T uo,
                                       T &diag) {
    T acc = T(0);
    if (VK) {
        const T *wi = gsel<T>(g.wi15, g.wi15f);
        diag = wi[t];
#pragma unroll
        for (int n = 1; n < 15; n++)
            acc += wi[(long long)n * ig.stride + t] * u[g.nb15[(long long)n * ig.stride + t]];
        // wider stencils of unstructured macro meshes (vertices of high valence)
        for (int n = 15; n < ig.w; n++)
            acc += wi[(long long)n * ig.stride + t] * u[g.nb15[(long long)n * ig.stride + t]];
    } else {
        const T *w = gsel<T>(g.wtab, g.wtabf) + 15LL * g.sid[t];
        diag = w[0];
#pragma unroll
        for (int n = 1; n < 15; n++) acc += w[n] * u[g.nb15[(long long)n * ig.stride + t]];
    }
    return diag * uo + acc;
}

// A u at a volume node of tetrahedron d.tet (c0: its slot in the closure);
// VK: forward edge n = 2e + 1 is weight e at the node's own slot, backward
// edge n = 2e + 2 is weight e at the neighbour's slot
template <typename T, bool VK>
__device__ __forceinline__ T volume_Au(const VolGeom &vg, const Gen15 &g, const VolDesc &d, const LNode &nd,
                                       const T *__restrict__ uv, int &c0, T &uo, T &diag) {
    const int4 *e4 = (const int4 *)(g.rowN15 + 16 * ((long long)((nd.i + nd.k) & 1) * vg.nrows + nd.r));
    const int4 E0 = e4[0], E1 = e4[1], E2 = e4[2], E3 = e4[3];
    const int t = nd.i >> 1;
    const int sl[15] = {E0.x, E0.y, E0.z, E0.w, E1.x, E1.y, E1.z, E1.w, E2.x, E2.y, E2.z, E2.w, E3.x, E3.y, E3.z};
    c0 = sl[0] + t;
    uo = uv[c0];
    T acc = T(0);
    if (VK) {
        const T *W = gsel<T>(g.wv, g.wvf) + d.w;
        diag = W[7 * g.ws + c0];
#pragma unroll
        for (int n = 1; n < 15; n++) {
            const int sn = sl[n] + t;
            const T w = (n & 1) ? W[((n - 1) >> 1) * g.ws + c0] : W[((n - 2) >> 1) * g.ws + sn];
            acc += w * uv[sn];
        }
    } else {
        const T *w = gsel<T>(g.w15, g.w15f) + 15LL * d.tet;
        diag = w[0];
#pragma unroll
        for (int n = 1; n < 15; n++) acc += w[n] * uv[sl[n] + t];
    }
    return diag * uo + acc;
}

// VKV: per-node volume weights (wv), VKI: per-master entries (wi15)
// TAIL as in k_colour: (1 - omega) r is a node's residual after its class
// pass (no 15-point stencil couples two nodes of one class)
template <typename T, bool VKV, bool VKI, int TAIL>
__global__ void __launch_bounds__(512) k_colour15(VolGeom vg, IfcGeom ig, Gen15 g, int nib, T *__restrict__ u,
                                                  const T *__restrict__ b, T omega, double *__restrict__ partial,
                                                  T *__restrict__ rout) {
    __shared__ double sh[64];
    const unsigned f = blockIdx.x;
    double r2 = 0.0;
    if (f < (unsigned)nib) {
        const int q = (int)(f * blockDim.x + threadIdx.x);
        if (q < g.nq) {
            const int t = g.ifcq[q];
            if (!(ig.frozen && ig.frozen[t])) {
                const long long sl = ig.base + t;
                const T uo = u[sl];
                T diag;
                const T rr = b[sl] - master_Au<T, VKI>(ig, g, u, t, uo, diag);
                const T un = uo + omega * rr / diag;
                u[sl] = un;
                if (ig.gptr)
                    for (int gq = ig.gptr[t]; gq < ig.gptr[t + 1]; gq++) u[ig.gidx[gq]] = un;
                if (TAIL == kTailNorm) {
                    const double e = (1.0 - (double)omega) * (double)rr;
                    r2 = e * e;
                }
                if (TAIL == kTailRes) rout[sl] = (T(1) - omega) * rr;
            }
        }
    } else {
        const unsigned per_vol = list_blocks_per_vol<1>(vg);
        const unsigned blk = block_order(f - nib, gridDim.x - nib, vg.remap);
        LNode nd;
        if (list_node<1>(vg, blk, per_vol, 0, nd)) {
            const VolDesc d = vg.vd[nd.v];
            T *uv = u + d.vec;
            int c0;
            T uo, diag;
            const T Au = volume_Au<T, VKV>(vg, g, d, nd, uv, c0, uo, diag);
            const T rr = (b + d.vec)[c0] - Au;
            uv[c0] = uo + omega * rr / diag;
            if (TAIL == kTailNorm) {
                const double e = (1.0 - (double)omega) * (double)rr;
                r2 = e * e;
            }
            if (TAIL == kTailRes) (rout + d.vec)[c0] = (T(1) - omega) * rr;
        }
    }
    if (TAIL == kTailNorm) {
        const double sum = block_sum_all(r2, sh);
        if (threadIdx.x == 0) partial[blockIdx.x] = sum;
    }
}

// r = b - A u in the value type T, written as TO
template <typename T, typename TO, bool WRITE, bool NORM, bool VKV, bool VKI>
__global__ void __launch_bounds__(512) k_residual15(VolGeom vg, IfcGeom ig, Gen15 g, int nib, const T *__restrict__ u,
                                                    const T *__restrict__ b, TO *__restrict__ r,
                                                    double *__restrict__ partial) {
    __shared__ double sh[64];
    const unsigned f = blockIdx.x;
    double acc2 = 0.0;
    if (f < (unsigned)nib) {
        // the masters g.ifcq[0 .. nq) if listed, else [ig.i0, ig.i1)
        const int q = (int)(f * blockDim.x + threadIdx.x);
        const int t = g.ifcq ? (q < g.nq ? g.ifcq[q] : -1) : (ig.i0 + q < ig.i1 ? ig.i0 + q : -1);
        if (t >= 0 && !(ig.frozen && ig.frozen[t])) {
            const long long sl = ig.base + t;
            T diag;
            const T res = b[sl] - master_Au<T, VKI>(ig, g, u, t, u[sl], diag);
            if (WRITE) r[sl] = (TO)res;
            acc2 = (double)res * (double)res;
        }
    } else {
        const unsigned per_vol = list_blocks_per_vol<1>(vg);
        const unsigned blk = block_order(f - nib, gridDim.x - nib, vg.remap);
        LNode nd;
        if (list_node<1>(vg, blk, per_vol, 0, nd)) {
            const VolDesc d = vg.vd[nd.v];
            int c0;
            T uo, diag;
            const T Au = volume_Au<T, VKV>(vg, g, d, nd, u + d.vec, c0, uo, diag);
            const T res = (b + d.vec)[c0] - Au;
            if (WRITE) r[d.vec + c0] = (TO)res;
            acc2 = (double)res * (double)res;
        }
    }
    if (NORM) {
        const double s = block_sum_all(acc2, sh);
        if (threadIdx.x == 0) partial[blockIdx.x] = s;
    }
}

// y = S x at every interior node of vg and every master of ig with the
// stencils of g (one per tetrahedron, and one per primitive or, with
// g.wi15, one per master; the mass matrix)
__global__ void __launch_bounds__(512) k_apply15(VolGeom vg, IfcGeom ig, Gen15 g, int nib, const double *__restrict__ x,
                                                 double *__restrict__ y) {
    const unsigned f = blockIdx.x;
    if (f < (unsigned)nib) {
        const int t = ig.i0 + (int)(f * blockDim.x + threadIdx.x);
        if (t >= ig.i1) return;
        double diag;
        y[ig.base + t] = g.wi15 ? master_Au<double, true>(ig, g, x, t, x[ig.base + t], diag)
                                : master_Au<double, false>(ig, g, x, t, x[ig.base + t], diag);
        return;
    }
    const unsigned per_vol = list_blocks_per_vol<1>(vg);
    const unsigned blk = block_order(f - nib, gridDim.x - nib, vg.remap);
    LNode nd;
    if (!list_node<1>(vg, blk, per_vol, 0, nd)) return;
    const VolDesc d = vg.vd[nd.v];
    int c0;
    double xo, diag;
    const double Sx = volume_Au<double, false>(vg, g, d, nd, x + d.vec, c0, xo, diag);
    y[d.vec + c0] = Sx;
}

// local coarsest level: u = b / diag at the single interior node (slot)
__global__ void k_local_coarse15(const VolDesc *__restrict__ vd, int nvol, int slot, Gen15 g,
                                 const double *__restrict__ b, double *__restrict__ u) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nvol) return;
    const VolDesc d = vd[v];
    const double diag = g.wv ? g.wv[7 * g.ws + d.w + slot] : g.w15[15LL * d.tet];
    (u + d.vec)[slot] = (b + d.vec)[slot] / diag;
}

// ---------------------------------------------------------------------------
// coarsest level: Jacobi-PCG in one workgroup, unknowns owned by threads,
// search direction shared through LDS
// ---------------------------------------------------------------------------
template <typename T, int NPT, int NB = 6>
__global__ void __launch_bounds__(1024) k_coarse_pcg(int n, const long long *__restrict__ slot,
                                                     const int *__restrict__ col, const double *__restrict__ val,
                                                     const unsigned char *__restrict__ frozen, const T *__restrict__ b,
                                                     T *__restrict__ u, const int *__restrict__ cptr,
                                                     const int *__restrict__ cidx, double rtol, int maxit,
                                                     int *__restrict__ iters) {
    __shared__ double p_sh[2048];
    __shared__ double red[64];
    const int tid = threadIdx.x, nt = blockDim.x;
    // every thread owns NPT unknowns; their matrix rows stay in registers
    double x[NPT], r[NPT], p[NPT], dinv[NPT], dg[NPT], av[NPT][NB];
    int ac[NPT][NB];
    bool act[NPT];
#pragma unroll
    for (int s = 0; s < NPT; s++) {
        const int q = tid + s * nt;
        act[s] = q < n && !(frozen && frozen[q]);
        x[s] = 0.0;
        r[s] = 0.0;
        p[s] = 0.0;
        dinv[s] = 0.0;
        dg[s] = 0.0;
#pragma unroll
        for (int e = 0; e < NB; e++) {
            ac[s][e] = 0;
            av[s][e] = 0.0;
        }
        if (q < n) {
            if (act[s]) {
                dg[s] = val[(NB + 1) * q];
                dinv[s] = 1.0 / dg[s];
                r[s] = (double)b[slot[q]];
#pragma unroll
                for (int e = 0; e < NB; e++) {
                    const int c = col[(NB + 1) * q + 1 + e];
                    ac[s][e] = c >= 0 ? c : 0;
                    av[s][e] = c >= 0 ? val[(NB + 1) * q + 1 + e] : 0.0;
                }
            }
            p[s] = r[s] * dinv[s];
            p_sh[q] = p[s];
        }
    }
    double rz = 0.0, rr0 = 0.0;
#pragma unroll
    for (int s = 0; s < NPT; s++) {
        rz += r[s] * p[s];
        rr0 += r[s] * r[s];
    }
    block_sum2_all(rz, rr0, red);
    int it = 0;
    if (rr0 > 0.0) {
        const double stop = rtol * rtol * rr0;
        for (it = 1; it <= maxit; it++) {
            __syncthreads();
            double qv[NPT];
            double pq = 0.0, dummy = 0.0;
#pragma unroll
            for (int s = 0; s < NPT; s++) {
                double a = 0.0;
                if (act[s]) {
                    a = dg[s] * p[s];
#pragma unroll
                    for (int e = 0; e < NB; e++) a += av[s][e] * p_sh[ac[s][e]];
                }
                qv[s] = a;
                pq += p[s] * a;
            }
            block_sum2_all(pq, dummy, red);
            const double alpha = rz / pq;
            double rr = 0.0, rz1 = 0.0;
#pragma unroll
            for (int s = 0; s < NPT; s++) {
                x[s] += alpha * p[s];
                r[s] -= alpha * qv[s];
                rr += r[s] * r[s];
                rz1 += r[s] * r[s] * dinv[s];
            }
            block_sum2_all(rr, rz1, red);
            if (rr <= stop) break;
            const double beta = rz1 / rz;
            rz = rz1;
#pragma unroll
            for (int s = 0; s < NPT; s++) {
                const int q = tid + s * nt;
                p[s] = r[s] * dinv[s] + beta * p[s];
                if (q < n) p_sh[q] = p[s];
            }
        }
    }
#pragma unroll
    for (int s = 0; s < NPT; s++) {
        const int q = tid + s * nt;
        if (!act[s]) continue;
        const T xv = (T)x[s];
        for (int c = cptr[q]; c < cptr[q + 1]; c++) u[cidx[c]] = xv;
    }
    if (tid == 0 && iters) *iters = it;
}

// the same Jacobi-PCG in a single wavefront (n <= 64 NPT): reductions are
// wave shuffles and the only barrier is the one that publishes p in LDS
template <typename T, int NPT, int NB = 6>
__global__ void __launch_bounds__(64) k_coarse_pcg_wave(int n, const long long *__restrict__ slot,
                                                        const int *__restrict__ col, const double *__restrict__ val,
                                                        const unsigned char *__restrict__ frozen,
                                                        const T *__restrict__ b, T *__restrict__ u,
                                                        const int *__restrict__ cptr, const int *__restrict__ cidx,
                                                        double rtol, int maxit, int *__restrict__ iters) {
    __shared__ double p_sh[64 * NPT];
    const int tid = threadIdx.x;
    double x[NPT], r[NPT], p[NPT], dinv[NPT], dg[NPT], av[NPT][NB];
    int ac[NPT][NB];
    bool act[NPT];
#pragma unroll
    for (int s = 0; s < NPT; s++) {
        const int q = tid + 64 * s;
        act[s] = q < n && !(frozen && frozen[q]);
        x[s] = 0.0;
        r[s] = 0.0;
        p[s] = 0.0;
        dinv[s] = 0.0;
        dg[s] = 0.0;
#pragma unroll
        for (int e = 0; e < NB; e++) {
            ac[s][e] = 0;
            av[s][e] = 0.0;
        }
        if (act[s]) {
            dg[s] = val[(NB + 1) * q];
            dinv[s] = 1.0 / dg[s];
            r[s] = (double)b[slot[q]];
#pragma unroll
            for (int e = 0; e < NB; e++) {
                const int c = col[(NB + 1) * q + 1 + e];
                ac[s][e] = c >= 0 ? c : 0;
                av[s][e] = c >= 0 ? val[(NB + 1) * q + 1 + e] : 0.0;
            }
        }
        p[s] = r[s] * dinv[s];
        p_sh[q] = p[s];
    }
    double rz = 0.0, rr0 = 0.0;
#pragma unroll
    for (int s = 0; s < NPT; s++) {
        rz += r[s] * p[s];
        rr0 += r[s] * r[s];
    }
    rz = wave_sum_dpp(rz);
    rr0 = wave_sum_dpp(rr0);
    int it = 0;
    if (rr0 > 0.0) {
        const double stop = rtol * rtol * rr0;
        for (it = 1; it <= maxit; it++) {
            __syncthreads();
            double qv[NPT];
            double pq = 0.0;
#pragma unroll
            for (int s = 0; s < NPT; s++) {
                double a = 0.0;
                if (act[s]) {
                    a = dg[s] * p[s];
#pragma unroll
                    for (int e = 0; e < NB; e++) a += av[s][e] * p_sh[ac[s][e]];
                }
                qv[s] = a;
                pq += p[s] * a;
            }
            pq = wave_sum_dpp(pq);
            const double alpha = rz / pq;
            double rr = 0.0, rz1 = 0.0;
#pragma unroll
            for (int s = 0; s < NPT; s++) {
                x[s] += alpha * p[s];
                r[s] -= alpha * qv[s];
                rr += r[s] * r[s];
                rz1 += r[s] * r[s] * dinv[s];
            }
            rr = wave_sum_dpp(rr);
            rz1 = wave_sum_dpp(rz1);
            if (rr <= stop) break;
            const double beta = rz1 / rz;
            rz = rz1;
            __syncthreads();  // every lane has finished reading p_sh
#pragma unroll
            for (int s = 0; s < NPT; s++) {
                p[s] = r[s] * dinv[s] + beta * p[s];
                p_sh[tid + 64 * s] = p[s];
            }
        }
    }
#pragma unroll
    for (int s = 0; s < NPT; s++) {
        const int q = tid + 64 * s;
        if (!act[s]) continue;
        const T xv = (T)x[s];
        for (int c = cptr[q]; c < cptr[q + 1]; c++) u[cidx[c]] = xv;
    }
    if (tid == 0 && iters) *iters = it;
}

// coarsest level with a precomputed dense inverse (row-major n x n): one
// wavefront per unknown q computes x_q = sum_j inv[q][j] b_j in a fixed order
// (the reduction leaves lane 63's total in every lane, so the master and its
// ghost copies receive the same value)
template <typename T>
__global__ void __launch_bounds__(256) k_coarse_dense(int n, const long long *__restrict__ slot,
                                                      const double *__restrict__ inv, const T *__restrict__ b,
                                                      T *__restrict__ u, const int *__restrict__ cptr,
                                                      const int *__restrict__ cidx) {
    const int q = (int)blockIdx.x * 4 + (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
    if (q >= n) return;  // uniform over the wavefront
    const double *a = inv + (long long)q * n;
    double acc = 0.0;
    for (int j = lane; j < n; j += 64) acc += a[j] * (double)b[slot[j]];
    const T xv = (T)wave_sum_dpp(acc);
    for (int c = cptr[q] + lane; c < cptr[q + 1]; c += 64) u[cidx[c]] = xv;
}

template <typename T, bool VK>
__global__ void k_local_coarse(const VolDesc *__restrict__ vd, int nvol, int4 sl, const T *__restrict__ b,
                               T *__restrict__ u, Weights<T> w, T h) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nvol) return;
    const VolDesc d = vd[v];
    // the single interior node (1,1,1) of a tetrahedron with 4 segments per edge
    const int c0 = sl.x;
    T diag;
    if (VK) {
        const T *w0 = w.w0 + d.w, *w1 = w.w1 + d.w, *w2 = w.w2 + d.w;
        diag = ((w0[c0] + w0[sl.y]) + (w1[c0] + w1[sl.z])) + (w2[c0] + w2[sl.w]);
    } else {
        diag = T(6) * h;
    }
    (u + d.vec)[c0] = (b + d.vec)[c0] / diag;
}

__global__ void __launch_bounds__(1024) k_reduce(const double *__restrict__ partial, int n, double *__restrict__ out) {
    __shared__ double sh[64];
    double s = 0.0;
    for (int q = threadIdx.x; q < n; q += blockDim.x) s += partial[q];
    s = block_sum_all(s, sh);
    if (threadIdx.x == 0) out[0] = s;
}

template <typename T>
__global__ void k_fill(T *__restrict__ p, long long n, T v) {
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x)
        p[q] = v;
}

template <typename TI, typename TO>
__global__ void k_cast(const TI *__restrict__ in, TO *__restrict__ out, long long n) {
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x)
        out[q] = (TO)in[q];
}

template <typename T>
__global__ void k_ghost_refresh(const int *__restrict__ dst, const int *__restrict__ src, int n, T *__restrict__ u) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) u[dst[q]] = u[src[q]];
}

// grid position of closure node (i,j,k) of tet t at a level with m segments
__device__ __forceinline__ void grid_pos(const int *tetinfo, int t, int m, int i, int j, int k, int X[3]) {
    const int *ti = tetinfo + 6 * t;
    X[0] = m * ti[0] + k;
    X[1] = m * ti[1] + k;
    X[2] = m * ti[2] + k;
    X[ti[3]] += i + j;
    X[ti[4]] += j;
}

template <typename T>
__global__ void __launch_bounds__(512) k_user_to_slots(VolGeom vg, const int *__restrict__ tetinfo, int m, int N,
                                                       IfcGeom ig, int nib, const int *__restrict__ ifc_dof,
                                                       const double *__restrict__ user, T *__restrict__ vec) {
    const unsigned f = blockIdx.x;
    if (f < (unsigned)nib) {
        const int t = ig.i0 + (int)(f * blockDim.x + threadIdx.x);
        if (t >= ig.i1) return;
        vec[ig.base + t] = (T)user[ifc_dof[t]];
        return;
    }
    const unsigned per_vol = list_blocks_per_vol<1>(vg);
    LNode n;
    if (!list_node<1>(vg, block_order(f - nib, gridDim.x - nib, vg.remap), per_vol, 0, n)) return;
    const VolDesc d = vg.vd[n.v];
    int X[3];
    grid_pos(tetinfo, d.tet, m, n.i, n.j, n.k, X);
    const bool in = X[0] > 0 && X[1] > 0 && X[2] > 0 && X[0] < N && X[1] < N && X[2] < N;
    const long long dof = (long long)(X[0] - 1) + (long long)(N - 1) * ((X[1] - 1) + (long long)(N - 1) * (X[2] - 1));
    const double uv = user[in ? dof : 0];  // boundary nodes read a valid address and store zero
    (vec + d.vec)[lslot(vg.rowC, vg.M, n.i, n.j, n.k)] = in ? (T)uv : T(0);
}

template <typename T, int CPB>
__global__ void __launch_bounds__(512) k_slots_to_user(VolGeom vg, const int *__restrict__ tetinfo, int m, int N,
                                                       IfcGeom ig, int nib, const int *__restrict__ ifc_dof,
                                                       const T *__restrict__ vec, double *__restrict__ user) {
    const unsigned f = blockIdx.x;
    if (f < (unsigned)nib) {
        const int t = ig.i0 + (int)(f * blockDim.x + threadIdx.x);
        if (t >= ig.i1) return;
        user[ifc_dof[t]] = (double)vec[ig.base + t];
        return;
    }
    const unsigned per_vol = list_blocks_per_vol<CPB>(vg);
    const unsigned blk = block_order(f - nib, gridDim.x - nib, vg.remap);
#pragma unroll
    for (int q = 0; q < CPB; q++) {
        LNode n;
        if (!list_node<CPB>(vg, blk, per_vol, q, n)) continue;
        const VolDesc d = vg.vd[n.v];
        int X[3];
        grid_pos(tetinfo, d.tet, m, n.i, n.j, n.k, X);
        const long long dof =
            (long long)(X[0] - 1) + (long long)(N - 1) * ((X[1] - 1) + (long long)(N - 1) * (X[2] - 1));
        user[dof] = (double)(vec + d.vec)[lslot(vg.rowC, vg.M, n.i, n.j, n.k)];
    }
}

// rank of interior node (i, j, k) among the interior nodes of a closure with
// m = M - 1 segments, in plane k, row j, i order: the planes below hold
// C(p,3) - C(p-k+1,3) nodes (p = m - 1), the rows below in plane k
// (j - 1)(p - k) - (j - 1) j / 2
__device__ __forceinline__ long long interior_rank(int M, int i, int j, int k) {
    const long long p = M - 2, a = p - k + 1;
    const long long below = (p * (p - 1) * (p - 2) - a * (a - 1) * (a - 2)) / 6;
    return below + (long long)(j - 1) * (p - k) - (long long)(j - 1) * j / 2 + (i - 1);
}

template <typename T>
__global__ void __launch_bounds__(512) k_mesh_user_to_slots(VolGeom vg, long long vbase, long long nint, IfcGeom ig,
                                                            int nib, const int *__restrict__ ifc_dof,
                                                            const double *__restrict__ user, T *__restrict__ vec) {
    const unsigned f = blockIdx.x;
    if (f < (unsigned)nib) {
        const int t = ig.i0 + (int)(f * blockDim.x + threadIdx.x);
        if (t >= ig.i1) return;
        vec[ig.base + t] = (T)user[ifc_dof[t]];
        return;
    }
    const unsigned per_vol = list_blocks_per_vol<1>(vg);
    LNode n;
    if (!list_node<1>(vg, block_order(f - nib, gridDim.x - nib, vg.remap), per_vol, 0, n)) return;
    const VolDesc d = vg.vd[n.v];
    const long long dof = vbase + (long long)d.tet * nint + interior_rank(vg.M, n.i, n.j, n.k);
    (vec + d.vec)[lslot(vg.rowC, vg.M, n.i, n.j, n.k)] = (T)user[dof];
}

template <typename T>
__global__ void __launch_bounds__(512) k_mesh_slots_to_user(VolGeom vg, long long vbase, long long nint, IfcGeom ig,
                                                            int nib, const int *__restrict__ ifc_dof,
                                                            const T *__restrict__ vec, double *__restrict__ user) {
    const unsigned f = blockIdx.x;
    if (f < (unsigned)nib) {
        const int t = ig.i0 + (int)(f * blockDim.x + threadIdx.x);
        if (t >= ig.i1) return;
        user[ifc_dof[t]] = (double)vec[ig.base + t];
        return;
    }
    const unsigned per_vol = list_blocks_per_vol<1>(vg);
    LNode n;
    if (!list_node<1>(vg, block_order(f - nib, gridDim.x - nib, vg.remap), per_vol, 0, n)) return;
    const VolDesc d = vg.vd[n.v];
    const long long dof = vbase + (long long)d.tet * nint + interior_rank(vg.M, n.i, n.j, n.k);
    user[dof] = (double)(vec + d.vec)[lslot(vg.rowC, vg.M, n.i, n.j, n.k)];
}

// consistent P1 mass matrix on the Kuhn meshes: diagonal 24 h^3/60, axis
// edges h^3/20 (6 tetrahedra), face diagonals h^3/30 (4), body diagonal h^3/20 (6)
template <int CPB>
__global__ void __launch_bounds__(512) k_mass(VolGeom vg, IfcGeom ig, int nib, const int *__restrict__ nb15,
                                              const double *__restrict__ x, double *__restrict__ y, double h3) {
    const double wc = 0.4 * h3, wax = h3 / 20.0, wfd = h3 / 30.0, wbd = h3 / 20.0;
    const unsigned f = blockIdx.x;
    if (f < (unsigned)nib) {
        const int t = ig.i0 + (int)(f * blockDim.x + threadIdx.x);
        if (t >= ig.i1) return;
        const long long st = ig.stride;
        double ax = 0.0, fd = 0.0, bd = 0.0;
        for (int e = 1; e < 7; e++) ax += x[nb15[e * st + t]];
        for (int e = 7; e < 13; e++) fd += x[nb15[e * st + t]];
        for (int e = 13; e < 15; e++) bd += x[nb15[e * st + t]];
        y[ig.base + t] = wc * x[nb15[t]] + wax * ax + wfd * fd + wbd * bd;
        return;
    }
    const unsigned per_vol = list_blocks_per_vol<CPB>(vg);
    const unsigned blk = block_order(f - nib, gridDim.x - nib, vg.remap);
    const int M = vg.M;
#pragma unroll
    for (int q = 0; q < CPB; q++) {
        LNode n;
        if (!list_node<CPB>(vg, blk, per_vol, q, n)) continue;
        const VolDesc d = vg.vd[n.v];
        const double *xv = x + d.vec;
        const int i = n.i, j = n.j, k = n.k;
        auto X = [&](int di, int dj, int dk) { return xv[lslot(vg.rowC, M, i + di, j + dj, k + dk)]; };
        // axis (a, b, c), face diagonals (a+b, b+c, a+c), body diagonal (a+b+c)
        const double ax =
            ((X(1, 0, 0) + X(-1, 0, 0)) + (X(-1, 1, 0) + X(1, -1, 0))) + (X(0, -1, 1) + X(0, 1, -1));
        const double fd =
            ((X(0, 1, 0) + X(0, -1, 0)) + (X(-1, 0, 1) + X(1, 0, -1))) + (X(1, -1, 1) + X(-1, 1, -1));
        const double bd = X(0, 0, 1) + X(0, 0, -1);
        (y + d.vec)[lslot(vg.rowC, M, i, j, k)] = wc * X(0, 0, 0) + wax * ax + wfd * fd + wbd * bd;
    }
}

// b = M f on the unit cube's Kuhn mesh in vector order (interior node
// (x, y, z) at (x-1) + (N-1)((y-1) + (N-1)(z-1)); f = 0 on the boundary).
// The consistent P1 mass matrix does not depend on k: 0.4 h^3 on the
// diagonal, h^3/20 to the 6 axis neighbours (6 elements share such an edge),
// h^3/30 to the face diagonals (1,1,0), (0,1,1), (1,0,1) (4 elements) and
// h^3/20 to the body diagonal (1,1,1) (6 elements), each in both signs.
__global__ void __launch_bounds__(256) k_mass_grid(int N, double h3, const double *__restrict__ f,
                                                   double *__restrict__ b) {
    const int n = N - 1;
    const long long sz = (long long)n * n;
    const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
    if (q >= sz * n) return;
    const int x = (int)(q % n), y = (int)((q / n) % n), z = (int)(q / sz);
    // a neighbour outside the interior reads the node itself (a valid
    // address) and contributes zero
    auto F = [&](int dx, int dy, int dz) -> double {
        const bool in = (unsigned)(x + dx) < (unsigned)n && (unsigned)(y + dy) < (unsigned)n &&
                        (unsigned)(z + dz) < (unsigned)n;
        const double v = f[in ? q + dx + (long long)dy * n + (long long)dz * sz : q];
        return in ? v : 0.0;
    };
    const double wc = 0.4 * h3, wax = h3 / 20.0, wfd = h3 / 30.0, wbd = h3 / 20.0;
    const double ax = ((F(1, 0, 0) + F(-1, 0, 0)) + (F(0, 1, 0) + F(0, -1, 0))) + (F(0, 0, 1) + F(0, 0, -1));
    const double fd = ((F(1, 1, 0) + F(-1, -1, 0)) + (F(0, 1, 1) + F(0, -1, -1))) + (F(1, 0, 1) + F(-1, 0, -1));
    const double bd = F(1, 1, 1) + F(-1, -1, -1);
    b[q] = wc * F(0, 0, 0) + wax * ax + wfd * fd + wbd * bd;
}

// per-block partial sums of v^2 over the volume nodes of vg's list and the
// interface masters of ig (every interior node once); CPB volume nodes per
// thread, whose load chains (list entry, row table, value) are independent
template <int CPB>
__global__ void __launch_bounds__(512) k_norm2(VolGeom vg, IfcGeom ig, int nib, const double *__restrict__ v,
                                               double *__restrict__ partial) {
    __shared__ double sh[64];
    const unsigned f = blockIdx.x;
    double acc = 0.0;
    if (f < (unsigned)nib) {
        const int t = ig.i0 + (int)(f * blockDim.x + threadIdx.x);
        if (t < ig.i1) {
            const double x = v[ig.base + t];
            acc = x * x;
        }
    } else {
        const unsigned per_vol = list_blocks_per_vol<CPB>(vg);
        const unsigned blk = block_order(f - nib, gridDim.x - nib, vg.remap);
        double x[CPB];
#pragma unroll
        for (int q = 0; q < CPB; q++) {
            x[q] = 0.0;
            LNode n;
            if (list_node<CPB>(vg, blk, per_vol, q, n)) x[q] = (v + vg.vd[n.v].vec)[lslot(vg.rowC, vg.M, n.i, n.j, n.k)];
        }
#pragma unroll
        for (int q = 0; q < CPB; q++) acc += x[q] * x[q];
    }
    const double s = block_sum_all(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ void __launch_bounds__(256) k_update_add(const VolDesc *__restrict__ vd, long long span, IfcGeom ig,
                                                    int nib, double *__restrict__ u, const float *__restrict__ e) {
    const unsigned f = blockIdx.x;
    if (f < (unsigned)nib) {
        const int t = ig.i0 + (int)(f * blockDim.x + threadIdx.x);
        if (t >= ig.i1) return;
        const long long sl = ig.base + t;
        u[sl] += (double)e[sl];
        return;
    }
    // span slots per volume, 4 per thread
    const long long per_vol = (span + 1023) / 1024;
    const long long g = f - nib;
    const long long v = g / per_vol, o0 = (g % per_vol) * 1024 + threadIdx.x;
    const long long base = vd[v].vec;
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const long long o = o0 + 256 * q;
        if (o < span) u[base + o] += (double)e[base + o];
    }
}

// ---------------------------------------------------------------------------
// coefficients
// ---------------------------------------------------------------------------
__device__ __constant__ int kPermD[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

__device__ __forceinline__ int perm_id(int a, int b) {
    // third axis is implied
    return a == 0 ? (b == 1 ? 0 : 1) : a == 1 ? (b == 0 ? 2 : 3) : (b == 0 ? 4 : 5);
}

// Bey children of coarse element (C, p) with a = e_p0, b = e_p1, c = e_p2:
// (2C,p) (2C+a,p) (2C+a+b,p) (2C+a+b+c,p) (2C+a,(p1,p2,p0)) (2C+a,(p1,p0,p2))
// (2C+a+b,(p2,p0,p1)) (2C+a+b,(p0,p2,p1)); coarse k = their mean.
__global__ void k_coarsen_k(const double *__restrict__ kf, int Nf, double *__restrict__ kc, int Nc) {
    const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const long long ne = 6LL * Nc * Nc * Nc;
    if (e >= ne) return;
    const int q = (int)(e % 6);
    long long cell = e / 6;
    const int cx = (int)(cell % Nc);
    cell /= Nc;
    const int cy = (int)(cell % Nc);
    const int cz = (int)(cell / Nc);
    const int p0 = kPermD[q][0], p1 = kPermD[q][1], p2 = kPermD[q][2];
    int base[3] = {2 * cx, 2 * cy, 2 * cz};
    auto fe = [&](int da, int db, int dc, int pa, int pb) {
        int X[3] = {base[0], base[1], base[2]};
        X[p0] += da;
        X[p1] += db;
        X[p2] += dc;
        return kf[6LL * (X[0] + (long long)Nf * (X[1] + (long long)Nf * X[2])) + perm_id(pa, pb)];
    };
    double s = fe(0, 0, 0, p0, p1);
    s += fe(1, 0, 0, p0, p1);
    s += fe(1, 1, 0, p0, p1);
    s += fe(1, 1, 1, p0, p1);
    s += fe(1, 0, 0, p1, p2);
    s += fe(1, 0, 0, p1, p0);
    s += fe(1, 1, 0, p2, p0);
    s += fe(1, 1, 0, p0, p2);
    kc[e] = s / 8.0;
}

// weight of grid edge (X, X + e_a): h/6 times the sum of k over the
// tetrahedra that have it on their axis path (a cell c = X - delta, delta_a = 0,
// and a permutation listing the axes set in delta first, then a)
__device__ double edge_w(const double *__restrict__ k, int N, double h, int x, int y, int z, int a) {
    double sum = 0.0;
    const int P[3] = {x, y, z};
    for (int dd = 0; dd < 8; dd++) {
        const int dl[3] = {dd & 1, (dd >> 1) & 1, (dd >> 2) & 1};
        if (dl[a]) continue;
        const int c[3] = {P[0] - dl[0], P[1] - dl[1], P[2] - dl[2]};
        if (c[0] < 0 || c[1] < 0 || c[2] < 0 || c[0] >= N || c[1] >= N || c[2] >= N) continue;
        const int ns = dl[0] + dl[1] + dl[2];
        for (int q = 0; q < 6; q++) {
            bool ok = kPermD[q][ns] == a;
            for (int s = 0; s < ns; s++) ok = ok && dl[kPermD[q][s]];
            if (ok) sum += k[6LL * (c[0] + (long long)N * (c[1] + (long long)N * c[2])) + q];
        }
    }
    return sum * h / 6.0;
}

__global__ void __launch_bounds__(512) k_vol_weights(VolGeom vg, const int *__restrict__ tetinfo, int m, int N,
                                                     double h, const double *__restrict__ k, double *__restrict__ w0,
                                                     double *__restrict__ w1, double *__restrict__ w2) {
    LNode n;
    if (!list_node<1>(vg, block_order(blockIdx.x, gridDim.x, vg.remap), list_blocks_per_vol<1>(vg), 0, n)) return;
    const VolDesc d = vg.vd[n.v];
    int X[3];
    grid_pos(tetinfo, d.tet, m, n.i, n.j, n.k, X);
    const int *ti = tetinfo + 6 * d.tet;
    const long long sl = d.w + lslot(vg.rowC, vg.M, n.i, n.j, n.k);
    // local direction s goes along grid axis p_s; skip edges that leave the cube
    double v[3];
    for (int s = 0; s < 3; s++) {
        const int ax = ti[3 + s];
        v[s] = (X[ax] < N) ? edge_w(k, N, h, X[0], X[1], X[2], ax) : 0.0;
    }
    w0[sl] = v[0];
    w1[sl] = v[1];
    w2[sl] = v[2];
}

__global__ void k_ifc_weights(int n_ifc, const int *__restrict__ xyz, int N, double h, const double *__restrict__ k,
                              double *__restrict__ wi) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_ifc) return;
    const int x = xyz[3 * t], y = xyz[3 * t + 1], z = xyz[3 * t + 2];
    const int X[3] = {x, y, z};
    for (int a = 0; a < 3; a++) {
        int Xm[3] = {x, y, z};
        Xm[a] -= 1;
        wi[(long long)(2 * a) * n_ifc + t] = X[a] < N ? edge_w(k, N, h, x, y, z, a) : 0.0;
        wi[(long long)(2 * a + 1) * n_ifc + t] = X[a] > 0 ? edge_w(k, N, h, Xm[0], Xm[1], Xm[2], a) : 0.0;
    }
}

__global__ void k_coarse_vals(int n, const int *__restrict__ pos, const int *__restrict__ col, int N, double h,
                              const double *__restrict__ k, double *__restrict__ val) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const int x = pos[3 * q], y = pos[3 * q + 1], z = pos[3 * q + 2];
    double diag = 0.0;
    for (int a = 0; a < 3; a++) {
        int Xm[3] = {x, y, z};
        Xm[a] -= 1;
        const double wp = edge_w(k, N, h, x, y, z, a);
        const double wm = edge_w(k, N, h, Xm[0], Xm[1], Xm[2], a);
        diag += wp + wm;
        val[7 * q + 1 + 2 * a] = col[7 * q + 1 + 2 * a] >= 0 ? -wp : 0.0;
        val[7 * q + 2 + 2 * a] = col[7 * q + 2 + 2 * a] >= 0 ? -wm : 0.0;
    }
    val[7 * q] = diag;
}

// Inhomogeneous Dirichlet data of eq. (1) moved to the right-hand side: an
// interior node couples only to its six axis neighbours (the other edges of a
// Kuhn simplex carry zero stiffness), so b_i = sum of w_ij g_j over those axis
// neighbours j that lie on the cube's boundary, w_ij = h for k = 1 (k null)
// and the edge weight of the coefficient otherwise.  Output in vector order.
__global__ void k_dirichlet_load(int N, double h, const double *__restrict__ k, const double *__restrict__ g,
                                 double *__restrict__ b) {
    const long long n1 = N - 1;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n1 * n1 * n1) return;
    const int P[3] = {(int)(t % n1) + 1, (int)((t / n1) % n1) + 1, (int)(t / (n1 * n1)) + 1};
    const long long M = N + 1;
    double s = 0.0;
    for (int a = 0; a < 3; a++) {
        for (int side = -1; side <= 1; side += 2) {
            int X[3] = {P[0], P[1], P[2]};
            X[a] += side;
            if (X[a] != 0 && X[a] != N) continue;
            const int *lo = side < 0 ? X : P;
            const double w = k ? edge_w(k, N, h, lo[0], lo[1], lo[2], a) : h;
            s += w * g[X[0] + M * (X[1] + M * (long long)X[2])];
        }
    }
    b[t] = s;
}

// Dirichlet-Neumann recovery (Sec. 4.3, eq. (5)): the intact side's
// sub-stencils are the stiffness assembled over the elements of intact macro
// tetrahedra only.  Fine element (cell c, permutation q) at a level with m
// segments per macro edge lies in the macro tetrahedron of macro cell c / m
// whose axis order sorts the element's centroid offsets in that macro cell.
__device__ int macro_tet_of(int cx, int cy, int cz, int q, int m, int n_sub) {
    const int C[3] = {cx / m, cy / m, cz / m};
    // centroid offsets in quarter units: 3, 2, 1 along the element's axes p0, p1, p2
    int D[3] = {4 * (cx - m * C[0]), 4 * (cy - m * C[1]), 4 * (cz - m * C[2])};
    D[kPermD[q][0]] += 3;
    D[kPermD[q][1]] += 2;
    D[kPermD[q][2]] += 1;
    const int a0 = D[0] > D[1] ? (D[0] > D[2] ? 0 : 2) : (D[1] > D[2] ? 1 : 2);
    const int a2 = D[0] < D[1] ? (D[0] < D[2] ? 0 : 2) : (D[1] < D[2] ? 1 : 2);
    const int a1 = 3 - a0 - a2;
    return 6 * (C[0] + n_sub * (C[1] + n_sub * C[2])) + perm_id(a0, a1);
}

// edge weight over intact elements: k (or 1 with k == nullptr) of each
// tetrahedron having the edge on its axis path, unless its macro
// tetrahedron is faulty
__device__ double edge_w_intact(const double *__restrict__ k, int N, double h, int x, int y, int z, int a, int m,
                                int n_sub, const unsigned char *__restrict__ faulty) {
    double sum = 0.0;
    const int P[3] = {x, y, z};
    for (int dd = 0; dd < 8; dd++) {
        const int dl[3] = {dd & 1, (dd >> 1) & 1, (dd >> 2) & 1};
        if (dl[a]) continue;
        const int c[3] = {P[0] - dl[0], P[1] - dl[1], P[2] - dl[2]};
        if (c[0] < 0 || c[1] < 0 || c[2] < 0 || c[0] >= N || c[1] >= N || c[2] >= N) continue;
        const int ns = dl[0] + dl[1] + dl[2];
        for (int q = 0; q < 6; q++) {
            bool ok = kPermD[q][ns] == a;
            for (int s = 0; s < ns; s++) ok = ok && dl[kPermD[q][s]];
            if (!ok || faulty[macro_tet_of(c[0], c[1], c[2], q, m, n_sub)]) continue;
            sum += k ? k[6LL * (c[0] + (long long)N * (c[1] + (long long)N * c[2])) + q] : 1.0;
        }
    }
    return sum * h / 6.0;
}

__global__ void k_ifc_weights_intact(int n_ifc, const int *__restrict__ xyz, int N, int m, int n_sub, double h,
                                     const double *__restrict__ k, const unsigned char *__restrict__ faulty,
                                     double *__restrict__ wi) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_ifc) return;
    const int x = xyz[3 * t], y = xyz[3 * t + 1], z = xyz[3 * t + 2];
    const int X[3] = {x, y, z};
    for (int a = 0; a < 3; a++) {
        int Xm[3] = {x, y, z};
        Xm[a] -= 1;
        wi[(long long)(2 * a) * n_ifc + t] = X[a] < N ? edge_w_intact(k, N, h, x, y, z, a, m, n_sub, faulty) : 0.0;
        wi[(long long)(2 * a + 1) * n_ifc + t] =
            X[a] > 0 ? edge_w_intact(k, N, h, Xm[0], Xm[1], Xm[2], a, m, n_sub, faulty) : 0.0;
    }
}

__global__ void k_coarse_vals_intact(int n, const int *__restrict__ pos, const int *__restrict__ col, int N, int m,
                                     int n_sub, double h, const double *__restrict__ k,
                                     const unsigned char *__restrict__ faulty, double *__restrict__ val) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const int x = pos[3 * q], y = pos[3 * q + 1], z = pos[3 * q + 2];
    double diag = 0.0;
    for (int a = 0; a < 3; a++) {
        int Xm[3] = {x, y, z};
        Xm[a] -= 1;
        const double wp = edge_w_intact(k, N, h, x, y, z, a, m, n_sub, faulty);
        const double wm = edge_w_intact(k, N, h, Xm[0], Xm[1], Xm[2], a, m, n_sub, faulty);
        diag += wp + wm;
        val[7 * q + 1 + 2 * a] = col[7 * q + 1 + 2 * a] >= 0 ? -wp : 0.0;
        val[7 * q + 2 + 2 * a] = col[7 * q + 2 + 2 * a] >= 0 ? -wm : 0.0;
    }
    val[7 * q] = diag;
}

// ---------------------------------------------------------------------------
// general macro meshes with a per-element coefficient (see GenK): the
// stiffness entry of grid nodes X and X + delta sums k_e K_e[r][r'] over the
// fine elements e holding both, K_e the matrix of e's macro tetrahedron and
// axis order at unit size, divided by m; the diagonal (delta = 0) sums over
// every element at X.  Elements outside the grid are skipped.
// ---------------------------------------------------------------------------
__device__ __constant__ int kIdx15D[15][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {-1, 1, 0}, {1, -1, 0},
                                              {0, -1, 1}, {0, 1, -1}, {0, 1, 0},  {0, -1, 0}, {-1, 0, 1},
                                              {1, 0, -1}, {1, -1, 1}, {-1, 1, -1}, {0, 0, 1}, {0, 0, -1}};
__device__ __constant__ int kGrid15D[15][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},   {0, -1, 0},
                                               {0, 0, 1},  {0, 0, -1}, {1, 1, 0},  {-1, -1, 0}, {0, 1, 1},
                                               {0, -1, -1}, {1, 0, 1}, {-1, 0, -1}, {1, 1, 1}, {-1, -1, -1}};

// offset of vertex v of an element with axis order q from its cube corner:
// 0, e_q0, e_q0 + e_q1, (1,1,1)
__device__ __forceinline__ void elem_vertex(int q, int v, int o[3]) {
    o[0] = o[1] = o[2] = 0;
    if (v >= 1) o[kPermD[q][0]] = 1;
    if (v >= 2) o[kPermD[q][1]] = 1;
    if (v >= 3) o[kPermD[q][2]] = 1;
}

__device__ double gen_entry(const GenK &G, const int X[3], int dx, int dy, int dz) {
    double s = 0.0;
    for (int q = 0; q < 6; q++)
        for (int r = 0; r < 4; r++) {
            int o[3];
            elem_vertex(q, r, o);
            const int c[3] = {X[0] - o[0], X[1] - o[1], X[2] - o[2]};
            if (c[0] < 0 || c[1] < 0 || c[2] < 0 || c[0] >= G.N || c[1] >= G.N || c[2] >= G.N) continue;
            int rr = -1;
            for (int v = 0; v < 4; v++) {
                int p[3];
                elem_vertex(q, v, p);
                if (p[0] - o[0] == dx && p[1] - o[1] == dy && p[2] - o[2] == dz) rr = v;
            }
            if (rr < 0) continue;
            const long long e = 6 * (c[0] + (long long)G.N * (c[1] + (long long)G.N * c[2])) + q;
            const int t = macro_tet_of(c[0], c[1], c[2], q, G.m, G.n_sub);
            if (G.faulty && G.faulty[t]) continue;
            s += (G.k ? G.k[e] : 1.0) * G.kel[(6LL * t + q) * 16 + 4 * r + rr];
        }
    return s / G.m;
}

// grid position of node (i,j,k) of tetrahedron t and the grid step of its
// index offset n
__device__ __forceinline__ void tet_grid(const int *__restrict__ tetinfo, int t, int m, int i, int j, int k, int X[3]) {
    for (int a = 0; a < 3; a++) X[a] = m * tetinfo[6 * t + a];
    X[tetinfo[6 * t + 3]] += i + j + k;
    X[tetinfo[6 * t + 4]] += j + k;
    X[tetinfo[6 * t + 5]] += k;
}
__device__ __forceinline__ void tet_step(const int *__restrict__ tetinfo, int t, int n, int g[3]) {
    g[0] = g[1] = g[2] = 0;
    g[tetinfo[6 * t + 3]] += kIdx15D[n][0] + kIdx15D[n][1] + kIdx15D[n][2];
    g[tetinfo[6 * t + 4]] += kIdx15D[n][1] + kIdx15D[n][2];
    g[tetinfo[6 * t + 5]] += kIdx15D[n][2];
}

// dJ/dk_e = -lambda_e^T K_e u_e for every element e of the level (element
// order), K_e its unit-coefficient matrix (kel / m); u and lambda in vector
// order, zero on the boundary
__global__ void k_grad_k15(int N, int m, int n_sub, const double *__restrict__ kel, const double *__restrict__ u,
                           const double *__restrict__ lam, double *__restrict__ out) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long ne = 6LL * N * N * N;
    if (e >= ne) return;
    const int q = (int)(e % 6);
    const long long cell = e / 6;
    const int c[3] = {(int)(cell % N), (int)((cell / N) % N), (int)(cell / ((long long)N * N))};
    const long long n1 = N - 1;
    double ul[4], ll[4];
    for (int v = 0; v < 4; v++) {
        int o[3];
        elem_vertex(q, v, o);
        const int X[3] = {c[0] + o[0], c[1] + o[1], c[2] + o[2]};
        const bool in = X[0] > 0 && X[1] > 0 && X[2] > 0 && X[0] < N && X[1] < N && X[2] < N;
        const long long d = (X[0] - 1) + n1 * ((X[1] - 1) + n1 * (X[2] - 1));
        ul[v] = in ? u[d] : 0.0;
        ll[v] = in ? lam[d] : 0.0;
    }
    const double *K = kel + (6LL * macro_tet_of(c[0], c[1], c[2], q, m, n_sub) + q) * 16;
    double g = 0.0;
    for (int a = 0; a < 4; a++)
        for (int b = 0; b < 4; b++) g += ll[a] * K[4 * a + b] * ul[b];
    out[e] = -g / m;
}

// every closure node (vg lists the full closure): the 7 forward edge weights
// of the edges that stay in the closure (0 otherwise) and the diagonal
__global__ void __launch_bounds__(256) k_gen_weights(VolGeom vg, const int *__restrict__ tetinfo, GenK G,
                                                     double *__restrict__ wv, long long ws) {
    const unsigned per_vol = list_blocks_per_vol<1>(vg);
    LNode nd;
    if (!list_node<1>(vg, blockIdx.x, per_vol, 0, nd)) return;
    const VolDesc d = vg.vd[nd.v];
    const int m = vg.M - 1;
    int X[3];
    tet_grid(tetinfo, d.tet, m, nd.i, nd.j, nd.k, X);
    const long long sl = d.w + lslot(vg.rowC, vg.M, nd.i, nd.j, nd.k);
    for (int e = 0; e < 7; e++) {
        const int n = 2 * e + 1;
        const int i2 = nd.i + kIdx15D[n][0], j2 = nd.j + kIdx15D[n][1], k2 = nd.k + kIdx15D[n][2];
        double w = 0.0;
        if (i2 >= 0 && j2 >= 0 && k2 >= 0 && i2 + j2 + k2 <= m) {
            int g[3];
            tet_step(tetinfo, d.tet, n, g);
            w = gen_entry(G, X, g[0], g[1], g[2]);
        }
        wv[e * ws + sl] = w;
    }
    wv[7 * ws + sl] = gen_entry(G, X, 0, 0, 0);
}

__global__ void k_gen_ifc_weights(int n_ifc, const int *__restrict__ xyz, GenK G, double *__restrict__ wi15) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= n_ifc) return;
    const int X[3] = {xyz[3 * f], xyz[3 * f + 1], xyz[3 * f + 2]};
    for (int n = 0; n < 15; n++)
        wi15[(long long)n * n_ifc + f] = gen_entry(G, X, kGrid15D[n][0], kGrid15D[n][1], kGrid15D[n][2]);
}

__global__ void k_gen_coarse_vals(int n, const int *__restrict__ pos, const int *__restrict__ col15, GenK G,
                                  double *__restrict__ val) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const int X[3] = {pos[3 * q], pos[3 * q + 1], pos[3 * q + 2]};
    for (int e = 0; e < 15; e++)
        val[15 * q + e] = e == 0 || col15[15 * q + e] >= 0
                              ? gen_entry(G, X, kGrid15D[e][0], kGrid15D[e][1], kGrid15D[e][2])
                              : 0.0;
}

// eliminated Dirichlet data on a general macro mesh: b = -sum over the
// boundary neighbours j of A_ij g_j at every interior node and master
// (g on the full (N+1)^3 grid, x fastest)
template <bool VK>
__global__ void __launch_bounds__(256) k_gen_dirichlet(VolGeom vg, IfcGeom ig, Gen15 g, int nib,
                                                       const int *__restrict__ tetinfo, const int *__restrict__ ifc_xyz,
                                                       int N, const double *__restrict__ gfull, double *__restrict__ b) {
    const long long M1 = N + 1;
    auto on_bnd = [&](const int *Y) {
        return Y[0] == 0 || Y[1] == 0 || Y[2] == 0 || Y[0] == N || Y[1] == N || Y[2] == N;
    };
    const unsigned f = blockIdx.x;
    if (f < (unsigned)nib) {
        const int t = (int)(f * blockDim.x + threadIdx.x);
        if (t >= ig.i1) return;
        const int X[3] = {ifc_xyz[3 * t], ifc_xyz[3 * t + 1], ifc_xyz[3 * t + 2]};
        const double *w = g.wi15 ? nullptr : g.wtab + 15LL * g.sid[t];
        double s = 0.0;
        for (int n = 1; n < 15; n++) {
            const int Y[3] = {X[0] + kGrid15D[n][0], X[1] + kGrid15D[n][1], X[2] + kGrid15D[n][2]};
            if (!on_bnd(Y)) continue;
            const double a = g.wi15 ? g.wi15[(long long)n * ig.stride + t] : w[n];
            s -= a * gfull[Y[0] + M1 * (Y[1] + M1 * Y[2])];
        }
        b[ig.base + t] = s;
        return;
    }
    const unsigned per_vol = list_blocks_per_vol<1>(vg);
    LNode nd;
    if (!list_node<1>(vg, f - nib, per_vol, 0, nd)) return;
    const VolDesc d = vg.vd[nd.v];
    const int m = vg.M - 1;
    int X[3];
    tet_grid(tetinfo, d.tet, m, nd.i, nd.j, nd.k, X);
    const long long c0 = lslot(vg.rowC, vg.M, nd.i, nd.j, nd.k);
    double s = 0.0;
    for (int n = 1; n < 15; n++) {
        int gs[3];
        tet_step(tetinfo, d.tet, n, gs);
        const int Y[3] = {X[0] + gs[0], X[1] + gs[1], X[2] + gs[2]};
        if (!on_bnd(Y)) continue;
        double a;
        if (VK) {
            const int e = (n - 1) >> 1;
            const long long sn =
                lslot(vg.rowC, vg.M, nd.i + kIdx15D[n][0], nd.j + kIdx15D[n][1], nd.k + kIdx15D[n][2]);
            a = (n & 1) ? g.wv[e * g.ws + d.w + c0] : g.wv[e * g.ws + d.w + sn];
        } else {
            a = g.w15[15LL * d.tet + n];
        }
        s -= a * gfull[Y[0] + M1 * (Y[1] + M1 * Y[2])];
    }
    b[d.vec + c0] = s;
}

// static Neumann data of the intact side on the interface (Alg. 2): at the
// nodes flagged in gamma, b_out = (A^I u) from the intact-side weights wi
__global__ void k_neumann_rhs(int n_ifc, long long base, const int *__restrict__ nbr, const double *__restrict__ wi,
                              const unsigned char *__restrict__ gamma, const double *__restrict__ u,
                              double *__restrict__ b_out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_ifc || !gamma[t]) return;
    const long long sl = base + t;
    const double uo = u[sl];
    double s = 0.0;
#pragma unroll
    for (int e = 0; e < 6; e++) s += wi[(long long)e * n_ifc + t] * (uo - u[nbr[(long long)e * n_ifc + t]]);
    b_out[sl] = s;
}

// the same on a general macro mesh: b_out = (A^I u) at the nodes of gamma
// with the intact side's 15 entries per master (kGrid15 order, entry 0 the
// diagonal at the master's own slot)
__global__ void k_neumann_rhs15(int n_ifc, long long base, const int *__restrict__ nb15,
                                const double *__restrict__ wi15, const unsigned char *__restrict__ gamma,
                                const double *__restrict__ u, double *__restrict__ b_out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_ifc || !gamma[t]) return;
    double s = 0.0;
#pragma unroll
    for (int e = 0; e < 15; e++) s += wi15[(long long)e * n_ifc + t] * u[nb15[(long long)e * n_ifc + t]];
    b_out[base + t] = s;
}

// Interface masks of a Dirichlet-Neumann recovery: a node whose ghost copies
// all lie in faulty closures is frozen, one with copies on both sides is on
// Gamma (gamma may be null).  The intact side's ghost list keeps the layout of
// the full list; a copy in a faulty closure is replaced by the master's own
// slot, so the scatter rewrites the master with the value it just stored.
__global__ void k_dn_masks(int n_ifc, long long base, long long C_pad, const int *__restrict__ gptr,
                           const int *__restrict__ gidx, const unsigned char *__restrict__ faulty,
                           unsigned char *__restrict__ frozen, unsigned char *__restrict__ gamma,
                           int *__restrict__ gidx_dn) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_ifc) return;
    int nf = 0, ni = 0;
    for (int g = gptr[t]; g < gptr[t + 1]; g++) {
        const int sl = gidx[g];
        if (faulty[sl / C_pad]) {
            nf++;
            gidx_dn[g] = (int)(base + t);
        } else {
            ni++;
            gidx_dn[g] = sl;
        }
    }
    frozen[t] = ni == 0;
    if (gamma) gamma[t] = nf > 0 && ni > 0;
}

// dJ/dk_T = -(h/6) sum over the 3 path edges (a,b) of T of (lam_a - lam_b)(u_a - u_b)
__global__ void k_grad_k(const double *__restrict__ u, const double *__restrict__ lam, int N, double h,
                         double *__restrict__ out) {
    const long long cell = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (cell >= (long long)N * N * N) return;
    const int cx = (int)(cell % N), cy = (int)((cell / N) % N), cz = (int)(cell / ((long long)N * N));
    double uc[8], lc[8];
    for (int d = 0; d < 8; d++) {
        const int x = cx + (d & 1), y = cy + ((d >> 1) & 1), z = cz + ((d >> 2) & 1);
        const bool in = x > 0 && y > 0 && z > 0 && x < N && y < N && z < N;
        const long long dof = (long long)(x - 1) + (long long)(N - 1) * ((y - 1) + (long long)(N - 1) * (z - 1));
        uc[d] = in ? u[dof] : 0.0;
        lc[d] = in ? lam[dof] : 0.0;
    }
    for (int q = 0; q < 6; q++) {
        int v = 0;
        double g = 0.0;
        for (int s = 0; s < 3; s++) {
            const int w = v | (1 << kPermD[q][s]);
            g += (lc[v] - lc[w]) * (uc[v] - uc[w]);
            v = w;
        }
        out[6 * cell + q] = -(h / 6.0) * g;
    }
}

// workgroups of a list-mode launch
inline long long list_blocks(const VolGeom &g, int cpb) {
    const long long per = ((long long)g.nlist + (long long)g.bs * cpb - 1) / ((long long)g.bs * cpb);
    return per * g.nvol;
}
inline long long list_blocks(const VolGeom &g) { return list_blocks(g, g.cpb); }

inline unsigned grid1d(long long n, int bs) {
    long long g = (n + bs - 1) / bs;
    if (g > 65535LL * 32) g = 65535LL * 32;
    return (unsigned)(g > 0 ? g : 1);
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename T>
void launch_colour(hipStream_t s, const VolGeom &vg, const IfcGeom &ig, T *u, const T *b, const Weights<T> &w, bool vk,
                   double h, double omega, bool own0, bool nb0) {
    const int nib = ifc_blocks(ig, vg.bs);
    const long long nvb = list_blocks(vg);
    const long long grid = nib + nvb;
    if (grid == 0) return;
    const T th = (T)h, to = (T)omega, tod = (T)(omega / (6.0 * h));
    const Prol<T> p;
    double *const np = nullptr;
    T *const nr = nullptr;
#define HHGR_COLOUR(VK, O0, N0)                                                                                 \
    do {                                                                                                       \
        if (vg.cpb == 1)                                                                                       \
            hipLaunchKernelGGL((k_colour<T, VK, O0, N0, false, kTailNone, 1>), dim3((unsigned)grid), dim3(vg.bs), 0, s, \
                               vg, ig, nib, u, b, w, th, to, tod, p, np, nr);                                 \
        else                                                                                                   \
            hipLaunchKernelGGL((k_colour<T, VK, O0, N0, false, kTailNone, 4>), dim3((unsigned)grid), dim3(vg.bs), 0, s, \
                               vg, ig, nib, u, b, w, th, to, tod, p, np, nr);                                 \
    } while (0)
    if (vk) {
        if (own0 && nb0) HHGR_COLOUR(true, true, true);
        else if (own0) HHGR_COLOUR(true, true, false);
        else HHGR_COLOUR(true, false, false);
    } else {
        if (own0 && nb0) HHGR_COLOUR(false, true, true);
        else if (own0) HHGR_COLOUR(false, true, false);
        else HHGR_COLOUR(false, false, false);
    }
#undef HHGR_COLOUR
}

template <typename T>
void launch_colour_prol(hipStream_t s, const VolGeom &vg, const IfcGeom &ig, T *u, const T *b, const Weights<T> &w,
                        bool vk, double h, double omega, const Prol<T> &p) {
    const int nib = ifc_blocks(ig, vg.bs);
    const long long nvb = list_blocks(vg);
    const long long grid = nib + nvb;
    if (grid == 0) return;
    const T th = (T)h, to = (T)omega, tod = (T)(omega / (6.0 * h));
    double *const np = nullptr;
    T *const nr = nullptr;
#define HHGR_COLOUR_PR(VK)                                                                                      \
    do {                                                                                                       \
        if (vg.cpb == 1)                                                                                       \
            hipLaunchKernelGGL((k_colour<T, VK, false, false, true, kTailNone, 1>), dim3((unsigned)grid), dim3(vg.bs), 0, \
                               s, vg, ig, nib, u, b, w, th, to, tod, p, np, nr);                              \
        else                                                                                                   \
            hipLaunchKernelGGL((k_colour<T, VK, false, false, true, kTailNone, 4>), dim3((unsigned)grid), dim3(vg.bs), 0, \
                               s, vg, ig, nib, u, b, w, th, to, tod, p, np, nr);                              \
    } while (0)
    if (vk)
        HHGR_COLOUR_PR(true);
    else
        HHGR_COLOUR_PR(false);
#undef HHGR_COLOUR_PR
}

int colour_blocks(const VolGeom &vg, const IfcGeom &ig) { return ifc_blocks(ig, vg.bs) + (int)list_blocks(vg); }

int launch_colour_norm(hipStream_t s, const VolGeom &vg, const IfcGeom &ig, double *u, const double *b,
                       const Weights<double> &w, bool vk, double h, double omega, double *partial) {
    const int nib = ifc_blocks(ig, vg.bs);
    const long long nvb = list_blocks(vg);
    const long long grid = nib + nvb;
    if (grid == 0) return 0;
    const Prol<double> p;
    const double tod = omega / (6.0 * h);
    double *const nr = nullptr;
#define HHGR_COLOUR_NRM(VK)                                                                                     \
    do {                                                                                                       \
        if (vg.cpb == 1)                                                                                       \
            hipLaunchKernelGGL((k_colour<double, VK, false, false, false, kTailNorm, 1>), dim3((unsigned)grid),      \
                               dim3(vg.bs), 0, s, vg, ig, nib, u, b, w, h, omega, tod, p, partial, nr);       \
        else                                                                                                   \
            hipLaunchKernelGGL((k_colour<double, VK, false, false, false, kTailNorm, 4>), dim3((unsigned)grid),      \
                               dim3(vg.bs), 0, s, vg, ig, nib, u, b, w, h, omega, tod, p, partial, nr);       \
    } while (0)
    if (vk)
        HHGR_COLOUR_NRM(true);
    else
        HHGR_COLOUR_NRM(false);
#undef HHGR_COLOUR_NRM
    return (int)grid;
}

template <typename T>
void launch_colour_res(hipStream_t s, const VolGeom &vg, const IfcGeom &ig, T *u, const T *b, const Weights<T> &w,
                       bool vk, double h, double omega, T *r) {
    const int nib = ifc_blocks(ig, vg.bs);
    const long long nvb = list_blocks(vg);
    const long long grid = nib + nvb;
    if (grid == 0) return;
    const T th = (T)h, to = (T)omega, tod = (T)(omega / (6.0 * h));
    const Prol<T> p;
    double *const np = nullptr;
#define HHGR_COLOUR_RES(VK)                                                                                     \
    do {                                                                                                       \
        if (vg.cpb == 1)                                                                                       \
            hipLaunchKernelGGL((k_colour<T, VK, false, false, false, kTailRes, 1>), dim3((unsigned)grid), dim3(vg.bs), 0, \
                               s, vg, ig, nib, u, b, w, th, to, tod, p, np, r);                               \
        else                                                                                                   \
            hipLaunchKernelGGL((k_colour<T, VK, false, false, false, kTailRes, 4>), dim3((unsigned)grid), dim3(vg.bs), 0, \
                               s, vg, ig, nib, u, b, w, th, to, tod, p, np, r);                               \
    } while (0)
    if (vk)
        HHGR_COLOUR_RES(true);
    else
        HHGR_COLOUR_RES(false);
#undef HHGR_COLOUR_RES
}

template <typename T, typename TO>
int launch_residual(hipStream_t s, const VolGeom &vg, const IfcGeom &ig, const T *u, const T *b, const Weights<T> &w,
                    bool vk, double h, TO *r, double *partial) {
    const int nib = ifc_blocks(ig, vg.bs);
    const long long nvb = list_blocks(vg);
    const long long grid = nib + nvb;
    if (grid == 0) return 0;
    const T th = (T)h;
#define HHGR_RES(VK, WR, NO)                                                                                   \
    do {                                                                                                       \
        if (vg.cpb == 1)                                                                                       \
            hipLaunchKernelGGL((k_residual<T, TO, VK, WR, NO, 1>), dim3((unsigned)grid), dim3(vg.bs), 0, s, vg, ig, nib, \
                               u, b, w, th, r, partial);                                                      \
        else                                                                                                   \
            hipLaunchKernelGGL((k_residual<T, TO, VK, WR, NO, 4>), dim3((unsigned)grid), dim3(vg.bs), 0, s, vg, ig, nib, \
                               u, b, w, th, r, partial);                                                      \
    } while (0)
    const bool wr = r != nullptr, no = partial != nullptr;
    if (vk) {
        if (wr && no) HHGR_RES(true, true, true);
        else if (wr) HHGR_RES(true, true, false);
        else HHGR_RES(true, false, true);
    } else {
        if (wr && no) HHGR_RES(false, true, true);
        else if (wr) HHGR_RES(false, true, false);
        else HHGR_RES(false, false, true);
    }
#undef HHGR_RES
    return (int)grid;
}

template <typename T>
void launch_restrict(hipStream_t s, const VolGeom &vc, const VolDesc *vdf, const int2 *fC, const IfcGeom &igc,
                     const int *rst, const T *rf, T *bc) {
    const int nib = ifc_blocks(igc, vc.bs);
    const long long grid = nib + list_blocks(vc);
    if (grid == 0) return;
    if (vc.cpb == 1)
        hipLaunchKernelGGL((k_restrict<T, 1>), dim3((unsigned)grid), dim3(vc.bs), 0, s, vc, vdf, fC, igc, nib, rst, rf, bc);
    else
        hipLaunchKernelGGL((k_restrict<T, 4>), dim3((unsigned)grid), dim3(vc.bs), 0, s, vc, vdf, fC, igc, nib, rst, rf, bc);
}

template <typename T>
void launch_prolong(hipStream_t s, const VolGeom &vf, const VolDesc *vdc, const int2 *cC, int Mc, const IfcGeom &igf,
                    const int *prl, const T *ec, T *uf) {
    const int nib = ifc_blocks(igf, vf.bs);
    const long long grid = nib + list_blocks(vf);
    if (grid == 0) return;
    if (vf.cpb == 1)
        hipLaunchKernelGGL((k_prolong<T, 1>), dim3((unsigned)grid), dim3(vf.bs), 0, s, vf, vdc, cC, Mc, igf, nib, prl, ec,
                           uf);
    else
        hipLaunchKernelGGL((k_prolong<T, 4>), dim3((unsigned)grid), dim3(vf.bs), 0, s, vf, vdc, cC, Mc, igf, nib, prl, ec,
                           uf);
}

template <typename T>
void launch_coarse_pcg(hipStream_t s, int n, const long long *slot, const int *col, const double *val,
                       const unsigned char *frozen, const T *b, T *u, const int *cptr, const int *cidx, double rtol,
                       int maxit, int *iters) {
    // up to 512 unknowns in a single wavefront; otherwise one unknown per
    // thread in as few waves as possible (cheaper barriers)
    if (n <= 64) {
        hipLaunchKernelGGL((k_coarse_pcg_wave<T, 1>), dim3(1), dim3(64), 0, s, n, slot, col, val, frozen, b, u, cptr,
                           cidx, rtol, maxit, iters);
    } else if (n <= 128) {
        hipLaunchKernelGGL((k_coarse_pcg_wave<T, 2>), dim3(1), dim3(64), 0, s, n, slot, col, val, frozen, b, u, cptr,
                           cidx, rtol, maxit, iters);
    } else if (n <= 256) {
        hipLaunchKernelGGL((k_coarse_pcg_wave<T, 4>), dim3(1), dim3(64), 0, s, n, slot, col, val, frozen, b, u, cptr,
                           cidx, rtol, maxit, iters);
    } else if (n <= 512) {
        hipLaunchKernelGGL((k_coarse_pcg_wave<T, 8>), dim3(1), dim3(64), 0, s, n, slot, col, val, frozen, b, u, cptr,
                           cidx, rtol, maxit, iters);
    } else if (n <= 1024) {
        const int bs = n <= 64 ? 64 : n <= 128 ? 128 : n <= 256 ? 256 : n <= 512 ? 512 : 1024;
        hipLaunchKernelGGL((k_coarse_pcg<T, 1>), dim3(1), dim3(bs), 0, s, n, slot, col, val, frozen, b, u, cptr, cidx,
                           rtol, maxit, iters);
    } else {
        hipLaunchKernelGGL((k_coarse_pcg<T, 2>), dim3(1), dim3(1024), 0, s, n, slot, col, val, frozen, b, u, cptr, cidx,
                           rtol, maxit, iters);
    }
}

template <typename T>
void launch_coarse_dense(hipStream_t s, int n, const long long *slot, const double *inv, const T *b, T *u,
                         const int *cptr, const int *cidx) {
    if (n <= 0) return;
    hipLaunchKernelGGL((k_coarse_dense<T>), dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, n, slot, inv, b, u, cptr,
                       cidx);
}

template <typename T>
void launch_local_coarse(hipStream_t s, const VolDesc *vd, int nvol, int4 sl, const T *b, T *u, const Weights<T> &w,
                         bool vk, double h) {
    if (nvol <= 0) return;
    const unsigned g = (unsigned)((nvol + 63) / 64);
    if (vk)
        hipLaunchKernelGGL((k_local_coarse<T, true>), dim3(g), dim3(64), 0, s, vd, nvol, sl, b, u, w, (T)h);
    else
        hipLaunchKernelGGL((k_local_coarse<T, false>), dim3(g), dim3(64), 0, s, vd, nvol, sl, b, u, w, (T)h);
}

void launch_reduce(hipStream_t s, const double *partial, int n, double *out) {
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(1024), 0, s, partial, n, out);
}

template <typename T>
void launch_fill(hipStream_t s, T *p, long long n, T v) {
    if (n <= 0) return;
    hipLaunchKernelGGL((k_fill<T>), dim3(grid1d(n, 256)), dim3(256), 0, s, p, n, v);
}

template <typename T>
void launch_user_to_slots(hipStream_t s, const VolGeom &vfull, const int *tetinfo, int m, int N, const IfcGeom &ig,
                          const int *ifc_dof, const double *user, T *vec) {
    const int nib = ifc_blocks(ig, vfull.bs);
    const long long grid = nib + list_blocks(vfull, 1);
    if (grid == 0) return;
    hipLaunchKernelGGL((k_user_to_slots<T>), dim3((unsigned)grid), dim3(vfull.bs), 0, s, vfull, tetinfo, m, N, ig, nib,
                       ifc_dof, user, vec);
}

template <typename T>
void launch_slots_to_user(hipStream_t s, const VolGeom &vint, const int *tetinfo, int m, int N, const IfcGeom &ig,
                          const int *ifc_dof, const T *vec, double *user) {
    const int nib = ifc_blocks(ig, vint.bs);
    const long long grid = nib + list_blocks(vint);
    if (grid == 0) return;
    if (vint.cpb == 1)
        hipLaunchKernelGGL((k_slots_to_user<T, 1>), dim3((unsigned)grid), dim3(vint.bs), 0, s, vint, tetinfo, m, N, ig,
                           nib, ifc_dof, vec, user);
    else
        hipLaunchKernelGGL((k_slots_to_user<T, 4>), dim3((unsigned)grid), dim3(vint.bs), 0, s, vint, tetinfo, m, N, ig,
                           nib, ifc_dof, vec, user);
}

template <typename T>
void launch_mesh_user_to_slots(hipStream_t s, const VolGeom &vint, long long vbase, long long nint, const IfcGeom &ig,
                               const int *ifc_dof, const double *user, T *vec) {
    const int nib = ifc_blocks(ig, vint.bs);
    const long long grid = nib + list_blocks(vint, 1);
    if (grid == 0) return;
    hipLaunchKernelGGL((k_mesh_user_to_slots<T>), dim3((unsigned)grid), dim3(vint.bs), 0, s, vint, vbase, nint, ig,
                       nib, ifc_dof, user, vec);
}

template <typename T>
void launch_mesh_slots_to_user(hipStream_t s, const VolGeom &vint, long long vbase, long long nint, const IfcGeom &ig,
                               const int *ifc_dof, const T *vec, double *user) {
    const int nib = ifc_blocks(ig, vint.bs);
    const long long grid = nib + list_blocks(vint, 1);
    if (grid == 0) return;
    hipLaunchKernelGGL((k_mesh_slots_to_user<T>), dim3((unsigned)grid), dim3(vint.bs), 0, s, vint, vbase, nint, ig,
                       nib, ifc_dof, vec, user);
}

template void launch_mesh_user_to_slots<double>(hipStream_t, const VolGeom &, long long, long long, const IfcGeom &,
                                                const int *, const double *, double *);
template void launch_mesh_slots_to_user<double>(hipStream_t, const VolGeom &, long long, long long, const IfcGeom &,
                                                const int *, const double *, double *);

void launch_mass(hipStream_t s, const VolGeom &vint, const IfcGeom &ig, const int *nb15, const double *x, double *y,
                 double h) {
    const int nib = ifc_blocks(ig, vint.bs);
    const long long grid = nib + list_blocks(vint);
    if (grid == 0) return;
    if (vint.cpb == 1)
        hipLaunchKernelGGL(k_mass<1>, dim3((unsigned)grid), dim3(vint.bs), 0, s, vint, ig, nib, nb15, x, y, h * h * h);
    else
        hipLaunchKernelGGL(k_mass<4>, dim3((unsigned)grid), dim3(vint.bs), 0, s, vint, ig, nib, nb15, x, y, h * h * h);
}

void launch_mass_grid(hipStream_t s, int N, double h, const double *f, double *b) {
    const long long n = (long long)(N - 1) * (N - 1) * (N - 1);
    if (n <= 0) return;
    hipLaunchKernelGGL(k_mass_grid, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, N, h * h * h, f, b);
}

int launch_norm2(hipStream_t s, const VolGeom &vg, const IfcGeom &ig, const double *v, double *partial) {
    VolGeom g = vg;
    g.cpb = 4;
    const int nib = ifc_blocks(ig, g.bs);
    const long long grid = nib + list_blocks(g);
    if (grid == 0) return 0;
    hipLaunchKernelGGL(k_norm2<4>, dim3((unsigned)grid), dim3(g.bs), 0, s, g, ig, nib, v, partial);
    return (int)grid;
}

void launch_update_add(hipStream_t s, const VolDesc *vd, int nvol, long long span, const IfcGeom &ig, double *u,
                       const float *e) {
    const int nib = ifc_blocks(ig, 256);
    const long long grid = nib + (long long)nvol * ((span + 1023) / 1024);
    if (grid == 0) return;
    hipLaunchKernelGGL(k_update_add, dim3((unsigned)grid), dim3(256), 0, s, vd, span, ig, nib, u, e);
}

template <typename T>
void launch_ghost_refresh(hipStream_t s, const int *dst, const int *src, int n, T *u) {
    if (n <= 0) return;
    hipLaunchKernelGGL((k_ghost_refresh<T>), dim3((n + 255) / 256), dim3(256), 0, s, dst, src, n, u);
}

template <typename TI, typename TO>
void launch_cast(hipStream_t s, const TI *in, TO *out, long long n) {
    if (n <= 0) return;
    hipLaunchKernelGGL((k_cast<TI, TO>), dim3(grid1d(n, 256)), dim3(256), 0, s, in, out, n);
}

void launch_coarsen_k(hipStream_t s, const double *kf, int Nf, double *kc, int Nc) {
    const long long ne = 6LL * Nc * Nc * Nc;
    hipLaunchKernelGGL(k_coarsen_k, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, s, kf, Nf, kc, Nc);
}

void launch_vol_weights(hipStream_t s, const VolGeom &vfull, const int *tetinfo, int m, int N, double h,
                        const double *k, double *w0, double *w1, double *w2) {
    const long long grid = list_blocks(vfull, 1);
    if (grid == 0) return;
    hipLaunchKernelGGL(k_vol_weights, dim3((unsigned)grid), dim3(vfull.bs), 0, s, vfull, tetinfo, m, N, h, k, w0, w1,
                       w2);
}

void launch_ifc_weights(hipStream_t s, int n_ifc, const int *ifc_xyz, int N, double h, const double *k, double *wi) {
    if (n_ifc <= 0) return;
    hipLaunchKernelGGL(k_ifc_weights, dim3((n_ifc + 255) / 256), dim3(256), 0, s, n_ifc, ifc_xyz, N, h, k, wi);
}

int colour15_blocks(const VolGeom &vg, const Gen15 &g) {
    const int nib = g.nq > 0 ? (((g.nq + vg.bs - 1) / vg.bs + 7) & ~7) : 0;
    return nib + (int)list_blocks(vg, 1);
}

template <typename T, int TAIL>
static int colour15_tail(hipStream_t s, const VolGeom &vg, const IfcGeom &ig, const Gen15 &g, T *u, const T *b,
                         double omega, double *partial, T *r) {
    const int nib = g.nq > 0 ? (((g.nq + vg.bs - 1) / vg.bs + 7) & ~7) : 0;
    const long long grid = nib + list_blocks(vg, 1);
    if (grid == 0) return 0;
    const dim3 gd((unsigned)grid), bd(vg.bs);
    if (g.wv)
        hipLaunchKernelGGL((k_colour15<T, true, true, TAIL>), gd, bd, 0, s, vg, ig, g, nib, u, b, (T)omega, partial, r);
    else if (g.wi15)
        hipLaunchKernelGGL((k_colour15<T, false, true, TAIL>), gd, bd, 0, s, vg, ig, g, nib, u, b, (T)omega, partial, r);
    else
        hipLaunchKernelGGL((k_colour15<T, false, false, TAIL>), gd, bd, 0, s, vg, ig, g, nib, u, b, (T)omega, partial, r);
    return (int)grid;
}

template <typename T>
void launch_colour15(hipStream_t s, const VolGeom &vg, const IfcGeom &ig, const Gen15 &g, T *u, const T *b,
                     double omega) {
    colour15_tail<T, kTailNone>(s, vg, ig, g, u, b, omega, nullptr, nullptr);
}

int launch_colour15_norm(hipStream_t s, const VolGeom &vg, const IfcGeom &ig, const Gen15 &g, double *u,
                         const double *b, double omega, double *partial) {
    return colour15_tail<double, kTailNorm>(s, vg, ig, g, u, b, omega, partial, nullptr);
}

template <typename T>
void launch_colour15_res(hipStream_t s, const VolGeom &vg, const IfcGeom &ig, const Gen15 &g, T *u, const T *b,
                         double omega, T *r) {
    colour15_tail<T, kTailRes>(s, vg, ig, g, u, b, omega, nullptr, r);
}

template <typename T, typename TO, bool VKV, bool VKI>
static void residual15(hipStream_t s, dim3 gd, dim3 bd, const VolGeom &vg, const IfcGeom &ig, const Gen15 &g, int nib,
                       const T *u, const T *b, TO *r, double *partial) {
    if (r && partial)
        hipLaunchKernelGGL((k_residual15<T, TO, true, true, VKV, VKI>), gd, bd, 0, s, vg, ig, g, nib, u, b, r, partial);
    else if (r)
        hipLaunchKernelGGL((k_residual15<T, TO, true, false, VKV, VKI>), gd, bd, 0, s, vg, ig, g, nib, u, b, r, partial);
    else
        hipLaunchKernelGGL((k_residual15<T, TO, false, true, VKV, VKI>), gd, bd, 0, s, vg, ig, g, nib, u, b, r, partial);
}

template <typename T, typename TO>
int launch_residual15(hipStream_t s, const VolGeom &vg, const IfcGeom &ig, const Gen15 &g, const T *u, const T *b,
                      TO *r, double *partial) {
    const int nib = g.ifcq ? (g.nq > 0 ? (((g.nq + vg.bs - 1) / vg.bs + 7) & ~7) : 0) : ifc_blocks(ig, vg.bs);
    const long long grid = nib + list_blocks(vg, 1);
    if (grid == 0) return 0;
    const dim3 gd((unsigned)grid), bd(vg.bs);
    if (g.wv)
        residual15<T, TO, true, true>(s, gd, bd, vg, ig, g, nib, u, b, r, partial);
    else if (g.wi15)
        residual15<T, TO, false, true>(s, gd, bd, vg, ig, g, nib, u, b, r, partial);
    else
        residual15<T, TO, false, false>(s, gd, bd, vg, ig, g, nib, u, b, r, partial);
    return (int)grid;
}

template void launch_colour15<double>(hipStream_t, const VolGeom &, const IfcGeom &, const Gen15 &, double *,
                                      const double *, double);
template void launch_colour15<float>(hipStream_t, const VolGeom &, const IfcGeom &, const Gen15 &, float *,
                                     const float *, double);
template void launch_colour15_res<double>(hipStream_t, const VolGeom &, const IfcGeom &, const Gen15 &, double *,
                                          const double *, double, double *);
template void launch_colour15_res<float>(hipStream_t, const VolGeom &, const IfcGeom &, const Gen15 &, float *,
                                         const float *, double, float *);
template int launch_residual15<double, double>(hipStream_t, const VolGeom &, const IfcGeom &, const Gen15 &,
                                               const double *, const double *, double *, double *);
template int launch_residual15<double, float>(hipStream_t, const VolGeom &, const IfcGeom &, const Gen15 &,
                                              const double *, const double *, float *, double *);
template int launch_residual15<float, float>(hipStream_t, const VolGeom &, const IfcGeom &, const Gen15 &,
                                             const float *, const float *, float *, double *);

template <typename T>
void launch_coarse_pcg15(hipStream_t s, int n, const long long *slot, const int *col, const double *val,
                         const unsigned char *frozen, const T *b, T *u, const int *cptr, const int *cidx,
                         double rtol, int maxit, int *iters) {
    // 14 off-diagonal entries per row stay in registers: at most 2 rows per
    // lane (more spill to scratch), so above 128 unknowns one row per thread
    if (n <= 64)
        hipLaunchKernelGGL((k_coarse_pcg_wave<T, 1, 14>), dim3(1), dim3(64), 0, s, n, slot, col, val, frozen, b, u, cptr,
                           cidx, rtol, maxit, iters);
    else if (n <= 128)
        hipLaunchKernelGGL((k_coarse_pcg_wave<T, 2, 14>), dim3(1), dim3(64), 0, s, n, slot, col, val, frozen, b, u, cptr,
                           cidx, rtol, maxit, iters);
    else if (n <= 1024) {
        const int bs = n <= 256 ? 256 : n <= 512 ? 512 : 1024;
        hipLaunchKernelGGL((k_coarse_pcg<T, 1, 14>), dim3(1), dim3(bs), 0, s, n, slot, col, val, frozen, b, u, cptr, cidx,
                           rtol, maxit, iters);
    } else
        hipLaunchKernelGGL((k_coarse_pcg<T, 2, 14>), dim3(1), dim3(1024), 0, s, n, slot, col, val, frozen, b, u, cptr,
                           cidx, rtol, maxit, iters);
}

template void launch_coarse_pcg15<double>(hipStream_t, int, const long long *, const int *, const double *,
                                          const unsigned char *, const double *, double *, const int *, const int *,
                                          double, int, int *);
template void launch_coarse_pcg15<float>(hipStream_t, int, const long long *, const int *, const double *,
                                         const unsigned char *, const float *, float *, const int *, const int *,
                                         double, int, int *);

void launch_local_coarse15(hipStream_t s, const VolDesc *vd, int nvol, int slot, const Gen15 &g, const double *b,
                           double *u) {
    if (nvol <= 0) return;
    hipLaunchKernelGGL(k_local_coarse15, dim3((unsigned)((nvol + 63) / 64)), dim3(64), 0, s, vd, nvol, slot, g, b, u);
}

void launch_gen_weights(hipStream_t s, const VolGeom &vfull, const int *tetinfo, const GenK &G, double *wv,
                        long long ws) {
    VolGeom v = vfull;
    v.bs = 256;
    const long long grid = list_blocks(v, 1);
    if (grid == 0) return;
    hipLaunchKernelGGL(k_gen_weights, dim3((unsigned)grid), dim3(256), 0, s, v, tetinfo, G, wv, ws);
}

void launch_gen_ifc_weights(hipStream_t s, int n_ifc, const int *ifc_xyz, const GenK &G, double *wi15) {
    if (n_ifc <= 0) return;
    hipLaunchKernelGGL(k_gen_ifc_weights, dim3((n_ifc + 255) / 256), dim3(256), 0, s, n_ifc, ifc_xyz, G, wi15);
}

void launch_gen_coarse_vals(hipStream_t s, int n, const int *pos, const int *col15, const GenK &G, double *val) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_gen_coarse_vals, dim3((n + 255) / 256), dim3(256), 0, s, n, pos, col15, G, val);
}

void launch_apply15(hipStream_t s, const VolGeom &vint, const IfcGeom &ig, const Gen15 &g, const double *x, double *y) {
    const int nib = ifc_blocks(ig, vint.bs);
    const long long grid = nib + list_blocks(vint, 1);
    if (grid == 0) return;
    hipLaunchKernelGGL(k_apply15, dim3((unsigned)grid), dim3(vint.bs), 0, s, vint, ig, g, nib, x, y);
}

void launch_grad_k15(hipStream_t s, int N, int m, int n_sub, const double *kel, const double *u, const double *lam,
                     double *out) {
    const long long ne = 6LL * N * N * N;
    hipLaunchKernelGGL(k_grad_k15, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, s, N, m, n_sub, kel, u, lam, out);
}

void launch_neumann_rhs15(hipStream_t s, int n_ifc, long long base, const int *nb15, const double *wi15,
                          const unsigned char *gamma, const double *u, double *b_out) {
    if (n_ifc <= 0) return;
    hipLaunchKernelGGL(k_neumann_rhs15, dim3((n_ifc + 255) / 256), dim3(256), 0, s, n_ifc, base, nb15, wi15, gamma, u,
                       b_out);
}

void launch_gen_dirichlet(hipStream_t s, const VolGeom &vint, const IfcGeom &ig, const Gen15 &g, const int *tetinfo,
                          const int *ifc_xyz, int N, const double *gfull, double *b) {
    VolGeom v = vint;
    v.bs = 256;
    const int nib = ig.i1 > 0 ? (ig.i1 + 255) / 256 : 0;
    const long long grid = nib + list_blocks(v, 1);
    if (grid == 0) return;
    if (g.wv)
        hipLaunchKernelGGL(k_gen_dirichlet<true>, dim3((unsigned)grid), dim3(256), 0, s, v, ig, g, nib, tetinfo,
                           ifc_xyz, N, gfull, b);
    else
        hipLaunchKernelGGL(k_gen_dirichlet<false>, dim3((unsigned)grid), dim3(256), 0, s, v, ig, g, nib, tetinfo,
                           ifc_xyz, N, gfull, b);
}

void launch_dirichlet_load(hipStream_t s, int N, double h, const double *k, const double *g, double *b) {
    const long long n = (long long)(N - 1) * (N - 1) * (N - 1);
    if (n <= 0) return;
    hipLaunchKernelGGL(k_dirichlet_load, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, N, h, k, g, b);
}

void launch_coarse_vals(hipStream_t s, int n, const int *pos, const int *col, int N, double h, const double *k,
                        double *val) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_coarse_vals, dim3((n + 255) / 256), dim3(256), 0, s, n, pos, col, N, h, k, val);
}

void launch_ifc_weights_intact(hipStream_t s, int n_ifc, const int *ifc_xyz, int N, int m, int n_sub, double h,
                               const double *k, const unsigned char *faulty, double *wi) {
    if (n_ifc <= 0) return;
    hipLaunchKernelGGL(k_ifc_weights_intact, dim3((n_ifc + 255) / 256), dim3(256), 0, s, n_ifc, ifc_xyz, N, m, n_sub, h,
                       k, faulty, wi);
}

void launch_coarse_vals_intact(hipStream_t s, int n, const int *pos, const int *col, int N, int m, int n_sub, double h,
                               const double *k, const unsigned char *faulty, double *val) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_coarse_vals_intact, dim3((n + 255) / 256), dim3(256), 0, s, n, pos, col, N, m, n_sub, h, k,
                       faulty, val);
}

void launch_neumann_rhs(hipStream_t s, int n_ifc, long long base, const int *nbr, const double *wi,
                        const unsigned char *gamma, const double *u, double *b_out) {
    if (n_ifc <= 0) return;
    hipLaunchKernelGGL(k_neumann_rhs, dim3((n_ifc + 255) / 256), dim3(256), 0, s, n_ifc, base, nbr, wi, gamma, u,
                       b_out);
}

void launch_dn_masks(hipStream_t s, int n_ifc, long long base, long long C_pad, const int *gptr, const int *gidx,
                     const unsigned char *faulty, unsigned char *frozen, unsigned char *gamma, int *gidx_dn) {
    if (n_ifc <= 0) return;
    hipLaunchKernelGGL(k_dn_masks, dim3((n_ifc + 255) / 256), dim3(256), 0, s, n_ifc, base, C_pad, gptr, gidx, faulty,
                       frozen, gamma, gidx_dn);
}

void launch_grad_k(hipStream_t s, const double *u, const double *lam, int N, double h, double *out) {
    const long long nc = (long long)N * N * N;
    hipLaunchKernelGGL(k_grad_k, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, s, u, lam, N, h, out);
}

// explicit instantiations
template void launch_colour<double>(hipStream_t, const VolGeom &, const IfcGeom &, double *, const double *,
                                    const Weights<double> &, bool, double, double, bool, bool);
template void launch_colour<float>(hipStream_t, const VolGeom &, const IfcGeom &, float *, const float *,
                                   const Weights<float> &, bool, double, double, bool, bool);
template void launch_colour_res<double>(hipStream_t, const VolGeom &, const IfcGeom &, double *, const double *,
                                        const Weights<double> &, bool, double, double, double *);
template void launch_colour_res<float>(hipStream_t, const VolGeom &, const IfcGeom &, float *, const float *,
                                       const Weights<float> &, bool, double, double, float *);
template void launch_colour_prol<double>(hipStream_t, const VolGeom &, const IfcGeom &, double *, const double *,
                                         const Weights<double> &, bool, double, double, const Prol<double> &);
template void launch_colour_prol<float>(hipStream_t, const VolGeom &, const IfcGeom &, float *, const float *,
                                        const Weights<float> &, bool, double, double, const Prol<float> &);
template int launch_residual<double, double>(hipStream_t, const VolGeom &, const IfcGeom &, const double *,
                                             const double *, const Weights<double> &, bool, double, double *, double *);
template int launch_residual<double, float>(hipStream_t, const VolGeom &, const IfcGeom &, const double *,
                                            const double *, const Weights<double> &, bool, double, float *, double *);
template int launch_residual<float, float>(hipStream_t, const VolGeom &, const IfcGeom &, const float *, const float *,
                                           const Weights<float> &, bool, double, float *, double *);
template void launch_restrict<double>(hipStream_t, const VolGeom &, const VolDesc *, const int2 *, const IfcGeom &,
                                      const int *, const double *, double *);
template void launch_restrict<float>(hipStream_t, const VolGeom &, const VolDesc *, const int2 *, const IfcGeom &,
                                     const int *, const float *, float *);
template void launch_prolong<double>(hipStream_t, const VolGeom &, const VolDesc *, const int2 *, int, const IfcGeom &,
                                     const int *, const double *, double *);
template void launch_prolong<float>(hipStream_t, const VolGeom &, const VolDesc *, const int2 *, int, const IfcGeom &,
                                    const int *, const float *, float *);
template void launch_coarse_pcg<double>(hipStream_t, int, const long long *, const int *, const double *,
                                        const unsigned char *, const double *, double *, const int *, const int *,
                                        double, int, int *);
template void launch_coarse_pcg<float>(hipStream_t, int, const long long *, const int *, const double *,
                                       const unsigned char *, const float *, float *, const int *, const int *, double,
                                       int, int *);
template void launch_coarse_dense<double>(hipStream_t, int, const long long *, const double *, const double *,
                                          double *, const int *, const int *);
template void launch_coarse_dense<float>(hipStream_t, int, const long long *, const double *, const float *, float *,
                                         const int *, const int *);
template void launch_local_coarse<double>(hipStream_t, const VolDesc *, int, int4, const double *, double *,
                                          const Weights<double> &, bool, double);
template void launch_local_coarse<float>(hipStream_t, const VolDesc *, int, int4, const float *, float *,
                                         const Weights<float> &, bool, double);
template void launch_fill<double>(hipStream_t, double *, long long, double);
template void launch_fill<float>(hipStream_t, float *, long long, float);
template void launch_fill<unsigned char>(hipStream_t, unsigned char *, long long, unsigned char);
template void launch_fill<unsigned int>(hipStream_t, unsigned int *, long long, unsigned int);
template void launch_user_to_slots<double>(hipStream_t, const VolGeom &, const int *, int, int, const IfcGeom &,
                                           const int *, const double *, double *);
template void launch_slots_to_user<double>(hipStream_t, const VolGeom &, const int *, int, int, const IfcGeom &,
                                           const int *, const double *, double *);
template void launch_ghost_refresh<double>(hipStream_t, const int *, const int *, int, double *);
template void launch_ghost_refresh<float>(hipStream_t, const int *, const int *, int, float *);
template void launch_cast<double, float>(hipStream_t, const double *, float *, long long);
template void launch_cast<float, double>(hipStream_t, const float *, double *, long long);

}  // namespace hhgr
