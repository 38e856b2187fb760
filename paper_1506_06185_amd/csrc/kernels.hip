// HIP kernels (gfx950) of the HHG multigrid engine.
//
// Volume containers are processed as structured arrays: a workgroup takes a
// chunk of consecutive slots of one plane of one tetrahedron, decodes (i,j,k)
// arithmetically and reads its stencil neighbours at closed-form offsets, so
// the loads of a wavefront are consecutive addresses.  Interface (face, edge,
// vertex) nodes are few and are handled through precomputed slot tables by
// the first workgroups of the same launch.  Block ids of the volume part are
// remapped so that each of the 8 XCDs walks a contiguous run of chunks, which
// keeps the neighbouring planes of a chunk in that XCD's L2.
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

__device__ __forceinline__ int tetnum_d(int x) { return x * (x + 1) * (x + 2) / 6; }
__device__ __forceinline__ int pstart_d(int M, int k) { return tetnum_d(M) - tetnum_d(M - k); }
__device__ __forceinline__ int rstart_d(int s, int j) { return j * s - ((j * (j - 1)) >> 1); }
__device__ __forceinline__ int cidx_d(int M, int i, int j, int k) { return pstart_d(M, k) + rstart_d(M - k, j) + i; }

// row j of a triangular plane with row-0 length s that holds plane offset o
__device__ __forceinline__ int decode_row(int s, int o) {
    const float b = 2.0f * (float)s + 1.0f;
    const float disc = fmaxf(b * b - 8.0f * (float)o, 0.0f);
    int j = (int)((b - sqrtf(disc)) * 0.5f);
    j = max(0, min(j, s - 1));
    while (j + 1 <= s - 1 && rstart_d(s, j + 1) <= o) ++j;
    while (j > 0 && rstart_d(s, j) > o) --j;
    return j;
}

// Workgroups are dispatched to the 8 XCDs round-robin; map so that each XCD
// receives a contiguous range of logical block ids.
__device__ __forceinline__ unsigned xcd_remap(unsigned f, unsigned total) {
    const unsigned per = total >> 3, rem = total & 7u, x = f & 7u, loc = f >> 3;
    return x < rem ? x * (per + 1) + loc : rem * (per + 1) + (x - rem) * per + loc;
}

struct VNode {
    int v, i, j, k, s, o, ps;
};

__device__ __forceinline__ bool vol_node(const VolGeom &g, unsigned lg, VNode &n) {
    n.v = (int)(lg / (unsigned)g.nchunks);
    const int c = (int)(lg % (unsigned)g.nchunks);
    const int2 ch = g.chunks[c];
    n.k = ch.x;
    n.s = g.M - n.k;
    n.o = ch.y + (int)threadIdx.x;
    if (n.o >= n.s * (n.s + 1) / 2) return false;
    n.j = decode_row(n.s, n.o);
    n.i = n.o - rstart_d(n.s, n.j);
    n.ps = pstart_d(g.M, n.k);
    return true;
}

__device__ __forceinline__ bool is_interior(const VNode &n, int M) {
    return n.i >= 1 && n.j >= 1 && n.k >= 1 && n.i + n.j + n.k <= M - 2;
}

// closure offsets of the 6 axis neighbours (local directions a, b, c)
struct Nb6 {
    int ap, am, bp, bm, cp, cm;
};
__device__ __forceinline__ Nb6 nb6(const VNode &n) {
    const int c0 = n.ps + n.o;
    const int rj = n.s - n.j;
    Nb6 r;
    r.ap = c0 + 1;
    r.am = c0 - 1;
    r.bp = c0 + rj - 1;                                                            // (i-1, j+1, k)
    r.bm = c0 - rj;                                                                // (i+1, j-1, k)
    r.cp = n.ps + n.s * (n.s + 1) / 2 + rstart_d(n.s - 1, n.j - 1) + n.i;          // (i, j-1, k+1)
    r.cm = n.ps - (n.s + 1) * (n.s + 2) / 2 + rstart_d(n.s + 1, n.j + 1) + n.i;    // (i, j+1, k-1)
    return r;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
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
// red-black SOR colour pass
// ---------------------------------------------------------------------------
template <typename T, bool VK, bool OWN0, bool NB0>
__global__ void __launch_bounds__(512) k_colour(VolGeom vg, IfcGeom ig, int nib, T *__restrict__ u,
                                                const T *__restrict__ b, Weights<T> w, T h, T omega, int colour) {
    const unsigned f = blockIdx.x;
    if (f < (unsigned)nib) {
        const int t = ig.i0 + (int)(f * blockDim.x + threadIdx.x);
        if (t >= ig.i1) return;
        if (ig.frozen && ig.frozen[t]) return;
        const long long sl = ig.base + t;
        const T uo = OWN0 ? T(0) : u[sl];
        T acc = T(0), diag;
        if (VK) {
            diag = T(0);
#pragma unroll
            for (int e = 0; e < 6; e++) {
                const T we = w.wi[(long long)e * ig.stride + t];
                diag += we;
                if (!NB0) acc += we * u[ig.nbr[(long long)e * ig.stride + t]];
            }
        } else {
            diag = T(6) * h;
            if (!NB0) {
#pragma unroll
                for (int e = 0; e < 6; e++) acc += u[ig.nbr[(long long)e * ig.stride + t]];
                acc *= h;
            }
        }
        const T Au = diag * uo - acc;
        const T un = uo + omega * (b[sl] - Au) / diag;
        u[sl] = un;
        if (ig.gptr)
            for (int g = ig.gptr[t]; g < ig.gptr[t + 1]; g++) u[ig.gidx[g]] = un;
        return;
    }
    VNode n;
    if (!vol_node(vg, xcd_remap(f - nib, gridDim.x - nib), n)) return;
    if (!is_interior(n, vg.M) || ((n.i + n.k) & 1) != colour) return;
    const VolDesc d = vg.vd[n.v];
    T *uv = u + d.vec;
    const int c0 = n.ps + n.o;
    const Nb6 q = nb6(n);
    const T uo = OWN0 ? T(0) : uv[c0];
    T diag, acc;
    if (VK) {
        const T *w0 = w.w0 + d.w, *w1 = w.w1 + d.w, *w2 = w.w2 + d.w;
        const T wap = w0[c0], wam = w0[q.am], wbp = w1[c0], wbm = w1[q.bm], wcp = w2[c0], wcm = w2[q.cm];
        diag = ((wap + wam) + (wbp + wbm)) + (wcp + wcm);
        acc = NB0 ? T(0)
                  : wap * uv[q.ap] + wam * uv[q.am] + wbp * uv[q.bp] + wbm * uv[q.bm] + wcp * uv[q.cp] +
                        wcm * uv[q.cm];
    } else {
        diag = T(6) * h;
        acc = NB0 ? T(0) : h * (((uv[q.ap] + uv[q.am]) + (uv[q.bp] + uv[q.bm])) + (uv[q.cp] + uv[q.cm]));
    }
    const T Au = diag * uo - acc;
    uv[c0] = uo + omega * ((b + d.vec)[c0] - Au) / diag;
}

// ---------------------------------------------------------------------------
// residual r = b - A u (+ block partial sums of r^2)
// ---------------------------------------------------------------------------
template <typename T, typename TO, bool VK, bool WRITE, bool NORM>
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
            if (VK) {
                diag = T(0);
#pragma unroll
                for (int e = 0; e < 6; e++) {
                    const T we = w.wi[(long long)e * ig.stride + t];
                    diag += we;
                    acc += we * u[ig.nbr[(long long)e * ig.stride + t]];
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
        VNode n;
        if (vol_node(vg, xcd_remap(f - nib, gridDim.x - nib), n) && is_interior(n, vg.M)) {
            const VolDesc d = vg.vd[n.v];
            const T *uv = u + d.vec;
            const int c0 = n.ps + n.o;
            const Nb6 q = nb6(n);
            const T uo = uv[c0];
            T diag, acc;
            if (VK) {
                const T *w0 = w.w0 + d.w, *w1 = w.w1 + d.w, *w2 = w.w2 + d.w;
                const T wap = w0[c0], wam = w0[q.am], wbp = w1[c0], wbm = w1[q.bm], wcp = w2[c0], wcm = w2[q.cm];
                diag = ((wap + wam) + (wbp + wbm)) + (wcp + wcm);
                acc = wap * uv[q.ap] + wam * uv[q.am] + wbp * uv[q.bp] + wbm * uv[q.bm] + wcp * uv[q.cp] +
                      wcm * uv[q.cm];
            } else {
                diag = T(6) * h;
                acc = h * (((uv[q.ap] + uv[q.am]) + (uv[q.bp] + uv[q.bm])) + (uv[q.cp] + uv[q.cm]));
            }
            const T res = (b + d.vec)[c0] - (diag * uo - acc);
            if (WRITE) (r + d.vec)[c0] = (TO)res;
            acc2 = (double)res * (double)res;
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
__device__ __constant__ int kD14[14][3] = {{1, 0, 0},  {-1, 0, 0}, {-1, 1, 0}, {1, -1, 0}, {0, -1, 1},
                                           {0, 1, -1}, {0, 1, 0},  {0, -1, 0}, {-1, 0, 1}, {1, 0, -1},
                                           {1, -1, 1}, {-1, 1, -1}, {0, 0, 1}, {0, 0, -1}};

template <typename T>
__global__ void __launch_bounds__(512) k_restrict(VolGeom vc, const VolDesc *__restrict__ vdf, int Mf, IfcGeom ig,
                                                  int nib, const int *__restrict__ rst, const T *__restrict__ rf,
                                                  T *__restrict__ bc) {
    const unsigned f = blockIdx.x;
    if (f < (unsigned)nib) {
        const int t = ig.i0 + (int)(f * blockDim.x + threadIdx.x);
        if (t >= ig.i1) return;
        if (ig.frozen && ig.frozen[t]) return;
        T s = T(0);
#pragma unroll
        for (int e = 1; e < 15; e++) s += rf[rst[(long long)e * ig.stride + t]];
        bc[ig.base + t] = rf[rst[t]] + T(0.5) * s;
        return;
    }
    VNode n;
    if (!vol_node(vc, xcd_remap(f - nib, gridDim.x - nib), n)) return;
    if (!is_interior(n, vc.M)) return;
    const T *rv = rf + vdf[n.v].vec;
    const int I = 2 * n.i, J = 2 * n.j, K = 2 * n.k;
    T s = T(0);
#pragma unroll
    for (int e = 0; e < 14; e++) s += rv[cidx_d(Mf, I + kD14[e][0], J + kD14[e][1], K + kD14[e][2])];
    (bc + vc.vd[n.v].vec)[n.ps + n.o] = rv[cidx_d(Mf, I, J, K)] + T(0.5) * s;
}

// ---------------------------------------------------------------------------
// prolongation u_f += P e_c (linear interpolation)
// ---------------------------------------------------------------------------
// index direction of the coarse edge bisected by a fine node with parity code
// (i&1) | (j&1)<<1 | (k&1)<<2
__device__ __constant__ int kParDir[8][3] = {{0, 0, 0},  {1, 0, 0}, {0, 1, 0},  {-1, 1, 0},
                                             {0, 0, 1},  {-1, 0, 1}, {0, -1, 1}, {1, -1, 1}};

template <typename T>
__global__ void __launch_bounds__(512) k_prolong(VolGeom vf, const VolDesc *__restrict__ vdc, int Mc, IfcGeom ig,
                                                 int nib, const int *__restrict__ prl, const T *__restrict__ ec,
                                                 T *__restrict__ uf) {
    const unsigned f = blockIdx.x;
    if (f < (unsigned)nib) {
        const int t = ig.i0 + (int)(f * blockDim.x + threadIdx.x);
        if (t >= ig.i1) return;
        if (ig.frozen && ig.frozen[t]) return;
        const long long sl = ig.base + t;
        const T v = uf[sl] + T(0.5) * (ec[prl[t]] + ec[prl[(long long)ig.stride + t]]);
        uf[sl] = v;
        if (ig.gptr)
            for (int g = ig.gptr[t]; g < ig.gptr[t + 1]; g++) uf[ig.gidx[g]] = v;
        return;
    }
    VNode n;
    if (!vol_node(vf, xcd_remap(f - nib, gridDim.x - nib), n)) return;
    if (!is_interior(n, vf.M)) return;
    const T *ev = ec + vdc[n.v].vec;
    T *uv = uf + vf.vd[n.v].vec;
    const int code = (n.i & 1) | ((n.j & 1) << 1) | ((n.k & 1) << 2);
    const int c0 = n.ps + n.o;
    if (code == 0) {
        uv[c0] = uv[c0] + ev[cidx_d(Mc, n.i >> 1, n.j >> 1, n.k >> 1)];
    } else {
        const int di = kParDir[code][0], dj = kParDir[code][1], dk = kParDir[code][2];
        const T e1 = ev[cidx_d(Mc, (n.i - di) >> 1, (n.j - dj) >> 1, (n.k - dk) >> 1)];
        const T e2 = ev[cidx_d(Mc, (n.i + di) >> 1, (n.j + dj) >> 1, (n.k + dk) >> 1)];
        uv[c0] = uv[c0] + T(0.5) * (e1 + e2);
    }
}

// ---------------------------------------------------------------------------
// coarsest level: Jacobi-PCG in one workgroup, unknowns owned by threads,
// search direction shared through LDS
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(1024) k_coarse_pcg(int n, const long long *__restrict__ slot,
                                                     const int *__restrict__ col, const double *__restrict__ val,
                                                     const unsigned char *__restrict__ frozen, const T *__restrict__ b,
                                                     T *__restrict__ u, const int *__restrict__ cptr,
                                                     const int *__restrict__ cidx, double rtol, int maxit,
                                                     int *__restrict__ iters) {
    __shared__ double p_sh[2048];
    __shared__ double red[64];
    const int tid = threadIdx.x;
    double x[2] = {0.0, 0.0}, r[2] = {0.0, 0.0}, p[2] = {0.0, 0.0}, d[2] = {1.0, 1.0};
    bool act[2], frz[2];
    for (int s = 0; s < 2; s++) {
        const int q = tid + s * 1024;
        act[s] = q < n;
        frz[s] = act[s] && frozen && frozen[q];
        if (act[s]) {
            d[s] = val[7 * q];
            r[s] = frz[s] ? 0.0 : (double)b[slot[q]];
            p[s] = r[s] / d[s];
            p_sh[q] = p[s];
        }
    }
    double rz = r[0] * p[0] + r[1] * p[1];
    double rr0 = r[0] * r[0] + r[1] * r[1];
    block_sum2_all(rz, rr0, red);
    int it = 0;
    if (rr0 > 0.0) {
        const double stop = rtol * rtol * rr0;
        for (it = 1; it <= maxit; it++) {
            __syncthreads();
            double qv[2] = {0.0, 0.0};
            for (int s = 0; s < 2; s++) {
                if (!act[s] || frz[s]) continue;
                const int q = tid + s * 1024;
                double a = d[s] * p[s];
                for (int e = 1; e < 7; e++) {
                    const int c = col[7 * q + e];
                    if (c >= 0) a += val[7 * q + e] * p_sh[c];
                }
                qv[s] = a;
            }
            double pq = p[0] * qv[0] + p[1] * qv[1];
            double dummy = 0.0;
            block_sum2_all(pq, dummy, red);
            const double alpha = rz / pq;
            for (int s = 0; s < 2; s++) {
                x[s] += alpha * p[s];
                r[s] -= alpha * qv[s];
            }
            double rr = r[0] * r[0] + r[1] * r[1];
            double rz1 = r[0] * r[0] / d[0] + r[1] * r[1] / d[1];
            block_sum2_all(rr, rz1, red);
            if (rr <= stop) break;
            const double beta = rz1 / rz;
            rz = rz1;
            for (int s = 0; s < 2; s++) {
                p[s] = r[s] / d[s] + beta * p[s];
                if (act[s]) p_sh[tid + s * 1024] = p[s];
            }
        }
    }
    for (int s = 0; s < 2; s++) {
        const int q = tid + s * 1024;
        if (!act[s] || frz[s]) continue;
        const T xv = (T)x[s];
        for (int c = cptr[q]; c < cptr[q + 1]; c++) u[cidx[c]] = xv;
    }
    if (tid == 0 && iters) *iters = it;
}

template <typename T, bool VK>
__global__ void k_local_coarse(const VolDesc *__restrict__ vd, int nvol, int M, const T *__restrict__ b,
                               T *__restrict__ u, Weights<T> w, T h) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nvol) return;
    const VolDesc d = vd[v];
    // the single interior node (1,1,1) of a tetrahedron with 4 segments per edge
    VNode n;
    n.i = 1;
    n.j = 1;
    n.k = 1;
    n.s = M - 1;
    n.ps = pstart_d(M, 1);
    n.o = rstart_d(n.s, 1) + 1;
    const int c0 = n.ps + n.o;
    T diag;
    if (VK) {
        const Nb6 q = nb6(n);
        const T *w0 = w.w0 + d.w, *w1 = w.w1 + d.w, *w2 = w.w2 + d.w;
        diag = ((w0[c0] + w0[q.am]) + (w1[c0] + w1[q.bm])) + (w2[c0] + w2[q.cm]);
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
    VNode n;
    if (!vol_node(vg, xcd_remap(f - nib, gridDim.x - nib), n)) return;
    const VolDesc d = vg.vd[n.v];
    int X[3];
    grid_pos(tetinfo, d.tet, m, n.i, n.j, n.k, X);
    const bool in = X[0] > 0 && X[1] > 0 && X[2] > 0 && X[0] < N && X[1] < N && X[2] < N;
    const long long dof = (long long)(X[0] - 1) + (long long)(N - 1) * ((X[1] - 1) + (long long)(N - 1) * (X[2] - 1));
    (vec + d.vec)[n.ps + n.o] = in ? (T)user[dof] : T(0);
}

template <typename T>
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
    VNode n;
    if (!vol_node(vg, xcd_remap(f - nib, gridDim.x - nib), n)) return;
    if (!is_interior(n, vg.M)) return;
    const VolDesc d = vg.vd[n.v];
    int X[3];
    grid_pos(tetinfo, d.tet, m, n.i, n.j, n.k, X);
    const long long dof = (long long)(X[0] - 1) + (long long)(N - 1) * ((X[1] - 1) + (long long)(N - 1) * (X[2] - 1));
    user[dof] = (double)(vec + d.vec)[n.ps + n.o];
}

// consistent P1 mass matrix on the Kuhn meshes: diagonal 24 h^3/60, axis
// edges h^3/20 (6 tetrahedra), face diagonals h^3/30 (4), body diagonal h^3/20 (6)
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
    VNode n;
    if (!vol_node(vg, xcd_remap(f - nib, gridDim.x - nib), n)) return;
    if (!is_interior(n, vg.M)) return;
    const VolDesc d = vg.vd[n.v];
    const double *xv = x + d.vec;
    const int M = vg.M;
    double ax = 0.0, fd = 0.0, bd = 0.0;
    // index directions: 0..5 axis (a,b,c), 6..11 face diagonals (a+b, b+c, a+c), 12..13 body (a+b+c)
    for (int e = 0; e < 6; e++) ax += xv[cidx_d(M, n.i + kD14[e][0], n.j + kD14[e][1], n.k + kD14[e][2])];
    for (int e = 6; e < 12; e++) fd += xv[cidx_d(M, n.i + kD14[e][0], n.j + kD14[e][1], n.k + kD14[e][2])];
    for (int e = 12; e < 14; e++) bd += xv[cidx_d(M, n.i + kD14[e][0], n.j + kD14[e][1], n.k + kD14[e][2])];
    (y + d.vec)[n.ps + n.o] = wc * xv[n.ps + n.o] + wax * ax + wfd * fd + wbd * bd;
}

__global__ void __launch_bounds__(512) k_update_add(VolGeom vg, IfcGeom ig, int nib, double *__restrict__ u,
                                                    const float *__restrict__ e) {
    const unsigned f = blockIdx.x;
    if (f < (unsigned)nib) {
        const int t = ig.i0 + (int)(f * blockDim.x + threadIdx.x);
        if (t >= ig.i1) return;
        const long long sl = ig.base + t;
        u[sl] += (double)e[sl];
        return;
    }
    VNode n;
    if (!vol_node(vg, xcd_remap(f - nib, gridDim.x - nib), n)) return;
    const long long sl = vg.vd[n.v].vec + n.ps + n.o;
    u[sl] += (double)e[sl];
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
    VNode n;
    if (!vol_node(vg, xcd_remap(blockIdx.x, gridDim.x), n)) return;
    const VolDesc d = vg.vd[n.v];
    int X[3];
    grid_pos(tetinfo, d.tet, m, n.i, n.j, n.k, X);
    const int *ti = tetinfo + 6 * d.tet;
    const long long sl = d.w + n.ps + n.o;
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
                   double h, double omega, int colour, bool own0, bool nb0) {
    const int nib = ifc_blocks(ig, vg.bs);
    const long long nvb = (long long)vg.nchunks * vg.nvol;
    const long long grid = nib + nvb;
    if (grid == 0) return;
    const T th = (T)h, to = (T)omega;
#define HHGR_COLOUR(VK, O0, N0) \
    hipLaunchKernelGGL((k_colour<T, VK, O0, N0>), dim3((unsigned)grid), dim3(vg.bs), 0, s, vg, ig, nib, u, b, w, th, to, colour)
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

template <typename T, typename TO>
int launch_residual(hipStream_t s, const VolGeom &vg, const IfcGeom &ig, const T *u, const T *b, const Weights<T> &w,
                    bool vk, double h, TO *r, double *partial) {
    const int nib = ifc_blocks(ig, vg.bs);
    const long long nvb = (long long)vg.nchunks * vg.nvol;
    const long long grid = nib + nvb;
    if (grid == 0) return 0;
    const T th = (T)h;
#define HHGR_RES(VK, WR, NO) \
    hipLaunchKernelGGL((k_residual<T, TO, VK, WR, NO>), dim3((unsigned)grid), dim3(vg.bs), 0, s, vg, ig, nib, u, b, w, th, r, partial)
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
void launch_restrict(hipStream_t s, const VolGeom &vc, const VolDesc *vdf, int Mf, const IfcGeom &igc, const int *rst,
                     const T *rf, T *bc) {
    const int nib = ifc_blocks(igc, vc.bs);
    const long long grid = nib + (long long)vc.nchunks * vc.nvol;
    if (grid == 0) return;
    hipLaunchKernelGGL((k_restrict<T>), dim3((unsigned)grid), dim3(vc.bs), 0, s, vc, vdf, Mf, igc, nib, rst, rf, bc);
}

template <typename T>
void launch_prolong(hipStream_t s, const VolGeom &vf, const VolDesc *vdc, int Mc, const IfcGeom &igf, const int *prl,
                    const T *ec, T *uf) {
    const int nib = ifc_blocks(igf, vf.bs);
    const long long grid = nib + (long long)vf.nchunks * vf.nvol;
    if (grid == 0) return;
    hipLaunchKernelGGL((k_prolong<T>), dim3((unsigned)grid), dim3(vf.bs), 0, s, vf, vdc, Mc, igf, nib, prl, ec, uf);
}

template <typename T>
void launch_coarse_pcg(hipStream_t s, int n, const long long *slot, const int *col, const double *val,
                       const unsigned char *frozen, const T *b, T *u, const int *cptr, const int *cidx, double rtol,
                       int maxit, int *iters) {
    hipLaunchKernelGGL((k_coarse_pcg<T>), dim3(1), dim3(1024), 0, s, n, slot, col, val, frozen, b, u, cptr, cidx, rtol,
                       maxit, iters);
}

template <typename T>
void launch_local_coarse(hipStream_t s, const VolDesc *vd, int nvol, int M, const T *b, T *u, const Weights<T> &w,
                         bool vk, double h) {
    if (nvol <= 0) return;
    const unsigned g = (unsigned)((nvol + 63) / 64);
    if (vk)
        hipLaunchKernelGGL((k_local_coarse<T, true>), dim3(g), dim3(64), 0, s, vd, nvol, M, b, u, w, (T)h);
    else
        hipLaunchKernelGGL((k_local_coarse<T, false>), dim3(g), dim3(64), 0, s, vd, nvol, M, b, u, w, (T)h);
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
    const long long grid = nib + (long long)vfull.nchunks * vfull.nvol;
    if (grid == 0) return;
    hipLaunchKernelGGL((k_user_to_slots<T>), dim3((unsigned)grid), dim3(vfull.bs), 0, s, vfull, tetinfo, m, N, ig, nib,
                       ifc_dof, user, vec);
}

template <typename T>
void launch_slots_to_user(hipStream_t s, const VolGeom &vint, const int *tetinfo, int m, int N, const IfcGeom &ig,
                          const int *ifc_dof, const T *vec, double *user) {
    const int nib = ifc_blocks(ig, vint.bs);
    const long long grid = nib + (long long)vint.nchunks * vint.nvol;
    if (grid == 0) return;
    hipLaunchKernelGGL((k_slots_to_user<T>), dim3((unsigned)grid), dim3(vint.bs), 0, s, vint, tetinfo, m, N, ig, nib,
                       ifc_dof, vec, user);
}

void launch_mass(hipStream_t s, const VolGeom &vint, const IfcGeom &ig, const int *nb15, const double *x, double *y,
                 double h) {
    const int nib = ifc_blocks(ig, vint.bs);
    const long long grid = nib + (long long)vint.nchunks * vint.nvol;
    if (grid == 0) return;
    hipLaunchKernelGGL(k_mass, dim3((unsigned)grid), dim3(vint.bs), 0, s, vint, ig, nib, nb15, x, y, h * h * h);
}

void launch_update_add(hipStream_t s, const VolGeom &vfull, const IfcGeom &ig, double *u, const float *e) {
    const int nib = ifc_blocks(ig, vfull.bs);
    const long long grid = nib + (long long)vfull.nchunks * vfull.nvol;
    if (grid == 0) return;
    hipLaunchKernelGGL(k_update_add, dim3((unsigned)grid), dim3(vfull.bs), 0, s, vfull, ig, nib, u, e);
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
    const long long grid = (long long)vfull.nchunks * vfull.nvol;
    if (grid == 0) return;
    hipLaunchKernelGGL(k_vol_weights, dim3((unsigned)grid), dim3(vfull.bs), 0, s, vfull, tetinfo, m, N, h, k, w0, w1,
                       w2);
}

void launch_ifc_weights(hipStream_t s, int n_ifc, const int *ifc_xyz, int N, double h, const double *k, double *wi) {
    if (n_ifc <= 0) return;
    hipLaunchKernelGGL(k_ifc_weights, dim3((n_ifc + 255) / 256), dim3(256), 0, s, n_ifc, ifc_xyz, N, h, k, wi);
}

void launch_coarse_vals(hipStream_t s, int n, const int *pos, const int *col, int N, double h, const double *k,
                        double *val) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_coarse_vals, dim3((n + 255) / 256), dim3(256), 0, s, n, pos, col, N, h, k, val);
}

void launch_grad_k(hipStream_t s, const double *u, const double *lam, int N, double h, double *out) {
    const long long nc = (long long)N * N * N;
    hipLaunchKernelGGL(k_grad_k, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, s, u, lam, N, h, out);
}

// explicit instantiations
template void launch_colour<double>(hipStream_t, const VolGeom &, const IfcGeom &, double *, const double *,
                                    const Weights<double> &, bool, double, double, int, bool, bool);
template void launch_colour<float>(hipStream_t, const VolGeom &, const IfcGeom &, float *, const float *,
                                   const Weights<float> &, bool, double, double, int, bool, bool);
template int launch_residual<double, double>(hipStream_t, const VolGeom &, const IfcGeom &, const double *,
                                             const double *, const Weights<double> &, bool, double, double *, double *);
template int launch_residual<double, float>(hipStream_t, const VolGeom &, const IfcGeom &, const double *,
                                            const double *, const Weights<double> &, bool, double, float *, double *);
template int launch_residual<float, float>(hipStream_t, const VolGeom &, const IfcGeom &, const float *, const float *,
                                           const Weights<float> &, bool, double, float *, double *);
template void launch_restrict<double>(hipStream_t, const VolGeom &, const VolDesc *, int, const IfcGeom &, const int *,
                                      const double *, double *);
template void launch_restrict<float>(hipStream_t, const VolGeom &, const VolDesc *, int, const IfcGeom &, const int *,
                                     const float *, float *);
template void launch_prolong<double>(hipStream_t, const VolGeom &, const VolDesc *, int, const IfcGeom &, const int *,
                                     const double *, double *);
template void launch_prolong<float>(hipStream_t, const VolGeom &, const VolDesc *, int, const IfcGeom &, const int *,
                                    const float *, float *);
template void launch_coarse_pcg<double>(hipStream_t, int, const long long *, const int *, const double *,
                                        const unsigned char *, const double *, double *, const int *, const int *,
                                        double, int, int *);
template void launch_coarse_pcg<float>(hipStream_t, int, const long long *, const int *, const double *,
                                       const unsigned char *, const float *, float *, const int *, const int *, double,
                                       int, int *);
template void launch_local_coarse<double>(hipStream_t, const VolDesc *, int, int, const double *, double *,
                                          const Weights<double> &, bool, double);
template void launch_local_coarse<float>(hipStream_t, const VolDesc *, int, int, const float *, float *,
                                         const Weights<float> &, bool, double);
template void launch_fill<double>(hipStream_t, double *, long long, double);
template void launch_fill<float>(hipStream_t, float *, long long, float);
template void launch_fill<unsigned char>(hipStream_t, unsigned char *, long long, unsigned char);
template void launch_user_to_slots<double>(hipStream_t, const VolGeom &, const int *, int, int, const IfcGeom &,
                                           const int *, const double *, double *);
template void launch_slots_to_user<double>(hipStream_t, const VolGeom &, const int *, int, int, const IfcGeom &,
                                           const int *, const double *, double *);
template void launch_ghost_refresh<double>(hipStream_t, const int *, const int *, int, double *);
template void launch_ghost_refresh<float>(hipStream_t, const int *, const int *, int, float *);
template void launch_cast<double, float>(hipStream_t, const double *, float *, long long);
template void launch_cast<float, double>(hipStream_t, const float *, double *, long long);

}  // namespace hhgr
