// HIP kernels of the unstructured-macro-mesh path that the structured
// kernels (kernels.hip) do not cover.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace hhgr {
namespace {

// eliminated Dirichlet data (eq. (1) into eq. (2)): b = -A_IB g at the rows
// coupled to boundary nodes, one thread per row, entries in a fixed order
__global__ void k_dirichlet_rows(int nrows, const int *__restrict__ rows, const int *__restrict__ ptr,
                                 const int *__restrict__ col, const double *__restrict__ val,
                                 const double *__restrict__ g, double *__restrict__ b) {
    const int q = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (q >= nrows) return;
    double s = 0.0;
    for (int e = ptr[q]; e < ptr[q + 1]; e++) s += val[e] * g[col[e]];
    b[rows[q]] = -s;
}

// static Neumann data of the intact side (Alg. 2) at the masters flagged in
// gamma: b_out = (A^I u) from the intact-side rows of width w (entry 0 the
// diagonal at the master's own slot), entries in a fixed order
__global__ void k_neumann_rhs_w(int n_ifc, long long base, const int *__restrict__ nb, const double *__restrict__ wi,
                                int w, const unsigned char *__restrict__ gamma, const double *__restrict__ u,
                                double *__restrict__ b_out) {
    const int t = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (t >= n_ifc || !gamma[t]) return;
    double s = 0.0;
    for (int e = 0; e < w; e++) s += wi[(long long)e * n_ifc + t] * u[nb[(long long)e * n_ifc + t]];
    b_out[base + t] = s;
}

// closure slot of node (i, j, k) from the level's row table (colour-split
// layout: row (j, k) of colour (i + k) & 1 starts at .x for 0, .y for 1)
__device__ __forceinline__ long long mesh_slot(const int2 *__restrict__ rowC, int M, int i, int j, int k) {
    const int2 r = rowC[k * M - ((k * (k - 1)) >> 1) + j];
    return (long long)((((i + k) & 1) ? r.y : r.x) + (i >> 1));
}

// dJ/dk per macro tetrahedron, first pass: block (pair, tet) sums
// lambda_e^T K_e u_e over the elements e of tetrahedron t whose lowest
// index-space corner X = (a, b, c) has (b, c) = the pair's, c <= b < m, over
// a in [b, m) and the 6 element types (those with every corner in the
// closure: X0 >= X1 >= X2 >= 0, X0 <= m); fixed summation order
__global__ void __launch_bounds__(256) k_mesh_grad_rows(int m, int M, const int2 *__restrict__ rowC, long long C_pad,
                                                       const double *__restrict__ kel, const double *__restrict__ u,
                                                       const double *__restrict__ lam, int npairs,
                                                       double *__restrict__ partial) {
    __shared__ double sh[256];
    const int t = (int)blockIdx.y, pr = (int)blockIdx.x;
    int b = (int)((sqrt(8.0 * pr + 1.0) - 1.0) * 0.5);
    while ((b + 1) * (b + 2) / 2 <= pr) b++;
    while (b * (b + 1) / 2 > pr) b--;
    const int c = pr - b * (b + 1) / 2;
    const long long base = (long long)t * C_pad;
    const double *Kt = kel + 96LL * t;
    double acc = 0.0;
    for (int q = (int)threadIdx.x; q < 6 * (m - b); q += (int)blockDim.x) {
        const int a = b + q / 6, p = q % 6;
        const int p0 = p >> 1, p1 = p0 == 0 ? 1 + (p & 1) : p0 == 1 ? ((p & 1) ? 2 : 0) : (p & 1);
        int X[4][3] = {{a, b, c}, {a, b, c}, {a, b, c}, {a + 1, b + 1, c + 1}};
        X[1][p0]++;
        X[2][p0]++;
        X[2][p1]++;
        bool in = true;
        for (int r = 0; r < 4; r++) in = in && X[r][0] >= X[r][1] && X[r][1] >= X[r][2] && X[r][2] >= 0 && X[r][0] <= m;
        if (!in) continue;
        double ul[4], ll[4];
        for (int r = 0; r < 4; r++) {
            const long long s = base + mesh_slot(rowC, M, X[r][0] - X[r][1], X[r][1] - X[r][2], X[r][2]);
            ul[r] = u[s];
            ll[r] = lam[s];
        }
        const double *K = Kt + 16 * p;
        double g = 0.0;
        for (int r = 0; r < 4; r++)
            for (int s2 = 0; s2 < 4; s2++) g += ll[r] * K[4 * r + s2] * ul[s2];
        acc += g;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[(long long)t * npairs + pr] = sh[0];
}

// second pass: dJ/dk_t = -(sum of the tetrahedron's row sums), fixed order
__global__ void __launch_bounds__(256) k_mesh_grad_sum(int npairs, const double *__restrict__ partial,
                                                      double *__restrict__ out) {
    __shared__ double sh[256];
    const int t = (int)blockIdx.x;
    double acc = 0.0;
    for (int q = (int)threadIdx.x; q < npairs; q += (int)blockDim.x) acc += partial[(long long)t * npairs + q];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[t] = -sh[0];
}

}  // namespace

void launch_mesh_grad_tet(hipStream_t s, int nt, int m, int M, const int2 *rowC, long long C_pad, const double *kel,
                          const double *u, const double *lam, double *partial, double *out) {
    if (nt <= 0) return;
    const int npairs = m * (m + 1) / 2;
    hipLaunchKernelGGL(k_mesh_grad_rows, dim3((unsigned)npairs, (unsigned)nt), dim3(256), 0, s, m, M, rowC, C_pad, kel,
                       u, lam, npairs, partial);
    hipLaunchKernelGGL(k_mesh_grad_sum, dim3((unsigned)nt), dim3(256), 0, s, npairs, partial, out);
}

void launch_neumann_rhs_w(hipStream_t s, int n_ifc, long long base, const int *nb, const double *wi, int w,
                          const unsigned char *gamma, const double *u, double *b_out) {
    if (n_ifc <= 0) return;
    hipLaunchKernelGGL(k_neumann_rhs_w, dim3((unsigned)((n_ifc + 255) / 256)), dim3(256), 0, s, n_ifc, base, nb, wi, w,
                       gamma, u, b_out);
}

void launch_dirichlet_rows(hipStream_t s, int nrows, const int *rows, const int *ptr, const int *col,
                           const double *val, const double *g, double *b) {
    if (nrows <= 0) return;
    hipLaunchKernelGGL(k_dirichlet_rows, dim3((unsigned)((nrows + 255) / 256)), dim3(256), 0, s, nrows, rows, ptr, col,
                       val, g, b);
}

}  // namespace hhgr
