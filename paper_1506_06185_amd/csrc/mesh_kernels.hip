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

}  // namespace

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
