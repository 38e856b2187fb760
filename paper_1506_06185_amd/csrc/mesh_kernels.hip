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

}  // namespace

void launch_dirichlet_rows(hipStream_t s, int nrows, const int *rows, const int *ptr, const int *col,
                           const double *val, const double *g, double *b) {
    if (nrows <= 0) return;
    hipLaunchKernelGGL(k_dirichlet_rows, dim3((unsigned)((nrows + 255) / 256)), dim3(256), 0, s, nrows, rows, ptr, col,
                       val, g, b);
}

}  // namespace hhgr
