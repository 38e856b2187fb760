// Host emulation of the HIP device-code subset used by fused.hip, for
// checking its indexing on the CPU: a workgroup runs as blockDim.x host
// threads that meet at a std::barrier in __syncthreads(); workgroups run one
// after another; dynamic LDS is one host array whose bytes beyond the
// launch's request are poisoned for AddressSanitizer.  Test use only.
#pragma once
#include <algorithm>
#include <barrier>
#include <cstddef>
#include <functional>
#include <thread>
#include <vector>

#include <sanitizer/asan_interface.h>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(x)
#define __shared__
#define __restrict__

typedef struct mockdev_stream *hipStream_t;
struct int2 {
    int x, y;
};
struct int4 {
    int x, y, z, w;
};
inline int2 make_int2(int x, int y) { return int2{x, y}; }
inline int4 make_int4(int x, int y, int z, int w) { return int4{x, y, z, w}; }
struct dim3 {
    unsigned x = 1, y = 1, z = 1;
    dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct mockdev_idx {
    unsigned x = 0, y = 0, z = 0;
};
extern thread_local mockdev_idx threadIdx, blockIdx;
extern dim3 gridDim, blockDim;
extern std::barrier<> *mockdev_barrier;
inline void __syncthreads() { mockdev_barrier->arrive_and_wait(); }
using std::min;
using std::max;

constexpr size_t kMockLds = size_t(1) << 20;
extern unsigned char fused_lds[kMockLds];

template <typename K, typename... A>
void mockdev_launch(K kernel, dim3 grid, dim3 block, size_t lds, A... args) {
    ASAN_UNPOISON_MEMORY_REGION(fused_lds, kMockLds);
    ASAN_POISON_MEMORY_REGION(fused_lds + lds, kMockLds - lds);
    gridDim = grid;
    blockDim = block;
    // one host thread per work item, reused for every workgroup in turn
    std::barrier<> bar((std::ptrdiff_t)block.x);
    mockdev_barrier = &bar;
    std::vector<std::thread> th;
    for (unsigned tx = 0; tx < block.x; tx++)
        th.emplace_back([&, tx]() {
            threadIdx.x = tx;
            for (unsigned bx = 0; bx < grid.x; bx++) {
                blockIdx.x = bx;
                kernel(args...);
                bar.arrive_and_wait();  // the next workgroup reuses the LDS
            }
        });
    for (auto &t : th) t.join();
    ASAN_UNPOISON_MEMORY_REGION(fused_lds, kMockLds);
}
#define hipLaunchKernelGGL(K, G, B, L, S, ...) mockdev_launch(K, G, B, L, __VA_ARGS__)
