// Host-only stand-in for the few HIP runtime declarations that the engine's
// host code uses, so that its control logic (set-up, recovery, batching,
// graph bookkeeping) can be compiled with g++ and run under AddressSanitizer
// on a machine without a GPU.  "Device" memory is host memory; copies are
// memcpy; streams, events and graphs are inert handles.  Test use only.
#pragma once
#include <cstddef>

typedef int hipError_t;
enum { hipSuccess = 0, hipErrorInvalidValue = 1 };
typedef struct mock_stream *hipStream_t;
typedef struct mock_event *hipEvent_t;
typedef struct mock_graph *hipGraph_t;
typedef struct mock_graph_exec *hipGraphExec_t;
enum hipMemcpyKind { hipMemcpyHostToHost, hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice };
enum { hipStreamNonBlocking = 1, hipEventDisableTiming = 2, hipHostMallocDefault = 0 };
typedef enum { hipStreamCaptureModeGlobal, hipStreamCaptureModeThreadLocal, hipStreamCaptureModeRelaxed } hipStreamCaptureMode;
struct hipDeviceProp_t {
    char name[256];
    char gcnArchName[256];
};
struct int2 {
    int x, y;
};
struct int4 {
    int x, y, z, w;
};
inline int2 make_int2(int x, int y) { return int2{x, y}; }
inline int4 make_int4(int x, int y, int z, int w) { return int4{x, y, z, w}; }

hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned flags);
hipError_t hipEventCreate(hipEvent_t *e);
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned flags);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s = nullptr);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b);
hipError_t hipMemcpyAsync(void *dst, const void *src, size_t n, hipMemcpyKind k, hipStream_t s = nullptr);
hipError_t hipHostMalloc(void **p, size_t n, unsigned flags);
hipError_t hipHostFree(void *p);
hipError_t hipGetLastError();
const char *hipGetErrorString(hipError_t e);
hipError_t hipGetDevice(int *d);
hipError_t hipGetDeviceProperties(hipDeviceProp_t *p, int d);
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode m);
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t *g);
hipError_t hipGraphInstantiate(hipGraphExec_t *x, hipGraph_t g, void *, char *, size_t);
hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t s);
hipError_t hipGraphExecDestroy(hipGraphExec_t x);
hipError_t hipGraphDestroy(hipGraph_t g);

// device-symbol stand-ins: a __device__ array is an ordinary host array and
// its "device address" is its host address
#define __device__
#define __align__(n) __attribute__((aligned(n)))
#define HIP_SYMBOL(X) X
hipError_t hipGetSymbolAddress(void **p, const void *symbol);
template <typename T>
hipError_t hipGetSymbolAddress(void **p, const T &symbol) {
    return hipGetSymbolAddress(p, (const void *)&symbol);
}
