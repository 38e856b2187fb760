// Inert host implementation of the declarations in mock/hip/hip_runtime.h
// (test use only): handles are heap objects so that AddressSanitizer sees
// use-after-destroy and leaks; copies are plain memcpy.
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "hip/hip_runtime.h"

struct mock_stream {
    int capturing = 0;
};
struct mock_event {
    int recorded = 0;
};
struct mock_graph {
    int n = 0;
};
struct mock_graph_exec {
    int n = 0;
};

int g_mock_captures = 0, g_mock_launches = 0;

hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) {
    *s = new mock_stream();
    return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
    delete s;
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) {
    if (s && s->capturing) return hipErrorInvalidValue;
    return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned) {
    if (!e) return hipErrorInvalidValue;
    (void)s;
    return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t *e) {
    *e = new mock_event();
    return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) {
    delete e;
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t) {
    if (!e) return hipErrorInvalidValue;
    e->recorded = 1;
    return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e) { return e ? hipSuccess : hipErrorInvalidValue; }
hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b) {
    if (!a || !b) return hipErrorInvalidValue;
    *ms = 0.001f;
    return hipSuccess;
}
hipError_t hipMemcpyAsync(void *dst, const void *src, size_t n, hipMemcpyKind, hipStream_t) {
    if (n) std::memcpy(dst, src, n);
    return hipSuccess;
}
hipError_t hipHostMalloc(void **p, size_t n, unsigned) {
    *p = std::calloc(1, n ? n : 1);
    return *p ? hipSuccess : hipErrorInvalidValue;
}
hipError_t hipHostFree(void *p) {
    std::free(p);
    return hipSuccess;
}
hipError_t hipGetLastError() { return hipSuccess; }
const char *hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "mock error"; }
hipError_t hipGetSymbolAddress(void **p, const void *symbol) {
    *p = const_cast<void *>(symbol);
    return hipSuccess;
}
hipError_t hipGetDevice(int *d) {
    *d = 0;
    return hipSuccess;
}
hipError_t hipGetDeviceProperties(hipDeviceProp_t *p, int) {
    std::memset(p, 0, sizeof(*p));
    std::strcpy(p->name, "mock");
    std::strcpy(p->gcnArchName, "mock");
    return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
    s->capturing = 1;
    g_mock_captures++;
    return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t *g) {
    s->capturing = 0;
    *g = new mock_graph();
    return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t *x, hipGraph_t g, void *, char *, size_t) {
    if (!g) return hipErrorInvalidValue;
    *x = new mock_graph_exec();
    return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t) {
    if (!x) return hipErrorInvalidValue;
    g_mock_launches++;
    return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t x) {
    delete x;
    return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
    delete g;
    return hipSuccess;
}
