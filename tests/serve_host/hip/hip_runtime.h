// Host-only stand-in for the HIP runtime calls the serving loop makes, so that
// its scheduler can be compiled and driven on a CPU (fake device).  "Device"
// memory is host memory.  Streams are FIFO queues run in order by one fake
// device thread (fake_device.cpp); events are markers in them.  hipFree and
// hipHostFree wait until every queue is empty, as the real calls synchronise
// the device.  Copies run at once on the calling thread.
#pragma once
#include <cstddef>
#include <cstdlib>
#include <cstring>

typedef int hipError_t;
typedef struct ihipStream_t *hipStream_t;
typedef struct ihipEvent_t *hipEvent_t;
enum { hipSuccess = 0, hipErrorNotReady = 600, hipErrorOutOfMemory = 2 };
enum hipMemcpyKind { hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice };
#define hipStreamNonBlocking 1
#define hipEventDisableTiming 2
#define hipHostMallocDefault 0

inline const char *hipGetErrorString(hipError_t) { return "fake device error"; }
inline hipError_t hipSetDevice(int) { return hipSuccess; }
inline hipError_t hipGetDevice(int *d) { *d = 0; return hipSuccess; }
inline hipError_t hipMemGetInfo(size_t *f, size_t *t) { *f = size_t(1) << 34; *t = *f; return hipSuccess; }
inline hipError_t hipGetLastError() { return hipSuccess; }

hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipStreamQuery(hipStream_t s);
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventQuery(hipEvent_t e);
hipError_t hipFreeVoid(void *p);
hipError_t hipHostFree(void *p);

template <class T>
inline hipError_t hipMalloc(T **p, size_t n) { *p = (T *)std::malloc(n ? n : 1); return *p ? hipSuccess : 2; }
template <class T>
inline hipError_t hipHostMalloc(T **p, size_t n, unsigned) { *p = (T *)std::malloc(n ? n : 1); return *p ? hipSuccess : 2; }
inline hipError_t hipFree(void *p) { return hipFreeVoid(p); }
// stream-ordered allocation: no device-wide synchronisation (the fake frees at once; the scheduler
// only frees buffers whose device work has completed)
template <class T>
inline hipError_t hipMallocAsync(T **p, size_t n, hipStream_t) { *p = (T *)std::malloc(n ? n : 1); return *p ? hipSuccess : 2; }
inline hipError_t hipFreeAsync(void *p, hipStream_t) { std::free(p); return hipSuccess; }
typedef struct ihipMemPool_t *hipMemPool_t;
enum hipMemPoolAttr { hipMemPoolAttrReleaseThreshold = 4 };
inline hipError_t hipDeviceGetDefaultMemPool(hipMemPool_t *p, int) { *p = nullptr; return hipSuccess; }
inline hipError_t hipMemPoolSetAttribute(hipMemPool_t, hipMemPoolAttr, void *) { return hipSuccess; }
inline hipError_t hipMemPoolTrimTo(hipMemPool_t, size_t) { return hipSuccess; }
inline hipError_t hipMemcpy(void *d, const void *s, size_t n, hipMemcpyKind) { std::memcpy(d, s, n); return hipSuccess; }
inline hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind, hipStream_t)
{
    std::memcpy(d, s, n);
    return hipSuccess;
}
