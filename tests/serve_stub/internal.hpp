// Host-only stand-in for the library's internal header, used to test the
// serving runtime's admission, ring and completion logic on the CPU.  The
// HIP calls the runtime makes are replaced by host functions: copies are
// memcpy, streams and events are no-ops, and the batched search writes one
// candidate per spectrum whose `bin` is the spectrum's first value.
#pragma once
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "pulscan.h"

typedef int hipError_t;
typedef void *hipStream_t;
typedef void *hipEvent_t;
enum { hipSuccess = 0, hipErrorOutOfMemory = 2 };
enum hipMemcpyKind { hipMemcpyHostToDevice, hipMemcpyDeviceToHost };
#define hipEventDisableTiming 0
#define hipHostMallocDefault 0

inline hipError_t hipSetDevice(int) { return hipSuccess; }
inline hipError_t hipGetLastError() { return hipSuccess; }
inline hipError_t hipDeviceSynchronize() { return hipSuccess; }
inline hipError_t hipStreamCreate(hipStream_t *s) { *s = malloc(1); return hipSuccess; }
inline hipError_t hipStreamDestroy(hipStream_t s) { free(s); return hipSuccess; }
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipEventCreateWithFlags(hipEvent_t *e, int) { *e = malloc(1); return hipSuccess; }
inline hipError_t hipEventDestroy(hipEvent_t e) { free(e); return hipSuccess; }
inline hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
inline hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
inline hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
inline hipError_t hipMalloc(void **p, size_t n) {
  *p = malloc(n ? n : 1);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
inline hipError_t hipFree(void *p) { free(p); return hipSuccess; }
// free device memory: PULSCAN_STUB_FREE_MIB MiB (default 16 GiB), half the total
inline hipError_t hipMemGetInfo(size_t *f, size_t *t) {
  const char *e = getenv("PULSCAN_STUB_FREE_MIB");
  const size_t mib = e ? (size_t)strtoull(e, nullptr, 10) : ((size_t)16 << 10);
  *f = mib << 20;
  *t = 2 * *f;
  return hipSuccess;
}
inline hipError_t hipHostMalloc(void **p, size_t n, int) { return hipMalloc(p, n); }
inline hipError_t hipHostFree(void *p) { free(p); return hipSuccess; }
inline hipError_t hipMemcpy(void *d, const void *s, size_t n, hipMemcpyKind) {
  memcpy(d, s, n);
  return hipSuccess;
}
inline hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind k, hipStream_t) {
  return hipMemcpy(d, s, n, k);
}
