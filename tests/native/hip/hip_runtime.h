// Host-only stand-in for the HIP runtime calls of the tile server, so that its
// scheduling logic (admission, FIFO order, completion records) can be tested
// on a machine without a GPU. Memory is host memory; streams complete at once.
#pragma once
#include <atomic>
#include <cstdlib>
#include <cstring>
#include <cstddef>
typedef int hipError_t;
typedef void* hipStream_t;
typedef void* hipEvent_t;
enum { hipSuccess = 0, hipMemcpyDeviceToHost = 2, hipMemcpyDeviceToDevice = 3, hipStreamNonBlocking = 1, hipEventBlockingSync = 1, hipEventDisableTiming = 2 };
inline hipError_t hipGetDevice(int* d) { *d = 0; return 0; }
inline hipError_t hipSetDevice(int) { return 0; }
inline hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) { *s = malloc(1); return 0; }
inline hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { *e = malloc(1); return 0; }
inline hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return 0; }
inline hipError_t hipEventSynchronize(hipEvent_t) { return 0; }
inline hipError_t hipEventDestroy(hipEvent_t e) { free(e); return 0; }
inline hipError_t hipStreamDestroy(hipStream_t s) { free(s); return 0; }
inline hipError_t hipStreamSynchronize(hipStream_t) { return 0; }
// Device memory: host memory, with an optional cap on the number of live
// allocations (0: none) so that out-of-memory paths can be exercised.
inline std::atomic<int>& hip_stub_alloc_cap() { static std::atomic<int> cap{0}; return cap; }
inline std::atomic<int>& hip_stub_live() { static std::atomic<int> live{0}; return live; }
inline hipError_t hipMalloc(void** p, size_t n) {
  const int cap = hip_stub_alloc_cap().load();
  if (cap > 0 && hip_stub_live().load() >= cap) { *p = nullptr; return 2; }
  *p = malloc(n);
  if (!*p) return 2;
  ++hip_stub_live();
  return 0;
}
inline hipError_t hipFree(void* p) {
  if (p) { --hip_stub_live(); free(p); }
  return 0;
}
inline hipError_t hipMemsetAsync(void* p, int v, size_t n, hipStream_t) { memset(p, v, n); return 0; }
inline hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, int, hipStream_t) { memcpy(d, s, n); return 0; }
