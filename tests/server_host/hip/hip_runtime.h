// Host-only stand-in for the HIP runtime (test infrastructure): lets the
// solve server, the device-memory cache and the C-ABI glue compile with g++
// so that their threads run under ThreadSanitizer and AddressSanitizer on
// the CPU.  Device memory is host memory; copies are memcpy; a device
// synchronisation sleeps briefly.
#pragma once
#include <cstddef>
#include <cstdlib>
#include <cstring>
#include <thread>
#include <chrono>
#define __device__
#define __host__
#define __global__
#define __forceinline__ inline
typedef int hipError_t;
enum { hipSuccess = 0, hipErrorOutOfMemory = 2 };
typedef struct ihipStream_t *hipStream_t;
typedef enum hipMemcpyKind { hipMemcpyHostToHost, hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice, hipMemcpyDefault } hipMemcpyKind;
#define hipStreamNonBlocking 1
inline hipError_t hipSetDevice(int) { return 0; }
inline hipError_t hipGetDevice(int *d) { *d = 0; return 0; }
inline hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) { *s = (hipStream_t) new char[16]; return 0; }
inline hipError_t hipStreamDestroy(hipStream_t s) { delete[] (char *)s; return 0; }
inline hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind, hipStream_t) { std::memcpy(d, s, n); return 0; }
inline hipError_t hipStreamSynchronize(hipStream_t) { return 0; }
inline hipError_t hipDeviceSynchronize() { std::this_thread::sleep_for(std::chrono::microseconds(200)); return 0; }
inline hipError_t hipMalloc(void **p, size_t n) { *p = std::malloc(n); return *p ? 0 : 2; }
inline hipError_t hipFree(void *p) { std::free(p); return 0; }
inline const char *hipGetErrorString(hipError_t) { return "stub error"; }
inline hipError_t hipGetLastError() { return 0; }
