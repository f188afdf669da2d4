// CPU stand-in for the part of the HIP runtime API that the library's host
// code calls (test infrastructure only).  It lets tests/test_host_sanitize.py
// compile csrc/lsm_api.hip with g++ under AddressSanitizer and
// UndefinedBehaviorSanitizer on a machine without a GPU: device memory is
// host memory from malloc (so a sanitizer sees every access the stand-in
// launchers make), stream operations run at once, events read a host clock.
#pragma once
#include <stddef.h>
#include <stdint.h>

#define __host__
#define __device__

typedef enum hipError_t {
  hipSuccess = 0,
  hipErrorInvalidValue = 1,
  hipErrorOutOfMemory = 2,
  hipErrorInvalidDevice = 101,
  hipErrorInvalidSymbol = 13,
  hipErrorNotReady = 600,
} hipError_t;

typedef enum hipMemcpyKind {
  hipMemcpyHostToHost = 0,
  hipMemcpyHostToDevice = 1,
  hipMemcpyDeviceToHost = 2,
  hipMemcpyDeviceToDevice = 3,
  hipMemcpyDefault = 4,
} hipMemcpyKind;

typedef struct ihipStream_t* hipStream_t;
typedef struct ihipEvent_t* hipEvent_t;

#define hipHostMallocDefault 0x0u
#define hipHostMallocMapped 0x2u

hipError_t hipGetDevice(int* dev);
hipError_t hipSetDevice(int dev);
hipError_t hipGetLastError(void);
hipError_t hipMalloc(void** p, size_t bytes);
hipError_t hipFree(void* p);
hipError_t hipHostMalloc(void** p, size_t bytes, unsigned int flags);
hipError_t hipHostFree(void* p);
hipError_t hipHostGetDevicePointer(void** dev, void* host, unsigned int flags);
hipError_t hipMemset(void* p, int value, size_t bytes);
hipError_t hipMemsetAsync(void* p, int value, size_t bytes, hipStream_t s);
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind kind,
                          hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipEventCreate(hipEvent_t* e);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float* ms, hipEvent_t start, hipEvent_t stop);
