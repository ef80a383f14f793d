// Test double of the HIP runtime interface, for building the library's host runtime and scheduler
// on the CPU (tests/test_scheduler_cpu.py).  Only what that host code uses is declared; the
// definitions, in tests/mock_hip/mock_device.cpp, keep "device" memory in host memory, run the
// kernel launches as small host functions that write stand-in results, and complete events a
// fixed latency after they are recorded, so that launches stay in flight for a while.
#pragma once

#include <cstddef>
#include <cstdint>

#define __host__
#define __device__
#define __global__
#define __shared__
#define __forceinline__ inline

enum hipError_t {
    hipSuccess = 0,
    hipErrorInvalidValue = 1,
    hipErrorOutOfMemory = 2,
    hipErrorLaunchFailure = 719,
    hipErrorNotReady = 600,
};

typedef struct MockStream* hipStream_t;
typedef struct MockEvent* hipEvent_t;

enum hipMemcpyKind {
    hipMemcpyHostToHost = 0,
    hipMemcpyHostToDevice = 1,
    hipMemcpyDeviceToHost = 2,
    hipMemcpyDeviceToDevice = 3,
    hipMemcpyDefault = 4,
};

enum hipDeviceAttribute_t { hipDeviceAttributeMultiprocessorCount = 1 };

constexpr unsigned hipStreamNonBlocking = 1u;
constexpr unsigned hipEventDisableTiming = 2u;
constexpr unsigned hipHostMallocDefault = 0u;

struct float4 { float x, y, z, w; };
struct double4 { double x, y, z, w; };
inline float4 make_float4(float x, float y, float z, float w) { return float4{x, y, z, w}; }
inline double4 make_double4(double x, double y, double z, double w) { return double4{x, y, z, w}; }

hipError_t hipGetDeviceCount(int* n);
hipError_t hipSetDevice(int device);
hipError_t hipDeviceGetAttribute(int* value, hipDeviceAttribute_t attr, int device);
hipError_t hipMemGetInfo(size_t* free_bytes, size_t* total_bytes);
hipError_t hipDeviceSynchronize();
const char* hipGetErrorString(hipError_t e);

hipError_t hipMalloc(void** p, size_t bytes);
hipError_t hipFree(void* p);
hipError_t hipHostMalloc(void** p, size_t bytes, unsigned flags);
hipError_t hipHostFree(void* p);
hipError_t hipMemcpy(void* dst, const void* src, size_t bytes, hipMemcpyKind kind);
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind kind, hipStream_t s);
template <class T>
hipError_t hipMalloc(T** p, size_t bytes) { return hipMalloc((void**)p, bytes); }

hipError_t hipStreamCreate(hipStream_t* s);
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned flags);

hipError_t hipEventCreate(hipEvent_t* e);
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned flags);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventQuery(hipEvent_t e);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float* ms, hipEvent_t start, hipEvent_t stop);
