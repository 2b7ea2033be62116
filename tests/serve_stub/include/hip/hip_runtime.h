// Host-only stand-in for the HIP runtime header, for building the serving
// runtime (rt_serve.cpp) on the CPU against a simulated device
// (stub_device.cpp) under ThreadSanitizer.  Only what the server and the
// library's internal header name is declared; test infrastructure only.
#pragma once

#include <cstddef>
#include <cstdint>

typedef int hipError_t;
enum : int { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorNotReady = 600 };

typedef struct StubStream* hipStream_t;
typedef struct StubEvent* hipEvent_t;

#define hipStreamNonBlocking 0x01u
#define hipEventDisableTiming 0x02u

struct float2 {
    float x, y;
};
struct float4 {
    float x, y, z, w;
};

hipError_t hipGetDevice(int* device);
hipError_t hipSetDevice(int device);
hipError_t hipStreamCreateWithFlags(hipStream_t* stream, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t stream);
hipError_t hipStreamSynchronize(hipStream_t stream);
hipError_t hipEventCreateWithFlags(hipEvent_t* event, unsigned flags);
hipError_t hipEventDestroy(hipEvent_t event);
hipError_t hipEventRecord(hipEvent_t event, hipStream_t stream);
hipError_t hipEventQuery(hipEvent_t event);
const char* hipGetErrorString(hipError_t e);
