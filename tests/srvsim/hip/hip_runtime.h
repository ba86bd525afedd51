// Test double of the HIP runtime API subset that the request loop uses, for
// running its host logic on the CPU.  Streams are command queues; one
// "device" thread executes the head commands of the streams in a random
// interleaving that honours stream order and event waits, so that any
// missing cross-stream ordering in the host logic shows up as wrong results.
#pragma once
#include <cstddef>
#include <cstdint>
#include <functional>

typedef int hipError_t;
enum { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorNotReady = 600 };
struct SimStream;
struct SimEvent;
typedef SimStream *hipStream_t;
typedef SimEvent *hipEvent_t;
enum { hipStreamNonBlocking = 1, hipEventDisableTiming = 2, hipHostMallocDefault = 0 };
enum hipMemcpyKind { hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice };

hipError_t hipSetDevice(int);
struct hipDeviceProp_t {
    int multiProcessorCount;
    char gcnArchName[256];
    size_t totalGlobalMem;
};
hipError_t hipGetDeviceCount(int *);
hipError_t hipGetDeviceProperties(hipDeviceProp_t *, int);
hipError_t hipMemcpy(void *, const void *, size_t, hipMemcpyKind);
hipError_t hipDeviceSynchronize();
hipError_t hipStreamCreateWithFlags(hipStream_t *, unsigned);
hipError_t hipStreamSynchronize(hipStream_t);
hipError_t hipStreamDestroy(hipStream_t);
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned);
hipError_t hipMalloc(void **, size_t);
hipError_t hipFree(void *);
hipError_t hipHostMalloc(void **, size_t, unsigned);
hipError_t hipHostFree(void *);
hipError_t hipHostGetDevicePointer(void **, void *, unsigned);
hipError_t hipMemset(void *, int, size_t);
hipError_t hipMemsetAsync(void *, int, size_t, hipStream_t);
hipError_t hipMemcpyAsync(void *, const void *, size_t, hipMemcpyKind, hipStream_t);
hipError_t hipEventCreate(hipEvent_t *);
hipError_t hipEventCreateWithFlags(hipEvent_t *, unsigned);
hipError_t hipEventRecord(hipEvent_t, hipStream_t);
hipError_t hipEventSynchronize(hipEvent_t);
hipError_t hipEventQuery(hipEvent_t);
hipError_t hipEventElapsedTime(float *, hipEvent_t, hipEvent_t);
hipError_t hipEventDestroy(hipEvent_t);
hipError_t hipGetLastError();
hipError_t hipRuntimeGetVersion(int *);
const char *hipGetErrorString(hipError_t);

// Append a command to a stream (the simulated kernels use it).
void sim_enqueue(hipStream_t s, std::function<void()> fn);
