/* Host-only stand-in for the few HIP runtime calls the batched and serving
 * executors make, so their scheduling logic can be built with a host compiler
 * (and a thread sanitizer) without a GPU.  Streams are plain tokens. */
#ifndef LEIDEN_HOST_MOCK_HIP_RUNTIME_H
#define LEIDEN_HOST_MOCK_HIP_RUNTIME_H
typedef int hipError_t;
typedef struct mock_stream* hipStream_t;
enum { hipSuccess = 0, hipStreamNonBlocking = 1 };
#ifdef __cplusplus
extern "C" {
#endif
hipError_t hipSetDevice(int device);
hipError_t hipGetDevice(int* device);
hipError_t hipGetDeviceCount(int* count);
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned flags);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipStreamDestroy(hipStream_t s);
#ifdef __cplusplus
}
#endif
#endif
