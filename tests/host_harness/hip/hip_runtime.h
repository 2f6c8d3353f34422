// Host-only stand-in for the HIP runtime header, used to build the
// library's host layer (argument checks, workspace layout, schedules,
// stream and event logic) as plain C++ under the sanitizers.  Only the
// names that layer uses are declared; "device" memory is host memory.
#pragma once
#include <cstddef>
#include <cstdint>

typedef int hipError_t;
enum : int {
  hipSuccess = 0,
  hipErrorInvalidValue = 1,
  hipErrorOutOfMemory = 2,
};
struct ihipStream_t;
typedef ihipStream_t* hipStream_t;
struct ihipEvent_t;
typedef ihipEvent_t* hipEvent_t;
struct ihipGraph;
typedef ihipGraph* hipGraph_t;
struct hipGraphExec;
typedef hipGraphExec* hipGraphExec_t;
struct hipGraphNode;
typedef hipGraphNode* hipGraphNode_t;

enum hipMemcpyKind {
  hipMemcpyHostToHost = 0,
  hipMemcpyHostToDevice = 1,
  hipMemcpyDeviceToHost = 2,
  hipMemcpyDeviceToDevice = 3,
};
enum hipStreamCaptureStatus {
  hipStreamCaptureStatusNone = 0,
  hipStreamCaptureStatusActive = 1,
  hipStreamCaptureStatusInvalidated = 2,
};
enum hipStreamCaptureMode {
  hipStreamCaptureModeGlobal = 0,
  hipStreamCaptureModeThreadLocal = 1,
  hipStreamCaptureModeRelaxed = 2,
};
#define hipStreamNonBlocking 0x01
#define hipEventDisableTiming 0x02

struct hipFuncAttributes {
  int maxThreadsPerBlock;
};
struct dim3 {
  unsigned x, y, z;
  dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};

hipError_t hipGetDevice(int* d);
hipError_t hipMallocBytes(void** p, size_t bytes);
template <class T>
inline hipError_t hipMalloc(T** p, size_t bytes) {
  void* q = nullptr;
  hipError_t e = hipMallocBytes(&q, bytes);
  *p = static_cast<T*>(q);
  return e;
}
hipError_t hipFree(void* p);
hipError_t hipHostMalloc(void** p, size_t bytes, unsigned flags);
hipError_t hipHostFree(void* p);
hipError_t hipMemcpy(void* dst, const void* src, size_t bytes, hipMemcpyKind k);
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes,
                          hipMemcpyKind k, hipStream_t st);
hipError_t hipDeviceSynchronize();
hipError_t hipEventCreate(hipEvent_t* e);
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned flags);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t st);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b);
hipError_t hipStreamCreateWithFlags(hipStream_t* st, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t st);
hipError_t hipStreamSynchronize(hipStream_t st);
hipError_t hipStreamWaitEvent(hipStream_t st, hipEvent_t e, unsigned flags);
hipError_t hipStreamBeginCapture(hipStream_t st, hipStreamCaptureMode mode);
hipError_t hipStreamIsCapturing(hipStream_t st, hipStreamCaptureStatus* s);
hipError_t hipStreamEndCapture(hipStream_t st, hipGraph_t* g);
hipError_t hipGraphInstantiate(hipGraphExec_t* ex, hipGraph_t g,
                               hipGraphNode_t* err_node, char* log,
                               size_t log_size);
hipError_t hipGraphLaunch(hipGraphExec_t ex, hipStream_t st);
hipError_t hipGraphDestroy(hipGraph_t g);
hipError_t hipGraphExecDestroy(hipGraphExec_t ex);
hipError_t hipFuncGetAttributes(hipFuncAttributes* a, const void* f);
// device variables are host variables here; a symbol's address is its own
#define __device__
#define __align__(n) alignas(n)
#define HIP_SYMBOL(X) (&(X))
hipError_t hipGetSymbolAddress(void** p, const void* symbol);
