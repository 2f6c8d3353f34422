// Host-only stand-in for the HIP runtime entry points the library's host
// layer calls.  Work is "complete" as soon as it is enqueued; copies are
// plain memcpy; device memory is host memory, so the sanitizers see every
// access the host layer and the stand-in launchers make.
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <cstring>

struct ihipStream_t { int unused; };
struct ihipEvent_t { int unused; };
struct ihipGraph { int unused; };
struct hipGraphExec { int unused; };

hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
hipError_t hipMallocBytes(void** p, size_t bytes) {
  *p = std::calloc(bytes ? bytes : 1, 1);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void* p) { std::free(p); return hipSuccess; }
hipError_t hipHostMalloc(void** p, size_t bytes, unsigned) { return hipMallocBytes(p, bytes); }
hipError_t hipHostFree(void* p) { std::free(p); return hipSuccess; }
hipError_t hipMemcpy(void* dst, const void* src, size_t bytes, hipMemcpyKind) {
  std::memcpy(dst, src, bytes);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes,
                          hipMemcpyKind, hipStream_t) {
  std::memcpy(dst, src, bytes);
  return hipSuccess;
}
hipError_t hipDeviceSynchronize() { return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t* e) { *e = new ihipEvent_t(); return hipSuccess; }
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) { delete e; return hipSuccess; }
hipError_t hipEventRecord(hipEvent_t e, hipStream_t) { return e ? hipSuccess : hipErrorInvalidValue; }
hipError_t hipEventSynchronize(hipEvent_t e) { return e ? hipSuccess : hipErrorInvalidValue; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
  if (!a || !b) return hipErrorInvalidValue;
  *ms = 0.125f;
  return hipSuccess;
}
hipError_t hipStreamCreateWithFlags(hipStream_t* st, unsigned) {
  *st = new ihipStream_t();
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t st) { delete st; return hipSuccess; }
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t e, unsigned) {
  return e ? hipSuccess : hipErrorInvalidValue;
}
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return hipSuccess; }
hipError_t hipStreamIsCapturing(hipStream_t, hipStreamCaptureStatus* s) {
  *s = hipStreamCaptureStatusNone;
  return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t* g) {
  *g = new ihipGraph();
  return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* ex, hipGraph_t, hipGraphNode_t*,
                               char*, size_t) {
  *ex = new hipGraphExec();
  return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t ex, hipStream_t) {
  return ex ? hipSuccess : hipErrorInvalidValue;
}
hipError_t hipGraphDestroy(hipGraph_t g) { delete g; return hipSuccess; }
hipError_t hipGraphExecDestroy(hipGraphExec_t ex) { delete ex; return hipSuccess; }
hipError_t hipGetSymbolAddress(void** p, const void* symbol) {
  *p = const_cast<void*>(symbol);
  return hipSuccess;
}
hipError_t hipFuncGetAttributes(hipFuncAttributes* a, const void* f) {
  if (!f) return hipErrorInvalidValue;
  a->maxThreadsPerBlock = 1024;
  return hipSuccess;
}
