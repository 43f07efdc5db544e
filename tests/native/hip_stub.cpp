// Host implementation of the HIP stand-in (hip_stub/hip/hip_runtime.h) and
// of the kernels' host entry points, for the ThreadSanitizer build of the
// gate.  Nothing here computes: launches are accepted and events complete
// kEventNs after they are recorded, on the host clock.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "kernels/fused.hpp"
#include "kernels/ops.hpp"

namespace {
constexpr int64_t kEventNs = 20000;
struct Event {
  std::mutex mu;
  int64_t ready = 0;   // host time at which it completes; 0: never recorded
};
int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}
}  // namespace

hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipGetDeviceCount(int* n) {
  *n = 1;
  return hipSuccess;
}
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t, int) {
  *v = 256;
  return hipSuccess;
}
hipError_t hipDeviceSynchronize() { return hipSuccess; }
hipError_t hipGetLastError() { return hipSuccess; }
const char* hipGetErrorString(hipError_t) { return "stub"; }
hipError_t hipMalloc(void** p, size_t n) {
  *p = std::calloc(1, n ? n : 1);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void* p) {
  std::free(p);
  return hipSuccess;
}
hipError_t hipMallocAsync(void** p, size_t n, hipStream_t) { return hipMalloc(p, n); }
hipError_t hipFreeAsync(void* p, hipStream_t) { return hipFree(p); }
hipError_t hipHostMalloc(void** p, size_t n, unsigned) { return hipMalloc(p, n); }
hipError_t hipHostFree(void* p) { return hipFree(p); }
hipError_t hipMemset(void* p, int v, size_t n) {
  std::memset(p, v, n);
  return hipSuccess;
}
hipError_t hipMemsetAsync(void* p, int v, size_t n, hipStream_t) { return hipMemset(p, v, n); }
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t) {
  std::memcpy(d, s, n);
  return hipSuccess;
}
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) {
  std::memcpy(d, s, n);
  return hipSuccess;
}
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
  *s = reinterpret_cast<hipStream_t>(new char);
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  delete reinterpret_cast<char*>(s);
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t* e) {
  *e = reinterpret_cast<hipEvent_t>(new Event);
  return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) {
  delete reinterpret_cast<Event*>(e);
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t) {
  Event* ev = reinterpret_cast<Event*>(e);
  std::lock_guard<std::mutex> lk(ev->mu);
  ev->ready = now_ns() + kEventNs;
  return hipSuccess;
}
hipError_t hipEventQuery(hipEvent_t e) {
  Event* ev = reinterpret_cast<Event*>(e);
  std::lock_guard<std::mutex> lk(ev->mu);
  return ev->ready && now_ns() >= ev->ready ? hipSuccess : hipErrorNotReady;
}
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) {
  *ms = 0.01f;
  return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return hipSuccess; }
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t* g) {
  *g = reinterpret_cast<hipGraph_t>(new char);
  return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* ge, hipGraph_t, hipGraphNode_t*, char*, size_t) {
  *ge = reinterpret_cast<hipGraphExec_t>(new char);
  return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipSuccess; }
hipError_t hipGraphDestroy(hipGraph_t g) {
  delete reinterpret_cast<char*>(g);
  return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t g) {
  delete reinterpret_cast<char*>(g);
  return hipSuccess;
}

// ---- kernels' host entry points: accepted, nothing computed
namespace ug {
namespace {
OpPlan one() {
  OpPlan p;
  p.func = reinterpret_cast<const void*>(&one);
  p.grid = dim3(4);
  p.block = dim3(256);
  return p;
}
}  // namespace
OpPlan gemm_f32_plan(int64_t, int64_t, int64_t, bool, int) { return one(); }
hipError_t gemm_f32_launch(const float*, const float*, float*, int64_t, int64_t, int64_t,
                           hipStream_t, unsigned*, int) { return hipSuccess; }
OpPlan conv3x3_f32_plan(int64_t, int64_t, int64_t, int64_t, int) { return one(); }
hipError_t conv3x3_f32_launch(const float*, const float*, float*, int64_t, int64_t, int64_t,
                              int64_t, hipStream_t, unsigned*, int) { return hipSuccess; }
OpPlan bias_relu_f32_plan(int64_t, int64_t, int, bool) { return one(); }
hipError_t bias_relu_f32_launch(const float*, const float*, float*, int64_t, int64_t, int,
                                hipStream_t) { return hipSuccess; }
OpPlan rowsum_f32_plan(int64_t, int64_t) { return one(); }
hipError_t rowsum_f32_launch(const float*, float*, int64_t, int64_t, hipStream_t) { return hipSuccess; }
OpPlan softmax_f32_plan(int64_t, int64_t, bool) { return one(); }
hipError_t softmax_f32_launch(const float*, float*, int64_t, int64_t, hipStream_t) { return hipSuccess; }
OpPlan gemm_fp8_plan(int64_t, int64_t, int64_t) { return one(); }
hipError_t gemm_fp8_launch(const unsigned char*, const unsigned char*, float*, int64_t, int64_t,
                           int64_t, hipStream_t) { return hipSuccess; }
OpPlan vecadd_f32_plan(int64_t, int64_t) { return one(); }
hipError_t vecadd_f32_launch(const float*, const float*, float*, int64_t, int64_t, int64_t,
                             hipStream_t) { return hipSuccess; }
OpPlan conv3x3_bf16_plan(int64_t, int64_t, int64_t) { return one(); }
hipError_t conv3x3_bf16_launch(const uint16_t*, const uint16_t*, float*, int64_t, int64_t,
                               int64_t, hipStream_t, unsigned*) { return hipSuccess; }
OpPlan accum_i32_plan(int64_t) { return one(); }
hipError_t accum_i32_launch(const int*, int*, int64_t, hipStream_t) { return hipSuccess; }
OpPlan gemm_bf16_plan(int64_t, int64_t, int64_t) { return one(); }
hipError_t gemm_bf16_launch(const uint16_t*, const uint16_t*, float*, int64_t, int64_t, int64_t,
                            hipStream_t, unsigned*) { return hipSuccess; }
size_t voxel_f32_workspace(int64_t, int, int) { return 0; }
OpPlan voxel_f32_plan(int64_t, int, int) { return one(); }
hipError_t voxel_f32_launch(const float*, int*, int*, float*, int*, int64_t, int, int, float,
                            float, float, void*, size_t, hipStream_t) { return hipSuccess; }
hipError_t static_scratch(void** p) {
  static char buf[256];
  *p = buf;
  return hipSuccess;
}
hipError_t stream_queue_classes(const std::vector<hipStream_t>& s, std::vector<int>* cls) {
  cls->assign(s.size(), 0);
  for (size_t i = 0; i < s.size(); ++i) (*cls)[i] = static_cast<int>(i % 4);
  return hipSuccess;
}
uint32_t fuse_rows_per_tile(uint32_t, uint32_t, uint32_t) { return 4; }
hipError_t fuse_executor_launch(FuseHost*, FuseDev*, uint32_t, uint32_t, int64_t, int64_t,
                                uint32_t, hipStream_t) { return hipSuccess; }
}  // namespace ug
