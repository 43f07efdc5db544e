// Which streams share a hardware queue.
//
// HIP multiplexes streams onto a fixed number of hardware queues
// (GPU_MAX_HW_QUEUES, 4 by default) and offers no call to ask or choose which
// one a stream uses; the assignment depends on the process's stream history.
// Two streams share a queue when a kernel on the second cannot start before
// a kernel queued earlier on the first has finished: a one-workgroup kernel
// that sleeps about 0.5 ms on stream a, then a one-workgroup kernel on stream
// b; each writes the device's constant-rate clock when it ends.
#include "ops.hpp"

namespace ug {
namespace {

__global__ void queue_probe_sleep(unsigned long long* t, int iters) {
  for (int i = 0; i < iters; ++i) __builtin_amdgcn_s_sleep(127);
  if (threadIdx.x == 0) t[0] = __builtin_amdgcn_s_memrealtime();
}

__global__ void queue_probe_stamp(unsigned long long* t) {
  if (threadIdx.x == 0) t[0] = __builtin_amdgcn_s_memrealtime();
}

}  // namespace

hipError_t stream_queue_classes(const std::vector<hipStream_t>& s, std::vector<int>* cls) {
  cls->assign(s.size(), -1);
  if (s.empty()) return hipSuccess;
  unsigned long long* d = nullptr;
  hipError_t e = hipMalloc(&d, 2 * sizeof(unsigned long long));
  if (e != hipSuccess) return e;
  std::vector<size_t> rep;  // first stream of each class
  for (size_t i = 0; i < s.size() && e == hipSuccess; ++i) {
    for (size_t c = 0; c < rep.size(); ++c) {
      hipLaunchKernelGGL(queue_probe_sleep, dim3(1), dim3(64), 0, s[rep[c]], d, 150);
      hipLaunchKernelGGL(queue_probe_stamp, dim3(1), dim3(64), 0, s[i], d + 1);
      if ((e = hipGetLastError()) != hipSuccess) break;
      if ((e = hipStreamSynchronize(s[rep[c]])) != hipSuccess) break;
      if ((e = hipStreamSynchronize(s[i])) != hipSuccess) break;
      unsigned long long h[2];
      if ((e = hipMemcpy(h, d, sizeof h, hipMemcpyDeviceToHost)) != hipSuccess) break;
      if (h[1] > h[0]) {  // the stamp waited for the sleeper: same queue
        (*cls)[i] = static_cast<int>(c);
        break;
      }
    }
    if (e == hipSuccess && (*cls)[i] < 0) {
      (*cls)[i] = static_cast<int>(rep.size());
      rep.push_back(i);
    }
  }
  const hipError_t f = hipFree(d);
  return e != hipSuccess ? e : f;
}

}  // namespace ug
