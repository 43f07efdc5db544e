// Completion counter of a contraction for the tail executor (fused.hpp):
// every wavefront adds one once all its stores are out, so the counter
// reaches (workgroups x wavefronts per workgroup) when the kernel's output is
// complete.  A null counter costs one comparison.
#pragma once

#include <hip/hip_runtime.h>

namespace ug {

__device__ __forceinline__ void wave_done(unsigned* sig) {
  if (sig == nullptr) return;
  __threadfence();   // this wavefront's stores, before its count
  if ((threadIdx.x & 63) == 0)
    __hip_atomic_fetch_add(sig, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace ug
