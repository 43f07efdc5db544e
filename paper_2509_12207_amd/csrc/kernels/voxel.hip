// Bird's-eye-view pillar binning of a point cloud (FP32 points -> int cells).
//
// Three launches on the caller's stream:
//   1. init:     count = 0, zmax = key(-inf), first = INT_MAX for every cell;
//   2. scatter:  one lane per point (float4 load): cell index, then three
//                order-independent atomics on its cell (count += 1, max of
//                the z key, min of the point index);
//   3. finalize: decode the z key back to float, empty cells' first = -1.
// zmax is kept as an order-preserving unsigned key of the float during the
// scatter so that a plain unsigned atomic max implements the float maximum
// (with -0 < +0).  Every output is independent of the atomics' order.
#include <climits>

#include "ops.hpp"

namespace ug {
namespace {

__device__ __forceinline__ unsigned zkey(float z) {
  const unsigned u = __float_as_uint(z);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float zval(unsigned k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

__global__ __launch_bounds__(256) void voxel_init(int* __restrict__ count,
                                                  unsigned* __restrict__ zk,
                                                  int* __restrict__ first, int64_t G) {
  const unsigned kneg = 0x007fffffu;  // key of -inf
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < G; i += stride) {
    count[i] = 0;
    zk[i] = kneg;
    first[i] = INT_MAX;
  }
}

__global__ __launch_bounds__(256) void voxel_scatter(const float4* __restrict__ pts,
                                                     int* __restrict__ vidx,
                                                     int* __restrict__ count,
                                                     unsigned* __restrict__ zk,
                                                     int* __restrict__ first, int64_t N, int nx,
                                                     int ny, float xmin, float ymin, float scale) {
#pragma clang fp contract(off)
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride) {
    const float4 p = pts[i];
    const float fx = (p.x - xmin) * scale;
    const float fy = (p.y - ymin) * scale;
    int v = -1;
    // NaN fails every comparison and lands outside
    if (fx >= 0.0f && fx < (float)nx && fy >= 0.0f && fy < (float)ny) {
      v = (int)fy * nx + (int)fx;
      atomicAdd(&count[v], 1);
      atomicMax(&zk[v], zkey(p.z));
      atomicMin(&first[v], (int)i);
    }
    vidx[i] = v;
  }
}

__global__ __launch_bounds__(256) void voxel_finalize(const int* __restrict__ count,
                                                      unsigned* __restrict__ zk,
                                                      int* __restrict__ first, int64_t G) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < G; i += stride) {
    // the z key buffer is the caller's float zmax buffer: decode in place
    reinterpret_cast<float*>(zk)[i] = zval(zk[i]);
    if (count[i] == 0) first[i] = -1;
  }
}

unsigned grid_for(int64_t work, int64_t cap) {
  int64_t g = (work + 255) / 256;
  if (g > cap) g = cap;
  if (g < 1) g = 1;
  return (unsigned)g;
}

}  // namespace

OpPlan voxel_f32_plan(int64_t N) {
  OpPlan p;
  p.func = reinterpret_cast<const void*>(&voxel_scatter);
  p.grid = dim3(grid_for(N, 256 * 32));
  p.block = dim3(256);
  return p;
}

hipError_t voxel_f32_launch(const float* pts, int* vidx, int* count, float* zmax, int* first,
                            int64_t N, int nx, int ny, float xmin, float ymin, float scale,
                            hipStream_t s) {
  const int64_t G = (int64_t)nx * ny;
  unsigned* zk = reinterpret_cast<unsigned*>(zmax);
  const dim3 blk(256);
  hipLaunchKernelGGL(voxel_init, dim3(grid_for(G, 256 * 8)), blk, 0, s, count, zk, first, G);
  if (N > 0) {
    OpPlan p = voxel_f32_plan(N);
    hipLaunchKernelGGL(voxel_scatter, p.grid, p.block, 0, s,
                       reinterpret_cast<const float4*>(pts), vidx, count, zk, first, N, nx, ny,
                       xmin, ymin, scale);
  }
  hipLaunchKernelGGL(voxel_finalize, dim3(grid_for(G, 256 * 8)), blk, 0, s, count, zk, first, G);
  return hipGetLastError();
}

}  // namespace ug
