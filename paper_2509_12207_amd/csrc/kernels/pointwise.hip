// HBM-bound kernels: bias + ReLU, row sum, row softmax (FP32).
//
// All three stream their input once and write their output once.  Accesses
// are float4 per lane where rows allow it, consecutive lanes touching
// consecutive 16-byte words; reductions are wavefront shuffles (plus one LDS
// exchange across the waves of a workgroup), in a fixed order, so results are
// reproducible run to run.
#include "ops.hpp"

namespace ug {
namespace {

// Streaming 16-byte accesses (nontemporal): they do not allocate in the
// caches, which pays for tensors far larger than L2 and the Infinity Cache
// (each byte is touched once); smaller tensors keep the cached path so that
// the next kernel of the task finds its input there.
typedef float f32x4v __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 load_stream(const float4* p) {
  const f32x4v v = __builtin_nontemporal_load(reinterpret_cast<const f32x4v*>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void store_stream(float4* p, float4 v) {
  const f32x4v w = {v.x, v.y, v.z, v.w};
  __builtin_nontemporal_store(w, reinterpret_cast<f32x4v*>(p));
}
template <bool NT>
__device__ __forceinline__ float4 ld4(const float4* p) {
  return NT ? load_stream(p) : *p;
}
template <bool NT>
__device__ __forceinline__ void st4(float4* p, float4 v) {
  if (NT) store_stream(p, v); else *p = v;
}

// ---------------------------------------------------------------- bias+ReLU
// y = s > 0 ? s : +0 with s = x + b (one FP32 add; -0 and NaN give +0).
__device__ __forceinline__ float relu_add(float x, float b) {
  const float s = x + b;
  return s > 0.0f ? s : 0.0f;
}

// axis 0: b[C] per column; axis 1: b[R] per row.  Vector path: C % 4 == 0.
// Each thread keeps UNROLL independent float4 loads in flight (consecutive
// lanes on consecutive 16-byte words); the row/column of a float4 comes from
// a 32-bit division when the tensor has fewer than 2^32 float4 (always in
// practice), avoiding 64-bit division in the stream.
constexpr int UNROLL = 4;

template <int AXIS, typename I>
__device__ __forceinline__ float4 bias_relu4(const float4 x, const float* __restrict__ b, I i,
                                             I c4) {
  if (AXIS == 0) {
    const float4 bb = reinterpret_cast<const float4*>(b)[i % c4];
    return make_float4(relu_add(x.x, bb.x), relu_add(x.y, bb.y), relu_add(x.z, bb.z),
                       relu_add(x.w, bb.w));
  }
  const float bb = b[i / c4];
  return make_float4(relu_add(x.x, bb), relu_add(x.y, bb), relu_add(x.z, bb), relu_add(x.w, bb));
}

template <int AXIS, typename I, bool NT>
__global__ __launch_bounds__(256) void bias_relu_vec(const float4* __restrict__ X,
                                                     const float* __restrict__ b,
                                                     float4* __restrict__ Y, I n, I c4) {
  const I stride = (I)gridDim.x * 256 * UNROLL;
  for (I base = (I)blockIdx.x * 256 * UNROLL + threadIdx.x; base < n; base += stride) {
    float4 x[UNROLL];
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
      const I i = base + (I)u * 256;
      if (i < n) x[u] = ld4<NT>(X + i);
    }
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
      const I i = base + (I)u * 256;
      if (i < n) st4<NT>(Y + i, bias_relu4<AXIS>(x[u], b, i, c4));
    }
  }
}

template <int AXIS>
__global__ __launch_bounds__(256) void bias_relu_scalar(const float* __restrict__ X,
                                                        const float* __restrict__ b,
                                                        float* __restrict__ Y, int64_t R,
                                                        int64_t C) {
  const int64_t n = R * C;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    Y[i] = relu_add(X[i], AXIS == 0 ? b[i % C] : b[i / C]);
}

// ---------------------------------------------------------------- reductions
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
  return v;
}

// One wave per row (4 rows per workgroup): rows of up to a few thousand.
__global__ __launch_bounds__(256) void rowsum_wave(const float* __restrict__ Z,
                                                   float* __restrict__ r, int64_t R, int64_t C) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= R) return;
  const float* z = Z + row * C;
  float s = 0.f;
  if ((C & 3) == 0 && ((reinterpret_cast<uintptr_t>(z) & 15) == 0)) {
    const float4* z4 = reinterpret_cast<const float4*>(z);
    for (int64_t j = lane; j < C / 4; j += 64) {
      const float4 v = load_stream(z4 + j);
      s += (v.x + v.y) + (v.z + v.w);
    }
  } else {
    for (int64_t j = lane; j < C; j += 64) s += z[j];
  }
  s = wave_sum(s);
  if (lane == 0) r[row] = s;
}

// One workgroup (4 waves) per row: long rows.
__global__ __launch_bounds__(256) void rowsum_block(const float* __restrict__ Z,
                                                    float* __restrict__ r, int64_t R, int64_t C) {
  __shared__ float part[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t row = blockIdx.x;
  const float* z = Z + row * C;
  float s = 0.f;
  if ((C & 3) == 0 && ((reinterpret_cast<uintptr_t>(z) & 15) == 0)) {
    // four independent loads in flight per lane, summed in a fixed order
    const float4* z4 = reinterpret_cast<const float4*>(z);
    const int64_t c4 = C / 4;
    float a[4] = {0.f, 0.f, 0.f, 0.f};
    int64_t j = threadIdx.x;
    for (; j + 768 < c4; j += 1024) {
      float4 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = load_stream(z4 + j + 256 * u);
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] += (v[u].x + v[u].y) + (v[u].z + v[u].w);
    }
    for (; j < c4; j += 256) {
      const float4 v = load_stream(z4 + j);
      a[0] += (v.x + v.y) + (v.z + v.w);
    }
    s = (a[0] + a[1]) + (a[2] + a[3]);
  } else {
    for (int64_t j = threadIdx.x; j < C; j += 256) s += z[j];
  }
  s = wave_sum(s);
  if (lane == 0) part[wave] = s;
  __syncthreads();
  if (threadIdx.x == 0) r[row] = (part[0] + part[1]) + (part[2] + part[3]);
}

// ---------------------------------------------------------------- softmax
// Row held in registers: NV float4 per lane, WAVES waves per row.
template <int WAVES, int NV, bool NT>
__global__ __launch_bounds__(256) void softmax_reg(const float* __restrict__ X,
                                                   float* __restrict__ Y, int64_t R, int64_t L) {
  constexpr int T = WAVES * 64;               // lanes per row
  constexpr int ROWS = 256 / T;               // rows per workgroup
  __shared__ float red[4];
  const int t = threadIdx.x % T;
  const int sub = threadIdx.x / T;
  const int lane = threadIdx.x & 63;
  const int wbase = sub * WAVES;              // first wave of this row
  const int64_t row = (int64_t)blockIdx.x * ROWS + sub;
  const bool live = row < R;
  const float* x = X + row * L;
  float* y = Y + row * L;
  float4 v[NV];
  const int64_t L4 = L / 4;
  float m = -INFINITY;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    const int64_t j = t + (int64_t)i * T;
    if (live && j < L4) {
      v[i] = ld4<NT>(reinterpret_cast<const float4*>(x) + j);
      m = fmaxf(m, fmaxf(fmaxf(v[i].x, v[i].y), fmaxf(v[i].z, v[i].w)));
    } else {
      v[i] = make_float4(-INFINITY, -INFINITY, -INFINITY, -INFINITY);
    }
  }
  m = wave_max(m);
  if (WAVES > 1) {
    if (lane == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    m = red[wbase];
#pragma unroll
    for (int w = 1; w < WAVES; ++w) m = fmaxf(m, red[wbase + w]);
    __syncthreads();
  }
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    v[i].x = expf(v[i].x - m);
    v[i].y = expf(v[i].y - m);
    v[i].z = expf(v[i].z - m);
    v[i].w = expf(v[i].w - m);
    s += (v[i].x + v[i].y) + (v[i].z + v[i].w);
  }
  s = wave_sum(s);
  if (WAVES > 1) {
    if (lane == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    s = red[wbase];
#pragma unroll
    for (int w = 1; w < WAVES; ++w) s += red[wbase + w];
  }
  const float inv = 1.0f / s;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    const int64_t j = t + (int64_t)i * T;
    if (live && j < L4)
      st4<NT>(reinterpret_cast<float4*>(y) + j,
              make_float4(v[i].x * inv, v[i].y * inv, v[i].z * inv, v[i].w * inv));
  }
}

// Any row length: one workgroup per row, three passes over the row.
__global__ __launch_bounds__(256) void softmax_any(const float* __restrict__ X,
                                                   float* __restrict__ Y, int64_t R, int64_t L) {
  __shared__ float red[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const float* x = X + (int64_t)blockIdx.x * L;
  float* y = Y + (int64_t)blockIdx.x * L;
  float m = -INFINITY;
  for (int64_t j = threadIdx.x; j < L; j += 256) m = fmaxf(m, x[j]);
  m = wave_max(m);
  if (lane == 0) red[wave] = m;
  __syncthreads();
  m = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
  __syncthreads();
  float s = 0.f;
  for (int64_t j = threadIdx.x; j < L; j += 256) s += expf(x[j] - m);
  s = wave_sum(s);
  if (lane == 0) red[wave] = s;
  __syncthreads();
  s = (red[0] + red[1]) + (red[2] + red[3]);
  const float inv = 1.0f / s;
  for (int64_t j = threadIdx.x; j < L; j += 256) y[j] = expf(x[j] - m) * inv;
}

unsigned grid_for(int64_t work, int64_t per_block, int64_t cap) {
  int64_t g = (work + per_block - 1) / per_block;
  if (g > cap) g = cap;
  if (g < 1) g = 1;
  return (unsigned)g;
}

}  // namespace

// ---------------------------------------------------------------- launchers
static bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

// Grid-stride kernels: up to 64 workgroups per CU on 256 CUs.
static constexpr int64_t kStreamGridCap = 256 * 64;
// Tensors from this size on are streamed with nontemporal accesses.
static constexpr int64_t kStreamBytes = int64_t(64) << 20;

OpPlan bias_relu_f32_plan(int64_t R, int64_t C, int axis, bool vec) {
  OpPlan p;
  const bool narrow = vec && R * (C / 4) < (int64_t(1) << 32);
  if (vec && narrow)
    p.func = axis == 0 ? reinterpret_cast<const void*>(&bias_relu_vec<0, uint32_t, false>)
                       : reinterpret_cast<const void*>(&bias_relu_vec<1, uint32_t, false>);
  else if (vec)
    p.func = axis == 0 ? reinterpret_cast<const void*>(&bias_relu_vec<0, int64_t, false>)
                       : reinterpret_cast<const void*>(&bias_relu_vec<1, int64_t, false>);
  else
    p.func = axis == 0 ? reinterpret_cast<const void*>(&bias_relu_scalar<0>)
                       : reinterpret_cast<const void*>(&bias_relu_scalar<1>);
  const int64_t work = vec ? R * (C / 4) : R * C;
  p.grid = dim3(grid_for(work, vec ? 256 * UNROLL : 256, kStreamGridCap));
  p.block = dim3(256);
  return p;
}

hipError_t bias_relu_f32_launch(const float* X, const float* b, float* Y, int64_t R, int64_t C,
                                int axis, hipStream_t s) {
  const bool vec = (C % 4 == 0) && aligned16(X) && aligned16(Y) && (axis == 1 || aligned16(b));
  OpPlan p = bias_relu_f32_plan(R, C, axis, vec);
  const int64_t n4 = R * (C / 4), c4 = C / 4;
  const float4* x4 = reinterpret_cast<const float4*>(X);
  float4* y4 = reinterpret_cast<float4*>(Y);
  const bool nt = R * C * 4 >= kStreamBytes;
  if (vec && n4 < (int64_t(1) << 32)) {
    const uint32_t n = (uint32_t)n4, c = (uint32_t)c4;
    if (axis == 0 && nt)
      hipLaunchKernelGGL((bias_relu_vec<0, uint32_t, true>), p.grid, p.block, 0, s, x4, b, y4, n, c);
    else if (axis == 0)
      hipLaunchKernelGGL((bias_relu_vec<0, uint32_t, false>), p.grid, p.block, 0, s, x4, b, y4, n, c);
    else if (nt)
      hipLaunchKernelGGL((bias_relu_vec<1, uint32_t, true>), p.grid, p.block, 0, s, x4, b, y4, n, c);
    else
      hipLaunchKernelGGL((bias_relu_vec<1, uint32_t, false>), p.grid, p.block, 0, s, x4, b, y4, n, c);
  } else if (vec) {
    if (axis == 0)
      hipLaunchKernelGGL((bias_relu_vec<0, int64_t, true>), p.grid, p.block, 0, s, x4, b, y4, n4, c4);
    else
      hipLaunchKernelGGL((bias_relu_vec<1, int64_t, true>), p.grid, p.block, 0, s, x4, b, y4, n4, c4);
  } else {
    if (axis == 0)
      hipLaunchKernelGGL(bias_relu_scalar<0>, p.grid, p.block, 0, s, X, b, Y, R, C);
    else
      hipLaunchKernelGGL(bias_relu_scalar<1>, p.grid, p.block, 0, s, X, b, Y, R, C);
  }
  return hipGetLastError();
}

OpPlan rowsum_f32_plan(int64_t R, int64_t C) {
  OpPlan p;
  p.block = dim3(256);
  if (C <= 2048) {
    p.func = reinterpret_cast<const void*>(&rowsum_wave);
    p.grid = dim3((unsigned)((R + 3) / 4));
  } else {
    p.func = reinterpret_cast<const void*>(&rowsum_block);
    p.grid = dim3((unsigned)R);
  }
  return p;
}

hipError_t rowsum_f32_launch(const float* Z, float* r, int64_t R, int64_t C, hipStream_t s) {
  OpPlan p = rowsum_f32_plan(R, C);
  if (C <= 2048)
    hipLaunchKernelGGL(rowsum_wave, p.grid, p.block, 0, s, Z, r, R, C);
  else
    hipLaunchKernelGGL(rowsum_block, p.grid, p.block, 0, s, Z, r, R, C);
  return hipGetLastError();
}

// Register-resident variants by row length (L % 4 == 0):
//   L <= 256: one wave per row, 1 float4 per lane; <= 1024: one wave, 4;
//   <= 2048: two waves, 4; <= 4096: four waves, 4.
OpPlan softmax_f32_plan(int64_t R, int64_t L, bool vec) {
  OpPlan p;
  p.block = dim3(256);
  if (!vec || L > 4096) {
    p.func = reinterpret_cast<const void*>(&softmax_any);
    p.grid = dim3((unsigned)R);
  } else if (L <= 256) {
    p.func = reinterpret_cast<const void*>(&softmax_reg<1, 1, false>);
    p.grid = dim3((unsigned)((R + 3) / 4));
  } else if (L <= 1024) {
    p.func = reinterpret_cast<const void*>(&softmax_reg<1, 4, false>);
    p.grid = dim3((unsigned)((R + 3) / 4));
  } else if (L <= 2048) {
    p.func = reinterpret_cast<const void*>(&softmax_reg<2, 4, false>);
    p.grid = dim3((unsigned)((R + 1) / 2));
  } else {
    p.func = reinterpret_cast<const void*>(&softmax_reg<4, 4, false>);
    p.grid = dim3((unsigned)R);
  }
  return p;
}

template <int W, int V>
static void launch_softmax_reg(bool nt, const OpPlan& p, hipStream_t s, const float* X, float* Y,
                               int64_t R, int64_t L) {
  if (nt)
    hipLaunchKernelGGL((softmax_reg<W, V, true>), p.grid, p.block, 0, s, X, Y, R, L);
  else
    hipLaunchKernelGGL((softmax_reg<W, V, false>), p.grid, p.block, 0, s, X, Y, R, L);
}

hipError_t softmax_f32_launch(const float* X, float* Y, int64_t R, int64_t L, hipStream_t s) {
  const bool vec = (L % 4 == 0) && aligned16(X) && aligned16(Y);
  OpPlan p = softmax_f32_plan(R, L, vec);
  const bool nt = R * L * 4 >= kStreamBytes;
  if (!vec || L > 4096)
    hipLaunchKernelGGL(softmax_any, p.grid, p.block, 0, s, X, Y, R, L);
  else if (L <= 256)
    launch_softmax_reg<1, 1>(nt, p, s, X, Y, R, L);
  else if (L <= 1024)
    launch_softmax_reg<1, 4>(nt, p, s, X, Y, R, L);
  else if (L <= 2048)
    launch_softmax_reg<2, 4>(nt, p, s, X, Y, R, L);
  else
    launch_softmax_reg<4, 4>(nt, p, s, X, Y, R, L);
  return hipGetLastError();
}

// ------------------------------------------------------------ vector add
// c = a + b over n floats by exactly `w` workgroups of 256 lanes (grid
// stride; float4 accesses when all three arrays are 16-byte aligned), the
// whole pass repeated `r` times (same result).  The custom kernel of the
// sensitivity experiments: its utilisation is w / CUs and its duration
// follows from n r / w, with small buffers.
namespace {
template <bool VEC>
__global__ __launch_bounds__(256) void vecadd_kernel(const float* __restrict__ a,
                                                     const float* __restrict__ b,
                                                     float* __restrict__ c, int64_t n, int r) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  const int64_t first = (int64_t)blockIdx.x * 256 + threadIdx.x;
  for (int rep = 0; rep < r; ++rep) {
    int64_t done = 0;
    if (VEC) {
      const int64_t n4 = n / 4;
      const float4* a4 = reinterpret_cast<const float4*>(a);
      const float4* b4 = reinterpret_cast<const float4*>(b);
      float4* c4 = reinterpret_cast<float4*>(c);
      for (int64_t i = first; i < n4; i += stride) {
        const float4 x = a4[i], y = b4[i];
        c4[i] = make_float4(x.x + y.x, x.y + y.y, x.z + y.z, x.w + y.w);
      }
      done = 4 * n4;
    }
    for (int64_t i = done + first; i < n; i += stride) c[i] = a[i] + b[i];
  }
}
}  // namespace

OpPlan vecadd_f32_plan(int64_t n, int64_t w) {
  (void)n;
  OpPlan p;
  p.func = reinterpret_cast<const void*>(&vecadd_kernel<true>);
  p.grid = dim3((unsigned)w);
  p.block = dim3(256);
  return p;
}

hipError_t vecadd_f32_launch(const float* a, const float* b, float* c, int64_t n, int64_t w,
                             int64_t r, hipStream_t s) {
  const bool vec = ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b) |
                     reinterpret_cast<uintptr_t>(c)) & 15) == 0;
  if (vec)
    hipLaunchKernelGGL(vecadd_kernel<true>, dim3((unsigned)w), dim3(256), 0, s, a, b, c, n,
                       (int)r);
  else
    hipLaunchKernelGGL(vecadd_kernel<false>, dim3((unsigned)w), dim3(256), 0, s, a, b, c, n,
                       (int)r);
  return hipGetLastError();
}


// ------------------------------------------------------------ state += x
// Device-resident chain state: s_i += x_i in int32 (two's-complement
// wrap), four lanes' worth per vector access when both are 16-byte aligned.
namespace {
template <bool Vec>
__global__ __launch_bounds__(256) void accum_i32_kernel(const int* __restrict__ x,
                                                        int* __restrict__ st, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (Vec) {
    const int64_t n4 = n / 4;
    const int4* x4 = reinterpret_cast<const int4*>(x);
    int4* s4 = reinterpret_cast<int4*>(st);
    for (int64_t i = t; i < n4; i += stride) {
      const int4 a = x4[i];
      int4 b = s4[i];
      b.x = (int)((unsigned)b.x + (unsigned)a.x);
      b.y = (int)((unsigned)b.y + (unsigned)a.y);
      b.z = (int)((unsigned)b.z + (unsigned)a.z);
      b.w = (int)((unsigned)b.w + (unsigned)a.w);
      s4[i] = b;
    }
    for (int64_t i = 4 * n4 + t; i < n; i += stride)
      st[i] = (int)((unsigned)st[i] + (unsigned)x[i]);
  } else {
    for (int64_t i = t; i < n; i += stride) st[i] = (int)((unsigned)st[i] + (unsigned)x[i]);
  }
}

unsigned accum_grid(int64_t n) {
  int64_t g = (n / 4 + 255) / 256;
  if (g > 2048) g = 2048;
  return (unsigned)(g < 1 ? 1 : g);
}
}  // namespace

OpPlan accum_i32_plan(int64_t n) {
  OpPlan p;
  p.func = reinterpret_cast<const void*>(&accum_i32_kernel<true>);
  p.grid = dim3(accum_grid(n));
  p.block = dim3(256);
  return p;
}

hipError_t accum_i32_launch(const int* x, int* st, int64_t n, hipStream_t s) {
  const bool vec = ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(st)) & 15) == 0;
  if (vec)
    hipLaunchKernelGGL(accum_i32_kernel<true>, dim3(accum_grid(n)), dim3(256), 0, s, x, st, n);
  else
    hipLaunchKernelGGL(accum_i32_kernel<false>, dim3(accum_grid(n)), dim3(256), 0, s, x, st, n);
  return hipGetLastError();
}

}  // namespace ug
