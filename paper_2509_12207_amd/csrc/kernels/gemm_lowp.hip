// Low-precision GEMMs on the matrix cores of gfx950, FP32 result:
//   FP8:  C[M,N] = A[M,K] B[K,N], A and B in OCP FP8 E4M3 (one byte each);
//   BF16: the same with A and B in bfloat16 (two bytes each).
//
// Operands are K-contiguous: A row-major [M, K], B given transposed as
// Bt [N, K] (row n holds column n of B).  M and N are arbitrary (rows past
// M or N are read from the matrix's first row or zero-filled, and never
// stored).  Workgroups are remapped so each XCD computes a contiguous band
// of output tiles.
//
// Instructions (both wave64, accumulator layout of the other 32x32
// instructions, mfma32_row):
// * v_mfma_scale_f32_32x32x64_f8f6f4, both scale exponents 127 (x1):
//   D[32x32] += A[32x64] B[64x32], 131072 FLOP.  Lane l feeds row (A) or
//   column (B) l % 32 with 32 bytes of K: bytes 32 (l / 32) .. +31 of the
//   64-byte K slice.
// * v_mfma_f32_32x32x16_bf16: D[32x32] += A[32x16] B[16x32], 32768 FLOP.
//   Lane l feeds row / column l % 32 with 8 values of K: k = 8 (l / 32) ..
//   +7.  A 64-byte K slice (32 values) takes two of them: lane l reads 16-
//   byte chunk l / 32 for the first and chunk 2 + l / 32 for the second.
//
// Kernels, all with a 256 x 256 workgroup tile:
//
// * gemm_ring<FP8 | BF16> (rows a multiple of 64 bytes: K % 64 == 0 for
//   FP8, K % 32 == 0 for BF16): eight waves of 128 x 64 (two per SIMD).
//   Global memory goes straight to LDS (global_load_lds_dwordx4) into a
//   ring of four 32 KiB stages, three stages ahead of the matrix cores; the
//   fragments of step s+1 are read from LDS while step s runs.  One barrier
//   a step.  LDS rows are 64 bytes with the four 16-byte chunks of row r
//   XOR-permuted by (r / 4) % 4: a 16-byte read by sixteen consecutive rows
//   then touches all 64 LDS banks once.  The direct-to-LDS loads are issued
//   from inline assembly so that the compiler, which cannot tell them apart
//   from the ring slots being read, does not wait for every load in flight
//   before each LDS read; their completion is waited for explicitly
//   (vmcnt) before each barrier.
//
// * gemm_fp8_kernel (FP8, any K multiple of 16): four waves of 128 x 128;
//   the next 128-byte K step is fetched into registers while the current
//   one, in two padded LDS stages, feeds the matrix cores.
#include "mfma.hpp"
#include "ops.hpp"
#include "signal.hpp"

namespace ug {
namespace {

typedef int i32x8 __attribute__((ext_vector_type(8)));

constexpr int BM = 256, BN = 256;   // workgroup tile
constexpr int BK = 128;             // bytes of K per step
constexpr int LDR = BK + 16;        // LDS row stride (bytes)
constexpr int ROWS = BM + BN;       // LDS rows per stage (A then B)
constexpr int STAGE = ROWS * LDR;   // bytes per stage
constexpr int CHUNKS = ROWS * BK / 16 / 256;   // 16-byte loads per thread per step
constexpr int kXcds = 8;
constexpr int kGroupM = 8;
// s_waitcnt lgkmcnt(0) with the vmcnt and expcnt fields at their maxima
constexpr int kWaitLdsOnly = 15 | (3 << 14) | (7 << 4) | (0 << 8);

// K offset (within a 64-byte slice) of the 8-byte piece p (0..3) of lane
// group g (= lane / 32) of a matrix-core operand.
__device__ __forceinline__ int kpos(int g, int p) { return 32 * g + 8 * p; }

__device__ __forceinline__ void tile_of(int wg, int tiles_m, int tiles_n, int* tm, int* tn) {
  const int total = tiles_m * tiles_n;
  int id = wg;
  if (total % kXcds == 0) id = (wg % kXcds) * (total / kXcds) + wg / kXcds;
  const int group = kGroupM * tiles_n;
  const int first_m = (id / group) * kGroupM;
  const int gm = min(tiles_m - first_m, kGroupM);
  const int r = id % group;
  *tm = first_m + r % gm;
  *tn = r / gm;
}

__device__ __forceinline__ i32x8 load_frag(const unsigned char* row, int g) {
  i32x8 v;
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const int2 w = *reinterpret_cast<const int2*>(row + kpos(g, p));
    v[2 * p] = w.x;
    v[2 * p + 1] = w.y;
  }
  return v;
}

__global__ __launch_bounds__(256, 1) void gemm_fp8_kernel(const unsigned char* __restrict__ A,
                                                          const unsigned char* __restrict__ Bt,
                                                          float* __restrict__ C, int M, int N,
                                                          int K) {
  __shared__ __attribute__((aligned(16))) unsigned char lds[2 * STAGE];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int tiles_m = (M + BM - 1) / BM, tiles_n = (N + BN - 1) / BN;
  int tm, tn;
  tile_of(blockIdx.x, tiles_m, tiles_n, &tm, &tn);
  const int m0 = tm * BM, n0 = tn * BN;

  // global -> register mapping: chunk c = tid + 256 u covers LDS row c / 8
  // (rows 0..255 of A, 256..511 of Bt), bytes 16 (c % 8) of the step, i.e.
  // row rA + 32 u of A (u < 8) or rB + 32 (u - 8) of Bt.  Chunks of rows
  // past M or N, or past K, are zeroed: the loads themselves are
  // unconditional (no branches in the stream).
  const int part = tid & 7;
  const int rA = m0 + (tid >> 3), rB = n0 + (tid >> 3);
  auto fetch = [&](uint4 (&reg)[CHUNKS], int k0) {
    const bool kin = k0 + 16 * part < K;
#pragma unroll
    for (int u = 0; u < CHUNKS; ++u) {
      const bool isa = u < CHUNKS / 2;
      const int row = (isa ? rA : rB) + 32 * (u % (CHUNKS / 2));
      const bool ok = row < (isa ? M : N) && kin;
      // a zeroed chunk reads the first 16 bytes of its matrix (always there:
      // K >= 16), never past the end
      const unsigned char* X = isa ? A : Bt;
      const unsigned char* p = ok ? X + (int64_t)row * K + 16 * part + k0 : X;
      const uint4 v = *reinterpret_cast<const uint4*>(p);
      reg[u] = ok ? v : make_uint4(0, 0, 0, 0);
    }
  };
  auto stash = [&](const uint4 (&reg)[CHUNKS], int stage) {
    unsigned char* base = lds + stage * STAGE;
#pragma unroll
    for (int u = 0; u < CHUNKS; ++u) {
      const int c = tid + 256 * u;
      *reinterpret_cast<uint4*>(base + (c >> 3) * LDR + 16 * (c & 7)) = reg[u];
    }
  };

  f32x16 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = zero16();

  const int g = lane >> 5, r32 = lane & 31;
  auto compute = [&](int stage) {
    const unsigned char* base = lds + stage * STAGE;
#pragma unroll
    for (int kk = 0; kk < BK; kk += 64) {
      i32x8 a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
        a[i] = load_frag(base + (wm * 128 + i * 32 + r32) * LDR + kk, g);
#pragma unroll
      for (int j = 0; j < 4; ++j)
        b[j] = load_frag(base + (BM + wn * 128 + j * 32 + r32) * LDR + kk, g);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a[i], b[j], acc[i][j], 0, 0,
                                                                      0, 127, 0, 127);
      // keep each 64-byte slice's operands live on their own (64 VGPRs)
      __builtin_amdgcn_sched_barrier(0);
    }
  };

  // the next step is fetched into registers while the current one, in LDS,
  // feeds the matrix cores
  const int steps = (K + BK - 1) / BK;
  uint4 reg[CHUNKS];
  fetch(reg, 0);
  stash(reg, 0);
  __syncthreads();
  for (int s = 0; s < steps; ++s) {
    if (s + 1 < steps) fetch(reg, (s + 1) * BK);
    compute(s & 1);
    if (s + 1 < steps) stash(reg, (s + 1) & 1);
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int col = n0 + wn * 128 + j * 32 + r32;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = m0 + wm * 128 + i * 32 + mfma32_row(r, lane);
        if (row < M && col < N) C[(int64_t)row * N + col] = acc[i][j][r];
      }
    }
}


// ------------------------------------------------------------ ring kernel
constexpr int RK = 64;                       // bytes of K per step
constexpr int RNST = 4;                      // ring stages
constexpr int RSTAGE = (BM + BN) * RK;       // 32 KiB per stage
constexpr int RWAVES = 8;
constexpr int RCPT = (BM + BN) * RK / 16 / (64 * RWAVES);   // 16-byte loads per lane per stage
constexpr int RNF = 2;                       // B fragments per wave (wave tile 128 x 64)
enum RingType { kRingFp8 = 0, kRingBf16 = 1 };

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ int ring_swz(int row) { return (row >> 2) & 3; }

// s_waitcnt vmcnt(N): all but this wave's N most recent ring loads are in LDS
template <int N>
__device__ __forceinline__ void ring_wait_loads() {
  asm volatile("s_waitcnt vmcnt(%0)" ::"i"(N) : "memory");
}

// One 16-byte direct-to-LDS load: lane l writes LDS bytes [lds + 16 l, +16).
// M0 holds the wave's LDS base; one wait state between writing M0 and the
// load that reads it.  M0 has no other use in these kernels.
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"
__device__ __forceinline__ void ring_load16(const unsigned char* g, unsigned lds) {
  asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off" ::"v"(g), "s"(lds)
               : "memory", "m0");
}
#pragma clang diagnostic pop

// The two 16-byte chunks of a 64-byte K slice that lane group g (= lane /
// 32) feeds to the matrix cores.
template <int T>
__device__ __forceinline__ int ring_chunk(int g, int h) {
  return T == kRingFp8 ? 2 * g + h : g + 2 * h;
}

__device__ __forceinline__ bf16x8 as_bf16x8(int4 v) { return __builtin_bit_cast(bf16x8, v); }

// 64 zero bytes: the K slice of a pixel outside the image (3x3 convolution)
__device__ __attribute__((aligned(64))) unsigned char kZeroSlice[64];

// Operands: A and Bt as bytes, `kb` bytes per row (a multiple of 64).
// CONV (BF16 only): the 3x3 convolution as an implicit GEMM on NHWC
// activations `Bt` ([H, W, Cc]) and OHWI weights `A` ([M, 3, 3, Cc], i.e.
// rows of kb = 18 Cc bytes): M output channels, N = H W pixels, and K slice
// s = (tap, 32-channel group) of a pixel row read at the pixel shifted by the
// tap (zero slice outside the image).
template <int T, bool CONV = false>
__global__ __launch_bounds__(64 * RWAVES, 1) void gemm_ring(const unsigned char* __restrict__ A,
                                                            const unsigned char* __restrict__ Bt,
                                                            float* __restrict__ C, int M, int N,
                                                            int kb, int H = 0, int W = 0,
                                                            int Cc = 0, unsigned* sig = nullptr) {
  __shared__ __attribute__((aligned(1024))) unsigned char lds[RNST * RSTAGE];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 2, wn = wave & 3;   // 2 x 4 waves
  const int tiles_m = (M + BM - 1) / BM, tiles_n = (N + BN - 1) / BN;
  int tm, tn;
  tile_of(blockIdx.x, tiles_m, tiles_n, &tm, &tn);
  const int m0 = tm * BM, n0 = tn * BN;
  const int steps = kb / RK;

  // A stage is 512 rows (256 of A, then 256 of Bt) of 64 bytes = 2048
  // chunks; load i of wave w fills the 1 KiB block w * RCPT + i, lane l the
  // chunk q = 64 (w RCPT + i) + l: row q / 4, stored chunk q % 4, which
  // holds K chunk (q % 4) ^ ring_swz(row).  Rows past M or N read the
  // matrix's first row (never stored).
  const unsigned char* src[RCPT];
  int py[RCPT], px[RCPT], kcs[RCPT];   // convolution: this lane's pixels
#pragma unroll
  for (int i = 0; i < RCPT; ++i) {
    const int q = (wave * RCPT + i) * 64 + lane;
    const int row = q >> 2, kc = (q & 3) ^ ring_swz(row);
    const bool isa = row < BM;
    const int grow = isa ? m0 + row : n0 + (row - BM);
    const bool ok = grow < (isa ? M : N);
    const unsigned char* X = isa ? A : Bt;
    src[i] = (ok ? X + (int64_t)grow * kb : X) + 16 * kc;
    if constexpr (CONV) {
      // pixel rows past the image get y = -2: outside for every tap
      py[i] = ok ? grow / W : -2;
      px[i] = ok ? grow % W : 0;
      kcs[i] = kc;
    }
  }
  const int groups = CONV ? Cc / 32 : 1;   // 32-channel groups per tap
  // Stages past the end re-load the last K slice into their own slot, which
  // is never read again: every step issues the same number of loads, so the
  // wait counts are constants.
  auto issue = [&](int step) {
    const int slot = step % RNST;
    const int sc = min(step, steps - 1);
    const int k0 = sc * RK;
    const int tap = sc / groups, grp = sc - tap * groups;
    const int dy = tap / 3 - 1, dx = tap % 3 - 1;
#pragma unroll
    for (int i = 0; i < RCPT; ++i) {
      const unsigned at = (unsigned)(uintptr_t)(lds + slot * RSTAGE + (wave * RCPT + i) * 1024);
      const unsigned char* g = src[i] + k0;
      if constexpr (CONV) {
        if (wave * RCPT + i >= BM / 16) {   // activation rows (wave-uniform)
          const int yy = py[i] + dy, xx = px[i] + dx;
          g = (yy >= 0 && yy < H && xx >= 0 && xx < W)
                  ? Bt + (((int64_t)yy * W + xx) * Cc + grp * 32) * 2 + 16 * kcs[i]
                  : kZeroSlice + 16 * kcs[i];
        }
      }
      ring_load16(g, __builtin_amdgcn_readfirstlane(at));
    }
  };

  f32x16 acc[4][RNF];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < RNF; ++j) acc[i][j] = zero16();

  // fragment of the 32 rows from `row0`: this lane's row, its two K chunks
  // (row0 is a multiple of 32, so row0 + r32 has the swizzle of r32)
  const int g = lane >> 5, r32 = lane & 31;
  const int c0 = 16 * (ring_chunk<T>(g, 0) ^ ring_swz(r32));
  const int c1 = 16 * (ring_chunk<T>(g, 1) ^ ring_swz(r32));
  auto frag = [&](const unsigned char* base, int row0) {
    const unsigned char* r = base + (row0 + r32) * RK;
    const int4 x = *reinterpret_cast<const int4*>(r + c0);
    const int4 y = *reinterpret_cast<const int4*>(r + c1);
    i32x8 v;
    v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
    v[4] = y.x; v[5] = y.y; v[6] = y.z; v[7] = y.w;
    return v;
  };
  auto read = [&](int step, i32x8 (&a)[4], i32x8 (&b)[RNF]) {
    const unsigned char* base = lds + (step % RNST) * RSTAGE;
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = frag(base, wm * 128 + i * 32);
#pragma unroll
    for (int j = 0; j < RNF; ++j) b[j] = frag(base, BM + wn * 64 + j * 32);
  };
  auto multiply = [&](const i32x8 (&a)[4], const i32x8 (&b)[RNF]) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < RNF; ++j) {
        if constexpr (T == kRingFp8) {
          acc[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a[i], b[j], acc[i][j], 0, 0,
                                                                      0, 127, 0, 127);
        } else {
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int4 x = {a[i][4 * h], a[i][4 * h + 1], a[i][4 * h + 2], a[i][4 * h + 3]};
            const int4 y = {b[j][4 * h], b[j][4 * h + 1], b[j][4 * h + 2], b[j][4 * h + 3]};
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(x), as_bf16x8(y),
                                                                acc[i][j], 0, 0, 0);
          }
        }
      }
  };
  // Step s: wait until stage s+1 is in LDS for every wave (this wave's loads
  // but the two latest stages, then the barrier) and this wave's reads of
  // stage s are done; refill the slot of stage s (its fragments are in
  // registers) with stage s+4; read stage s+1 (past the end: stale bytes,
  // never used); multiply stage s.
  auto step = [&](int s, const i32x8 (&ca)[4], const i32x8 (&cb)[RNF], i32x8 (&na)[4],
                  i32x8 (&nb)[RNF]) {
    ring_wait_loads<2 * RCPT>();
    __builtin_amdgcn_s_waitcnt(kWaitLdsOnly);
    asm volatile("s_barrier" ::: "memory");
    issue(s + RNST);
    read(s + 1, na, nb);
    multiply(ca, cb);
  };

  for (int s = 0; s < RNST; ++s) issue(s);
  ring_wait_loads<3 * RCPT>();
  asm volatile("s_barrier" ::: "memory");
  i32x8 a0[4], b0[RNF], a1[4], b1[RNF];
  read(0, a0, b0);
  for (int s = 0; s < steps; s += 2) {
    step(s, a0, b0, a1, b1);
    if (s + 1 < steps) step(s + 1, a1, b1, a0, b0);
  }
  // no load may still be writing LDS when the workgroup ends
  ring_wait_loads<0>();

#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < RNF; ++j) {
      const int col = n0 + wn * 64 + j * 32 + r32;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = m0 + wm * 128 + i * 32 + mfma32_row(r, lane);
        if (row < M && col < N) C[(int64_t)row * N + col] = acc[i][j][r];
      }
    }
  group_done(sig);
}

}  // namespace

OpPlan gemm_fp8_plan(int64_t M, int64_t N, int64_t K) {
  OpPlan p;
  const bool ring = K % RK == 0;
  p.func = ring ? reinterpret_cast<const void*>(&gemm_ring<kRingFp8>)
                : reinterpret_cast<const void*>(&gemm_fp8_kernel);
  p.grid = dim3((unsigned)(((M + BM - 1) / BM) * ((N + BN - 1) / BN)));
  p.block = dim3(ring ? 64 * RWAVES : 256);
  return p;
}

hipError_t gemm_fp8_launch(const unsigned char* A, const unsigned char* Bt, float* C, int64_t M,
                           int64_t N, int64_t K, hipStream_t s) {
  OpPlan p = gemm_fp8_plan(M, N, K);
  if (K % RK == 0)
    hipLaunchKernelGGL(gemm_ring<kRingFp8>, p.grid, p.block, 0, s, A, Bt, C, (int)M, (int)N,
                       (int)K);
  else
    hipLaunchKernelGGL(gemm_fp8_kernel, p.grid, p.block, 0, s, A, Bt, C, (int)M, (int)N, (int)K);
  return hipGetLastError();
}

OpPlan gemm_bf16_plan(int64_t M, int64_t N, int64_t K) {
  (void)K;
  OpPlan p;
  p.func = reinterpret_cast<const void*>(&gemm_ring<kRingBf16>);
  p.grid = dim3((unsigned)(((M + BM - 1) / BM) * ((N + BN - 1) / BN)));
  p.block = dim3(64 * RWAVES);
  return p;
}

hipError_t gemm_bf16_launch(const uint16_t* A, const uint16_t* Bt, float* C, int64_t M,
                            int64_t N, int64_t K, hipStream_t s, unsigned* sig) {
  OpPlan p = gemm_bf16_plan(M, N, K);
  hipLaunchKernelGGL(gemm_ring<kRingBf16>, p.grid, p.block, 0, s,
                     reinterpret_cast<const unsigned char*>(A),
                     reinterpret_cast<const unsigned char*>(Bt), C, (int)M, (int)N, (int)(2 * K),
                     0, 0, 0, sig);
  return hipGetLastError();
}

OpPlan conv3x3_bf16_plan(int64_t C, int64_t H, int64_t W) {
  OpPlan p;
  p.func = reinterpret_cast<const void*>(&gemm_ring<kRingBf16, true>);
  p.grid = dim3((unsigned)(((C + BM - 1) / BM) * ((H * W + BN - 1) / BN)));
  p.block = dim3(64 * RWAVES);
  return p;
}

hipError_t conv3x3_bf16_launch(const uint16_t* X, const uint16_t* Wt, float* Y, int64_t C,
                               int64_t H, int64_t W, hipStream_t s, unsigned* sig) {
  OpPlan p = conv3x3_bf16_plan(C, H, W);
  hipLaunchKernelGGL((gemm_ring<kRingBf16, true>), p.grid, p.block, 0, s,
                     reinterpret_cast<const unsigned char*>(Wt),
                     reinterpret_cast<const unsigned char*>(X), Y, (int)C, (int)(H * W),
                     (int)(18 * C), (int)H, (int)W, (int)C, sig);
  return hipGetLastError();
}

}  // namespace ug
