// C[M,N] = A[M,K] B[K,N] with A and B in OCP FP8 E4M3 and an FP32 result,
// on the FP8 matrix cores of gfx950.
//
// Operands are K-contiguous: A row-major [M, K], B given transposed as
// Bt [N, K] (row n holds column n of B).  K must be a multiple of 16 (one
// 16-byte load); M and N are arbitrary (tails are zero-filled on load and
// masked on store).
//
// v_mfma_scale_f32_32x32x64_f8f6f4 with both scale exponents 127 (x1):
// D[32x32] += A[32x64] B[64x32], 131072 FLOP per instruction.  Lane l feeds
// row (A) or column (B) l % 32 with 32 bytes of K; the K positions of those
// bytes are given by kpos() below.  The accumulator layout is that of the
// other 32x32 instructions (mfma32_row).
//
// Workgroup tile 256 x 256, four waves of 128 x 128 (4 x 4 instructions per
// 64-byte K slice, 256 accumulators per lane).  K advances 128 bytes a step:
// the next step is fetched into registers (16 x 16 bytes a lane, loads
// without branches) while the current one, in LDS, feeds the matrix cores;
// one barrier per step, two LDS stages of 2 x 256 rows x 144 bytes (rows
// padded by 16 bytes so the 16-byte fragment reads of 16 consecutive rows
// hit distinct banks).  Workgroups are remapped so each XCD computes a
// contiguous band of output tiles.
#include "mfma.hpp"
#include "ops.hpp"

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

}  // namespace

OpPlan gemm_fp8_plan(int64_t M, int64_t N, int64_t K) {
  (void)K;
  OpPlan p;
  p.func = reinterpret_cast<const void*>(&gemm_fp8_kernel);
  p.grid = dim3((unsigned)(((M + BM - 1) / BM) * ((N + BN - 1) / BN)));
  p.block = dim3(256);
  return p;
}

hipError_t gemm_fp8_launch(const unsigned char* A, const unsigned char* Bt, float* C, int64_t M,
                           int64_t N, int64_t K, hipStream_t s) {
  OpPlan p = gemm_fp8_plan(M, N, K);
  hipLaunchKernelGGL(gemm_fp8_kernel, p.grid, p.block, 0, s, A, Bt, C, (int)M, (int)N, (int)K);
  return hipGetLastError();
}

}  // namespace ug
