// C[M,N] = A[M,K] B[K,N], row-major FP32, on the FP32 matrix cores of gfx950.
//
// One kernel template, three tile shapes, always four waves per workgroup:
//   <WM, WN, TM, TN, KS>: the workgroup tile is (WM*TM*32) x (WN*TN*32); its
//   waves form a WM x WN x KS grid; each wave owns TM x TN MFMA 32x32x2 tiles
//   and one of KS slices of every K step.
//   big   <2,2,2,2,1>: 128 x 128 tiles, 64 accumulators per lane;
//   mid   <2,2,1,1,1>:  64 x  64 tiles;
//   small <1,1,1,1,4>:  32 x  32 tiles, K split four ways inside the
//                       workgroup and summed through LDS in a fixed order
//                       (results do not depend on scheduling).
// The launcher takes the largest tile that still gives two workgroups per CU
// (or the small one), so a 256^3 product spreads over 64 CUs instead of 4,
// unless the tuning table (an autotuner's measurements) names a variant
// (0 big, 1 mid, 2 small) for the shape.
//
// Operand tiles are staged through LDS, double buffered: the next K step is
// fetched into registers while the current one feeds the matrix cores, then
// written to the other buffer (one barrier per step).  A is stored K-major so
// both operands are read as 32 consecutive floats per half-wave.
//
// Workgroups are dispatched round-robin over the 8 XCDs; the linear id is
// remapped so each XCD works on a contiguous band of output tiles (sharing A
// and B panels in its own L2), walked in groups of 8 tile-rows.
#include "mfma.hpp"
#include "ops.hpp"
#include "signal.hpp"

namespace ug {
namespace {

constexpr int BK = 16;      // K values per wave per step
constexpr int kXcds = 8;
constexpr int kGroupM = 8;

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

template <int WM, int WN, int TM, int TN, int KS>
struct GemmCfg {
  static constexpr int BM = WM * TM * 32, BN = WN * TN * 32;
  static constexpr int BKT = BK * KS;                  // K values per step
  static constexpr int SA = BM + 4, SB = BN + 4;       // LDS row strides
  static constexpr int A4 = BM * BKT / 4 / 256;        // float4 per thread
  static constexpr int B4 = BKT * BN / 4 / 256;
  static constexpr int LDS = 2 * BKT * (SA + SB);      // floats
  static_assert(WM * WN * KS == 4, "four waves");
  static_assert(A4 >= 1 && B4 >= 1, "tile too small for 256 threads");
  static_assert(BM * BKT % 1024 == 0 && BKT * BN % 1024 == 0, "even float4 split");
  static_assert(KS == 1 || LDS >= (KS - 1) * 1024 * TM * TN, "reduction fits in LDS");
};

template <int WM, int WN, int TM, int TN, int KS, bool VEC>
__global__ __launch_bounds__(256) void gemm_f32_kernel(const float* __restrict__ A,
                                                        const float* __restrict__ B,
                                                        float* __restrict__ C, int M, int N,
                                                        int K, unsigned* sig) {
  using G = GemmCfg<WM, WN, TM, TN, KS>;
  constexpr int BM = G::BM, BN = G::BN, BKT = G::BKT, SA = G::SA, SB = G::SB;
  __shared__ float lds[G::LDS];
  float* As0 = lds;
  float* Bs0 = lds + 2 * BKT * SA;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int ks = wave / (WM * WN);
  const int wm = (wave % (WM * WN)) / WN, wn = wave % WN;
  const int tiles_m = (M + BM - 1) / BM, tiles_n = (N + BN - 1) / BN;
  int tm, tn;
  tile_of(blockIdx.x, tiles_m, tiles_n, &tm, &tn);
  const int m0 = tm * BM, n0 = tn * BN;

  float4 ra[G::A4], rb[G::B4];
  auto load = [&](int k0) {
#pragma unroll
    for (int i = 0; i < G::A4; ++i) {
      const int q = tid + 256 * i;
      const int m = m0 + q / (BKT / 4);
      const int k = k0 + 4 * (q % (BKT / 4));
      if (VEC) {
        ra[i] = (m < M && k < K) ? *reinterpret_cast<const float4*>(A + (size_t)m * K + k)
                                 : make_float4(0.f, 0.f, 0.f, 0.f);
      } else {
        float v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = (m < M && k + j < K) ? A[(size_t)m * K + k + j] : 0.f;
        ra[i] = make_float4(v[0], v[1], v[2], v[3]);
      }
    }
#pragma unroll
    for (int i = 0; i < G::B4; ++i) {
      const int q = tid + 256 * i;
      const int k = k0 + q / (BN / 4);
      const int n = n0 + 4 * (q % (BN / 4));
      if (VEC) {
        rb[i] = (k < K && n < N) ? *reinterpret_cast<const float4*>(B + (size_t)k * N + n)
                                 : make_float4(0.f, 0.f, 0.f, 0.f);
      } else {
        float v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = (k < K && n + j < N) ? B[(size_t)k * N + n + j] : 0.f;
        rb[i] = make_float4(v[0], v[1], v[2], v[3]);
      }
    }
  };
  auto store = [&](int buf) {
    float* As = As0 + buf * BKT * SA;
    float* Bs = Bs0 + buf * BKT * SB;
#pragma unroll
    for (int i = 0; i < G::A4; ++i) {
      const int q = tid + 256 * i;
      float* a = As + (4 * (q % (BKT / 4))) * SA + q / (BKT / 4);
      a[0 * SA] = ra[i].x;
      a[1 * SA] = ra[i].y;
      a[2 * SA] = ra[i].z;
      a[3 * SA] = ra[i].w;
    }
#pragma unroll
    for (int i = 0; i < G::B4; ++i) {
      const int q = tid + 256 * i;
      *reinterpret_cast<float4*>(Bs + (q / (BN / 4)) * SB + 4 * (q % (BN / 4))) = rb[i];
    }
  };

  f32x16 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = zero16();

  const int nk = (K + BKT - 1) / BKT;
  load(0);
  store(0);
  __syncthreads();

  const int half = lane >> 5, col = lane & 31;
  const int am = wm * TM * 32 + col, bn = wn * TN * 32 + col;
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) load((kt + 1) * BKT);
    const float* as = As0 + buf * BKT * SA + ks * BK * SA;
    const float* bs = Bs0 + buf * BKT * SB + ks * BK * SB;
#pragma unroll
    for (int kk = 0; kk < BK / 2; ++kk) {
      const int k = 2 * kk + half;
      float a[TM], b[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) a[i] = as[k * SA + am + 32 * i];
#pragma unroll
      for (int j = 0; j < TN; ++j) b[j] = bs[k * SB + bn + 32 * j];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = mfma_32x32x2(a[i], b[j], acc[i][j]);
    }
    if (kt + 1 < nk) store(buf ^ 1);
    __syncthreads();
  }

  if (KS > 1) {
    // K slices 1..KS-1 hand their partial sums to slice 0 through LDS; slice
    // 0 adds them in slice order.
    constexpr int PER = TM * TN * 16 * 64;   // floats per wave
    if (ks > 0) {
      float* red = lds + (ks - 1) * PER * (WM * WN) + (wave % (WM * WN)) * PER;
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
          for (int r = 0; r < 16; ++r) red[((i * TN + j) * 16 + r) * 64 + lane] = acc[i][j][r];
    }
    __syncthreads();
    if (ks > 0) {   // handed over: meet slice 0 at the counter's barrier, then leave
      group_done(sig);
      return;
    }
#pragma unroll
    for (int s = 1; s < KS; ++s) {
      const float* red = lds + (s - 1) * PER * (WM * WN) + (wave % (WM * WN)) * PER;
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
          for (int r = 0; r < 16; ++r) acc[i][j][r] += red[((i * TN + j) * 16 + r) * 64 + lane];
    }
  }

#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int n = n0 + wn * TN * 32 + 32 * j + col;
      if (n >= N) continue;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int m = m0 + wm * TM * 32 + 32 * i + mfma32_row(r, lane);
        if (m < M) C[(size_t)m * N + n] = acc[i][j][r];
      }
    }
  group_done(sig);
}

enum Shape { kBig = 0, kMid = 1, kSmall = 2 };

int64_t tiles(int64_t M, int64_t N, int bm, int bn) { return ((M + bm - 1) / bm) * ((N + bn - 1) / bn); }

Shape pick(int64_t M, int64_t N) {
  constexpr int64_t kWant = 512;   // two workgroups per CU
  if (tiles(M, N, 128, 128) >= kWant) return kBig;
  if (tiles(M, N, 64, 64) >= kWant / 2) return kMid;
  return kSmall;
}

// The variant asked for, else the tuning table's, else the rule above.
Shape choose(int64_t M, int64_t N, int64_t K, int variant) {
  if (variant < 0) {
    const int64_t key[4] = {M, N, K, 0};
    variant = tune_get(UG_OP_GEMM_F32, key);
  }
  return variant >= 0 && variant < 3 ? static_cast<Shape>(variant) : pick(M, N);
}

template <int WM, int WN, int TM, int TN, int KS>
const void* fn(bool vec) {
  return vec ? reinterpret_cast<const void*>(&gemm_f32_kernel<WM, WN, TM, TN, KS, true>)
             : reinterpret_cast<const void*>(&gemm_f32_kernel<WM, WN, TM, TN, KS, false>);
}

template <int WM, int WN, int TM, int TN, int KS>
void launch(bool vec, dim3 grid, hipStream_t s, const float* A, const float* B, float* C, int M,
            int N, int K, unsigned* sig) {
  if (vec)
    hipLaunchKernelGGL((gemm_f32_kernel<WM, WN, TM, TN, KS, true>), grid, dim3(256), 0, s, A, B,
                       C, M, N, K, sig);
  else
    hipLaunchKernelGGL((gemm_f32_kernel<WM, WN, TM, TN, KS, false>), grid, dim3(256), 0, s, A, B,
                       C, M, N, K, sig);
}

}  // namespace

static bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

OpPlan gemm_f32_plan(int64_t M, int64_t N, int64_t K, bool vec, int variant) {
  OpPlan p;
  p.block = dim3(256);
  switch (choose(M, N, K, variant)) {
    case kBig:
      p.func = fn<2, 2, 2, 2, 1>(vec);
      p.grid = dim3((unsigned)tiles(M, N, 128, 128));
      break;
    case kMid:
      p.func = fn<2, 2, 1, 1, 1>(vec);
      p.grid = dim3((unsigned)tiles(M, N, 64, 64));
      break;
    default:
      p.func = fn<1, 1, 1, 1, 4>(vec);
      p.grid = dim3((unsigned)tiles(M, N, 32, 32));
  }
  return p;
}

hipError_t gemm_f32_launch(const float* A, const float* B, float* C, int64_t M, int64_t N,
                           int64_t K, hipStream_t s, unsigned* sig, int variant) {
  const bool vec = (K % 4 == 0) && (N % 4 == 0) && aligned16(A) && aligned16(B);
  const Shape sh = choose(M, N, K, variant);
  OpPlan p = gemm_f32_plan(M, N, K, vec, static_cast<int>(sh));
  switch (sh) {
    case kBig:
      launch<2, 2, 2, 2, 1>(vec, p.grid, s, A, B, C, (int)M, (int)N, (int)K, sig);
      break;
    case kMid:
      launch<2, 2, 1, 1, 1>(vec, p.grid, s, A, B, C, (int)M, (int)N, (int)K, sig);
      break;
    default:
      launch<1, 1, 1, 1, 4>(vec, p.grid, s, A, B, C, (int)M, (int)N, (int)K, sig);
  }
  return hipGetLastError();
}

}  // namespace ug
