// 3x3 convolution (cross-correlation, stride 1, zero pad 1, C_out = C_in),
// NCHW FP32, as an implicit GEMM on the FP32 matrix cores of gfx950:
//   Y[o, p] = sum_{c, dy, dx} W[o, c, dy, dx] * X[c, py + dy - 1, px + dx - 1]
// i.e. M = output channels, N = pixels, K = 9 * input channels.
//
// Template <WM, WN, TM, TN, KS, TH, TW>: a workgroup owns BM = WM*TM*32
// output channels x a TH x TW pixel patch (TH*TW = WN*TN*32 pixels); its four
// waves form a WM x WN x KS grid.  The reduction runs over chunks of 4 input
// channels (36 K values): per step the workgroup stages KS chunks, each wave
// consumes the chunk of its K slice: the chunk's weights (BM x 36, K-major in
// LDS) and the input patch with its one-pixel halo (4 x (TH+2) x (TW+2)).
// The im2col operand is never materialised: each MFMA lane reads its
// (c, dy, dx)-shifted pixel straight from the patch.  The next step is
// prefetched into registers while the current one is consumed (32-bit
// offsets from a per-step uniform base).  With KS > 1
// the K slices are summed through LDS in slice order at the end, so results
// do not depend on scheduling.
//
// The launcher picks the largest tile that still gives ~two workgroups per CU,
// or one per CU for a tile without a K split (measured faster than a K split),
// unless the tuning table (an autotuner's measurements) names a variant
// (0..4, the order of kShapes) for the shape.
#include "mfma.hpp"
#include "ops.hpp"
#include "signal.hpp"

namespace ug {
namespace {

constexpr int CC = 4;          // input channels per chunk
constexpr int KC = CC * 9;     // K values per chunk

template <int WM, int WN, int TM, int TN, int KS, int TH, int TW>
struct ConvCfg {
  static constexpr int BM = WM * TM * 32;
  static constexpr int PH = TH + 2, PW = TW + 2, PLANE = PH * PW;
  static constexpr int SW = BM + 33;                  // LDS stride, K-major weights
  static constexpr int WS = KC * SW;                  // weight floats per chunk
  static constexpr int XS = CC * PLANE;               // patch floats per chunk
  static constexpr int W_PER = (KS * BM * KC + 255) / 256;
  static constexpr int X_PER = (KS * XS + 255) / 256;
  static constexpr int LDS = KS * (WS + XS);
  static_assert(WM * WN * KS == 4, "four waves");
  static_assert(WN * TN * 32 == TH * TW, "pixel tile");
  static_assert(KS == 1 || LDS >= (KS - 1) * 1024 * TM * TN, "reduction fits in LDS");
};

template <int WM, int WN, int TM, int TN, int KS, int TH, int TW>
__global__ __launch_bounds__(256) void conv3x3_f32_kernel(const float* __restrict__ X,
                                                           const float* __restrict__ Wt,
                                                           float* __restrict__ Y, int C, int H,
                                                           int W, unsigned* sig) {
  using Cf = ConvCfg<WM, WN, TM, TN, KS, TH, TW>;
  constexpr int BM = Cf::BM, SW = Cf::SW, PW = Cf::PW, PLANE = Cf::PLANE;
  __shared__ float lds[Cf::LDS];
  float* Ws0 = lds;                     // [KS][KC][SW]
  float* Xs0 = lds + KS * Cf::WS;       // [KS][CC][PLANE]

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int ks = wave / (WM * WN);
  const int wm = (wave % (WM * WN)) / WN, wn = wave % WN;
  const int tiles_x = (W + TW - 1) / TW, tiles_y = (H + TH - 1) / TH;
  const int pt = blockIdx.x % (tiles_x * tiles_y);
  const int n = blockIdx.x / (tiles_x * tiles_y);
  const int y0 = (pt / tiles_x) * TH, x0 = (pt % tiles_x) * TW;
  const int o0 = blockIdx.y * BM;
  const size_t plane = (size_t)H * W;
  const float* Xn = X + (size_t)n * C * plane;

  float rw[Cf::W_PER];
  float rx[Cf::X_PER];

  // Byte offsets of this thread's staged elements from the step's base
  // (weights: row o0, input channel c0; input: image n, channel c0), fixed
  // for the whole K loop; ~0u marks padding (outside the tile, the output
  // channels or the image).  32-bit offsets from a uniform base keep one
  // register per element instead of a 64-bit address; the operation's
  // validation keeps H * W below 2^26, so the byte offsets of the KS * CC
  // (at most 16) planes of one step fit in 32 bits.
  uint32_t wo[Cf::W_PER], xo[Cf::X_PER];
#pragma unroll
  for (int i = 0; i < Cf::W_PER; ++i) {
    const int idx = tid + 256 * i;
    const int s = idx / (BM * KC), rem = idx % (BM * KC);
    const int o = rem / KC, k = rem % KC;
    wo[i] = (idx < KS * BM * KC && o0 + o < C)
                ? (uint32_t)(((int64_t)(o * C + s * CC) * 9 + k) * 4) : ~0u;
  }
#pragma unroll
  for (int i = 0; i < Cf::X_PER; ++i) {
    const int idx = tid + 256 * i;
    const int s = idx / Cf::XS, rem = idx % Cf::XS;
    const int c = rem / PLANE, r = rem % PLANE;
    const int yy = y0 - 1 + r / PW, xx = x0 - 1 + r % PW;
    xo[i] = (idx < KS * Cf::XS && yy >= 0 && yy < H && xx >= 0 && xx < W)
                ? (uint32_t)((((int64_t)(s * CC + c) * H + yy) * W + xx) * 4) : ~0u;
  }

  // stage KS chunks starting at input channel c0 (chunk s covers c0 + 4 s ..);
  // only a step that runs past the last channel checks channels per element
  auto load = [&](int c0) {
    const char* wbase = reinterpret_cast<const char*>(Wt + ((size_t)o0 * C + c0) * 9);
    const char* xbase = reinterpret_cast<const char*>(Xn + (size_t)c0 * plane);
    if (c0 + KS * CC <= C) {
#pragma unroll
      for (int i = 0; i < Cf::W_PER; ++i)
        rw[i] = wo[i] != ~0u ? *reinterpret_cast<const float*>(wbase + wo[i]) : 0.f;
#pragma unroll
      for (int i = 0; i < Cf::X_PER; ++i)
        rx[i] = xo[i] != ~0u ? *reinterpret_cast<const float*>(xbase + xo[i]) : 0.f;
    } else {
#pragma unroll
      for (int i = 0; i < Cf::W_PER; ++i) {
        const int idx = tid + 256 * i;
        const int s = idx / (BM * KC), k = (idx % (BM * KC)) % KC;
        rw[i] = (wo[i] != ~0u && c0 + s * CC + k / 9 < C)
                    ? *reinterpret_cast<const float*>(wbase + wo[i]) : 0.f;
      }
#pragma unroll
      for (int i = 0; i < Cf::X_PER; ++i) {
        const int idx = tid + 256 * i;
        const int s = idx / Cf::XS, c = (idx % Cf::XS) / PLANE;
        rx[i] = (xo[i] != ~0u && c0 + s * CC + c < C)
                    ? *reinterpret_cast<const float*>(xbase + xo[i]) : 0.f;
      }
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int i = 0; i < Cf::W_PER; ++i) {
      const int idx = tid + 256 * i;
      if (idx < KS * BM * KC) {
        const int s = idx / (BM * KC), rem = idx % (BM * KC);
        Ws0[s * Cf::WS + (rem % KC) * SW + rem / KC] = rw[i];
      }
    }
#pragma unroll
    for (int i = 0; i < Cf::X_PER; ++i) {
      const int idx = tid + 256 * i;
      if (idx < KS * Cf::XS) Xs0[idx] = rx[i];
    }
  };

  f32x16 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = zero16();

  // MFMA step kk of a chunk: lane half h supplies K index k = kk + 18 h, so
  // the lower half walks input channels 0-1 of the chunk and the upper half
  // channels 2-3.  Both operands' LDS offsets then differ between the halves
  // by a per-lane constant, and every step's offset is a compile-time
  // immediate once the loop is unrolled.
  const int half = lane >> 5, col = lane & 31;
  const float* wb = Ws0 + ks * Cf::WS + half * (KC / 2) * SW + wm * TM * 32 + col;
  const float* xb[TN];
#pragma unroll
  for (int j = 0; j < TN; ++j) {
    const int p = (wn * TN + j) * 32 + col;
    xb[j] = Xs0 + ks * Cf::XS + half * (CC / 2) * PLANE + (p / TW) * PW + (p % TW);
  }

  const int nsteps = (C + KS * CC - 1) / (KS * CC);
  load(0);
  for (int st = 0; st < nsteps; ++st) {
    __syncthreads();          // previous step fully consumed
    store();
    __syncthreads();
    if (st + 1 < nsteps) load((st + 1) * KS * CC);
#pragma unroll
    for (int kk = 0; kk < KC / 2; ++kk) {
      const int r = kk % 9;
      const int xo = (kk / 9) * PLANE + (r / 3) * PW + (r % 3);
      float a[TM], b[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) a[i] = wb[kk * SW + 32 * i];
#pragma unroll
      for (int j = 0; j < TN; ++j) b[j] = xb[j][xo];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = mfma_32x32x2(a[i], b[j], acc[i][j]);
    }
  }

  if (KS > 1) {
    constexpr int PER = TM * TN * 16 * 64;
    __syncthreads();
    if (ks > 0) {
      float* red = lds + (ks - 1) * PER * (WM * WN) + (wave % (WM * WN)) * PER;
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
          for (int q = 0; q < 16; ++q) red[((i * TN + j) * 16 + q) * 64 + lane] = acc[i][j][q];
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
          for (int q = 0; q < 16; ++q) acc[i][j][q] += red[((i * TN + j) * 16 + q) * 64 + lane];
    }
  }

  float* Yn = Y + (size_t)n * C * plane;
#pragma unroll
  for (int j = 0; j < TN; ++j) {
    const int p = (wn * TN + j) * 32 + col;
    const int yy = y0 + p / TW, xx = x0 + p % TW;
    if (yy >= H || xx >= W) continue;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int o = o0 + wm * TM * 32 + 32 * i + mfma32_row(q, lane);
        if (o < C) Yn[(size_t)o * plane + (size_t)yy * W + xx] = acc[i][j][q];
      }
  }
  group_done(sig);
}

// Tile shapes, largest first: {BM, TH, TW}.
struct Shape {
  int bm, th, tw;
};
constexpr Shape kShapes[] = {
    {128, 8, 16},   // <2,2,2,2,1>
    {64, 8, 16},    // <1,4,2,1,1>
    {32, 8, 16},    // <1,4,1,1,1>
    {64, 2, 16},    // <1,1,2,1,4>
    {32, 2, 16},    // <1,1,1,1,4>
};

int64_t wgs(const Shape& s, int64_t N, int64_t C, int64_t H, int64_t W) {
  return ((H + s.th - 1) / s.th) * ((W + s.tw - 1) / s.tw) * N * ((C + s.bm - 1) / s.bm);
}

// First (largest) tile with ~two workgroups per CU, or one per CU if it has no
// K split; else the one with the most workgroups.
int pick(int64_t N, int64_t C, int64_t H, int64_t W);

// The variant asked for, else the tuning table's, else the rule below.
int choose(int64_t N, int64_t C, int64_t H, int64_t W, int variant) {
  if (variant < 0) {
    const int64_t key[4] = {N, C, H, W};
    variant = tune_get(UG_OP_CONV3X3_F32, key);
  }
  return variant >= 0 && variant < 5 ? variant : pick(N, C, H, W);
}

int pick(int64_t N, int64_t C, int64_t H, int64_t W) {
  constexpr int64_t kWant = 480, kOnePerCu = 256;
  int best = 4;
  int64_t most = 0;
  for (int i = 0; i < 5; ++i) {
    if (kShapes[i].bm > 32 && C <= kShapes[i].bm / 2) continue;   // mostly padding
    const int64_t n = wgs(kShapes[i], N, C, H, W);
    if (n >= kWant || (i < 3 && n >= kOnePerCu)) return i;       // tiles 0-2: no K split
    if (n > most) {
      most = n;
      best = i;
    }
  }
  return best;
}

template <int WM, int WN, int TM, int TN, int KS, int TH, int TW>
void launch(dim3 grid, hipStream_t s, const float* X, const float* Wt, float* Y, int C, int H,
            int W, unsigned* sig) {
  hipLaunchKernelGGL((conv3x3_f32_kernel<WM, WN, TM, TN, KS, TH, TW>), grid, dim3(256), 0, s, X,
                     Wt, Y, C, H, W, sig);
}

}  // namespace

OpPlan conv3x3_f32_plan(int64_t N, int64_t C, int64_t H, int64_t W, int variant) {
  OpPlan p;
  const int i = choose(N, C, H, W, variant);
  const Shape& s = kShapes[i];
  const void* f[] = {reinterpret_cast<const void*>(&conv3x3_f32_kernel<2, 2, 2, 2, 1, 8, 16>),
                     reinterpret_cast<const void*>(&conv3x3_f32_kernel<1, 4, 2, 1, 1, 8, 16>),
                     reinterpret_cast<const void*>(&conv3x3_f32_kernel<1, 4, 1, 1, 1, 8, 16>),
                     reinterpret_cast<const void*>(&conv3x3_f32_kernel<1, 1, 2, 1, 4, 2, 16>),
                     reinterpret_cast<const void*>(&conv3x3_f32_kernel<1, 1, 1, 1, 4, 2, 16>)};
  p.func = f[i];
  p.grid = dim3((unsigned)(((H + s.th - 1) / s.th) * ((W + s.tw - 1) / s.tw) * N),
                (unsigned)((C + s.bm - 1) / s.bm));
  p.block = dim3(256);
  return p;
}

hipError_t conv3x3_f32_launch(const float* X, const float* Wt, float* Y, int64_t N, int64_t C,
                              int64_t H, int64_t W, hipStream_t s, unsigned* sig, int variant) {
  const int v = choose(N, C, H, W, variant);
  OpPlan p = conv3x3_f32_plan(N, C, H, W, v);
  const int c = (int)C, h = (int)H, w = (int)W;
  switch (v) {
    case 0: launch<2, 2, 2, 2, 1, 8, 16>(p.grid, s, X, Wt, Y, c, h, w, sig); break;
    case 1: launch<1, 4, 2, 1, 1, 8, 16>(p.grid, s, X, Wt, Y, c, h, w, sig); break;
    case 2: launch<1, 4, 1, 1, 1, 8, 16>(p.grid, s, X, Wt, Y, c, h, w, sig); break;
    case 3: launch<1, 1, 2, 1, 4, 2, 16>(p.grid, s, X, Wt, Y, c, h, w, sig); break;
    default: launch<1, 1, 1, 1, 4, 2, 16>(p.grid, s, X, Wt, Y, c, h, w, sig); break;
  }
  return hipGetLastError();
}

}  // namespace ug
