// Operation-level validation and dispatch to the gfx950 kernels.
#include "ops.hpp"

namespace ug {

namespace {
constexpr int64_t kMaxDim = int64_t(1) << 31;

bool slot_ok(int32_t s, uint32_t n) { return s >= 0 && static_cast<uint32_t>(s) < n; }
bool pos(int64_t v) { return v > 0 && v < kMaxDim; }
}  // namespace

const char* validate_kernel(const ug_kernel& k, uint32_t nb) {
  const int64_t* s = k.shape;
  switch (k.op) {
    case UG_OP_GEMM_F32:
      if (!pos(s[0]) || !pos(s[1]) || !pos(s[2])) return "gemm: M, N, K must be in [1, 2^31)";
      if (s[0] * s[2] >= kMaxDim * 8 || s[2] * s[1] >= kMaxDim * 8 || s[0] * s[1] >= kMaxDim * 8)
        return "gemm: operand too large";
      if (!slot_ok(k.in[0], nb) || !slot_ok(k.in[1], nb) || !slot_ok(k.out[0], nb))
        return "gemm: needs in {A, B}, out {C}";
      return nullptr;
    case UG_OP_BIAS_RELU_F32:
      if (!pos(s[0]) || !pos(s[1]) || (s[2] != 0 && s[2] != 1))
        return "bias_relu: shape {R, C, axis in {0,1}}";
      if (!slot_ok(k.in[0], nb) || !slot_ok(k.in[1], nb) || !slot_ok(k.out[0], nb))
        return "bias_relu: needs in {X, b}, out {Y}";
      return nullptr;
    case UG_OP_CONV3X3_F32:
      if (!pos(s[0]) || !pos(s[1]) || !pos(s[2]) || !pos(s[3]))
        return "conv3x3: shape {N, C, H, W} must be positive";
      if (s[2] * s[3] >= (int64_t(1) << 26) || s[1] * s[1] * 9 >= kMaxDim * 4)
        return "conv3x3: H * W must be below 2^26 and 9 C^2 below 2^33";
      if (!slot_ok(k.in[0], nb) || !slot_ok(k.in[1], nb) || !slot_ok(k.out[0], nb))
        return "conv3x3: needs in {X, W}, out {Y}";
      return nullptr;
    case UG_OP_ROWSUM_F32:
      if (!pos(s[0]) || !pos(s[1])) return "rowsum: shape {R, C} must be positive";
      if (!slot_ok(k.in[0], nb) || !slot_ok(k.out[0], nb)) return "rowsum: needs in {Z}, out {r}";
      return nullptr;
    case UG_OP_SOFTMAX_F32:
      if (!pos(s[0]) || !pos(s[1])) return "softmax: shape {R, L} must be positive";
      if (!slot_ok(k.in[0], nb) || !slot_ok(k.out[0], nb)) return "softmax: needs in {X}, out {Y}";
      return nullptr;
    case UG_OP_VOXEL_F32:
      if (s[0] < 0 || s[0] >= kMaxDim) return "voxel: N must be in [0, 2^31)";
      if (!pos(s[1]) || !pos(s[2]) || s[1] * s[2] >= kMaxDim) return "voxel: bad grid nx, ny";
      if (!(k.fparam[2] > 0.0f)) return "voxel: scale must be positive";
      if (!slot_ok(k.in[0], nb) || !slot_ok(k.out[0], nb) || !slot_ok(k.out[1], nb) ||
          !slot_ok(k.out[2], nb) || !slot_ok(k.out[3], nb))
        return "voxel: needs in {pts}, out {vidx, count, zmax, first}";
      return nullptr;
    case UG_OP_GEMM_FP8:
      if (!pos(s[0]) || !pos(s[1]) || !pos(s[2])) return "gemm_fp8: M, N, K must be in [1, 2^31)";
      if (s[2] % 16 != 0) return "gemm_fp8: K must be a multiple of 16";
      if (s[3] < 0 || s[3] >= kMaxDim) return "gemm_fp8: the row offset must be in [0, 2^31)";
      if ((s[0] + s[3]) * s[2] >= kMaxDim * 32 || s[1] * s[2] >= kMaxDim * 32 ||
          (s[0] + s[3]) * s[1] >= kMaxDim * 8)
        return "gemm_fp8: operand too large";
      if (!slot_ok(k.in[0], nb) || !slot_ok(k.in[1], nb) || !slot_ok(k.out[0], nb))
        return "gemm_fp8: needs in {A, Bt}, out {C}";
      return nullptr;
    case UG_OP_CONV3X3_BF16:
      if (s[0] != 1) return "conv3x3_bf16: one image (N = 1)";
      if (!pos(s[1]) || s[1] % 32 != 0 || s[1] > 8192) return "conv3x3_bf16: C a multiple of 32, <= 8192";
      if (!pos(s[2]) || !pos(s[3]) || s[2] * s[3] >= kMaxDim / 64) return "conv3x3_bf16: bad H, W";
      if (!slot_ok(k.in[0], nb) || !slot_ok(k.in[1], nb) || !slot_ok(k.out[0], nb))
        return "conv3x3_bf16: needs in {X, W}, out {Y}";
      return nullptr;
    case UG_OP_VECADD_F32:
      if (!pos(s[0]) || s[1] < 1 || s[1] > 65536 || s[2] < 0 || s[2] > 65536)
        return "vecadd: N >= 1, 1 <= W <= 65536, 0 <= R <= 65536 (0 = 1)";
      if (!slot_ok(k.in[0], nb) || !slot_ok(k.in[1], nb) || !slot_ok(k.out[0], nb))
        return "vecadd: needs in {A, B}, out {C}";
      return nullptr;
    case UG_OP_UPLOAD_H2D:
      if (s[0] < 0 || s[0] >= kMaxDim || !pos(s[1]) || s[0] * s[1] >= kMaxDim * 32)
        return "upload: shape {N >= 0, unit bytes >= 1}, at most 64 GiB";
      if (!slot_ok(k.in[0], nb) || !slot_ok(k.out[0], nb))
        return "upload: needs in {host source}, out {device destination}";
      return nullptr;
    case UG_OP_ACCUM_I32:
      if (s[0] < 0 || s[0] >= kMaxDim) return "accum_i32: N must be in [0, 2^31)";
      if (!slot_ok(k.in[0], nb) || !slot_ok(k.out[0], nb))
        return "accum_i32: needs in {x}, out {state}";
      return nullptr;
    case UG_OP_GEMM_BF16:
      if (!pos(s[0]) || !pos(s[1]) || !pos(s[2]) || s[2] >= kMaxDim / 2)
        return "gemm_bf16: M, N in [1, 2^31), K in [1, 2^30)";
      if (s[2] % 32 != 0) return "gemm_bf16: K must be a multiple of 32";
      if (s[0] * s[2] >= kMaxDim * 16 || s[1] * s[2] >= kMaxDim * 16 || s[0] * s[1] >= kMaxDim * 8)
        return "gemm_bf16: operand too large";
      if (!slot_ok(k.in[0], nb) || !slot_ok(k.in[1], nb) || !slot_ok(k.out[0], nb))
        return "gemm_bf16: needs in {A, Bt}, out {C}";
      return nullptr;
    default:
      return "unknown op";
  }
}

size_t workspace_bytes(const ug_kernel& k) {
  if (k.op == UG_OP_VOXEL_F32) return voxel_f32_workspace(k.shape[0], (int)k.shape[1], (int)k.shape[2]);
  return 0;
}

namespace {
int64_t isqrt(int64_t x) {
  int64_t r = 0;
  while ((r + 1) * (r + 1) <= x) ++r;
  return r;
}
}  // namespace

bool frame_range(const ug_kernel& k, int64_t* lo, int64_t* hi) {
  const int64_t* s = k.shape;
  int64_t smin = 1, smax = 0;
  switch (k.op) {
    case UG_OP_VOXEL_F32:
    case UG_OP_UPLOAD_H2D:
      smin = 0;
      smax = s[0];
      break;
    case UG_OP_GEMM_F32:
    case UG_OP_SOFTMAX_F32:
      smax = s[0];
      break;
    case UG_OP_CONV3X3_F32:
    case UG_OP_CONV3X3_BF16:
      if (s[2] != s[3]) return false;   // square images
      smax = s[2];
      break;
    case UG_OP_BIAS_RELU_F32:
      smax = s[2] == 1 ? isqrt(s[1]) : s[0];
      break;
    case UG_OP_ROWSUM_F32:
      smax = isqrt(s[1]);
      break;
    default:
      return false;
  }
  if (k.frame_shift < 0 || k.frame_shift > 30 || smax < smin || smax < 1) return false;
  *lo = smin << k.frame_shift;
  *hi = (smax << k.frame_shift) | ((int64_t(1) << k.frame_shift) - 1);
  return true;
}

ug_kernel frame_kernel(const ug_kernel& k, int64_t v) {
  ug_kernel f = k;
  const int64_t s = v >> k.frame_shift;
  switch (k.op) {
    case UG_OP_VOXEL_F32:
    case UG_OP_UPLOAD_H2D:
    case UG_OP_GEMM_F32:
    case UG_OP_SOFTMAX_F32:
      f.shape[0] = s;
      break;
    case UG_OP_CONV3X3_F32:
    case UG_OP_CONV3X3_BF16:
      f.shape[2] = f.shape[3] = s;
      break;
    case UG_OP_BIAS_RELU_F32:
      if (k.shape[2] == 1)
        f.shape[1] = s * s;   // per-channel bias over an image plane
      else
        f.shape[0] = s;       // per-column bias over s rows
      break;
    case UG_OP_ROWSUM_F32:
      f.shape[1] = s * s;     // the row is an image plane
      break;
    default:
      break;
  }
  return f;
}

hipError_t launch_kernel(const ug_kernel& k, void* const* b, hipStream_t st, void* ws,
                         size_t ws_bytes, unsigned* sig, int variant) {
  if (sig && signal_waves(k) == 0) return hipErrorInvalidValue;
  const int64_t* s = k.shape;
  auto F = [&](int32_t slot) { return static_cast<float*>(b[slot]); };
  auto I = [&](int32_t slot) { return static_cast<int*>(b[slot]); };
  switch (k.op) {
    case UG_OP_GEMM_F32:
      return gemm_f32_launch(F(k.in[0]), F(k.in[1]), F(k.out[0]), s[0], s[1], s[2], st, sig,
                             variant);
    case UG_OP_BIAS_RELU_F32:
      return bias_relu_f32_launch(F(k.in[0]), F(k.in[1]), F(k.out[0]), s[0], s[1], (int)s[2], st);
    case UG_OP_CONV3X3_F32:
      return conv3x3_f32_launch(F(k.in[0]), F(k.in[1]), F(k.out[0]), s[0], s[1], s[2], s[3], st,
                                sig, variant);
    case UG_OP_ROWSUM_F32:
      return rowsum_f32_launch(F(k.in[0]), F(k.out[0]), s[0], s[1], st);
    case UG_OP_SOFTMAX_F32:
      return softmax_f32_launch(F(k.in[0]), F(k.out[0]), s[0], s[1], st);
    case UG_OP_VOXEL_F32:
      return voxel_f32_launch(F(k.in[0]), I(k.out[0]), I(k.out[1]), F(k.out[2]), I(k.out[3]),
                              s[0], (int)s[1], (int)s[2], k.fparam[0], k.fparam[1], k.fparam[2],
                              ws, ws_bytes, st);
    case UG_OP_GEMM_FP8: {
      // rows [m0, m0 + M) of A and C (a row band: one sub-kernel of a split
      // product); K is a multiple of 16, so the band of A stays aligned
      const int64_t m0 = s[3];
      const auto* a = static_cast<const unsigned char*>(b[k.in[0]]) + m0 * s[2];
      const auto* bt = static_cast<const unsigned char*>(b[k.in[1]]);
      if ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(bt)) & 15)
        return hipErrorInvalidValue;
      return gemm_fp8_launch(a, bt, F(k.out[0]) + m0 * s[1], s[0], s[1], s[2], st);
    }
    case UG_OP_CONV3X3_BF16: {
      const auto* x = static_cast<const uint16_t*>(b[k.in[0]]);
      const auto* w = static_cast<const uint16_t*>(b[k.in[1]]);
      if ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(w)) & 15)
        return hipErrorInvalidValue;
      return conv3x3_bf16_launch(x, w, F(k.out[0]), s[1], s[2], s[3], st, sig);
    }
    case UG_OP_VECADD_F32:
      return vecadd_f32_launch(F(k.in[0]), F(k.in[1]), F(k.out[0]), s[0], s[1],
                               s[2] > 0 ? s[2] : 1, st);
    case UG_OP_UPLOAD_H2D:
      // a per-frame input arriving from host memory (pinned by the caller)
      if (s[0] == 0) return hipSuccess;
      return hipMemcpyAsync(b[k.out[0]], b[k.in[0]], static_cast<size_t>(s[0] * s[1]),
                            hipMemcpyHostToDevice, st);
    case UG_OP_ACCUM_I32:
      if (s[0] == 0) return hipSuccess;
      return accum_i32_launch(I(k.in[0]), I(k.out[0]), s[0], st);
    case UG_OP_GEMM_BF16: {
      const auto* a = static_cast<const uint16_t*>(b[k.in[0]]);
      const auto* bt = static_cast<const uint16_t*>(b[k.in[1]]);
      if ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(bt)) & 15)
        return hipErrorInvalidValue;
      return gemm_bf16_launch(a, bt, F(k.out[0]), s[0], s[1], s[2], st, sig);
    }
    default:
      return hipErrorInvalidValue;
  }
}

uint32_t signal_waves(const ug_kernel& k) {
  switch (k.op) {
    case UG_OP_GEMM_F32:
    case UG_OP_CONV3X3_F32:
    case UG_OP_GEMM_BF16:
    case UG_OP_CONV3X3_BF16: {
      const OpPlan p = plan_kernel(k);
      return p.grid.x * p.grid.y * p.grid.z * (p.block.x * p.block.y * p.block.z / 64);
    }
    default:
      return 0;
  }
}

int chosen_variant(const ug_kernel& k) {
  const int64_t* s = k.shape;
  const int64_t gkey[4] = {s[0], s[1], s[2], 0};
  switch (k.op) {
    case UG_OP_GEMM_F32: {
      const int v = tune_get(UG_OP_GEMM_F32, gkey);
      if (v >= 0) return v;
      // the plan's function tells the rule's choice apart
      for (int i = 0; i < tile_variants(UG_OP_GEMM_F32); ++i)
        if (gemm_f32_plan(s[0], s[1], s[2], true, i).func == gemm_f32_plan(s[0], s[1], s[2], true).func)
          return i;
      return -1;
    }
    case UG_OP_CONV3X3_F32: {
      for (int i = 0; i < tile_variants(UG_OP_CONV3X3_F32); ++i)
        if (conv3x3_f32_plan(s[0], s[1], s[2], s[3], i).func ==
            conv3x3_f32_plan(s[0], s[1], s[2], s[3]).func)
          return i;
      return -1;
    }
    default:
      return -1;
  }
}

OpPlan plan_kernel(const ug_kernel& k, int variant) {
  const int64_t* s = k.shape;
  switch (k.op) {
    case UG_OP_GEMM_F32:
      return gemm_f32_plan(s[0], s[1], s[2], (s[2] % 4 == 0) && (s[1] % 4 == 0), variant);
    case UG_OP_BIAS_RELU_F32:
      return bias_relu_f32_plan(s[0], s[1], (int)s[2], s[1] % 4 == 0);
    case UG_OP_CONV3X3_F32:
      return conv3x3_f32_plan(s[0], s[1], s[2], s[3], variant);
    case UG_OP_ROWSUM_F32:
      return rowsum_f32_plan(s[0], s[1]);
    case UG_OP_SOFTMAX_F32:
      return softmax_f32_plan(s[0], s[1], s[1] % 4 == 0);
    case UG_OP_VOXEL_F32:
      return voxel_f32_plan(s[0], (int)s[1], (int)s[2]);
    case UG_OP_GEMM_FP8:
      return gemm_fp8_plan(s[0], s[1], s[2]);
    case UG_OP_GEMM_BF16:
      return gemm_bf16_plan(s[0], s[1], s[2]);
    case UG_OP_VECADD_F32:
      return vecadd_f32_plan(s[0], s[1]);
    case UG_OP_CONV3X3_BF16:
      return conv3x3_bf16_plan(s[1], s[2], s[3]);
    case UG_OP_ACCUM_I32:
      return accum_i32_plan(s[0]);
    default:
      return OpPlan{};
  }
}

}  // namespace ug
