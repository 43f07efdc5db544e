// Host-side entry points of the gfx950 kernels (one per operation), and the
// operation-level validation and dispatch used by the gate and the C-ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "ug.h"

namespace ug {

// Launch shape of an operation's main kernel (for the utilisation estimate).
struct OpPlan {
  const void* func = nullptr;
  dim3 grid{1, 1, 1};
  dim3 block{1, 1, 1};
  size_t lds = 0;
};

OpPlan gemm_f32_plan(int64_t M, int64_t N, int64_t K, bool vec, int variant = -1);
hipError_t gemm_f32_launch(const float* A, const float* B, float* C, int64_t M, int64_t N,
                           int64_t K, hipStream_t s, unsigned* sig = nullptr, int variant = -1);

OpPlan conv3x3_f32_plan(int64_t N, int64_t C, int64_t H, int64_t W, int variant = -1);
hipError_t conv3x3_f32_launch(const float* X, const float* Wt, float* Y, int64_t N, int64_t C,
                              int64_t H, int64_t W, hipStream_t s, unsigned* sig = nullptr,
                              int variant = -1);

OpPlan bias_relu_f32_plan(int64_t R, int64_t C, int axis, bool vec);
hipError_t bias_relu_f32_launch(const float* X, const float* b, float* Y, int64_t R, int64_t C,
                                int axis, hipStream_t s);

OpPlan rowsum_f32_plan(int64_t R, int64_t C);
hipError_t rowsum_f32_launch(const float* Z, float* r, int64_t R, int64_t C, hipStream_t s);

OpPlan softmax_f32_plan(int64_t R, int64_t L, bool vec);
hipError_t softmax_f32_launch(const float* X, float* Y, int64_t R, int64_t L, hipStream_t s);

OpPlan gemm_fp8_plan(int64_t M, int64_t N, int64_t K);
hipError_t gemm_fp8_launch(const unsigned char* A, const unsigned char* Bt, float* C, int64_t M,
                           int64_t N, int64_t K, hipStream_t s);

OpPlan vecadd_f32_plan(int64_t n, int64_t w);
hipError_t vecadd_f32_launch(const float* a, const float* b, float* c, int64_t n, int64_t w,
                             int64_t r, hipStream_t s);

OpPlan conv3x3_bf16_plan(int64_t C, int64_t H, int64_t W);
hipError_t conv3x3_bf16_launch(const uint16_t* X, const uint16_t* Wt, float* Y, int64_t C,
                               int64_t H, int64_t W, hipStream_t s, unsigned* sig = nullptr);

OpPlan accum_i32_plan(int64_t n);
hipError_t accum_i32_launch(const int* x, int* st, int64_t n, hipStream_t s);

OpPlan gemm_bf16_plan(int64_t M, int64_t N, int64_t K);
hipError_t gemm_bf16_launch(const uint16_t* A, const uint16_t* Bt, float* C, int64_t M,
                            int64_t N, int64_t K, hipStream_t s, unsigned* sig = nullptr);

// Device workspace the voxel scatter needs (0: none); the launch fails with
// hipErrorInvalidValue if it needs one and `ws` is missing or too small.
size_t voxel_f32_workspace(int64_t N, int nx, int ny);
OpPlan voxel_f32_plan(int64_t N, int nx, int ny);
hipError_t voxel_f32_launch(const float* pts, int* vidx, int* count, float* zmax, int* first,
                            int64_t N, int nx, int ny, float xmin, float ymin, float scale,
                            void* ws, size_t ws_bytes, hipStream_t s);

// Size of the static device workspace of ug_kernel_launch_noalloc, per GPU.
constexpr size_t kStaticScratchBytes = size_t(UG_STATIC_SCRATCH_BYTES);

// Device address of the static workspace on the current device (located on
// the first call per device, then cached).  Allocates nothing.
hipError_t static_scratch(void** ptr);

// Per-frame sizes (ug_kernel.frame_dim > 0): the range [lo, hi] of the
// frame's value v that kernel k accepts (false: the op takes no per-frame
// size, or the registered shape cannot carry one), and the kernel's shape
// for a frame with value v (s = v >> frame_shift sets the op's frame
// dimension; see include/ug.h).
bool frame_range(const ug_kernel& k, int64_t* lo, int64_t* hi);
ug_kernel frame_kernel(const ug_kernel& k, int64_t v);

// Checks a descriptor against n_buffers slots.  Returns nullptr if valid,
// else a static message.
const char* validate_kernel(const ug_kernel& k, uint32_t n_buffers);

// Bytes of device workspace the operation needs beside its buffers (0 for
// most operations).  The workspace holds no state between launches.
size_t workspace_bytes(const ug_kernel& k);

// Launches the operation with buffers[slot] pointers and a workspace of
// ws_bytes >= workspace_bytes(k) (may be null when none is needed).
// `sig` (contractions only, see signal_waves) is a device counter to which
// every wavefront of the kernel adds one once its results are stored.
// Asynchronous.
hipError_t launch_kernel(const ug_kernel& k, void* const* buffers, hipStream_t s,
                         void* ws = nullptr, size_t ws_bytes = 0, unsigned* sig = nullptr,
                         int variant = -1);

// Wavefronts that add to a completion counter when the operation is
// launched with one: 0 if the operation takes no counter (only the FP32 and
// BF16 GEMM and 3x3 convolution do).
uint32_t signal_waves(const ug_kernel& k);

// Main-kernel launch shape of an operation (at a tile variant, -1: the
// launcher's choice).
OpPlan plan_kernel(const ug_kernel& k, int variant = -1);
// The tile variant the launcher takes for k (-1 for operations with one).
int chosen_variant(const ug_kernel& k);

// Tile variants of an operation's launcher (0: one tile shape only): FP32
// GEMM 3 (128x128, 64x64, 32x32 with a four-way K split), FP32 convolution
// 5 (see conv3x3_f32.hip).  The launchers and plans of those operations take
// a variant; -1 means: the tuning table's entry for the shape, else the
// launcher's fixed rule.
int tile_variants(int32_t op);
// Tuning table, process-wide, keyed (op, shape[0..3]): the variant, or -1.
int tune_get(int32_t op, const int64_t* shape);
bool tune_set(int32_t op, const int64_t* shape, int variant);   // -1 removes
void tune_clear();
size_t tune_size();
// Adds the entries of a table file (lines "op s0 s1 s2 s3 variant", '#'
// comments): returns the number added, -1 if unreadable, -2 if a line is
// malformed (then nothing is added).
int tune_load(const char* path);

// Hardware-queue class of each stream (streams with equal class share a
// hardware queue), measured with two tiny kernels per pair of streams
// tested; classes are numbered in order of first appearance.  Synchronous;
// the device should be otherwise idle.
hipError_t stream_queue_classes(const std::vector<hipStream_t>& s, std::vector<int>* cls);

}  // namespace ug
