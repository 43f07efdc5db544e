// Bird's-eye-view pillar binning of a point cloud (FP32 points -> int cells).
//
// Per cell: count, maximum z and smallest point index; per point: its cell.
// zmax is kept as an order-preserving unsigned key of the float while it is
// reduced, so that an unsigned maximum implements the float maximum (with
// -0 < +0).  All three reductions are order independent, so every path below
// gives bit-identical outputs.
//
// Two paths, chosen by size:
//
// * direct (small clouds, and grids of more than kMaxTiles tiles): init,
//   then one lane per point with three atomics on its cell in global memory,
//   then finalize.  Device-wide atomics run at a fraction of HBM bandwidth,
//   which is fine for the 30k-120k-point frames of a LiDAR chain.
//
// * binned (large clouds): the grid is cut into tiles of kTileCells
//   consecutive cells, small enough that one tile's accumulators live in LDS.
//     1. bin:    per chunk of kChunk points (read once), the cell of every
//                point (vidx) and an 8-byte record (z key, cell in tile,
//                index in chunk) per point, counting-sorted by tile in LDS
//                and written as one contiguous block, with the offsets of
//                its tile runs;
//     2. reduce: per (tile, group of chunks), the tile's runs of those
//                chunks reduced in LDS (count / max / min), written out as a
//                partial tile;
//     3. merge:  per cell, the partial tiles of its tile combined into the
//                outputs (empty cells: count 0, zmax -inf, first -1).
//   Global traffic is about 36 bytes per point (16 read and 4 written by
//   the points themselves, a record written and read back), with no global
//   atomics.
#include <algorithm>
#include <climits>
#include <cstdint>

#include "ops.hpp"

namespace ug {
namespace {

constexpr int kTileBits = 12;
constexpr int kTileCells = 1 << kTileBits;        // cells per tile (48 KiB of LDS)
constexpr int kMaxTiles = 1024;                   // binned grids: <= 4 Mi cells
constexpr int64_t kChunk = 8192;                  // points per bin workgroup
static_assert(kChunk <= 8192, "a record keeps the index in its chunk in 13 bits");
constexpr int64_t kBinnedMinPoints = int64_t(1) << 20;
constexpr int64_t kMinChunksPerGroup = 64;        // tile reduce: chunks per workgroup, at least
constexpr unsigned kKeyNegInf = 0x007fffffu;      // key of -inf

__device__ __forceinline__ unsigned zkey(float z) {
  const unsigned u = __float_as_uint(z);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float zval(unsigned k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

// Cell of a point, or -1.  Both subtractions and products are single FP32
// operations (no contraction), as the cell definition requires.
__device__ __forceinline__ int cell_of(float4 p, int nx, int ny, float xmin, float ymin,
                                       float scale) {
#pragma clang fp contract(off)
  const float fx = (p.x - xmin) * scale;
  const float fy = (p.y - ymin) * scale;
  // NaN fails every comparison and lands outside
  if (fx >= 0.0f && fx < (float)nx && fy >= 0.0f && fy < (float)ny) return (int)fy * nx + (int)fx;
  return -1;
}

// ------------------------------------------------------------------ direct
__global__ __launch_bounds__(256) void voxel_init(int* __restrict__ count,
                                                  unsigned* __restrict__ zk,
                                                  int* __restrict__ first, int64_t G) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < G; i += stride) {
    count[i] = 0;
    zk[i] = kKeyNegInf;
    first[i] = INT_MAX;
  }
}

__global__ __launch_bounds__(256) void voxel_scatter(const float4* __restrict__ pts,
                                                     int* __restrict__ vidx,
                                                     int* __restrict__ count,
                                                     unsigned* __restrict__ zk,
                                                     int* __restrict__ first, int64_t N, int nx,
                                                     int ny, float xmin, float ymin, float scale) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride) {
    const float4 p = pts[i];
    const int v = cell_of(p, nx, ny, xmin, ymin, scale);
    if (v >= 0) {
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

// ------------------------------------------------------------------ binned
// Exclusive prefix sums of n <= kMaxTiles values (val(i) for i < n) into
// out[0..n], out[n] = total, by one 256-lane workgroup (four values a lane).
// `wsum` is 4 ints of LDS.  Ends with a barrier.
template <typename F>
__device__ void block_scan_tiles(int n, F val, int* out, int* wsum) {
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  int a[4], s = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int i = 4 * t + k;
    a[k] = i < n ? val(i) : 0;
    s += a[k];
  }
  int incl = s;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(incl, d, 64);
    if (lane >= d) incl += y;
  }
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  int off = incl - s;
  for (int w = 0; w < wave; ++w) off += wsum[w];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int i = 4 * t + k;
    if (i < n) out[i] = off;
    off += a[k];
  }
  if (t == 255) out[n] = off;
  __syncthreads();
}

// 1. bin: one chunk of kChunk points per workgroup, read once.  Every lane
//    keeps its 32 points' cells and z keys in registers while the chunk's
//    tile histogram builds up in LDS; the exclusive scan of the histogram
//    gives each tile's run, the points are placed into their runs in LDS
//    (a counting sort by tile), and the chunk's records go out as one
//    contiguous block (chunk-major) with the run offsets H[c][0..T].  A
//    record is 8 bytes: z key (bits 0-31), cell within the tile (32-43),
//    point index within the chunk (44-56).
constexpr int kPerLane = kChunk / 256;

__device__ __forceinline__ uint64_t record(unsigned zk, int cell, int idx) {
  return (uint64_t)zk | ((uint64_t)(cell & (kTileCells - 1)) << 32) | ((uint64_t)idx << 44);
}

__global__ __launch_bounds__(256) void voxel_bin(const float4* __restrict__ pts,
                                                 int* __restrict__ vidx, int* __restrict__ H,
                                                 uint64_t* __restrict__ R, int64_t N, int nx,
                                                 int ny, float xmin, float ymin, float scale,
                                                 int T) {
  __shared__ int cur[kMaxTiles];       // histogram, then cursors
  __shared__ int off[kMaxTiles + 1];   // exclusive scan of the histogram
  __shared__ int wsum[4];
  __shared__ uint64_t rec[kChunk];     // the chunk's records, sorted by tile
  const int c = blockIdx.x;
  for (int t = threadIdx.x; t < T; t += 256) cur[t] = 0;
  __syncthreads();
  const int64_t beg = (int64_t)c * kChunk;
  const int64_t end = beg + kChunk < N ? beg + kChunk : N;
  int cell[kPerLane];
  unsigned zk[kPerLane];
  // eight points a lane in flight
#pragma unroll
  for (int u0 = 0; u0 < kPerLane; u0 += 8) {
    float4 p[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t j = beg + threadIdx.x + (int64_t)(u0 + u) * 256;
      p[u] = j < end ? pts[j] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t j = beg + threadIdx.x + (int64_t)(u0 + u) * 256;
      int v = -1;
      if (j < end) {
        v = cell_of(p[u], nx, ny, xmin, ymin, scale);
        vidx[j] = v;
        if (v >= 0) atomicAdd(&cur[v >> kTileBits], 1);
      }
      cell[u0 + u] = v;
      zk[u0 + u] = zkey(p[u].z);
    }
  }
  __syncthreads();
  block_scan_tiles(T, [&](int i) { return cur[i]; }, off, wsum);
  int* h = H + (int64_t)c * (T + 1);
  for (int t = threadIdx.x; t <= T; t += 256) h[t] = off[t];
  for (int t = threadIdx.x; t < T; t += 256) cur[t] = off[t];
  __syncthreads();
#pragma unroll
  for (int u = 0; u < kPerLane; ++u) {
    if (cell[u] >= 0) {
      const int lp = atomicAdd(&cur[cell[u] >> kTileBits], 1);
      rec[lp] = record(zk[u], cell[u], threadIdx.x + u * 256);
    }
  }
  __syncthreads();
  const int n = off[T];
  uint64_t* out = R + beg;
  for (int i = threadIdx.x; i < n; i += 256) out[i] = rec[i];
}

// 2. one workgroup per (tile, group of chunks): the tile's runs of those
//    chunks reduced into LDS accumulators, written out as a partial tile.
//    The runs' bounds of the group's chunks (up to kStage at a time) are
//    staged in LDS first, all loaded at once; then each wavefront takes
//    eight chunks at a time (every fourth block of eight) and reduces their
//    runs in rounds of 128 records of every run, loaded together (sixteen
//    loads a lane in flight) before their atomics.
constexpr int kRunsAtOnce = 8;
constexpr int kStage = 1024;   // chunks whose run bounds sit in LDS at once

__device__ __forceinline__ void reduce_record(uint64_t r, int base, int* acc_c, unsigned* acc_z,
                                              int* acc_f) {
  const int cc = (int)((r >> 32) & (kTileCells - 1));
  atomicAdd(&acc_c[cc], 1);
  atomicMax(&acc_z[cc], (unsigned)r);
  atomicMin(&acc_f[cc], base + (int)(r >> 44));
}

__global__ __launch_bounds__(256) void voxel_tile_reduce(const int* __restrict__ H,
                                                         const uint64_t* __restrict__ R,
                                                         int* __restrict__ pc,
                                                         unsigned* __restrict__ pz,
                                                         int* __restrict__ pf, int T, int nb,
                                                         int groups, int cpg) {
  // 48 KiB of accumulators and 8 KiB of run bounds: two workgroups a CU
  __shared__ int acc_c[kTileCells];
  __shared__ unsigned acc_z[kTileCells];
  __shared__ int acc_f[kTileCells];
  __shared__ int2 bnd[kStage];
  // chunk-group major: the workgroups resident together are the tiles of
  // a few chunk groups, which read neighbouring pieces of the same chunk
  // blocks (fewer distinct pages in flight than one tile's groups, which
  // span the whole record array)
  const int g = blockIdx.x / T, t = blockIdx.x % T;
  const int c0 = g * cpg, c1 = c0 + cpg < nb ? c0 + cpg : nb;
  for (int i = threadIdx.x; i < kTileCells; i += 256) {
    acc_c[i] = 0;
    acc_z[i] = kKeyNegInf;
    acc_f[i] = INT_MAX;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int s0 = c0; s0 < c1; s0 += kStage) {
    const int s1 = s0 + kStage < c1 ? s0 + kStage : c1;
    __syncthreads();   // the previous stage's bounds are no longer read
    for (int c = s0 + threadIdx.x; c < s1; c += 256) {
      const int* h = H + (int64_t)c * (T + 1) + t;
      bnd[c - s0] = make_int2(h[0], h[1]);
    }
    __syncthreads();
    for (int cb = s0 + wave * kRunsAtOnce; cb < s1; cb += 4 * kRunsAtOnce) {
      int ra[kRunsAtOnce], rb[kRunsAtOnce];
      int longest = 0;   // the same in every lane
#pragma unroll
      for (int k = 0; k < kRunsAtOnce; ++k) {
        const int c = cb + k;
        const int2 ab = c < s1 ? bnd[c - s0] : make_int2(0, 0);
        ra[k] = ab.x;
        rb[k] = ab.y;
        longest = max(longest, ab.y - ab.x);
      }
      // rounds of 128 records of every run: sixteen loads a lane in flight
      for (int off = 0; off < longest; off += 128) {
        uint64_t r0[kRunsAtOnce], r1[kRunsAtOnce];
#pragma unroll
        for (int k = 0; k < kRunsAtOnce; ++k) {
          const uint64_t* run = R + (int64_t)(cb + k) * kChunk;
          const int i = ra[k] + off + lane;
          r0[k] = i < rb[k] ? run[i] : 0;
          r1[k] = i + 64 < rb[k] ? run[i + 64] : 0;
        }
#pragma unroll
        for (int k = 0; k < kRunsAtOnce; ++k) {
          const int base = (cb + k) * (int)kChunk;
          const int i = ra[k] + off + lane;
          if (i < rb[k]) reduce_record(r0[k], base, acc_c, acc_z, acc_f);
          if (i + 64 < rb[k]) reduce_record(r1[k], base, acc_c, acc_z, acc_f);
        }
      }
    }
  }
  __syncthreads();
  const int64_t o = ((int64_t)t * groups + g) * kTileCells;
  for (int i = threadIdx.x; i < kTileCells; i += 256) {
    pc[o + i] = acc_c[i];
    pz[o + i] = acc_z[i];
    pf[o + i] = acc_f[i];
  }
}

// 3. per cell: combine the partial tiles of its tile (the groups' partials
//    of tile t are partial tiles t * groups .. t * groups + groups - 1)
__global__ __launch_bounds__(256) void voxel_merge(const int* __restrict__ pc,
                                                   const unsigned* __restrict__ pz,
                                                   const int* __restrict__ pf,
                                                   int* __restrict__ count, float* __restrict__ zmax,
                                                   int* __restrict__ first, int64_t G, int groups) {
  const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (v >= G) return;
  const int t = (int)(v >> kTileBits);
  const int l = (int)(v & (kTileCells - 1));
  int c = 0, f = INT_MAX;
  unsigned z = kKeyNegInf;
  for (int s = t * groups; s < (t + 1) * groups; ++s) {
    const int64_t o = (int64_t)s * kTileCells + l;
    c += pc[o];
    z = max(z, pz[o]);
    f = min(f, pf[o]);
  }
  count[v] = c;
  zmax[v] = zval(z);
  first[v] = c ? f : -1;
}

unsigned grid_for(int64_t work, int64_t cap) {
  int64_t g = (work + 255) / 256;
  if (g > cap) g = cap;
  if (g < 1) g = 1;
  return (unsigned)g;
}

// Workspace of the binned path, in 256-byte aligned pieces: the chunks' run
// offsets, their records (kChunk slots per chunk), the partial tiles.
struct Binned {
  int T = 0, nb = 0, groups = 0, cpg = 0;
  size_t H = 0, R = 0, pc = 0, pz = 0, pf = 0, total = 0;
};

bool use_binned(int64_t N, int64_t G) {
  return N >= kBinnedMinPoints && (G + kTileCells - 1) / kTileCells <= kMaxTiles;
}

Binned binned_layout(int64_t N, int64_t G) {
  Binned b;
  b.T = (int)((G + kTileCells - 1) / kTileCells);
  b.nb = (int)((N + kChunk - 1) / kChunk);
  // about 2048 reduce workgroups (groups of chunks per tile), four times
  // the resident ones: the tiles of a clustered cloud hold very different
  // record counts, and the workgroup dispatcher evens them out.  A group
  // takes at least kMinChunksPerGroup chunks, so that a smaller cloud does
  // not pay for (and hold) more partial tiles than records.
  b.groups = (int)std::max<int64_t>(
      1, std::min<int64_t>(b.nb / kMinChunksPerGroup, (2048 + b.T - 1) / b.T));
  b.cpg = (b.nb + b.groups - 1) / b.groups;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += (bytes + 255) / 256 * 256;
    return at;
  };
  b.H = take(sizeof(int) * (size_t)b.nb * (b.T + 1));
  b.R = take(sizeof(uint64_t) * (size_t)b.nb * kChunk);
  const size_t parts = (size_t)b.T * b.groups * kTileCells;
  b.pc = take(sizeof(int) * parts);
  b.pz = take(sizeof(unsigned) * parts);
  b.pf = take(sizeof(int) * parts);
  b.total = off;
  return b;
}

}  // namespace

size_t voxel_f32_workspace(int64_t N, int nx, int ny) {
  const int64_t G = (int64_t)nx * ny;
  return use_binned(N, G) ? binned_layout(N, G).total : 0;
}

OpPlan voxel_f32_plan(int64_t N, int nx, int ny) {
  OpPlan p;
  p.block = dim3(256);
  const int64_t G = (int64_t)nx * ny;
  if (use_binned(N, G)) {
    // the widest of the five launches: one lane per cell in the merge
    p.func = reinterpret_cast<const void*>(&voxel_merge);
    p.grid = dim3(grid_for(G, INT_MAX));
  } else {
    p.func = reinterpret_cast<const void*>(&voxel_scatter);
    p.grid = dim3(grid_for(N, 256 * 32));
  }
  return p;
}

hipError_t voxel_f32_launch(const float* pts, int* vidx, int* count, float* zmax, int* first,
                            int64_t N, int nx, int ny, float xmin, float ymin, float scale,
                            void* ws, size_t ws_bytes, hipStream_t s) {
  const int64_t G = (int64_t)nx * ny;
  const dim3 blk(256);
  const float4* p4 = reinterpret_cast<const float4*>(pts);
  if (use_binned(N, G)) {
    const Binned b = binned_layout(N, G);
    if (!ws || ws_bytes < b.total || (reinterpret_cast<uintptr_t>(ws) & 255))
      return hipErrorInvalidValue;
    char* w = static_cast<char*>(ws);
    int* H = reinterpret_cast<int*>(w + b.H);
    uint64_t* R = reinterpret_cast<uint64_t*>(w + b.R);
    int* pc = reinterpret_cast<int*>(w + b.pc);
    unsigned* pz = reinterpret_cast<unsigned*>(w + b.pz);
    int* pf = reinterpret_cast<int*>(w + b.pf);
    hipLaunchKernelGGL(voxel_bin, dim3(b.nb), blk, 0, s, p4, vidx, H, R, N, nx, ny, xmin, ymin,
                       scale, b.T);
    hipLaunchKernelGGL(voxel_tile_reduce, dim3(b.T * b.groups), blk, 0, s, H, R, pc, pz, pf, b.T,
                       b.nb, b.groups, b.cpg);
    hipLaunchKernelGGL(voxel_merge, dim3(grid_for(G, INT_MAX)), blk, 0, s, pc, pz, pf, count,
                       zmax, first, G, b.groups);
    return hipGetLastError();
  }
  unsigned* zk = reinterpret_cast<unsigned*>(zmax);
  hipLaunchKernelGGL(voxel_init, dim3(grid_for(G, 256 * 8)), blk, 0, s, count, zk, first, G);
  if (N > 0) {
    hipLaunchKernelGGL(voxel_scatter, dim3(grid_for(N, 256 * 32)), blk, 0, s, p4, vidx, count, zk,
                       first, N, nx, ny, xmin, ymin, scale);
  }
  hipLaunchKernelGGL(voxel_finalize, dim3(grid_for(G, 256 * 8)), blk, 0, s, count, zk, first, G);
  return hipGetLastError();
}

}  // namespace ug
