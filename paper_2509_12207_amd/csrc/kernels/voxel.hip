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
//     1. count:  per chunk of kChunk points, a histogram of tiles (LDS),
//                stored tile-major in the workspace;
//     2. scan:   per tile, exclusive offsets of the chunks and the tile total;
//     3. place:  per chunk, the cell of every point (vidx), and a record
//                (z key, index, cell in tile) per point, sorted by tile in
//                LDS and written as one run per tile;
//     4. reduce: per segment of at most kSeg records of one tile, count /
//                max / min in LDS, written out as a partial tile;
//     5. merge:  per cell, the partial tiles of its tile combined into the
//                outputs (empty cells: count 0, zmax -inf, first -1).
//   Global traffic is about 50 bytes per point, with no global atomics.
#include <climits>
#include <cstdint>

#include "ops.hpp"

namespace ug {
namespace {

constexpr int kTileBits = 12;
constexpr int kTileCells = 1 << kTileBits;        // cells per tile (48 KiB of LDS)
constexpr int kMaxTiles = 1024;                   // binned grids: <= 4 Mi cells
constexpr int64_t kChunk = 8192;                  // points per count/place block
static_assert(kChunk <= 65536, "place keeps in-chunk indices in 16 bits");
constexpr int64_t kSeg = 65536;                   // records per reduce block
constexpr int64_t kBinnedMinPoints = int64_t(1) << 20;
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

// 1. tile histogram of each chunk; H is tile-major: H[tile * nb + chunk]
__global__ __launch_bounds__(256) void voxel_count(const float4* __restrict__ pts,
                                                   int* __restrict__ H, int64_t N, int nx, int ny,
                                                   float xmin, float ymin, float scale, int T,
                                                   int nb) {
  __shared__ int hist[kMaxTiles];
  for (int i = threadIdx.x; i < T; i += 256) hist[i] = 0;
  __syncthreads();
  const int64_t beg = (int64_t)blockIdx.x * kChunk;
  const int64_t end = beg + kChunk < N ? beg + kChunk : N;
  for (int64_t i = beg + threadIdx.x; i < end; i += 4 * 256) {
    float4 p[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i + u * 256 < end) p[u] = pts[i + u * 256];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (i + u * 256 < end) {
        const int v = cell_of(p[u], nx, ny, xmin, ymin, scale);
        if (v >= 0) atomicAdd(&hist[v >> kTileBits], 1);
      }
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < T; t += 256) H[(int64_t)t * nb + blockIdx.x] = hist[t];
}

// 2. per tile (one workgroup each): exclusive scan of its nb chunk counts in
//    place, and the tile total
__global__ __launch_bounds__(256) void voxel_scan(int* __restrict__ H, int* __restrict__ tcount,
                                                  int nb) {
  __shared__ int wsum[4];
  __shared__ int carry;
  int* h = H + (int64_t)blockIdx.x * nb;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < nb; base += 256) {
    const int i = base + threadIdx.x;
    const int x = i < nb ? h[i] : 0;
    int incl = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int y = __shfl_up(incl, d, 64);
      if (lane >= d) incl += y;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    int off = carry + incl - x;
    for (int w = 0; w < wave; ++w) off += wsum[w];
    if (i < nb) h[i] = off;
    __syncthreads();  // every lane has read carry and wsum
    if (threadIdx.x == 255) carry = off + x;
    __syncthreads();
  }
  if (threadIdx.x == 0) tcount[blockIdx.x] = carry;
}

// 3. cells and records, one chunk per workgroup.  The chunk's records are
//    first sorted by tile in LDS (a counting sort: the chunk's tile counts
//    are known from step 1), then written out as one contiguous run per
//    tile, so that the stores coalesce.  Record r of tile t lies in
//    [tbase[t], tbase[t] + tcount[t]); within a chunk's run the order is
//    arbitrary (the reductions do not depend on it).
__global__ __launch_bounds__(256) void voxel_place(const float4* __restrict__ pts,
                                                   int* __restrict__ vidx,
                                                   const int* __restrict__ H,
                                                   const int* __restrict__ tcount,
                                                   unsigned* __restrict__ rz,
                                                   int* __restrict__ ri,
                                                   unsigned short* __restrict__ rc, int64_t N,
                                                   int nx, int ny, float xmin, float ymin,
                                                   float scale, int T, int nb) {
  __shared__ int gbase[kMaxTiles];     // global position of the chunk's run of tile t
  __shared__ int loff[kMaxTiles + 1];  // local position of that run (exclusive scan)
  __shared__ int cur[kMaxTiles];       // local cursors
  __shared__ int wsum[4];
  __shared__ unsigned sz[kChunk];         // z keys, by local position
  __shared__ unsigned short si[kChunk];   // point index within the chunk
  __shared__ unsigned short sc[kChunk];   // cell within the tile
  const int c = blockIdx.x;
  block_scan_tiles(T, [&](int i) { return tcount[i]; }, loff, wsum);
  for (int t = threadIdx.x; t < T; t += 256) gbase[t] = loff[t] + H[(int64_t)t * nb + c];
  __syncthreads();
  // H holds, per tile, the exclusive scan over chunks: this chunk's count of
  // tile t is the step to the next chunk (or to the tile total)
  block_scan_tiles(T, [&](int i) {
    const int64_t h = (int64_t)i * nb + c;
    return (c + 1 < nb ? H[h + 1] : tcount[i]) - H[h];
  }, loff, wsum);
  for (int t = threadIdx.x; t < T; t += 256) cur[t] = loff[t];
  __syncthreads();
  const int64_t beg = (int64_t)c * kChunk;
  const int64_t end = beg + kChunk < N ? beg + kChunk : N;
  // eight points a lane in flight (two workgroups fit a CU)
  for (int64_t i = beg + threadIdx.x; i < end; i += 8 * 256) {
    float4 p[8];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (i + u * 256 < end) p[u] = pts[i + u * 256];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t j = i + u * 256;
      if (j < end) {
        const int v = cell_of(p[u], nx, ny, xmin, ymin, scale);
        vidx[j] = v;
        if (v >= 0) {
          const int t = v >> kTileBits;
          const int lp = atomicAdd(&cur[t], 1);
          if (lp < loff[t + 1]) {  // always true when counting and placing agree
            sz[lp] = zkey(p[u].z);
            si[lp] = (unsigned short)(j - beg);
            sc[lp] = (unsigned short)(v & (kTileCells - 1));
          }
        }
      }
    }
  }
  __syncthreads();
  // one wavefront per tile run (tiles dealt round-robin to the four)
  const int lane = threadIdx.x & 63;
  for (int t = threadIdx.x >> 6; t < T; t += 4) {
    const int a = loff[t], n = loff[t + 1] - a, g = gbase[t];
    for (int k = lane; k < n; k += 64) {
      rz[g + k] = sz[a + k];
      ri[g + k] = (int)(beg + si[a + k]);
      rc[g + k] = sc[a + k];
    }
  }
}

// 4. one workgroup per segment of a tile's records: LDS reduction, then the
//    partial tile.  Workgroups beyond the number of segments exit at once.
__global__ __launch_bounds__(256) void voxel_reduce(const int* __restrict__ tcount,
                                                    const unsigned* __restrict__ rz,
                                                    const int* __restrict__ ri,
                                                    const unsigned short* __restrict__ rc,
                                                    int* __restrict__ pc,
                                                    unsigned* __restrict__ pz,
                                                    int* __restrict__ pf, int T) {
  // 52 KiB of LDS: three workgroups fit a CU
  __shared__ int segb[kMaxTiles + 1];
  __shared__ int wsum[4];
  __shared__ int acc_c[kTileCells];
  __shared__ unsigned acc_z[kTileCells];
  __shared__ int acc_f[kTileCells];
  block_scan_tiles(T, [&](int i) { return (int)((tcount[i] + kSeg - 1) / kSeg); }, segb, wsum);
  const int s = blockIdx.x;
  if (s >= segb[T]) return;  // uniform across the workgroup
  // tile of segment s: the last t with segb[t] <= s (segb is non-decreasing)
  int lo = 0, hi = T - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (segb[mid] <= s) lo = mid; else hi = mid - 1;
  }
  const int t = lo;
  // first record of tile t: the sum of the totals of the tiles before it
  int part = 0;
  for (int i = threadIdx.x; i < t; i += 256) part += tcount[i];
  for (int d = 32; d >= 1; d >>= 1) part += __shfl_xor(part, d, 64);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = part;
  __syncthreads();
  const int tbase = wsum[0] + wsum[1] + wsum[2] + wsum[3];
  const int64_t start = (int64_t)tbase + (int64_t)(s - segb[t]) * kSeg;
  const int64_t tend = (int64_t)tbase + tcount[t];
  const int64_t end = start + kSeg < tend ? start + kSeg : tend;
  for (int c = threadIdx.x; c < kTileCells; c += 256) {
    acc_c[c] = 0;
    acc_z[c] = kKeyNegInf;
    acc_f[c] = INT_MAX;
  }
  __syncthreads();
  // eight records a lane per round (32-, 32- and 16-byte loads: the record
  // arrays are 256-byte aligned and padded to a multiple of 8 records),
  // from the multiple of 8 at or below the segment start; records outside
  // [start, end) are read and skipped
  for (int64_t r0 = (start & ~int64_t(7)) + 8 * threadIdx.x; r0 < end; r0 += 8 * 256) {
    const uint4 z0 = *reinterpret_cast<const uint4*>(rz + r0);
    const uint4 z1 = *reinterpret_cast<const uint4*>(rz + r0 + 4);
    const int4 f0 = *reinterpret_cast<const int4*>(ri + r0);
    const int4 f1 = *reinterpret_cast<const int4*>(ri + r0 + 4);
    const uint4 c8 = *reinterpret_cast<const uint4*>(rc + r0);
    const unsigned zz[8] = {z0.x, z0.y, z0.z, z0.w, z1.x, z1.y, z1.z, z1.w};
    const int ff[8] = {f0.x, f0.y, f0.z, f0.w, f1.x, f1.y, f1.z, f1.w};
    const unsigned cc[4] = {c8.x, c8.y, c8.z, c8.w};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int64_t r = r0 + k;
      if (r >= start && r < end) {
        const int c = (int)((cc[k >> 1] >> (16 * (k & 1))) & (kTileCells - 1));
        atomicAdd(&acc_c[c], 1);
        atomicMax(&acc_z[c], zz[k]);
        atomicMin(&acc_f[c], ff[k]);
      }
    }
  }
  __syncthreads();
  const int64_t o = (int64_t)s * kTileCells;
  for (int c = threadIdx.x; c < kTileCells; c += 256) {
    pc[o + c] = acc_c[c];
    pz[o + c] = acc_z[c];
    pf[o + c] = acc_f[c];
  }
}

// 5. per cell: combine the partial tiles of its tile
__global__ __launch_bounds__(256) void voxel_merge(const int* __restrict__ tcount,
                                                   const int* __restrict__ pc,
                                                   const unsigned* __restrict__ pz,
                                                   const int* __restrict__ pf,
                                                   int* __restrict__ count, float* __restrict__ zmax,
                                                   int* __restrict__ first, int64_t G, int T) {
  __shared__ int segb[kMaxTiles + 1];
  __shared__ int wsum[4];
  block_scan_tiles(T, [&](int i) { return (int)((tcount[i] + kSeg - 1) / kSeg); }, segb, wsum);
  const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (v >= G) return;
  const int t = (int)(v >> kTileBits);
  const int l = (int)(v & (kTileCells - 1));
  int c = 0, f = INT_MAX;
  unsigned z = kKeyNegInf;
  for (int s = segb[t]; s < segb[t + 1]; ++s) {
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

// Workspace of the binned path, in 256-byte aligned pieces.
struct Binned {
  int T = 0, nb = 0, smax = 0;
  size_t H = 0, tcount = 0, rz = 0, ri = 0, rc = 0, pc = 0, pz = 0, pf = 0, total = 0;
};

bool use_binned(int64_t N, int64_t G) {
  return N >= kBinnedMinPoints && (G + kTileCells - 1) / kTileCells <= kMaxTiles;
}

Binned binned_layout(int64_t N, int64_t G) {
  Binned b;
  b.T = (int)((G + kTileCells - 1) / kTileCells);
  b.nb = (int)((N + kChunk - 1) / kChunk);
  b.smax = b.T + (int)((N + kSeg - 1) / kSeg);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += (bytes + 255) / 256 * 256;
    return at;
  };
  b.H = take(sizeof(int) * (size_t)b.T * b.nb);
  b.tcount = take(sizeof(int) * (size_t)b.T);
  // record arrays padded to a multiple of 8 records (vector loads of eight)
  const size_t n8 = (size_t)(N + 7) / 8 * 8;
  b.rz = take(sizeof(unsigned) * n8);
  b.ri = take(sizeof(int) * n8);
  b.rc = take(sizeof(unsigned short) * n8);
  b.pc = take(sizeof(int) * (size_t)b.smax * kTileCells);
  b.pz = take(sizeof(unsigned) * (size_t)b.smax * kTileCells);
  b.pf = take(sizeof(int) * (size_t)b.smax * kTileCells);
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
    int* tc = reinterpret_cast<int*>(w + b.tcount);
    unsigned* rz = reinterpret_cast<unsigned*>(w + b.rz);
    int* ri = reinterpret_cast<int*>(w + b.ri);
    unsigned short* rc = reinterpret_cast<unsigned short*>(w + b.rc);
    int* pc = reinterpret_cast<int*>(w + b.pc);
    unsigned* pz = reinterpret_cast<unsigned*>(w + b.pz);
    int* pf = reinterpret_cast<int*>(w + b.pf);
    hipLaunchKernelGGL(voxel_count, dim3(b.nb), blk, 0, s, p4, H, N, nx, ny, xmin, ymin, scale,
                       b.T, b.nb);
    hipLaunchKernelGGL(voxel_scan, dim3(b.T), blk, 0, s, H, tc, b.nb);
    hipLaunchKernelGGL(voxel_place, dim3(b.nb), blk, 0, s, p4, vidx, H, tc, rz, ri, rc, N, nx, ny,
                       xmin, ymin, scale, b.T, b.nb);
    hipLaunchKernelGGL(voxel_reduce, dim3(b.smax), blk, 0, s, tc, rz, ri, rc, pc, pz, pf, b.T);
    hipLaunchKernelGGL(voxel_merge, dim3(grid_for(G, INT_MAX)), blk, 0, s, tc, pc, pz, pf, count,
                       zmax, first, G, b.T);
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
