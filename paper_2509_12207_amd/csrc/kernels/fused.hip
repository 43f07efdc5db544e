// Tail executor (see fused.hpp for the protocol).
//
// Workgroup 0, wave 0 is the dispatcher: eight queue slots per lane, it
// polls the host's publication and key-rewrite counts and, when they move, copies new
// descriptors to device memory, marks items ready once their producer's
// counter is complete and mirrors the host's keys.  Workers (workgroups 1..)
// repeatedly let their first wave pick the ready item with the smallest key
// that has tiles left (one slot per lane, a wave-wide minimum), claim its
// next tile with a compare-and-swap on (generation, next tile) so that a
// slot re-used for a new item can never hand out the old item's tiles, and
// run the tile with all four waves: each wave takes whole rows, applies
// y = max(x + b, +0) (one FP32 add, -0 and NaN to +0, the bias+ReLU
// kernel's arithmetic), stores y, and reduces the row in registers for the
// softmax and the row sum.  The last finished tile marks the item done and
// reports it to the host.
#include "fused.hpp"

namespace ug {
namespace {

__device__ __forceinline__ uint64_t now_ticks() { return __builtin_amdgcn_s_memrealtime(); }

template <typename T>
__device__ __forceinline__ T ld_sys(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
}
template <typename T>
__device__ __forceinline__ void st_sys(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}
template <typename T>
__device__ __forceinline__ T ld_dev(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_dev(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ float relu_add(float x, float b) {
  const float s = x + b;
  return s > 0.0f ? s : 0.0f;
}

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

// Descriptor as 10 words of 64 bits (FuseItem is 80 bytes).
constexpr int kItemWords = sizeof(FuseItem) / 8;

__device__ void dispatcher(FuseHost* __restrict__ H, FuseDev* __restrict__ D, uint64_t t0,
                           uint64_t idle, uint64_t lease) {
  const int lane = threadIdx.x;
  uint64_t last = t0;
  // publications and key rewrites already taken in (all-ones: none yet, so
  // the first pass reads every slot)
  uint64_t seen_npub = ~0ull, seen_kepoch = ~0ull;
  for (;;) {
    const uint64_t now = now_ticks();
    const uint32_t ctl = (ld_sys(&H->stop) ? 1u : 0u) | (ld_sys(&H->pause) ? 2u : 0u);
    if (lane == 0) st_dev(&D->ctl, ctl);
    if ((ctl & 1u) || now - t0 > lease) break;
    const uint64_t npub = ld_sys(&H->npub), kepoch = ld_sys(&H->kepoch);
    const bool scan_pub = npub != seen_npub, scan_key = kepoch != seen_kepoch;
    seen_npub = npub;
    seen_kepoch = kepoch;
    bool act = false;
    for (uint32_t s = lane; s < kFuseSlots; s += 64) {
      if (scan_pub) {
        const uint64_t p = ld_sys(&H->pub[s]);
        if (p != ld_dev(&D->seen[s])) {
          // a new item: copy its descriptor, restart the slot's counters
          // under a new generation, then let it wait for its producer
          const uint64_t* src = reinterpret_cast<const uint64_t*>(&H->item[s]);
          uint64_t* dst = reinterpret_cast<uint64_t*>(&D->item[s]);
#pragma unroll
          for (int w = 0; w < kItemWords; ++w)
            __hip_atomic_store(dst + w, ld_sys(src + w), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
          const uint32_t g = ld_dev(&D->gen[s]) + 1u;
          st_dev(&D->gen[s], g);
          st_dev(&D->next[s], uint64_t(g) << 32);
          st_dev(&D->fin[s], 0u);
          st_dev(&D->key[s], ld_sys(&H->key[s]));
          st_dev(&D->seen[s], p);
          st_dev(&D->state[s], 1u);
          act = true;
        }
      }
      const uint32_t st = ld_dev(&D->state[s]);
      if (st == 1u) {
        unsigned* sig = reinterpret_cast<unsigned*>(ld_dev(&D->item[s].sig));
        if (sig == nullptr || ld_dev(sig) >= ld_dev(&D->item[s].sig_expected)) {
          if (sig) st_dev(sig, 0u);   // ready for the producer's next launch
          st_dev(&D->key[s], ld_sys(&H->key[s]));
          st_dev(&D->state[s], 2u);
          act = true;
        }
      } else if (st == 2u && scan_key) {
        const uint64_t k = ld_sys(&H->key[s]);
        if (k != ld_dev(&D->key[s])) st_dev(&D->key[s], k);
      }
    }
    if (__ballot(act) != 0) {
      last = now;
      if (lane == 0)
        __hip_atomic_fetch_max(&D->progress, now, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      const uint64_t pr = max(last, ld_dev(&D->progress));
      if (now > pr && now - pr > idle) break;
      __builtin_amdgcn_s_sleep(20);
    }
  }
}

// One row r of an item, by one wave.
__device__ void tail_row(const FuseItem& it, uint32_t r, int lane) {
  const uint32_t c4 = it.C / 4;
  const float4* x = reinterpret_cast<const float4*>(it.x) + (size_t)r * c4;
  float4* y = reinterpret_cast<float4*>(it.y) + (size_t)r * c4;
  const float* b = reinterpret_cast<const float*>(it.bias);
  const float4* b4 = reinterpret_cast<const float4*>(it.bias);
  const bool per_col = it.axis == 0;
  const float brow = per_col ? 0.0f : b[r];
  auto apply = [&](float4 v, uint32_t j) {
    const float4 bb = per_col ? b4[j] : make_float4(brow, brow, brow, brow);
    return make_float4(relu_add(v.x, bb.x), relu_add(v.y, bb.y), relu_add(v.z, bb.z),
                       relu_add(v.w, bb.w));
  };
  if (it.flags & kFuseSoftmax) {
    // row held in registers: at most 16 float4 per lane (C <= 4096)
    constexpr int NV = kFuseMaxSoftmaxRow / 256;
    float4 v[NV];
    float m = -INFINITY, sum = 0.0f;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const uint32_t j = lane + 64u * i;
      if (j < c4) {
        v[i] = apply(x[j], j);
        y[j] = v[i];
        sum += (v[i].x + v[i].y) + (v[i].z + v[i].w);
        m = fmaxf(m, fmaxf(fmaxf(v[i].x, v[i].y), fmaxf(v[i].z, v[i].w)));
      }
    }
    if (it.flags & kFuseRowsum) {
      sum = wave_sum(sum);
      if (lane == 0) reinterpret_cast<float*>(it.rs)[r] = sum;
    }
    m = wave_max(m);
    float e = 0.0f;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const uint32_t j = lane + 64u * i;
      if (j < c4) {
        v[i].x = expf(v[i].x - m);
        v[i].y = expf(v[i].y - m);
        v[i].z = expf(v[i].z - m);
        v[i].w = expf(v[i].w - m);
        e += (v[i].x + v[i].y) + (v[i].z + v[i].w);
      }
    }
    const float inv = 1.0f / wave_sum(e);
    float4* o = reinterpret_cast<float4*>(it.sm) + (size_t)r * c4;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const uint32_t j = lane + 64u * i;
      if (j < c4) o[j] = make_float4(v[i].x * inv, v[i].y * inv, v[i].z * inv, v[i].w * inv);
    }
    return;
  }
  // streaming: four loads in flight per lane
  float sum = 0.0f;
  uint32_t j = lane;
  for (; j + 192 < c4; j += 256) {
    float4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = x[j + 64 * u];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      v[u] = apply(v[u], j + 64 * u);
      y[j + 64 * u] = v[u];
      sum += (v[u].x + v[u].y) + (v[u].z + v[u].w);
    }
  }
  for (; j < c4; j += 64) {
    const float4 v = apply(x[j], j);
    y[j] = v;
    sum += (v.x + v.y) + (v.z + v.w);
  }
  if (it.flags & kFuseRowsum) {
    sum = wave_sum(sum);
    if (lane == 0) reinterpret_cast<float*>(it.rs)[r] = sum;
  }
}

__device__ void worker(FuseHost* __restrict__ H, FuseDev* __restrict__ D, uint64_t t0,
                       uint64_t idle, uint64_t lease, uint32_t log_cap) {
  __shared__ uint64_t sh_item[kItemWords];
  __shared__ uint32_t sh_cmd, sh_slot, sh_tile;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint64_t last = t0;
  for (;;) {
    if (wave == 0) {
      const uint64_t now = now_ticks();
      const uint32_t ctl = ld_dev(&D->ctl);
      uint32_t cmd;   // 0 run a tile, 1 leave, 2 wait, 3 retry
      uint64_t bk = ~0ull, bn = 0;
      int bs = -1;
      if ((ctl & 1u) || now - t0 > lease) {
        cmd = 1;
      } else {
        if (!(ctl & 2u)) {
          for (uint32_t s = lane; s < kFuseSlots; s += 64) {
            if (ld_dev(&D->state[s]) != 2u) continue;
            const uint64_t nx = ld_dev(&D->next[s]);
            if (uint32_t(nx) >= ld_dev(&D->item[s].tiles)) continue;
            const uint64_t k = ld_dev(&D->key[s]);
            if (bs < 0 || k < bk) {
              bk = k;
              bs = (int)s;
              bn = nx;
            }
          }
        }
        // wave-wide minimum of (key, slot)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
          const uint64_t ok = __shfl_xor(bk, off, 64);
          const int os = __shfl_xor(bs, off, 64);
          const uint64_t on = __shfl_xor(bn, off, 64);
          const bool take = os >= 0 && (bs < 0 || ok < bk || (ok == bk && os < bs));
          if (take) {
            bk = ok;
            bs = os;
            bn = on;
          }
        }
        if (bs < 0) {
          const uint64_t pr = max(last, ld_dev(&D->progress));
          cmd = (now > pr && now - pr > idle) ? 1u : 2u;
        } else {
          cmd = 3;
          if (lane == 0) {
            uint64_t expect = bn;
            if (__hip_atomic_compare_exchange_strong(&D->next[bs], &expect, bn + 1,
                                                     __ATOMIC_ACQ_REL, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT)) {
              cmd = 0;
              const uint64_t* src = reinterpret_cast<const uint64_t*>(&D->item[bs]);
#pragma unroll
              for (int w = 0; w < kItemWords; ++w) sh_item[w] = ld_dev(src + w);
              sh_slot = (uint32_t)bs;
              sh_tile = uint32_t(bn);
            }
          }
          cmd = __shfl(cmd, 0, 64);
        }
      }
      if (lane == 0) sh_cmd = cmd;
    }
    __syncthreads();
    const uint32_t cmd = sh_cmd;
    if (cmd == 1u) break;
    if (cmd == 2u) {
      if (wave == 0) __builtin_amdgcn_s_sleep(20);
    } else if (cmd == 0u) {
      FuseItem it;
      __builtin_memcpy(&it, sh_item, sizeof(FuseItem));
      const uint32_t tile = sh_tile, slot = sh_slot;
      const uint32_t r0 = tile * it.rows_per_tile;
      const uint32_t r1 = min(it.R, r0 + it.rows_per_tile);
      for (uint32_t r = r0 + wave; r < r1; r += 4) tail_row(it, r, lane);
      __syncthreads();
      if (threadIdx.x == 0) {
        __threadfence();   // the tile's results before its count
        const uint32_t f = __hip_atomic_fetch_add(&D->fin[slot], 1u, __ATOMIC_ACQ_REL,
                                                  __HIP_MEMORY_SCOPE_AGENT) + 1u;
        const uint64_t pubn = ld_dev(&D->seen[slot]);
        if (log_cap) {
          const uint32_t i = __hip_atomic_fetch_add(&D->log_n, 1u, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
          if (i < log_cap && i < kFuseLogCap) st_sys(&H->log[i], (pubn << 24) | tile);
        }
        __hip_atomic_fetch_add(&D->tiles_run, uint64_t(1), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        if (f == it.tiles) {
          st_dev(&D->state[slot], 0u);
          __threadfence_system();
          st_sys(&H->done[slot], pubn);
        }
        const uint64_t t = now_ticks();
        __hip_atomic_fetch_max(&D->progress, t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      last = now_ticks();
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void tail_executor(FuseHost* __restrict__ H,
                                                     FuseDev* __restrict__ D, uint64_t idle,
                                                     uint64_t lease, uint32_t log_cap) {
  const uint64_t t0 = now_ticks();
  if (blockIdx.x == 0) {
    if (threadIdx.x < 64) dispatcher(H, D, t0, idle, lease);
    return;
  }
  worker(H, D, t0, idle, lease, log_cap);
}

}  // namespace

uint32_t fuse_rows_per_tile(uint32_t C) {
  uint32_t r = C >= 8192 ? 4u : (32768u + C - 1) / C;
  return (r + 3u) & ~3u;
}

hipError_t fuse_executor_launch(FuseHost* h, FuseDev* d, uint32_t workers, int64_t idle_ns,
                                int64_t lease_ns, uint32_t log_cap, hipStream_t s) {
  if (workers < 1 || workers > 1024 || idle_ns <= 0 || lease_ns <= 0) return hipErrorInvalidValue;
  // device clock: 100 MHz
  const uint64_t idle = (uint64_t)idle_ns / 10u, lease = (uint64_t)lease_ns / 10u;
  hipLaunchKernelGGL(tail_executor, dim3(1 + workers), dim3(256), 0, s, h, d, idle, lease,
                     log_cap);
  return hipGetLastError();
}

}  // namespace ug
