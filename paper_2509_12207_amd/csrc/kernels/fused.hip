// Tail executor (see fused.hpp for the protocol).
//
// The dispatcher (workgroup 0, wave 0) keeps eight queue slots per lane and
// one lane per 64th worker.  Each round it reads the host's control words,
// takes in new publications from the ring, re-reads keys after a rewrite,
// checks the counters of items waiting for their producer, collects the
// workers' acknowledgements, and gives every idle worker the next tile of
// the ready item with the smallest (key, slot), several workers at once
// when the item has tiles enough.
//
// A worker's four waves each take every fourth row of the tile and apply
// y = max(x + b, +0) (one FP32 add, -0 and NaN to +0: the bias+ReLU
// kernel's arithmetic), store y, and reduce the row for the row sum and
// the softmax.  Short rows are batched so that every lane has eight 16-byte
// loads in flight; a softmax row of up to 2048 floats stays in registers,
// a longer one (up to 4096) takes its maximum and its sum of exponentials
// in one pass (the online normaliser of Milakov and Gimelshein, 2018) and
// reads the stored y back, still in cache, for the output.
#include "fused.hpp"

namespace ug {
namespace {

constexpr uint32_t kPer = kFuseSlots / 64;   // slots per dispatcher lane
constexpr uint32_t kNoSlot = ~0u;
constexpr int kMailWords = 13;               // FuseItem, cmd, (slot, tile), op
constexpr uint64_t kTicksPerNs10 = 10;       // device clock: 100 MHz
constexpr uint32_t kBiasLds = 1024;          // float4 of per-column bias staged in LDS
constexpr uint32_t kLdsBytes = 24576;        // the executor's LDS (24 KiB: six workgroups a CU)

// Global-memory pointers (address space 1): the items' pointers arrive as
// integers, and without this the compiler would use flat accesses.
#define UG_GLOBAL __attribute__((address_space(1)))

__device__ __forceinline__ uint64_t now_ticks() { return __builtin_amdgcn_s_memrealtime(); }

template <typename T>
__device__ __forceinline__ T ld_sys(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
template <typename T>
__device__ __forceinline__ void st_sys(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
template <typename T>
__device__ __forceinline__ T ld(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// every memory operation of this wave issued so far has completed
__device__ __forceinline__ void settle() { __builtin_amdgcn_s_waitcnt(0); }

__device__ __forceinline__ float relu_add(float x, float b) {
  const float s = x + b;
  return s > 0.0f ? s : 0.0f;
}
// four floats in one 16-byte access
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 relu_add4(f4 v, f4 b) {
  return f4{relu_add(v.x, b.x), relu_add(v.y, b.y), relu_add(v.z, b.z), relu_add(v.w, b.w)};
}
__device__ __forceinline__ float sum4(f4 v) { return (v.x + v.y) + (v.z + v.w); }
__device__ __forceinline__ float max4(f4 v) { return fmaxf(fmaxf(v.x, v.y), fmaxf(v.z, v.w)); }
__device__ __forceinline__ f4 exp4(f4 v, float m) {
  return f4{expf(v.x - m), expf(v.y - m), expf(v.z - m), expf(v.w - m)};
}
__device__ __forceinline__ f4 scale4(f4 v, float s) { return v * s; }

// Wave-wide sum and maximum: xor swizzles within each half of the wave
// (no lane-index registers), then the two halves' results added.  The order
// is fixed, so the results are reproducible.
template <int X>
__device__ __forceinline__ float swz_xor(float v) {
  return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x1F | (X << 10)));
}
__device__ __forceinline__ float wave_sum(float v) {
  v += swz_xor<1>(v);
  v += swz_xor<2>(v);
  v += swz_xor<4>(v);
  v += swz_xor<8>(v);
  v += swz_xor<16>(v);
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0)) +
         __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
}
__device__ __forceinline__ float wave_max(float v) {
  v = fmaxf(v, swz_xor<1>(v));
  v = fmaxf(v, swz_xor<2>(v));
  v = fmaxf(v, swz_xor<4>(v));
  v = fmaxf(v, swz_xor<8>(v));
  v = fmaxf(v, swz_xor<16>(v));
  return fmaxf(__int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0)),
               __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32)));
}

// ------------------------------------------------------------- dispatcher

// The dispatcher's view of the slots, in LDS while it runs (kept in
// FuseDev::slot between launches).
struct SlotsLds {
  uint64_t key[kFuseSlots], pub[kFuseSlots], sig[kFuseSlots];
  uint32_t next[kFuseSlots], tiles[kFuseSlots], state[kFuseSlots], fin[kFuseSlots];
  uint32_t expected[kFuseSlots];
};

__device__ void dispatcher(FuseHost* __restrict__ H, FuseDev* __restrict__ D, uint32_t workers,
                           uint32_t launch, uint64_t t0, uint64_t idle, uint64_t lease,
                           uint32_t log_cap, unsigned char* lds) {
  SlotsLds& L = *reinterpret_cast<SlotsLds*>(lds);
  const uint32_t lane = threadIdx.x;
  const uint64_t tag = uint64_t(launch) << 32;
  const uint32_t groups = (workers + 63) / 64;   // workers per lane, at most 16
  const uint64_t drain = uint64_t(kFuseDrainNs) / kTicksPerNs10;
  // a new launch: no worker holds a command of it; the slots come in
  for (uint32_t w = lane; w < workers; w += 64) st(&D->wstate[w], uint64_t(kNoSlot));
#pragma unroll 2
  for (uint32_t i = 0; i < kPer; ++i) {
    const uint32_t s = lane + 64 * i;
    const FuseSlot* sl = &D->slot[s];
    L.key[s] = ld(&sl->key);
    L.pub[s] = ld(&sl->pub);
    L.sig[s] = ld(&sl->sig);
    L.next[s] = ld(&sl->next);
    L.tiles[s] = ld(&sl->tiles);
    L.state[s] = ld(&sl->state);
    L.fin[s] = ld(&sl->fin);
    L.expected[s] = ld(&sl->sig_expected);
  }
  // statistics of this launch (wave-uniform): rounds, their ticks, tiles;
  // finished items add their phases to FuseDev::stats when reported
  uint64_t st_rounds = 0, st_round_ticks = 0, st_tiles = 0;
  uint64_t npub_seen = ld(&D->npub_seen);
  uint32_t log_n = ld(&D->log_n);
  uint64_t kepoch_seen = ~0ull;   // keys are read again at the start
  uint64_t last = t0, t_leave = 0;
  bool leaving = false;
  // slots finished but not yet reported (an item of no tiles, or a launch
  // that left before reporting) are looked for in the next round
  bool report = true;
  settle();
  // control words of the first round; later rounds' are loaded at the end of
  // the round before, so that the PCIe read overlaps the round's work
  uint64_t cw = lane < 4 ? ld_sys(&H->ctl[lane]) : 0ull;
  for (;;) {
    const uint64_t now = now_ticks();
    bool act = false;

    // 3. items waiting for their producer (every counter loaded at once),
    // beside the first 64 workers' acknowledgements
    uint64_t ws0 = 0, a0 = 0;
    if (lane < workers) {
      ws0 = ld(&D->wstate[lane]);   // (sequence << 32) | slot in progress
      a0 = ld(&D->ack[lane]);
    }
    {
      unsigned cnt[kPer];
#pragma unroll
      for (uint32_t i = 0; i < kPer; ++i) {
        const uint32_t s = lane + 64 * i;
        cnt[i] = L.state[s] == 1u ? ld(reinterpret_cast<UG_GLOBAL unsigned*>(L.sig[s])) : 0u;
      }
      bool ready_any = false;
#pragma unroll
      for (uint32_t i = 0; i < kPer; ++i) {
        const uint32_t s = lane + 64 * i;
        if (L.state[s] == 1u && cnt[i] >= L.expected[s]) {
          // ready for the producer's next launch
          __hip_atomic_store(reinterpret_cast<UG_GLOBAL unsigned*>(L.sig[s]), 0u,
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          L.state[s] = 2u;
          st(&D->slot[s].t_ready, uint32_t(now));
          ready_any = true;
        }
      }
      if (__ballot(ready_any)) act = true;
    }

    // 4. acknowledgements: finished tiles, idle workers
    uint32_t avail = 0;   // bit g: worker lane + 64 g is alive and idle
    bool busy = false, fin_any = report;
    report = false;
#pragma unroll 2
    for (uint32_t g = 0; g < groups; ++g) {
      const uint32_t w = lane + 64 * g;
      if (w >= workers) break;
      const uint64_t ws = g == 0 ? ws0 : ld(&D->wstate[w]);
      const uint64_t a = g == 0 ? a0 : ld(&D->ack[w]);
      const uint32_t q = uint32_t(ws >> 32), sl = uint32_t(ws);
      if (a != (tag | q)) {
        busy |= sl != kNoSlot;
        continue;
      }
      avail |= 1u << g;
      if (sl == kNoSlot) continue;
      // the same lane reads wstate[w] next: program order keeps this store
      // ahead of that load
      st(&D->wstate[w], (uint64_t(q) << 32) | kNoSlot);
      if (atomicAdd(&L.fin[sl], 1u) + 1u == L.tiles[sl]) {
        L.state[sl] = 3u;   // finished, to be reported
        fin_any = true;
      }
    }
    if (__ballot(fin_any)) {
      act = true;
      // the workers' results (released before their acknowledgements) ahead
      // of the reports; each slot is reported by its own lane
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
#pragma unroll 2
      for (uint32_t i = 0; i < kPer; ++i) {
        const uint32_t s = lane + 64 * i;
        if (L.state[s] == 3u) {
          L.state[s] = 0u;
          st_sys(&H->done[s], L.pub[s]);
          const uint32_t ts = ld(&D->slot[s].t_seen), tr = ld(&D->slot[s].t_ready),
                         tf = ld(&D->slot[s].t_first);
          const uint64_t ph[4] = {1, uint32_t(tr - ts), uint32_t(tf - tr),
                                  uint32_t(uint32_t(now) - tf)};
#pragma unroll
          for (int k = 0; k < 4; ++k)
            __hip_atomic_fetch_add(&D->stats[kStatItems + k], ph[k], __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
      }
    }

    // the control words (read during the previous round)
    const uint64_t stop = __shfl(cw, kCtlStop, 64), pause = __shfl(cw, kCtlPause, 64);
    const uint64_t npub = __shfl(cw, kCtlNpub, 64), kepoch = __shfl(cw, kCtlKepoch, 64);
    if (!leaving && (stop || now - t0 > lease)) {
      leaving = true;
      t_leave = now;
    }

    // 1. new publications, in order, one per lane
    if (npub != npub_seen) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");   // the host's stores before npub
      bool empty = false;
      for (uint64_t base = npub_seen; base < npub; base += 64) {
        const uint64_t p = base + 1 + lane;
        if (p <= npub) {
          const uint32_t s = ld_sys(&H->ring[(p - 1) % kFuseSlots]) % kFuseSlots;
          const uint64_t* src = reinterpret_cast<const uint64_t*>(&H->item[s]);
          uint64_t* dst = reinterpret_cast<uint64_t*>(&D->item[s]);
          // the descriptor in two halves of five words (fewer registers)
          uint64_t wv[5];
#pragma unroll
          for (int i = 0; i < 5; ++i) wv[i] = ld_sys(src + i);
#pragma unroll
          for (int i = 0; i < 5; ++i) st(dst + i, wv[i]);
#pragma unroll
          for (int i = 0; i < 5; ++i) wv[i] = ld_sys(src + 5 + i);
          const uint64_t key = ld_sys(&H->key[s]);
#pragma unroll
          for (int i = 0; i < 5; ++i) st(dst + 5 + i, wv[i]);
          const uint32_t tiles = uint32_t(wv[4]);   // words 5..9: sig, (expected, R), .., tiles
          L.key[s] = key;
          L.pub[s] = p;
          L.sig[s] = wv[0];
          L.expected[s] = uint32_t(wv[1]);
          L.next[s] = 0u;
          L.fin[s] = 0u;
          L.tiles[s] = tiles;
          L.state[s] = tiles == 0u ? 3u : (wv[0] ? 1u : 2u);
          // the item's phase clock stays in device memory (read rarely)
          st(&D->slot[s].t_seen, uint32_t(now));
          st(&D->slot[s].t_ready, uint32_t(now));
          st(&D->slot[s].t_first, uint32_t(now));
          empty |= tiles == 0u;
        }
      }
      report = __ballot(empty) != 0ull;
      npub_seen = npub;
      act = true;
      // other lanes copy these descriptors into mailboxes below
      settle();
    }

    // 2. keys rewritten by the host
    if (kepoch != kepoch_seen) {
      kepoch_seen = kepoch;
#pragma unroll 2
      for (uint32_t i = 0; i < kPer; ++i) {
        const uint32_t s = lane + 64 * i;
        if (L.state[s] != 0u) L.key[s] = ld_sys(&H->key[s]);
      }
    }

    // 5. hand out tiles: idle workers take the ready tiles with the
    // smallest (key, slot), in order
    if (!pause && !leaving && __ballot(avail != 0u)) {
      // this lane's best slot: (key, slot) smallest, ready, with tiles left
      auto best = [&]() {
        uint32_t bi = kNoSlot;
        uint64_t bk = ~0ull;
#pragma unroll 2
        for (uint32_t i = 0; i < kPer; ++i) {
          const uint32_t s = lane + 64 * i;
          if (L.state[s] == 2u && L.next[s] < L.tiles[s] && (bi == kNoSlot || L.key[s] < bk)) {
            bk = L.key[s];
            bi = s;
          }
        }
        return bi;
      };
      uint32_t mine_best = best();
      for (uint32_t g = 0; g < groups; ++g) {
        uint64_t mask = __ballot((avail >> g) & 1u);
        while (mask) {
          // wave-wide minimum of (key, slot) over the lanes' best slots
          uint32_t bs = mine_best;
          uint64_t bk = bs == kNoSlot ? ~0ull : L.key[bs];
#pragma unroll
          for (int off = 32; off > 0; off >>= 1) {
            const uint64_t ok2 = __shfl_xor(bk, off, 64);
            const uint32_t os = __shfl_xor(bs, off, 64);
            if (os != kNoSlot && (bs == kNoSlot || ok2 < bk || (ok2 == bk && os < bs))) {
              bk = ok2;
              bs = os;
            }
          }
          bs = __builtin_amdgcn_readfirstlane(bs);
          if (bs == kNoSlot) break;   // nothing ready
          const uint32_t base = L.next[bs];
          const uint32_t rem = L.tiles[bs] - base;
          const uint32_t n_idle = uint32_t(__popcll(mask));
          const uint32_t take = n_idle < rem ? n_idle : rem;
          const uint64_t below = mask & ((1ull << lane) - 1ull);
          const uint32_t rank = uint32_t(__popcll(below));
          const bool mine = ((mask >> lane) & 1ull) && rank < take;
          if (mine) {
            const uint32_t w = lane + 64 * g;
            const uint32_t tile = base + rank;
            const uint32_t q = uint32_t(ld(&D->wstate[w]) >> 32) + 1u;
            FuseMail* mb = &D->mail[w];
            const uint64_t* src = reinterpret_cast<const uint64_t*>(&D->item[bs]);
            uint64_t* dst = reinterpret_cast<uint64_t*>(&mb->it);
#pragma unroll
            for (int i = 0; i < int(sizeof(FuseItem) / 8); ++i) st(dst + i, ld(src + i));
            st(&mb->slot, bs);
            st(&mb->tile, tile);
            st(&mb->op, 0u);
            st(&D->wstate[w], (uint64_t(q) << 32) | bs);
            if (log_cap && log_n + rank < log_cap && log_n + rank < kFuseLogCap)
              st_sys(&H->log[log_n + rank], (L.pub[bs] << 24) | tile);
            // the mailbox before its command
            __hip_atomic_store(&mb->cmd, tag | q, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
          }
          if (lane == bs % 64) {
            if (base == 0u) st(&D->slot[bs].t_first, uint32_t(now));
            L.next[bs] = base + take;
            mine_best = best();
          }
          log_n += take;
          st_tiles += take;
          // the lowest `take` idle lanes are served
          for (uint32_t t = 0; t < take; ++t) mask &= mask - 1ull;
          if (mine) avail &= ~(1u << g);
          busy |= mine;
          act = true;
        }
      }
    }

    // the next round's control words, in flight while this round ends
    cw = lane < 4 ? ld_sys(&H->ctl[lane]) : 0ull;

    // 6. progress, leaving
    const bool busy_any = __ballot(busy) != 0ull;
    if (__ballot(act) != 0ull) last = now;
    if (!leaving && !busy_any && now - last > idle) {
      leaving = true;
      t_leave = now;
    }
    st_rounds++;
    st_round_ticks += now_ticks() - now;
    if (leaving && (!busy_any || now - t_leave > drain)) break;
    if (__ballot(act) == 0ull) __builtin_amdgcn_s_sleep(4);
  }
  // every worker leaves
  for (uint32_t w = lane; w < workers; w += 64) st(&D->mail[w].op, 1u);
  for (uint32_t w = lane; w < workers; w += 64) {
    const uint32_t q = uint32_t(ld(&D->wstate[w]) >> 32) + 1u;
    __hip_atomic_store(&D->mail[w].cmd, tag | q, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
  // the slots go back to device memory for the next launch
#pragma unroll 2
  for (uint32_t i = 0; i < kPer; ++i) {
    const uint32_t s = lane + 64 * i;
    FuseSlot* sl = &D->slot[s];
    st(&sl->key, L.key[s]);
    st(&sl->pub, L.pub[s]);
    st(&sl->sig, L.sig[s]);
    st(&sl->next, L.next[s]);
    st(&sl->tiles, L.tiles[s]);
    st(&sl->state, L.state[s]);
    st(&sl->fin, L.fin[s]);
    st(&sl->sig_expected, L.expected[s]);
  }
  if (lane == 0) {
    __hip_atomic_fetch_add(&D->stats[kStatRounds], st_rounds, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_add(&D->stats[kStatRoundTicks], st_round_ticks, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_add(&D->stats[kStatTiles], st_tiles, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
  }
  if (lane == 0) {
    st(&D->npub_seen, npub_seen);
    st(&D->log_n, log_n);
  }
}

// ---------------------------------------------------------------- workers

using gfloat4 = UG_GLOBAL f4;
using gfloat = UG_GLOBAL float;

// Element j of a row whose base is uniform across the wave: scalar base,
// 32-bit vector offset.
__device__ __forceinline__ f4 ld4(const gfloat4* row, uint32_t j) {
  return *reinterpret_cast<const gfloat4*>(reinterpret_cast<const UG_GLOBAL char*>(row) + j * 16u);
}
__device__ __forceinline__ void st4(gfloat4* row, uint32_t j, f4 v) {
  *reinterpret_cast<gfloat4*>(reinterpret_cast<UG_GLOBAL char*>(row) + j * 16u) = v;
}

struct Rows {
  const gfloat4* x;
  gfloat4* y;
  const gfloat* b;    // the bias in global memory
  const f4* lb;       // a per-column bias staged in LDS (C <= 4096)
  gfloat4* sm;
  gfloat* rs;
  uint32_t c4;
  bool per_col, do_rs;
};

template <bool LB>
__device__ __forceinline__ f4 bias_of(const Rows& t, uint32_t j, float br) {
  if (!t.per_col) return f4{br, br, br, br};
  return LB ? t.lb[j] : ld4(reinterpret_cast<const gfloat4*>(t.b), j);
}

// Rows r, r + 4, ... below r1 of rows of at most 64 * NB float4 (NB <= 4),
// G = 8 / NB rows at a time; softmax rows stay in registers.  Loads are never skipped
// (an index past the row or the tile reads the last valid element again) so
// that all eight are issued back to back; stores and sums are masked.
template <int NB, bool SM>
__device__ void rows_short(const Rows& t, uint32_t r, uint32_t r1, uint32_t lane) {
  constexpr int G = 8 / NB;
  const uint32_t jmax = t.c4 - 1;
  for (; r < r1; r += 4 * G) {
    f4 v[G * NB];
#pragma unroll
    for (int q = 0; q < G; ++q) {
      const uint32_t row = min(r + 4 * q, r1 - 1);
#pragma unroll
      for (int u = 0; u < NB; ++u)
        v[q * NB + u] = ld4(t.x + size_t(row) * t.c4, min(lane + 64 * u, jmax));
    }
#pragma unroll
    for (int q = 0; q < G; ++q) {
      const uint32_t row = r + 4 * q;
      if (row >= r1) break;
      const float br = t.per_col ? 0.0f : t.b[row];
      float s = 0.0f, m = -INFINITY;
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const uint32_t j = lane + 64 * u;
        const bool in = j < t.c4;
        f4& e = v[q * NB + u];
        e = relu_add4(e, bias_of<true>(t, min(j, jmax), br));
        if (in) st4(t.y + size_t(row) * t.c4, j, e);
        s += in ? sum4(e) : 0.0f;
        if (SM) m = in ? fmaxf(m, max4(e)) : m;
      }
      if (t.do_rs) {
        s = wave_sum(s);
        if (lane == 0) t.rs[row] = s;
      }
      if (SM) {
        m = wave_max(m);
        float es = 0.0f;
#pragma unroll
        for (int u = 0; u < NB; ++u) {
          f4& e = v[q * NB + u];
          e = exp4(e, m);
          es += lane + 64 * u < t.c4 ? sum4(e) : 0.0f;
        }
        const float inv = 1.0f / wave_sum(es);
#pragma unroll
        for (int u = 0; u < NB; ++u) {
          const uint32_t j = lane + 64 * u;
          if (j < t.c4) st4(t.sm + size_t(row) * t.c4, j, scale4(v[q * NB + u], inv));
        }
      }
    }
  }
}

// Long rows, one per wave at a time, U float4 per lane in flight, loads
// clamped as above.  With SM
// the row's maximum and sum of exponentials are kept as a running pair,
// rescaled when a chunk raises the maximum; the softmax is then written
// from the stored y.
template <bool SM, bool LB, int U>
__device__ void rows_long(const Rows& t, uint32_t r, uint32_t r1, uint32_t lane) {
  const uint32_t jmax = t.c4 - 1;
  for (; r < r1; r += 4) {
    const float br = t.per_col ? 0.0f : t.b[r];
    const gfloat4* x = t.x + size_t(r) * t.c4;
    gfloat4* y = t.y + size_t(r) * t.c4;
    float s = 0.0f, m = -INFINITY, es = 0.0f;
    for (uint32_t j0 = lane; j0 < t.c4; j0 += 64 * U) {
      f4 v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = ld4(x, min(j0 + 64 * u, jmax));
      float cm = -INFINITY;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint32_t j = j0 + 64 * u;
        const bool in = j < t.c4;
        v[u] = relu_add4(v[u], bias_of<LB>(t, min(j, jmax), br));
        if (in) st4(y, j, v[u]);
        s += in ? sum4(v[u]) : 0.0f;
        if (SM) cm = in ? fmaxf(cm, max4(v[u])) : cm;
      }
      if (SM) {
        if (cm > m) {
          es *= expf(m - cm);
          m = cm;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) es += j0 + 64 * u < t.c4 ? sum4(exp4(v[u], m)) : 0.0f;
      }
    }
    if (t.do_rs) {
      const float rsum = wave_sum(s);
      if (lane == 0) t.rs[r] = rsum;
    }
    if (SM) {
      const float M = wave_max(m);
      const float inv = 1.0f / wave_sum(m == -INFINITY ? 0.0f : es * expf(m - M));
      gfloat4* o = t.sm + size_t(r) * t.c4;
      for (uint32_t j0 = lane; j0 < t.c4; j0 += 64 * U) {
        f4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = ld4(y, min(j0 + 64 * u, jmax));
#pragma unroll
        for (int u = 0; u < U; ++u)
          if (j0 + 64 * u < t.c4) st4(o, j0 + 64 * u, scale4(exp4(v[u], M), inv));
      }
    }
  }
}

// Long rows without a softmax whose per-column bias is too long for LDS:
// two rows a pass (this wave's rows r and r + 4), so that each chunk of the
// bias, read from global memory, serves both, and eight loads of x are in
// flight beside four of the bias.
__device__ void rows_long_pair(const Rows& t, uint32_t r, uint32_t r1, uint32_t lane) {
  constexpr int U = 4;
  const uint32_t jmax = t.c4 - 1;
  const gfloat4* b4 = reinterpret_cast<const gfloat4*>(t.b);
  for (; r < r1; r += 8) {
    const bool two = r + 4 < r1;   // the same in every lane
    const uint32_t r2 = two ? r + 4 : r;
    const gfloat4* xa = t.x + size_t(r) * t.c4;
    const gfloat4* xb = t.x + size_t(r2) * t.c4;
    gfloat4* ya = t.y + size_t(r) * t.c4;
    gfloat4* yb = t.y + size_t(r2) * t.c4;
    float sa = 0.0f, sb = 0.0f;
    for (uint32_t j0 = lane; j0 < t.c4; j0 += 64 * U) {
      f4 bb[U], va[U], vb[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint32_t jj = min(j0 + 64 * u, jmax);
        bb[u] = ld4(b4, jj);
        va[u] = ld4(xa, jj);
        vb[u] = ld4(xb, jj);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint32_t j = j0 + 64 * u;
        const bool in = j < t.c4;
        va[u] = relu_add4(va[u], bb[u]);
        vb[u] = relu_add4(vb[u], bb[u]);
        if (in) st4(ya, j, va[u]);
        if (in && two) st4(yb, j, vb[u]);
        sa += in ? sum4(va[u]) : 0.0f;
        sb += in ? sum4(vb[u]) : 0.0f;
      }
    }
    if (t.do_rs) {
      const float ra = wave_sum(sa), rb = wave_sum(sb);
      if (lane == 0) {
        t.rs[r] = ra;
        if (two) t.rs[r2] = rb;
      }
    }
  }
}

__device__ void run_tile(const FuseItem& it, uint32_t tile, uint32_t wave, uint32_t lane,
                         const f4* lb) {
  Rows t;
  t.x = reinterpret_cast<const gfloat4*>(it.x);
  t.y = reinterpret_cast<gfloat4*>(it.y);
  t.b = reinterpret_cast<const gfloat*>(it.bias);
  t.lb = lb;
  t.sm = reinterpret_cast<gfloat4*>(it.sm);
  t.rs = reinterpret_cast<gfloat*>(it.rs);
  t.c4 = it.C / 4;
  t.per_col = it.axis == 0;
  t.do_rs = (it.flags & kFuseRowsum) != 0;
  const uint32_t r0 = tile * it.rows_per_tile + wave;
  const uint32_t r1 = min(it.R, (tile + 1) * it.rows_per_tile);
  const uint32_t nb = (t.c4 + 63) / 64;
  if (it.flags & kFuseSoftmax) {
    if (nb <= 1) rows_short<1, true>(t, r0, r1, lane);
    else if (nb <= 2) rows_short<2, true>(t, r0, r1, lane);
    else if (nb <= 4) rows_short<4, true>(t, r0, r1, lane);
    else rows_long<true, true, 8>(t, r0, r1, lane);
  } else {
    if (nb <= 1) rows_short<1, false>(t, r0, r1, lane);
    else if (nb <= 2) rows_short<2, false>(t, r0, r1, lane);
    else if (nb <= 4) rows_short<4, false>(t, r0, r1, lane);
    else if (!t.per_col || nb <= kBiasLds / 64) rows_long<false, true, 8>(t, r0, r1, lane);
    else rows_long_pair(t, r0, r1, lane);
  }
}

__device__ void worker(FuseDev* __restrict__ D, uint32_t w, uint32_t launch, uint64_t t0,
                       uint64_t lease, unsigned char* lds) {
  f4* lb = reinterpret_cast<f4*>(lds);
  uint64_t lb_src = 0;   // the bias staged in lb (pointer), and its length
  uint32_t lb_c4 = 0;
  __shared__ uint64_t sh[kMailWords];
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint64_t tag = uint64_t(launch) << 32;
  const uint64_t give_up = lease + 2 * (uint64_t(kFuseDrainNs) / kTicksPerNs10);
  FuseMail* mb = &D->mail[w];
  if (threadIdx.x == 0) st(&D->ack[w], tag);   // alive and idle
  uint32_t seq = 0;
  for (;;) {
    if (wave == 0) {
      uint64_t c = 0;
      bool quit = false;
      for (;;) {
        const uint64_t v = ld(&mb->cmd);   // the same word in every lane
        c = (uint64_t(__builtin_amdgcn_readfirstlane(uint32_t(v >> 32))) << 32) |
            __builtin_amdgcn_readfirstlane(uint32_t(v));
        if ((c >> 32) == launch && uint32_t(c) != seq) break;
        if (now_ticks() - t0 > give_up) {
          quit = true;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
      if (quit) {
        if (lane == 0) sh[12] = 1;   // op: leave
      } else {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // the item's inputs
        const uint64_t* mw = reinterpret_cast<const uint64_t*>(mb);
        if (lane < 10 || lane == 11) sh[lane] = ld(mw + lane);   // descriptor, (slot, tile)
        if (lane == 10) sh[10] = c;
        if (lane == 12) sh[12] = ld(&mb->op);
      }
    }
    __syncthreads();
    const uint64_t cmd = sh[10];
    const uint32_t op = uint32_t(sh[12]);
    if (op != 0u) break;
    // the descriptor is the same in every lane: scalar registers
    FuseItem it;
    uint32_t* iw = reinterpret_cast<uint32_t*>(&it);
    const uint32_t* sw = reinterpret_cast<const uint32_t*>(sh);
#pragma unroll
    for (int i = 0; i < int(sizeof(FuseItem) / 4); ++i) iw[i] = __builtin_amdgcn_readfirstlane(sw[i]);
    const uint32_t tile = __builtin_amdgcn_readfirstlane(uint32_t(sh[11] >> 32));
    const uint32_t c4 = it.C / 4;
    const bool stage = it.axis == 0 && c4 <= kBiasLds;
    if (stage && (it.bias != lb_src || c4 != lb_c4)) {
      // a per-column bias is read by every row: staged once per item
      const gfloat4* b4 = reinterpret_cast<const gfloat4*>(it.bias);
      for (uint32_t j = threadIdx.x; j < c4; j += 256) lb[j] = ld4(b4, j);
      lb_src = it.bias;
      lb_c4 = c4;
      __syncthreads();
    }
    run_tile(it, tile, wave, lane, stage ? lb : nullptr);
    __syncthreads();
    if (threadIdx.x == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");   // the tile's results first
      st(&D->ack[w], cmd);
    }
    seq = uint32_t(cmd);
  }
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void tail_executor(
    FuseHost* __restrict__ H, FuseDev* __restrict__ D, uint32_t workers, uint32_t launch,
    uint64_t idle, uint64_t lease, uint32_t log_cap) {
  // the dispatcher's slot staging, or a worker's bias
  __shared__ __attribute__((aligned(16))) unsigned char lds[kLdsBytes];
  static_assert(kLdsBytes >= sizeof(SlotsLds) && kLdsBytes >= 16 * kBiasLds, "LDS use fits");
  const uint64_t t0 = now_ticks();
  if (blockIdx.x == 0) {
    if (threadIdx.x < 64) dispatcher(H, D, workers, launch, t0, idle, lease, log_cap, lds);
    return;
  }
  worker(D, blockIdx.x - 1, launch, t0, lease, lds);
}

}  // namespace

uint32_t fuse_rows_per_tile(uint32_t R, uint32_t C, uint32_t workers) {
  const uint64_t row = 4ull * (C ? C : 1);
  const uint64_t hi = row >= 524288 ? 1 : 524288 / row;
  uint64_t lo = (65536 + row - 1) / row;
  if (lo > hi) lo = hi;
  const uint64_t w = workers ? workers : 1;
  uint64_t r = (uint64_t(R) + w - 1) / w;
  r = r < lo ? lo : (r > hi ? hi : r);
  return uint32_t((r + 3) & ~3ull);
}

hipError_t fuse_executor_launch(FuseHost* h, FuseDev* d, uint32_t workers, uint32_t launch,
                                int64_t idle_ns, int64_t lease_ns, uint32_t log_cap,
                                hipStream_t s) {
  if (workers < 1 || workers > kFuseMaxWorkers || launch == 0 || idle_ns <= 0 || lease_ns <= 0)
    return hipErrorInvalidValue;
  const uint64_t idle = uint64_t(idle_ns) / kTicksPerNs10;
  const uint64_t lease = uint64_t(lease_ns) / kTicksPerNs10;
  hipLaunchKernelGGL(tail_executor, dim3(1 + workers), dim3(256), 0, s, h, d, workers, launch,
                     idle, lease, log_cap);
  return hipGetLastError();
}

}  // namespace ug
