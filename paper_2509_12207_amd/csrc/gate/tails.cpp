// Host side of the tail executor: slots, publication, keys, relaunches.
#include "tails.hpp"

#include <atomic>
#include <cstring>
#include <set>

#include "../kernels/ops.hpp"

namespace ug {

namespace {
// Stores seen by the executor through PCIe: plain stores in program order,
// the publication number last (release).
template <typename T>
void store_release(T* p, T v) {
  __atomic_store_n(p, v, __ATOMIC_RELEASE);
}
template <typename T>
T load_acquire(const T* p) {
  return __atomic_load_n(p, __ATOMIC_ACQUIRE);
}
}  // namespace

TailQueue::~TailQueue() {
  if (h_) (void)halt();
  if (ev_) (void)hipEventDestroy(ev_);
  if (own_stream_ && s_) (void)hipStreamDestroy(s_);
  if (d_) (void)hipFree(d_);
  if (h_) (void)hipHostFree(h_);
}

hipError_t TailQueue::open(int device, uint32_t workers, int64_t idle_ns, int64_t lease_ns,
                           uint32_t log_cap, hipStream_t stream) {
  if (h_) return hipErrorInvalidValue;
  if (workers < 1 || workers > kFuseMaxWorkers || idle_ns <= 0 || lease_ns <= 0 || log_cap > kFuseLogCap)
    return hipErrorInvalidValue;
  hipError_t e = hipSetDevice(device);
  if (e != hipSuccess) return e;
  // coherent pinned memory: the executor reads what the host writes (and the
  // host what it writes) without caching
  void* hp = nullptr;
  if ((e = hipHostMalloc(&hp, sizeof(FuseHost), hipHostMallocCoherent | hipHostMallocMapped)) !=
      hipSuccess)
    return e;
  h_ = static_cast<FuseHost*>(hp);
  std::memset(h_, 0, sizeof(FuseHost));
  void* dp = nullptr;
  if ((e = hipMalloc(&dp, sizeof(FuseDev))) != hipSuccess) return e;
  d_ = static_cast<FuseDev*>(dp);
  if ((e = hipMemset(d_, 0, sizeof(FuseDev))) != hipSuccess) return e;
  if (stream) {
    s_ = stream;
  } else {
    if ((e = hipStreamCreateWithFlags(&s_, hipStreamNonBlocking)) != hipSuccess) return e;
    own_stream_ = true;
  }
  if ((e = hipEventCreateWithFlags(&ev_, hipEventDisableTiming)) != hipSuccess) return e;
  workers_ = workers;
  idle_ns_ = idle_ns;
  lease_ns_ = lease_ns;
  log_cap_ = log_cap;
  free_.clear();
  for (uint32_t s = kFuseSlots; s-- > 0;) free_.push_back(s);
  busy_.assign(kFuseSlots, 0);
  return hipDeviceSynchronize();
}

bool TailQueue::reserve(uint32_t* slot) {
  if (free_.empty()) return false;
  *slot = free_.back();
  free_.pop_back();
  return true;
}

void TailQueue::unreserve(uint32_t slot) { free_.push_back(slot); }

uint64_t TailQueue::publish(uint32_t slot, const FuseItem& it, uint64_t key) {
  const uint64_t pub = ++next_pub_;
  h_->item[slot] = it;
  h_->item[slot].rows_per_tile = fuse_rows_per_tile(it.R, it.C, workers_);
  h_->item[slot].tiles = (it.R + h_->item[slot].rows_per_tile - 1) / h_->item[slot].rows_per_tile;
  store_release(&h_->key[slot], key);
  store_release(&h_->pub[slot], pub);
  store_release(&h_->ring[(pub - 1) % kFuseSlots], slot);
  store_release(&h_->ctl[kCtlNpub], pub);
  busy_[slot] = 1;
  ++outstanding_;
  return pub;
}

void TailQueue::set_key(uint32_t slot, uint64_t key) {
  if (load_acquire(&h_->key[slot]) == key) return;
  store_release(&h_->key[slot], key);
  keys_dirty_ = true;
}

void TailQueue::commit_keys() {
  if (!keys_dirty_) return;
  keys_dirty_ = false;
  store_release(&h_->ctl[kCtlKepoch], load_acquire(&h_->ctl[kCtlKepoch]) + 1);
}

bool TailQueue::finished(uint32_t slot, uint64_t pub) {
  if (!busy_[slot]) return true;
  if (load_acquire(&h_->done[slot]) != pub) return false;
  busy_[slot] = 0;
  --outstanding_;
  free_.push_back(slot);
  return true;
}

void TailQueue::set_pause(bool on) { store_release(&h_->ctl[kCtlPause], uint64_t(on ? 1 : 0)); }

hipError_t TailQueue::kick() {
  if (outstanding_ == 0) return hipSuccess;
  if (launched_) {
    const hipError_t q = hipEventQuery(ev_);
    if (q == hipErrorNotReady) return hipSuccess;   // still running
    if (q != hipSuccess) return q;
  }
  // launches are numbered from 1, modulo 2^32 but never 0 (a worker tells
  // this launch's commands from the previous one's)
  uint32_t launch = static_cast<uint32_t>(launches_ + 1);
  if (launch == 0) launch = 1;
  hipError_t e = fuse_executor_launch(h_, d_, workers_, launch, idle_ns_, lease_ns_, log_cap_, s_);
  if (e != hipSuccess) return e;
  if ((e = hipEventRecord(ev_, s_)) != hipSuccess) return e;
  launched_ = true;
  ++launches_;
  store_release(&h_->launches, launches_);
  return hipSuccess;
}

hipError_t TailQueue::halt() {
  if (!h_) return hipSuccess;
  store_release(&h_->ctl[kCtlStop], uint64_t(1));
  hipError_t e = hipStreamSynchronize(s_);
  store_release(&h_->ctl[kCtlStop], uint64_t(0));
  launched_ = false;
  return e;
}

uint32_t TailQueue::read_log(uint64_t* out, uint32_t cap) const {
  uint32_t n = 0;
  for (; n < cap && n < log_cap_; ++n) {
    const uint64_t v = load_acquire(&h_->log[n]);
    if (v == 0) break;
    out[n] = v;
  }
  return n;
}

hipError_t TailQueue::stats(uint64_t* out) const {
  if (!d_) return hipErrorInvalidValue;
  return hipMemcpy(out, d_->stats, sizeof(d_->stats), hipMemcpyDeviceToHost);
}

bool tail_item(const std::vector<ug_kernel>& ks, int32_t first, int32_t end,
               void* const* buffers, FuseItem* it) {
  const ug_kernel& k = ks[first];
  std::memset(it, 0, sizeof(*it));
  it->x = reinterpret_cast<uint64_t>(buffers[k.in[0]]);
  it->bias = reinterpret_cast<uint64_t>(buffers[k.in[1]]);
  it->y = reinterpret_cast<uint64_t>(buffers[k.out[0]]);
  it->R = static_cast<uint32_t>(k.shape[0]);
  it->C = static_cast<uint32_t>(k.shape[1]);
  it->axis = static_cast<uint32_t>(k.shape[2]);
  for (int32_t g = first + 1; g < end; ++g) {
    if (ks[g].op == UG_OP_SOFTMAX_F32) {
      it->sm = reinterpret_cast<uint64_t>(buffers[ks[g].out[0]]);
      it->flags |= kFuseSoftmax;
    } else {
      it->rs = reinterpret_cast<uint64_t>(buffers[ks[g].out[0]]);
      it->flags |= kFuseRowsum;
    }
  }
  uint64_t align = it->x | it->y | it->sm;
  if (it->axis == 0) align |= it->bias;
  return (align & 15) == 0;
}

void tail_runs(const std::vector<ug_kernel>& ks, int32_t lo, int32_t hi,
               std::vector<int32_t>* mark) {
  if (mark->size() < static_cast<size_t>(hi)) mark->resize(hi, -1);
  for (int32_t g = lo; g < hi; ++g) (*mark)[g] = -1;
  auto slots = [](const int32_t* v, int n, std::set<int32_t>* s) {
    for (int i = 0; i < n; ++i)
      if (v[i] >= 0) s->insert(v[i]);
  };
  auto contraction = [](int32_t op) {
    return op == UG_OP_GEMM_F32 || op == UG_OP_CONV3X3_F32 || op == UG_OP_GEMM_BF16 ||
           op == UG_OP_CONV3X3_BF16;
  };
  int32_t i = lo + 1;
  while (i < hi) {
    const ug_kernel& k = ks[i];
    const ug_kernel& prev = ks[i - 1];
    if (!(k.op == UG_OP_BIAS_RELU_F32 && contraction(prev.op) && k.in[0] == prev.out[0])) {
      ++i;
      continue;
    }
    const int64_t R = k.shape[0], C = k.shape[1];
    const int32_t y = k.out[0];
    int32_t end = i + 1;
    bool has_sm = false, has_rs = false;
    while (end < hi) {
      const ug_kernel& t = ks[end];
      const bool sm = t.op == UG_OP_SOFTMAX_F32, rs = t.op == UG_OP_ROWSUM_F32;
      if (!(sm || rs) || (sm && has_sm) || (rs && has_rs) || t.in[0] != y ||
          t.shape[0] != R || t.shape[1] != C)
        break;
      has_sm |= sm;
      has_rs |= rs;
      ++end;
    }
    bool ok = C % 4 == 0 && !(has_sm && C > kFuseMaxSoftmaxRow) && R < (int64_t(1) << 31) &&
              C < (int64_t(1) << 31) && 4 * R * C <= kFuseMaxTailBytes;
    for (int32_t g = i - 1; g < end && ok; ++g) ok = ks[g].frame_dim == 0;
    if (ok) {
      std::set<int32_t> reads, writes;
      for (int32_t g = i; g < end; ++g) {
        slots(ks[g].in, 3, &reads);
        slots(ks[g].out, 4, &writes);
      }
      for (int32_t g = end; g < hi && ok; ++g) {
        std::set<int32_t> r, w;
        slots(ks[g].in, 3, &r);
        slots(ks[g].out, 4, &w);
        for (int32_t s : w)
          if (reads.count(s) || writes.count(s)) ok = false;
        for (int32_t s : r)
          if (writes.count(s)) ok = false;
      }
    }
    if (ok) {
      (*mark)[i] = end;
      for (int32_t g = i + 1; g < end; ++g) (*mark)[g] = -2;
    }
    i = end;
  }
}

}  // namespace ug
