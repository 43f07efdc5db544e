// Host side of the tail executor (kernels/fused.hpp): the queue slots, the
// executor's stream and its relaunches.  One TailQueue per gate (or per
// direct user of the C-ABI); every call comes from one thread at a time.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "../kernels/fused.hpp"
#include "ug.h"

namespace ug {

// The gate fuses short kernels only: a tail's bias+ReLU input is at most
// this many bytes (larger tails launch as usual, at full-device bandwidth).
constexpr int64_t kFuseMaxTailBytes = int64_t(1) << 20;

class TailQueue {
 public:
  TailQueue() = default;
  TailQueue(const TailQueue&) = delete;
  TailQueue& operator=(const TailQueue&) = delete;
  ~TailQueue();

  // Allocates the shared memory (pinned host, device) and, unless `stream`
  // is given, a stream of its own at the default priority.
  hipError_t open(int device, uint32_t workers, int64_t idle_ns, int64_t lease_ns,
                  uint32_t log_cap, hipStream_t stream = nullptr);
  hipStream_t stream() const { return s_; }
  bool is_open() const { return h_ != nullptr; }

  // Takes a free slot (false: all kSlots are taken).
  bool reserve(uint32_t* slot);
  // Returns a reserved slot that was never published.
  void unreserve(uint32_t slot);
  // Publication number the next publish will give.
  uint64_t next_pub() const { return next_pub_ + 1; }
  // Publishes an item into a reserved slot with its first key (the item's
  // rows per tile and tile count are set here, for this queue's workers);
  // returns its publication number.
  uint64_t publish(uint32_t slot, const FuseItem& it, uint64_t key);
  // Rewrites a published item's key (takes effect at the next commit_keys).
  void set_key(uint32_t slot, uint64_t key);
  void commit_keys();
  // True once the item published as `pub` in `slot` has finished; the slot
  // is then free again.
  bool finished(uint32_t slot, uint64_t pub);
  void set_pause(bool on);
  // Launches the executor if items are outstanding and it is not running.
  hipError_t kick();
  // Stops the executor and waits for its stream.
  hipError_t halt();
  uint32_t outstanding() const { return outstanding_; }
  uint64_t launches() const { return launches_; }
  // Service log entries (pub << 24 | tile) written so far, up to cap.
  uint32_t read_log(uint64_t* out, uint32_t cap) const;
  // The executor's statistics (FuseStat), as of its last exit.
  hipError_t stats(uint64_t* out) const;

 private:
  FuseHost* h_ = nullptr;
  FuseDev* d_ = nullptr;
  hipStream_t s_ = nullptr;
  bool own_stream_ = false;
  hipEvent_t ev_ = nullptr;
  bool launched_ = false;
  uint32_t workers_ = 0, log_cap_ = 0;
  int64_t idle_ns_ = 0, lease_ns_ = 0;
  std::vector<uint32_t> free_;
  std::vector<uint8_t> busy_;     // published, not yet seen finished
  uint64_t next_pub_ = 0;
  uint32_t outstanding_ = 0;
  uint64_t launches_ = 0;
  bool keys_dirty_ = false;
};

// Descriptor of the tail that kernel `first` of a task starts (kernels
// [first, end) of `ks`), for the frame's buffers; false if the frame's
// buffers are not 16-byte aligned (the tail then runs as ordinary launches).
bool tail_item(const std::vector<ug_kernel>& ks, int32_t first, int32_t end,
               void* const* buffers, FuseItem* it);

// Tails of the kernels [lo, hi) of one task: for each kernel, the end of
// the tail it starts (> index), or -1; a kernel inside a tail (not its
// first) gets -2.  The rule: a bias+ReLU right after a contraction (FP32 or
// BF16 GEMM or 3x3 convolution) whose output it reads, with at most one
// row softmax and one row sum of its output after it (same rows and row
// length), row length a multiple of 4 (at most 4096 with a softmax), at
// most kFuseMaxTailBytes of input, no per-frame sizes, and no later kernel
// of the task writing a buffer the tail reads or writes or reading one it
// writes.
void tail_runs(const std::vector<ug_kernel>& ks, int32_t lo, int32_t hi,
               std::vector<int32_t>* mark);

}  // namespace ug
