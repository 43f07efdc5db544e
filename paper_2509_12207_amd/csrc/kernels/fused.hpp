// Tail executor: a long-lived kernel that runs fused tails (bias+ReLU of a
// contraction's output, then optionally the row softmax and the row sum of
// that result) taken from a queue in device memory, most urgent first.
//
// Memory shared by the host gate and the executor:
//   FuseHost  pinned, coherent host memory.  The gate writes an item's
//             descriptor and key, then its publication number (pub) and
//             the publication count (npub, last); it rewrites keys whenever
//             its urgency order changes, then bumps kepoch.  The executor
//             polls only npub and kepoch while nothing changes.  The
//             executor writes `done` (the publication number of the slot's
//             finished item) and the service log.
//   FuseDev   device memory (zeroed before the first launch, then kept
//             across launches).  Workgroup 0 of the executor (the
//             dispatcher) copies new descriptors from the host, watches the
//             producers' completion counters and mirrors keys and control
//             words; the other workgroups (workers) claim tiles of ready
//             items with device-scope atomics and never read host memory
//             but to report completion.
//
// A producer (a contraction launched with a completion counter) adds one to
// the counter per wavefront once that wavefront's results are stored; the
// item is ready when the counter reaches the producer's wavefront count, and
// the dispatcher then resets it to zero for the producer's next launch.
//
// Every wait of the executor is bounded: it leaves when the host sets
// `stop`, when nothing has progressed for `idle` nanoseconds, or at the end
// of its lease; claimed tiles are always finished first.  The host launches
// it again while items are pending and it is not running.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ug {

constexpr uint32_t kFuseSlots = 512;      // items queued at once (8 per lane of a wave)
constexpr uint32_t kFuseLogCap = 8192;    // service-log entries (tests)
constexpr uint32_t kFuseMaxSoftmaxRow = 4096;   // softmax rows held in registers

// Stages of an item (FuseItem::flags).
constexpr uint32_t kFuseSoftmax = 1u;
constexpr uint32_t kFuseRowsum = 2u;

struct FuseItem {
  uint64_t x;              // const float X[R, C]: the bias+ReLU input
  uint64_t y;              // float Y[R, C]: its output (may equal X)
  uint64_t bias;           // const float b[C] (axis 0) or b[R] (axis 1)
  uint64_t sm;             // float SM[R, C]: softmax of the rows of Y
  uint64_t rs;             // float RS[R]: sums of the rows of Y
  uint64_t sig;            // unsigned*: the producer's counter (0: ready at once)
  uint32_t sig_expected;   // wavefronts of the producer
  uint32_t R, C, axis, flags;
  uint32_t rows_per_tile, tiles;
  uint32_t pad;
};
static_assert(sizeof(FuseItem) == 80, "descriptor layout");

struct FuseHost {
  uint64_t stop;
  uint64_t pause;
  uint64_t npub;                   // host: publications so far (after each pub)
  uint64_t kepoch;                 // host: key rewrites so far (after the keys)
  uint64_t pub[kFuseSlots];
  uint64_t key[kFuseSlots];
  uint64_t done[kFuseSlots];
  FuseItem item[kFuseSlots];
  uint64_t launches;               // host: executor launches so far
  uint64_t log[kFuseLogCap];       // device: (pub << 24) | tile, per served tile
};

struct FuseDev {
  uint64_t seen[kFuseSlots];       // publication number copied
  uint64_t key[kFuseSlots];
  uint64_t next[kFuseSlots];       // (generation << 32) | next tile to claim
  uint32_t state[kFuseSlots];      // 0 idle/finished, 1 waiting for producer, 2 ready
  uint32_t fin[kFuseSlots];        // tiles finished
  uint32_t gen[kFuseSlots];
  uint32_t ctl;                    // bit 0 stop, bit 1 pause (mirrored by the dispatcher)
  uint32_t log_n;                  // service-log entries written
  uint64_t progress;               // device clock of the last progress
  uint64_t tiles_run;              // tiles served since the memory was zeroed
  FuseItem item[kFuseSlots];
};

// Launches the executor: one dispatcher workgroup and `workers` worker
// workgroups of 256 threads.  idle_ns and lease_ns bound its life (device
// clock, 100 MHz); log_cap > 0 records the first log_cap served tiles.
hipError_t fuse_executor_launch(FuseHost* h, FuseDev* d, uint32_t workers, int64_t idle_ns,
                                int64_t lease_ns, uint32_t log_cap, hipStream_t s);

// Rows per tile of an item with rows of C floats (a multiple of 4, about
// 128 KiB of input per tile, at least 4 rows).
uint32_t fuse_rows_per_tile(uint32_t C);

}  // namespace ug
