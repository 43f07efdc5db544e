// Tail executor: a long-lived kernel that runs fused tails (bias+ReLU of a
// contraction's output, then optionally the row softmax and the row sum of
// that result) taken from a queue, most urgent first.
//
// Memory shared by the host gate and the executor:
//   FuseHost  pinned, coherent host memory.  The gate writes an item's
//             descriptor and key into a free slot, the slot's number into
//             the publication ring, then the publication count (npub,
//             last); it rewrites keys whenever its urgency order changes,
//             then bumps kepoch.  While nothing changes the executor reads
//             only the four control words.  The executor writes `done` (the
//             publication number of the slot's finished item) and the
//             service log.
//   FuseDev   device memory, zeroed once and kept across launches.
//
// Workgroup 0, wave 0 of the executor is the dispatcher; it alone owns the
// slots' state (FuseSlot, held in its LDS while it runs).  It takes in new publications, marks an item
// ready once its producer's counter is complete, and hands tiles of ready
// items, smallest key first, to idle workers through one mailbox each.
// A worker (workgroups 1..) waits on its mailbox, runs the tile with its
// four waves and acknowledges it; the dispatcher counts finished tiles and
// reports a finished item to the host.  Polling loops use relaxed loads
// only: one acquire per command taken and one release per tile finished
// (and per batch of commands or reports), so that the caches the other
// kernels share are not flushed on every poll.
//
// A producer (a contraction launched with a completion counter) adds each
// workgroup's wavefront count to the counter once the workgroup's results
// are stored (signal.hpp); the item is ready when the counter reaches the
// producer's wavefront count, and the dispatcher then resets it to zero for
// the producer's next launch.
//
// Every wait of the executor is bounded: the dispatcher leaves when the host
// sets `stop`, when nothing has progressed for `idle` nanoseconds, or at the
// end of its lease, after the tiles it handed out are finished (at most
// kFuseDrainNs more); it then sends every worker a command to leave, and a
// worker that hears nothing leaves after the lease and twice the drain
// bound.  The host launches the executor again while items are pending and
// it is not running.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ug {

constexpr uint32_t kFuseSlots = 512;      // items queued at once (8 per dispatcher lane)
constexpr uint32_t kFuseMaxWorkers = 1024;
constexpr uint32_t kFuseLogCap = 8192;    // service-log entries (tests)
constexpr uint32_t kFuseMaxSoftmaxRow = 4096;   // longest row with a fused softmax
constexpr int64_t kFuseDrainNs = 2000000000;    // tiles handed out finish within this

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

// FuseHost::ctl words.
constexpr int kCtlStop = 0, kCtlPause = 1, kCtlNpub = 2, kCtlKepoch = 3;

struct FuseHost {
  uint64_t ctl[4];                 // host: stop, pause, npub (after each publication),
                                   // kepoch (after each batch of key rewrites)
  uint64_t pub[kFuseSlots];        // host: publication number of the slot's item
  uint64_t key[kFuseSlots];        // host: the slot's key (smaller is served first)
  uint64_t done[kFuseSlots];       // device: publication number of the slot's finished item
  uint32_t ring[kFuseSlots];       // host: slot of publication p at ring[(p - 1) % kFuseSlots]
  FuseItem item[kFuseSlots];       // host: the slot's descriptor
  uint64_t launches;               // host: executor launches so far
  uint64_t log[kFuseLogCap];       // device: (pub << 24) | tile, per tile handed out
};

// The dispatcher's record of a slot.
struct FuseSlot {
  uint64_t key, pub, sig;
  uint32_t state;                  // 0 free or finished, 1 waiting for the producer, 2 ready
  uint32_t next;                   // next tile to hand out
  uint32_t tiles, fin;             // tiles in all, tiles finished
  uint32_t sig_expected;
  uint32_t t_seen, t_ready, t_first;   // device clock (low 32 bits): taken in, ready,
                                       // first tile handed out
  uint32_t pad[2];
};
static_assert(sizeof(FuseSlot) == 64, "slot layout");

// FuseDev::stats, accumulated over the executor's launches (device clock
// ticks of 10 ns).
enum FuseStat {
  kStatRounds = 0,     // dispatcher rounds
  kStatRoundTicks,     // their total duration
  kStatItems,          // items finished
  kStatWaitTicks,      // taken in -> ready (waiting for the producer), summed
  kStatQueueTicks,     // ready -> first tile handed out, summed
  kStatServeTicks,     // first tile handed out -> finished, summed
  kStatTiles,          // tiles handed out
  kStatCount = 8
};

// A command from the dispatcher to one worker.
struct FuseMail {
  FuseItem it;
  uint64_t cmd;                    // (launch << 32) | sequence number
  uint32_t slot, tile;
  uint32_t op;                     // 0 run the tile, 1 leave
  uint32_t pad[7];
};
static_assert(sizeof(FuseMail) == 128, "mailbox layout");

struct FuseDev {
  FuseSlot slot[kFuseSlots];
  FuseItem item[kFuseSlots];       // descriptors taken in from the host
  uint64_t ack[kFuseMaxWorkers];   // worker: last command finished, (launch << 32) | seq
  uint64_t wstate[kFuseMaxWorkers];// dispatcher: (last sequence number sent << 32) |
                                   // slot of the tile in progress (or ~0u)
  FuseMail mail[kFuseMaxWorkers];
  uint64_t npub_seen;              // publications taken in
  uint32_t log_n;                  // service-log entries written
  uint32_t pad;
  uint64_t stats[kStatCount];
};

// Launches the executor: one dispatcher workgroup and `workers` worker
// workgroups of 256 threads.  `launch` numbers the launch (from 1, distinct
// from the previous launch's); idle_ns and lease_ns bound its life (device
// clock, 100 MHz); log_cap > 0 records the first log_cap tiles handed out.
hipError_t fuse_executor_launch(FuseHost* h, FuseDev* d, uint32_t workers, uint32_t launch,
                                int64_t idle_ns, int64_t lease_ns, uint32_t log_cap,
                                hipStream_t s);

// Rows per tile of an item of R rows of C floats served by `workers`
// workers: about R / workers, kept between 64 KiB and 512 KiB of input (at
// least one row), rounded up to a multiple of 4 (one row per wave).  A
// tile costs one dispatcher round trip of a few microseconds, which a
// 512 KiB tile (tens of microseconds on one workgroup) makes small, and the
// worker's L2 invalidate and write-back (its acquire and release), which
// the other kernels on that XCD feel: the floor keeps a short tail to a
// few tiles.
uint32_t fuse_rows_per_tile(uint32_t R, uint32_t C, uint32_t workers);

}  // namespace ug
