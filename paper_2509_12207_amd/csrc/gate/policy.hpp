// Urgency-ordered launch policy (UrgenGo, arXiv 2509.12207, Sec. 4.2-4.4),
// as a pure state machine over decision instants.  No clock, no HIP: the
// gate thread (runtime.cpp) feeds it the inputs it observed at an instant and
// executes the decisions it returns; ug_replay_instant feeds it a recorded
// instant offline.
//
// Per instant t:
//   1. apply inputs in canonical order: arrivals by (chain, frame), then
//      observed events by (chain, frame, task, seq).  A batch-start event
//      moves the chain instance's executing-kernel index to the first kernel
//      of that batch (every earlier batch is done); a task-end event finishes
//      the task, frees its per-chain task slot and queues the frame for its
//      next task (or completes the frame).
//   2. start tasks: for each (chain, task) whose slot is free, the oldest
//      waiting frame starts the task's CPU segment.
//   3. CPU segments whose time has elapsed finish; the task may launch.
//   4. one urgency snapshot (Eq. 2) for every active instance.
//   5. launch requests are served from the most to the least urgent; each
//      releases kernels until its batch closes, its task ends, or delayed
//      launching holds it.
#pragma once

#include <array>
#include <climits>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <map>
#include <utility>
#include <vector>

#include "ug.h"

namespace ug {

struct PolicyConfig {
  int policy = UG_POLICY_URGENCY;
  bool bind = true, delay = true, batch = true, calibrate = false, admit = true, exit = false;
  bool no_overlap = false;             // wait for a closed batch to finish
  bool graph = false;                  // tasks launch as one graph each
  int order_key = UG_KEY_URGENCY;      // ranking order (UG_KEY_*)
  int32_t est_noise_permille = 0;      // estimate noise n (per task instance)
  uint64_t noise_seed = 0;
  int64_t admit_tasks = 4;             // tasks in flight before new ones wait
  int64_t delta_eval_ns = 500000;
  int64_t delay_poll_ns = 1000000;
  float util_exempt = 0.1f;
  int64_t th_slack_ns = 0;
  int64_t calib_period_ns = 1000000;   // at most one calibration sample per period
  int64_t max_hold_ns = 0;             // hold-age bound per deadline task; 0 = none
  int32_t cpu_cores = 0;               // cores of the CPU segments; 0 = one each
  bool cpu_prio = false;               // urgency-centric CPU scheduling (Sec. 4.3)
  bool keep_order = false;             // keep each instant's full ranking (order())
  std::vector<int32_t> lanes{2, 6};
};

// Slack of an instance of a best-effort chain (registered with deadline 0):
// no urgency at all, below every deadline instance including late ones.
constexpr int64_t kBestEffortSlack = INT64_MIN;

struct ChainSpec {
  int64_t period_ns = 0, deadline_ns = 0;
  bool best_effort = false;           // deadline 0: never urgent, always delayable
  uint32_t n_buffers = 0;
  std::vector<ug_kernel> kernels;     // all tasks, in order
  std::vector<int64_t> est;           // E_k
  std::vector<float> util;            // U_k
  std::vector<int32_t> task_first, task_end;
  std::vector<int64_t> cpu;           // CPU segment of each task
  std::vector<int64_t> gpu_rem;       // sum_{k >= g} E_k, size N + 1
  std::vector<int64_t> cpu_rem;       // sum_{j' >= j} E^cpu_j', size M + 1
  // per-frame sizes: the frame dimension each kernel takes (0 = none) and
  // its profile points (v, E) sorted by v; a kernel with points has a
  // per-frame estimate
  std::vector<int32_t> fdim;
  std::vector<std::vector<std::pair<int64_t, int64_t>>> prof;
  bool per_frame = false;             // some kernel has a per-frame estimate
  void finalize();
};

// Estimate of a kernel for a frame of size v from its profile points:
// linear between neighbouring points (floor), the end point's value beyond
// either end.
int64_t profile_estimate(const std::vector<std::pair<int64_t, int64_t>>& p, int64_t v);

struct Wait {
  int32_t kind;  // 0 batch start, 1 task end
  int32_t seq;
  bool operator==(const Wait& o) const { return kind == o.kind && seq == o.seq; }
};

enum Phase { kWait = 0, kCpu = 1, kLaunch = 2, kDone = 3 };

struct Instance {
  int32_t c = 0;
  int64_t f = 0;
  int64_t t_arr = 0;
  int phase = kWait;
  int32_t task = -1;
  int64_t task_t0 = 0;                 // when the current task started
  // CPU segment on the shared cores (cpu_cores > 0): work still to run, when
  // it asked for a core, whether it holds one (since cpu_since), and its
  // priority rank (1 = most urgent; urgency-centric scheduling)
  int64_t cpu_left = 0, cpu_req = 0, cpu_since = 0;
  bool cpu_run = false;
  int32_t cpu_prio = 0;
  int64_t cpu_ready = 0;
  int32_t i_gpu = 0, i_cpu = 0;        // executing-kernel / CPU-segment index
  int32_t g_next = 0, released_hi = 0;
  int32_t batch = 0;
  bool batch_open = false;
  int64_t batch_sum = 0;
  std::vector<int32_t> batch_first;
  std::deque<Wait> waits;
  bool bound = false;
  int32_t level = -1, lane = -1;
  bool has_wake = false;
  int64_t wake = 0;
  // hold-age bound: time of the task's first hold, and while the task is
  // held the time at which that age reaches the bound
  bool has_held = false;
  int64_t held_since = 0;
  bool has_expire = false;
  int64_t expire = 0;
  int32_t n_holds = 0, n_batches = 0;
  // per-frame estimates (chains with per-frame sizes): E of every kernel
  // for this frame and their suffix sums; empty otherwise
  std::vector<int64_t> est, gpu_rem;
  bool in_flight() const { return released_hi > i_gpu; }
};

struct Arrival {
  int32_t c;
  int64_t f;
  int64_t t_arr;
  std::vector<int64_t> dims;  // the frame's sizes (chains with per-frame sizes)
};
struct EvDone {
  int32_t c;
  int64_t f;
  int32_t task, kind, seq;
};
struct Finished {
  int32_t c;
  int64_t f, t_arr, t_done;
  int32_t n_holds, n_batches;
  bool exited = false;        // left the chain early (negative urgency at a task start)
};

using Key = std::pair<int32_t, int64_t>;  // (chain, frame)

class Policy {
 public:
  explicit Policy(const PolicyConfig& cfg) : cfg_(cfg) {}

  uint32_t add_chain(ChainSpec&& spec);
  void finalize();                       // recompute remaining-work sums
  void reset();                          // drop every instance and sample
  const PolicyConfig& config() const { return cfg_; }
  PolicyConfig& mutable_config() { return cfg_; }
  std::vector<ChainSpec>& chains() { return chains_; }
  const std::vector<ChainSpec>& chains() const { return chains_; }

  // Process one instant; decisions are appended to `out`.  Returns false
  // (and leaves `err`) if an input does not match the state.
  bool instant(int64_t t, std::vector<Arrival>& arrivals,
               std::vector<EvDone>& evdones, std::vector<ug_record>& out,
               const char** err);

  // Earliest pending timer (CPU segment end, sleep-loop wake); false if none.
  bool next_timer(int64_t* t) const;

  const std::map<Key, Instance>& instances() const { return inst_; }
  std::vector<Finished>& finished() { return finished_; }
  std::vector<int64_t>& samples() { return samples_; }
  uint64_t collisions() const { return collisions_; }
  // collisions by the number of other chains' instances in flight (1, 2,
  // ..., kCollisionBins or more)
  static constexpr size_t kCollisionBins = 8;
  const std::array<uint64_t, kCollisionBins>& collision_hist() const { return collision_hist_; }
  int32_t fifo_lane(int32_t c, int32_t task) const { return fifo_base_[c] + task; }
  int32_t fifo_lanes() const { return fifo_total_; }
  // Every active instance of the last instant, most urgent first under the
  // configured order (FIFO policy: (chain, frame) order); kept only with
  // keep_order.
  const std::vector<Key>& order() const { return order_; }

 private:
  bool urgent(int64_t slack) const;
  // remaining GPU + CPU work of Eq. (2) as the gate estimates it (with
  // estimate noise, each task's part scaled by its instance's factor)
  int64_t remaining(const Instance& in) const;
  // true iff `a` ranks before `b` under the configured order at the
  // current instant (strict total order)
  bool before(const Instance& a, const Instance& b, const std::map<Key, int64_t>& slack) const;
  // deadline of the instance's current task under SAEDF / EQDF, as the
  // rational base + num / den (den > 0)
  void cpu_cores(int64_t t, const std::vector<Instance*>& active, bool started,
                 std::vector<ug_record>& out);
  void subtask_deadline(const Instance& in, __int128* base, __int128* num, __int128* den) const;
  bool blocked(const Instance& me, const std::vector<Instance*>& active,
               const std::map<Key, int64_t>& slack) const;
  void bind(Instance& me, const std::vector<Instance*>& active,
            const std::map<Key, int64_t>& slack, std::vector<ug_record>& out);
  void release(Instance& me, int64_t t, const std::vector<Instance*>& active,
               const std::map<Key, int64_t>& slack, std::vector<ug_record>& out);
  void start_task(Instance& in, int32_t j, int64_t t, std::vector<ug_record>& out);

  PolicyConfig cfg_;
  std::vector<ChainSpec> chains_;
  std::vector<int32_t> fifo_base_;
  int32_t fifo_total_ = 0;
  std::map<Key, Instance> inst_;
  std::map<std::pair<int32_t, int32_t>, int64_t> slot_;      // -1 = free
  std::map<std::pair<int32_t, int32_t>, std::deque<int64_t>> queue_;
  std::map<std::pair<int32_t, int32_t>, int32_t> lane_load_;
  std::vector<Finished> finished_;
  std::vector<int64_t> samples_;
  std::vector<Key> order_;
  int64_t active_ = 0;         // instances with launched, unconfirmed kernels
  bool sampled_ = false;       // a sample has been taken
  int64_t next_sample_ = 0;    // earliest time of the next sample
  uint64_t collisions_ = 0;
  std::array<uint64_t, kCollisionBins> collision_hist_{};
  int64_t now_ = 0;            // time of the instant being decided
};

// SplitMix64 output for the state x (Steele, Lea and Flood, 2014).
uint64_t splitmix64(uint64_t x);
// Estimate noise of task j of frame f of chain c: k uniform in [-n, n] from
// three chained SplitMix64 outputs of (seed, c, f, j); estimates become
// E * (1000 + k) / 1000.
int32_t noise_permille(uint64_t seed, int32_t c, int64_t f, int32_t j, int32_t n);

// Exact comparison of urgency levels UL = 1/slack (Eq. 2): true iff
// 1/s1 > 1/s2, with 1/0 = +infinity and kBestEffortSlack below everything.
bool ul_greater(int64_t s1, int64_t s2);
// Strict total order: higher UL first, then lower (chain, frame).
bool more_urgent(int64_t s1, const Key& k1, int64_t s2, const Key& k2);

}  // namespace ug
