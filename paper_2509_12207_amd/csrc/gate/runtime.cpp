// libug runtime: context, gate thread, streams, events and the C-ABI.
//
// One gate thread per context owns the policy (policy.hpp), every stream and
// every event.  Each loop iteration it
//   1. polls, for every active chain instance, the events at the head of its
//      wait list (hipEventQuery; completed prefix only),
//   2. reads the clock (t), takes the frames whose arrival time has come,
//   3. if anything was observed or a timer expired, runs one decision instant
//      at t and executes the decisions: event records and kernel launches on
//      the bound stream, completions to the caller's queue,
//   4. logs the instant (inputs and decisions) for offline replay.
// Callers talk to the gate only through two mutex-protected queues
// (submissions in, completions out).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <ctime>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "../kernels/ops.hpp"
#include "policy.hpp"
#include "tails.hpp"
#include "ug.h"

namespace {

int64_t mono_ns() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return static_cast<int64_t>(ts.tv_sec) * 1000000000LL + ts.tv_nsec;
}

struct Frame {
  uint32_t chain = 0;
  int64_t f = 0;
  int64_t t_arr = 0;
  std::vector<void*> buffers;
  std::vector<int64_t> dims;  // per-frame sizes (kernels with frame_dim > 0)
};

// Per-frame sizes a chain accepts: dims[d] in [lo[d], hi[d]].
struct DimRange {
  std::vector<int64_t> lo, hi;
};

using EvKey = std::tuple<int32_t, int64_t, int32_t, int32_t, int32_t>;  // c, f, task, kind, seq
// a captured task: chain, task, the frame's buffer pointers and sizes, and
// whether its tails are fused (left out of the graph, producers counted)
using GraphKey = std::tuple<int32_t, int32_t, std::vector<void*>, std::vector<int64_t>, bool>;
using TaskKey = std::tuple<int32_t, int64_t, int32_t>;  // c, f, task

// A captured task graph.  A fused graph's producers count on counters of
// its own (one per producer, by kernel index in the task; null elsewhere),
// so it is launched fused only while no item of an earlier launch still
// uses them (`busy` counts those items until they are seen finished).
struct GraphRec {
  hipGraphExec_t ge = nullptr;
  std::vector<unsigned*> sig;
  uint32_t busy = 0;
};

// A tail published to the executor for an instance's task, and the graph
// whose counter it waits on (null: a slot's own counter).
struct TailRec {
  uint32_t slot;
  uint64_t pub;
  GraphRec* graph;
};

struct Ctx {
  ug_config cfg{};
  ug::Policy policy{ug::PolicyConfig{}};
  bool has_device = false;
  bool started = false;
  bool finalized = false;

  std::vector<std::vector<hipStream_t>> level_streams;  // [level][lane]
  int queue_classes = 0;                                // hardware queues the lanes use
  std::vector<hipStream_t> fifo_streams;                // one per task of every chain
  // streams attached by the caller (ug_attach_streams) are borrowed; only
  // streams the library created itself (own_streams) are destroyed
  bool streams_attached = false;
  std::vector<hipStream_t> owned_streams;
  std::vector<hipEvent_t> event_pool;
  std::vector<hipEvent_t> all_events;
  std::map<EvKey, hipEvent_t> live_events;
  std::map<ug::Key, hipStream_t> bound;
  // device workspace of each registered kernel ([chain][kernel], null when
  // the kernel needs none): a kernel runs for one frame at a time, so one
  // workspace per kernel suffices
  std::vector<std::vector<void*>> ws;
  std::vector<std::vector<size_t>> ws_bytes;
  std::map<ug::Key, Frame> frames;                      // arrived, not completed
  // task graphs (UG_F_GRAPH): captured on their own stream, launched on the
  // task's bound stream; kept until the context is destroyed
  std::map<GraphKey, GraphRec> graphs;
  hipStream_t capture_stream = nullptr;
  std::vector<Frame> pending;                           // submitted, not arrived

  // fused tails (UG_F_FUSE): the tails of every chain ([chain][kernel]: the
  // end of the tail the kernel starts, -1, or -2 inside a tail), the
  // executor's queue and stream, the completion counters (one per queue
  // slot for producers launched one by one: a slot's item is the only user
  // of its counter; fused graphs take theirs from `counter_chunks`), the
  // items published per task instance (in order) with the prefix seen
  // finished, slots reserved by a producer's launch for its tail, the
  // kernel up to which an instance's launches are covered by a fused tail,
  // and the items each recorded event waits for.  Counters live as long as
  // the context (captured graphs hold their addresses) and are zeroed at
  // every start.
  std::vector<std::vector<int32_t>> tail_mark;
  std::unique_ptr<ug::TailQueue> tails;
  hipStream_t fuse_stream = nullptr;
  unsigned* slot_counters = nullptr;
  std::vector<unsigned*> counter_chunks;
  size_t chunk_used = 0;
  std::map<TaskKey, std::vector<TailRec>> inst_tails;
  std::map<TaskKey, size_t> inst_tails_done;
  std::map<std::pair<ug::Key, int32_t>, uint32_t> reserved;
  std::map<ug::Key, int32_t> covered_to;
  std::map<EvKey, size_t> ev_tails;
  std::vector<ug::Key> last_order;   // the ranking the queue's keys follow
  std::atomic<uint64_t> st_tails{0}, st_tails_unfused{0};
  uint64_t executor_launches = 0;    // of the last run (counted at ug_stop)
  uint64_t fuse_stats[ug::kStatCount] = {};   // the executor's, of the last run

  std::mutex mu;  // inbox, outbox, counters, next_frame
  std::condition_variable cv_done;
  std::deque<Frame> inbox;
  std::deque<ug_completion> outbox;
  std::vector<int64_t> next_frame;
  uint64_t outstanding = 0;
  // serving admission (under mu): footprint of one frame per chain, bytes
  // held by the frames in flight and their peak
  std::vector<uint64_t> footprint;
  std::vector<DimRange> dim_range;
  uint64_t inflight_bytes = 0, hbm_peak = 0, st_deferred = 0;

  // completed-frame latencies and per-chain counts since start (under mu)
  std::vector<int64_t> latencies;
  std::vector<uint64_t> chain_done, chain_missed;

  std::mutex trace_mu;
  std::vector<ug_record> trace;
  uint64_t trace_dropped = 0;

  std::thread thr;
  std::atomic<bool> stop{false};
  std::atomic<int> device_error{0};
  // messages written by caller threads and the gate thread alike
  std::mutex err_mu;
  std::string last_error;
  std::string device_msg;

  // statistics (written by the gate thread; read racily by ug_get_stats
  // through atomics)
  std::atomic<uint64_t> st_submitted{0}, st_completed{0}, st_missed{0}, st_launches{0},
      st_holds{0}, st_batches{0}, st_instants{0};
  std::atomic<int64_t> st_decide_ns{0}, st_launch_ns{0};
};

void set_error(Ctx* c, const std::string& msg, bool device) {
  std::lock_guard<std::mutex> lk(c->err_mu);
  c->last_error = msg;
  if (device) c->device_msg = msg;
}

ug_status fail(Ctx* c, ug_status s, const std::string& msg) {
  if (c) set_error(c, msg, false);
  return s;
}

// Message of the last failure of a call that has no context yet (ug_create).
std::mutex g_create_mu;
std::string g_create_error;

ug_status hip_fail(Ctx* c, hipError_t e, const char* what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  if (!c) {
    std::lock_guard<std::mutex> lk(g_create_mu);
    g_create_error = m;
  }
  if (c) {
    set_error(c, m, true);
    c->device_error.store(1);
  }
  return UG_EDEVICE;
}

bool sticky(Ctx* c) { return c->device_error.load() != 0; }

ug::PolicyConfig policy_config(const ug_config& cfg) {
  ug::PolicyConfig p;
  p.policy = cfg.policy;
  p.bind = (cfg.flags & UG_F_BIND) != 0;
  p.delay = (cfg.flags & UG_F_DELAY) != 0;
  p.batch = (cfg.flags & UG_F_BATCH) != 0;
  p.calibrate = (cfg.flags & UG_F_CALIBRATE) != 0;
  p.delta_eval_ns = cfg.delta_eval_ns;
  p.delay_poll_ns = cfg.delay_poll_ns;
  p.util_exempt = cfg.util_exempt;
  p.th_slack_ns = cfg.th_slack_ns;
  p.calib_period_ns = cfg.calib_period_ns;
  p.admit = (cfg.flags & UG_F_ADMIT) != 0;
  p.exit = (cfg.flags & UG_F_EXIT) != 0;
  p.no_overlap = (cfg.flags & UG_F_NO_OVERLAP) != 0;
  p.graph = (cfg.flags & UG_F_GRAPH) != 0;
  p.order_key = cfg.order_key;
  p.est_noise_permille = cfg.est_noise_permille;
  p.noise_seed = cfg.noise_seed;
  p.admit_tasks = cfg.admit_tasks;
  p.max_hold_ns = cfg.max_hold_ns;
  p.cpu_cores = cfg.cpu_cores;
  p.cpu_prio = (cfg.flags & UG_F_CPU_PRIO) != 0;
  p.keep_order = (cfg.flags & UG_F_FUSE) != 0;
  p.lanes.assign(cfg.lanes, cfg.lanes + cfg.n_levels);
  return p;
}

void push_trace(Ctx* c, const ug_record& r) {
  if (c->cfg.trace_capacity == 0) return;
  if (c->trace.size() >= c->cfg.trace_capacity) {
    ++c->trace_dropped;
    return;
  }
  c->trace.push_back(r);
}

ug_record make_rec(int32_t type, int32_t chain, int64_t frame, int32_t task, int32_t kernel,
                   int32_t a, int32_t b, int64_t t) {
  ug_record r;
  r.type = type;
  r.chain = chain;
  r.frame = frame;
  r.task = task;
  r.kernel = kernel;
  r.a = a;
  r.b = b;
  r.t = t;
  return r;
}

hipEvent_t take_event(Ctx* c) {
  if (c->event_pool.empty()) {
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    c->all_events.push_back(e);
    return e;
  }
  hipEvent_t e = c->event_pool.back();
  c->event_pool.pop_back();
  return e;
}

// True if the tail that kernel g of a chain starts is fused for this
// frame: it qualifies (tail_mark) and the frame's buffers are aligned.
bool tail_ok(const Ctx* c, int32_t chain, int32_t g, const Frame& fr, ug::FuseItem* it) {
  const int32_t end = c->tail_mark[chain][g];
  if (end <= g) return false;
  ug::FuseItem tmp;
  return ug::tail_item(c->policy.chains()[chain].kernels, g, end, fr.buffers.data(), it ? it : &tmp);
}

constexpr size_t kCounterChunk = 4096;   // graph counters per allocation

// The slots' completion counters, allocated once per context.
hipError_t alloc_counters(Ctx* c) {
  if (c->slot_counters) return hipSuccess;
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, ug::kFuseSlots * sizeof(unsigned));
  if (e == hipSuccess) e = hipMemset(p, 0, ug::kFuseSlots * sizeof(unsigned));
  if (e != hipSuccess) {
    if (p) (void)hipFree(p);
    return e;
  }
  c->slot_counters = static_cast<unsigned*>(p);
  return hipSuccess;
}

// A zeroed counter of a fused graph's own (null on failure, *err set).
unsigned* graph_counter(Ctx* c, hipError_t* err) {
  if (c->counter_chunks.empty() || c->chunk_used == kCounterChunk) {
    void* p = nullptr;
    *err = hipMalloc(&p, kCounterChunk * sizeof(unsigned));
    if (*err == hipSuccess) *err = hipMemset(p, 0, kCounterChunk * sizeof(unsigned));
    if (*err != hipSuccess) {
      if (p) (void)hipFree(p);
      return nullptr;
    }
    c->counter_chunks.push_back(static_cast<unsigned*>(p));
    c->chunk_used = 0;
  }
  return c->counter_chunks.back() + c->chunk_used++;
}

// Zeroes every counter (at start: an earlier run may have left counts).
hipError_t zero_counters(Ctx* c) {
  hipError_t e = alloc_counters(c);
  if (e == hipSuccess) e = hipMemset(c->slot_counters, 0, ug::kFuseSlots * sizeof(unsigned));
  for (unsigned* p : c->counter_chunks)
    if (e == hipSuccess) e = hipMemset(p, 0, kCounterChunk * sizeof(unsigned));
  for (auto& kv : c->graphs) kv.second.busy = 0;
  return e;
}

// Graph of task j of a chain for a frame's buffers and sizes: captured on
// first use (every kernel of the task in order on the capture stream, in
// relaxed mode so other threads' HIP calls are unaffected), instantiated and
// cached.  With `fused`, the task's fused tails are left out and their
// producers count their wavefronts.  On failure returns null with *err set.
GraphRec* task_graph(Ctx* c, int32_t chain, int32_t j, const Frame& fr, bool fused,
                     hipError_t* err) {
  GraphKey gk{chain, j, fr.buffers, fr.dims, fused};
  auto it = c->graphs.find(gk);
  if (it != c->graphs.end()) return &it->second;
  if (!c->capture_stream) {
    *err = hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking);
    if (*err != hipSuccess) return nullptr;
  }
  const ug::ChainSpec& ch = c->policy.chains()[chain];
  GraphRec rec;
  rec.sig.assign(static_cast<size_t>(ch.task_end[j] - ch.task_first[j]), nullptr);
  if (fused) {
    // the graph's own counters, made before the capture
    for (int32_t g = ch.task_first[j]; g + 1 < ch.task_end[j]; ++g)
      if (tail_ok(c, chain, g + 1, fr, nullptr) &&
          !(rec.sig[g - ch.task_first[j]] = graph_counter(c, err)))
        return nullptr;
  }
  *err = hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeRelaxed);
  if (*err != hipSuccess) return nullptr;
  hipError_t launch_err = hipSuccess;
  for (int32_t g = ch.task_first[j]; g < ch.task_end[j] && launch_err == hipSuccess; ++g) {
    if (fused && tail_ok(c, chain, g, fr, nullptr)) {
      g = c->tail_mark[chain][g] - 1;   // the tail runs on the executor
      continue;
    }
    ug_kernel k = ch.kernels[g];
    if (k.frame_dim > 0) k = ug::frame_kernel(k, fr.dims[k.frame_dim - 1]);
    launch_err = ug::launch_kernel(k, fr.buffers.data(), c->capture_stream, c->ws[chain][g],
                                   c->ws_bytes[chain][g], rec.sig[g - ch.task_first[j]]);
  }
  hipGraph_t graph = nullptr;
  *err = hipStreamEndCapture(c->capture_stream, &graph);
  if (launch_err != hipSuccess) *err = launch_err;
  if (*err != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return nullptr;
  }
  *err = hipGraphInstantiate(&rec.ge, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (*err != hipSuccess) return nullptr;
  return &c->graphs.emplace(std::move(gk), std::move(rec)).first->second;
}

// Key of an item of instance `key`: the instance's rank in the gate's last
// urgency order (1 = most urgent), then the publication number; FIFO
// launch serves items in publication order.
uint64_t tail_key(const Ctx* c, const ug::Key& key, uint64_t pub) {
  if (c->cfg.policy == UG_POLICY_FIFO) return pub;
  uint64_t rank = 0xffffffffull;
  const auto& order = c->policy.order();
  for (size_t r = 0; r < order.size(); ++r)
    if (order[r] == key) {
      rank = r + 1;
      break;
    }
  return (rank << 32) | (pub & 0xffffffffull);
}

// Publishes the tail [g, end) of an instance's task into a reserved slot;
// its producer counts on `sig` (a counter of `graph`'s, or the slot's own
// when `graph` is null).
void publish_tail(Ctx* c, const ug::Key& key, int32_t task, int32_t g, uint32_t slot,
                  const Frame& fr, unsigned* sig, GraphRec* graph) {
  const ug::ChainSpec& ch = c->policy.chains()[key.first];
  ug::FuseItem it;
  (void)tail_item(ch.kernels, g, c->tail_mark[key.first][g], fr.buffers.data(), &it);
  it.sig = reinterpret_cast<uint64_t>(sig);
  it.sig_expected = ug::signal_waves(ch.kernels[g - 1]);
  const uint64_t pub = c->tails->publish(slot, it, tail_key(c, key, c->tails->next_pub()));
  if (graph) graph->busy++;
  c->inst_tails[TaskKey{key.first, key.second, task}].push_back({slot, pub, graph});
  c->covered_to[key] = c->tail_mark[key.first][g];
  c->st_tails++;
}

// Orders `pool` so that consecutive entries sit on different hardware queues
// wherever the queues allow: streams are grouped by the queue the probe finds
// them on, then taken round-robin over the groups.  Returns the number of
// queues seen in *n_queues.
hipError_t place_over_queues(std::vector<hipStream_t>* pool, int* n_queues) {
  std::vector<int> cls;
  hipError_t e = ug::stream_queue_classes(*pool, &cls);
  if (e != hipSuccess) return e;
  std::vector<std::vector<hipStream_t>> by_queue;
  for (size_t i = 0; i < pool->size(); ++i) {
    if (static_cast<size_t>(cls[i]) >= by_queue.size()) by_queue.resize(cls[i] + 1);
    by_queue[cls[i]].push_back((*pool)[i]);
  }
  std::vector<hipStream_t> order;
  for (size_t round = 0; order.size() < pool->size(); ++round)
    for (auto& q : by_queue)
      if (round < q.size()) order.push_back(q[round]);
  *pool = std::move(order);
  *n_queues = static_cast<int>(by_queue.size());
  return hipSuccess;
}

uint32_t streams_used(const Ctx* c);

// Gives the policy its streams: the lanes of every level in order (urgency
// policy) or one stream per task of every chain (FIFO), from `pool`, placed
// over the hardware queues first when UG_F_PLACE is set.
hipError_t assign_streams(Ctx* c, std::vector<hipStream_t> pool) {
  if (c->cfg.flags & UG_F_FUSE) {
    // the executor's own stream, and the pool without the streams on its
    // hardware queue (while any other remains); short of streams, lanes
    // share the remaining ones in turn
    hipError_t e = hipSuccess;
    if (!c->fuse_stream &&
        (e = hipStreamCreateWithFlags(&c->fuse_stream, hipStreamNonBlocking)) != hipSuccess)
      return e;
    std::vector<hipStream_t> probe{c->fuse_stream};
    probe.insert(probe.end(), pool.begin(), pool.end());
    std::vector<int> cls;
    if ((e = ug::stream_queue_classes(probe, &cls)) != hipSuccess) return e;
    std::vector<hipStream_t> keep;
    for (size_t i = 1; i < probe.size(); ++i)
      if (cls[i] != cls[0]) keep.push_back(probe[i]);
    if (!keep.empty()) pool = std::move(keep);
    const size_t n = streams_used(c), have = pool.size();
    for (size_t i = have; i < n; ++i) pool.push_back(pool[i % have]);
    pool.resize(n);
  }
  if (c->cfg.flags & UG_F_PLACE) {
    hipError_t e = place_over_queues(&pool, &c->queue_classes);
    if (e != hipSuccess) return e;
  }
  if (c->cfg.policy == UG_POLICY_FIFO) {
    c->fifo_streams = std::move(pool);
    return hipSuccess;
  }
  c->level_streams.assign(c->cfg.n_levels, {});
  size_t next = 0;
  for (int lv = 0; lv < c->cfg.n_levels; ++lv)
    for (int ln = 0; ln < c->cfg.lanes[lv]; ++ln) c->level_streams[lv].push_back(pool[next++]);
  return hipSuccess;
}

// Streams the policy uses: the lanes of every level, or one per task.
uint32_t streams_used(const Ctx* c) {
  if (c->cfg.policy == UG_POLICY_FIFO) return static_cast<uint32_t>(c->policy.fifo_lanes());
  uint32_t n = 0;
  for (int lv = 0; lv < c->cfg.n_levels; ++lv) n += static_cast<uint32_t>(c->cfg.lanes[lv]);
  return n;
}

// Streams to attach: with fused tails half as many again, so that the
// streams sharing the executor's hardware queue can be set aside.
uint32_t streams_needed(const Ctx* c) {
  const uint32_t n = streams_used(c);
  return (c->cfg.flags & UG_F_FUSE) ? n + (n + 1) / 2 : n;
}

// Library-owned streams (own_streams): created at the default priority.
hipError_t create_own_streams(Ctx* c) {
  std::vector<hipStream_t> pool;
  const uint32_t n = streams_needed(c);
  for (uint32_t i = 0; i < n; ++i) {
    hipStream_t st = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    c->owned_streams.push_back(st);
    pool.push_back(st);
  }
  return assign_streams(c, std::move(pool));
}

// Executes the decisions of one instant.  Returns false on a device error.
bool execute(Ctx* c, const std::vector<ug_record>& dec) {
  for (const ug_record& d : dec) {
    const ug::Key key{d.chain, d.frame};
    switch (d.type) {
      case UG_REC_BIND: {
        hipStream_t s = c->cfg.policy == UG_POLICY_FIFO ? c->fifo_streams[d.b]
                                                        : c->level_streams[d.a][d.b];
        c->bound[key] = s;
        break;
      }
      case UG_REC_EVREC: {
        hipEvent_t e = take_event(c);
        if (!e) {
          hip_fail(c, hipErrorOutOfMemory, "hipEventCreateWithFlags");
          return false;
        }
        const int64_t t0 = mono_ns();
        hipError_t err = hipEventRecord(e, c->bound.at(key));
        c->st_launch_ns += mono_ns() - t0;
        if (err != hipSuccess) {
          hip_fail(c, err, "hipEventRecord");
          return false;
        }
        c->live_events[EvKey{d.chain, d.frame, d.task, d.a, d.b}] = e;
        if (c->tails && d.a == 1) {
          // a task-end event stands for every tail of the task as well; a
          // batch-start event does not wait for the earlier batches' tails
          // (no later kernel reads what a tail writes)
          auto t = c->inst_tails.find(TaskKey{d.chain, d.frame, d.task});
          c->ev_tails[EvKey{d.chain, d.frame, d.task, d.a, d.b}] =
              t == c->inst_tails.end() ? 0 : t->second.size();
        }
        if (d.a == 0) c->st_batches++;
        break;
      }
      case UG_REC_LAUNCH: {
        const ug::ChainSpec& ch = c->policy.chains()[d.chain];
        const Frame& fr = c->frames.at(key);
        const int64_t t0 = mono_ns();
        const ug_kernel& kd = ch.kernels[d.kernel];
        hipError_t err;
        const std::vector<int32_t>* mark = c->tails ? &c->tail_mark[d.chain] : nullptr;
        if (c->cfg.flags & UG_F_GRAPH) {
          // the task's first kernel launches the task's graph; its other
          // kernels are inside it.  With fused tails, every tail of the task
          // that qualifies takes a slot and is published once the graph is
          // launched; the unfused graph runs instead when slots are short or
          // the fused graph's counters still serve an earlier launch's items.
          err = hipSuccess;
          if (d.kernel == ch.task_first[d.task]) {
            std::vector<std::pair<int32_t, uint32_t>> pubs;
            GraphRec* rec = nullptr;
            if (mark) {
              bool fused = true;
              for (int32_t g = ch.task_first[d.task]; g < ch.task_end[d.task]; ++g) {
                if (!tail_ok(c, d.chain, g, fr, nullptr)) continue;
                uint32_t slot = 0;
                if (!c->tails->reserve(&slot)) {
                  fused = false;
                  break;
                }
                pubs.push_back({g, slot});
              }
              if (fused && !pubs.empty()) {
                rec = task_graph(c, d.chain, d.task, fr, true, &err);
                if (rec && rec->busy) {
                  rec = nullptr;
                  fused = false;
                }
              }
              if (!fused || !rec) {
                for (auto& p : pubs) c->tails->unreserve(p.second);
                if (err == hipSuccess) c->st_tails_unfused += pubs.size();
                pubs.clear();
              }
            }
            if (!rec && err == hipSuccess) rec = task_graph(c, d.chain, d.task, fr, false, &err);
            if (rec) err = hipGraphLaunch(rec->ge, c->bound.at(key));
            if (err == hipSuccess)
              for (auto& p : pubs)
                publish_tail(c, key, d.task, p.first, p.second, fr,
                             rec->sig[p.first - 1 - ch.task_first[d.task]], rec);
          }
        } else if (mark && (*mark)[d.kernel] == -2 && d.kernel < c->covered_to[key]) {
          // inside a fused tail: the executor runs it
          err = hipSuccess;
        } else if (mark && (*mark)[d.kernel] > d.kernel) {
          // the first kernel of a tail: published if its producer reserved
          // a slot, else launched as usual
          auto r = c->reserved.find({key, d.kernel});
          if (r != c->reserved.end()) {
            publish_tail(c, key, d.task, d.kernel, r->second, fr, c->slot_counters + r->second,
                         nullptr);
            c->reserved.erase(r);
            err = hipSuccess;
          } else {
            err = ug::launch_kernel(kd, fr.buffers.data(), c->bound.at(key));
          }
        } else if (mark && d.kernel + 1 < ch.task_end[d.task] &&
                   tail_ok(c, d.chain, d.kernel + 1, fr, nullptr)) {
          // the producer of a tail: counts its wavefronts on the slot's
          // counter when a slot is free for the tail
          uint32_t slot = 0;
          unsigned* sig = nullptr;
          if (c->tails->reserve(&slot)) {
            c->reserved[{key, d.kernel + 1}] = slot;
            sig = c->slot_counters + slot;
          } else {
            c->st_tails_unfused++;
          }
          err = ug::launch_kernel(kd, fr.buffers.data(), c->bound.at(key),
                                  c->ws[d.chain][d.kernel], c->ws_bytes[d.chain][d.kernel], sig);
        } else if (kd.frame_dim > 0) {
          // this frame's size (checked at submission)
          const ug_kernel kf = ug::frame_kernel(kd, fr.dims[kd.frame_dim - 1]);
          err = ug::launch_kernel(kf, fr.buffers.data(), c->bound.at(key),
                                  c->ws[d.chain][d.kernel], c->ws_bytes[d.chain][d.kernel]);
        } else {
          err = ug::launch_kernel(kd, fr.buffers.data(), c->bound.at(key),
                                  c->ws[d.chain][d.kernel], c->ws_bytes[d.chain][d.kernel]);
        }
        c->st_launch_ns += mono_ns() - t0;
        if (err != hipSuccess) {
          hip_fail(c, err, "kernel launch");
          return false;
        }
        c->st_launches++;
        break;
      }
      case UG_REC_HOLD:
        c->st_holds++;
        break;
      default:
        break;
    }
  }
  return true;
}

void deliver_completions(Ctx* c) {
  auto& fin = c->policy.finished();
  if (fin.empty()) return;
  std::lock_guard<std::mutex> lk(c->mu);
  for (const ug::Finished& f : fin) {
    const ug::ChainSpec& ch = c->policy.chains()[f.c];
    ug_completion out{};
    out.chain = static_cast<uint32_t>(f.c);
    out.frame = static_cast<uint64_t>(f.f);
    out.t_arr_ns = f.t_arr;
    out.t_done_ns = f.t_done;
    out.latency_ns = f.t_done - f.t_arr;
    // best-effort chains have no deadline: never missed, and outside the
    // miss ratio and the latency percentiles
    // an exited frame counts as missed and stays out of the latencies
    out.missed = (!ch.best_effort && (f.exited || out.latency_ns > ch.deadline_ns)) ? 1 : 0;
    out.n_holds = f.n_holds;
    out.n_batches = f.n_batches;
    out.exited = f.exited ? 1 : 0;
    c->outbox.push_back(out);
    if (!ch.best_effort) {
      if (!f.exited) c->latencies.push_back(out.latency_ns);
      c->chain_done[f.c] += 1;
      c->chain_missed[f.c] += out.missed;
    }
    c->frames.erase({f.c, f.f});
    c->bound.erase({f.c, f.f});
    c->covered_to.erase({f.c, f.f});
    c->st_completed++;
    if (out.missed) c->st_missed++;
    if (c->outstanding > 0) --c->outstanding;
    c->inflight_bytes -= std::min(c->inflight_bytes, c->footprint[f.c]);
  }
  fin.clear();
  c->cv_done.notify_all();
}

void gate_main(Ctx* c) {
  (void)hipSetDevice(c->cfg.device);
  std::vector<ug::Arrival> arr;
  std::vector<ug::EvDone> evs;
  std::vector<ug_record> dec;
  std::vector<Frame> incoming;
  while (!c->stop.load(std::memory_order_relaxed)) {
    {
      std::lock_guard<std::mutex> lk(c->mu);
      while (!c->inbox.empty()) {
        incoming.push_back(std::move(c->inbox.front()));
        c->inbox.pop_front();
      }
    }
    for (Frame& f : incoming) c->pending.push_back(std::move(f));
    incoming.clear();

    // the tail executor runs while items are unfinished (it leaves when
    // idle; launched again here)
    if (c->tails && c->tails->outstanding()) {
      const hipError_t e = c->tails->kick();
      if (e != hipSuccess) {
        hip_fail(c, e, "tail executor launch");
        break;
      }
    }

    // 1. observe events: completed prefix of each instance's wait list
    evs.clear();
    bool dev_err = false;
    for (const auto& kv : c->policy.instances()) {
      const ug::Instance& in = kv.second;
      for (const ug::Wait& w : in.waits) {
        auto it = c->live_events.find(EvKey{in.c, in.f, in.task, w.kind, w.seq});
        if (it == c->live_events.end()) break;
        hipError_t q = hipEventQuery(it->second);
        if (q == hipErrorNotReady) break;
        if (q != hipSuccess) {
          hip_fail(c, q, "hipEventQuery");
          dev_err = true;
          break;
        }
        if (c->tails) {
          // and the tails published before the event have finished
          auto need = c->ev_tails.find(it->first);
          if (need != c->ev_tails.end() && need->second > 0) {
            const TaskKey tk{in.c, in.f, in.task};
            const std::vector<TailRec>& recs = c->inst_tails[tk];
            size_t& seen = c->inst_tails_done[tk];
            while (seen < need->second && c->tails->finished(recs[seen].slot, recs[seen].pub)) {
              if (recs[seen].graph) recs[seen].graph->busy--;
              ++seen;
            }
            if (seen < need->second) break;
          }
        }
        evs.push_back({in.c, in.f, in.task, w.kind, w.seq});
      }
      if (dev_err) break;
    }
    if (dev_err) break;

    // 2. clock, arrivals, timers
    const int64_t now = mono_ns();
    arr.clear();
    for (size_t i = 0; i < c->pending.size();) {
      if (c->pending[i].t_arr <= now) {
        Frame& f = c->pending[i];
        arr.push_back({static_cast<int32_t>(f.chain), f.f, f.t_arr, f.dims});
        c->frames[{static_cast<int32_t>(f.chain), f.f}] = std::move(f);
        if (i + 1 != c->pending.size()) c->pending[i] = std::move(c->pending.back());
        c->pending.pop_back();
      } else {
        ++i;
      }
    }
    int64_t tt = 0;
    const bool timer = c->policy.next_timer(&tt) && tt <= now;
    if (arr.empty() && evs.empty() && !timer) {
      if (c->cfg.idle_sleep_ns > 0)
        std::this_thread::sleep_for(std::chrono::nanoseconds(c->cfg.idle_sleep_ns));
      else
        std::this_thread::yield();
      continue;
    }

    // 3. decide
    dec.clear();
    const char* err = nullptr;
    const int64_t t0 = mono_ns();
    const bool ok = c->policy.instant(now, arr, evs, dec, &err);
    c->st_decide_ns += mono_ns() - t0;
    c->st_instants++;
    if (!ok) {
      set_error(c, err ? err : "policy error", true);
      c->device_error.store(1);
      break;
    }
    {
      std::lock_guard<std::mutex> lk(c->trace_mu);
      push_trace(c, make_rec(UG_REC_INSTANT, 0, 0, 0, 0, (int32_t)arr.size(), (int32_t)evs.size(), now));
      for (const auto& a : arr) {
        push_trace(c, make_rec(UG_REC_ARRIVE, a.c, a.f, 0, 0, 0, 0, a.t_arr));
        for (size_t d = 0; d < a.dims.size(); ++d)
          push_trace(c, make_rec(UG_REC_DIMS, a.c, a.f, 0, 0, static_cast<int32_t>(d), 0, a.dims[d]));
      }
      for (const auto& e : evs)
        push_trace(c, make_rec(UG_REC_EVDONE, e.c, e.f, e.task, 0, e.kind, e.seq, 0));
      for (const auto& d : dec) push_trace(c, d);
    }
    for (const auto& e : evs) {
      auto it = c->live_events.find(EvKey{e.c, e.f, e.task, e.kind, e.seq});
      c->event_pool.push_back(it->second);
      c->live_events.erase(it);
      if (c->tails) {
        c->ev_tails.erase(EvKey{e.c, e.f, e.task, e.kind, e.seq});
        if (e.kind == 1) {   // task end: every item of the task has finished
          c->inst_tails.erase(TaskKey{e.c, e.f, e.task});
          c->inst_tails_done.erase(TaskKey{e.c, e.f, e.task});
        }
      }
    }
    if (!execute(c, dec)) break;
    if (c->tails && c->tails->outstanding() && c->cfg.policy == UG_POLICY_URGENCY &&
        c->policy.order() != c->last_order) {
      // the device queue follows the gate's new ranking
      c->last_order = c->policy.order();
      std::map<ug::Key, uint64_t> rank;
      for (size_t r = 0; r < c->last_order.size(); ++r) rank[c->last_order[r]] = r + 1;
      for (const auto& kv : c->inst_tails) {
        const ug::Key key{std::get<0>(kv.first), std::get<1>(kv.first)};
        auto rk = rank.find(key);
        const uint64_t hi = (rk == rank.end() ? 0xffffffffull : rk->second) << 32;
        auto dn = c->inst_tails_done.find(kv.first);
        for (size_t i = dn == c->inst_tails_done.end() ? 0 : dn->second; i < kv.second.size(); ++i)
          c->tails->set_key(kv.second[i].slot, hi | (kv.second[i].pub & 0xffffffffull));
      }
      c->tails->commit_keys();
    }
    deliver_completions(c);
  }
  c->cv_done.notify_all();
}

void stop_thread(Ctx* c) {
  if (c->thr.joinable()) {
    c->stop.store(true);
    c->thr.join();
  }
  c->stop.store(false);
}

ug_status submit_frame(Ctx* c, uint32_t chain, int64_t t_arr_ns, void* const* buffers,
                 uint32_t n_buffers, const int64_t* dims, uint32_t n_dims, uint64_t* frame) {
  if (!c) return UG_EINVAL;
  if (sticky(c)) return UG_EDEVICE;
  if (!c->started) return fail(c, UG_ESTATE, "not started");
  const auto& chs = c->policy.chains();
  if (chain >= chs.size() || !buffers || n_buffers != chs[chain].n_buffers)
    return fail(c, UG_EINVAL, "submit: bad chain or buffer count");
  for (uint32_t i = 0; i < n_buffers; ++i)
    if (!buffers[i]) return fail(c, UG_EINVAL, "submit: null buffer");
  const DimRange& dr = c->dim_range[chain];
  if (n_dims < dr.lo.size() || (n_dims && !dims))
    return fail(c, UG_EINVAL, "submit: the chain needs per-frame sizes (ug_frame_submit_dims)");
  for (size_t d = 0; d < dr.lo.size(); ++d)
    if (dims[d] < dr.lo[d] || dims[d] > dr.hi[d])
      return fail(c, UG_EINVAL, "submit: per-frame size out of the registered range");
  Frame f;
  f.chain = chain;
  f.t_arr = t_arr_ns < 0 ? mono_ns() : t_arr_ns;
  f.buffers.assign(buffers, buffers + n_buffers);
  if (n_dims) f.dims.assign(dims, dims + n_dims);
  std::lock_guard<std::mutex> lk(c->mu);
  if (c->outstanding >= c->cfg.queue_capacity) return UG_EAGAIN;
  const uint64_t fp = c->footprint[chain];
  if (c->cfg.hbm_budget_bytes && fp > c->cfg.hbm_budget_bytes - std::min(c->inflight_bytes,
                                                                          c->cfg.hbm_budget_bytes)) {
    ++c->st_deferred;
    return UG_EAGAIN;
  }
  c->inflight_bytes += fp;
  c->hbm_peak = std::max(c->hbm_peak, c->inflight_bytes);
  f.f = c->next_frame[chain]++;
  if (frame) *frame = static_cast<uint64_t>(f.f);
  c->inbox.push_back(std::move(f));
  ++c->outstanding;
  c->st_submitted++;
  return UG_OK;
}
}  // namespace

// ========================================================================
extern "C" {

void ug_config_default(ug_config* cfg) {
  if (!cfg) return;
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->abi_version = UG_ABI_VERSION;
  cfg->policy = UG_POLICY_URGENCY;
  cfg->flags = UG_F_BIND | UG_F_DELAY | UG_F_BATCH | UG_F_ADMIT | UG_F_PLACE;
  cfg->device = 0;
  cfg->delta_eval_ns = 500000;
  cfg->delay_poll_ns = 1000000;
  cfg->util_exempt = 0.1f;
  cfg->n_levels = 2;
  cfg->lanes[0] = 2;
  cfg->lanes[1] = 6;
  cfg->th_slack_ns = 0;
  cfg->idle_sleep_ns = 0;
  cfg->queue_capacity = 4096;
  cfg->trace_capacity = 0;
  cfg->calib_period_ns = 1000000;
  cfg->admit_tasks = 4;
  cfg->hbm_budget_bytes = 0;
  cfg->order_key = UG_KEY_URGENCY;
  cfg->est_noise_permille = 0;
  cfg->noise_seed = 0;
  cfg->own_streams = 0;
  cfg->max_hold_ns = 0;
  cfg->cpu_cores = 0;
  cfg->fuse_workers = 64;
  cfg->fuse_idle_ns = 500000;
}

int64_t ug_now_ns(void) { return mono_ns(); }

const char* ug_status_str(ug_status s) {
  switch (s) {
    case UG_OK: return "ok";
    case UG_EINVAL: return "invalid argument";
    case UG_ENOMEM: return "out of memory";
    case UG_EDEVICE: return "device error";
    case UG_EAGAIN: return "queue full";
    case UG_ETIMEDOUT: return "timed out";
    case UG_ESTATE: return "invalid state";
    case UG_ENODEV: return "no device";
    default: return "unknown status";
  }
}

ug_status ug_create(const ug_config* cfg, void** out) {
  if (!cfg || !out) return UG_EINVAL;
  *out = nullptr;
  if (cfg->abi_version != UG_ABI_VERSION) return UG_EINVAL;
  if (cfg->policy != UG_POLICY_FIFO && cfg->policy != UG_POLICY_URGENCY) return UG_EINVAL;
  if (cfg->n_levels < 1 || cfg->n_levels > 8) return UG_EINVAL;
  for (int i = 0; i < cfg->n_levels; ++i)
    if (cfg->lanes[i] < 1 || cfg->lanes[i] > 64) return UG_EINVAL;
  if (cfg->own_streams != 0 && cfg->own_streams != 1) return UG_EINVAL;
  if (cfg->max_hold_ns < 0) return UG_EINVAL;
  if (cfg->cpu_cores < 0 || cfg->cpu_cores > 1024) return UG_EINVAL;
  if ((cfg->flags & UG_F_FUSE) &&
      (cfg->fuse_workers < 1 || cfg->fuse_workers > 1024 || cfg->fuse_idle_ns <= 0))
    return UG_EINVAL;
  if (cfg->delta_eval_ns < 0 || cfg->delay_poll_ns < 0 || cfg->queue_capacity == 0 ||
      cfg->calib_period_ns < 0 || cfg->admit_tasks < 1 || cfg->order_key < UG_KEY_URGENCY ||
      cfg->order_key > UG_KEY_EQDF || cfg->est_noise_permille < 0 ||
      cfg->est_noise_permille > 1000)
    return UG_EINVAL;
  if (cfg->tile_table && ug::tune_load(cfg->tile_table) < 0) {
    std::lock_guard<std::mutex> lk(g_create_mu);
    g_create_error = std::string("tile table unreadable or malformed: ") + cfg->tile_table;
    return UG_EINVAL;
  }
  std::unique_ptr<Ctx> c(new (std::nothrow) Ctx());
  if (!c) return UG_ENOMEM;
  c->cfg = *cfg;
  c->cfg.tile_table = nullptr;   // read here; the caller's string is not kept
  c->policy = ug::Policy(policy_config(*cfg));
  c->has_device = cfg->device >= 0;
  if (c->has_device) {
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || cfg->device >= n) {
      return e != hipSuccess ? hip_fail(nullptr, e, "hipGetDeviceCount") : UG_EINVAL;
    }
    if ((e = hipSetDevice(cfg->device)) != hipSuccess) return hip_fail(nullptr, e, "hipSetDevice");
    for (int i = 0; i < 1024; ++i) {
      hipEvent_t ev = nullptr;
      if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess)
        return hip_fail(nullptr, e, "hipEventCreateWithFlags");
      c->event_pool.push_back(ev);
      c->all_events.push_back(ev);
    }
  }
  c->trace.reserve(std::min<uint32_t>(cfg->trace_capacity, 1u << 22));
  *out = c.release();
  return UG_OK;
}

void ug_destroy(void* ctx) {
  Ctx* c = static_cast<Ctx*>(ctx);
  if (!c) return;
  stop_thread(c);
  if (c->has_device) {
    (void)hipSetDevice(c->cfg.device);
    // the executor first: a stream on its hardware queue waits behind it
    c->tails.reset();
    if (c->fuse_stream) {
      (void)hipStreamSynchronize(c->fuse_stream);
      (void)hipStreamDestroy(c->fuse_stream);
    }
    // every stream the gate launched on has drained before anything is freed
    for (auto& lv : c->level_streams)
      for (hipStream_t s : lv) (void)hipStreamSynchronize(s);
    for (hipStream_t s : c->fifo_streams) (void)hipStreamSynchronize(s);
    if (c->capture_stream) (void)hipStreamSynchronize(c->capture_stream);
    if (c->slot_counters) (void)hipFree(c->slot_counters);
    for (unsigned* p : c->counter_chunks) (void)hipFree(p);
    for (hipStream_t s : c->owned_streams) (void)hipStreamDestroy(s);
    for (hipEvent_t e : c->all_events) (void)hipEventDestroy(e);
    for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second.ge);
    if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
    for (auto& v : c->ws)
      for (void* p : v)
        if (p) (void)hipFree(p);
  }
  delete c;
}

const char* ug_last_error(void* ctx) {
  // a copy per calling thread: the context's message may be replaced by
  // another thread at any time
  static thread_local std::string copy;
  Ctx* c = static_cast<Ctx*>(ctx);
  if (c) {
    std::lock_guard<std::mutex> lk(c->err_mu);
    copy = c->last_error;
  } else {
    std::lock_guard<std::mutex> lk(g_create_mu);
    copy = g_create_error;
  }
  return copy.c_str();
}

ug_status ug_chain_register(void* ctx, int64_t period_ns, int64_t deadline_ns,
                            const ug_task* tasks, uint32_t n_tasks, uint32_t n_buffers,
                            uint32_t* chain_id) {
  Ctx* c = static_cast<Ctx*>(ctx);
  if (!c) return UG_EINVAL;
  if (sticky(c)) return UG_EDEVICE;
  if (c->started || c->finalized) return fail(c, UG_ESTATE, "chains are registered before start");
  if (!tasks || n_tasks == 0 || deadline_ns < 0 || period_ns < 0)
    return fail(c, UG_EINVAL, "chain needs tasks and a deadline >= 0");
  ug::ChainSpec spec;
  spec.period_ns = period_ns;
  spec.deadline_ns = deadline_ns;
  spec.best_effort = deadline_ns == 0;
  spec.n_buffers = n_buffers;
  DimRange dr;
  for (uint32_t j = 0; j < n_tasks; ++j) {
    const ug_task& t = tasks[j];
    if (!t.kernels || t.n_kernels == 0 || t.cpu_ns < 0)
      return fail(c, UG_EINVAL, "every task needs at least one kernel and cpu_ns >= 0");
    spec.task_first.push_back(static_cast<int32_t>(spec.kernels.size()));
    for (uint32_t k = 0; k < t.n_kernels; ++k) {
      const ug_kernel& kd = t.kernels[k];
      if (const char* why = ug::validate_kernel(kd, n_buffers)) return fail(c, UG_EINVAL, why);
      if (kd.est_ns < 0) return fail(c, UG_EINVAL, "est_ns must be >= 0");
      if (kd.frame_dim < 0 || kd.frame_dim > 4) return fail(c, UG_EINVAL, "frame_dim must be in 0..4");
      if (kd.frame_dim > 0) {
        // the per-frame values this kernel accepts, by its op's frame
        // dimension (at most the registered size)
        int64_t lo = 0, hi = 0;
        if (!ug::frame_range(kd, &lo, &hi))
          return fail(c, UG_EINVAL, "this op or registered shape takes no per-frame size");
        const size_t d = static_cast<size_t>(kd.frame_dim - 1);
        if (dr.lo.size() <= d) {
          dr.lo.resize(d + 1, 0);
          dr.hi.resize(d + 1, INT64_MAX);
        }
        dr.lo[d] = std::max(dr.lo[d], lo);
        dr.hi[d] = std::min(dr.hi[d], hi);
        if (dr.lo[d] > dr.hi[d])
          return fail(c, UG_EINVAL, "the kernels sharing a per-frame size admit no common value");
      } else if (kd.frame_shift != 0) {
        return fail(c, UG_EINVAL, "frame_shift without frame_dim");
      }
      float u = kd.util;
      if (u < 0.f && kd.op == UG_OP_UPLOAD_H2D) u = 1.0f;   // delayed like a full launch
      if (u < 0.f) {
        if (c->has_device) {
          if (ug_kernel_util(&kd, c->cfg.device, &u) != UG_OK) u = 1.0f;
        } else {
          u = 1.0f;
        }
      }
      spec.kernels.push_back(kd);
      spec.est.push_back(kd.est_ns);
      spec.util.push_back(u);
      spec.fdim.push_back(kd.frame_dim);
    }
    spec.task_end.push_back(static_cast<int32_t>(spec.kernels.size()));
    spec.cpu.push_back(t.cpu_ns);
  }
  std::vector<void*> ws(spec.kernels.size(), nullptr);
  std::vector<size_t> wsb(spec.kernels.size(), 0);
  for (size_t k = 0; k < spec.kernels.size(); ++k) {
    wsb[k] = ug::workspace_bytes(spec.kernels[k]);
    if (wsb[k] == 0 || !c->has_device) continue;
    (void)hipSetDevice(c->cfg.device);
    if (hipMalloc(&ws[k], wsb[k]) != hipSuccess) {
      (void)hipGetLastError();
      for (void* p : ws)
        if (p) (void)hipFree(p);
      return fail(c, UG_ENOMEM, "kernel workspace allocation failed");
    }
  }
  for (size_t d = 0; d < dr.lo.size(); ++d)
    if (dr.hi[d] == INT64_MAX) dr.lo[d] = dr.hi[d] = 0;  // an unused index accepts 0
  c->ws.push_back(std::move(ws));
  c->ws_bytes.push_back(std::move(wsb));
  std::vector<int32_t> mark(spec.kernels.size(), -1);
  for (size_t j = 0; j < spec.task_first.size(); ++j)
    ug::tail_runs(spec.kernels, spec.task_first[j], spec.task_end[j], &mark);
  c->tail_mark.push_back(std::move(mark));
  const uint32_t id = c->policy.add_chain(std::move(spec));
  c->next_frame.push_back(0);
  c->footprint.push_back(0);
  c->dim_range.push_back(std::move(dr));
  if (chain_id) *chain_id = id;
  return UG_OK;
}

ug_status ug_kernel_set_estimate(void* ctx, uint32_t chain, uint32_t kernel, int64_t est_ns,
                                 float util) {
  Ctx* c = static_cast<Ctx*>(ctx);
  if (!c) return UG_EINVAL;
  if (c->started) return fail(c, UG_ESTATE, "estimates are set before start");
  auto& chs = c->policy.chains();
  if (chain >= chs.size() || kernel >= chs[chain].est.size() || est_ns < 0)
    return fail(c, UG_EINVAL, "no such kernel");
  chs[chain].est[kernel] = est_ns;
  if (util >= 0.f) chs[chain].util[kernel] = util;
  chs[chain].finalize();
  return UG_OK;
}

ug_status ug_kernel_get_estimate(void* ctx, uint32_t chain, uint32_t kernel, int64_t* est_ns,
                                 float* util) {
  Ctx* c = static_cast<Ctx*>(ctx);
  if (!c) return UG_EINVAL;
  const auto& chs = c->policy.chains();
  if (chain >= chs.size() || kernel >= chs[chain].est.size())
    return fail(c, UG_EINVAL, "no such kernel");
  if (est_ns) *est_ns = chs[chain].est[kernel];
  if (util) *util = chs[chain].util[kernel];
  return UG_OK;
}

ug_status ug_profile(void* ctx, uint32_t chain, void* const* buffers, uint32_t n_buffers,
                     uint32_t warmup, uint32_t reps) {
  Ctx* c = static_cast<Ctx*>(ctx);
  if (!c) return UG_EINVAL;
  if (sticky(c)) return UG_EDEVICE;
  if (!c->has_device) return fail(c, UG_ENODEV, "profiling needs a device");
  if (c->started) return fail(c, UG_ESTATE, "profile before start");
  auto& chs = c->policy.chains();
  if (chain >= chs.size() || !buffers || n_buffers != chs[chain].n_buffers || reps == 0)
    return fail(c, UG_EINVAL, "profile: bad chain, buffers or reps");
  for (uint32_t i = 0; i < n_buffers; ++i)
    if (!buffers[i]) return fail(c, UG_EINVAL, "profile: null buffer");
  (void)hipSetDevice(c->cfg.device);
  hipStream_t s = nullptr;
  hipError_t e;
  if ((e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) != hipSuccess)
    return hip_fail(c, e, "hipStreamCreateWithFlags");
  std::vector<hipEvent_t> ev(2 * reps);
  for (auto& x : ev) (void)hipEventCreate(&x);
  std::map<std::vector<int64_t>, int64_t> measured;
  ug::ChainSpec& ch = chs[chain];
  ug_status st = UG_OK;
  // median of `reps` isolated runs of one kernel shape (shared by equal shapes)
  auto measure = [&](const ug_kernel& kd, void* w, size_t wb, int64_t* out) -> bool {
    std::vector<int64_t> key{kd.op, kd.shape[0], kd.shape[1], kd.shape[2], kd.shape[3]};
    auto it = measured.find(key);
    if (it != measured.end()) {
      *out = it->second;
      return true;
    }
    for (uint32_t i = 0; i < warmup; ++i)
      if ((e = ug::launch_kernel(kd, buffers, s, w, wb)) != hipSuccess) {
        st = hip_fail(c, e, "profile launch");
        return false;
      }
    std::vector<float> ms(reps);
    for (uint32_t r = 0; r < reps; ++r) {
      (void)hipEventRecord(ev[2 * r], s);
      if ((e = ug::launch_kernel(kd, buffers, s, w, wb)) != hipSuccess) {
        st = hip_fail(c, e, "profile launch");
        return false;
      }
      (void)hipEventRecord(ev[2 * r + 1], s);
    }
    if ((e = hipStreamSynchronize(s)) != hipSuccess) {
      st = hip_fail(c, e, "hipStreamSynchronize");
      return false;
    }
    for (uint32_t r = 0; r < reps; ++r) (void)hipEventElapsedTime(&ms[r], ev[2 * r], ev[2 * r + 1]);
    std::sort(ms.begin(), ms.end());
    *out = static_cast<int64_t>(ms[reps / 2] * 1.0e6);
    measured[key] = *out;
    return true;
  };
  for (size_t k = 0; k < ch.kernels.size() && st == UG_OK; ++k) {
    const ug_kernel& kd = ch.kernels[k];
    void* w = c->ws[chain][k];
    const size_t wb = c->ws_bytes[chain][k];
    if (kd.frame_dim <= 0) {
      int64_t est = 0;
      if (!measure(kd, w, wb, &est)) break;
      ch.est[k] = est;
      continue;
    }
    // a per-frame size: profile points at the largest value the chain
    // accepts and at 1/2, 1/4, 1/8 of it (no lower than the smallest)
    const DimRange& dr = c->dim_range[chain];
    const size_t d = static_cast<size_t>(kd.frame_dim - 1);
    const int64_t hi = dr.hi[d], lo = std::max<int64_t>(dr.lo[d], 1);
    std::vector<std::pair<int64_t, int64_t>> pts;
    for (int q = 3; q >= 0 && st == UG_OK; --q) {
      const int64_t v = std::max(lo, hi >> q);
      if (!pts.empty() && pts.back().first >= v) continue;
      int64_t est = 0;
      if (!measure(ug::frame_kernel(kd, v), w, wb, &est)) break;
      pts.push_back({v, est});
    }
    if (st != UG_OK) break;
    ch.prof[k] = pts;
    ch.est[k] = pts.back().second;
  }
  ch.finalize();
  for (auto& x : ev) (void)hipEventDestroy(x);
  (void)hipStreamDestroy(s);
  return st;
}

ug_status ug_kernel_set_profile(void* ctx, uint32_t chain, uint32_t kernel, const int64_t* v,
                                const int64_t* e, uint32_t n) {
  Ctx* c = static_cast<Ctx*>(ctx);
  if (!c) return UG_EINVAL;
  if (c->started) return fail(c, UG_ESTATE, "profiles are set before start");
  auto& chs = c->policy.chains();
  if (chain >= chs.size() || kernel >= chs[chain].est.size())
    return fail(c, UG_EINVAL, "no such kernel");
  ug::ChainSpec& ch = chs[chain];
  if (ch.fdim[kernel] <= 0) return fail(c, UG_EINVAL, "the kernel has no per-frame size");
  if (n > 16 || (n && (!v || !e))) return fail(c, UG_EINVAL, "profile: at most 16 points");
  std::vector<std::pair<int64_t, int64_t>> pts;
  for (uint32_t i = 0; i < n; ++i) {
    if (e[i] < 0 || (i && v[i] <= v[i - 1]))
      return fail(c, UG_EINVAL, "profile: values increasing, estimates >= 0");
    pts.push_back({v[i], e[i]});
  }
  ch.prof[kernel] = pts;
  ch.finalize();
  return UG_OK;
}

ug_status ug_kernel_get_profile(void* ctx, uint32_t chain, uint32_t kernel, int64_t* v,
                                int64_t* e, uint32_t cap, uint32_t* n) {
  Ctx* c = static_cast<Ctx*>(ctx);
  if (!c || !n || (cap && (!v || !e))) return UG_EINVAL;
  const auto& chs = c->policy.chains();
  if (chain >= chs.size() || kernel >= chs[chain].est.size())
    return fail(c, UG_EINVAL, "no such kernel");
  const auto& pts = chs[chain].prof[kernel];
  *n = static_cast<uint32_t>(pts.size());
  for (uint32_t i = 0; i < cap && i < pts.size(); ++i) {
    v[i] = pts[i].first;
    e[i] = pts[i].second;
  }
  return UG_OK;
}

ug_status ug_set_threshold(void* ctx, int64_t th_slack_ns) {
  Ctx* c = static_cast<Ctx*>(ctx);
  if (!c) return UG_EINVAL;
  if (c->started) return fail(c, UG_ESTATE, "stop before changing the threshold");
  c->cfg.th_slack_ns = th_slack_ns;
  c->policy.mutable_config().th_slack_ns = th_slack_ns;
  return UG_OK;
}

ug_status ug_set_flags(void* ctx, int32_t policy, uint32_t flags) {
  Ctx* c = static_cast<Ctx*>(ctx);
  if (!c) return UG_EINVAL;
  if (c->started) return fail(c, UG_ESTATE, "stop before changing flags");
  if (policy != c->cfg.policy) return fail(c, UG_EINVAL, "the policy is fixed at creation");
  c->cfg.flags = flags;
  ug::PolicyConfig& p = c->policy.mutable_config();
  p.bind = (flags & UG_F_BIND) != 0;
  p.delay = (flags & UG_F_DELAY) != 0;
  p.batch = (flags & UG_F_BATCH) != 0;
  p.calibrate = (flags & UG_F_CALIBRATE) != 0;
  p.admit = (flags & UG_F_ADMIT) != 0;
  p.exit = (flags & UG_F_EXIT) != 0;
  p.no_overlap = (flags & UG_F_NO_OVERLAP) != 0;
  p.graph = (flags & UG_F_GRAPH) != 0;
  p.cpu_prio = (flags & UG_F_CPU_PRIO) != 0;
  p.keep_order = (flags & UG_F_FUSE) != 0;
  return UG_OK;
}

ug_status ug_start(void* ctx) {
  Ctx* c = static_cast<Ctx*>(ctx);
  if (!c) return UG_EINVAL;
  if (sticky(c)) return UG_EDEVICE;
  if (!c->has_device) return fail(c, UG_ENODEV, "no device");
  if (c->started) return fail(c, UG_ESTATE, "already started");
  (void)hipSetDevice(c->cfg.device);
  if (!c->streams_attached) {
    if (!c->cfg.own_streams)
      return fail(c, UG_ESTATE, "no streams: attach them with ug_attach_streams (or set own_streams)");
    if (c->policy.chains().empty()) return fail(c, UG_ESTATE, "no chain registered");
    hipError_t e = create_own_streams(c);
    if (e != hipSuccess) return hip_fail(c, e, "stream creation");
    c->streams_attached = true;
  }
  c->policy.reset();
  c->finalized = true;
  c->inst_tails.clear();
  c->inst_tails_done.clear();
  c->reserved.clear();
  c->covered_to.clear();
  c->executor_launches = 0;
  for (uint64_t& v : c->fuse_stats) v = 0;
  c->ev_tails.clear();
  c->last_order.clear();
  if (c->cfg.flags & UG_F_FUSE) {
    if (c->cfg.fuse_workers < 1 || c->cfg.fuse_workers > 1024 || c->cfg.fuse_idle_ns <= 0)
      return fail(c, UG_EINVAL, "fused tails need fuse_workers in 1..1024 and fuse_idle_ns > 0");
    // the completion counters, zeroed at every start
    hipError_t e = hipSuccess;
    if (!c->fuse_stream &&
        (e = hipStreamCreateWithFlags(&c->fuse_stream, hipStreamNonBlocking)) != hipSuccess)
      return hip_fail(c, e, "tail executor stream");
    if ((e = zero_counters(c)) != hipSuccess) return hip_fail(c, e, "completion counters");
    c->tails.reset(new ug::TailQueue());
    // lease: a minute per launch, renewed by the next launch
    if ((e = c->tails->open(c->cfg.device, c->cfg.fuse_workers, c->cfg.fuse_idle_ns,
                            int64_t(60) * 1000000000, 0, c->fuse_stream)) != hipSuccess) {
      c->tails.reset();
      return hip_fail(c, e, "tail executor");
    }
  }
  c->live_events.clear();
  c->event_pool = c->all_events;
  c->bound.clear();
  c->frames.clear();
  c->pending.clear();
  {
    std::lock_guard<std::mutex> lk(c->mu);
    c->latencies.clear();
    c->chain_done.assign(c->policy.chains().size(), 0);
    c->chain_missed.assign(c->policy.chains().size(), 0);
    c->inflight_bytes = 0;   // no frame is outstanding at a start
    c->hbm_peak = 0;
    c->st_deferred = 0;
  }
  // counters cover the frames since this start, like the metrics
  for (auto* a : {&c->st_submitted, &c->st_completed, &c->st_missed, &c->st_launches,
                  &c->st_holds, &c->st_batches, &c->st_instants, &c->st_tails,
                  &c->st_tails_unfused})
    a->store(0);
  c->st_decide_ns.store(0);
  c->st_launch_ns.store(0);
  c->stop.store(false);
  c->started = true;
  c->thr = std::thread(gate_main, c);
  return UG_OK;
}

ug_status ug_frame_submit(void* ctx, uint32_t chain, int64_t t_arr_ns, void* const* buffers,
                          uint32_t n_buffers, uint64_t* frame) {
  return submit_frame(static_cast<Ctx*>(ctx), chain, t_arr_ns, buffers, n_buffers, nullptr, 0, frame);
}

ug_status ug_frame_submit_dims(void* ctx, uint32_t chain, int64_t t_arr_ns, void* const* buffers,
                               uint32_t n_buffers, const int64_t* dims, uint32_t n_dims,
                               uint64_t* frame) {
  return submit_frame(static_cast<Ctx*>(ctx), chain, t_arr_ns, buffers, n_buffers, dims, n_dims, frame);
}

ug_status ug_chain_set_footprint(void* ctx, uint32_t chain, uint64_t bytes) {
  Ctx* c = static_cast<Ctx*>(ctx);
  if (!c) return UG_EINVAL;
  if (c->started || c->finalized) return fail(c, UG_ESTATE, "footprints are set before start");
  if (chain >= c->footprint.size()) return fail(c, UG_EINVAL, "no such chain");
  c->footprint[chain] = bytes;
  return UG_OK;
}

ug_status ug_streams_needed(void* ctx, uint32_t* n) {
  Ctx* c = static_cast<Ctx*>(ctx);
  if (!c || !n) return UG_EINVAL;
  *n = streams_needed(c);
  return UG_OK;
}

ug_status ug_attach_streams(void* ctx, void* const* hip_streams, uint32_t n) {
  Ctx* c = static_cast<Ctx*>(ctx);
  if (!c) return UG_EINVAL;
  if (sticky(c)) return UG_EDEVICE;
  if (!c->has_device) return fail(c, UG_ENODEV, "streams need a device");
  if (c->started) return fail(c, UG_ESTATE, "streams are attached before start");
  if (c->streams_attached) return fail(c, UG_ESTATE, "streams are already attached");
  if (c->cfg.policy == UG_POLICY_FIFO && c->policy.chains().empty())
    return fail(c, UG_ESTATE, "FIFO launch: register the chains before attaching streams");
  if (!hip_streams || n != streams_needed(c))
    return fail(c, UG_EINVAL, "attach: wrong number of streams (see ug_streams_needed)");
  std::vector<hipStream_t> pool;
  for (uint32_t i = 0; i < n; ++i) {
    if (!hip_streams[i]) return fail(c, UG_EINVAL, "attach: null stream (the default stream is not accepted)");
    pool.push_back(static_cast<hipStream_t>(hip_streams[i]));
  }
  std::vector<hipStream_t> sorted_pool = pool;
  std::sort(sorted_pool.begin(), sorted_pool.end());
  if (std::adjacent_find(sorted_pool.begin(), sorted_pool.end()) != sorted_pool.end())
    return fail(c, UG_EINVAL, "attach: a stream is given twice");
  (void)hipSetDevice(c->cfg.device);
  hipError_t e = assign_streams(c, std::move(pool));
  if (e != hipSuccess) return hip_fail(c, e, "hardware-queue probe");
  c->streams_attached = true;
  return UG_OK;
}

int32_t ug_poll_complete(void* ctx, ug_completion* out, uint32_t cap) {
  Ctx* c = static_cast<Ctx*>(ctx);
  if (!c || (!out && cap)) return UG_EINVAL;
  std::lock_guard<std::mutex> lk(c->mu);
  uint32_t n = 0;
  while (n < cap && !c->outbox.empty()) {
    out[n++] = c->outbox.front();
    c->outbox.pop_front();
  }
  if (n == 0 && sticky(c)) return UG_EDEVICE;
  return static_cast<int32_t>(n);
}

ug_status ug_drain(void* ctx, int64_t timeout_ns) {
  Ctx* c = static_cast<Ctx*>(ctx);
  if (!c) return UG_EINVAL;
  if (!c->started) return UG_OK;
  std::unique_lock<std::mutex> lk(c->mu);
  const auto deadline = std::chrono::steady_clock::now() + std::chrono::nanoseconds(timeout_ns);
  while (c->outstanding > 0) {
    if (sticky(c)) return UG_EDEVICE;
    if (c->cv_done.wait_until(lk, deadline) == std::cv_status::timeout && c->outstanding > 0)
      return fail(c, UG_ETIMEDOUT, "drain timed out");
  }
  return sticky(c) ? UG_EDEVICE : UG_OK;
}

ug_status ug_stop(void* ctx) {
  Ctx* c = static_cast<Ctx*>(ctx);
  if (!c) return UG_EINVAL;
  if (!c->started) return UG_OK;
  stop_thread(c);
  c->started = false;
  if (c->has_device) {
    (void)hipSetDevice(c->cfg.device);
    // the executor first: a stream on its hardware queue waits behind it
    if (c->tails) {
      c->executor_launches += c->tails->launches();
      uint64_t st[ug::kStatCount] = {};
      if (c->tails->halt() == hipSuccess && c->tails->stats(st) == hipSuccess)
        for (int k = 0; k < ug::kStatCount; ++k) c->fuse_stats[k] += st[k];
    }
    c->tails.reset();
    for (auto& lv : c->level_streams)
      for (hipStream_t s : lv) (void)hipStreamSynchronize(s);
    for (hipStream_t s : c->fifo_streams) (void)hipStreamSynchronize(s);
  }
  {
    std::lock_guard<std::mutex> lk(c->mu);
    c->inbox.clear();
    c->outstanding = 0;
    for (auto& n : c->next_frame) n = 0;
  }
  return sticky(c) ? UG_EDEVICE : UG_OK;
}

ug_status ug_get_stats(void* ctx, ug_stats* out) {
  Ctx* c = static_cast<Ctx*>(ctx);
  if (!c || !out) return UG_EINVAL;
  std::memset(out, 0, sizeof(*out));
  out->frames_submitted = c->st_submitted.load();
  out->frames_completed = c->st_completed.load();
  out->frames_missed = c->st_missed.load();
  out->launches = c->st_launches.load();
  out->holds = c->st_holds.load();
  out->batches = c->st_batches.load();
  out->instants = c->st_instants.load();
  out->collisions = c->started ? 0 : c->policy.collisions();
  if (!c->started)
    for (size_t i = 0; i < 8; ++i) out->collision_hist[i] = c->policy.collision_hist()[i];
  out->decide_ns = c->st_decide_ns.load();
  out->launch_ns = c->st_launch_ns.load();
  out->tails_fused = c->st_tails.load();
  out->tails_unfused = c->st_tails_unfused.load();
  out->executor_launches = c->executor_launches;
  {
    std::lock_guard<std::mutex> lk(c->mu);
    out->frames_deferred = c->st_deferred;
    out->hbm_peak_bytes = c->hbm_peak;
  }
  std::lock_guard<std::mutex> lk(c->trace_mu);
  out->trace_records = c->trace.size();
  out->trace_dropped = c->trace_dropped;
  return UG_OK;
}

int32_t ug_trace_read(void* ctx, ug_record* out, uint32_t cap) {
  Ctx* c = static_cast<Ctx*>(ctx);
  if (!c || (!out && cap)) return UG_EINVAL;
  std::lock_guard<std::mutex> lk(c->trace_mu);
  const uint32_t n = static_cast<uint32_t>(std::min<size_t>(cap, c->trace.size()));
  std::copy(c->trace.begin(), c->trace.begin() + n, out);
  c->trace.erase(c->trace.begin(), c->trace.begin() + n);
  return static_cast<int32_t>(n);
}

int32_t ug_calibration_read(void* ctx, int64_t* out, uint32_t cap) {
  Ctx* c = static_cast<Ctx*>(ctx);
  if (!c || (!out && cap)) return UG_EINVAL;
  if (c->started) return fail(c, UG_ESTATE, "stop before reading samples");
  const auto& s = c->policy.samples();
  const uint32_t n = static_cast<uint32_t>(std::min<size_t>(cap, s.size()));
  std::copy(s.begin(), s.begin() + n, out);
  return static_cast<int32_t>(n);
}

ug_status ug_calibration_threshold(void* ctx, int32_t pct, int64_t* th_slack_ns) {
  Ctx* c = static_cast<Ctx*>(ctx);
  if (!c || !th_slack_ns || pct < 1 || pct > 100) return UG_EINVAL;
  if (c->started) return fail(c, UG_ESTATE, "stop before computing the threshold");
  std::vector<int64_t> s = c->policy.samples();
  *th_slack_ns = 0;
  if (s.empty()) return UG_OK;
  // ascending urgency: a before b iff UL(b) > UL(a)
  std::sort(s.begin(), s.end(), [](int64_t a, int64_t b) { return ug::ul_greater(b, a); });
  const size_t n = s.size();
  const size_t idx = (static_cast<size_t>(pct) * n + 99) / 100 - 1;
  *th_slack_ns = s[idx] > 0 ? s[idx] : 0;
  return UG_OK;
}

ug_status ug_get_metrics(void* ctx, ug_metrics* out) {
  Ctx* c = static_cast<Ctx*>(ctx);
  if (!c || !out) return UG_EINVAL;
  std::memset(out, 0, sizeof(*out));
  std::vector<int64_t> lat;
  {
    std::lock_guard<std::mutex> lk(c->mu);
    lat = c->latencies;
    double ratio_sum = 0.0;
    for (size_t i = 0; i < c->chain_done.size(); ++i) {
      if (c->chain_done[i] == 0) continue;
      out->n_chains += 1;
      out->missed += c->chain_missed[i];
      ratio_sum += static_cast<double>(c->chain_missed[i]) / static_cast<double>(c->chain_done[i]);
    }
    out->miss_ratio = out->n_chains ? ratio_sum / out->n_chains : 0.0;
  }
  out->frames = lat.size();
  if (lat.empty()) return UG_OK;
  std::sort(lat.begin(), lat.end());
  const size_t n = lat.size();
  out->p50_ns = lat[(50 * n + 99) / 100 - 1];
  out->p99_ns = lat[(99 * n + 99) / 100 - 1];
  out->max_ns = lat.back();
  double sum = 0.0;
  for (int64_t v : lat) sum += static_cast<double>(v);
  out->mean_ns = sum / static_cast<double>(n);
  return UG_OK;
}

ug_status ug_replay_instant(void* ctx, int64_t t, const ug_record* inputs, uint32_t n_inputs,
                            ug_record* out, uint32_t cap, uint32_t* n_out) {
  Ctx* c = static_cast<Ctx*>(ctx);
  if (!c || (!inputs && n_inputs) || !n_out) return UG_EINVAL;
  if (c->has_device) return fail(c, UG_ESTATE, "replay runs on a context without a device");
  if (!c->finalized) {
    c->policy.reset();
    c->finalized = true;
  }
  std::vector<ug::Arrival> arr;
  std::vector<ug::EvDone> evs;
  for (uint32_t i = 0; i < n_inputs; ++i) {
    const ug_record& r = inputs[i];
    if (r.type == UG_REC_ARRIVE) {
      arr.push_back({r.chain, r.frame, r.t, {}});
    } else if (r.type == UG_REC_DIMS) {
      if (arr.empty() || arr.back().c != r.chain || arr.back().f != r.frame ||
          r.a != static_cast<int32_t>(arr.back().dims.size()))
        return fail(c, UG_EINVAL, "replay: DIMS follow their frame's ARRIVE, in index order");
      arr.back().dims.push_back(r.t);
    } else if (r.type == UG_REC_EVDONE)
      evs.push_back({r.chain, r.frame, r.task, r.a, r.b});
    else
      return fail(c, UG_EINVAL, "replay inputs are ARRIVE, DIMS and EVDONE records");
  }
  std::vector<ug_record> dec;
  const char* err = nullptr;
  if (!c->policy.instant(t, arr, evs, dec, &err)) return fail(c, UG_EINVAL, err ? err : "replay");
  c->policy.finished().clear();
  *n_out = static_cast<uint32_t>(dec.size());
  if (dec.size() > cap) return fail(c, UG_ENOMEM, "replay: output buffer too small");
  std::copy(dec.begin(), dec.end(), out);
  return UG_OK;
}

ug_status ug_kernel_launch(const ug_kernel* k, void* const* buffers, uint32_t n_buffers,
                           void* hip_stream) {
  if (!k || !buffers) return UG_EINVAL;
  if (ug::validate_kernel(*k, n_buffers)) return UG_EINVAL;
  const int32_t* slots[2] = {k->in, k->out};
  const int counts[2] = {3, 4};
  for (int a = 0; a < 2; ++a)
    for (int i = 0; i < counts[a]; ++i) {
      const int32_t s = slots[a][i];
      if (s >= 0 && (static_cast<uint32_t>(s) >= n_buffers || !buffers[s])) return UG_EINVAL;
    }
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const size_t wb = ug::workspace_bytes(*k);
  void* w = nullptr;
  // stream-ordered workspace: served from the device's memory pool after
  // the first call, released once the kernel has finished
  if (wb && hipMallocAsync(&w, wb, st) != hipSuccess) return UG_ENOMEM;
  hipError_t e = ug::launch_kernel(*k, buffers, st, w, wb);
  if (w) (void)hipFreeAsync(w, st);
  return e == hipSuccess ? UG_OK : UG_EDEVICE;
}

ug_status ug_kernel_launch_noalloc(const ug_kernel* k, void* const* buffers, uint32_t n_buffers,
                                   void* hip_stream) {
  if (!k || !buffers) return UG_EINVAL;
  if (ug::validate_kernel(*k, n_buffers)) return UG_EINVAL;
  const int32_t* slots[2] = {k->in, k->out};
  const int counts[2] = {3, 4};
  for (int a = 0; a < 2; ++a)
    for (int i = 0; i < counts[a]; ++i) {
      const int32_t s = slots[a][i];
      if (s >= 0 && (static_cast<uint32_t>(s) >= n_buffers || !buffers[s])) return UG_EINVAL;
    }
  const size_t wb = ug::workspace_bytes(*k);
  if (wb > ug::kStaticScratchBytes) return UG_EINVAL;
  void* w = nullptr;
  if (wb && ug::static_scratch(&w) != hipSuccess) return UG_EDEVICE;
  hipError_t e = ug::launch_kernel(*k, buffers, static_cast<hipStream_t>(hip_stream), w, wb);
  return e == hipSuccess ? UG_OK : UG_EDEVICE;
}

ug_status ug_kernel_workspace(const ug_kernel* k, uint64_t* bytes) {
  if (!k || !bytes) return UG_EINVAL;
  if (ug::validate_kernel(*k, 16)) return UG_EINVAL;
  *bytes = ug::workspace_bytes(*k);
  return UG_OK;
}

ug_status ug_kernel_launch_ws(const ug_kernel* k, void* const* buffers, uint32_t n_buffers,
                              void* workspace, uint64_t workspace_bytes, void* hip_stream) {
  if (!k || !buffers) return UG_EINVAL;
  if (ug::validate_kernel(*k, n_buffers)) return UG_EINVAL;
  const int32_t* slots[2] = {k->in, k->out};
  const int counts[2] = {3, 4};
  for (int a = 0; a < 2; ++a)
    for (int i = 0; i < counts[a]; ++i) {
      const int32_t s = slots[a][i];
      if (s >= 0 && (static_cast<uint32_t>(s) >= n_buffers || !buffers[s])) return UG_EINVAL;
    }
  const size_t need = ug::workspace_bytes(*k);
  if (need && (!workspace || workspace_bytes < need ||
               (reinterpret_cast<uintptr_t>(workspace) & 255)))
    return UG_EINVAL;
  hipError_t e = ug::launch_kernel(*k, buffers, static_cast<hipStream_t>(hip_stream), workspace,
                                   static_cast<size_t>(workspace_bytes));
  return e == hipSuccess ? UG_OK : UG_EDEVICE;
}

ug_status ug_kernel_util(const ug_kernel* k, int32_t device, float* util) {
  if (!k || !util) return UG_EINVAL;
  if (ug::validate_kernel(*k, 16)) return UG_EINVAL;
  ug::OpPlan p = ug::plan_kernel(*k);
  if (!p.func) return UG_EINVAL;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
      cus <= 0)
    return UG_EDEVICE;
  // fraction of the device's compute units the launch occupies
  const double wgs = static_cast<double>(p.grid.x) * p.grid.y * p.grid.z;
  *util = static_cast<float>(std::min(1.0, wgs / static_cast<double>(cus)));
  return UG_OK;
}

// ---------------------------------------------------------------- tails

ug_status ug_tails_open(int32_t device, uint32_t workers, int64_t idle_ns, uint32_t log_cap,
                        void** queue) {
  if (!queue || device < 0 || workers < 1 || workers > 1024 || idle_ns <= 0 ||
      log_cap > ug::kFuseLogCap)
    return UG_EINVAL;
  *queue = nullptr;
  std::unique_ptr<ug::TailQueue> q(new (std::nothrow) ug::TailQueue());
  if (!q) return UG_ENOMEM;
  const hipError_t e = q->open(device, workers, idle_ns, int64_t(60) * 1000000000, log_cap);
  if (e != hipSuccess) return e == hipErrorInvalidValue ? UG_EINVAL : UG_EDEVICE;
  *queue = q.release();
  return UG_OK;
}

ug_status ug_tails_publish(void* queue, const ug_tail* t, uint64_t key, uint32_t* slot,
                           uint64_t* pub) {
  auto* q = static_cast<ug::TailQueue*>(queue);
  if (!q || !t || !slot || !pub || !t->x || !t->y || !t->bias) return UG_EINVAL;
  if (t->rows == 0 || t->cols == 0 || t->cols % 4 || t->axis > 1 ||
      (t->sm && t->cols > ug::kFuseMaxSoftmaxRow) || (t->counter && t->counter_target == 0))
    return UG_EINVAL;
  uint64_t align = reinterpret_cast<uint64_t>(t->x) | reinterpret_cast<uint64_t>(t->y) |
                   reinterpret_cast<uint64_t>(t->sm);
  if (t->axis == 0) align |= reinterpret_cast<uint64_t>(t->bias);
  if (align & 15) return UG_EINVAL;
  ug::FuseItem it{};
  it.x = reinterpret_cast<uint64_t>(t->x);
  it.y = reinterpret_cast<uint64_t>(t->y);
  it.bias = reinterpret_cast<uint64_t>(t->bias);
  it.sm = reinterpret_cast<uint64_t>(t->sm);
  it.rs = reinterpret_cast<uint64_t>(t->rs);
  it.sig = reinterpret_cast<uint64_t>(t->counter);
  it.sig_expected = t->counter_target;
  it.R = t->rows;
  it.C = t->cols;
  it.axis = t->axis;
  it.flags = (t->sm ? ug::kFuseSoftmax : 0u) | (t->rs ? ug::kFuseRowsum : 0u);
  if (!q->reserve(slot)) return UG_EAGAIN;
  *pub = q->publish(*slot, it, key);
  return UG_OK;
}

ug_status ug_tails_set_key(void* queue, uint32_t slot, uint64_t key) {
  auto* q = static_cast<ug::TailQueue*>(queue);
  if (!q || slot >= ug::kFuseSlots) return UG_EINVAL;
  q->set_key(slot, key);
  q->commit_keys();
  return UG_OK;
}

ug_status ug_tails_pause(void* queue, int32_t on) {
  auto* q = static_cast<ug::TailQueue*>(queue);
  if (!q) return UG_EINVAL;
  q->set_pause(on != 0);
  return UG_OK;
}

ug_status ug_tails_kick(void* queue) {
  auto* q = static_cast<ug::TailQueue*>(queue);
  if (!q) return UG_EINVAL;
  return q->kick() == hipSuccess ? UG_OK : UG_EDEVICE;
}

int32_t ug_tails_finished(void* queue, uint32_t slot, uint64_t pub) {
  auto* q = static_cast<ug::TailQueue*>(queue);
  if (!q || slot >= ug::kFuseSlots) return UG_EINVAL;
  return q->finished(slot, pub) ? 1 : 0;
}

ug_status ug_tails_stats(void* queue, uint64_t* out, uint32_t n) {
  auto* q = static_cast<ug::TailQueue*>(queue);
  if (!q || (!out && n)) return UG_EINVAL;
  uint64_t st[ug::kStatCount] = {};
  if (q->stats(st) != hipSuccess) return UG_EDEVICE;
  for (uint32_t k = 0; k < n && k < static_cast<uint32_t>(ug::kStatCount); ++k) out[k] = st[k];
  return UG_OK;
}

ug_status ug_fuse_stats(void* ctx, uint64_t* out, uint32_t n) {
  Ctx* c = static_cast<Ctx*>(ctx);
  if (!c || (!out && n)) return UG_EINVAL;
  for (uint32_t k = 0; k < n && k < static_cast<uint32_t>(ug::kStatCount); ++k)
    out[k] = c->fuse_stats[k];
  return UG_OK;
}

int32_t ug_tails_log(void* queue, uint64_t* out, uint32_t cap) {
  auto* q = static_cast<ug::TailQueue*>(queue);
  if (!q || (!out && cap)) return UG_EINVAL;
  return static_cast<int32_t>(q->read_log(out, cap));
}

ug_status ug_tails_close(void* queue) {
  auto* q = static_cast<ug::TailQueue*>(queue);
  if (!q) return UG_EINVAL;
  const hipError_t e = q->halt();
  delete q;
  return e == hipSuccess ? UG_OK : UG_EDEVICE;
}

ug_status ug_kernel_launch_signal(const ug_kernel* k, void* const* buffers, uint32_t n_buffers,
                                  uint32_t* counter, uint32_t* waves, void* hip_stream) {
  if (!k || !buffers || !counter || !waves) return UG_EINVAL;
  if (ug::validate_kernel(*k, n_buffers) || ug::signal_waves(*k) == 0) return UG_EINVAL;
  const int32_t* slots[2] = {k->in, k->out};
  const int counts[2] = {3, 4};
  for (int a = 0; a < 2; ++a)
    for (int i = 0; i < counts[a]; ++i) {
      const int32_t s = slots[a][i];
      if (s >= 0 && (static_cast<uint32_t>(s) >= n_buffers || !buffers[s])) return UG_EINVAL;
    }
  *waves = ug::signal_waves(*k);
  const hipError_t e = ug::launch_kernel(*k, buffers, static_cast<hipStream_t>(hip_stream),
                                         nullptr, 0, counter);
  return e == hipSuccess ? UG_OK : UG_EDEVICE;
}

ug_status ug_graph_prepare(void* ctx, uint32_t chain, void* const* buffers, uint32_t n_buffers,
                           const int64_t* dims, uint32_t n_dims) {
  Ctx* c = static_cast<Ctx*>(ctx);
  if (!c) return UG_EINVAL;
  if (sticky(c)) return UG_EDEVICE;
  if (!c->has_device) return fail(c, UG_ENODEV, "graphs need a device");
  if (c->started) return fail(c, UG_ESTATE, "graphs are prepared before start");
  const auto& chs = c->policy.chains();
  if (chain >= chs.size() || !buffers || n_buffers != chs[chain].n_buffers)
    return fail(c, UG_EINVAL, "graph_prepare: bad chain or buffer count");
  for (uint32_t i = 0; i < n_buffers; ++i)
    if (!buffers[i]) return fail(c, UG_EINVAL, "graph_prepare: null buffer");
  const DimRange& dr = c->dim_range[chain];
  if (n_dims < dr.lo.size() || (n_dims && !dims))
    return fail(c, UG_EINVAL, "graph_prepare: the chain needs per-frame sizes");
  for (size_t d = 0; d < dr.lo.size(); ++d)
    if (dims[d] < dr.lo[d] || dims[d] > dr.hi[d])
      return fail(c, UG_EINVAL, "graph_prepare: per-frame size out of the registered range");
  (void)hipSetDevice(c->cfg.device);
  Frame fr;
  fr.chain = chain;
  fr.buffers.assign(buffers, buffers + n_buffers);
  if (n_dims) fr.dims.assign(dims, dims + n_dims);
  for (size_t j = 0; j < chs[chain].task_first.size(); ++j) {
    for (int fused = 0; fused < ((c->cfg.flags & UG_F_FUSE) ? 2 : 1); ++fused) {
      hipError_t err = hipSuccess;
      if (!task_graph(c, static_cast<int32_t>(chain), static_cast<int32_t>(j), fr, fused != 0, &err))
        return hip_fail(c, err, "graph capture");
    }
  }
  return UG_OK;
}

int32_t ug_tile_variants(int32_t op) { return ug::tile_variants(op); }

ug_status ug_tile_set(int32_t op, const int64_t* shape, int32_t variant) {
  if (!shape) return UG_EINVAL;
  return ug::tune_set(op, shape, variant) ? UG_OK : UG_EINVAL;
}

ug_status ug_tile_clear(void) {
  ug::tune_clear();
  return UG_OK;
}

int32_t ug_tile_get(const ug_kernel* k) {
  if (!k || ug::validate_kernel(*k, 16)) return UG_EINVAL;
  return ug::chosen_variant(*k);
}

ug_status ug_tile_load(const char* path, uint32_t* n_added) {
  if (!path) return UG_EINVAL;
  const int n = ug::tune_load(path);
  if (n < 0) return UG_EINVAL;
  if (n_added) *n_added = static_cast<uint32_t>(n);
  return UG_OK;
}

ug_status ug_kernel_launch_variant(const ug_kernel* k, void* const* buffers, uint32_t n_buffers,
                                   int32_t variant, void* hip_stream) {
  if (!k || !buffers || ug::validate_kernel(*k, n_buffers)) return UG_EINVAL;
  if (variant < 0 || variant >= ug::tile_variants(k->op)) return UG_EINVAL;
  const int32_t* slots[2] = {k->in, k->out};
  const int counts[2] = {3, 4};
  for (int a = 0; a < 2; ++a)
    for (int i = 0; i < counts[a]; ++i) {
      const int32_t s = slots[a][i];
      if (s >= 0 && (static_cast<uint32_t>(s) >= n_buffers || !buffers[s])) return UG_EINVAL;
    }
  const hipError_t e = ug::launch_kernel(*k, buffers, static_cast<hipStream_t>(hip_stream),
                                         nullptr, 0, nullptr, variant);
  return e == hipSuccess ? UG_OK : UG_EDEVICE;
}

ug_status ug_launch_cost(const ug_kernel* k, void* const* buffers, uint32_t n_buffers,
                         uint32_t n, void* hip_stream, int64_t* host_ns, int64_t* gpu_ns) {
  if (!k || !buffers || !host_ns || !gpu_ns || n == 0) return UG_EINVAL;
  if (ug::validate_kernel(*k, n_buffers) || ug::workspace_bytes(*k)) return UG_EINVAL;
  const int32_t* slots[2] = {k->in, k->out};
  const int counts[2] = {3, 4};
  for (int a = 0; a < 2; ++a)
    for (int i = 0; i < counts[a]; ++i) {
      const int32_t s = slots[a][i];
      if (s >= 0 && (static_cast<uint32_t>(s) >= n_buffers || !buffers[s])) return UG_EINVAL;
    }
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipSuccess;
  for (int i = 0; i < 8 && e == hipSuccess; ++i) e = ug::launch_kernel(*k, buffers, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) e = hipEventRecord(e0, st);
  const int64_t t0 = mono_ns();
  for (uint32_t i = 0; i < n && e == hipSuccess; ++i) e = ug::launch_kernel(*k, buffers, st);
  const int64_t t1 = mono_ns();
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e != hipSuccess) return UG_EDEVICE;
  *host_ns = (t1 - t0) / n;
  *gpu_ns = static_cast<int64_t>(static_cast<double>(ms) * 1e6 / n);
  return UG_OK;
}

int32_t ug_chain_tails(void* ctx, uint32_t chain, int32_t* first, int32_t* end, uint32_t cap) {
  Ctx* c = static_cast<Ctx*>(ctx);
  if (!c || chain >= c->tail_mark.size() || (cap && (!first || !end))) return UG_EINVAL;
  const std::vector<int32_t>& m = c->tail_mark[chain];
  uint32_t n = 0;
  for (size_t g = 0; g < m.size(); ++g)
    if (m[g] > static_cast<int32_t>(g)) {
      if (n < cap) {
        first[n] = static_cast<int32_t>(g);
        end[n] = m[g];
      }
      ++n;
    }
  return static_cast<int32_t>(std::min(n, cap));
}

}  // extern "C"
