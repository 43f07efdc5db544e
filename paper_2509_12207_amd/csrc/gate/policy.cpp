// Urgency-ordered launch policy: see policy.hpp for the per-instant order.
#include "policy.hpp"

#include <algorithm>

namespace ug {

// ---------------------------------------------------------------- Eq. (2)
bool ul_greater(int64_t s1, int64_t s2) {
  // best-effort instances have no urgency: below every deadline instance
  if (s1 == kBestEffortSlack) return false;
  if (s2 == kBestEffortSlack) return true;
  // 1/0 is +infinity: above every finite level, not above itself.
  if (s1 == 0) return s2 != 0;
  if (s2 == 0) return false;
  // 1/s1 - 1/s2 = (s2 - s1) / (s1 s2): positive iff the numerator and the
  // product have the same sign.  The numerator is formed in 128 bits.
  __int128 num = static_cast<__int128>(s2) - static_cast<__int128>(s1);
  if (num == 0) return false;
  bool prod_pos = (s1 > 0) == (s2 > 0);
  return (num > 0) == prod_pos;
}

uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

int32_t noise_permille(uint64_t seed, int32_t c, int64_t f, int32_t j, int32_t n) {
  const uint64_t h = splitmix64(splitmix64(splitmix64(seed ^ static_cast<uint64_t>(c)) ^
                                           static_cast<uint64_t>(f)) ^
                                static_cast<uint64_t>(j));
  return static_cast<int32_t>(h % static_cast<uint64_t>(2 * n + 1)) - n;
}

bool more_urgent(int64_t s1, const Key& k1, int64_t s2, const Key& k2) {
  if (ul_greater(s1, s2)) return true;
  if (ul_greater(s2, s1)) return false;
  return k1 < k2;
}

// ---------------------------------------------------------------- chains
void ChainSpec::finalize() {
  const size_t n = est.size();
  gpu_rem.assign(n + 1, 0);
  for (size_t g = n; g-- > 0;) gpu_rem[g] = gpu_rem[g + 1] + est[g];
  const size_t m = cpu.size();
  cpu_rem.assign(m + 1, 0);
  for (size_t j = m; j-- > 0;) cpu_rem[j] = cpu_rem[j + 1] + cpu[j];
  fdim.resize(n, 0);
  prof.resize(n);
  per_frame = false;
  for (size_t g = 0; g < n; ++g)
    if (fdim[g] > 0 && !prof[g].empty()) per_frame = true;
}

static int64_t floor_div(__int128 a, int64_t b) {
  __int128 q = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
  return static_cast<int64_t>(q);
}

int64_t profile_estimate(const std::vector<std::pair<int64_t, int64_t>>& p, int64_t v) {
  if (v <= p.front().first) return p.front().second;
  if (v >= p.back().first) return p.back().second;
  size_t i = 0;
  while (p[i + 1].first <= v) ++i;
  const int64_t v0 = p[i].first, v1 = p[i + 1].first;
  const int64_t e0 = p[i].second, e1 = p[i + 1].second;
  return e0 + floor_div(static_cast<__int128>(e1 - e0) * (v - v0), v1 - v0);
}

uint32_t Policy::add_chain(ChainSpec&& spec) {
  spec.finalize();
  const int32_t c = static_cast<int32_t>(chains_.size());
  fifo_base_.push_back(fifo_total_);
  fifo_total_ += static_cast<int32_t>(spec.task_first.size());
  for (int32_t j = 0; j < static_cast<int32_t>(spec.task_first.size()); ++j) {
    slot_[{c, j}] = -1;
    queue_[{c, j}];
  }
  chains_.push_back(std::move(spec));
  return static_cast<uint32_t>(c);
}

void Policy::finalize() {
  for (auto& ch : chains_) ch.finalize();
  lane_load_.clear();
  for (int32_t lv = 0; lv < static_cast<int32_t>(cfg_.lanes.size()); ++lv)
    for (int32_t ln = 0; ln < cfg_.lanes[lv]; ++ln) lane_load_[{lv, ln}] = 0;
}

void Policy::reset() {
  inst_.clear();
  for (auto& s : slot_) s.second = -1;
  for (auto& q : queue_) q.second.clear();
  finished_.clear();
  samples_.clear();
  sampled_ = false;
  next_sample_ = 0;
  collisions_ = 0;
  collision_hist_.fill(0);
  finalize();
}

bool Policy::urgent(int64_t slack) const {
  // UL > TH_urgent with TH = 1/th_slack; th_slack <= 0 is TH = +infinity.
  if (cfg_.th_slack_ns <= 0) return false;
  return ul_greater(slack, cfg_.th_slack_ns);
}

static ug_record rec(int32_t type, int32_t c, int64_t f, int32_t task,
                     int32_t kernel, int32_t a, int32_t b, int64_t t) {
  ug_record r;
  r.type = type;
  r.chain = c;
  r.frame = f;
  r.task = task;
  r.kernel = kernel;
  r.a = a;
  r.b = b;
  r.t = t;
  return r;
}

void Policy::start_task(Instance& in, int32_t j, int64_t t, std::vector<ug_record>& out) {
  const ChainSpec& ch = chains_[in.c];
  in.task = j;
  in.task_t0 = t;
  in.phase = kCpu;
  in.cpu_ready = t + ch.cpu[j];
  in.cpu_left = ch.cpu[j];
  in.cpu_req = t;
  in.cpu_run = false;
  in.cpu_since = 0;
  in.g_next = ch.task_first[j];
  in.released_hi = ch.task_first[j];
  in.batch = 0;
  in.batch_open = false;
  in.batch_sum = 0;
  in.batch_first.clear();
  in.waits.clear();
  in.bound = false;
  in.level = in.lane = -1;
  in.has_wake = false;
  in.has_held = false;
  in.has_expire = false;
  slot_[{in.c, j}] = in.f;
  out.push_back(rec(UG_REC_TSTART, in.c, in.f, j, 0, 0, 0, 0));
}

// ------------------------------------------------------------ one instant
bool Policy::instant(int64_t t, std::vector<Arrival>& arrivals,
                     std::vector<EvDone>& evdones, std::vector<ug_record>& out,
                     const char** err) {
  now_ = t;
  const size_t out0 = out.size();
  // 1. inputs in canonical order
  std::sort(arrivals.begin(), arrivals.end(), [](const Arrival& a, const Arrival& b) {
    return a.c != b.c ? a.c < b.c : a.f < b.f;
  });
  for (const Arrival& a : arrivals) {
    if (a.c < 0 || a.c >= static_cast<int32_t>(chains_.size()) || inst_.count({a.c, a.f})) {
      *err = "arrival of an unknown chain or a frame seen before";
      return false;
    }
    Instance in;
    in.c = a.c;
    in.f = a.f;
    in.t_arr = a.t_arr;
    const ChainSpec& ch = chains_[a.c];
    if (ch.per_frame) {
      // this frame's estimates: a kernel with profile points takes the
      // estimate of the frame's size, the others their fixed one
      const size_t n = ch.est.size();
      in.est = ch.est;
      for (size_t g = 0; g < n; ++g) {
        if (ch.fdim[g] <= 0 || ch.prof[g].empty()) continue;
        const size_t d = static_cast<size_t>(ch.fdim[g] - 1);
        if (d >= a.dims.size()) {
          *err = "arrival without the frame's sizes";
          return false;
        }
        in.est[g] = profile_estimate(ch.prof[g], a.dims[d]);
      }
      in.gpu_rem.assign(n + 1, 0);
      for (size_t g = n; g-- > 0;) in.gpu_rem[g] = in.gpu_rem[g + 1] + in.est[g];
    }
    inst_.emplace(Key{a.c, a.f}, std::move(in));
    queue_[{a.c, 0}].push_back(a.f);
  }
  std::sort(evdones.begin(), evdones.end(), [](const EvDone& a, const EvDone& b) {
    if (a.c != b.c) return a.c < b.c;
    if (a.f != b.f) return a.f < b.f;
    if (a.task != b.task) return a.task < b.task;
    if (a.seq != b.seq) return a.seq < b.seq;
    return a.kind < b.kind;
  });
  std::vector<Key> completed;
  for (const EvDone& e : evdones) {
    auto it = inst_.find({e.c, e.f});
    if (it == inst_.end()) {
      *err = "event of an unknown frame";
      return false;
    }
    Instance& in = it->second;
    if (in.task != e.task || in.waits.empty() || !(in.waits.front() == Wait{e.kind, e.seq})) {
      *err = "event the instance is not waiting for";
      return false;
    }
    in.waits.pop_front();
    const ChainSpec& ch = chains_[e.c];
    if (e.kind == 0) {
      // batch e.seq has started on the device: all earlier batches are done
      in.i_gpu = in.batch_first[e.seq];
    } else {
      in.i_gpu = ch.task_end[e.task];
      if (in.bound && cfg_.policy == UG_POLICY_URGENCY) lane_load_[{in.level, in.lane}] -= 1;
      slot_[{e.c, e.task}] = -1;
      if (e.task + 1 == static_cast<int32_t>(ch.task_first.size())) {
        in.phase = kDone;
        completed.push_back({e.c, e.f});
      } else {
        in.phase = kWait;
        queue_[{e.c, e.task + 1}].push_back(e.f);
      }
    }
  }
  for (const Key& k : completed) {  // already in (chain, frame) order
    Instance& in = inst_.at(k);
    out.push_back(rec(UG_REC_COMPLETE, in.c, in.f, 0, 0, 0, 0, t));
    finished_.push_back({in.c, in.f, in.t_arr, t, in.n_holds, in.n_batches});
    inst_.erase(k);
  }
  // 2. task starts, in (chain, task) order.  With early exit, a frame whose
  //    urgency is negative (slack < 0) when its task would start leaves the
  //    chain instead (Sec. 4.3)
  const bool exiting = cfg_.policy == UG_POLICY_URGENCY && cfg_.exit;
  for (int32_t c = 0; c < static_cast<int32_t>(chains_.size()); ++c) {
    const ChainSpec& ch = chains_[c];
    const int32_t nt = static_cast<int32_t>(ch.task_first.size());
    for (int32_t j = 0; j < nt; ++j) {
      auto& q = queue_[{c, j}];
      while (slot_[{c, j}] < 0 && !q.empty()) {
        int64_t f = q.front();
        q.pop_front();
        Instance& in = inst_.at({c, f});
        if (exiting && !ch.best_effort &&
            in.t_arr + ch.deadline_ns - remaining(in) - t < 0) {
          out.push_back(rec(UG_REC_EXIT, c, f, j, 0, 0, 0, t));
          finished_.push_back({c, f, in.t_arr, t, in.n_holds, in.n_batches, true});
          inst_.erase({c, f});
          continue;
        }
        start_task(in, j, t, out);
      }
    }
  }
  // 3. finished CPU segments
  std::vector<Instance*> active;
  active.reserve(inst_.size());
  for (auto& kv : inst_) {
    Instance& in = kv.second;
    if (cfg_.cpu_cores <= 0 && in.phase == kCpu && in.cpu_ready <= t) {
      in.phase = kLaunch;
      in.i_cpu = in.task + 1;
    }
    active.push_back(&in);
  }
  if (cfg_.cpu_cores > 0) {
    bool started = false;
    for (size_t i = out0; i < out.size(); ++i) started |= out[i].type == UG_REC_TSTART;
    cpu_cores(t, active, started, out);
  }
  // 4. urgency snapshot: slack = t_arr + D - sum E^gpu - sum E^cpu - t
  std::map<Key, int64_t> slack;
  for (Instance* in : active) {
    const ChainSpec& ch = chains_[in->c];
    slack[{in->c, in->f}] =
        ch.best_effort
            ? kBestEffortSlack
            : in->t_arr + ch.deadline_ns - remaining(*in) - t;
  }
  // the whole ranking, when asked for (the fused-tail queue's keys): every
  // active instance, most urgent first
  if (cfg_.keep_order) {
    std::vector<Instance*> order(active);
    if (cfg_.policy == UG_POLICY_URGENCY)
      std::sort(order.begin(), order.end(),
                [&](const Instance* a, const Instance* b) { return before(*a, *b, slack); });
    order_.clear();
    for (const Instance* in : order) order_.push_back({in->c, in->f});
  }
  // 5. highest urgency among active kernels, for TH_urgent calibration,
  //    sampled periodically: at the first instant at or after each sampling
  //    time
  if (cfg_.calibrate && (!sampled_ || t >= next_sample_)) {
    const Instance* top = nullptr;
    for (Instance* in : active) {
      if (!in->in_flight() || chains_[in->c].best_effort) continue;
      if (!top || more_urgent(slack[{in->c, in->f}], {in->c, in->f},
                              slack[{top->c, top->f}], {top->c, top->f}))
        top = in;
    }
    if (top) {
      samples_.push_back(slack[{top->c, top->f}]);
      sampled_ = true;
      next_sample_ = t + cfg_.calib_period_ns;
    }
  }
  // instances with launched, unconfirmed kernels (the AKB's entries)
  active_ = 0;
  for (Instance* in : active)
    if (in->in_flight()) ++active_;
  // 6. launch requests, most urgent first
  std::vector<Instance*> ready;
  for (Instance* in : active) {
    if (in->phase != kLaunch) continue;
    if (in->g_next >= chains_[in->c].task_end[in->task]) continue;
    if (!in->waits.empty()) continue;
    if (in->has_wake && in->wake > t && !(in->has_expire && in->expire <= t)) continue;
    ready.push_back(in);
  }
  if (cfg_.policy == UG_POLICY_URGENCY) {
    std::sort(ready.begin(), ready.end(), [&](const Instance* a, const Instance* b) {
      return before(*a, *b, slack);
    });
  }
  for (Instance* in : ready) release(*in, t, active, slack, out);
  return true;
}

void Policy::cpu_cores(int64_t t, const std::vector<Instance*>& active, bool started,
                       std::vector<ug_record>& out) {
  // CPU segments on cfg_.cpu_cores cores.  Segments that held a core since
  // the last instant are credited the time in between; those with no work
  // left finish (the task may launch).  Without urgency-centric scheduling
  // the cores serve segments first come, first served, each to its end.
  // With it (Sec. 4.3), a chain starting a new CPU segment ranks every active
  // instance by urgency (rank 1 the most urgent), and the cores run the
  // segments of the best ranks, preempting worse ones (fixed priorities,
  // ties in (chain, frame) order).
  std::vector<Instance*> waiting;
  for (Instance* in : active) {
    if (in->phase != kCpu) continue;
    if (in->cpu_run) {
      in->cpu_left = std::max<int64_t>(0, in->cpu_left - (t - in->cpu_since));
      in->cpu_since = t;
    }
    if (in->cpu_left == 0) {
      in->phase = kLaunch;
      in->i_cpu = in->task + 1;
      in->cpu_run = false;
    } else {
      waiting.push_back(in);
    }
  }
  const bool prio = cfg_.policy == UG_POLICY_URGENCY && cfg_.cpu_prio;
  if (prio && started) {
    std::map<Key, int64_t> slack;
    for (Instance* in : active) {
      const ChainSpec& ch = chains_[in->c];
      slack[{in->c, in->f}] = ch.best_effort ? kBestEffortSlack
                                             : in->t_arr + ch.deadline_ns - remaining(*in) - t;
    }
    std::vector<Instance*> order(active);
    std::sort(order.begin(), order.end(),
              [&](const Instance* a, const Instance* b) { return before(*a, *b, slack); });
    for (size_t r = 0; r < order.size(); ++r) order[r]->cpu_prio = static_cast<int32_t>(r + 1);
  }
  const size_t k = static_cast<size_t>(cfg_.cpu_cores);
  std::vector<Instance*> want;
  if (prio) {
    want = waiting;
    std::sort(want.begin(), want.end(), [](const Instance* a, const Instance* b) {
      return a->cpu_prio != b->cpu_prio ? a->cpu_prio < b->cpu_prio
                                        : Key{a->c, a->f} < Key{b->c, b->f};
    });
    if (want.size() > k) want.resize(k);
  } else {
    std::vector<Instance*> queued;
    for (Instance* in : waiting) (in->cpu_run ? want : queued).push_back(in);
    std::sort(queued.begin(), queued.end(), [](const Instance* a, const Instance* b) {
      return a->cpu_req != b->cpu_req ? a->cpu_req < b->cpu_req
                                      : Key{a->c, a->f} < Key{b->c, b->f};
    });
    for (Instance* in : queued)
      if (want.size() < k) want.push_back(in);
  }
  auto chosen = [&](const Instance* in) {
    return std::find(want.begin(), want.end(), in) != want.end();
  };
  for (Instance* in : waiting) {
    if (in->cpu_run && !chosen(in)) {
      in->cpu_run = false;
      out.push_back(rec(UG_REC_CPU, in->c, in->f, in->task, 0, 0, 0, 0));
    }
  }
  std::sort(want.begin(), want.end(), [](const Instance* a, const Instance* b) {
    return Key{a->c, a->f} < Key{b->c, b->f};
  });
  for (Instance* in : want) {
    if (!in->cpu_run) {
      in->cpu_run = true;
      in->cpu_since = t;
      out.push_back(rec(UG_REC_CPU, in->c, in->f, in->task, 0, 1, 0, 0));
    }
  }
}

int64_t Policy::remaining(const Instance& in) const {
  const ChainSpec& ch = chains_[in.c];
  const int32_t n = cfg_.est_noise_permille;
  const std::vector<int64_t>& rem = in.gpu_rem.empty() ? ch.gpu_rem : in.gpu_rem;
  if (n <= 0) return rem[in.i_gpu] + ch.cpu_rem[in.i_cpu];
  int64_t gpu = 0, cpu = 0;
  const int32_t nt = static_cast<int32_t>(ch.task_first.size());
  for (int32_t j = 0; j < nt; ++j) {
    const int64_t fac = 1000 + noise_permille(cfg_.noise_seed, in.c, in.f, j, n);
    const int32_t lo = std::max(in.i_gpu, ch.task_first[j]);
    if (lo < ch.task_end[j]) gpu += (rem[lo] - rem[ch.task_end[j]]) * fac / 1000;
    if (j >= in.i_cpu) cpu += ch.cpu[j] * fac / 1000;
  }
  return gpu + cpu;
}

bool Policy::before(const Instance& a, const Instance& b,
                    const std::map<Key, int64_t>& slack) const {
  if (cfg_.order_key == UG_KEY_URGENCY)
    return more_urgent(slack.at({a.c, a.f}), {a.c, a.f}, slack.at({b.c, b.f}), {b.c, b.f});
  const ChainSpec& ca = chains_[a.c];
  const ChainSpec& cb = chains_[b.c];
  if (ca.best_effort != cb.best_effort) return cb.best_effort;
  if (!ca.best_effort) {
    int cmp = 0;  // < 0: a first
    const int64_t ra = remaining(a);
    const int64_t rb = remaining(b);
    auto sign = [](__int128 x, __int128 y) { return x < y ? -1 : (x > y ? 1 : 0); };
    switch (cfg_.order_key) {
      case UG_KEY_EDF:
        cmp = sign(a.t_arr + ca.deadline_ns, b.t_arr + cb.deadline_ns);
        break;
      case UG_KEY_SJF:
        cmp = sign(ra, rb);
        break;
      case UG_KEY_HRRN:
        // (w_a + R_a) / R_a > (w_b + R_b) / R_b, cross-multiplied; R = 0 first
        if (ra == 0 || rb == 0)
          cmp = (ra == 0) == (rb == 0) ? 0 : (ra == 0 ? -1 : 1);
        else
          cmp = -sign(static_cast<__int128>(now_ - a.t_arr + ra) * rb,
                      static_cast<__int128>(now_ - b.t_arr + rb) * ra);
        break;
      case UG_KEY_SAEDF:
      case UG_KEY_EQDF: {
        // earliest deadline of the current task: t_ref + w + num / den
        // for each side, compared as (base * den + num) / den cross-multiplied
        __int128 base_a, num_a, den_a, base_b, num_b, den_b;
        subtask_deadline(a, &base_a, &num_a, &den_a);
        subtask_deadline(b, &base_b, &num_b, &den_b);
        cmp = sign((base_a * den_a + num_a) * den_b, (base_b * den_b + num_b) * den_a);
        break;
      }
      case UG_KEY_LCUF: {
        // E_a / P_a < E_b / P_b, cross-multiplied; P = 0 last
        const int64_t pa = ca.period_ns, pb = cb.period_ns;
        if (pa <= 0 || pb <= 0)
          cmp = (pa <= 0) == (pb <= 0) ? 0 : (pa <= 0 ? 1 : -1);
        else
          cmp = sign(static_cast<__int128>(ca.gpu_rem[0] + ca.cpu_rem[0]) * pb,
                     static_cast<__int128>(cb.gpu_rem[0] + cb.cpu_rem[0]) * pa);
        break;
      }
      default:
        break;
    }
    if (cmp) return cmp < 0;
  }
  return Key{a.c, a.f} < Key{b.c, b.f};
}

void Policy::subtask_deadline(const Instance& in, __int128* base, __int128* num,
                              __int128* den) const {
  // The chain's remaining slack S = t_arr + D - t_ref - w_rem split over its
  // remaining tasks: SAEDF gives the current task S / m (equal slack), EQDF
  // S * w / w_rem (equal flexibility; all of S when w_rem = 0).  The current
  // task is the one that has started (from its start), else the next one
  // (from now).  Estimates: the profiled ones (the frame's own with
  // per-frame sizes), without estimate noise.
  const ChainSpec& ch = chains_[in.c];
  const std::vector<int64_t>& rem = in.gpu_rem.empty() ? ch.gpu_rem : in.gpu_rem;
  int32_t j;
  int64_t t_ref;
  if (in.phase == kCpu || in.phase == kLaunch) {
    j = in.task;
    t_ref = in.task_t0;
  } else {
    j = in.task + 1;
    t_ref = now_;
  }
  const int64_t w = ch.cpu[j] + rem[ch.task_first[j]] - rem[ch.task_end[j]];
  const int64_t w_rem = ch.cpu_rem[j] + rem[ch.task_first[j]];
  const int64_t m = static_cast<int64_t>(ch.task_first.size()) - j;
  const __int128 s = static_cast<__int128>(in.t_arr) + ch.deadline_ns - t_ref - w_rem;
  *base = static_cast<__int128>(t_ref) + w;
  if (cfg_.order_key == UG_KEY_SAEDF) {
    *num = s;
    *den = m;
  } else if (w_rem == 0) {
    *num = s;
    *den = 1;
  } else {
    *num = s * w;
    *den = w_rem;
  }
}

bool Policy::blocked(const Instance& me, const std::vector<Instance*>& active,
                     const std::map<Key, int64_t>& slack) const {
  // Delayed launching: another chain has an active kernel that is truly
  // urgent and ranks before this one.
  for (const Instance* o : active) {
    if (o->c == me.c || !o->in_flight()) continue;
    const int64_t so = slack.at({o->c, o->f});
    if (urgent(so) && before(*o, me, slack)) return true;
  }
  return false;
}

void Policy::bind(Instance& me, const std::vector<Instance*>& active,
                  const std::map<Key, int64_t>& slack, std::vector<ug_record>& out) {
  if (cfg_.policy != UG_POLICY_URGENCY) {
    me.level = 0;
    me.lane = fifo_lane(me.c, me.task);
  } else {
    const int32_t n_levels = static_cast<int32_t>(cfg_.lanes.size());
    const int64_t sm = slack.at({me.c, me.f});
    int32_t level;
    if (!cfg_.bind) {
      level = std::min<int32_t>(1, n_levels - 1);
    } else if (n_levels <= 1) {
      level = 0;
    } else if (urgent(sm)) {
      level = 0;  // reserved for truly urgent tasks
    } else {
      // rank among active, not truly urgent instances (and this one)
      int32_t rank = 1, n = 1;
      for (const Instance* o : active) {
        if (o == &me || !o->in_flight()) continue;
        const int64_t so = slack.at({o->c, o->f});
        if (urgent(so)) continue;
        ++n;
        if (before(*o, me, slack)) ++rank;
      }
      level = 1 + static_cast<int32_t>((static_cast<int64_t>(rank - 1) * (n_levels - 1)) / n);
    }
    int32_t best = 0;
    for (int32_t ln = 1; ln < cfg_.lanes[level]; ++ln)
      if (lane_load_[{level, ln}] < lane_load_[{level, best}]) best = ln;
    lane_load_[{level, best}] += 1;
    me.level = level;
    me.lane = best;
  }
  me.bound = true;
  out.push_back(rec(UG_REC_BIND, me.c, me.f, me.task, 0, me.level, me.lane, 0));
}

void Policy::release(Instance& me, int64_t t, const std::vector<Instance*>& active,
                     const std::map<Key, int64_t>& slack, std::vector<ug_record>& out) {
  const ChainSpec& ch = chains_[me.c];
  const int32_t end = ch.task_end[me.task];
  const bool gated = cfg_.policy == UG_POLICY_URGENCY;
  const bool graph = gated && cfg_.graph;
  const bool batching = gated && cfg_.batch && !graph;
  // a hold of the task at t: the first one starts the hold age; while the
  // task waits, a timer fires when the age reaches the bound (best-effort
  // tasks have no deadline to protect and no bound)
  auto held = [&]() {
    if (cfg_.max_hold_ns <= 0 || ch.best_effort) return;
    if (!me.has_held) {
      me.has_held = true;
      me.held_since = t;
    }
    me.has_expire = true;
    me.expire = me.held_since + cfg_.max_hold_ns;
  };
  while (me.g_next < end && me.waits.empty()) {
    const int32_t g = me.g_next;
    // hold-age bound: once the task has waited max_hold_ns since its first
    // hold, neither delayed launching nor admission holds it again
    const bool aged = cfg_.max_hold_ns > 0 && !ch.best_effort && me.has_held &&
                      t >= me.held_since + cfg_.max_hold_ns;
    // with task graphs the task is one launch: it is gated at its first
    // kernel, with the largest utilisation of its kernels
    const bool gate_here = !graph || g == ch.task_first[me.task];
    float u = ch.util[g];
    if (graph && gate_here)
      for (int32_t k = g; k < end; ++k) u = std::max(u, ch.util[k]);
    if (gated && cfg_.delay && gate_here && !aged && (ch.best_effort || u >= cfg_.util_exempt) &&
        blocked(me, active, slack)) {
      out.push_back(rec(UG_REC_HOLD, me.c, me.f, me.task, g, 0, 0, 0));
      me.n_holds += 1;
      if (cfg_.delay_poll_ns > 0) {
        me.has_wake = true;
        me.wake = t + cfg_.delay_poll_ns;
      } else {
        me.has_wake = false;
      }
      held();
      return;
    }
    // admission: a task that is not truly urgent starts only while fewer
    // than admit_tasks instances have kernels in flight; waiting tasks are
    // re-checked at every instant, most urgent first
    if (gated && cfg_.admit && !me.bound && !aged && active_ >= cfg_.admit_tasks &&
        !urgent(slack.at({me.c, me.f}))) {
      out.push_back(rec(UG_REC_HOLD, me.c, me.f, me.task, g, 1, 0, 0));
      me.n_holds += 1;
      me.has_wake = false;
      held();
      return;
    }
    if (!me.bound && !me.in_flight()) ++active_;
    me.has_wake = false;
    me.has_expire = false;
    if (!me.bound) bind(me, active, slack, out);
    if (!me.batch_open) {
      me.batch_open = true;
      me.batch_first.push_back(g);
      me.n_batches += 1;
      out.push_back(rec(UG_REC_EVREC, me.c, me.f, me.task, 0, 0, me.batch, 0));
    }
    if (gated && urgent(slack.at({me.c, me.f}))) {
      // a collision, and how many other chains' instances it met
      size_t others = 0;
      for (const Instance* o : active)
        if (o->c != me.c && o->in_flight()) ++others;
      if (others) {
        ++collisions_;
        ++collision_hist_[std::min<size_t>(others, kCollisionBins) - 1];
      }
    }
    out.push_back(rec(UG_REC_LAUNCH, me.c, me.f, me.task, g, me.level, me.lane, 0));
    me.released_hi = g + 1;
    me.g_next = g + 1;
    me.batch_sum += me.est.empty() ? ch.est[g] : me.est[g];
    const bool last = g == end - 1;
    // a best-effort kernel is a batch of its own, so the gate decides again
    // before each one
    if (last || (batching && (ch.best_effort || me.batch_sum > cfg_.delta_eval_ns))) {
      // the start event of a batch opened ahead (no overlap) has already
      // been waited for, before its first kernel was released
      if (!(gated && cfg_.no_overlap && me.batch > 0)) me.waits.push_back({0, me.batch});
      if (last) {
        out.push_back(rec(UG_REC_EVREC, me.c, me.f, me.task, 0, 1, me.batch + 1, 0));
        me.waits.push_back({1, me.batch + 1});
      }
      me.batch += 1;
      me.batch_open = false;
      me.batch_sum = 0;
      if (!last && gated && cfg_.no_overlap) {
        // no overlap: the next batch's start event is recorded now, right
        // after this batch's last kernel, and waited for as well, so the
        // next batch is launched only once this one has finished
        me.batch_open = true;
        me.batch_first.push_back(g + 1);
        me.n_batches += 1;
        out.push_back(rec(UG_REC_EVREC, me.c, me.f, me.task, 0, 0, me.batch, 0));
        me.waits.push_back({0, me.batch});
      }
    }
  }
}

bool Policy::next_timer(int64_t* t) const {
  bool any = false;
  int64_t best = 0;
  for (const auto& kv : inst_) {
    const Instance& in = kv.second;
    if (in.phase == kCpu && cfg_.cpu_cores <= 0 && (!any || in.cpu_ready < best)) {
      best = in.cpu_ready;
      any = true;
    }
    if (in.phase == kCpu && cfg_.cpu_cores > 0 && in.cpu_run &&
        (!any || in.cpu_since + in.cpu_left < best)) {
      best = in.cpu_since + in.cpu_left;
      any = true;
    }
    if (in.phase == kLaunch && in.has_wake && (!any || in.wake < best)) {
      best = in.wake;
      any = true;
    }
    if (in.phase == kLaunch && in.has_expire && (!any || in.expire < best)) {
      best = in.expire;
      any = true;
    }
  }
  if (any) *t = best;
  return any;
}

}  // namespace ug
