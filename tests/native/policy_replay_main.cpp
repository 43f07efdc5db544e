// Host-only driver of the policy core (policy.cpp) for sanitizer builds: reads
// chains, a configuration and recorded decision instants from a text file,
// replays every instant through ug::Policy and prints the decisions, one per
// line, in the record format of include/ug.h.
//
// input:
//   cfg <policy> <bind> <delay> <batch> <calibrate> <delta> <poll> <th> <exempt>
//       <calib_period> <admit> <admit_tasks> <exit> <no_overlap> <graph> <key>
//       <noise_permille> <noise_seed> <max_hold> <cpu_cores> <cpu_prio> <nlevels>
//       <lanes...>
//   chain <deadline> <period> <ntasks>   (deadline 0: a best-effort chain)
//     task <cpu_ns> <nkernels> (<est_ns> <util> <frame_dim> <npts> (<v> <e>)*)*
//   instant <t> <narr> <nev>
//     a <chain> <frame> <t_arr> <ndims> <dims...>
//     e <chain> <frame> <task> <kind> <seq>
// output: per instant "instant <t> <ndecisions>" then one line per record:
//   <type> <chain> <frame> <task> <kernel> <a> <b> <t>
#include <cstdio>
#include <iostream>
#include <string>
#include <vector>

#include "gate/policy.hpp"

int main() {
  std::string tok;
  ug::PolicyConfig cfg;
  std::cin >> tok;
  if (tok != "cfg") return 2;
  int bind, delay, batch, cal, admit, ext, nov, graph, cprio, nlev;
  std::cin >> cfg.policy >> bind >> delay >> batch >> cal >> cfg.delta_eval_ns >>
      cfg.delay_poll_ns >> cfg.th_slack_ns >> cfg.util_exempt >> cfg.calib_period_ns >> admit >>
      cfg.admit_tasks >> ext >> nov >> graph >> cfg.order_key >> cfg.est_noise_permille >>
      cfg.noise_seed >> cfg.max_hold_ns >> cfg.cpu_cores >> cprio >> nlev;
  cfg.bind = bind, cfg.delay = delay, cfg.batch = batch, cfg.calibrate = cal, cfg.admit = admit;
  cfg.exit = ext, cfg.no_overlap = nov, cfg.graph = graph, cfg.cpu_prio = cprio;
  cfg.lanes.assign(nlev, 0);
  for (int i = 0; i < nlev; ++i) std::cin >> cfg.lanes[i];
  ug::Policy pol(cfg);
  std::vector<ug_record> out;
  bool finalized = false;
  while (std::cin >> tok) {
    if (tok == "chain") {
      ug::ChainSpec ch;
      int nt;
      std::cin >> ch.deadline_ns >> ch.period_ns >> nt;
      ch.best_effort = ch.deadline_ns == 0;
      for (int j = 0; j < nt; ++j) {
        std::string t;
        int64_t cpu;
        int nk;
        std::cin >> t >> cpu >> nk;
        ch.task_first.push_back(static_cast<int32_t>(ch.est.size()));
        for (int k = 0; k < nk; ++k) {
          int64_t e;
          float u;
          int fd, np;
          std::cin >> e >> u >> fd >> np;
          ch.est.push_back(e);
          ch.util.push_back(u);
          ch.kernels.push_back(ug_kernel{});
          ch.fdim.push_back(fd);
          std::vector<std::pair<int64_t, int64_t>> pts(np);
          for (auto& p : pts) std::cin >> p.first >> p.second;
          ch.prof.push_back(pts);
        }
        ch.task_end.push_back(static_cast<int32_t>(ch.est.size()));
        ch.cpu.push_back(cpu);
      }
      pol.add_chain(std::move(ch));
    } else if (tok == "instant") {
      if (!finalized) {
        pol.reset();
        finalized = true;
      }
      int64_t t;
      int na, ne;
      std::cin >> t >> na >> ne;
      std::vector<ug::Arrival> arr(na);
      std::vector<ug::EvDone> ev(ne);
      for (auto& a : arr) {
        int nd;
        std::cin >> tok >> a.c >> a.f >> a.t_arr >> nd;
        a.dims.resize(nd);
        for (auto& d : a.dims) std::cin >> d;
      }
      for (auto& e : ev) std::cin >> tok >> e.c >> e.f >> e.task >> e.kind >> e.seq;
      out.clear();
      const char* err = nullptr;
      if (!pol.instant(t, arr, ev, out, &err)) {
        std::printf("error %s\n", err ? err : "?");
        return 1;
      }
      pol.finished().clear();
      std::printf("instant %lld %zu\n", static_cast<long long>(t), out.size());
      for (const auto& r : out)
        std::printf("%d %d %lld %d %d %d %d %lld\n", r.type, r.chain, static_cast<long long>(r.frame),
                    r.task, r.kernel, r.a, r.b, static_cast<long long>(r.t));
    }
  }
  std::printf("samples %zu\n", pol.samples().size());
  return 0;
}
