// The gate under ThreadSanitizer: the real runtime (gate thread, queues,
// policy, stream pool, graphs, tiles table) built for the host against the
// HIP stand-in in hip_stub/, driven by a caller thread that submits frames,
// a thread that polls completions and reads statistics and errors, and a
// thread that makes failing calls (so the error messages are written from
// several threads at once).  Exits 0 when every submitted frame completed
// once; ThreadSanitizer reports any data race on stderr (and the test
// treats any report as a failure).
#include <atomic>
#include <chrono>
#include <cstdio>
#include <thread>
#include <vector>

#include "ug.h"

static ug_kernel gemm(int a, int b, int c) {
  ug_kernel k{};
  k.op = UG_OP_GEMM_F32;
  for (int i = 0; i < 3; ++i) k.in[i] = -1;
  for (int i = 0; i < 4; ++i) k.out[i] = -1;
  k.in[0] = a;
  k.in[1] = b;
  k.out[0] = c;
  k.shape[0] = k.shape[1] = k.shape[2] = 64;
  k.est_ns = 30000;
  k.util = 0.5f;
  return k;
}

static ug_kernel bias_relu(int x, int b) {
  ug_kernel k{};
  k.op = UG_OP_BIAS_RELU_F32;
  for (int i = 0; i < 3; ++i) k.in[i] = -1;
  for (int i = 0; i < 4; ++i) k.out[i] = -1;
  k.in[0] = x;
  k.in[1] = b;
  k.out[0] = x;
  k.shape[0] = k.shape[1] = 64;
  k.est_ns = 5000;
  k.util = 0.05f;
  return k;
}

int main(int argc, char** argv) {
  const bool graphs = argc > 1 && argv[1][0] == 'g';
  ug_config cfg;
  ug_config_default(&cfg);
  cfg.own_streams = 1;
  cfg.th_slack_ns = 2000000;
  cfg.trace_capacity = 1 << 16;
  cfg.delay_poll_ns = 200000;
  if (graphs) cfg.flags |= UG_F_GRAPH;
  void* ctx = nullptr;
  if (ug_create(&cfg, &ctx) != UG_OK) return 2;
  const int n_chains = 4, n_frames = 60;
  std::vector<float> buf(64 * 64 * 4);
  void* ptrs[4] = {buf.data(), buf.data() + 4096, buf.data() + 8192, buf.data() + 12288};
  for (int c = 0; c < n_chains; ++c) {
    ug_kernel t0[3] = {gemm(0, 1, 2), bias_relu(2, 3), gemm(2, 1, 0)};
    ug_kernel t1[2] = {gemm(0, 1, 2), bias_relu(2, 3)};
    ug_task tasks[2] = {{t0, 3, 0, 100000}, {t1, 2, 0, 0}};
    uint32_t id = 0;
    if (ug_chain_register(ctx, 5000000 * (c + 1), 4000000 * (c + 1), tasks, 2, 4, &id) != UG_OK)
      return 3;
  }
  if (ug_start(ctx) != UG_OK) return 4;
  std::atomic<bool> done{false};
  std::atomic<long> completed{0};
  std::thread poller([&] {
    ug_completion out[64];
    ug_stats st;
    while (!done.load()) {
      const int32_t n = ug_poll_complete(ctx, out, 64);
      if (n > 0) completed += n;
      (void)ug_get_stats(ctx, &st);
      (void)ug_last_error(ctx);
      std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
    int32_t n;
    while ((n = ug_poll_complete(ctx, out, 64)) > 0) completed += n;
  });
  std::thread failer([&] {
    void* bad[4] = {nullptr, nullptr, nullptr, nullptr};
    while (!done.load()) {
      uint64_t f;
      (void)ug_frame_submit(ctx, 99, -1, ptrs, 4, &f);    // no such chain
      (void)ug_frame_submit(ctx, 0, -1, bad, 4, &f);      // null buffer
      (void)ug_last_error(ctx);
      std::this_thread::sleep_for(std::chrono::microseconds(30));
    }
  });
  long submitted = 0;
  for (int f = 0; f < n_frames; ++f) {
    for (int c = 0; c < n_chains; ++c) {
      uint64_t id;
      while (ug_frame_submit(ctx, c, -1, ptrs, 4, &id) == UG_EAGAIN)
        std::this_thread::sleep_for(std::chrono::microseconds(100));
      ++submitted;
    }
    std::this_thread::sleep_for(std::chrono::microseconds(500));
  }
  const ug_status dr = ug_drain(ctx, 30000000000LL);
  done.store(true);
  poller.join();
  failer.join();
  (void)ug_stop(ctx);
  ug_record recs[256];
  while (ug_trace_read(ctx, recs, 256) > 0) {
  }
  ug_destroy(ctx);
  std::printf("submitted %ld completed %ld drain %d\n", submitted, completed.load(), dr);
  return dr == UG_OK && completed.load() == submitted ? 0 : 1;
}
