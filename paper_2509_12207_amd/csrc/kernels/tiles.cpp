// Tile-variant table: the tile shape each (operation, shape) launches with,
// as an autotuner measured it.  Set before launches, read on every launch
// without a lock: a table is never changed once published; a change
// publishes a new copy (the old ones stay until the process ends, a few
// entries each).
#include <atomic>
#include <cstdio>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "ops.hpp"

namespace ug {
namespace {

using TileKey = std::tuple<int32_t, int64_t, int64_t, int64_t, int64_t>;
using Table = std::map<TileKey, int>;

std::mutex g_mu;                         // writers
std::vector<const Table*> g_all;         // every table published (kept)
std::atomic<const Table*> g_table{nullptr};

TileKey key_of(int32_t op, const int64_t* s) { return TileKey{op, s[0], s[1], s[2], s[3]}; }

void publish(Table&& t) {
  const Table* p = new Table(std::move(t));
  g_all.push_back(p);
  g_table.store(p, std::memory_order_release);
}

}  // namespace

int tile_variants(int32_t op) {
  switch (op) {
    case UG_OP_GEMM_F32: return 3;
    case UG_OP_CONV3X3_F32: return 5;
    default: return 0;
  }
}

int tune_get(int32_t op, const int64_t* shape) {
  const Table* t = g_table.load(std::memory_order_acquire);
  if (!t) return -1;
  auto it = t->find(key_of(op, shape));
  return it == t->end() ? -1 : it->second;
}

bool tune_set(int32_t op, const int64_t* shape, int variant) {
  if (tile_variants(op) == 0 || variant < -1 || variant >= tile_variants(op)) return false;
  std::lock_guard<std::mutex> lk(g_mu);
  const Table* cur = g_table.load(std::memory_order_acquire);
  Table t = cur ? *cur : Table{};
  if (variant < 0)
    t.erase(key_of(op, shape));
  else
    t[key_of(op, shape)] = variant;
  publish(std::move(t));
  return true;
}

void tune_clear() {
  std::lock_guard<std::mutex> lk(g_mu);
  publish(Table{});
}

size_t tune_size() {
  const Table* t = g_table.load(std::memory_order_acquire);
  return t ? t->size() : 0;
}

int tune_load(const char* path) {
  FILE* f = std::fopen(path, "r");
  if (!f) return -1;
  Table add;
  char line[512];
  int n = 0, bad = 0;
  while (std::fgets(line, sizeof line, f)) {
    // "op s0 s1 s2 s3 variant", '#' starts a comment
    for (char* c = line; *c; ++c)
      if (*c == '#') {
        *c = 0;
        break;
      }
    long long v[6];
    const int got = std::sscanf(line, "%lld %lld %lld %lld %lld %lld", &v[0], &v[1], &v[2], &v[3],
                                &v[4], &v[5]);
    if (got <= 0) continue;
    const int32_t op = static_cast<int32_t>(v[0]);
    if (got != 6 || tile_variants(op) == 0 || v[5] < 0 || v[5] >= tile_variants(op)) {
      ++bad;
      continue;
    }
    const int64_t s[4] = {v[1], v[2], v[3], v[4]};
    add[key_of(op, s)] = static_cast<int>(v[5]);
    ++n;
  }
  std::fclose(f);
  if (bad) return -2;
  std::lock_guard<std::mutex> lk(g_mu);
  const Table* cur = g_table.load(std::memory_order_acquire);
  Table t = cur ? *cur : Table{};
  for (auto& kv : add) t[kv.first] = kv.second;
  publish(std::move(t));
  return n;
}

}  // namespace ug
