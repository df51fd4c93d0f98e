// autotune.hip -- cache of measured join settings per workload class, with
// fixed fallbacks.  The measurements themselves (knn_autotune) live with the
// join in index.hip.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>

#include "autotune.hpp"

namespace knn {

namespace {

// Workload class: dims, K bucket (power of two), N bucket (power of 4).
using Class = std::tuple<int, int, int>;

std::mutex g_mu;
std::map<Class, TuneEntry> g_cache;
bool g_loaded = false;

int log2_bucket(int64_t v) {
  int b = 0;
  while ((int64_t(1) << (b + 1)) <= v) ++b;
  return b;
}

Class class_of(int dims, int K, int64_t N) {
  return Class(dims, log2_bucket(K), log2_bucket(N) / 2);
}

void load_file_locked(const char* p) {
  if (!p || !*p) return;
  FILE* f = std::fopen(p, "r");
  if (!f) return;
  // one entry per line: 11 fields, or the 10 of files written before the
  // queue granularity was measured
  char line[512];
  while (std::fgets(line, sizeof(line), f)) {
    int d, kb, nb, lanes, lin, ls, z, pp = 0;
    double wf, gr, tp;
    const int got = std::sscanf(line, "%d %d %d %lf %lf %d %d %lf %d %d %d", &d, &kb, &nb, &wf, &gr,
                                &lanes, &lin, &tp, &ls, &z, &pp);
    if (got < 10) continue;
    if (got == 10) pp = 0;
    g_cache[Class(d, kb, nb)] = TuneEntry{wf, gr, lanes, lin, tp, ls, z, pp};
  }
  std::fclose(f);
}

void ensure_loaded_locked() {
  if (g_loaded) return;
  g_loaded = true;
  load_file_locked(std::getenv("KNN_AUTOTUNE_CACHE"));
}

}  // namespace

TuneEntry autotune_get(int dims, int K, int64_t N) {
  std::lock_guard<std::mutex> lk(g_mu);
  ensure_loaded_locked();
  auto it = g_cache.find(class_of(dims, K, N));
  return it != g_cache.end() ? it->second : TuneEntry{0.0, 0.0, 0};
}

int autotune_lanes(int dims, int K, int64_t N) { return autotune_get(dims, K, N).lanes; }

double autotune_w_factor(int dims, int K, int64_t N) {
  const double f = autotune_get(dims, K, N).w_factor;
  return f > 0 ? f : 1.0;
}

double autotune_growth(int dims, int K, int64_t N) { return autotune_get(dims, K, N).growth; }

int autotune_linear(int dims, int K, int64_t N) { return autotune_get(dims, K, N).linear; }

double autotune_tail_pairs(int dims, int K, int64_t N) {
  return autotune_get(dims, K, N).tail_pairs;
}

int autotune_lanes_shift(int dims, int K, int64_t N) {
  return autotune_get(dims, K, N).lanes_shift;
}

int autotune_zorder(int dims, int K, int64_t N) { return autotune_get(dims, K, N).zorder; }
int autotune_pops(int dims, int K, int64_t N) { return autotune_get(dims, K, N).pops; }

void autotune_store(int dims, int K, int64_t N, const TuneEntry& e) {
  std::lock_guard<std::mutex> lk(g_mu);
  ensure_loaded_locked();
  g_cache[class_of(dims, K, N)] = e;
}

int autotune_load(const char* path) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_loaded = true;
  const char* p = path ? path : std::getenv("KNN_AUTOTUNE_CACHE");
  if (!p) return -1;
  FILE* f = std::fopen(p, "r");
  if (!f) return -1;
  std::fclose(f);
  load_file_locked(p);
  return 0;
}

int autotune_save(const char* path) {
  std::lock_guard<std::mutex> lk(g_mu);
  const char* p = path ? path : std::getenv("KNN_AUTOTUNE_CACHE");
  if (!p) return -1;
  FILE* f = std::fopen(p, "w");
  if (!f) return -1;
  for (auto& kv : g_cache)
    std::fprintf(f, "%d %d %d %.17g %.17g %d %d %.17g %d %d %d\n", std::get<0>(kv.first),
                 std::get<1>(kv.first), std::get<2>(kv.first), kv.second.w_factor,
                 kv.second.growth, kv.second.lanes, kv.second.linear, kv.second.tail_pairs,
                 kv.second.lanes_shift, kv.second.zorder, kv.second.pops);
  std::fclose(f);
  return 0;
}

void autotune_clear() {
  std::lock_guard<std::mutex> lk(g_mu);
  g_cache.clear();
  g_loaded = true;
}

}  // namespace knn
