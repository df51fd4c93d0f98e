// autotune.hip -- cache of measured (cell-side factor, lanes per query)
// settings per workload class, with fixed fallback rules.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>

#include "autotune.hpp"
#include "kernels.hpp"

namespace knn {

namespace {

// Workload class: dims, K bucket (power of two), N bucket (power of 4).
using Class = std::tuple<int, int, int>;
struct Entry {
  double w_factor;
  int lanes;
};

std::mutex g_mu;
std::map<Class, Entry> g_cache;
bool g_loaded = false;

int log2_bucket(int64_t v) {
  int b = 0;
  while ((int64_t(1) << (b + 1)) <= v) ++b;
  return b;
}

Class class_of(int dims, int K, int64_t N) {
  return Class(dims, log2_bucket(K), log2_bucket(N) / 2);
}

void ensure_loaded() {
  if (g_loaded) return;
  g_loaded = true;
  const char* p = std::getenv("KNN_AUTOTUNE_CACHE");
  if (!p || !*p) return;
  FILE* f = std::fopen(p, "r");
  if (!f) return;
  int d, kb, nb, lanes;
  double wf;
  while (std::fscanf(f, "%d %d %d %lf %d", &d, &kb, &nb, &wf, &lanes) == 5)
    g_cache[Class(d, kb, nb)] = Entry{wf, lanes};
  std::fclose(f);
}

}  // namespace

int autotune_lanes(int dims, int K, int64_t N) {
  {
    std::lock_guard<std::mutex> lk(g_mu);
    ensure_loaded();
    auto it = g_cache.find(class_of(dims, K, N));
    if (it != g_cache.end() && it->second.lanes > 0) return it->second.lanes;
  }
  return 0;  // no measurement: chosen per level from the candidate counts
}

double autotune_w_factor(int dims, int K, int64_t N) {
  std::lock_guard<std::mutex> lk(g_mu);
  ensure_loaded();
  auto it = g_cache.find(class_of(dims, K, N));
  if (it != g_cache.end() && it->second.w_factor > 0) return it->second.w_factor;
  return 1.0;
}

void autotune_store(int dims, int K, int64_t N, double w_factor, int lanes) {
  std::lock_guard<std::mutex> lk(g_mu);
  ensure_loaded();
  g_cache[class_of(dims, K, N)] = Entry{w_factor, lanes};
}

int autotune_load(const char* path) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_loaded = true;
  const char* p = path ? path : std::getenv("KNN_AUTOTUNE_CACHE");
  if (!p) return -1;
  FILE* f = std::fopen(p, "r");
  if (!f) return -1;
  int d, kb, nb, lanes;
  double wf;
  while (std::fscanf(f, "%d %d %d %lf %d", &d, &kb, &nb, &wf, &lanes) == 5)
    g_cache[Class(d, kb, nb)] = Entry{wf, lanes};
  std::fclose(f);
  return 0;
}

int autotune_save(const char* path) {
  std::lock_guard<std::mutex> lk(g_mu);
  const char* p = path ? path : std::getenv("KNN_AUTOTUNE_CACHE");
  if (!p) return -1;
  FILE* f = std::fopen(p, "w");
  if (!f) return -1;
  for (auto& kv : g_cache)
    std::fprintf(f, "%d %d %d %.17g %d\n", std::get<0>(kv.first), std::get<1>(kv.first),
                 std::get<2>(kv.first), kv.second.w_factor, kv.second.lanes);
  std::fclose(f);
  return 0;
}

}  // namespace knn
