// autotune.hpp -- cache of measured join settings per workload class: the
// level-0 cell-side factor (cell side = factor * eps_min(K), Sec. 4.4), the
// geometric growth of the cell side between levels, and the lanes per query
// of level 0 (the paper's t, Sec. 4.7).  Filled by knn_autotune()
// measurements; fixed rules are the fallback.
#pragma once

#include <cstdint>

namespace knn {

struct TuneEntry {
  double w_factor;  // 0 = no measurement
  double growth;    // 0 = no measurement
  int lanes;        // 0 = chosen per level from the candidate counts
  int linear = 0;   // linear growths: 0 = not measured (default), 1, or -1 (none)
  double tail_pairs = 0;  // brute-force tail budget, 0 = not measured
  int lanes_shift = 0;    // the per-level lanes-per-query rule times 2^shift
  int zorder = 0;         // Z-order levels: 1 on, -1 off, 0 = not measured
  int pops = 0;           // persistent queue: pops per wavefront, 0 = not measured
};

// Cached entry for the class of (dims, K, N), or all zeros.
TuneEntry autotune_get(int dims, int K, int64_t N);
// Level-0 lanes (0 if none cached), cell-side factor (1 if none cached: the
// paper's choice, cell side = eps_min) and growth (0 if none cached).
int autotune_lanes(int dims, int K, int64_t N);
double autotune_w_factor(int dims, int K, int64_t N);
double autotune_growth(int dims, int K, int64_t N);
// Linear growths before the geometric ones (0 if none cached: the default).
int autotune_linear(int dims, int K, int64_t N);
// Brute-force tail budget (0 if none cached).
double autotune_tail_pairs(int dims, int K, int64_t N);
// Shift of the per-level lanes-per-query rule (0 if none cached).
int autotune_lanes_shift(int dims, int K, int64_t N);
// Z-order levels: 1 / -1 as measured, 0 if none cached.
int autotune_zorder(int dims, int K, int64_t N);
// Pops per wavefront and queue of the persistent search (0 if none cached).
int autotune_pops(int dims, int K, int64_t N);
// Records a measured best setting for the class of (dims, K, N).
void autotune_store(int dims, int K, int64_t N, const TuneEntry& e);
// Loads / saves the cache file (path from KNN_AUTOTUNE_CACHE when path is NULL).
int autotune_load(const char* path);
int autotune_save(const char* path);
void autotune_clear();

}  // namespace knn
