// autotune.hpp -- choice of the level-0 cell-side factor and of the lanes per
// query (the paper's t, Sec. 4.7) for a workload class, from a cache filled by
// knn_autotune() measurements, with fixed rules as the fallback.
#pragma once

#include <cstdint>

namespace knn {

// Lanes per query of level 0 for (dims, K, N): cached measurement, else 0
// (the join then picks it from the level's candidate counts).
int autotune_lanes(int dims, int K, int64_t N);
// Cell side as a multiple of eps_min(K): cached measurement, else 1 (the
// paper's choice, cell side = eps_min).
double autotune_w_factor(int dims, int K, int64_t N);
// Records a measured best setting for the class of (dims, K, N).
void autotune_store(int dims, int K, int64_t N, double w_factor, int lanes);
// Loads / saves the cache file (path from KNN_AUTOTUNE_CACHE when path is NULL).
int autotune_load(const char* path);
int autotune_save(const char* path);

}  // namespace knn
