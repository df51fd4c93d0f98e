// index.hpp -- host-side objects of the library: the resident dataset
// (knn_index) and the per-join scratch (JoinContext).
#pragma once

#include <atomic>
#include <mutex>
#include <vector>

#include "kernels.hpp"

struct knn_index {
  int64_t N = 0;
  int n = 0;
  int device = 0;
  knn::DevBuf<double> X;   // SoA coordinates in id order, X[j*N + i]
  knn::DevBuf<double> XA;  // the same, row-major N x n (one point = one read in gathers)
  double lo[KNN_MAX_DIMS] = {0};
  double hi[KNN_MAX_DIMS] = {0};
  // search-distance selection (Sec. 4.4)
  double eps_mean = 0;
  double bin_width = 0;
  int n_bins = 0;
  int n_sample = 0;
  std::vector<uint64_t> cum;  // cumulative histogram counts
  std::atomic<int> busy{0};
  struct JoinContextHolder* ctx = nullptr;  // scratch of knn_self_join*
};

namespace knn {

// One grid level (Sec. 3.1) plus every temporary of the level loop.  A
// context serves one join at a time; concurrent joins use separate contexts.
struct JoinContext {
  int device = 0;
  // level arrays
  GridGeom gg{};
  int64_t M = 0;
  DevBuf<double> Xs;
  DevBuf<int32_t> perm;
  DevBuf<uint32_t> cell_of;
  DevBuf<uint64_t> cell_key;
  DevBuf<uint32_t> cell_start;
  DevBuf<uint32_t> ranges;  // compacted non-empty row segments, R slots per cell
  DevBuf<uint8_t> rslot;    // segment index of each compacted entry
  DevBuf<uint32_t> nrng;    // non-empty segments per cell
  DevBuf<uint32_t> cand_count;
  DevBuf<uint32_t> dense;
  // temporaries
  DevBuf<uint64_t> keys, keys2;
  DevBuf<int32_t> vals2;
  DevBuf<uint32_t> flags, tmp;
  DevBuf<uint32_t> scal;  // [0] = M, [1] = active count
  DevBuf<int32_t> iscal;  // [0] = head, [1] = fail count, [2] = refine rounds
  DevBuf<int32_t> active, fail_list;
  DevBuf<uint8_t> failed;
  DevBuf<uint64_t> ikeys, ikeys2;
  DevBuf<int32_t> ivals, ivals2;
  DevBuf<int32_t> out_ids;  // staging for host-destination joins
  DevBuf<double> out_d;

  int64_t device_bytes() const;
};

struct JoinParams {
  int32_t K;
  knn_join_opts opts;
};

// Builds the grid level of cell side w into ctx (Sec. 3.1 / 4.6).
void build_level(const knn_index& idx, JoinContext& ctx, double w, hipStream_t s);
// The whole GPU-only KNN self-join (Alg. 1 with n_large = 1): level loop with
// failures re-queued and the cell side grown until every query succeeds.
void self_join(const knn_index& idx, JoinContext& ctx, int32_t K, int32_t* d_ids,
               double* d_dists, const knn_join_opts& o, hipStream_t s);
// Device bytes a join of (idx, K) needs beyond the index (admission control).
uint64_t join_footprint(const knn_index& idx, int32_t K, bool host_output);
double eps_min_of(const knn_index& idx, int32_t K);
void validate_join(const knn_index* idx, int32_t K);

}  // namespace knn

struct JoinContextHolder {
  knn::JoinContext ctx;
};
