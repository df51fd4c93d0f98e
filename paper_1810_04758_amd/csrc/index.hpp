// index.hpp -- host-side objects of the library: the resident dataset
// (knn_index) and the per-join scratch (JoinContext).
#pragma once

#include <atomic>
#include <mutex>
#include <vector>

#include "kernels.hpp"

namespace knn {
struct GraphPlan;
struct EpsJoinState;
struct HybridState;
}

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
  // cumulative histogram counts, exact up to the first bin where they reach
  // KNN_MAX_K per sample point (later bins are not counted)
  std::vector<uint64_t> cum;
  std::vector<int64_t> hist_sample;  // ids of the histogram's sample points
  std::vector<int64_t> mean_sample;  // ids of the eps_mean sample
  std::atomic<int> busy{0};
  struct JoinContextHolder* ctx = nullptr;  // scratch of knn_self_join*
  knn::GraphPlan* graph = nullptr;          // last captured join (use_graph)
  knn::EpsJoinState* eps = nullptr;         // distance similarity join state
  knn::HybridState* hybrid = nullptr;       // the hybrid join's host index
};

namespace knn {

// Copies of large results from device memory into caller (pageable) host
// memory: chunks of kStageBytes through two pinned buffers, the copy of the
// next chunk in flight while host threads move the current one, so the
// transfer runs near the link's rate instead of the runtime's pageable path.
// The buffers are kept for later copies.
struct HostStage {
  static constexpr size_t kStageBytes = (size_t)64 << 20;
  HostBuf<char> buf[2];
  hipEvent_t ev[2] = {nullptr, nullptr};
  HostStage() = default;
  HostStage(const HostStage&) = delete;
  HostStage& operator=(const HostStage&) = delete;
  ~HostStage() {
    for (auto e : ev)
      if (e) (void)hipEventDestroy(e);
  }
};
// dst (host) <- src (device, bytes), on stream s; returns when done.
void copy_to_host(HostStage& st, void* dst, const void* src, size_t bytes, hipStream_t s);

// One grid level (Sec. 3.1) plus every temporary of the level loop.  A
// context serves one join at a time; concurrent joins use separate contexts.
struct JoinContext {
  int device = 0;
  // level arrays
  GridGeom gg{};
  GridGeom gz0{};  // Z-order levels: the level-0 geometry the keys were sorted for
  // bounds the grid levels cover: the index's, joined with an external query
  // set's when there is one
  double blo[KNN_MAX_DIMS] = {0};
  double bhi[KNN_MAX_DIMS] = {0};
  bool zmode = false;  // the current level is a Z-order level
  // the Z-order levels' sorted keys are held as uint32 in keys / keys2
  // (level-0 keys of at most 32 bits)
  bool zkeys32 = false;
  int64_t M = 0;
  DevBuf<double> Xs, Xs2;      // sorted points (Xs2: the other of a level pair)
  DevBuf<int32_t> perm, perm2;  // sorted position -> id
  DevBuf<int32_t> pos;          // sort values of a level sorted from the previous one
  DevBuf<uint32_t> pending;     // Z-order levels: queries flagged for each later level
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
  DevBuf<uint32_t> scan_state;  // single-pass scan epoch, ticket, tile words
  DevBuf<uint32_t> scal;  // [0] = M, [1] = active count
  DevBuf<int32_t> iscal;  // level counters (kCounterInts, one 128-byte line each)
  DevBuf<int32_t> active, fail_list;
  DevBuf<int32_t> active2;  // the level's active list after the deferral filter
  DevBuf<uint8_t> failed;
  DevBuf<uint64_t> ikeys, ikeys2;
  DevBuf<int32_t> ivals, ivals2;
  DevBuf<int32_t> out_ids;  // staging for host-destination joins
  DevBuf<double> out_d;
  DevBuf<char> tail_scratch;
  // [0] candidates of the active queries, [1] their maximum
  DevBuf<int32_t> heavy;      // heavy queries of the level
  DevBuf<uint8_t> cell_active;  // cells holding an active query (levels > 0)
  const uint32_t* dense_used = nullptr;  // the level's dense key table, if any
  DevBuf<uint2> rowtab;                  // row table (cells of each grid row)
  HostBuf<int32_t> pinned;               // read-backs of the level loop
  HostStage stage;                       // host-destination result copies
  const uint2* rowtab_used = nullptr;
  bool graph_owned = false;  // scratch of a captured graph: buffers are never released
  // buffers carved from one fixed region (reserve_fixed_scratch): none is
  // released or regrown during the join, and the dense key table and the row
  // table are used only up to kFixedTableFactor * N entries
  bool fixed = false;
  int64_t table_cap = 0;  // > 0: that limit; 0: the default limits
  // level 0 of a query-set join kept for the next one (JoinLimit::reuse_level0)
  bool l0_cached = false;
  double l0_w = 0;
  bool l0_zl = false;

  int64_t device_bytes() const;
};

// Device buffers of a JoinContext (the DevBuf members above).
constexpr int kContextBuffers = 36;

// What one level of a join did, recorded by an eager run so that the same
// launch sequence can be issued again without host round trips (a join on the
// same index, K and options is deterministic: the same levels, active counts,
// lanes per query and launch shapes).
struct LevelPlan {
  bool tail = false;
  int64_t A = 0;        // active queries
  int T = 0;            // lanes per query
  int64_t n_items = 0;
  int blocks = 0;       // persistent grid
  int grain = 1;
  int64_t Mcap = 0;     // cells, when the level sized its ranges by them
  uint32_t heavy_min = 0;
  int tail_rounds = 0;
  // statistics of the recorded run
  double cand = 0;
  int32_t fails = 0;
  int32_t refine = 0;
  int32_t spec = 0;
  int32_t deferred = 0;
  int64_t A_kept = 0;  // active queries after the deferral filter
  int64_t heavy = 0;
  int64_t heavy_failed = 0;
  double heavy_cand = 0;
  int64_t M = 0;
  double cell_w = 0;
  int64_t remaining = 0;  // queries left after the level (its failures and the deferred)
  int64_t failed_stat = 0;  // failed queries as the statistics count them (deferred included)
};

// A join captured in a HIP graph with the scratch it writes (its own context,
// so eager joins on the same index cannot reallocate memory the graph uses).
struct GraphPlan {
  int32_t K = 0;
  knn_join_opts opts{};  // stats pointer cleared
  int32_t* ids = nullptr;
  double* dists = nullptr;
  std::vector<LevelPlan> levels;
  double eps_min = 0;
  JoinContext ctx;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t done = nullptr;  // end of the last replay
  bool matches(int32_t K_, const knn_join_opts& o, int32_t* ids_, double* dists_) const;
  ~GraphPlan();
};

// The query set of a join of two sets, R join_KNN S (Sec. 2.1): R = Q on the
// device, row-major NQ x n (QA) and as SoA (QX[j*NQ + i]), with its bounds.
// Its points are searched against the index's points S; nothing is excluded.
struct JoinQueries {
  const double* QA = nullptr;
  const double* QX = nullptr;
  int64_t NQ = 0;
  double lo[KNN_MAX_DIMS] = {0};
  double hi[KNN_MAX_DIMS] = {0};
};

// A query-set join cut short after max_levels levels (the GPU component of
// the hybrid join, Alg. 1: each batch is searched at one eps and the queries
// that fail go back to the work queue): the query indices left unsolved go
// to `unsolved` (device, NQ entries; their output rows are not written) and
// their number to n_unsolved.  reuse_level0: keep the level-0 grid in the
// context and skip its build when the next such join asks for the same cell
// side (the indexed points never change).
struct JoinLimit {
  int max_levels = 0;
  int32_t* unsolved = nullptr;
  int64_t n_unsolved = 0;
  bool reuse_level0 = false;
};

struct JoinParams {
  int32_t K;
  knn_join_opts opts;
};

// The grid of cell side w (keys, sort, cell table, sorted coordinates, dense
// key table) into ctx, then the neighbour ranges of every cell (cell_active
// NULL) or of the flagged cells only.
// from_prev: sort from the sorted order the context holds (a previous level
// of the same join, same points) instead of from the original order.
void build_grid(const knn_index& idx, JoinContext& ctx, double w, hipStream_t s,
                bool from_prev = false);
int64_t build_ranges(const knn_index& idx, JoinContext& ctx, hipStream_t s, int64_t Mcap_known,
                     const uint8_t* cell_active, uint8_t active_tag);
// Z-order level `level` (cell side w0 * 2^level) into ctx: level 0 computes
// the interleaved keys, sorts them once and gathers the points; a later level
// only rebuilds the cell table from the same sorted keys shifted by
// dims * level bits (cell sides double exactly, so each coarse cell is a run
// of the sorted order).  Neighbour ranges follow with build_ranges.
void build_grid_z(const knn_index& idx, JoinContext& ctx, double w0, int level, hipStream_t s);
// Whether a join of (idx, K) with options o runs on Z-order levels.
bool use_zorder(const knn_index& idx, int32_t K, const knn_join_opts& o);
// Builds the grid level of cell side w into ctx (Sec. 3.1 / 4.6).
// Mcap_known > 0: the cell count that sizes the 5-6 dimension range arrays
// (no round trip); else it is read back when needed.  Returns the Mcap used.
int64_t build_level(const knn_index& idx, JoinContext& ctx, double w, hipStream_t s,
                    int64_t Mcap_known = 0);
// The whole GPU-only KNN self-join (Alg. 1 with n_large = 1): level loop with
// failures re-queued and the cell side grown until every query succeeds.
// record: filled with the levels of this run.  replay: issue exactly these
// levels with no host round trip (stream capture), statistics not written.
// jq non-NULL: the join of the query set jq with the index's points instead
// (rows of the outputs = query ids; K <= N; no replay).
void self_join(const knn_index& idx, JoinContext& ctx, int32_t K, int32_t* d_ids,
               double* d_dists, const knn_join_opts& o, hipStream_t s,
               std::vector<LevelPlan>* record = nullptr,
               const std::vector<LevelPlan>* replay = nullptr,
               const JoinQueries* jq = nullptr, JoinLimit* lim = nullptr);
// use_graph: the first join of (index, K, options, outputs) runs eagerly and
// captures its launch sequence; later ones launch the graph.
void self_join_graph(knn_index& idx, int32_t K, int32_t* d_ids, double* d_dists,
                     const knn_join_opts& o, hipStream_t s);
constexpr int64_t kFixedTableFactor = 4;
// Device bytes a join of (idx, K) needs beyond the index (admission control).
uint64_t join_footprint(const knn_index& idx, int32_t K, bool host_output);
double eps_min_of(const knn_index& idx, int32_t K);
// Brute-force tail budget of a join in (remaining queries) x N pairs; <= 0: no tail.
double tail_budget_of(const knn_index& idx, int32_t K, const knn_join_opts& o);
// A join whose every buffer comes from one fixed region: the bytes it needs
// (each buffer at its largest size for (idx, K, o), 256-byte aligned), and
// the reservation of all of them in ctx at those sizes (so the level loop
// never grows one).  ctx.table_cap must be set first.
uint64_t fixed_scratch_bytes(const knn_index& idx, int32_t K, const knn_join_opts& o);
void reserve_fixed_scratch(const knn_index& idx, JoinContext& ctx, int32_t K,
                           const knn_join_opts& o, hipStream_t s);
void validate_join(const knn_index* idx, int32_t K);
// Geometry of the level with cell side w.  The side is enlarged (w updated)
// if the grid would not fit the 62-bit key space or 2^30 cells per dimension
// (a performance policy only: any side gives exact results).
GridGeom make_geom(int n, const double* lo, const double* hi, double& w);

// The state of the distance similarity self-join an index keeps between
// calls (epsjoin_rt.hip); freed with the index.
struct EpsJoinState;
void destroy_eps_state(EpsJoinState* st);
// The hybrid join's host-side index (hybrid.hip); freed with the index.
struct HybridState;
void destroy_hybrid_state(HybridState* h);

// Makes `dev` current for a scope.
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    KNN_HIP(hipGetDevice(&prev));
    if (prev != dev) KNN_HIP(hipSetDevice(dev));
  }
  ~DeviceGuard() {
    int cur = -1;
    if (hipGetDevice(&cur) == hipSuccess && cur != prev && prev >= 0) (void)hipSetDevice(prev);
  }
};

// One join at a time per index (KNN_EBUSY otherwise).
struct BusyGuard {
  knn_index* idx;
  explicit BusyGuard(knn_index* i) : idx(i) {
    int expect = 0;
    KNN_CHECK(idx->busy.compare_exchange_strong(expect, 1), KNN_EBUSY,
              "another join is running on this index");
  }
  ~BusyGuard() { idx->busy.store(0); }
};

// Runs f at the C ABI edge: KNN_OK, or the code of the exception it threw
// (its message to knn_last_error).
template <class F>
int guarded(F&& f) {
  try {
    f();
    set_last_error("");
    return KNN_OK;
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  } catch (const std::bad_alloc&) {
    set_last_error("host allocation failed");
    return KNN_ENOMEM;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return KNN_EINTERNAL;
  } catch (...) {
    set_last_error("unknown error");
    return KNN_EINTERNAL;
  }
}

}  // namespace knn

struct JoinContextHolder {
  knn::JoinContext ctx;
};
