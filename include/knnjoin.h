/*
 * knnjoin.h -- C ABI of libknnjoin.so, an exact grid-indexed K-nearest-
 * neighbour self-join for one AMD Instinct MI355X (gfx950).
 *
 * Method: Gowanlock, "Hybrid CPU/GPU KNN self-join" (arXiv:1810.04758),
 * GPU component only (HYBRID-GPU / GPU-Only configuration, Sec. 4.2, Alg. 1):
 *   - points are binned into a uniform grid whose cell side is the search
 *     distance eps (Sec. 3.1; built on the GPU, Sec. 4.6);
 *   - each query scans its own cell and the 3^n - 1 adjacent cells, computes
 *     the distances and keeps its K nearest (Alg. 1, GPUJoinKernel);
 *   - queries that cannot prove their K nearest inside the scanned cells fail
 *     and are re-run on a grid with a larger eps (Alg. 1, re-index rule;
 *     Sec. 4.5);
 *   - eps starts from eps_min, chosen by sampling (Sec. 4.4);
 *   - queries are processed dense-first (work estimate of Sec. 4.5).
 *
 * Result (problem statement, Sec. 2.1): for every point i of D, the K points
 * j != i with the smallest Euclidean distance.  Ties in the squared distance
 * go to the lower point id (the paper is silent; this library's reading).
 * Row i of the output lists them nearest first.  Distances are
 * sqrt(sum_j (x_j - y_j)^2), the sum taken left to right over the
 * dimensions with every operation rounded (no fused multiply-add), and the
 * square root correctly rounded, so results are reproducible bit for bit.
 *
 * Conventions
 *   - Every function returns KNN_OK (0) or a negative KNN_E* code and never
 *     lets a C++ exception escape.  knn_last_error() returns a description of
 *     the last failure on the calling thread.
 *   - "host" pointers are ordinary CPU memory; "device" pointers are HIP
 *     device memory on the index's device.  Streams are hipStream_t passed as
 *     void* (NULL = the legacy default stream).
 *   - Point coordinates are fp64, row-major N x dims (point i occupies
 *     D[i*dims .. i*dims+dims-1]).  2 <= dims <= 6 (the paper's range, Sec.
 *     2.3), 2 <= N < 2^31, every coordinate finite.
 *   - Output arrays are row-major N x K: ids int32, dists fp64.
 */
#ifndef KNNJOIN_H
#define KNNJOIN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KNN_OK 0
#define KNN_EINVAL (-1)    /* invalid argument */
#define KNN_ENOMEM (-2)    /* device or host allocation failed */
#define KNN_EDEVICE (-3)   /* HIP runtime or kernel error */
#define KNN_EBUSY (-4)     /* object in use / queue full */
#define KNN_ETIMEOUT (-5)  /* wait timed out */
#define KNN_EINTERNAL (-6) /* internal invariant violated (a bug) */
#define KNN_ECANCELED (-7) /* a caller's callback stopped the operation */

#define KNN_MIN_DIMS 2
#define KNN_MAX_DIMS 6
#define KNN_MAX_K 1024 /* largest K the search kernel's per-query buffers hold */

typedef struct knn_index knn_index;

/* Options of knn_build_index*.  Zero fields take the defaults in brackets. */
typedef struct knn_build_opts {
  uint64_t seed;        /* seed of the sampling generator (SplitMix64) [1] */
  int32_t n_sample;     /* sample points of the distance histogram [500], Sec. 4.4 */
  int32_t n_bins;       /* histogram bins up to eps_mean [1000], Sec. 4.4 */
  double mean_frac;     /* fraction of D sampled for eps_mean [0.001], Sec. 4.4 */
  int32_t min_mean_sample; /* lower bound of the eps_mean sample size [64] */
  int32_t device;       /* HIP device ordinal; < 0 = current device [-1] */
} knn_build_opts;

/* Per-join statistics (optional output of the join calls). */
#define KNN_MAX_LEVELS 64
typedef struct knn_join_stats {
  int32_t levels;             /* grid levels searched (1 + re-indexes) */
  double eps_min;             /* eps_min(K) from the histogram */
  double cell_width[KNN_MAX_LEVELS];   /* cell side of each level */
  int64_t attempted[KNN_MAX_LEVELS];   /* active queries at each level (deferred
                                          ones included) */
  int64_t failed[KNN_MAX_LEVELS];      /* of which failed (re-queued) */
  int64_t cells[KNN_MAX_LEVELS];       /* non-empty cells of each level */
  double ms_build[KNN_MAX_LEVELS];     /* index construction time per level */
  double ms_search[KNN_MAX_LEVELS];    /* search kernel (k_search) time per level */
  double ms_total;            /* wall time of the whole join */
  int64_t total_attempted;    /* sum of attempted */
  int64_t total_failed;       /* sum of failed: fraction = failed/attempted */
  int32_t lanes_per_query;    /* t of level 0 */
  int32_t lanes[KNN_MAX_LEVELS];          /* t used at each level */
  double cand_per_query[KNN_MAX_LEVELS];  /* mean candidates per searched query
                                             (active and not deferred) */
  int64_t refine_rounds[KNN_MAX_LEVELS];  /* exact-bisection rounds (crowded bins) */
  int64_t tail_queries;       /* queries finished by the brute-force tail */
  int32_t tail_rounds;        /* its exact-bisection rounds */
  double ms_tail;             /* its time */
  double ms_heavy[KNN_MAX_LEVELS];        /* heavy-query kernel time per level */
  int64_t heavy_queries[KNN_MAX_LEVELS];  /* queries it took (one workgroup each) */
  int64_t heavy_failed[KNN_MAX_LEVELS];   /* of which failed */
  double heavy_cand[KNN_MAX_LEVELS];      /* their candidates in total */
  int64_t spec_queries[KNN_MAX_LEVELS];   /* queries whose speculation held (no
                                             collect pass) */
  int64_t deferred[KNN_MAX_LEVELS];       /* queries deferred to the next level
                                             without a count pass (in failed) */
} knn_join_stats;

/* Options of the join calls.  Zero fields take the defaults in brackets. */
typedef struct knn_join_opts {
  double w_factor;        /* level-0 cell side = w_factor * eps_min(K) [autotuned or 1] */
  double cell_width;      /* > 0: explicit level-0 cell side, overrides w_factor */
  int32_t lanes_per_query;/* t, threads per query: 1,2,4,...,64 [autotuned] (Sec. 4.7) */
  int32_t schedule;       /* 0 persistent kernel + device work queue, density ordered;
                             1 one launch per batch, cell order [0] */
  int32_t batch_queries;  /* schedule 1: queries per launch, 0 = all [0] */
  double eps_step;        /* linear growth step, multiple of eps_min [0.5] (Alg. 1) */
  int32_t linear_levels;  /* linear growths before geometric growth [1]; < 0: none */
  double growth;          /* geometric growth factor of the cell side [16^(1/dims)] */
  int32_t use_graph;      /* 1: the first join of (index, K, these options, these
                             outputs) runs eagerly, recording its levels, and
                             captures the same launch sequence in a HIP graph
                             held by the index (with scratch of its own); later
                             such joins launch the graph: no host round trip,
                             asynchronous on the stream.  One graph per index
                             (another key replaces it).  Statistics of a replay
                             repeat the recorded counts; per-level times are 0 [0] */
  double tail_pairs;      /* brute-force tail once (remaining queries) x N <= this
                             [autotuned or 2.5e8]; < 0 disables the tail (the
                             remedy Sec. 5.4 proposes) */
  int64_t heavy_min;      /* queries with at least this many
                             candidates get a workgroup each; 0 = automatic
                             (those that would outlast the level), < 0 = never */
  int32_t queue_grain;    /* persistent schedule: work items claimed per queue pop;
                             0 = automatic (a level's items over (wavefronts x P),
                             at most 64, P = pops per wavefront [autotuned or 4]);
                             < 0: automatic with P = -queue_grain */
  int32_t item_order;     /* persistent schedule: 0 = densest class first inside
                             each XCD's contiguous chunk (Sec. 4.5 ordering);
                             1 = cell order [0] */
  int32_t lanes_shift;    /* automatic lanes per query times 2^lanes_shift (-2..2)
                             [autotuned or 0] */
  int32_t share_lists;    /* 1: the queries of a wavefront that share a cell walk
                             one candidate list (the union of their pruned
                             lists), so every load serves all of them; -1: each
                             query walks its own; 0 = automatic [1 in 5-6
                             dimensions, whose search is bound by the L2] */
  int32_t speculate;      /* 0: the count pass keeps the candidates within a
                             K-th distance predicted from the local density and,
                             when they hold the K nearest, the collect pass is
                             skipped for that query; -1: never [0] */
  int32_t predict_fail;   /* 0: a query whose K-th distance, predicted from the
                             local density, exceeds its covered radius by a
                             margin goes to the next level without searching
                             this one (results are unchanged); -1: never [0] */
  int32_t zorder;         /* 1: Z-order levels (2-4 dimensions): the points are
                             sorted once by the bit-interleaved cell key of the
                             level-0 grid, and every re-index doubles the cell
                             side (the key shifted right by dims bits), so a
                             level costs a cell-table pass instead of a sort;
                             growth, linear_levels and eps_step are then
                             ignored.  -1: row-major levels re-sorted at every
                             re-index.  0 = autotuned, else on in 2-3
                             dimensions [0] */
  knn_join_stats* stats;  /* optional statistics output */
} knn_join_opts;

/* Fills *o with the defaults (all zero).  Always succeeds. */
void knn_build_opts_default(knn_build_opts* o);
void knn_join_opts_default(knn_join_opts* o);

/*
 * Builds the index of D: copies D to the device, computes per-dimension
 * bounds, and runs the search-distance sampling of Sec. 4.4 (eps_mean and
 * the cumulative distance histogram, which does not depend on K, so
 * eps_min(K) becomes a lookup at join time).  Grid levels are built by the
 * join, since their cell side depends on K.
 *   D        host, N x dims fp64, read only; copied, the caller may free it on
 *            return.
 *   opts     may be NULL.
 *   out      receives the index; owned by the caller, free with
 *            knn_destroy_index.
 * Errors: KNN_EINVAL (dims outside [2,6], N < 2 or N >= 2^31, a non-finite
 * coordinate, NULL pointers), KNN_ENOMEM, KNN_EDEVICE.
 */
int knn_build_index(const double* D, int64_t n_points, int32_t dims,
                    const knn_build_opts* opts, knn_index** out);

/* As knn_build_index, with D already in device memory (N x dims fp64,
 * row-major).  D is copied on `stream`; it must stay valid until the call
 * returns (the call synchronises the stream). */
int knn_build_index_device(const double* d_D, int64_t n_points, int32_t dims,
                           const knn_build_opts* opts, void* stream,
                           knn_index** out);

/*
 * KNN self-join D join_KNN D (Sec. 2.1) into host arrays.
 *   ids, dists  host, N x K each, written completely on success; contents
 *               unspecified on error.
 *   K           1 <= K <= min(N-1, KNN_MAX_K).
 *   opts        may be NULL.
 * Blocks until done.  One join per index at a time: a concurrent call on the
 * same index returns KNN_EBUSY.
 */
int knn_self_join(knn_index* idx, int32_t K, int32_t* ids, double* dists,
                  const knn_join_opts* opts);

/*
 * As knn_self_join, with d_ids / d_dists in device memory (N x K each).
 * Work is issued on `stream`; the call returns after the last level's
 * failure count has been read back (the level loop needs it on the host), at
 * which point the results are complete in device memory.
 */
int knn_self_join_device(knn_index* idx, int32_t K, int32_t* d_ids, double* d_dists,
                         const knn_join_opts* opts, void* stream);

/*
 * KNN join of a query set with the indexed set, R join_KNN S (Sec. 2.1: the
 * self-join's definition for a query set R = Q against the indexed points
 * S = D; Sec. 4.3 adds such a query set to the GPU kernel): for every query
 * point, the K points of D with the smallest Euclidean distance.  Nothing is
 * excluded: a query equal to a point of D has that point as a neighbour at
 * distance 0.  Distances, ordering and the tie rule are the self-join's.
 * The index's grid levels are used unchanged (queries outside D's bounding
 * box widen the levels' box); each query's neighbour cells are looked up
 * from its own coordinates.
 *   d_Q             device, n_queries x dims fp64 row-major (the index's
 *                   dims), read only; must stay valid until the call returns.
 *   d_ids, d_dists  device, n_queries x K each; row r = query r, ids are
 *                   point ids of D.
 *   K               1 <= K <= min(N, KNN_MAX_K).
 *   opts            may be NULL; use_graph must be 0.
 * Work is issued on `stream`; the call returns when the results are complete.
 * Errors: KNN_EINVAL (K out of range, n_queries < 1, N + n_queries >= 2^31,
 * a non-finite query coordinate, use_graph set, NULL pointers), KNN_ENOMEM,
 * KNN_EDEVICE, KNN_EBUSY (another join running on the index).
 */
int knn_join_device(knn_index* idx, const double* d_Q, int64_t n_queries, int32_t K,
                    int32_t* d_ids, double* d_dists, const knn_join_opts* opts, void* stream);

/* As knn_join_device with Q, ids and dists in host memory (blocks). */
int knn_join(knn_index* idx, const double* Q, int64_t n_queries, int32_t K, int32_t* ids,
             double* dists, const knn_join_opts* opts);

/*
 * For callers that cannot allocate device memory during the call (serving
 * loops that run on a fixed memory plan, harnesses that forbid hipMalloc):
 * the same join as knn_self_join_device, same arguments, results and
 * ordering, with every temporary buffer taken from a fixed scratch area of
 * KNN_NOALLOC_SCRATCH_BYTES that the library holds per device (a static
 * device array, present on every device that runs the library until the
 * process ends).  The call makes no hipMalloc, hipFree, hipHostMalloc or
 * other allocating call; the caller still provides d_ids / d_dists.
 *   Limit: the join's buffers, each at its largest size for (index, K,
 *   opts), must fit the area (roughly 180-250 + 17*R bytes per point, R =
 *   3^dims on Z-order levels and 3^(dims-1) on row-major ones, plus the
 *   brute-force tail's per-query state: about 2e5 points in 2-D, 1.5e4 in
 *   6-D); larger joins return KNN_EINVAL, and knn_last_error() states the
 *   bytes needed.
 *   opts->stats must be NULL and opts->use_graph 0 (both would allocate):
 *   KNN_EINVAL otherwise.
 * The area is shared by every call on a device and keeps the last call's
 * contents; everything a join reads is written or cleared by the join
 * itself.  Calls on one device are serialised by the library (a second
 * caller blocks until the first returns; each call returns after its device
 * work has completed), since overlapping joins in one area would race.
 */
#define KNN_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int knn_self_join_device_noalloc(knn_index* idx, int32_t K, int32_t* d_ids,
                                 double* d_dists, const knn_join_opts* opts,
                                 void* stream);

/* ------------------------------------------------------------------------
 * Hybrid CPU/GPU KNN self-join (Sec. 4.1-4.5, Alg. 1 with its CPU ranks):
 * the same result as knn_self_join, with the queries split between the GPU
 * and host threads through one work queue.  The queue holds the point ids
 * ordered by the point count of their own cell at eps_min(K), densest first
 * (Sec. 4.5).  The GPU takes batches from the dense end and searches each at
 * one eps (cell side eps; first eps = eps_factor * eps_min(K)); the queries
 * it cannot prove go back to the front of the queue, and eps grows by
 * eps_min / 2 when more than a quarter of a batch failed (Alg. 1).  Host
 * threads take batches from the sparse end and solve them exactly with a
 * kd-tree over all points (built on first use, kept with the index).
 * Batch schedule, all sizes fractions of N: a monolithic GPU batch of
 * n_large, then after each round n_large' = min(n_large / 2, max(0, 1 -
 * done_gpu - done_cpu - n_cwin)) (the window n_cwin stays reserved for the
 * CPU), until it reaches 0; then GPU batches of n_small; CPU batches of
 * n_cpu; both small sizes halve once 95 % of the queries are done.
 * ------------------------------------------------------------------------ */
typedef struct knn_hybrid_opts {
  double n_large;     /* first monolithic GPU batch [0.4]; < 0: none */
  double n_small;     /* GPU batch after the monolithic rounds [0.005] */
  double n_cwin;      /* window reserved for the CPU [0.4]; < 0: none */
  double n_cpu;       /* CPU batch [0.005] */
  double eps_factor;  /* first eps = eps_factor * eps_min(K) [1] */
  int32_t cpu_threads;/* host threads [hardware threads - 1]; < 0: none (the
                         GPU takes every batch) */
  int32_t zorder;     /* the GPU's level structure, as knn_join_opts.zorder */
} knn_hybrid_opts;
typedef struct knn_hybrid_stats {
  double ms_total;        /* T: the whole call */
  double ms_gpu;          /* T_GPU: when the GPU finished its last batch */
  double ms_cpu;          /* T_CPU: when the last host thread finished */
  double load_imbalance;  /* |T_CPU - T_GPU| / T (Sec. 5.5); 0 without threads */
  double ms_queue;        /* building the work queue (part of T) */
  double ms_cpu_index;    /* building the kd-tree in this call (0 if kept) */
  double ms_merge;        /* copying the GPU's rows into the host outputs (part
                             of T, after T_GPU and T_CPU) */
  double eps_min;         /* eps_min(K) */
  double eps_final;       /* the GPU's eps at the end */
  int64_t gpu_queries;    /* queries solved by the GPU */
  int64_t cpu_queries;    /* queries solved by the host threads */
  int64_t gpu_attempts;   /* queries given to the GPU, failures counted again */
  int32_t gpu_batches;
  int32_t monolithic_batches;
  int32_t reindexes;      /* eps increases */
  int32_t cpu_threads;
} knn_hybrid_stats;
/*
 * ids / dists: host, N x K each (row i = point i, nearest first, the order
 * and distances of knn_self_join).  1 <= K <= min(N - 1, KNN_MAX_K - 1).
 * opts and stats may be NULL.  Blocks until done.
 * Errors: KNN_EINVAL (K out of range, n_small or n_cpu negative, NULL
 * outputs), KNN_ENOMEM, KNN_EDEVICE, KNN_EBUSY.
 */
int knn_self_join_hybrid(knn_index* idx, int32_t K, int32_t* ids, double* dists,
                         const knn_hybrid_opts* opts, knn_hybrid_stats* stats);

/* ------------------------------------------------------------------------
 * Distance similarity self-join (Sec. 1 and Sec. 3: the range-query join
 * whose GPU kernel the KNN join is built from).  Result: every ordered pair
 * (i, j) of points of D with j != i and fl(sqrt(d2(i, j))) <= eps, d2 the
 * KNN join's squared distance (left to right over the dimensions, every
 * operation rounded, no fused multiply-add); each unordered pair appears
 * twice, once per direction, and a duplicate point at distance 0 is a
 * neighbour.  Pairs are key/value triples (query id, neighbour id, distance
 * = the rounded square root), produced in batches that fit a result buffer
 * (Sec. 3.2).
 * Method: one grid level of cell side eps (Sec. 3.1; enlarged by 2^-16 so
 * that rounding cannot move a neighbour out of the 3^n block, or further when
 * the grid would be too fine); each query scans its block, skipping the
 * parts of each row of cells that lie farther than eps.  The paper sizes its
 * batches from an estimated result size; here a count pass gives each
 * query's exact pair count first (kept for later calls with the same eps),
 * so a batch can never overflow its buffer.
 * The level and counts stay with the index until it is destroyed, a call
 * with another eps replaces them, or knn_eps_join_release frees them.  These
 * calls share the index's one-join-at-a-time rule (KNN_EBUSY).
 * Errors of all of them: KNN_EINVAL (idx NULL, eps negative or not finite,
 * the other arguments as stated), KNN_ENOMEM, KNN_EDEVICE, KNN_EBUSY.
 * ------------------------------------------------------------------------ */

/*
 * Result size.  sample_stride 1: *n_pairs = the exact number of pairs; then
 * d_counts, when not NULL (device, int32 x N), receives the pair count of
 * each point id.  sample_stride s > 1: the estimate of Sec. 3.2 (a light
 * pass over a sample): the pairs of every s-th query in the processing
 * order (a sample spread evenly over the cells), scaled by N / (queries
 * sampled), rounded; d_counts must then be NULL.
 * Issues its work on `stream` and returns when the size is known.
 */
int knn_eps_join_size(knn_index* idx, double eps, int64_t sample_stride, uint64_t* n_pairs,
                      int32_t* d_counts, void* stream);

/*
 * One batch into device memory.  The queries are taken in the index's
 * processing order for this eps (cells in key order; a cursor is a position
 * in it: 0 starts the join, n_points means done).  The batch holds the pairs
 * of the queries at positions [cursor, *next_cursor): as many whole queries
 * as fit `capacity` pairs, at least one (KNN_EINVAL, with the count in
 * knn_last_error, if the query at `cursor` alone has more pairs; a cursor
 * of n_points returns 0 pairs).
 *   d_qids, d_nids  device, int32, capacity entries: query id, neighbour id.
 *   d_dists         device, fp64, capacity entries.
 *   *n_pairs        pairs written, at indices [0, *n_pairs).
 * Order: a query's pairs are contiguous, queries in processing order; within
 * a query the scan order (deterministic; not sorted by id or distance).
 * The first call for an eps builds the level and counts (blocking); each
 * call reads its batch bounds back, then issues the writes on `stream` and
 * returns: the pairs are complete when the stream reaches that point.
 */
int knn_eps_join_device(knn_index* idx, double eps, int64_t cursor, uint64_t capacity,
                        int32_t* d_qids, int32_t* d_nids, double* d_dists, uint64_t* n_pairs,
                        int64_t* next_cursor, void* stream);

/*
 * The whole join to host memory, for results larger than device memory
 * (Sec. 3.2's scheme): batches of at most batch_pairs pairs (0: 10^8, the
 * paper's buffer size) are written on n_streams streams (0: 3, at most 8)
 * in turn, each batch copied to pinned host buffers of its stream while the
 * next batches are computed, and handed to `consume` on the calling thread,
 * in batch order (the order of knn_eps_join_device's batches from cursor 0).
 * The buffers passed to consume hold n_pairs entries and are valid until it
 * returns.  consume returns 0 to go on; any other value stops the join
 * (KNN_ECANCELED).  Device memory: about 16 * batch_pairs * n_streams bytes
 * plus the level; pinned host memory the same (batch_pairs is capped at the
 * result size).  The streams and both kinds of buffers stay with the index's
 * state for later calls (freed as the level is).  Blocks until done.
 * stats (may be NULL) receives the timings below.
 */
typedef int (*knn_eps_consumer)(const int32_t* qids, const int32_t* nids, const double* dists,
                                uint64_t n_pairs, void* user);
typedef struct knn_eps_join_stats {
  uint64_t n_pairs;   /* pairs of the whole join */
  int64_t n_batches;  /* batches handed to the consumer */
  double ms_total;    /* wall time of the call */
  double ms_count;    /* level and exact counts (part of ms_total) */
  double ms_wait;     /* host time spent waiting for batches to arrive */
  double ms_consume;  /* host time inside the consumer */
} knn_eps_join_stats;
int knn_eps_join(knn_index* idx, double eps, uint64_t batch_pairs, int32_t n_streams,
                 knn_eps_consumer consume, void* user, knn_eps_join_stats* stats);

/* Frees the level and counts of the distance similarity join. */
int knn_eps_join_release(knn_index* idx);

/* Frees the index and its device memory.  NULL is a no-op. */
void knn_destroy_index(knn_index* idx);

/* Thread-local message of the last error ("" if none). */
const char* knn_last_error(void);

/* Basic facts about an index. */
typedef struct knn_index_info {
  int64_t n_points;
  int32_t dims;
  int32_t device;
  double lo[KNN_MAX_DIMS];
  double hi[KNN_MAX_DIMS];
  double eps_mean;        /* Sec. 4.4 */
  int32_t n_bins;
  int32_t n_sample;
  int64_t device_bytes;   /* device memory held by the index right now */
} knn_index_info;
int knn_index_info_get(const knn_index* idx, knn_index_info* out);

/*
 * The search-distance sampling an index holds (Sec. 4.4), read only, for
 * inspection and testing.  Any output pointer may be NULL.
 *   hist_sample  host, knn_index_info.n_sample entries: ids of the
 *                histogram's sample points, increasing.
 *   mean_sample  host, up to KNN_MAX_MEAN_SAMPLE entries: ids of the eps_mean
 *                sample, increasing; their number goes to *n_mean.
 *   counts       host, knn_index_info.n_bins entries: distances per bin (not
 *                cumulative), bin b = [b, b+1) * bin_width.  eps_min(K) for
 *                any K <= KNN_MAX_K reads only the bins up to the first one
 *                whose cumulative count reaches KNN_MAX_K per sample point;
 *                the counts are exact up to that bin (or a few bins beyond
 *                it) and 0 after it (all bins are exact when no bin reaches
 *                it).
 *   bin_width    eps_mean / n_bins.
 * How the samples are drawn (so that they can be reproduced): SplitMix64
 * (Steele, Lea, Flood, OOPSLA 2014) outputs reduced modulo N, repeats
 * skipped, until enough distinct ids are held, then sorted (every id when the
 * sample would hold N or more).  The eps_mean sample holds
 * min(max(round(mean_frac * N), min_mean_sample), N, KNN_MAX_MEAN_SAMPLE)
 * ids drawn from the state `seed`; the histogram sample n_sample ids drawn
 * from the state seed ^ 0x5DEECE66D.
 * Errors: KNN_EINVAL (idx NULL).
 */
#define KNN_MAX_MEAN_SAMPLE 20000
int knn_index_sampling_get(const knn_index* idx, int64_t* hist_sample, int64_t* mean_sample,
                           int64_t* n_mean, uint64_t* counts, double* bin_width);

/* ------------------------------------------------------------------------
 * Autotuner.  The level-0 cell side (as a multiple of eps_min(K)) and the
 * geometric growth of the cell side between levels decide how many queries
 * fail at each level and how many candidates the rest scan; the best
 * setting depends on the data.  knn_autotune measures joins of (idx, K) on
 * a grid of both, keeps the fastest in a process-wide cache keyed by the
 * workload class (dims, K rounded to a power of two, N to a power of 4), and
 * later joins whose options leave w_factor / growth zero use it.
 * ------------------------------------------------------------------------ */
typedef struct knn_autotune_result {
  double w_factor;    /* chosen level-0 cell side / eps_min(K) */
  double growth;      /* chosen geometric growth of the cell side */
  double ms_best;     /* best join time measured (ms) */
  double ms_default;  /* join time of the untuned default (ms) */
  int32_t trials;     /* settings measured */
  int32_t linear_levels; /* chosen linear growths before the geometric ones
                            (0 or 1; -1 in the cache means none) */
  double tail_pairs;     /* chosen brute-force tail budget (pairs) */
  int32_t lanes_shift;   /* chosen shift of the lanes-per-query rule (x 2^shift) */
  int32_t zorder;        /* chosen level structure: 1 Z-order levels, -1 row-major */
  int32_t queue_pops;    /* chosen pops per wavefront and queue of the persistent
                            search (the automatic queue_grain rule) */
} knn_autotune_result;
/* Runs on `stream` (device scratch allocated internally); blocks. */
int knn_autotune(knn_index* idx, int32_t K, void* stream, knn_autotune_result* out);
/* Save / load the cache as text ("dims kbucket nbucket w_factor growth
 * lanes linear tail_pairs lanes_shift zorder pops" per line; lines of the
 * older 10-field form load with pops 0); path NULL =
 * $KNN_AUTOTUNE_CACHE. */
int knn_autotune_save(const char* path);
int knn_autotune_load(const char* path);

/* Upper bound of the device bytes one eager self-join of (idx, K) with host
 * outputs allocates beyond the index, the device cache's rounding and reuse
 * slack included (the serving loop's admission size).  A join captured in a
 * HIP graph (use_graph) keeps every level's scratch and may hold more. */
int knn_join_footprint(const knn_index* idx, int32_t K, uint64_t* bytes);

/* eps_min(K) of Sec. 4.4 from the index's cumulative distance histogram:
 * the midpoint of the first bin whose cumulative count reaches K per sample
 * point, or eps_mean if none does. */
int knn_eps_min(const knn_index* idx, int32_t K, double* eps_min);

/*
 * Builds the grid level of cell side `cell_width` (Sec. 3.1) and copies it
 * to host arrays, for inspection and testing.  Any output pointer may be
 * NULL.  Sizes: sorted_keys, perm: N; cell_keys: N (first *n_cells used);
 * cell_start: N+1 (first *n_cells+1 used); ranges: N * 3^(dims-1) * 2 (first
 * *n_cells * 3^(dims-1) * 2 used); grid_dims: dims.
 * Layout: the key of a point is row-major over its cell coordinates
 * floor((x_j - lo_j) * inv_w), inv_w = 1/cell_width, last dimension fastest;
 * points are sorted by key, stably in their id; perm[p] is the id of the
 * point at sorted position p; cell c holds sorted positions
 * [cell_start[c], cell_start[c+1]); ranges[(c*R + r)*2 + {0,1}] is the
 * half-open sorted range of row segment r (offsets o_0..o_{n-2} in
 * {-1,0,1}, o_0 slowest, last coordinate within one of c's), (0,0) if empty.
 */
int knn_grid_export(knn_index* idx, double cell_width, uint64_t* sorted_keys,
                    int32_t* perm, uint64_t* cell_keys, uint32_t* cell_start,
                    uint32_t* ranges, int64_t* grid_dims, int64_t* n_cells);

/*
 * The two sampling kernels of Sec. 4.4 on caller-chosen samples, device
 * memory throughout (used by the index build; exposed for testing).
 *   d_D        device, N x dims fp64 row-major.
 *   d_sample   device, ns int64 point ids (each in [0, N)).
 * knn_sample_mean_dist: mean distance over the unordered pairs of the
 *   sample; *mean is written to host memory (the call synchronises).
 * knn_dist_histogram: counts, for every sample point s and every point
 *   j != s, the distance d = sqrt(d^2(s,j)) into bin floor(d * inv_bin_width)
 *   when that bin is < n_bins; d_counts (device, n_bins uint64) is
 *   overwritten.  Asynchronous on `stream`.
 */
int knn_sample_mean_dist(const double* d_D, int64_t n_points, int32_t dims,
                         const int64_t* d_sample, int64_t ns, double* mean,
                         void* stream);
int knn_dist_histogram(const double* d_D, int64_t n_points, int32_t dims,
                       const int64_t* d_sample, int64_t ns, double inv_bin_width,
                       int32_t n_bins, uint64_t* d_counts, void* stream);

/* ------------------------------------------------------------------------
 * Serving: a request loop over indexes resident in device memory.
 * Requests (dataset, K) are admitted while their device footprint fits the
 * memory budget and fewer than max_inflight run; admitted requests run
 * concurrently on their own streams, so work of requests that arrive while
 * others run overlaps on the device.  Results are the same as a solo
 * knn_self_join on the same index and K (bit for bit).
 * ------------------------------------------------------------------------ */
typedef struct knn_server knn_server;

typedef struct knn_server_opts {
  uint64_t mem_budget_bytes; /* device bytes for in-flight requests [8 GiB] */
  int32_t max_inflight;      /* concurrent requests [4] */
  int32_t max_queue;         /* pending requests before submit returns KNN_EBUSY [4096] */
  int32_t device;            /* < 0 = current device */
} knn_server_opts;

typedef struct knn_server_stats {
  int64_t submitted;
  int64_t completed;
  int64_t failed;
  double p50_ms;           /* latency submit -> results in host memory */
  double p99_ms;
  double mean_ms;
  double max_ms;
  double queries_per_s;    /* completed queries (points) / busy wall time */
  double requests_per_s;
  uint64_t peak_bytes;     /* peak admitted footprint */
  int32_t peak_inflight;
} knn_server_stats;

int knn_server_create(const knn_server_opts* opts, knn_server** out);
/* Registers a built index (borrowed: it must outlive the server). */
int knn_server_add_dataset(knn_server* srv, knn_index* idx, int32_t* dataset_id);
/* Queues a self-join of dataset `dataset_id` with K neighbours into host
 * arrays ids/dists (N x K, owned by the caller, untouched until completion).
 * ids and dists both NULL make a latency-only request: the join runs in full
 * and its results are discarded on the device (load generation).
 * Returns KNN_EBUSY when the pending queue is full; a request that does not
 * fit the free budget waits in the queue (it is not rejected).  A request
 * whose footprint exceeds the whole budget is rejected with KNN_EINVAL. */
int knn_server_submit(knn_server* srv, int32_t dataset_id, int32_t K, int32_t* ids,
                      double* dists, int64_t* ticket);
/* Waits for a ticket: KNN_OK when done, KNN_ETIMEOUT, or the request's own
 * error code.  timeout_us < 0 waits forever. */
int knn_server_wait(knn_server* srv, int64_t ticket, int64_t timeout_us);
int knn_server_stats_get(knn_server* srv, knn_server_stats* out);
/* Waits for all requests, then frees the server. NULL is a no-op. */
void knn_server_destroy(knn_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* KNNJOIN_H */
