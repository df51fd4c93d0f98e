// kernels.hpp -- host-side launchers of the HIP kernels (gfx950).
#pragma once

#include "common.hpp"

namespace knn {

constexpr int kMaxDims = KNN_MAX_DIMS;
constexpr int kXcds = 8;  // accelerator complex dies of an MI355X, each with its own L2

// Device counters of a search level, each on a 128-byte line of its own:
// device-scope atomics on one line serialize, and the queue heads of the
// eight XCDs are hit concurrently.
constexpr int kLineInts = 32;
constexpr int kFailSlot = kXcds * kLineInts;       // failed queries
constexpr int kRefineSlot = kFailSlot + kLineInts;   // refinement rounds (diagnostics)
constexpr int kHeavySlot = kRefineSlot + kLineInts;  // heavy queries
constexpr int kHeavyFailSlot = kHeavySlot + kLineInts;      // of which failed (diagnostics)
constexpr int kHeavyCandSlot = kHeavyFailSlot + kLineInts;  // their candidates (uint64)
constexpr int kWalkErrSlot = kHeavyCandSlot + kLineInts;    // candidate-list overruns
constexpr int kSpecSlot = kWalkErrSlot + kLineInts;          // speculations that held
constexpr int kCandSumSlot = kSpecSlot + kLineInts;          // candidate sum, max (2 x u64)
constexpr int kCounterInts = kCandSumSlot + kLineInts;

// Geometry of one grid level (Sec. 3.1): cell side 1/inv_w, origin lo.
struct GridGeom {
  int32_t dims;
  double lo[kMaxDims];
  double inv_w;
  int64_t g[kMaxDims];        // cells per dimension
  uint64_t stride[kMaxDims];  // key stride per dimension (last = 1)
  int32_t key_bits;           // bits of the largest key
  int64_t g_max;
  // Z-order levels: keys interleave the bits of the cell coordinates (bit b
  // of dimension j at position b*dims + dims-1-j), zbits bits per dimension
  // at this level.  The cell key of a point at level L is its level-0 key
  // shifted right by zshift = dims*L, so one sort of the level-0 keys orders
  // the points for every level.  zbits = 0: row-major keys (stride).
  int32_t zbits;
  int32_t zshift;
};

// ---- elementwise / reductions (grid.hip) ----
// Row-major N x n (AoS) -> SoA X[j*N + i]; counts non-finite coordinates into *bad.
void launch_aos_to_soa(const double* D, int64_t N, int n, double* X, uint32_t* bad,
                       hipStream_t s);
// Per-dimension min/max of SoA X into lo[n], hi[n] (device).  part: scratch of
// at least 2*n*kBoundsBlocks doubles.
constexpr int kBoundsBlocks = 512;
void launch_bounds(const double* X, int64_t N, int n, double* part, double* lo, double* hi,
                   hipStream_t s);

// ---- scan (grid.hip) ----
// Exclusive scan of n uint32 values (out may equal in) in one pass.  If
// total != nullptr the sum of all values is written there (device).  state:
// state_elems >= scan_state_elems(n) uint32 owned by one stream's work,
// zero-filled once when allocated and kept between scans (it carries the
// scans' epoch and ticket); state[2] counts look-back errors (must stay 0).
// Users of the state take tiles of at least kLbMinTile elements.  Beyond the
// look-back words the state holds a tile area for compactions of up to n
// elements (counts, then their scan, then the writes: tile counts and ballot
// masks, rewritten by every compaction).
constexpr int kLbMinTile = 2048;
size_t scan_state_elems(int64_t n);
// The tile area's first `words` uint32 (8-byte aligned) of a state of
// state_elems words made by scan_state_elems for at least the compaction's n.
uint32_t* scan_tile_area(uint32_t* state, int64_t state_elems, int64_t words);
void launch_exclusive_scan(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total,
                           uint32_t* state, int64_t state_elems, hipStream_t s);

// ---- radix sort (grid.hip) ----
// Stable LSD sort of (key, val) pairs by the low `bits` bits of the keys.
// keys/vals hold the input; keys2/vals2 are same-size scratch; tmp:
// radix_tmp_elems(n) uint32; state: scan state (launch_exclusive_scan).
// Returns true when the sorted output ended up in keys2/vals2 (odd number of
// passes), false when it is in keys/vals.
size_t radix_tmp_elems(int64_t n);
bool radix_sort_pairs(uint64_t* keys, int32_t* vals, uint64_t* keys2, int32_t* vals2,
                      int64_t n, int bits, uint32_t* tmp, uint32_t* state, int64_t state_elems,
                      hipStream_t s);
// The same for keys of at most 32 bits held as uint32 (a third less traffic
// per pass than 64-bit keys).
bool radix_sort_pairs(uint32_t* keys, int32_t* vals, uint32_t* keys2, int32_t* vals2,
                      int64_t n, int bits, uint32_t* tmp, uint32_t* state, int64_t state_elems,
                      hipStream_t s);

// ---- grid level construction (grid.hip) ----
// keys[i] = cell key of point i (original order, SoA X; row-major or Z-order
// as gg says); vals[i] = i.
void launch_cell_keys(const double* X, int64_t N, const GridGeom& gg, uint64_t* keys,
                      int32_t* vals, hipStream_t s);
// uint32 keys (gg.key_bits <= 32)
void launch_cell_keys(const double* X, int64_t N, const GridGeom& gg, uint32_t* keys,
                      int32_t* vals, hipStream_t s);
// From sorted keys (cell starts counted per tile, the counts scanned, then
// written): the cell table.  cell_of (N), cell_key (N),
// cell_start (N+1), d_M (device scalar) written.  state: scan state and its
// tile area (flags unused).  shift: the cells are those of sorted_keys >>
// shift (a Z-order level above the one the keys were sorted for); cell_key
// holds the shifted keys (64-bit whatever the width of sorted_keys).
void build_cell_table(const uint64_t* sorted_keys, int64_t N, uint32_t* flags,
                      uint32_t* cell_of, uint64_t* cell_key, uint32_t* cell_start,
                      uint32_t* d_M, uint32_t* state, int64_t state_elems, hipStream_t s,
                      int shift = 0);
void build_cell_table(const uint32_t* sorted_keys, int64_t N, uint32_t* flags,
                      uint32_t* cell_of, uint64_t* cell_key, uint32_t* cell_start,
                      uint32_t* d_M, uint32_t* state, int64_t state_elems, hipStream_t s,
                      int shift = 0);
// list[i] = perm[list[i]] for i < n (sorted positions -> point ids).
void launch_pos_to_id(int32_t* list, int64_t n, const int32_t* perm, hipStream_t s);
// keys[p] = cell key of the point at sorted position p of the previous level
// (point-major Xs), vals[p] = p.
void launch_cell_keys_points(const double* Xs, int64_t N, const GridGeom& gg, uint64_t* keys,
                             int32_t* vals, hipStream_t s);
// perm[p] = perm_prev[pos[p]], point p of Xs = point pos[p] of Xs_prev.
void launch_gather_prev(const double* Xs_prev, const int32_t* perm_prev, const int32_t* pos,
                        int64_t N, int n, double* Xs, int32_t* perm, hipStream_t s);
// Doubles per point in the sorted coordinate array: n rounded up to even, so
// a point is whole 16-byte pairs (a padding coordinate is 0).
inline constexpr int point_stride(int n) { return (n + 1) & ~1; }
// Xs[p*S + j] = XA[perm[p]*n + j] for j < n, Xs[p*S + n] = 0 when n is odd
// (S = point_stride(n); XA row-major N x n)
void launch_gather_points(const double* XA, const int32_t* perm, int64_t N, int n, double* Xs,
                          hipStream_t s);
// Row table: for every row of the grid (the cells sharing coordinates
// 0..n-2, row = key / g_last), [rowtab[row].x, rowtab[row].y) = its
// non-empty cells (empty rows: 0, 0).  rows entries.
void launch_row_table(const uint64_t* cell_key, const uint32_t* d_M, int64_t N, uint64_t g_last,
                      uint2* rowtab, int64_t rows, hipStream_t s);
// Dense key -> cell lookup table (table_size entries, set to ~0 where empty).
void launch_dense_table(const uint64_t* cell_key, const uint32_t* d_M, int64_t N,
                        uint32_t* table, int64_t table_size, hipStream_t s);
// Row-segment neighbour ranges of every cell: the non-empty ones of the
// 3^(n-1) segments, compacted in segment order into
// ranges[(c*R + i)*4 + {0..3}] = (start, mid0, mid1, end): the segment's
// points, split where the last cell coordinate reaches the cell's and where
// it passes it; their segment index in rslot[c*R + i], their number in
// nrng[c], and the candidate count (sum of lengths) in cand_count[c].
// cell_active (nullable): only the cells flagged with active_tag get ranges
// (the others' entries are left as they were).
void launch_neighbor_ranges(const double* Xs, int64_t N, const uint32_t* cell_start,
                            const uint64_t* cell_key, const uint32_t* d_M,
                            const uint32_t* dense /*nullable*/, const uint2* rowtab /*nullable*/,
                            const uint8_t* cell_active /*nullable*/, uint8_t active_tag,
                            const GridGeom& gg, uint32_t* ranges, uint8_t* rslot,
                            uint32_t* nrng, uint32_t* cand_count, hipStream_t s);
// Z-order level: neighbour ranges of the cells flagged with active_tag
// (every cell when cell_active is NULL), one entry per non-empty cell of the
// 3^n block, compacted in block order (offsets o_0..o_{n-1} in {-1,0,1}, the
// last fastest) in the row-segment format above: rslot = the offsets of
// dimensions 0..n-2, and the cell is the lower part (o_{n-1} = -1: start,
// end, end, end), the middle (0: start, start, end, end) or the upper part
// (+1: start, start, start, end) of its segment, so the search's pruning
// reads it unchanged.  Neighbours are found by a galloping search outward
// from the cell's own position in cell_key (Z-order neighbours are mostly
// close in the sorted cell table).  ranges: R = 3^n entries per cell.
// dense (nullable, dense_size >= the level's prod(g) entries, contents
// arbitrary): first filled with each cell's position at its row-major index,
// then neighbours are looked up there (one load and a key check) instead of
// by the galloping search.
void launch_neighbor_ranges_z(const uint32_t* cell_start, const uint64_t* cell_key,
                              const uint32_t* d_M, int64_t N, const uint8_t* cell_active,
                              uint8_t active_tag, const GridGeom& gg, uint32_t* dense,
                              int64_t dense_size, uint32_t* ranges, uint8_t* rslot,
                              uint32_t* nrng, uint32_t* cand_count, hipStream_t s);
// A Z-order level's ranges without its cell table, for few active queries:
// slot i (the i-th active sorted position q, the first min(n_active,
// *n_dev) of the list) gets the ranges of q's 3^n block in the format above,
// each neighbour cell's points found by binary search in the sorted level-0
// keys (keys >> gg.zshift == the cell's key); cell_of[q] = i, nrng and
// cand_count by slot, and *d_M = the number of slots.
void launch_sparse_ranges_z(const uint64_t* sorted_keys, int64_t N, const int32_t* active,
                            int64_t n_active, const uint32_t* n_dev, const GridGeom& gg,
                            uint32_t* ranges, uint8_t* rslot, uint32_t* nrng,
                            uint32_t* cand_count, uint32_t* cell_of, uint32_t* d_M,
                            hipStream_t s);
void launch_sparse_ranges_z(const uint32_t* sorted_keys, int64_t N, const int32_t* active,
                            int64_t n_active, const uint32_t* n_dev, const GridGeom& gg,
                            uint32_t* ranges, uint8_t* rslot, uint32_t* nrng,
                            uint32_t* cand_count, uint32_t* cell_of, uint32_t* d_M,
                            hipStream_t s);
// flags[cell_of[active[i]]] = tag for every active query (n_dev non-NULL:
// the first min(n_active, *n_dev) of the list).
void launch_mark_cells_of(const int32_t* active, int64_t n_active, const uint32_t* cell_of,
                          uint8_t* flags, uint8_t tag, hipStream_t s,
                          const uint32_t* n_dev = nullptr);

// ---- work items (grid.hip) ----
// Work item i = G consecutive active slots.  Its estimate is the sum of the
// candidate counts of its queries' cells; its sort key is (XCD chunk, density
// class): chunk = i*8/n_items (contiguous in cell order), class = half-octaves
// of the estimate, densest first.  A stable sort keeps cell order inside.
void launch_item_keys(const int32_t* active /*nullable: identity*/, int64_t n_active,
                      int G, const uint32_t* cell_of, const uint32_t* cand_count,
                      uint64_t* keys, int32_t* vals, int64_t n_items, hipStream_t s);
// sum[0] = total and sum[1] = maximum of the candidate counts of the cells of
// the active queries (uint64, device).
void launch_active_cand_sum(const int32_t* active /*nullable*/, int64_t n_active,
                            const uint32_t* cell_of, const uint32_t* cand_count, uint64_t* sum,
                            hipStream_t s);
// list[0 .. *count) = the active sorted positions whose cell has at least
// heavy_min candidates (order unspecified); *cand_sum += their candidates.
void launch_heavy_list(const int32_t* active /*nullable*/, int64_t n_active,
                       const uint32_t* cell_of, const uint32_t* cand_count, uint32_t heavy_min,
                       int32_t* list, int32_t* count, unsigned long long* cand_sum,
                       hipStream_t s);
// failed[e] = tag for the entries e of the failure list (ids, or sorted
// positions on Z-order levels; the next level's active queries carry that
// level's tag).
void launch_mark_failed(const int32_t* fail_list, const int32_t* d_fail_count,
                        int64_t max_fail, uint8_t* failed, uint8_t tag, hipStream_t s);
// out = the sorted positions p with failed[perm[p]] == tag (perm NULL:
// failed[p] == tag; at_least: >= tag instead of ==), in order; their
// number to *count (device).  One pass (scan state as launch_exclusive_scan).
void launch_active_list(const uint8_t* failed, uint8_t tag, const int32_t* perm, int64_t N,
                        int32_t* out, uint32_t* count, uint32_t* state, int64_t state_elems,
                        hipStream_t s, bool at_least = false, int32_t base = 0);
// (base: added to every position written, for flags of a sub-array.)
// Ranges of external queries: for the active queries q (point positions
// base + i of Xs, i in [0, count of queries)), their 3^n block's ranges in
// the level's cell table, in the format of launch_neighbor_ranges (zl:
// launch_neighbor_ranges_z), written to slot i (ranges[i*R...], rslot, nrng,
// cand_count), and cell_of[q] = i.
// (n_dev non-NULL: the list's count is min(n_active, *n_dev); list entries
// outside [base, base + nq) are skipped.)
void launch_query_ranges(const double* Xs, const int32_t* active, int64_t n_active,
                         const uint32_t* n_dev, int64_t base, int64_t nq,
                         const uint32_t* cell_start, const uint64_t* cell_key,
                         const uint32_t* d_M, const uint32_t* dense, const uint2* rowtab,
                         const GridGeom& gg, bool zl, uint32_t* cell_of, uint32_t* ranges,
                         uint8_t* rslot, uint32_t* nrng, uint32_t* cand_count, hipStream_t s);
// out[i] = base + i for i < n.
void launch_iota(int32_t* out, int64_t n, int32_t base, hipStream_t s);
// Zeroes `bytes` bytes at p (4-byte aligned) with a kernel, not a memset node.
void launch_zero(void* p, size_t bytes, hipStream_t s);

// ---- search-distance sampling (eps.hip) ----
// Partial sums of pair distances inside the sample: one double per block of
// rows; returns the number of partials written to part (host reads them).
// SX: scratch of ns * n doubles (the sample's coordinates, gathered first).
int launch_sample_pair_sums(const double* X, int64_t N, int n, const int64_t* sample,
                            int64_t ns, double* SX, double* part, hipStream_t s);
// Histogram of the distances from the sample points to the points p =
// 0, pstride, 2 pstride, ... of X (all points when pstride = 1), bins of width
// 1/inv_bw; only the first count_bins bins are counted (the rest stay 0;
// count_bins <= 0: all n_bins).  max_abs: a bound on every |coordinate|
// (< 0: unknown), which lets far pairs be rejected in single precision first
// (the counts are the same).
void launch_dist_histogram(const double* X, int64_t N, int n, const int64_t* sample,
                           int64_t ns, double inv_bw, int n_bins, uint64_t* counts,
                           hipStream_t s, int count_bins = 0, int64_t pstride = 1,
                           double max_abs = -1.0);

// ---- distance similarity self-join (epsjoin.hip) ----
// One row-major grid level (ranges / rslot / nrng, R segments per cell) whose
// cell side w covers the search distance, and the squared-distance limit t
// (the largest d^2 whose correctly rounded square root is <= eps).
// Count pass: counts[slot] = the points j != p of position p = slot * stride
// with d^2(p, j) <= t.  Write pass (counts of every position, off = their
// exclusive prefix, N + 1 entries): the pairs of the positions [first, last)
// at out + off[p] - off[first], as (id of p, id of j, sqrt(d^2)).
struct EpsPassArgs {
  const double* Xs;        // sorted coordinates, point-major: Xs[p*point_stride(n) + j]
  int64_t N;
  const int32_t* perm;     // sorted position -> id
  const uint32_t* cell_of;
  const uint32_t* ranges;
  const uint8_t* rslot;
  const uint32_t* nrng;
  int32_t R;
  GridGeom gg;
  double w;                // the level's cell side
  double margin;           // rounding of a cell coordinate, in cells
  double t;
  int64_t stride = 1;      // count pass: every stride-th position
  int64_t first = 0, last = 0;  // write pass: sorted positions
  uint32_t* counts = nullptr;
  const uint64_t* off = nullptr;
  int32_t* out_q = nullptr;
  int32_t* out_j = nullptr;
  double* out_d = nullptr;
};
void launch_eps_count(const EpsPassArgs& a, hipStream_t s);
void launch_eps_write(const EpsPassArgs& a, hipStream_t s);
// Elements of the tile array launch_offsets needs for n counts.
int64_t eps_scan_tiles(int64_t n);
// off[0..n] = exclusive prefix of counts[0..n) (off[n] = the total).
void launch_offsets(const uint32_t* counts, int64_t n, uint64_t* tiles, uint64_t* off,
                    hipStream_t s);
// Greedy batches of positions from `first` whose pairs fit cap: bounds[2b] =
// end position of batch b, bounds[2b+1] = its end offset; status[0] = the
// batches written (at most maxb; -1: one position alone exceeds cap, its
// pair count in status[2]), status[1] = off[first].
void launch_batch_bounds(const uint64_t* off, int64_t n, int64_t first, uint64_t cap,
                         int64_t maxb, int64_t* bounds, int64_t* status, hipStream_t s);
// out[perm[p]] = counts[p].
void launch_counts_by_id(const uint32_t* counts, const int32_t* perm, int64_t n, int32_t* out,
                         hipStream_t s);

// ---- search (search.hip) ----
struct SearchArgs {
  const double* Xs;        // sorted coordinates, point-major: Xs[p*point_stride(n) + j]
  int64_t N;
  const int32_t* perm;     // sorted position -> point id
  const uint32_t* cell_of; // sorted position -> cell
  const uint32_t* ranges;  // cell*R*4 compacted non-empty row segments (start, mid0, mid1, end)
  const uint8_t* rslot;    // cell*R: segment index of each compacted range
  const uint32_t* nrng;    // non-empty segments per cell
  const uint32_t* cand;    // candidates per cell
  const int32_t* active;   // active sorted positions (nullptr: identity)
  int64_t n_active;
  const int32_t* order;    // item order (nullptr: identity)
  int64_t n_items;
  int64_t item_base;       // first item of this launch (schedule 1)
  int32_t* head;           // persistent work-queue heads: XCD x at head[x * kLineInts]
  int64_t qbeg[kXcds + 1]; // queue x = order positions [qbeg[x], qbeg[x+1])
  int32_t grain;           // items claimed per queue pop
  int32_t persistent;
  int32_t share_lists;     // wavefronts whose queries share a cell walk one list
  int32_t zl;              // Z-order level: 3^n single-cell ranges per cell (else 3^(n-1))
  int32_t self_in_list;    // the query is a point of its own list (self-join), counted and
                           // taken back; 0: external queries, not in any list
  double lo[kMaxDims];
  double inv_w;
  double w;                // fl(1 / inv_w)
  int64_t g[kMaxDims];
  double margin;           // relative shrink of the covered radius (rounding)
  int32_t K;
  int32_t cap;             // per-query survivor buffer entries (>= K)
  int32_t* out_ids;        // N x K, row = point id
  double* out_d;
  int32_t* fail_list;      // point ids of failed queries (sorted positions if fail_pos)
  int32_t* fail_count;
  int32_t fail_pos;        // Z-order levels: failures listed by sorted position
  int32_t* refine_count;   // diagnostics: refinement rounds executed
  uint32_t heavy_min;      // > 0: k_search leaves queries with this many candidates or more
  const int32_t* heavy;    // to k_search_heavy: their sorted positions
  const int32_t* n_heavy;  // and their number (device)
  int32_t* heavy_fail;     // failures among them (diagnostics)
  int32_t* walk_error;     // candidate-list walks that ran past their list (must stay 0)
  int32_t spec_slots;      // speculative survivor slots per query (0: off)
  int32_t* spec_count;     // diagnostics: queries whose speculation held
  double spec_coef;        // speculation limit = spec_coef * C^(-2/n), C = candidates of the cell
};
// Deferral filter of a level's active queries: a query whose K-th squared
// distance, predicted from its 3^n block's density, exceeds its covered
// radius^2 by the defer margin goes straight to the failure list; the others
// form the level's new active list (cell order kept).
struct DeferArgs {
  const double* Xs;
  const int32_t* perm;
  const uint32_t* cell_of;
  const uint32_t* cand;       // candidates per cell
  const int32_t* active;      // active sorted positions (nullptr: identity)
  int64_t n_active;
  const uint32_t* n_active_dev;  // nullable: the count is min(n_active, *n_active_dev)
  // Z-order levels, before the neighbour ranges exist: with cell_key set, the
  // density comes from the query's parent group (the 2^n cells whose keys
  // agree above the last n bits, a cell of twice the side) instead of cand
  const uint64_t* cell_key;
  const uint32_t* cell_start;
  const uint32_t* d_M;
  int32_t fail_pos;           // deferred queries listed by sorted position (else id)
  // Z-order levels: with failed set, a deferred query is not listed but
  // flagged for the first level whose cell side could hold its predicted
  // K-th distance (1.5 times the side at least covers that distance):
  // failed[q] = that level (at most top_level) and pending[that level] += 1
  uint8_t* failed;
  uint32_t* pending;
  int32_t level;
  int32_t top_level;
  double lo[kMaxDims];
  double inv_w;
  double w;
  int64_t g[kMaxDims];
  double margin;
  double defer_coef;          // deferred when defer_coef * C^(-2/n) > thr
  int32_t* out_active;        // kept positions
  uint32_t* out_count;        // their number (device)
  int32_t* fail_list;         // deferred ids appended here
  int32_t* fail_count;
  unsigned long long* cand_sum;  // nullable: [0] += candidates of kept queries, [1] = max
                                 // (pre-zeroed)
  uint32_t* state;            // scan state (launch_exclusive_scan) and its tile area
  int64_t state_elems;
  // set by launch_defer_filter (carved from the tile area)
  uint32_t* tile_counts;
  uint32_t* tile_masks;
};
void launch_defer_filter(const DeferArgs& a, int dims, hipStream_t s);

// Returns the number of waves per block used.
void launch_search(const SearchArgs& a, int dims, int lanes_per_query, int grid_blocks,
                   hipStream_t s);
// One workgroup of kHeavyThreads per query for the heavy queries a.heavy[0 ..
// *a.n_heavy), grid-stride over them (blocks: any positive count).
constexpr int kHeavyThreads = 1024;
void launch_search_heavy(const SearchArgs& a, int dims, int blocks, hipStream_t s);
// Dynamic LDS bytes per wave for a given (lanes_per_query, cap); zl: a
// Z-order level (3^n range slots per cell).
size_t search_lds_per_wave(int dims, int lanes_per_query, int cap, bool zl = false);
// Speculative survivor slots per query for a given (lanes_per_query, cap), and
// the coefficient of the predicted K-th squared distance at cell side w.
int search_spec_slots(int dims, int lanes_per_query, int cap, bool zl = false);
double search_density_coef(int dims, int K, double w);
int search_waves_per_block(int dims, int lanes_per_query, int cap, bool zl = false);
// Resident blocks per CU of the search kernel (occupancy API).
int search_blocks_per_cu(int dims, int lanes_per_query, int cap, bool zl = false);
// Largest dimension count with Z-order levels.
constexpr int kZMaxDims = 4;

}  // namespace knn
