// index.hip -- host runtime of the library: index build with the sampling of
// Sec. 4.4, grid levels (Sec. 3.1, built on the GPU as in Sec. 4.6), the
// GPU-only level loop of Alg. 1 (failures re-queued, cell side grown,
// re-index), and the C ABI of knnjoin.h.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>

#include "autotune.hpp"
#include "index.hpp"
#include "tail.hpp"

namespace knn {

static thread_local std::string g_last_error;
void set_last_error(const std::string& msg) { g_last_error = msg; }

namespace {

// SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
// generators", OOPSLA 2014): the counter-based generator of the sampling.
struct SplitMix64 {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
};

// `count` distinct ids in [0, N), drawn with SplitMix64 (all ids if count >= N).
std::vector<int64_t> sample_ids(int64_t N, int64_t count, uint64_t seed) {
  std::vector<int64_t> out;
  if (count >= N) {
    out.resize(N);
    for (int64_t i = 0; i < N; ++i) out[i] = i;
    return out;
  }
  SplitMix64 g{seed};
  // ids seen so far: open addressing, linear probing, at most a quarter full
  size_t cap = 16;
  while (cap < (size_t)count * 4) cap <<= 1;
  std::vector<uint64_t> seen(cap, ~0ull);
  out.reserve((size_t)count);
  while ((int64_t)out.size() < count) {
    const uint64_t id = g.next() % (uint64_t)N;
    size_t h = (size_t)((id * 0x9E3779B97F4A7C15ull) >> 20) & (cap - 1);
    while (seen[h] != ~0ull && seen[h] != id) h = (h + 1) & (cap - 1);
    if (seen[h] == ~0ull) {
      seen[h] = id;
      out.push_back((int64_t)id);
    }
  }
  // ascending: LSD radix sort, 11 bits a pass (ids < N < 2^31)
  std::vector<int64_t> tmp(out.size());
  for (int sh = 0; sh < 33; sh += 11) {
    size_t cnt[2049] = {};
    for (int64_t v : out) ++cnt[((uint64_t)v >> sh & 2047) + 1];
    for (int b = 0; b < 2048; ++b) cnt[b + 1] += cnt[b];
    for (int64_t v : out) tmp[cnt[(uint64_t)v >> sh & 2047]++] = v;
    out.swap(tmp);
  }
  return out;
}

int current_device() {
  int d = 0;
  KNN_HIP(hipGetDevice(&d));
  return d;
}

int cu_count(int dev) {
  int v = 0;
  KNN_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev));
  return v > 0 ? v : 1;
}

int64_t pow3(int e) {
  int64_t r = 1;
  for (int i = 0; i < e; ++i) r *= 3;
  return r;
}

}  // namespace

GridGeom make_geom(int n, const double* lo, const double* hi, double& w) {
  GridGeom gg{};
  gg.dims = n;
  double ext = 0;
  for (int j = 0; j < n; ++j) ext = std::max(ext, hi[j] - lo[j]);
  if (!(w > 0) || !std::isfinite(w)) w = ext > 0 ? ext : 1.0;
  for (int attempt = 0; attempt < 200; ++attempt) {
    double inv_w = 1.0 / w;
    bool fits = std::isfinite(inv_w) && inv_w > 0;
    long double prod = 1;
    int64_t gmax = 1;
    for (int j = 0; fits && j < n; ++j) {
      double u = std::floor((hi[j] - lo[j]) * inv_w);
      if (!(u < (double)(1ll << 30))) {
        fits = false;
        break;
      }
      gg.g[j] = (int64_t)u + 1;
      gmax = std::max(gmax, gg.g[j]);
      prod *= (long double)gg.g[j];
    }
    if (fits && prod < (long double)(1ull << 62)) {
      gg.inv_w = inv_w;
      gg.g_max = gmax;
      uint64_t st = 1;
      for (int j = n - 1; j >= 0; --j) {
        gg.stride[j] = st;
        st *= (uint64_t)gg.g[j];
      }
      for (int j = 0; j < n; ++j) gg.lo[j] = lo[j];
      uint64_t maxkey = st - 1;
      int bits = 0;
      while (bits < 64 && (maxkey >> bits) != 0) ++bits;
      gg.key_bits = bits;
      return gg;
    }
    w *= 2;
  }
  throw Error(KNN_EINTERNAL, "could not choose a grid geometry");
}

namespace {

// Geometry of the level-0 Z-order grid of cell side w: row-major sizes, and
// the bits per dimension of the interleaved keys (dims * bits <= 62).  The
// side is enlarged until that fits (a performance policy only).
GridGeom make_geom_z(int n, const double* lo, const double* hi, double& w) {
  for (int attempt = 0; attempt < 200; ++attempt) {
    GridGeom gg = make_geom(n, lo, hi, w);  // may enlarge w for its own limits
    int bits = 0;
    while (bits < 62 && ((gg.g_max - 1) >> bits) != 0) ++bits;
    if (n * bits <= 62) {
      gg.zbits = bits;
      gg.zshift = 0;
      gg.key_bits = n * bits;
      return gg;
    }
    w *= 2;
  }
  throw Error(KNN_EINTERNAL, "could not choose a Z-order grid geometry");
}

// Level L of a Z-order ladder: cell side w0 * 2^L, so inv_w is the level-0
// one times 2^-L exactly and every cell coordinate is the level-0 one shifted
// right by L (floor(u / 2^L) = floor(floor(u) / 2^L) for u >= 0, and scaling
// by a power of two rounds identically).
GridGeom z_level_geom(const GridGeom& g0, int L) {
  GridGeom gg = g0;
  gg.inv_w = std::ldexp(g0.inv_w, -L);
  gg.g_max = 1;
  for (int j = 0; j < g0.dims; ++j) {
    gg.g[j] = ((g0.g[j] - 1) >> L) + 1;
    gg.g_max = std::max(gg.g_max, gg.g[j]);
  }
  uint64_t st = 1;
  for (int j = g0.dims - 1; j >= 0; --j) {
    gg.stride[j] = st;
    st *= (uint64_t)gg.g[j];
  }
  gg.zbits = std::max(g0.zbits - L, 0);
  gg.zshift = g0.dims * std::min(L, g0.zbits);
  gg.key_bits = g0.dims * gg.zbits;
  return gg;
}

// Flag value of a level (> 0) in the failure and active-cell arrays: 1..255.
uint8_t level_tag(int level) { return (uint8_t)(1 + (level - 1) % 255); }

double elapsed_ms(hipEvent_t a, hipEvent_t b) {
  float ms = 0;
  KNN_HIP(hipEventElapsedTime(&ms, a, b));
  return (double)ms;
}

struct Events {
  hipEvent_t e[4] = {nullptr, nullptr, nullptr, nullptr};
  bool on = false;
  explicit Events(bool enable) : on(enable) {
    if (on)
      for (auto& x : e) KNN_HIP(hipEventCreate(&x));
  }
  ~Events() {
    for (auto& x : e)
      if (x) (void)hipEventDestroy(x);
  }
  void rec(int i, hipStream_t s) {
    if (on) KNN_HIP(hipEventRecord(e[i], s));
  }
};

}  // namespace

void copy_to_host(HostStage& st, void* dst, const void* src, size_t bytes, hipStream_t s) {
  const size_t C = HostStage::kStageBytes;
  if (bytes <= C / 4) {  // small: one direct copy
    if (bytes) KNN_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s));
    KNN_HIP(hipStreamSynchronize(s));
    return;
  }
  for (int i = 0; i < 2; ++i) {
    st.buf[i].reserve(C);
    if (!st.ev[i]) KNN_HIP(hipEventCreateWithFlags(&st.ev[i], hipEventDisableTiming));
  }
  const size_t n = (bytes + C - 1) / C;
  auto issue = [&](size_t k) {
    const size_t off = k * C, len = std::min(C, bytes - off);
    KNN_HIP(hipMemcpyAsync(st.buf[k & 1].p, static_cast<const char*>(src) + off, len,
                           hipMemcpyDeviceToHost, s));
    KNN_HIP(hipEventRecord(st.ev[k & 1], s));
  };
  const int nt = (int)std::max(1u, std::min(8u, std::thread::hardware_concurrency()));
  issue(0);
  for (size_t k = 0; k < n; ++k) {
    KNN_HIP(hipEventSynchronize(st.ev[k & 1]));
    if (k + 1 < n) issue(k + 1);
    const size_t off = k * C, len = std::min(C, bytes - off);
    const char* from = st.buf[k & 1].p;
    char* to = static_cast<char*>(dst) + off;
    auto part = [&](int t) {
      const size_t a = len * t / nt, b = len * (t + 1) / nt;
      std::memcpy(to + a, from + a, b - a);
    };
    std::vector<std::thread> th;
    for (int t = 1; t < nt; ++t) th.emplace_back(part, t);
    part(0);
    for (auto& x : th) x.join();
  }
}

int64_t JoinContext::device_bytes() const {
  return (int64_t)(Xs.bytes() + perm.bytes() + cell_of.bytes() + cell_key.bytes() +
                   cell_start.bytes() + ranges.bytes() + rslot.bytes() + nrng.bytes() +
                   cand_count.bytes() + dense.bytes() +
                   keys.bytes() + keys2.bytes() + vals2.bytes() + flags.bytes() + tmp.bytes() +
                   scal.bytes() + iscal.bytes() + active.bytes() + fail_list.bytes() +
                   failed.bytes() + ikeys.bytes() + ikeys2.bytes() + ivals.bytes() +
                   ivals2.bytes() + out_ids.bytes() + out_d.bytes() + tail_scratch.bytes() +
                   heavy.bytes() + cell_active.bytes() + rowtab.bytes() +
                   Xs2.bytes() + perm2.bytes() + pos.bytes() + active2.bytes() +
                   scan_state.bytes() + pending.bytes());
}

double eps_min_of(const knn_index& idx, int32_t K) {
  const uint64_t need = (uint64_t)K * (uint64_t)idx.n_sample;
  for (int d = 0; d < idx.n_bins; ++d) {
    if (idx.cum[d] >= need) {
      double start = (double)d * idx.bin_width;
      double end = (double)(d + 1) * idx.bin_width;
      return (start + end) / 2.0;
    }
  }
  return (double)idx.n_bins * idx.bin_width;
}

void validate_join(const knn_index* idx, int32_t K) {
  KNN_CHECK(idx != nullptr, KNN_EINVAL, "index is NULL");
  KNN_CHECK(K >= 1, KNN_EINVAL, "K must be >= 1");
  KNN_CHECK((int64_t)K <= idx->N - 1, KNN_EINVAL, "K must be <= N-1");
  KNN_CHECK(K <= KNN_MAX_K, KNN_EINVAL, "K above KNN_MAX_K");
}

void build_grid(const knn_index& idx, JoinContext& c, double w, hipStream_t s, bool from_prev) {
  const int64_t N = idx.N;
  const int n = idx.n;
  c.zmode = false;
  c.gg = make_geom(n, c.blo, c.bhi, w);
  c.Xs.reserve((size_t)N * point_stride(n));
  c.perm.reserve(N);
  c.cell_of.reserve(N);
  c.cell_key.reserve(N);
  c.cell_start.reserve(N + 1);
  c.cand_count.reserve(N);
  c.keys.reserve(N);
  c.keys2.reserve(N);
  c.vals2.reserve(N);
  c.flags.reserve(N);
  c.tmp.reserve(radix_tmp_elems(N));
  // scan state: zero-filled once per allocation (it carries the scans' epoch)
  if (c.scan_state.reserve(scan_state_elems(N)))
    launch_zero(c.scan_state.p, c.scan_state.bytes(), s);
  c.scal.reserve(4);
  if (from_prev) {
    // sort the previous level's order (spatially coherent: each new cell's
    // points come from a few runs of it) by the new keys, then carry the
    // coordinates and ids over
    c.pos.reserve(N);
    c.Xs2.reserve((size_t)N * point_stride(n));
    c.perm2.reserve(N);
    launch_cell_keys_points(c.Xs.p, N, c.gg, c.keys.p, c.pos.p, s);
    if (radix_sort_pairs(c.keys.p, c.pos.p, c.keys2.p, c.vals2.p, N, c.gg.key_bits, c.tmp.p,
                         c.scan_state.p, (int64_t)c.scan_state.n, s)) {
      std::swap(c.keys, c.keys2);
      std::swap(c.pos, c.vals2);
    }
    launch_gather_prev(c.Xs.p, c.perm.p, c.pos.p, N, n, c.Xs2.p, c.perm2.p, s);
    std::swap(c.Xs, c.Xs2);
    std::swap(c.perm, c.perm2);
  } else {
    launch_cell_keys(idx.X.p, N, c.gg, c.keys.p, c.perm.p, s);
    if (radix_sort_pairs(c.keys.p, c.perm.p, c.keys2.p, c.vals2.p, N, c.gg.key_bits, c.tmp.p,
                         c.scan_state.p, (int64_t)c.scan_state.n, s)) {
      std::swap(c.keys, c.keys2);  // sorted output is in the scratch pair
      std::swap(c.perm, c.vals2);
    }
  }
  build_cell_table(c.keys.p, N, c.flags.p, c.cell_of.p, c.cell_key.p, c.cell_start.p, c.scal.p,
                   c.scan_state.p, (int64_t)c.scan_state.n, s);
  if (!from_prev) launch_gather_points(idx.XA.p, c.perm.p, N, n, c.Xs.p, s);
  // The number of cells M stays on the device (kernels read it there), so the
  // level is built without a host round trip; per-cell arrays are sized for
  // the worst case M = N.
  c.M = -1;
  // dense key -> cell table when the grid is small enough
  long double cells = 1;
  for (int j = 0; j < n; ++j) cells *= (long double)c.gg.g[j];
  const uint32_t* dense = nullptr;
  const int64_t dense_lim = c.table_cap > 0 ? c.table_cap : std::max<int64_t>(16 * N, 1 << 22);
  const int64_t rows_lim = c.table_cap > 0 ? c.table_cap : std::max<int64_t>(32 * N, 1 << 22);
  if (n > 2 && cells <= (long double)dense_lim) {
    c.dense.reserve((size_t)cells);
    launch_dense_table(c.cell_key.p, c.scal.p, N, c.dense.p, (int64_t)cells, s);
    dense = c.dense.p;
  }
  c.dense_used = dense;
  // otherwise a row table, when the rows (cells sharing coordinates 0..n-2)
  // are few enough: a range lookup is then a short search within one row
  c.rowtab_used = nullptr;
  if (!dense) {
    const long double rows = cells / (long double)c.gg.g[n - 1];
    if (rows <= (long double)rows_lim) {
      c.rowtab.reserve((size_t)rows);
      launch_row_table(c.cell_key.p, c.scal.p, N, (uint64_t)c.gg.g[n - 1], c.rowtab.p,
                       (int64_t)rows, s);
      c.rowtab_used = c.rowtab.p;
    }
  }
  // An eager join holds at most one of the two lookup tables (the join
  // footprint counts the larger): the one this level does not use goes back
  // to the device cache.  No wait is needed: its last user was the range
  // kernel of an earlier level or join, and the host has synchronised with
  // the stream since (each level reads its counters back, each join returns
  // after its work).  A context owned by a captured graph keeps both, since
  // the graph's nodes refer to them.
  if (!c.graph_owned && !c.fixed) {
    if (!c.dense_used) c.dense.release();
    if (!c.rowtab_used) c.rowtab.release();
  }
}

void build_grid_z(const knn_index& idx, JoinContext& c, double w0, int level, hipStream_t s) {
  const int64_t N = idx.N;
  const int n = idx.n;
  KNN_CHECK(n <= kZMaxDims, KNN_EINTERNAL, "Z-order levels take 2-4 dimensions");
  c.zmode = true;
  if (level == 0) {
    c.gz0 = make_geom_z(n, c.blo, c.bhi, w0);
    c.Xs.reserve((size_t)N * point_stride(n));
    c.perm.reserve(N);
    c.keys.reserve(N);
    c.keys2.reserve(N);
    c.vals2.reserve(N);
    c.tmp.reserve(radix_tmp_elems(N));
    if (c.scan_state.reserve(scan_state_elems(N)))
      launch_zero(c.scan_state.p, c.scan_state.bytes(), s);
    // keys of at most 32 bits are sorted as uint32 (in the same buffers)
    c.zkeys32 = c.gz0.key_bits <= 32;
    bool swapped;
    if (c.zkeys32) {
      uint32_t* k = reinterpret_cast<uint32_t*>(c.keys.p);
      uint32_t* k2 = reinterpret_cast<uint32_t*>(c.keys2.p);
      launch_cell_keys(idx.X.p, N, c.gz0, k, c.perm.p, s);
      swapped = radix_sort_pairs(k, c.perm.p, k2, c.vals2.p, N, c.gz0.key_bits, c.tmp.p,
                                 c.scan_state.p, (int64_t)c.scan_state.n, s);
    } else {
      launch_cell_keys(idx.X.p, N, c.gz0, c.keys.p, c.perm.p, s);
      swapped = radix_sort_pairs(c.keys.p, c.perm.p, c.keys2.p, c.vals2.p, N, c.gz0.key_bits,
                                 c.tmp.p, c.scan_state.p, (int64_t)c.scan_state.n, s);
    }
    if (swapped) {
      std::swap(c.keys, c.keys2);  // sorted output is in the scratch pair
      std::swap(c.perm, c.vals2);
    }
    launch_gather_points(idx.XA.p, c.perm.p, N, n, c.Xs.p, s);
  }
  c.gg = z_level_geom(c.gz0, level);
  c.cell_of.reserve(N);
  c.cell_key.reserve(N);
  c.cell_start.reserve(N + 1);
  c.cand_count.reserve(N);
  c.flags.reserve(N);
  c.scal.reserve(4);
  if (c.zkeys32)
    build_cell_table(reinterpret_cast<const uint32_t*>(c.keys.p), N, c.flags.p, c.cell_of.p,
                     c.cell_key.p, c.cell_start.p, c.scal.p, c.scan_state.p,
                     (int64_t)c.scan_state.n, s, c.gg.zshift);
  else
    build_cell_table(c.keys.p, N, c.flags.p, c.cell_of.p, c.cell_key.p, c.cell_start.p, c.scal.p,
                     c.scan_state.p, (int64_t)c.scan_state.n, s, c.gg.zshift);
  c.M = -1;
  c.dense_used = nullptr;
  c.rowtab_used = nullptr;
  if (!c.graph_owned && !c.fixed) c.rowtab.release();  // the dense table serves the ranges
}

bool use_zorder(const knn_index& idx, int32_t K, const knn_join_opts& o) {
  if (idx.n > kZMaxDims || o.zorder < 0) return false;
  if (o.zorder > 0) return true;
  const int tuned = autotune_zorder(idx.n, K, idx.N);
  return tuned != 0 ? tuned > 0 : idx.n <= 3;
}

int64_t build_ranges(const knn_index& idx, JoinContext& c, hipStream_t s, int64_t Mcap_known,
                     const uint8_t* cell_active, uint8_t active_tag) {
  const int64_t N = idx.N;
  const int n = idx.n;
  const int64_t R = c.zmode ? pow3(n) : pow3(n - 1);
  int64_t Mcap = N;
  if (R >= 81) {
    // 5-6 dims: 81-243 segments per cell make the worst case large; size the
    // segment arrays from the actual cell count (one round trip)
    if (Mcap_known > 0) {
      Mcap = Mcap_known;
    } else {
      c.pinned.reserve(kCounterInts + 16 + KNN_MAX_LEVELS);
      KNN_HIP(hipMemcpyAsync(c.pinned.p, c.scal.p, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
      KNN_HIP(hipStreamSynchronize(s));
      Mcap = std::max<int64_t>((uint32_t)c.pinned.p[0], 1);
    }
  }
  c.ranges.reserve((size_t)Mcap * R * 4);
  c.rslot.reserve((size_t)Mcap * R);
  c.nrng.reserve(N);
  if (c.zmode) {
    // neighbours through a row-major table of the level's cells (never
    // cleared: entries are checked against the cell keys) when it has at
    // most 16 N entries: on a sparser grid the scatter of the cells into the
    // table costs more than the galloping lookups it replaces (clustered
    // 2-D, 2e7 points: 6.5e8 entries at level 0, 280 us of scatter)
    long double cells = 1;
    for (int j = 0; j < n; ++j) cells *= (long double)c.gg.g[j];
    const int64_t lim = c.table_cap > 0 ? c.table_cap : std::max<int64_t>(16 * N, 1 << 22);
    uint32_t* dense = nullptr;
    if (cells <= (long double)lim && (!c.fixed || (long double)c.dense.n >= cells)) {
      c.dense.reserve((size_t)cells);
      dense = c.dense.p;
    }
    launch_neighbor_ranges_z(c.cell_start.p, c.cell_key.p, c.scal.p, N, cell_active, active_tag,
                             c.gg, dense, dense ? (int64_t)c.dense.n : 0, c.ranges.p, c.rslot.p,
                             c.nrng.p, c.cand_count.p, s);
  } else {
    launch_neighbor_ranges(c.Xs.p, N, c.cell_start.p, c.cell_key.p, c.scal.p, c.dense_used,
                           c.rowtab_used, cell_active, active_tag, c.gg, c.ranges.p, c.rslot.p,
                           c.nrng.p, c.cand_count.p, s);
  }
  return Mcap;
}

int64_t build_level(const knn_index& idx, JoinContext& c, double w, hipStream_t s,
                    int64_t Mcap_known) {
  c.zmode = false;
  std::copy(idx.lo, idx.lo + idx.n, c.blo);
  std::copy(idx.hi, idx.hi + idx.n, c.bhi);
  build_grid(idx, c, w, s);
  return build_ranges(idx, c, s, Mcap_known, nullptr, 0);
}

// Z-order self-join levels after the first with at most this many active
// queries build no cell table (launch_sparse_ranges_z): on 2e7 points the
// table's two sweeps cost about 0.1 ms, the sparse lookups of 1.6e4 queries
// (3^n blocks, two binary searches each) a few tens of microseconds.
constexpr int64_t kSparseLevelQueries = 16384;

uint64_t join_footprint(const knn_index& idx, int32_t K, bool host_output) {
  // Upper bound of everything a JoinContext allocates, with the worst case of
  // one non-empty cell per point (M = N), and of what the device cache hands
  // out for it: at most kPoolSlack times each request rounded up, i.e.
  // kPoolSlack (b + kPoolRound) for each of the context's buffers.
  const uint64_t N = (uint64_t)idx.N, n = (uint64_t)idx.n;
  // Z-order levels list the 3^n cells of a block, row-major ones 3^(n-1) segments
  const uint64_t R = (uint64_t)pow3(idx.n <= kZMaxDims ? idx.n : idx.n - 1);
  const uint64_t cap = (uint64_t)K + std::max<uint64_t>(16, (uint64_t)K / 2);
  uint64_t b = 0;
  b += 16 * (uint64_t)point_stride(idx.n) * N;  // Xs and the previous level's
  b += 8 * N;                                    // perm2, pos
  b += (4 + 4 + 8 + 4 + 4 + 4) * N;    // perm, cell_of, cell_key, cell_start, nrng, cand_count
  b += 17 * R * N;                     // ranges (4 x u32) + rslot
  b += std::max<uint64_t>(256 * N, 32ull << 20);  // dense key table or row table
  b += (16 + 4 + 4) * N;               // keys, keys2, vals2, flags
  b += (uint64_t)radix_tmp_elems((int64_t)N) * 4;
  b += (uint64_t)scan_state_elems((int64_t)N) * 4;
  b += (4 + 4 + 4 + 1 + 1 + 4) * N;    // active, active2, fail_list, failed, cell_active, heavy
  b += 24 * N;                         // work-item keys and order (at most one item per query)
  b += std::min<uint64_t>(N, 65535) * (512 + cap * 12);  // brute-force tail scratch
  b += 4096;                           // scalars
  if (host_output) b += N * (uint64_t)K * 12;
  b += (uint64_t)kContextBuffers * kPoolRound;
  return (uint64_t)std::ceil((double)b * kPoolSlack);
}

double tail_budget_of(const knn_index& idx, int32_t K, const knn_join_opts& o) {
  // with levels this cheap the tail only pays off for a few hundred queries
  // (it scans all N points per query)
  const double tuned_tail = o.tail_pairs == 0 ? autotune_tail_pairs(idx.n, K, idx.N) : 0.0;
  return o.tail_pairs > 0 ? o.tail_pairs
         : o.tail_pairs < 0 ? -1.0
         : tuned_tail > 0  ? tuned_tail
                           : 2.5e8;
}

namespace {

// Every buffer a join can reserve, at its largest size for (idx, K, o) with
// the lookup tables limited to table_cap entries: f(buffer, elements).
template <class F>
void for_each_join_buffer(const knn_index& idx, JoinContext& c, int32_t K,
                          const knn_join_opts& o, int64_t table_cap, F&& f) {
  const int64_t N = idx.N;
  const int n = idx.n;
  const int64_t S = point_stride(n), R = use_zorder(idx, K, o) ? pow3(n) : pow3(n - 1);
  const int cap = K + std::max(16, K / 2);
  f(c.Xs, N * S);
  f(c.Xs2, N * S);
  f(c.perm, N);
  f(c.perm2, N);
  f(c.pos, N);
  f(c.cell_of, N);
  f(c.cell_key, N);
  f(c.cell_start, N + 1);
  f(c.cand_count, N);
  f(c.nrng, N);
  f(c.ranges, N * R * 4);  // at most one cell per point
  f(c.rslot, N * R);
  f(c.keys, N);
  f(c.keys2, N);
  f(c.vals2, N);
  f(c.flags, N);
  f(c.tmp, (int64_t)radix_tmp_elems(N));
  f(c.scan_state, (int64_t)scan_state_elems(N));
  f(c.scal, 4);
  f(c.iscal, kCounterInts);
  f(c.pending, KNN_MAX_LEVELS);
  f(c.active, N);
  f(c.active2, N);
  f(c.fail_list, N);
  f(c.heavy, N);
  f(c.failed, N);
  f(c.cell_active, N);
  f(c.ikeys, N);  // at most one work item per active query
  f(c.ikeys2, N);
  f(c.ivals, N);
  f(c.ivals2, N);
  f(c.dense, table_cap);  // row-major levels of 3-6 dims, Z-order levels
  f(c.rowtab, table_cap);
  // the tail runs once A * N <= budget with A <= 65535 remaining queries
  const double budget = tail_budget_of(idx, K, o);
  int64_t a_max = 0;
  if (budget > 0) a_max = std::min<int64_t>({(int64_t)(budget / (double)N), 65535, N});
  f(c.tail_scratch, (int64_t)tail_state_bytes(std::max<int64_t>(a_max, 1), cap));
}

}  // namespace

uint64_t fixed_scratch_bytes(const knn_index& idx, int32_t K, const knn_join_opts& o) {
  JoinContext probe;
  uint64_t total = 0;
  for_each_join_buffer(idx, probe, K, o, kFixedTableFactor * idx.N, [&](auto& buf, int64_t count) {
    using T = std::remove_reference_t<decltype(*buf.p)>;
    total += ((uint64_t)std::max<int64_t>(count, 1) * sizeof(T) + 255) / 256 * 256;
  });
  return total;
}

void reserve_fixed_scratch(const knn_index& idx, JoinContext& c, int32_t K,
                           const knn_join_opts& o, hipStream_t s) {
  for_each_join_buffer(idx, c, K, o, c.table_cap,
                       [&](auto& buf, int64_t count) { buf.reserve((size_t)count); });
  // the single-pass scans' epoch and ticket start from zero
  launch_zero(c.scan_state.p, c.scan_state.bytes(), s);
}

// Lanes per query for a level of A active queries that see `cand` candidates
// on average (measured on MI355X over t in 2..64 and 2-6 dims): the power of
// two nearest cand^0.6 / 4, raised until the level has enough lanes to fill
// the GPU (A * t >= 2^18) and the per-wave LDS buffers stay within 16 KiB.
static int lanes_for(int dims, double cand, int64_t A, int cap, bool zl) {
  const double want = std::pow(std::max(cand, 1.0), 0.6) / 4.0;
  int T = 2;
  while (T < 64 && (double)T * 1.41421356 < want) T *= 2;
  while (T < 64 && (double)A * T < (double)(1 << 18)) T *= 2;
  while (T < 64 && search_lds_per_wave(dims, T, cap, zl) > 16384) T *= 2;
  return T;
}

void self_join(const knn_index& idx, JoinContext& c, int32_t K, int32_t* d_ids, double* d_dists,
               const knn_join_opts& o, hipStream_t s, std::vector<LevelPlan>* record,
               const std::vector<LevelPlan>* replay, const JoinQueries* jq, JoinLimit* lim) {
  // rj: a join of the query set jq with the index's points (R join S,
  // Sec. 2.1); the queries are appended to the sorted point array (positions
  // N .. N + NQ - 1), lie in no cell, and get their ranges slot by slot
  const bool rj = jq != nullptr;
  if (rj) {
    KNN_CHECK(K >= 1 && (int64_t)K <= idx.N && K <= KNN_MAX_K, KNN_EINVAL,
              "K must be in [1, min(N, KNN_MAX_K)]");
    KNN_CHECK(jq->NQ >= 1 && idx.N + jq->NQ < ((int64_t)1 << 31), KNN_EINVAL,
              "the query count must be >= 1 and N + queries < 2^31");
    KNN_CHECK(!replay && !record, KNN_EINTERNAL, "joins of a query set are not captured");
  } else {
    validate_join(&idx, K);
  }
  KNN_CHECK(d_ids && d_dists, KNN_EINVAL, "output pointers are NULL");
  KNN_CHECK(!lim || (rj && !replay && !record && (lim->max_levels <= 0 || lim->unsolved)),
            KNN_EINTERNAL, "a level limit needs a query set and an unsolved list");
  if (lim) lim->n_unsolved = 0;
  const bool keep_l0 = lim && lim->reuse_level0;
  if (!keep_l0) c.l0_cached = false;  // this join rebuilds the context's levels
  auto t_start = std::chrono::steady_clock::now();
  const int64_t N = idx.N;
  const int64_t NQ = rj ? jq->NQ : 0;
  const int64_t NP = N + NQ;  // points of the sorted array (queries after the indexed points)
  knn_join_stats* st = replay ? nullptr : o.stats;
  if (record) record->clear();
  if (st) std::memset(st, 0, sizeof(*st));
  // the levels cover the index's bounds, joined with the queries'
  for (int j = 0; j < idx.n; ++j) {
    c.blo[j] = rj ? std::min(idx.lo[j], jq->lo[j]) : idx.lo[j];
    c.bhi[j] = rj ? std::max(idx.hi[j], jq->hi[j]) : idx.hi[j];
  }

  // level-0 cell side: w = w_factor * eps_min(K) (Sec. 4.4), or explicit
  const double eps_min = eps_min_of(idx, K);
  double ext = 0;
  for (int j = 0; j < idx.n; ++j) ext = std::max(ext, c.bhi[j] - c.blo[j]);
  double w;
  if (o.cell_width > 0) {
    w = o.cell_width;
  } else {
    double f = o.w_factor > 0 ? o.w_factor : autotune_w_factor(idx.n, K, idx.N);
    w = f * eps_min;
  }
  if (!(w > 0) || !std::isfinite(w)) w = ext > 0 ? ext * 1e-6 : 1.0;
  const double w0 = w;
  const double step = (o.eps_step > 0 ? o.eps_step : 0.5) * w0;
  // growth: the paper's linear step (eps += eps_step * eps_min) for the first
  // `linear` re-indexes, then geometric growth whose default multiplies the
  // scanned volume by 16 per level (the non-linear expansion Sec. 5.4
  // proposes for the GPU-Only tail)
  int linear = o.linear_levels > 0 ? o.linear_levels : (o.linear_levels < 0 ? 0 : 1);
  if (o.linear_levels == 0) {
    const int tl = autotune_linear(idx.n, K, idx.N);
    if (tl != 0) linear = tl > 0 ? tl : 0;
  }
  const double tuned_growth = o.growth > 1.0 ? 0.0 : autotune_growth(idx.n, K, idx.N);
  const double growth = o.growth > 1.0 ? o.growth
                        : tuned_growth > 1.0 ? tuned_growth
                                             : std::pow(16.0, 1.0 / idx.n);

  const int T_fixed = o.lanes_per_query;
  KNN_CHECK(T_fixed == 0 || (T_fixed >= 1 && T_fixed <= 64 && (T_fixed & (T_fixed - 1)) == 0),
            KNN_EINVAL, "lanes_per_query must be a power of two in [1, 64]");
  const int T_tuned = T_fixed > 0 ? 0 : autotune_lanes(idx.n, K, idx.N);
  const int lanes_shift = std::max(-2, std::min(2, o.lanes_shift != 0
                                                       ? o.lanes_shift
                                                       : autotune_lanes_shift(idx.n, K, idx.N)));
  const int pad = std::max(16, K / 2);
  const int cap = K + pad;
  // Z-order levels: one sort, cell side doubling per level (growth,
  // linear_levels and eps_step do not apply)
  const bool zl = use_zorder(idx, K, o);
  if (st) st->eps_min = eps_min;
  const double tail_budget = tail_budget_of(idx, K, o);
  double diag2 = 0;
  for (int j = 0; j < idx.n; ++j) diag2 += (c.bhi[j] - c.blo[j]) * (c.bhi[j] - c.blo[j]);

  c.iscal.reserve(kCounterInts);  // queue heads, failures, refinement rounds, heavy queries
  c.scal.reserve(4);
  c.active.reserve(std::max(N, NQ));
  c.fail_list.reserve(std::max(N, NQ));
  c.failed.reserve(NP);
  c.cell_active.reserve(N);
  // sorted failures are listed by position (Z-order levels keep the order;
  // external queries keep theirs at every level)
  const bool fpos = zl || rj;
  if (rj) {
    // the point arrays hold the queries after the indexed points, in both
    // buffers of the row-major level pair
    const int S = point_stride(idx.n);
    // a kept level 0 lives in these buffers: growing one drops it
    bool moved = c.Xs.reserve((size_t)NP * S);
    moved |= c.perm.reserve(NP);
    c.vals2.reserve(NP);
    moved |= c.cell_of.reserve(NP);
    if (!zl) {
      moved |= c.Xs2.reserve((size_t)NP * S);
      moved |= c.perm2.reserve(NP);
    }
    if (moved) c.l0_cached = false;
    const int64_t NM = std::max(N, NQ);
    c.tmp.reserve(radix_tmp_elems(NM));
    if (c.scan_state.reserve(scan_state_elems(NM)))
      launch_zero(c.scan_state.p, c.scan_state.bytes(), s);
  }
  // Failure and active-cell flags carry the level's tag (level_tag), so they
  // are cleared only when the tags start over (before level 1's marks).
  const int ncu = cu_count(c.device);

  Events ev(st != nullptr);
  int64_t A = rj ? NQ : N;          // active queries of the level
  int64_t remaining = A;            // queries not solved yet
  for (int level = 0;; ++level) {
    if (level >= KNN_MAX_LEVELS - 1) w = std::max(w, 2.0 * ext + 1.0);  // everything in one block
    const LevelPlan* rp = nullptr;
    if (replay) {
      KNN_CHECK(level < (int)replay->size(), KNN_EINTERNAL, "replayed join ran past its plan");
      rp = &(*replay)[level];
    }
    LevelPlan lp;
    if (lim && lim->max_levels > 0 && level == lim->max_levels) {
      // cut short: list the queries left (as the tail below does) and hand
      // their query indices back
      int32_t* list = c.fail_list.p;
      if (zl) {
        launch_active_list(c.failed.p + N, level_tag(level), nullptr, NQ, c.active.p,
                           c.scal.p + 1, c.scan_state.p, (int64_t)c.scan_state.n, s, true,
                           (int32_t)N);
        c.pinned.reserve(kCounterInts + 16 + KNN_MAX_LEVELS);
        KNN_HIP(hipMemcpyAsync(c.pinned.p, c.scal.p + 1, sizeof(uint32_t), hipMemcpyDeviceToHost,
                               s));
        KNN_HIP(hipStreamSynchronize(s));
        KNN_CHECK((int64_t)(uint32_t)c.pinned.p[0] == remaining, KNN_EINTERNAL,
                  "cut: the flagged queries differ from the count left");
        list = c.active.p;
      }
      launch_pos_to_id(list, remaining, c.perm.p, s);
      KNN_HIP(hipMemcpyAsync(lim->unsolved, list, (size_t)remaining * sizeof(int32_t),
                             hipMemcpyDeviceToDevice, s));
      lim->n_unsolved = remaining;
      break;
    }
    // brute-force tail once few queries remain (their ids are in fail_list)
    // (remaining: the queries left, A of them active at this level; Z-order
    // levels may hold more, deferred to later levels)
    const bool tail = rp ? rp->tail
                         : (level > 0 && tail_budget > 0 && remaining <= 65535 &&
                            (double)remaining * (double)N <= tail_budget);
    if (tail) {
      ev.rec(0, s);
      TailArgs ta{};
      ta.X = idx.X.p;
      ta.N = N;
      ta.n = idx.n;
      if (rj) {
        ta.QX = jq->QX;
        ta.QN = NQ;
      }
      if (rp) remaining = rp->A;
      if (zl) {
        // every query left is flagged with this level or a later one: list
        // them (sorted positions) and take their ids
        launch_active_list(c.failed.p + (rj ? N : 0), level_tag(level), nullptr, rj ? NQ : N,
                           c.active.p, c.scal.p + 1, c.scan_state.p, (int64_t)c.scan_state.n, s,
                           true, rj ? (int32_t)N : 0);
        if (!rp) {  // the flags must account for exactly the queries left
          c.pinned.reserve(kCounterInts + 16 + KNN_MAX_LEVELS);
          KNN_HIP(hipMemcpyAsync(c.pinned.p, c.scal.p + 1, sizeof(uint32_t),
                                 hipMemcpyDeviceToHost, s));
          KNN_HIP(hipStreamSynchronize(s));
          KNN_CHECK((int64_t)(uint32_t)c.pinned.p[0] == remaining, KNN_EINTERNAL,
                    "tail: the flagged queries differ from the count left");
        }
        launch_pos_to_id(c.active.p, remaining, c.perm.p, s);
        ta.q_ids = c.active.p;
      } else {
        if (rj) launch_pos_to_id(c.fail_list.p, remaining, c.perm.p, s);
        ta.q_ids = c.fail_list.p;
      }
      A = remaining;
      ta.A = (int32_t)A;
      const double top_ref = std::max(diag2, 1e-290);
      uint64_t tb;
      std::memcpy(&tb, &top_ref, 8);
      ta.top = (int64_t)(tb >> 50);
      ta.K = K;
      ta.cap = cap;
      ta.out_ids = d_ids;
      ta.out_d = d_dists;
      c.tail_scratch.reserve(tail_state_bytes(A, cap));
      const int rounds = tail_run(ta, c.tail_scratch.p, s, rp ? rp->tail_rounds : -1);
      ev.rec(1, s);
      if (!rp) KNN_HIP(hipStreamSynchronize(s));
      if (st) {
        st->tail_queries = A;
        st->tail_rounds = rounds;
        st->ms_tail = elapsed_ms(ev.e[0], ev.e[1]);
      }
      if (record) {
        lp.tail = true;
        lp.A = A;
        lp.tail_rounds = rounds;
        record->push_back(lp);
      }
      break;
    }
    ev.rec(0, s);
    // level 0 sorts the points from their original order, later levels from
    // the previous level's order (row-major) or not at all (Z-order)
    const bool reuse = level == 0 && keep_l0 && c.l0_cached && c.l0_w == w && c.l0_zl == zl;
    // a later Z-order level of a self-join with few active queries builds no
    // cell table: each query's block is looked up in the sorted level-0 keys
    // (the table over all N points would cost more than their searches)
    const bool sparse = zl && !rj && level > 0 && A <= kSparseLevelQueries;
    if (reuse) {
      // level 0 of the previous query-set join with this cell side: the
      // indexed points' grid is unchanged (only the appended queries differ)
    } else if (sparse) {
      KNN_CHECK(level <= c.gz0.zbits, KNN_EINTERNAL,
                "Z-order levels ran past their single-cell top");
      c.zmode = true;
      c.gg = z_level_geom(c.gz0, level);
      c.M = -1;
      c.dense_used = nullptr;
      c.rowtab_used = nullptr;
    } else if (zl) {
      // the top of the ladder is one cell, where every query succeeds
      KNN_CHECK(level == 0 || level <= c.gz0.zbits, KNN_EINTERNAL,
                "Z-order levels ran past their single-cell top");
      build_grid_z(idx, c, w0, level, s);
    } else {
      build_grid(idx, c, w, s, level > 0);
    }
    if (level == 0 && keep_l0) {
      c.l0_cached = true;
      c.l0_w = w;
      c.l0_zl = zl;
    } else if (level > 0) {
      c.l0_cached = false;
    }
    if (rj && level == 0) {
      // the queries, sorted by their level-0 cell key (locality), appended
      // after the indexed points: coordinates and ids (row-major levels: in
      // both buffers of the pair, which later levels swap)
      const GridGeom& g0 = zl ? c.gz0 : c.gg;
      const int S = point_stride(idx.n);
      c.ikeys.reserve(NQ);
      c.ikeys2.reserve(NQ);
      c.ivals.reserve(NQ);
      c.ivals2.reserve(NQ);
      launch_cell_keys(jq->QX, NQ, g0, c.ikeys.p, c.ivals.p, s);
      const int32_t* qperm =
          radix_sort_pairs(c.ikeys.p, c.ivals.p, c.ikeys2.p, c.ivals2.p, NQ, g0.key_bits,
                           c.tmp.p, c.scan_state.p, (int64_t)c.scan_state.n, s)
              ? c.ivals2.p
              : c.ivals.p;
      launch_gather_points(jq->QA, qperm, NQ, idx.n, c.Xs.p + (size_t)N * S, s);
      KNN_HIP(hipMemcpyAsync(c.perm.p + N, qperm, (size_t)NQ * sizeof(int32_t),
                             hipMemcpyDeviceToDevice, s));
      if (!zl) {
        KNN_HIP(hipMemcpyAsync(c.Xs2.p + (size_t)N * S, c.Xs.p + (size_t)N * S,
                               (size_t)NQ * S * sizeof(double), hipMemcpyDeviceToDevice, s));
        KNN_HIP(hipMemcpyAsync(c.perm2.p + N, qperm, (size_t)NQ * sizeof(int32_t),
                               hipMemcpyDeviceToDevice, s));
      }
    }
    // active list of this level (cell order): level 0 = every point
    const int32_t* active = nullptr;
    const uint8_t* cell_active = nullptr;
    if (rj && level == 0) {
      launch_iota(c.active.p, NQ, (int32_t)N, s);  // every query
      active = c.active.p;
    } else if (level > 0) {
      // failures flagged by position (Z-order levels, external queries) are
      // read without a gather through perm
      if (rj)
        launch_active_list(c.failed.p + N, level_tag(level), nullptr, NQ, c.active.p,
                           c.scal.p + 1, c.scan_state.p, (int64_t)c.scan_state.n, s, false,
                           (int32_t)N);
      else
        launch_active_list(c.failed.p, level_tag(level), zl ? nullptr : c.perm.p, N, c.active.p,
                           c.scal.p + 1, c.scan_state.p, (int64_t)c.scan_state.n, s);
      active = c.active.p;
    }
    // Z-order levels: deferred queries are flagged straight for later levels,
    // so the flags and the per-level pending counts start clean here
    if (zl && level == 0) {
      c.pending.reserve(KNN_MAX_LEVELS);
      launch_zero(c.failed.p, (size_t)NP, s);
      launch_zero(c.cell_active.p, (size_t)N, s);
      launch_zero(c.pending.p, KNN_MAX_LEVELS * sizeof(uint32_t), s);
    }
    // the level's counters start here: the deferral filters append to the
    // failure list
    const int64_t A_in = A;
    launch_zero(c.iscal.p, kCounterInts * sizeof(int32_t), s);
    const bool filt = o.predict_fail >= 0;
    auto defer_args = [&](const int32_t* in, int32_t* out, uint32_t* out_count) {
      DeferArgs da{};
      da.Xs = c.Xs.p;
      da.perm = c.perm.p;
      da.cell_of = c.cell_of.p;
      da.cand = c.cand_count.p;
      da.active = in;
      da.n_active = A;
      for (int j = 0; j < kMaxDims; ++j) {
        da.lo[j] = c.gg.lo[j];
        da.g[j] = c.gg.g[j];
      }
      da.inv_w = c.gg.inv_w;
      da.w = 1.0 / c.gg.inv_w;
      da.margin = (8.0 * (double)c.gg.g_max + 4.0 * idx.n + 32.0) * std::ldexp(1.0, -53);
      da.defer_coef = search_density_coef(idx.n, K, da.w) / 1.3;
      da.out_active = out;
      da.out_count = out_count;
      da.fail_list = c.fail_list.p;
      da.fail_count = c.iscal.p + kFailSlot;
      da.fail_pos = fpos ? 1 : 0;
      if (zl) {  // skip ahead to the level the prediction asks for
        da.failed = c.failed.p;
        da.pending = c.pending.p;
        da.level = level;
        da.top_level = c.gz0.zbits;
      }
      da.cand_sum = reinterpret_cast<unsigned long long*>(c.iscal.p + kCandSumSlot);
      da.state = c.scan_state.p;
      da.state_elems = (int64_t)c.scan_state.n;
      return da;
    };
    const uint32_t* n_pre = nullptr;  // device count of the list the prefilter kept
    if (zl && filt && !rj && !sparse) {
      // Z-order levels: a first deferral from the parent-group density, before
      // any neighbour range exists, so that ranges are built only for the
      // cells of the queries it keeps (most of a fine level's queries are
      // deferred); a deliberately loose margin (2 on the squared distance,
      // against 1.3 for the block estimate that follows)
      c.active2.reserve(N);
      DeferArgs pa = defer_args(active, c.active2.p, c.scal.p + 3);
      pa.cand = nullptr;
      pa.cell_key = c.cell_key.p;
      pa.cell_start = c.cell_start.p;
      pa.d_M = c.scal.p;
      pa.cand_sum = nullptr;
      pa.defer_coef = search_density_coef(idx.n, K, pa.w) * (4.0 / 9.0) / 2.0;
      launch_defer_filter(pa, idx.n, s);
      active = c.active2.p;
      n_pre = c.scal.p + 3;
    }
    if (rj) {
      // external queries: ranges slot by slot, for the active ones
      const int64_t R = zl ? pow3(idx.n) : pow3(idx.n - 1);
      c.ranges.reserve((size_t)NQ * R * 4);
      c.rslot.reserve((size_t)NQ * R);
      c.nrng.reserve(NQ);
      c.cand_count.reserve(std::max(N, NQ));
      launch_query_ranges(c.Xs.p, active, A, level > 0 ? c.scal.p + 1 : nullptr, N, NQ,
                          c.cell_start.p, c.cell_key.p, c.scal.p,
                          c.dense_used, c.rowtab_used, c.gg, zl, c.cell_of.p, c.ranges.p,
                          c.rslot.p, c.nrng.p, c.cand_count.p, s);
    } else if (sparse) {
      const int64_t R = pow3(idx.n);
      c.ranges.reserve((size_t)A * R * 4);
      c.rslot.reserve((size_t)A * R);
      if (c.zkeys32)
        launch_sparse_ranges_z(reinterpret_cast<const uint32_t*>(c.keys.p), N, active, A,
                               c.scal.p + 1, c.gg, c.ranges.p, c.rslot.p, c.nrng.p,
                               c.cand_count.p, c.cell_of.p, c.scal.p, s);
      else
        launch_sparse_ranges_z(c.keys.p, N, active, A, c.scal.p + 1, c.gg, c.ranges.p, c.rslot.p,
                               c.nrng.p, c.cand_count.p, c.cell_of.p, c.scal.p, s);
      lp.Mcap = A;
    } else {
      if (level > 0 || n_pre) {
        // neighbour ranges only for the cells that hold an active query
        // (level 0 of Z-order levels, whose flag array was just cleared,
        // marks with a tag no later level uses)
        const uint8_t tag = level == 0 ? (uint8_t)0xFF : level_tag(level);
        launch_mark_cells_of(active, A, c.cell_of.p, c.cell_active.p, tag, s, n_pre);
        cell_active = c.cell_active.p;
      }
      lp.Mcap = build_ranges(idx, c, s, rp ? rp->Mcap : 0, cell_active,
                             level == 0 ? (uint8_t)0xFF : level_tag(level));
    }
    if (filt) {
      // the deferral filter on the block density (candidate counts)
      int32_t* out = n_pre ? c.active.p : (c.active2.reserve(std::max(N, NQ)), c.active2.p);
      DeferArgs da = defer_args(active, out, c.scal.p + 2);
      da.n_active_dev = n_pre ? n_pre : sparse ? c.scal.p + 1 : nullptr;
      launch_defer_filter(da, idx.n, s);
      active = out;
    }
    // lanes per query from the level's mean candidate count (the paper's t,
    // Sec. 4.7, chosen per level: the tail levels see far more candidates)
    double cand = 0;
    uint64_t cand_max = 0;
    int T = T_fixed;
    if (rp) {
      cand = rp->cand;
      c.M = rp->M;
      T = rp->T;
      if (filt) A = rp->A_kept;
    } else {
      uint64_t* csum = reinterpret_cast<uint64_t*>(c.iscal.p + kCandSumSlot);
      if (!filt) launch_active_cand_sum(active, A, c.cell_of.p, c.cand_count.p, csum, s);
      c.pinned.reserve(kCounterInts + 16 + KNN_MAX_LEVELS);
      int32_t* hp = c.pinned.p;
      KNN_HIP(hipMemcpyAsync(hp, csum, 2 * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
      KNN_HIP(hipMemcpyAsync(hp + 4, c.scal.p, 3 * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
      KNN_HIP(hipStreamSynchronize(s));  // the level's one round trip before the search
      uint64_t tot[2];
      std::memcpy(tot, hp, sizeof(tot));
      const uint32_t M = (uint32_t)hp[4];
      if (filt) A = (int64_t)(uint32_t)hp[6];
      cand = (double)tot[0] / (double)std::max<int64_t>(A, 1);
      cand_max = tot[1];
      c.M = M;
      if (T == 0) {
        T = (level == 0 && T_tuned > 0) ? T_tuned : lanes_for(idx.n, cand, A, cap, zl);
        for (int sft = lanes_shift; sft > 0 && T < 64; --sft) T *= 2;
        for (int sft = lanes_shift; sft < 0 && T > 1; ++sft) T /= 2;
      }
    }
    // the per-wave buffers of small T grow with 3^(n-1) segment lists: raise
    // T until one wavefront's LDS fits
    while (T < 64 && search_lds_per_wave(idx.n, T, cap, zl) > 65536) T *= 2;
    const int G = 64 / T;
    const int waves = search_waves_per_block(idx.n, T, cap, zl);
    // Heavy queries: a query on one wavefront costs about C/T lane steps, the
    // level about A*cand/(64*W) (W resident wavefronts); a query above half of
    // that (and above 4096 candidates) would outlast the level, so it gets a
    // workgroup of its own.
    uint32_t heavy_min = 0;
    if (rp) {
      heavy_min = rp->heavy_min;
    } else if (o.heavy_min >= 0) {
      double hm;
      if (o.heavy_min > 0) {
        hm = (double)o.heavy_min;
      } else {
        const double W = (double)ncu * search_blocks_per_cu(idx.n, T, cap, zl) * waves;
        hm = std::max(4096.0, (double)T * (double)A * cand / (128.0 * W));
      }
      if ((double)cand_max >= hm) heavy_min = (uint32_t)std::min(hm, 4294967295.0);
    }
    // work items, densest first (Sec. 4.5 work estimate; persistent schedule)
    const int64_t n_items = ceil_div(A, G);
    const int32_t* order = nullptr;
    if (o.schedule == 0 && o.item_order == 0 && n_items > 1) {
      c.ikeys.reserve(n_items);
      c.ikeys2.reserve(n_items);
      c.ivals.reserve(n_items);
      c.ivals2.reserve(n_items);
      launch_item_keys(active, A, G, c.cell_of.p, c.cand_count.p, c.ikeys.p, c.ivals.p, n_items,
                       s);
      if (radix_sort_pairs(c.ikeys.p, c.ivals.p, c.ikeys2.p, c.ivals2.p, n_items, 9, c.tmp.p,
                           c.scan_state.p, (int64_t)c.scan_state.n, s)) {
        std::swap(c.ikeys, c.ikeys2);
        std::swap(c.ivals, c.ivals2);
      }
      order = c.ivals.p;
    }
    ev.rec(1, s);

    SearchArgs a{};
    a.Xs = c.Xs.p;
    a.N = N;
    a.perm = c.perm.p;
    a.cell_of = c.cell_of.p;
    a.ranges = c.ranges.p;
    a.rslot = c.rslot.p;
    a.nrng = c.nrng.p;
    a.cand = c.cand_count.p;
    a.active = active;
    a.n_active = A;
    a.order = order;
    a.n_items = n_items;
    a.item_base = 0;
    a.head = c.iscal.p;
    for (int x = 0; x <= kXcds; ++x)  // queue x: items of chunk x (ceil(x * n_items / 8) onwards)
      a.qbeg[x] = (x * n_items + kXcds - 1) / kXcds;
    a.persistent = o.schedule == 0 ? 1 : 0;
    a.share_lists = o.share_lists > 0 ? 1 : (o.share_lists < 0 ? 0 : (idx.n >= 5 ? 1 : 0));
    a.zl = zl ? 1 : 0;
    for (int j = 0; j < kMaxDims; ++j) {
      a.lo[j] = c.gg.lo[j];
      a.g[j] = c.gg.g[j];
    }
    a.inv_w = c.gg.inv_w;
    a.w = 1.0 / c.gg.inv_w;
    a.margin = (8.0 * (double)c.gg.g_max + 4.0 * idx.n + 32.0) * std::ldexp(1.0, -53);
    a.K = K;
    a.cap = cap;
    a.spec_slots = o.speculate < 0 ? 0 : search_spec_slots(idx.n, T, cap, zl);
    a.spec_coef = std::pow(1.7, 2.0 / idx.n) * search_density_coef(idx.n, K, a.w);
    a.out_ids = d_ids;
    a.out_d = d_dists;
    a.fail_list = c.fail_list.p;
    a.fail_count = c.iscal.p + kFailSlot;
    a.fail_pos = fpos ? 1 : 0;
    a.self_in_list = rj ? 0 : 1;
    a.refine_count = c.iscal.p + kRefineSlot;
    a.walk_error = c.iscal.p + kWalkErrSlot;
    a.spec_count = c.iscal.p + kSpecSlot;
    lp.heavy_min = heavy_min;
    if (heavy_min > 0 && A > 0) {
      // heavy queries first, one workgroup each (count stays on the device)
      c.heavy.reserve(std::max(N, NQ));
      a.heavy_min = heavy_min;
      a.heavy = c.heavy.p;
      a.n_heavy = c.iscal.p + kHeavySlot;
      a.heavy_fail = c.iscal.p + kHeavyFailSlot;
      launch_heavy_list(active, A, c.cell_of.p, c.cand_count.p, heavy_min, c.heavy.p,
                        c.iscal.p + kHeavySlot,
                        reinterpret_cast<unsigned long long*>(c.iscal.p + kHeavyCandSlot), s);
      launch_search_heavy(a, idx.n, ncu, s);
    }
    ev.rec(3, s);
    if (A == 0) {
      // every query of the level was deferred
    } else if (o.schedule == 0) {
      int blocks;
      if (rp) {
        blocks = rp->blocks;
        a.grain = rp->grain;
      } else {
        // persistent grid: exactly what can be resident at once
        int64_t want = ceil_div(n_items, waves);
        blocks = (int)std::min<int64_t>(want,
                                        (int64_t)ncu * search_blocks_per_cu(idx.n, T, cap, zl));
        // a few pops per wavefront and queue: few atomics, fine enough
        // granularity for the dense-first balance at the end of each queue
        const int64_t total_waves = (int64_t)blocks * waves;
        const int tuned_pops = o.queue_grain == 0 ? autotune_pops(idx.n, K, idx.N) : 0;
        const int64_t pops = o.queue_grain < 0 ? -(int64_t)o.queue_grain
                             : tuned_pops > 0  ? tuned_pops
                                               : 4;
        a.grain = o.queue_grain > 0
                      ? o.queue_grain
                      : (int32_t)std::max<int64_t>(1, std::min<int64_t>(64, n_items / (total_waves * pops)));
      }
      lp.blocks = blocks;
      lp.grain = a.grain;
      launch_search(a, idx.n, T, blocks, s);
    } else {
      // one launch per batch of queries, cell order, one item per wavefront
      int64_t per = o.batch_queries > 0 ? ceil_div(o.batch_queries, G) : n_items;
      for (int64_t base = 0; base < n_items; base += per) {
        a.item_base = base;
        a.n_items = std::min<int64_t>(n_items, base + per);
        int64_t blocks = ceil_div(a.n_items - base, waves);
        launch_search(a, idx.n, T, (int)blocks, s);
      }
    }
    ev.rec(2, s);
    int32_t sc[2] = {0, 0};
    int32_t spec_held = 0, deferred = 0;
    int64_t hq = 0, hf = 0;
    double hc = 0;
    if (rp) {
      sc[0] = rp->fails;
      sc[1] = rp->refine;
      spec_held = rp->spec;
      deferred = rp->deferred;
      hq = rp->heavy;
      hf = rp->heavy_failed;
      hc = rp->heavy_cand;
    } else {
      c.pinned.reserve(kCounterInts + 16 + KNN_MAX_LEVELS);
      int32_t* cnt = c.pinned.p;
      KNN_HIP(hipMemcpyAsync(cnt, c.iscal.p, kCounterInts * sizeof(int32_t), hipMemcpyDeviceToHost,
                             s));
      // the single-pass scans' look-back error count of this level's build
      // (must stay 0), in the same round trip
      KNN_HIP(hipMemcpyAsync(cnt + kCounterInts, c.scan_state.p + 2, sizeof(uint32_t),
                             hipMemcpyDeviceToHost, s));
      if (zl)  // queries flagged for each later level
        KNN_HIP(hipMemcpyAsync(cnt + kCounterInts + 16, c.pending.p,
                               KNN_MAX_LEVELS * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
      KNN_HIP(hipStreamSynchronize(s));
      if (cnt[kCounterInts] != 0) {
        // cleared, so that later joins on this context start clean
        launch_zero(c.scan_state.p + 2, sizeof(uint32_t), s);
        KNN_HIP(hipStreamSynchronize(s));
        throw Error(KNN_EINTERNAL, "scan: a look-back found no prefix");
      }
      KNN_CHECK(cnt[kWalkErrSlot] == 0, KNN_EINTERNAL,
                "search: a candidate list was inconsistent with its count");
      sc[0] = cnt[kFailSlot];
      sc[1] = cnt[kRefineSlot];
      spec_held = cnt[kSpecSlot];
      deferred = (int32_t)(A_in - A);
      hq = cnt[kHeavySlot];
      hf = cnt[kHeavyFailSlot];
      uint64_t hcu = 0;
      std::memcpy(&hcu, &cnt[kHeavyCandSlot], sizeof(hcu));
      hc = (double)hcu;
    }
    const int32_t fails = sc[0];
    // the next level's active queries: this level's search failures and, on
    // Z-order levels, the queries flagged for it by earlier deferrals; the
    // queries left: those and every later level's
    int64_t A_next = fails;
    if (rp) {
      remaining = rp->remaining;
      if (level + 1 < (int)replay->size()) A_next = (*replay)[level + 1].A;
    } else {
      remaining = fails;
      if (zl) {
        const uint32_t* pend = reinterpret_cast<const uint32_t*>(c.pinned.p + kCounterInts + 16);
        for (int L = level + 1; L < KNN_MAX_LEVELS; ++L) remaining += pend[L];
        if (level + 1 < KNN_MAX_LEVELS) A_next += pend[level + 1];
      }
    }
    if (record) {
      lp.A = A_in;
      lp.A_kept = A;
      lp.T = T;
      lp.n_items = n_items;
      lp.cand = cand;
      lp.fails = fails;
      lp.refine = sc[1];
      lp.spec = spec_held;
      lp.deferred = deferred;
      lp.heavy = hq;
      lp.heavy_failed = hf;
      lp.heavy_cand = hc;
      lp.M = c.M;
      lp.cell_w = 1.0 / c.gg.inv_w;
      lp.remaining = remaining;
      lp.failed_stat = fails + (zl ? deferred : 0);
      record->push_back(lp);
    }
    if (st && level < KNN_MAX_LEVELS) {
      if (level == 0) st->lanes_per_query = T;
      st->lanes[level] = T;
      st->cand_per_query[level] = cand;
      st->refine_rounds[level] = sc[1];
      st->spec_queries[level] = spec_held;
      st->deferred[level] = deferred;
      st->levels = level + 1;
      st->cell_width[level] = 1.0 / c.gg.inv_w;
      st->attempted[level] = A_in;
      // deferred queries count as failed (Z-order levels flag them without
      // the failure list)
      st->failed[level] = fails + (zl ? deferred : 0);
      st->cells[level] = c.M;
      st->ms_build[level] = elapsed_ms(ev.e[0], ev.e[1]);
      st->ms_heavy[level] = elapsed_ms(ev.e[1], ev.e[3]);
      st->ms_search[level] = elapsed_ms(ev.e[3], ev.e[2]);
      st->heavy_queries[level] = hq;
      st->heavy_failed[level] = hf;
      st->heavy_cand[level] = hc;
      st->total_attempted += A_in;
      st->total_failed += fails + (zl ? deferred : 0);
    }
    if (remaining == 0) break;
    KNN_CHECK(fails <= A_in, KNN_EINTERNAL, "more failures than attempted queries");
    // failures are re-queued on a grid with a larger cell side (Alg. 1):
    // linear growth by eps_step * w0 first, then geometric growth
    if (!zl && level_tag(level + 1) == 1) {  // tags wrapped: clear the stale ones
      launch_zero(c.failed.p, (size_t)NP, s);
      launch_zero(c.cell_active.p, (size_t)N, s);
    }
    launch_mark_failed(c.fail_list.p, c.iscal.p + kFailSlot, fails, c.failed.p,
                       level_tag(level + 1), s);
    A = A_next;
    w = (1.0 / c.gg.inv_w);
    if (level < linear)
      w = w + step;
    else
      w = w * growth;
  }
  if (st) {
    st->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() -
                                                             t_start)
                       .count();
  }
}

bool GraphPlan::matches(int32_t K_, const knn_join_opts& o, int32_t* ids_, double* dists_) const {
  return K == K_ && ids == ids_ && dists == dists_ && opts.w_factor == o.w_factor &&
         opts.cell_width == o.cell_width && opts.lanes_per_query == o.lanes_per_query &&
         opts.schedule == o.schedule && opts.batch_queries == o.batch_queries &&
         opts.eps_step == o.eps_step && opts.linear_levels == o.linear_levels &&
         opts.growth == o.growth && opts.tail_pairs == o.tail_pairs &&
         opts.heavy_min == o.heavy_min && opts.queue_grain == o.queue_grain &&
         opts.item_order == o.item_order && opts.share_lists == o.share_lists &&
         opts.lanes_shift == o.lanes_shift && opts.speculate == o.speculate &&
         opts.predict_fail == o.predict_fail && opts.zorder == o.zorder;
}

GraphPlan::~GraphPlan() {
  if (done) (void)hipEventSynchronize(done);  // a replay may still use the scratch
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  if (done) (void)hipEventDestroy(done);
}

namespace {

void stats_from_plan(const GraphPlan& gp, knn_join_stats* st) {
  std::memset(st, 0, sizeof(*st));
  st->eps_min = gp.eps_min;
  int L = 0;
  for (const LevelPlan& lp : gp.levels) {
    if (lp.tail) {
      st->tail_queries = lp.A;
      st->tail_rounds = lp.tail_rounds;
      continue;
    }
    if (L >= KNN_MAX_LEVELS) break;
    if (L == 0) st->lanes_per_query = lp.T;
    st->lanes[L] = lp.T;
    st->cand_per_query[L] = lp.cand;
    st->refine_rounds[L] = lp.refine;
    st->spec_queries[L] = lp.spec;
    st->deferred[L] = lp.deferred;
    st->heavy_queries[L] = lp.heavy;
    st->heavy_failed[L] = lp.heavy_failed;
    st->heavy_cand[L] = lp.heavy_cand;
    st->cell_width[L] = lp.cell_w;
    st->attempted[L] = lp.A;
    st->failed[L] = lp.failed_stat;
    st->cells[L] = lp.M;
    st->total_attempted += lp.A;
    st->total_failed += lp.failed_stat;
    st->levels = ++L;
  }
}

}  // namespace

void self_join_graph(knn_index& idx, int32_t K, int32_t* d_ids, double* d_dists,
                     const knn_join_opts& o, hipStream_t s) {
  knn_join_stats* st = o.stats;
  GraphPlan* gp = idx.graph;
  if (gp && gp->matches(K, o, d_ids, d_dists)) {
    // replay: the whole join as one graph launch, ordered after the previous
    // replay (they share the graph's scratch)
    Events ev(st != nullptr);
    KNN_HIP(hipStreamWaitEvent(s, gp->done, 0));
    ev.rec(0, s);
    KNN_HIP(hipGraphLaunch(gp->exec, s));
    ev.rec(1, s);
    KNN_HIP(hipEventRecord(gp->done, s));
    if (st) {
      // a replay has no host round trip; when the caller waits for its
      // statistics, the error counters of its scratch are checked too
      KNN_HIP(hipEventSynchronize(ev.e[1]));
      stats_from_plan(*gp, st);
      st->ms_total = elapsed_ms(ev.e[0], ev.e[1]);
      gp->ctx.pinned.reserve(kCounterInts + 16);
      int32_t* cnt = gp->ctx.pinned.p;
      KNN_HIP(hipMemcpyAsync(cnt, gp->ctx.iscal.p + kWalkErrSlot, sizeof(int32_t),
                             hipMemcpyDeviceToHost, s));
      KNN_HIP(hipMemcpyAsync(cnt + 1, gp->ctx.scan_state.p + 2, sizeof(uint32_t),
                             hipMemcpyDeviceToHost, s));
      KNN_HIP(hipStreamSynchronize(s));
      if (cnt[0] != 0 || cnt[1] != 0) {
        launch_zero(gp->ctx.scan_state.p + 2, sizeof(uint32_t), s);
        KNN_HIP(hipStreamSynchronize(s));
        throw Error(KNN_EINTERNAL,
                    "replayed join: a candidate list or a scan look-back was inconsistent");
      }
    }
    return;
  }
  // first join of this (K, options, outputs): run it eagerly, recording its
  // levels, then capture the same launch sequence on a private stream
  if (gp) {
    delete gp;
    idx.graph = nullptr;
  }
  std::unique_ptr<GraphPlan> np(new GraphPlan());
  np->K = K;
  np->opts = o;
  np->opts.stats = nullptr;
  np->ids = d_ids;
  np->dists = d_dists;
  np->ctx.device = idx.device;
  np->ctx.graph_owned = true;
  np->eps_min = eps_min_of(idx, K);
  KNN_HIP(hipEventCreateWithFlags(&np->done, hipEventDisableTiming));
  self_join(idx, np->ctx, K, d_ids, d_dists, o, s, &np->levels, nullptr);
  hipStream_t cs = nullptr;
  KNN_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipGraph_t g = nullptr;
  try {
    KNN_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    try {
      self_join(idx, np->ctx, K, d_ids, d_dists, np->opts, cs, nullptr, &np->levels);
    } catch (...) {
      (void)hipStreamEndCapture(cs, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    KNN_HIP(hipStreamEndCapture(cs, &g));
    np->graph = g;
    KNN_HIP(hipGraphInstantiate(&np->exec, g, nullptr, nullptr, 0));
  } catch (...) {
    (void)hipStreamDestroy(cs);
    throw;
  }
  KNN_HIP(hipStreamDestroy(cs));
  KNN_HIP(hipEventRecord(np->done, s));
  idx.graph = np.release();
}

}  // namespace knn

using namespace knn;

namespace {

knn_build_opts resolve(const knn_build_opts* in) {
  knn_build_opts o{};
  if (in) o = *in;
  if (o.seed == 0) o.seed = 1;
  if (o.n_sample <= 0) o.n_sample = 500;
  if (o.n_bins <= 0) o.n_bins = 1000;
  if (!(o.mean_frac > 0)) o.mean_frac = 0.001;
  if (o.min_mean_sample <= 0) o.min_mean_sample = 64;
  return o;
}

// Common part of both build entry points: D_dev is AoS on the device.
knn_index* build_from_device(const double* D_dev, int64_t N, int n, const knn_build_opts& o,
                             hipStream_t s) {
  auto* idx = new knn_index();
  try {
    idx->N = N;
    idx->n = n;
    idx->device = current_device();
    idx->X.alloc((size_t)N * n);
    idx->XA.alloc((size_t)N * n);
    KNN_HIP(hipMemcpyAsync(idx->XA.p, D_dev, (size_t)N * n * sizeof(double),
                           hipMemcpyDeviceToDevice, s));
    DevBuf<uint32_t> bad(1);
    KNN_HIP(hipMemsetAsync(bad.p, 0, sizeof(uint32_t), s));
    launch_aos_to_soa(D_dev, N, n, idx->X.p, bad.p, s);
    // bounds (a non-finite coordinate is reported below, before they are used)
    DevBuf<double> part((size_t)2 * n * kBoundsBlocks), lohi(2 * kMaxDims);
    launch_bounds(idx->X.p, N, n, part.p, lohi.p, lohi.p + kMaxDims, s);
    double hb[2 * kMaxDims];
    uint32_t nbad = 0;
    KNN_HIP(hipMemcpyAsync(&nbad, bad.p, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    KNN_HIP(hipMemcpyAsync(hb, lohi.p, sizeof(hb), hipMemcpyDeviceToHost, s));
    // the samples of Sec. 4.4 are drawn on the host while the device works:
    // eps_mean over mean_frac * N points, the histogram over n_sample points
    int64_t nm = (int64_t)std::llround(o.mean_frac * (double)N);
    nm = std::max<int64_t>(nm, o.min_mean_sample);
    nm = std::min<int64_t>(nm, std::min<int64_t>(N, KNN_MAX_MEAN_SAMPLE));
    std::vector<int64_t> sm = sample_ids(N, nm, o.seed);
    std::vector<int64_t> sh = sample_ids(N, o.n_sample, o.seed ^ 0x5DEECE66Dull);
    KNN_HIP(hipStreamSynchronize(s));
    KNN_CHECK(nbad == 0, KNN_EINVAL, "D holds non-finite coordinates");
    for (int j = 0; j < n; ++j) {
      idx->lo[j] = hb[j];
      idx->hi[j] = hb[kMaxDims + j];
    }
    DevBuf<int64_t> d_sm(sm.size()), d_sh(sh.size());
    KNN_HIP(hipMemcpyAsync(d_sm.p, sm.data(), sm.size() * 8, hipMemcpyHostToDevice, s));
    KNN_HIP(hipMemcpyAsync(d_sh.p, sh.data(), sh.size() * 8, hipMemcpyHostToDevice, s));
    DevBuf<double> psum(std::max<size_t>(sm.size(), 1));
    DevBuf<double> sx(std::max<size_t>(sm.size() * n, 1));
    int np = launch_sample_pair_sums(idx->X.p, N, n, d_sm.p, (int64_t)sm.size(), sx.p, psum.p, s);
    std::vector<double> hp(np);
    if (np) KNN_HIP(hipMemcpyAsync(hp.data(), psum.p, np * 8, hipMemcpyDeviceToHost, s));
    KNN_HIP(hipStreamSynchronize(s));
    double sum = 0;
    for (double v : hp) sum += v;
    double pairs = (double)sm.size() * (double)(sm.size() - 1) / 2.0;
    double eps_mean = pairs > 0 ? sum / pairs : 0.0;
    double ext = 0;
    for (int j = 0; j < n; ++j) ext = std::max(ext, idx->hi[j] - idx->lo[j]);
    if (!(eps_mean > 0)) eps_mean = ext > 0 ? ext : 1.0;
    idx->eps_mean = eps_mean;
    idx->n_bins = o.n_bins;
    idx->n_sample = (int)sh.size();
    idx->bin_width = eps_mean / o.n_bins;
    // eps_min(K) reads the cumulative histogram only up to the first bin
    // where it reaches K per sample point, so for every K <= KNN_MAX_K only
    // the bins up to where it reaches KNN_MAX_K per sample point matter.
    // That bin is estimated on every pstride-th point (with a margin of 4),
    // the bins below it are counted exactly over all points (the far pairs,
    // most of them, skip the bin arithmetic), and all bins are counted when
    // the estimate fell short.
    const int64_t ns = (int64_t)sh.size();
    const double inv_bw = 1.0 / idx->bin_width;
    const uint64_t need = (uint64_t)KNN_MAX_K * (uint64_t)ns;
    DevBuf<uint64_t> counts(o.n_bins);
    std::vector<uint64_t> hc(o.n_bins);
    double max_abs = 0;  // every |coordinate| is at most this
    for (int j = 0; j < n; ++j)
      max_abs = std::max(max_abs, std::max(std::fabs(idx->lo[j]), std::fabs(idx->hi[j])));
    auto histogram = [&](int count_bins, int64_t pstride) {
      launch_dist_histogram(idx->X.p, N, n, d_sh.p, ns, inv_bw, o.n_bins, counts.p, s,
                            count_bins, pstride, max_abs);
      KNN_HIP(hipMemcpyAsync(hc.data(), counts.p, o.n_bins * 8, hipMemcpyDeviceToHost, s));
      KNN_HIP(hipStreamSynchronize(s));
    };
    int count_bins = o.n_bins;
    const int64_t pstride = N / (int64_t)262144;
    if (pstride >= 8) {
      histogram(o.n_bins, pstride);
      uint64_t c = 0;
      for (int b = 0; b < o.n_bins; ++b) {
        c += hc[b] * (uint64_t)pstride;
        if (c >= 4 * need) {
          count_bins = b + 1;
          break;
        }
      }
    }
    histogram(count_bins, 1);
    auto cumulate = [&] {
      idx->cum.assign(o.n_bins, 0);
      uint64_t c = 0;
      for (int b = 0; b < o.n_bins; ++b) {
        c += hc[b];
        idx->cum[b] = c;
      }
    };
    cumulate();
    if (count_bins < o.n_bins && idx->cum[count_bins - 1] < need) {
      histogram(o.n_bins, 1);
      cumulate();
    }
    idx->hist_sample = sh;
    idx->mean_sample = sm;
    return idx;
  } catch (...) {
    delete idx;
    throw;
  }
}

void check_build_args(const void* D, int64_t N, int32_t dims, knn_index** out) {
  KNN_CHECK(D != nullptr && out != nullptr, KNN_EINVAL, "NULL pointer");
  KNN_CHECK(dims >= KNN_MIN_DIMS && dims <= KNN_MAX_DIMS, KNN_EINVAL, "dims must be in [2, 6]");
  KNN_CHECK(N >= 2 && N < (int64_t(1) << 31), KNN_EINVAL, "N must be in [2, 2^31)");
}

JoinContext& index_ctx(knn_index* idx) {
  if (!idx->ctx) {
    idx->ctx = new JoinContextHolder();
    idx->ctx->ctx.device = idx->device;
  }
  return idx->ctx->ctx;
}

knn_join_opts resolve_join(const knn_join_opts* o) {
  knn_join_opts r{};
  if (o) r = *o;
  return r;
}

// The fixed scratch area of knn_self_join_device_noalloc.  Each device that
// runs the library holds its own copy until the process ends.  Host code
// never passes the array's name to a kernel: the device address comes from
// hipGetSymbolAddress, taken once per device with that device current.
static __device__ __align__(256) char scratch[KNN_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
std::map<int, char*> g_scratch_addr;           // device -> address of its copy
std::map<int, std::mutex> g_scratch_call_mu;   // device -> serialises its users

// Address of `scratch` on device dev (dev must be current).
char* scratch_of_device(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_addr.find(dev);
  if (it != g_scratch_addr.end()) return it->second;
  void* ptr = nullptr;
  KNN_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  KNN_CHECK(ptr != nullptr, KNN_EDEVICE, "no device address for the scratch area");
  g_scratch_addr[dev] = static_cast<char*>(ptr);
  return static_cast<char*>(ptr);
}

std::mutex& scratch_call_mutex(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_call_mu[dev];  // constructed in place, never moved
}

// The join of the query set Q (device, row-major NQ x n) with the index's
// points: the queries' SoA copy and bounds (non-finite coordinates refused),
// then the level loop with the query set.
void join_query_set(knn_index* idx, const double* d_Q, int64_t NQ, int32_t K, int32_t* d_ids,
                    double* d_dists, const knn_join_opts& o, hipStream_t s) {
  const int n = idx->n;
  JoinQueries jq;
  jq.QA = d_Q;
  jq.NQ = NQ;
  DevBuf<double> QX((size_t)NQ * n);
  DevBuf<uint32_t> bad(1);
  launch_zero(bad.p, sizeof(uint32_t), s);
  launch_aos_to_soa(d_Q, NQ, n, QX.p, bad.p, s);
  DevBuf<double> part((size_t)2 * n * kBoundsBlocks), lohi(2 * kMaxDims);
  launch_bounds(QX.p, NQ, n, part.p, lohi.p, lohi.p + kMaxDims, s);
  double hb[2 * kMaxDims];
  uint32_t nbad = 0;
  KNN_HIP(hipMemcpyAsync(hb, lohi.p, sizeof(hb), hipMemcpyDeviceToHost, s));
  KNN_HIP(hipMemcpyAsync(&nbad, bad.p, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  KNN_HIP(hipStreamSynchronize(s));
  KNN_CHECK(nbad == 0, KNN_EINVAL, "Q holds non-finite coordinates");
  for (int j = 0; j < n; ++j) {
    jq.lo[j] = hb[j];
    jq.hi[j] = hb[kMaxDims + j];
  }
  jq.QX = QX.p;
  // the level loop returns after its device work completed: QX may go
  self_join(*idx, index_ctx(idx), K, d_ids, d_dists, o, s, nullptr, nullptr, &jq);
}

}  // namespace

extern "C" {

void knn_build_opts_default(knn_build_opts* o) {
  if (o) std::memset(o, 0, sizeof(*o)), o->device = -1;
}

void knn_join_opts_default(knn_join_opts* o) {
  if (o) std::memset(o, 0, sizeof(*o));
}

const char* knn_last_error(void) { return g_last_error.c_str(); }

int knn_build_index(const double* D, int64_t n_points, int32_t dims, const knn_build_opts* opts,
                    knn_index** out) {
  return guarded([&] {
    check_build_args(D, n_points, dims, out);
    knn_build_opts o = resolve(opts);
    int dev = o.device >= 0 ? o.device : current_device();
    DeviceGuard dg(dev);
    hipStream_t s = nullptr;
    KNN_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    try {
      DevBuf<double> dD((size_t)n_points * dims);
      KNN_HIP(hipMemcpyAsync(dD.p, D, (size_t)n_points * dims * sizeof(double),
                             hipMemcpyHostToDevice, s));
      *out = build_from_device(dD.p, n_points, dims, o, s);
      KNN_HIP(hipStreamSynchronize(s));
    } catch (...) {
      (void)hipStreamDestroy(s);
      throw;
    }
    KNN_HIP(hipStreamDestroy(s));
  });
}

int knn_build_index_device(const double* d_D, int64_t n_points, int32_t dims,
                           const knn_build_opts* opts, void* stream, knn_index** out) {
  return guarded([&] {
    check_build_args(d_D, n_points, dims, out);
    knn_build_opts o = resolve(opts);
    int dev = o.device >= 0 ? o.device : current_device();
    DeviceGuard dg(dev);
    *out = build_from_device(d_D, n_points, dims, o, (hipStream_t)stream);
  });
}

int knn_self_join_device(knn_index* idx, int32_t K, int32_t* d_ids, double* d_dists,
                         const knn_join_opts* opts, void* stream) {
  return guarded([&] {
    validate_join(idx, K);
    BusyGuard bg(idx);
    DeviceGuard dg(idx->device);
    knn_join_opts o = resolve_join(opts);
    if (o.use_graph)
      self_join_graph(*idx, K, d_ids, d_dists, o, (hipStream_t)stream);
    else
      self_join(*idx, index_ctx(idx), K, d_ids, d_dists, o, (hipStream_t)stream);
  });
}

int knn_join_device(knn_index* idx, const double* d_Q, int64_t n_queries, int32_t K,
                    int32_t* d_ids, double* d_dists, const knn_join_opts* opts, void* stream) {
  return guarded([&] {
    KNN_CHECK(idx != nullptr, KNN_EINVAL, "index is NULL");
    KNN_CHECK(d_Q && d_ids && d_dists, KNN_EINVAL, "NULL pointer");
    KNN_CHECK(n_queries >= 1, KNN_EINVAL, "n_queries must be >= 1");
    knn_join_opts o = resolve_join(opts);
    KNN_CHECK(o.use_graph == 0, KNN_EINVAL, "use_graph is not available for a query set");
    BusyGuard bg(idx);
    DeviceGuard dg(idx->device);
    join_query_set(idx, d_Q, n_queries, K, d_ids, d_dists, o, (hipStream_t)stream);
  });
}

int knn_join(knn_index* idx, const double* Q, int64_t n_queries, int32_t K, int32_t* ids,
             double* dists, const knn_join_opts* opts) {
  return guarded([&] {
    KNN_CHECK(idx != nullptr, KNN_EINVAL, "index is NULL");
    KNN_CHECK(Q && ids && dists, KNN_EINVAL, "NULL pointer");
    KNN_CHECK(n_queries >= 1 && n_queries < ((int64_t)1 << 31), KNN_EINVAL,
              "n_queries must be in [1, 2^31)");
    KNN_CHECK(K >= 1 && K <= KNN_MAX_K, KNN_EINVAL, "K out of range");
    knn_join_opts o = resolve_join(opts);
    KNN_CHECK(o.use_graph == 0, KNN_EINVAL, "use_graph is not available for a query set");
    BusyGuard bg(idx);
    DeviceGuard dg(idx->device);
    hipStream_t s = nullptr;
    KNN_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    try {
      const size_t nq = (size_t)n_queries * idx->n, nk = (size_t)n_queries * K;
      DevBuf<double> dQ(nq);
      DevBuf<int32_t> dI(nk);
      DevBuf<double> dD(nk);
      KNN_HIP(hipMemcpyAsync(dQ.p, Q, nq * sizeof(double), hipMemcpyHostToDevice, s));
      join_query_set(idx, dQ.p, n_queries, K, dI.p, dD.p, o, s);
      JoinContext& c = index_ctx(idx);
      copy_to_host(c.stage, ids, dI.p, nk * sizeof(int32_t), s);
      copy_to_host(c.stage, dists, dD.p, nk * sizeof(double), s);
    } catch (...) {
      (void)hipStreamSynchronize(s);
      (void)hipStreamDestroy(s);
      throw;
    }
    KNN_HIP(hipStreamDestroy(s));
  });
}

int knn_self_join_device_noalloc(knn_index* idx, int32_t K, int32_t* d_ids, double* d_dists,
                                 const knn_join_opts* opts, void* stream) {
  return guarded([&] {
    validate_join(idx, K);
    KNN_CHECK(d_ids && d_dists, KNN_EINVAL, "output pointers are NULL");
    knn_join_opts o = resolve_join(opts);
    KNN_CHECK(o.stats == nullptr, KNN_EINVAL,
              "no-allocation join: statistics (HIP events) are not available");
    KNN_CHECK(o.use_graph == 0, KNN_EINVAL,
              "no-allocation join: use_graph (a graph with scratch of its own) is not available");
    const uint64_t need = fixed_scratch_bytes(*idx, K, o);
    KNN_CHECK(need <= (uint64_t)KNN_NOALLOC_SCRATCH_BYTES, KNN_EINVAL,
              "no-allocation join: this index and K need " + std::to_string(need) +
                  " bytes of scratch, above the fixed area of " +
                  std::to_string((uint64_t)KNN_NOALLOC_SCRATCH_BYTES));
    BusyGuard bg(idx);
    DeviceGuard dg(idx->device);
    hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lk(scratch_call_mutex(idx->device));
    ArenaScope arena(scratch_of_device(idx->device), (size_t)KNN_NOALLOC_SCRATCH_BYTES);
    JoinContext c;  // destroyed before the arena scope ends
    c.device = idx->device;
    c.fixed = true;
    c.table_cap = kFixedTableFactor * idx->N;
    try {
      reserve_fixed_scratch(*idx, c, K, o, s);
      self_join(*idx, c, K, d_ids, d_dists, o, s);
    } catch (...) {
      // the next call reuses the area: let this one's work finish first
      (void)hipStreamSynchronize(s);
      throw;
    }
  });
}

int knn_self_join(knn_index* idx, int32_t K, int32_t* ids, double* dists,
                  const knn_join_opts* opts) {
  return guarded([&] {
    validate_join(idx, K);
    KNN_CHECK(ids && dists, KNN_EINVAL, "output pointers are NULL");
    BusyGuard bg(idx);
    DeviceGuard dg(idx->device);
    knn_join_opts o = resolve_join(opts);
    JoinContext& c = index_ctx(idx);
    hipStream_t s = nullptr;
    KNN_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    try {
      const size_t NK = (size_t)idx->N * K;
      c.out_ids.reserve(NK);
      c.out_d.reserve(NK);
      if (o.use_graph)
        self_join_graph(*idx, K, c.out_ids.p, c.out_d.p, o, s);
      else
        self_join(*idx, c, K, c.out_ids.p, c.out_d.p, o, s);
      copy_to_host(c.stage, ids, c.out_ids.p, NK * sizeof(int32_t), s);
      copy_to_host(c.stage, dists, c.out_d.p, NK * sizeof(double), s);
    } catch (...) {
      (void)hipStreamSynchronize(s);
      (void)hipStreamDestroy(s);
      throw;
    }
    KNN_HIP(hipStreamDestroy(s));
  });
}

void knn_destroy_index(knn_index* idx) {
  if (!idx) return;
  try {
    DeviceGuard dg(idx->device);
    delete idx->graph;
    idx->graph = nullptr;
    delete idx->ctx;
    idx->ctx = nullptr;
    destroy_eps_state(idx->eps);
    idx->eps = nullptr;
    destroy_hybrid_state(idx->hybrid);
    idx->hybrid = nullptr;
    delete idx;
  } catch (...) {
  }
}

int knn_index_info_get(const knn_index* idx, knn_index_info* out) {
  return guarded([&] {
    KNN_CHECK(idx && out, KNN_EINVAL, "NULL pointer");
    std::memset(out, 0, sizeof(*out));
    out->n_points = idx->N;
    out->dims = idx->n;
    out->device = idx->device;
    for (int j = 0; j < idx->n; ++j) {
      out->lo[j] = idx->lo[j];
      out->hi[j] = idx->hi[j];
    }
    out->eps_mean = idx->eps_mean;
    out->n_bins = idx->n_bins;
    out->n_sample = idx->n_sample;
    out->device_bytes = (int64_t)(idx->X.bytes() + idx->XA.bytes()) +
                        (idx->ctx ? idx->ctx->ctx.device_bytes() : 0) +
                        (idx->graph ? idx->graph->ctx.device_bytes() : 0);
  });
}

int knn_index_sampling_get(const knn_index* idx, int64_t* hist_sample, int64_t* mean_sample,
                           int64_t* n_mean, uint64_t* counts, double* bin_width) {
  return guarded([&] {
    KNN_CHECK(idx != nullptr, KNN_EINVAL, "index is NULL");
    if (hist_sample)
      std::copy(idx->hist_sample.begin(), idx->hist_sample.end(), hist_sample);
    if (mean_sample)
      std::copy(idx->mean_sample.begin(), idx->mean_sample.end(), mean_sample);
    if (n_mean) *n_mean = (int64_t)idx->mean_sample.size();
    if (counts)
      for (int b = 0; b < idx->n_bins; ++b) counts[b] = idx->cum[b] - (b ? idx->cum[b - 1] : 0);
    if (bin_width) *bin_width = idx->bin_width;
  });
}

int knn_autotune(knn_index* idx, int32_t K, void* stream, knn_autotune_result* out) {
  return guarded([&] {
    validate_join(idx, K);
    KNN_CHECK(out != nullptr, KNN_EINVAL, "NULL pointer");
    BusyGuard bg(idx);
    DeviceGuard dg(idx->device);
    hipStream_t s = (hipStream_t)stream;
    JoinContext& c = index_ctx(idx);
    const size_t NK = (size_t)idx->N * K;
    c.out_ids.reserve(NK);
    c.out_d.reserve(NK);
    int ls_cur = 0;  // lanes shift of the trials (last stages)
    int pops_cur = 4;  // pops per wavefront of the trials (last stage)
    int z_cur = -1;  // level structure of the trials: -1 row-major, 1 Z-order
    auto time_join = [&](double wf, double gr, int lin, double tp) {
      double best = 1e300;
      for (int rep = 0; rep < 2; ++rep) {
        knn_join_opts o{};
        o.w_factor = wf;
        o.growth = gr;
        o.linear_levels = lin;
        o.tail_pairs = tp;
        o.lanes_shift = ls_cur;
        o.zorder = z_cur;
        o.queue_grain = -pops_cur;
        KNN_HIP(hipStreamSynchronize(s));
        auto t0 = std::chrono::steady_clock::now();
        self_join(*idx, c, K, c.out_ids.p, c.out_d.p, o, s);
        KNN_HIP(hipStreamSynchronize(s));
        best = std::min(best, std::chrono::duration<double, std::milli>(
                                  std::chrono::steady_clock::now() - t0).count());
      }
      return best;
    };
    // Staged search.  Row-major levels: the level-0 cell side first (default
    // growth, the paper's linear first step), then growth x linear step for
    // the best side, then the side again around the best at that growth,
    // then the brute-force tail budget.  Z-order levels (2-4 dimensions,
    // growth 2 by construction): the level-0 side, then the tail budget.
    // Last, the lanes-per-query rule for the overall best.
    const double n = (double)idx->n;
    const double g16 = std::pow(16.0, 1.0 / n);
    const double tp0 = 2.5e8;
    std::memset(out, 0, sizeof(*out));
    out->ms_default = time_join(1.0, g16, 1, tp0);
    out->ms_best = out->ms_default;
    out->w_factor = 1.0;
    out->growth = g16;
    out->linear_levels = 1;
    out->tail_pairs = tp0;
    out->zorder = -1;
    out->trials = 1;
    auto consider = [&](double wf, double gr, int lin, double tp) {
      const double ms = time_join(wf, gr, lin, tp);
      ++out->trials;
      if (ms < out->ms_best) {
        out->ms_best = ms;
        out->w_factor = wf;
        out->growth = gr;
        out->linear_levels = lin;
        out->tail_pairs = tp;
        out->zorder = z_cur;
      }
    };
    for (double wf : {0.25, 0.5, 0.7, 1.4, 2.0}) consider(wf, g16, 1, tp0);
    // the best side at the edge of the range: two more beyond it
    if (out->w_factor >= 2.0)
      for (double wf : {2.8, 4.0}) consider(wf, g16, 1, tp0);
    const double wf1 = out->w_factor;
    for (double gb : {4.0, 16.0, 64.0})
      for (int lin : {1, -1}) {
        const double gr = std::pow(gb, 1.0 / n);
        if (gb == 16.0 && lin == 1) continue;  // measured in the first stage
        consider(wf1, gr, lin, tp0);
      }
    // the fastest (slowest) growth best: one faster (slower)
    if (out->growth >= std::pow(64.0, 1.0 / n) * 0.999)
      consider(wf1, std::pow(256.0, 1.0 / n), out->linear_levels, tp0);
    else if (out->growth <= std::pow(4.0, 1.0 / n) * 1.001)
      consider(wf1, std::pow(2.0, 1.0 / n), out->linear_levels, tp0);
    const double gr2 = out->growth;
    const int lin2 = out->linear_levels;
    for (double f : {0.8, 1.25}) consider(wf1 * f, gr2, lin2, tp0);
    // the best uses the linear first step: also start straight at that
    // step's side (w + 0.5 w), without it (a level 0 that defers nearly every
    // query costs its whole build for nothing)
    if (out->linear_levels == 1) consider(out->w_factor * 1.5, out->growth, -1, tp0);
    const double wf3 = out->w_factor;
    const double gr3 = out->growth;
    const int lin3 = out->linear_levels;
    for (double tp : {6e7, 1e9}) consider(wf3, gr3, lin3, tp);
    if (idx->n <= kZMaxDims) {
      // Z-order levels: levels are cheap, so finer level-0 sides are in range
      z_cur = 1;
      const double rm_best = out->ms_best;
      double zbest = 1e300, zwf = 0;
      auto try_z = [&](double wf) {
        const double ms = time_join(wf, 2.0, -1, tp0);
        ++out->trials;
        if (ms < zbest) {
          zbest = ms;
          zwf = wf;
        }
      };
      for (double wf : {0.0625, 0.125, 0.25, 0.5, 1.0}) try_z(wf);
      // the best side at the edge of the range: one more beyond it
      if (zwf <= 0.0625)
        try_z(0.03125);
      else if (zwf >= 1.0)
        try_z(2.0);
      const double zwf1 = zwf;
      for (double f : {0.7, 1.4}) try_z(zwf1 * f);
      // and once more, finer, around the best of those
      const double zwf2 = zwf;
      for (double f : {0.85, 1.18}) try_z(zwf2 * f);
      if (zbest < rm_best) {
        out->ms_best = zbest;
        out->w_factor = zwf;
        out->growth = 2.0;
        out->linear_levels = -1;
        out->tail_pairs = tp0;
        out->zorder = 1;
        for (double tp : {6e7, 1e9}) consider(zwf, 2.0, -1, tp);
      }
      z_cur = out->zorder;
    }
    // the lanes-per-query rule, halved or doubled at every level
    const double wf4 = out->w_factor, gr4 = out->growth, tp4 = out->tail_pairs;
    const int lin4 = out->linear_levels;
    out->lanes_shift = 0;
    for (int ls : {-1, 1}) {
      ls_cur = ls;
      const double before = out->ms_best;
      consider(wf4, gr4, lin4, tp4);
      if (out->ms_best < before) out->lanes_shift = ls;
    }
    // the queue granularity of the persistent search: pops per wavefront and
    // queue (few: fewer atomics on the queue heads; many: finer balance at the
    // end of each queue when dense items cluster)
    ls_cur = out->lanes_shift;
    out->queue_pops = 4;
    for (int pp : {8, 16, 32, 64}) {
      pops_cur = pp;
      const double before = out->ms_best;
      consider(wf4, gr4, lin4, tp4);
      if (out->ms_best < before) out->queue_pops = pp;
    }
    // last, the level-0 side once more with the chosen lanes and queue
    // granularity (the best side shifts with them)
    pops_cur = out->queue_pops;
    for (double f : {0.8, 1.25})
      consider(out->w_factor * f, out->growth, out->linear_levels, out->tail_pairs);
    pops_cur = 4;
    ls_cur = 0;
    autotune_store(idx->n, K, idx->N,
                   TuneEntry{out->w_factor, out->growth, 0, out->linear_levels > 0 ? 1 : -1,
                             out->tail_pairs, out->lanes_shift, out->zorder, out->queue_pops});
  });
}

int knn_autotune_save(const char* path) {
  return guarded([&] { KNN_CHECK(autotune_save(path) == 0, KNN_EINVAL, "cannot write the cache"); });
}

int knn_autotune_load(const char* path) {
  return guarded([&] { KNN_CHECK(autotune_load(path) == 0, KNN_EINVAL, "cannot read the cache"); });
}

int knn_join_footprint(const knn_index* idx, int32_t K, uint64_t* bytes) {
  return guarded([&] {
    KNN_CHECK(bytes != nullptr, KNN_EINVAL, "NULL pointer");
    validate_join(idx, K);
    *bytes = join_footprint(*idx, K, true);
  });
}

int knn_eps_min(const knn_index* idx, int32_t K, double* eps_min) {
  return guarded([&] {
    KNN_CHECK(idx && eps_min, KNN_EINVAL, "NULL pointer");
    KNN_CHECK(K >= 1, KNN_EINVAL, "K must be >= 1");
    *eps_min = eps_min_of(*idx, K);
  });
}

int knn_grid_export(knn_index* idx, double cell_width, uint64_t* sorted_keys, int32_t* perm,
                    uint64_t* cell_keys, uint32_t* cell_start, uint32_t* ranges,
                    int64_t* grid_dims, int64_t* n_cells) {
  return guarded([&] {
    KNN_CHECK(idx != nullptr, KNN_EINVAL, "index is NULL");
    KNN_CHECK(cell_width > 0 && std::isfinite(cell_width), KNN_EINVAL, "cell_width must be > 0");
    BusyGuard bg(idx);
    DeviceGuard dg(idx->device);
    JoinContext& c = index_ctx(idx);
    hipStream_t s = nullptr;
    KNN_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    try {
      build_level(*idx, c, cell_width, s);
      uint32_t M32 = 0;
      KNN_HIP(hipMemcpyAsync(&M32, c.scal.p, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
      KNN_HIP(hipStreamSynchronize(s));
      c.M = M32;
      const int64_t N = idx->N, M = c.M, R = pow3(idx->n - 1);
      if (sorted_keys)
        KNN_HIP(hipMemcpyAsync(sorted_keys, c.keys.p, N * 8, hipMemcpyDeviceToHost, s));
      if (perm) KNN_HIP(hipMemcpyAsync(perm, c.perm.p, N * 4, hipMemcpyDeviceToHost, s));
      if (cell_keys) KNN_HIP(hipMemcpyAsync(cell_keys, c.cell_key.p, M * 8, hipMemcpyDeviceToHost, s));
      if (cell_start)
        KNN_HIP(hipMemcpyAsync(cell_start, c.cell_start.p, (M + 1) * 4, hipMemcpyDeviceToHost, s));
      std::vector<uint32_t> hr, hn;
      std::vector<uint8_t> hs;
      if (ranges) {
        hr.resize((size_t)M * R * 4);
        hs.resize((size_t)M * R);
        hn.resize((size_t)M);
        KNN_HIP(hipMemcpyAsync(hr.data(), c.ranges.p, M * R * 4 * 4, hipMemcpyDeviceToHost, s));
        KNN_HIP(hipMemcpyAsync(hs.data(), c.rslot.p, M * R, hipMemcpyDeviceToHost, s));
        KNN_HIP(hipMemcpyAsync(hn.data(), c.nrng.p, M * 4, hipMemcpyDeviceToHost, s));
      }
      KNN_HIP(hipStreamSynchronize(s));
      if (ranges) {
        // compacted segments -> one slot per segment, (0, 0) where empty
        std::memset(ranges, 0, (size_t)M * R * 2 * 4);
        for (int64_t cc = 0; cc < M; ++cc)
          for (uint32_t i = 0; i < hn[cc]; ++i) {
            const int64_t r = hs[cc * R + i];
            ranges[(cc * R + r) * 2] = hr[(cc * R + i) * 4];
            ranges[(cc * R + r) * 2 + 1] = hr[(cc * R + i) * 4 + 3];
          }
      }
      if (grid_dims)
        for (int j = 0; j < idx->n; ++j) grid_dims[j] = c.gg.g[j];
      if (n_cells) *n_cells = M;
    } catch (...) {
      (void)hipStreamSynchronize(s);
      (void)hipStreamDestroy(s);
      throw;
    }
    KNN_HIP(hipStreamDestroy(s));
  });
}

int knn_sample_mean_dist(const double* d_D, int64_t n_points, int32_t dims,
                         const int64_t* d_sample, int64_t ns, double* mean, void* stream) {
  return guarded([&] {
    KNN_CHECK(d_D && d_sample && mean, KNN_EINVAL, "NULL pointer");
    KNN_CHECK(dims >= 1 && dims <= KNN_MAX_DIMS && n_points >= 1 && ns >= 0, KNN_EINVAL,
              "bad sizes");
    hipStream_t s = (hipStream_t)stream;
    DevBuf<double> X((size_t)n_points * dims);
    DevBuf<uint32_t> bad(1);
    KNN_HIP(hipMemsetAsync(bad.p, 0, 4, s));
    launch_aos_to_soa(d_D, n_points, dims, X.p, bad.p, s);
    DevBuf<double> part(std::max<int64_t>(ns, 1));
    DevBuf<double> sx(std::max<int64_t>(ns * dims, 1));
    int np = launch_sample_pair_sums(X.p, n_points, dims, d_sample, ns, sx.p, part.p, s);
    std::vector<double> hp(np);
    if (np) KNN_HIP(hipMemcpyAsync(hp.data(), part.p, np * 8, hipMemcpyDeviceToHost, s));
    KNN_HIP(hipStreamSynchronize(s));
    double sum = 0;
    for (double v : hp) sum += v;
    double pairs = (double)ns * (double)(ns - 1) / 2.0;
    *mean = pairs > 0 ? sum / pairs : 0.0;
  });
}

int knn_dist_histogram(const double* d_D, int64_t n_points, int32_t dims, const int64_t* d_sample,
                       int64_t ns, double inv_bin_width, int32_t n_bins, uint64_t* d_counts,
                       void* stream) {
  return guarded([&] {
    KNN_CHECK(d_D && d_sample && d_counts, KNN_EINVAL, "NULL pointer");
    KNN_CHECK(dims >= 1 && dims <= KNN_MAX_DIMS && n_points >= 1 && ns >= 0, KNN_EINVAL,
              "bad sizes");
    KNN_CHECK(inv_bin_width > 0 && std::isfinite(inv_bin_width), KNN_EINVAL,
              "inv_bin_width must be > 0");
    hipStream_t s = (hipStream_t)stream;
    DevBuf<double> X((size_t)n_points * dims);
    DevBuf<uint32_t> bad(1);
    KNN_HIP(hipMemsetAsync(bad.p, 0, 4, s));
    launch_aos_to_soa(d_D, n_points, dims, X.p, bad.p, s);
    launch_dist_histogram(X.p, n_points, dims, d_sample, ns, inv_bin_width, n_bins, d_counts, s);
    KNN_HIP(hipStreamSynchronize(s));  // X is freed on return
  });
}

}  // extern "C"
