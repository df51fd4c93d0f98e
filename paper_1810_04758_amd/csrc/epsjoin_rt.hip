// epsjoin_rt.hip -- host runtime of the distance similarity self-join (every
// pair within eps; Sec. 1 and Sec. 3): the grid level of cell side eps
// (Sec. 3.1), exact per-query counts and their prefix, the sampled result-size
// estimate, batches that fit a result buffer (Sec. 3.2), and the streaming of
// batches to host memory on several streams with copies overlapping the
// kernels (Sec. 3.2's multi-stream scheme).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "index.hpp"

namespace knn {

// One stream of the host streaming path with its batch buffers (device and
// pinned host), kept between calls.
struct EpsSlot {
  hipStream_t s = nullptr;
  hipEvent_t done = nullptr;
  DevBuf<int32_t> dq, dj;
  DevBuf<double> dd;
  int32_t* hq = nullptr;
  int32_t* hj = nullptr;
  double* hd = nullptr;
  size_t host_cap = 0;
  EpsSlot() = default;
  EpsSlot(const EpsSlot&) = delete;
  EpsSlot& operator=(const EpsSlot&) = delete;
  void free_host() {
    if (hq) (void)hipHostFree(hq);
    if (hj) (void)hipHostFree(hj);
    if (hd) (void)hipHostFree(hd);
    hq = hj = nullptr;
    hd = nullptr;
    host_cap = 0;
  }
  void ensure(size_t per) {
    if (!s) {
      KNN_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
      KNN_HIP(hipEventCreateWithFlags(&done, hipEventDisableTiming));
    }
    dq.reserve(per);
    dj.reserve(per);
    dd.reserve(per);
    if (host_cap < per) {
      free_host();
      KNN_HIP(hipHostMalloc((void**)&hq, per * sizeof(int32_t), hipHostMallocDefault));
      KNN_HIP(hipHostMalloc((void**)&hj, per * sizeof(int32_t), hipHostMallocDefault));
      KNN_HIP(hipHostMalloc((void**)&hd, per * sizeof(double), hipHostMallocDefault));
      host_cap = per;
    }
  }
  ~EpsSlot() {
    if (s) (void)hipStreamSynchronize(s);
    free_host();
    if (done) (void)hipEventDestroy(done);
    if (s) (void)hipStreamDestroy(s);
  }
};

// What an index keeps between calls for the eps it last joined with: the
// grid level (sorted order = the processing order the cursors refer to) and,
// once counted, the exact per-position counts and their prefix.
struct EpsJoinState {
  bool level = false;
  uint64_t eps_bits = 0;  // eps of the level (bit pattern)
  double w = 0, t = 0, margin = 0;
  int32_t R = 0;
  bool counted = false;  // counts / off hold the exact counts of this level
  uint64_t total = 0;
  JoinContext ctx;
  DevBuf<uint32_t> counts;
  DevBuf<uint64_t> off, tiles;
  DevBuf<int64_t> small;  // batch bounds read-back
  HostBuf<int64_t> pinned;
  // host streaming: a control stream and the batch streams, created on
  // first use (the buffers grow to the largest batch asked for)
  hipStream_t control = nullptr;
  std::vector<std::unique_ptr<EpsSlot>> slots;
  ~EpsJoinState() {
    slots.clear();
    if (control) {
      (void)hipStreamSynchronize(control);
      (void)hipStreamDestroy(control);
    }
  }
};

void destroy_eps_state(EpsJoinState* st) { delete st; }

namespace {

constexpr int64_t kBoundsPerLaunch = 4096;

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

uint64_t bits_of(double x) {
  uint64_t b;
  std::memcpy(&b, &x, sizeof b);
  return b;
}

// The largest double t with fl(sqrt(t)) <= eps: sqrt is monotone and
// correctly rounded, so fl(sqrt(d2)) <= eps exactly when d2 <= t.
double sq_limit(double eps) {
  double t = eps * eps;
  while (t > 0 && std::sqrt(t) > eps) t = std::nextafter(t, 0.0);
  for (;;) {
    const double up = std::nextafter(t, INFINITY);
    if (!std::isfinite(up) || std::sqrt(up) > eps) break;
    t = up;
  }
  return t;
}

void check_eps(const knn_index* idx, double eps) {
  KNN_CHECK(idx != nullptr, KNN_EINVAL, "index is NULL");
  KNN_CHECK(std::isfinite(eps) && eps >= 0, KNN_EINVAL, "eps must be finite and >= 0");
}

EpsJoinState& state_of(knn_index* idx) {
  if (!idx->eps) {
    idx->eps = new EpsJoinState();
    idx->eps->ctx.device = idx->device;
  }
  return *idx->eps;
}

// The grid level of eps into st (kept while eps stays the same).  Cell side
// w = eps (1 + 2^-16): a cell coordinate carries at most (8 g + 4n + 32)
// 2^-53 cells of rounding (g <= 2^30 cells per dimension), far below 2^-16,
// so every point within eps of a query -- in fact within
// eps (1 + 2^-17) -- lies in the 3^n block of its cell.  A pair whose
// squared distance underflows can be computed as within eps while its true
// distance is not (below 2^-500 the squares are subnormal); a side of at
// least 2^-500 covers those too.  The side is also kept at or above 2^-29 of
// the largest extent (a grid of at most 2^29 cells per dimension).
void ensure_level(const knn_index& idx, EpsJoinState& st, double eps, hipStream_t s) {
  if (st.level && st.eps_bits == bits_of(eps)) return;
  st.level = false;
  st.counted = false;
  const int n = idx.n;
  double ext = 0;
  for (int j = 0; j < n; ++j) ext = std::max(ext, idx.hi[j] - idx.lo[j]);
  double w = std::max({eps * (1.0 + 0x1p-16), 0x1p-500, ext * 0x1p-29});
  (void)make_geom(n, idx.lo, idx.hi, w);  // the side the level will really use
  build_level(idx, st.ctx, w, s);
  st.w = w;
  st.t = sq_limit(eps);
  st.margin = (8.0 * (double)st.ctx.gg.g_max + 4.0 * n + 32.0) * 0x1p-53;
  int64_t R = 1;
  for (int j = 0; j + 1 < n; ++j) R *= 3;
  st.R = (int32_t)R;
  st.eps_bits = bits_of(eps);
  st.level = true;
}

EpsPassArgs pass_args(const knn_index& idx, EpsJoinState& st) {
  EpsPassArgs a{};
  JoinContext& c = st.ctx;
  a.Xs = c.Xs.p;
  a.N = idx.N;
  a.perm = c.perm.p;
  a.cell_of = c.cell_of.p;
  a.ranges = c.ranges.p;
  a.rslot = c.rslot.p;
  a.nrng = c.nrng.p;
  a.R = st.R;
  a.gg = c.gg;
  a.w = st.w;
  a.margin = st.margin;
  a.t = st.t;
  return a;
}

// Exact counts of every position and their prefix (kept for this eps).
void ensure_counts(const knn_index& idx, EpsJoinState& st, hipStream_t s) {
  if (st.counted) return;
  const int64_t N = idx.N;
  st.counts.reserve(N);
  st.off.reserve(N + 1);
  st.tiles.reserve(eps_scan_tiles(N));
  EpsPassArgs a = pass_args(idx, st);
  a.stride = 1;
  a.counts = st.counts.p;
  launch_eps_count(a, s);
  launch_offsets(st.counts.p, N, st.tiles.p, st.off.p, s);
  st.pinned.reserve(4);
  KNN_HIP(hipMemcpyAsync(st.pinned.p, st.off.p + N, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
  KNN_HIP(hipStreamSynchronize(s));
  std::memcpy(&st.total, st.pinned.p, sizeof(uint64_t));
  st.counted = true;
}

// Up to maxb batches from position `first` (cap pairs each): end positions
// and end offsets into `ends` (pairs), the offset of `first` into *start.
void batch_bounds(const knn_index& idx, EpsJoinState& st, int64_t first, uint64_t cap,
                  int64_t maxb, std::vector<int64_t>& ends, uint64_t* start, hipStream_t s) {
  st.small.reserve(3 + 2 * maxb);
  st.pinned.reserve(3 + 2 * maxb);
  launch_batch_bounds(st.off.p, idx.N, first, cap, maxb, st.small.p + 3, st.small.p, s);
  KNN_HIP(hipMemcpyAsync(st.pinned.p, st.small.p, 3 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  KNN_HIP(hipStreamSynchronize(s));
  const int64_t nb = st.pinned.p[0];
  *start = (uint64_t)st.pinned.p[1];
  KNN_CHECK(nb >= 0, KNN_EINVAL,
            "capacity of " + std::to_string(cap) + " pairs is below the " +
                std::to_string(st.pinned.p[2]) + " pairs of the query at cursor " +
                std::to_string(first));
  ends.resize(2 * nb);
  if (nb > 0) {
    KNN_HIP(hipMemcpyAsync(st.pinned.p + 3, st.small.p + 3, 2 * nb * sizeof(int64_t),
                           hipMemcpyDeviceToHost, s));
    KNN_HIP(hipStreamSynchronize(s));
    std::memcpy(ends.data(), st.pinned.p + 3, 2 * nb * sizeof(int64_t));
  }
}

void write_batch(const knn_index& idx, EpsJoinState& st, int64_t first, int64_t last,
                 int32_t* q, int32_t* j, double* d, hipStream_t s) {
  EpsPassArgs a = pass_args(idx, st);
  a.first = first;
  a.last = last;
  a.off = st.off.p;
  a.out_q = q;
  a.out_j = j;
  a.out_d = d;
  launch_eps_write(a, s);
}

}  // namespace

}  // namespace knn

using namespace knn;

extern "C" {

int knn_eps_join_size(knn_index* idx, double eps, int64_t sample_stride, uint64_t* n_pairs,
                      int32_t* d_counts, void* stream) {
  return guarded([&] {
    check_eps(idx, eps);
    KNN_CHECK(n_pairs != nullptr, KNN_EINVAL, "n_pairs is NULL");
    KNN_CHECK(sample_stride >= 1, KNN_EINVAL, "sample_stride must be >= 1");
    KNN_CHECK(d_counts == nullptr || sample_stride == 1, KNN_EINVAL,
              "per-point counts need sample_stride 1");
    BusyGuard bg(idx);
    DeviceGuard dg(idx->device);
    hipStream_t s = (hipStream_t)stream;
    EpsJoinState& st = state_of(idx);
    ensure_level(*idx, st, eps, s);
    const int64_t N = idx->N;
    if (sample_stride == 1) {
      ensure_counts(*idx, st, s);
      if (d_counts) {
        launch_counts_by_id(st.counts.p, st.ctx.perm.p, N, d_counts, s);
        KNN_HIP(hipStreamSynchronize(s));
      }
      *n_pairs = st.total;
      return;
    }
    // the estimate: the pairs of every sample_stride-th position (a sample
    // spread evenly over the cells), scaled to all positions
    const int64_t ns = ceil_div(N, sample_stride);
    st.counted = false;  // the count buffer now holds the sample's
    st.counts.reserve(N);
    st.off.reserve(N + 1);
    st.tiles.reserve(eps_scan_tiles(N));
    EpsPassArgs a = pass_args(*idx, st);
    a.stride = sample_stride;
    a.counts = st.counts.p;
    launch_eps_count(a, s);
    launch_offsets(st.counts.p, ns, st.tiles.p, st.off.p, s);
    st.pinned.reserve(4);
    KNN_HIP(hipMemcpyAsync(st.pinned.p, st.off.p + ns, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    KNN_HIP(hipStreamSynchronize(s));
    uint64_t sampled = 0;
    std::memcpy(&sampled, st.pinned.p, sizeof(uint64_t));
    *n_pairs = (uint64_t)std::llround((double)sampled * (double)N / (double)ns);
  });
}

int knn_eps_join_device(knn_index* idx, double eps, int64_t cursor, uint64_t capacity,
                        int32_t* d_qids, int32_t* d_nids, double* d_dists, uint64_t* n_pairs,
                        int64_t* next_cursor, void* stream) {
  return guarded([&] {
    check_eps(idx, eps);
    KNN_CHECK(n_pairs && next_cursor, KNN_EINVAL, "n_pairs / next_cursor is NULL");
    KNN_CHECK(cursor >= 0 && cursor <= idx->N, KNN_EINVAL, "cursor outside [0, n_points]");
    KNN_CHECK(capacity == 0 || (d_qids && d_nids && d_dists), KNN_EINVAL, "output pointer is NULL");
    BusyGuard bg(idx);
    DeviceGuard dg(idx->device);
    hipStream_t s = (hipStream_t)stream;
    EpsJoinState& st = state_of(idx);
    ensure_level(*idx, st, eps, s);
    ensure_counts(*idx, st, s);
    *n_pairs = 0;
    *next_cursor = cursor;
    if (cursor == idx->N) return;
    std::vector<int64_t> ends;
    uint64_t start = 0;
    batch_bounds(*idx, st, cursor, capacity, 1, ends, &start, s);
    const int64_t last = ends[0];
    write_batch(*idx, st, cursor, last, d_qids, d_nids, d_dists, s);
    *n_pairs = (uint64_t)ends[1] - start;
    *next_cursor = last;
  });
}

int knn_eps_join(knn_index* idx, double eps, uint64_t batch_pairs, int32_t n_streams,
                 knn_eps_consumer consume, void* user, knn_eps_join_stats* stats) {
  return guarded([&] {
    check_eps(idx, eps);
    KNN_CHECK(consume != nullptr, KNN_EINVAL, "consumer is NULL");
    KNN_CHECK(n_streams >= 0 && n_streams <= 8, KNN_EINVAL, "n_streams must be in [0, 8]");
    const int S = n_streams == 0 ? 3 : n_streams;
    const uint64_t cap = batch_pairs == 0 ? (uint64_t)100000000 : batch_pairs;
    BusyGuard bg(idx);
    DeviceGuard dg(idx->device);
    const double t0 = now_ms();
    knn_eps_join_stats sts{};
    EpsJoinState& st = state_of(idx);
    if (!st.control) KNN_HIP(hipStreamCreateWithFlags(&st.control, hipStreamNonBlocking));
    hipStream_t s0 = st.control;
    ensure_level(*idx, st, eps, s0);
    ensure_counts(*idx, st, s0);  // synchronises s0: the level and counts are done
    sts.ms_count = now_ms() - t0;
    sts.n_pairs = st.total;
    // batch b runs on slot b % S: its kernel and its copy to the slot's host
    // buffers are queued while earlier batches are still copied or consumed;
    // a slot's buffers are reused only after the consumer has returned from
    // the batch S before
    const size_t per = (size_t)std::min<uint64_t>(cap, std::max<uint64_t>(st.total, 1));
    while ((int)st.slots.size() < S) st.slots.emplace_back(new EpsSlot());
    std::vector<uint64_t> count_of;  // pairs of the batches issued, by batch
    int64_t issued = 0, consumed = 0;
    auto finish = [&](int64_t b) {
      EpsSlot& sl = *st.slots[b % S];
      const double w0 = now_ms();
      KNN_HIP(hipEventSynchronize(sl.done));
      const double w1 = now_ms();
      sts.ms_wait += w1 - w0;
      const int rc = consume(sl.hq, sl.hj, sl.hd, count_of[b], user);
      sts.ms_consume += now_ms() - w1;
      KNN_CHECK(rc == 0, KNN_ECANCELED,
                "the consumer stopped the join (returned " + std::to_string(rc) + ")");
      ++consumed;
    };
    try {
      int64_t cursor = 0;
      std::vector<int64_t> ends;
      while (cursor < idx->N) {
        uint64_t start = 0;
        batch_bounds(*idx, st, cursor, cap, kBoundsPerLaunch, ends, &start, s0);
        const int64_t nb = (int64_t)ends.size() / 2;
        for (int64_t k = 0; k < nb; ++k) {
          const int64_t b = issued;
          if (b >= S) finish(b - S);
          EpsSlot& sl = *st.slots[b % S];
          sl.ensure(per);  // no-op once sized (the slot's last batch is consumed)
          const int64_t last = ends[2 * k];
          const uint64_t np = (uint64_t)ends[2 * k + 1] - start;
          write_batch(*idx, st, cursor, last, sl.dq.p, sl.dj.p, sl.dd.p, sl.s);
          if (np > 0) {
            KNN_HIP(hipMemcpyAsync(sl.hq, sl.dq.p, np * sizeof(int32_t), hipMemcpyDeviceToHost, sl.s));
            KNN_HIP(hipMemcpyAsync(sl.hj, sl.dj.p, np * sizeof(int32_t), hipMemcpyDeviceToHost, sl.s));
            KNN_HIP(hipMemcpyAsync(sl.hd, sl.dd.p, np * sizeof(double), hipMemcpyDeviceToHost, sl.s));
          }
          KNN_HIP(hipEventRecord(sl.done, sl.s));
          count_of.push_back(np);
          ++issued;
          cursor = last;
          start = (uint64_t)ends[2 * k + 1];
        }
      }
      while (consumed < issued) finish(consumed);
      sts.n_batches = issued;
    } catch (...) {
      for (auto& sl : st.slots)
        if (sl->s) (void)hipStreamSynchronize(sl->s);
      throw;
    }
    sts.ms_total = now_ms() - t0;
    if (stats) *stats = sts;
  });
}

int knn_eps_join_release(knn_index* idx) {
  return guarded([&] {
    KNN_CHECK(idx != nullptr, KNN_EINVAL, "index is NULL");
    BusyGuard bg(idx);
    DeviceGuard dg(idx->device);
    destroy_eps_state(idx->eps);
    idx->eps = nullptr;
  });
}

}  // extern "C"
