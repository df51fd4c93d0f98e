// hybrid.hip -- the hybrid CPU/GPU KNN self-join (Sec. 4.1-4.5): one work
// queue of the query points ordered from most to least estimated work (the
// point count of each point's cell at eps_min, Sec. 4.5); the GPU takes
// batches from the dense end, searches each at one eps and hands the queries
// that fail back to the queue (Alg. 1), growing eps by eps_min / 2 when more
// than a quarter of a batch failed; host threads take small batches from the
// sparse end and solve them with an exact kd-tree search (Sec. 4.2.1, Fig. of
// the work example).  Batch schedule: monolithic GPU batches that halve
// every round while a window of queries stays reserved for the CPU, then
// small GPU batches; at 95 % of the queries done the small batch sizes halve
// (Sec. 4.5, Table of the reconfiguration operations).
#pragma clang fp contract(off)

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "index.hpp"

namespace knn {

// ---------------------------------------------------------------------------
// Host kd-tree of the CPU component: median splits on the dimension of the
// largest spread (Bentley 1975), leaves of at most kLeaf points stored
// contiguously, an implicit complete binary tree (node i has children 2i+1
// and 2i+2), so subtrees are built in parallel without sharing anything.
// Searches keep the K smallest (d^2, id) and prune a subtree only when the
// squared distance to its splitting plane, rounded as the distances are,
// exceeds the current K-th d^2: exact under the library's distance rounding.
// ---------------------------------------------------------------------------
struct HostKdTree {
  static constexpr int kLeaf = 12;
  int n = 0;
  int64_t N = 0;
  int depth = 0;                // internal levels
  std::vector<double> pts;      // leaf order, point-major N x n
  std::vector<int32_t> ids;     // id of each leaf-order point
  std::vector<double> split;    // internal nodes
  std::vector<int8_t> sdim;
  std::vector<int64_t> first;   // leaves: start of each leaf (size leaves + 1)

  static int64_t count_leaves(int64_t N_, int& d) {
    d = 0;
    while ((N_ >> d) > kLeaf) ++d;
    return (int64_t)1 << d;
  }
};

namespace {

using Clock = std::chrono::steady_clock;

double ms_since(Clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
}

// Builds the subtree of node `node` (internal level `lvl`) over ord[b, e).
void kd_build(HostKdTree& t, const double* X, std::vector<int32_t>& ord, int64_t b, int64_t e,
              int64_t node, int lvl, int par_levels) {
  const int n = t.n;
  if (lvl == t.depth) {
    const int64_t leaf = node - (((int64_t)1 << t.depth) - 1);
    t.first[leaf] = b;
    for (int64_t i = b; i < e; ++i) {
      const int32_t id = ord[i];
      t.ids[i] = id;
      for (int j = 0; j < n; ++j) t.pts[(size_t)i * n + j] = X[(size_t)id * n + j];
    }
    return;
  }
  int dim = 0;
  double best = -1;
  for (int j = 0; j < n; ++j) {
    double lo = INFINITY, hi = -INFINITY;
    for (int64_t i = b; i < e; ++i) {
      const double v = X[(size_t)ord[i] * n + j];
      lo = std::min(lo, v);
      hi = std::max(hi, v);
    }
    if (e > b && hi - lo > best) {
      best = hi - lo;
      dim = j;
    }
  }
  // the halves' sizes follow the leaf count of each subtree, so every leaf
  // holds about N / 2^depth points
  const int64_t m = b + (e - b) / 2;
  if (e > b) {
    std::nth_element(ord.begin() + b, ord.begin() + m, ord.begin() + e,
                     [&](int32_t a, int32_t c) { return X[(size_t)a * n + dim] < X[(size_t)c * n + dim]; });
    t.split[node] = X[(size_t)ord[m] * n + dim];
  } else {
    t.split[node] = 0.0;
  }
  t.sdim[node] = (int8_t)dim;
  // left: values <= split, right: values >= split
  if (lvl < par_levels) {
    std::thread th([&] { kd_build(t, X, ord, b, m, 2 * node + 1, lvl + 1, par_levels); });
    kd_build(t, X, ord, m, e, 2 * node + 2, lvl + 1, par_levels);
    th.join();
  } else {
    kd_build(t, X, ord, b, m, 2 * node + 1, lvl + 1, par_levels);
    kd_build(t, X, ord, m, e, 2 * node + 2, lvl + 1, par_levels);
  }
}

std::unique_ptr<HostKdTree> kd_create(const double* X, int64_t N, int n, int threads) {
  auto t = std::make_unique<HostKdTree>();
  t->n = n;
  t->N = N;
  const int64_t leaves = HostKdTree::count_leaves(N, t->depth);
  t->pts.resize((size_t)N * n);
  t->ids.resize(N);
  t->split.assign(((size_t)1 << t->depth) - 1 + 1, 0.0);
  t->sdim.assign(((size_t)1 << t->depth) - 1 + 1, 0);
  t->first.assign(leaves + 1, 0);
  t->first[leaves] = N;
  std::vector<int32_t> ord(N);
  for (int64_t i = 0; i < N; ++i) ord[i] = (int32_t)i;
  int par = 0;
  while ((1 << (par + 1)) <= std::max(threads, 1) && par < t->depth) ++par;
  kd_build(*t, X, ord, 0, N, 0, 0, par);
  return t;
}

struct Cand {
  double d2;
  int32_t id;
};
inline bool cand_less(const Cand& a, const Cand& b) {
  return a.d2 < b.d2 || (a.d2 == b.d2 && a.id < b.id);
}

// The K nearest points j != qid of point qid (coordinates q), ascending
// (d^2, id), into ids / dists (K entries).
void kd_knn(const HostKdTree& t, const double* q, int32_t qid, int K, std::vector<Cand>& heap,
            std::vector<std::pair<int64_t, double>>& stack, int32_t* out_ids, double* out_d) {
  const int n = t.n;
  heap.clear();
  stack.clear();
  stack.emplace_back(0, 0.0);
  const int64_t internal = ((int64_t)1 << t.depth) - 1;
  while (!stack.empty()) {
    const auto [node, bound] = stack.back();
    stack.pop_back();
    if ((int)heap.size() == K && bound > heap.front().d2) continue;
    if (node >= internal) {
      const int64_t leaf = node - internal;
      for (int64_t i = t.first[leaf]; i < t.first[leaf + 1]; ++i) {
        const int32_t id = t.ids[i];
        if (id == qid) continue;
        const double* p = &t.pts[(size_t)i * n];
        double s = 0.0;
        for (int j = 0; j < n; ++j) {
          const double a = p[j] - q[j];
          s = s + a * a;
        }
        const Cand c{s, id};
        if ((int)heap.size() < K) {
          heap.push_back(c);
          std::push_heap(heap.begin(), heap.end(), cand_less);
        } else if (cand_less(c, heap.front())) {
          std::pop_heap(heap.begin(), heap.end(), cand_less);
          heap.back() = c;
          std::push_heap(heap.begin(), heap.end(), cand_less);
        }
      }
      continue;
    }
    const int dim = t.sdim[node];
    const double diff = q[dim] - t.split[node];
    const double b2 = diff * diff;  // a far-side point's d^2 is at least this
    const int64_t near = diff <= 0 ? 2 * node + 1 : 2 * node + 2;
    const int64_t far = diff <= 0 ? 2 * node + 2 : 2 * node + 1;
    stack.emplace_back(far, std::max(bound, b2));
    stack.emplace_back(near, bound);
  }
  std::sort_heap(heap.begin(), heap.end(), cand_less);
  for (int k = 0; k < K; ++k) {
    out_ids[k] = heap[k].id;
    out_d[k] = std::sqrt(heap[k].d2);
  }
}

// ---------------------------------------------------------------------------
// Device helpers of the GPU component
// ---------------------------------------------------------------------------
constexpr int kBlock = 256;

// QA[b] = XA[ids[b]] (row-major) and QX[j * nb + b] (SoA).
__global__ void k_gather_queries(const double* __restrict__ XA, int n,
                                 const int32_t* __restrict__ ids, int64_t nb,
                                 double* __restrict__ QA, double* __restrict__ QX) {
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nb;
       b += (int64_t)gridDim.x * blockDim.x) {
    const int64_t id = ids[b];
    for (int j = 0; j < n; ++j) {
      const double v = XA[id * n + j];
      QA[b * n + j] = v;
      QX[(int64_t)j * nb + b] = v;
    }
  }
}

__global__ void k_mark_rows(const int32_t* __restrict__ rows, int64_t nr, uint8_t* __restrict__ flag) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nr;
       i += (int64_t)gridDim.x * blockDim.x)
    flag[rows[i]] = 1;
}

// out[i] = ids[rows[i]].
__global__ void k_take_ids(const int32_t* __restrict__ rows, int64_t nr,
                           const int32_t* __restrict__ ids, int32_t* __restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nr;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = ids[rows[i]];
}

// Row b of the K+1 nearest of query point ids[b] among all points (itself
// included, at distance 0) -> its K nearest j != ids[b]: the list without
// that id, or its first K entries when the id is not in it (K+1 other
// points at distance 0 with lower ids).  Rows flagged unsolved are skipped.
// The rows go to out_ids / out_d row `self` (N x K, by id), and solved[self]
// is set.
__global__ void k_drop_self(const int32_t* __restrict__ ids1, const double* __restrict__ d1,
                            const int32_t* __restrict__ qid, const uint8_t* __restrict__ unsolved,
                            int64_t nb, int K, int32_t* __restrict__ out_ids,
                            double* __restrict__ out_d, uint8_t* __restrict__ solved) {
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nb;
       b += (int64_t)gridDim.x * blockDim.x) {
    if (unsolved[b]) continue;
    const int32_t self = qid[b];
    const int32_t* ri = ids1 + b * (K + 1);
    const double* rd = d1 + b * (K + 1);
    int32_t* oi = out_ids + (int64_t)self * K;
    double* od = out_d + (int64_t)self * K;
    int o = 0;
    for (int k = 0; k <= K && o < K; ++k) {
      if (ri[k] == self) continue;
      oi[o] = ri[k];
      od[o] = rd[k];
      ++o;
    }
    solved[self] = 1;
  }
}

// Rows list[r] of the N x K arrays into consecutive rows of the outputs.
__global__ void k_gather_rows(const int32_t* __restrict__ list, int64_t nr, int K,
                              const int32_t* __restrict__ ids, const double* __restrict__ d,
                              int32_t* __restrict__ out_ids, double* __restrict__ out_d) {
  const int64_t total = nr * K;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / K, k = e - r * K;
    const int64_t src = (int64_t)list[r] * K + k;
    out_ids[e] = ids[src];
    out_d[e] = d[src];
  }
}

// Work estimate of Sec. 4.5 per sorted position: key = ~(points of its cell)
// (so an ascending sort puts the densest first).
__global__ void k_work_keys(const uint32_t* __restrict__ cell_of,
                            const uint32_t* __restrict__ cell_start, int64_t N,
                            uint64_t* __restrict__ keys) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < N;
       p += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t c = cell_of[p];
    keys[p] = (uint64_t)(0xFFFFFFFFu - (cell_start[c + 1] - cell_start[c]));
  }
}

int grid_of(int64_t n) { return (int)std::min<int64_t>(std::max<int64_t>(ceil_div(n, kBlock), 1), 8192); }

}  // namespace

// The CPU component's kd-tree, kept with the index (built on first use).
struct HybridState {
  std::mutex mu;
  std::vector<double> XA;  // the points, id order, row-major N x n
  std::unique_ptr<HostKdTree> tree;
};

void destroy_hybrid_state(HybridState* h) { delete h; }

}  // namespace knn

using namespace knn;

namespace {

struct Schedule {
  double n_large, n_small, n_cwin, n_cpu, eps_factor;
  int threads;
};

Schedule resolve_hybrid(const knn_hybrid_opts* o) {
  knn_hybrid_opts z{};
  if (o) z = *o;
  auto frac = [](double v, double def) { return v > 0 ? std::min(v, 1.0) : (v < 0 ? 0.0 : def); };
  Schedule s;
  s.n_large = frac(z.n_large, 0.4);
  s.n_small = frac(z.n_small, 0.005);
  s.n_cwin = frac(z.n_cwin, 0.4);
  s.n_cpu = frac(z.n_cpu, 0.005);
  KNN_CHECK(s.n_small > 0 && s.n_cpu > 0, KNN_EINVAL, "n_small and n_cpu must be > 0");
  s.eps_factor = z.eps_factor > 0 ? z.eps_factor : 1.0;
  const int hw = (int)std::max(2u, std::thread::hardware_concurrency());
  s.threads = z.cpu_threads > 0 ? z.cpu_threads : (z.cpu_threads < 0 ? 0 : hw - 1);
  return s;
}

HybridState& hybrid_of(knn_index* idx) {
  if (!idx->hybrid) idx->hybrid = new HybridState();
  return *idx->hybrid;
}

}  // namespace

extern "C" {

int knn_self_join_hybrid(knn_index* idx, int32_t K, int32_t* ids, double* dists,
                         const knn_hybrid_opts* opts, knn_hybrid_stats* stats) {
  return guarded([&] {
    validate_join(idx, K);
    KNN_CHECK(K + 1 <= KNN_MAX_K, KNN_EINVAL, "the hybrid join needs K < KNN_MAX_K");
    KNN_CHECK(ids && dists, KNN_EINVAL, "output pointers are NULL");
    const Schedule sch = resolve_hybrid(opts);
    const int32_t zorder = opts ? opts->zorder : 0;
    BusyGuard bg(idx);
    DeviceGuard dg(idx->device);
    const int64_t N = idx->N;
    const int n = idx->n;
    const auto t0 = Clock::now();
    knn_hybrid_stats hs{};
    hs.cpu_threads = sch.threads;
    hipStream_t s = nullptr;
    KNN_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    struct StreamGuard {
      hipStream_t s;
      ~StreamGuard() {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
      }
    } sg{s};

    // ---- the CPU component's index (kept with the index once built) -------
    HybridState& hst = hybrid_of(idx);
    const bool need_tree = sch.threads > 0 && !hst.tree;
    const double eps_min = eps_min_of(*idx, K);
    hs.eps_min = eps_min;

    // ---- work queue (Sec. 4.5): ids by non-increasing own-cell count -------
    JoinContext qc;
    qc.device = idx->device;
    DevBuf<int32_t> dqueue(N);
    {
      build_level(*idx, qc, eps_min > 0 ? eps_min : 1.0, s);
      qc.keys2.reserve(N);
      DevBuf<uint64_t> wk(N), wk2(N);
      DevBuf<int32_t> wv2(N);
      k_work_keys<<<grid_of(N), kBlock, 0, s>>>(qc.cell_of.p, qc.cell_start.p, N, wk.p);
      KNN_LAUNCHED();
      KNN_HIP(hipMemcpyAsync(dqueue.p, qc.perm.p, N * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
      // stable: equal counts keep the cell order, and ids ascending inside a cell
      if (radix_sort_pairs(wk.p, dqueue.p, wk2.p, wv2.p, N, 32, qc.tmp.p, qc.scan_state.p,
                           (int64_t)qc.scan_state.n, s))
        KNN_HIP(hipMemcpyAsync(dqueue.p, wv2.p, N * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    }
    std::vector<int32_t> hqueue(N);
    KNN_HIP(hipMemcpyAsync(hqueue.data(), dqueue.p, N * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    if (need_tree) {
      hst.XA.resize((size_t)N * n);
      KNN_HIP(hipMemcpyAsync(hst.XA.data(), idx->XA.p, (size_t)N * n * sizeof(double),
                             hipMemcpyDeviceToHost, s));
    }
    const double* XA_host = hst.XA.data();
    KNN_HIP(hipStreamSynchronize(s));
    hs.ms_queue = ms_since(t0);

    // ---- shared queue state --------------------------------------------------
    std::mutex mu;
    std::condition_variable cv;
    int64_t qf = 0, qb = N;         // queue [qf, qb): GPU takes from qf, CPU from qb
    int64_t done_g = 0, done_c = 0;  // queries solved by each side
    bool gpu_active = true;          // the GPU may still hand failures back
    bool halved = false;             // the 95 % rule applied
    double n_cpu = sch.n_cpu;
    std::atomic<bool> abort{false};
    std::string cpu_error;
    double t_cpu_end = 0;

    // ---- CPU workers -------------------------------------------------------------
    auto cpu_worker = [&](HostKdTree* tree) {
      std::vector<Cand> heap;
      std::vector<std::pair<int64_t, double>> stack;
      heap.reserve(K + 1);
      std::vector<int32_t> batch;
      for (;;) {
        int64_t b0, nb;
        {
          std::unique_lock<std::mutex> lk(mu);
          cv.wait(lk, [&] { return abort.load() || qf < qb || !gpu_active; });
          if (abort.load() || qf >= qb) break;
          nb = std::max<int64_t>(1, (int64_t)std::llround(n_cpu * (double)N));
          nb = std::min(nb, qb - qf);
          qb -= nb;
          b0 = qb;
          batch.assign(hqueue.begin() + b0, hqueue.begin() + b0 + nb);
        }
        for (int32_t id : batch)
          kd_knn(*tree, &XA_host[(size_t)id * n], id, K, heap, stack, ids + (size_t)id * K,
                 dists + (size_t)id * K);
        {
          std::lock_guard<std::mutex> lk(mu);
          done_c += nb;
          if (!halved && done_g + done_c >= (int64_t)std::ceil(0.95 * (double)N)) {
            halved = true;
            n_cpu = sch.n_cpu / 2;
          }
          t_cpu_end = std::max(t_cpu_end, ms_since(t0));
        }
        cv.notify_all();
      }
      std::lock_guard<std::mutex> lk(mu);
      t_cpu_end = std::max(t_cpu_end, ms_since(t0));
    };
    std::vector<std::thread> workers;
    std::thread cpu_launcher;
    if (sch.threads > 0) {
      // the kd-tree is built (once per index) by the CPU side while the GPU
      // starts on its first batch
      cpu_launcher = std::thread([&] {
        try {
          HostKdTree* tree = nullptr;
          {
            std::lock_guard<std::mutex> lk(hst.mu);
            if (!hst.tree) {
              const auto tb = Clock::now();
              hst.tree = kd_create(XA_host, N, n, sch.threads);
              hs.ms_cpu_index = ms_since(tb);
            }
            tree = hst.tree.get();
          }
          for (int i = 0; i < sch.threads; ++i) workers.emplace_back(cpu_worker, tree);
          for (auto& w : workers) w.join();
        } catch (const std::exception& e) {
          std::lock_guard<std::mutex> lk(mu);
          cpu_error = e.what();
          abort = true;
          cv.notify_all();
        }
      });
    }

    // ---- GPU component (this thread) ---------------------------------------------
    double eps = sch.eps_factor * eps_min;
    if (!(eps > 0)) eps = 1.0;
    double n_large = sch.n_large, n_cwin = sch.n_cwin, n_small = sch.n_small;
    JoinContext gc;
    gc.device = idx->device;
    DevBuf<double> QA, QX, d1;
    DevBuf<int32_t> i1, unsolved, uids;
    DevBuf<uint8_t> flags;
    HostBuf<int32_t> h_uids;
    // the GPU's rows stay on the device (by id) until the end
    DevBuf<int32_t> g_ids((size_t)N * K);
    DevBuf<double> g_d((size_t)N * K);
    DevBuf<uint8_t> g_solved(N);
    launch_zero(g_solved.p, (size_t)N, s);
    double t_gpu_end = 0;
    try {
      for (;;) {
        int64_t f0, nb;
        bool mono;
        {
          std::lock_guard<std::mutex> lk(mu);
          if (abort.load() || qf >= qb) break;
          mono = n_large > 0;
          const double frac = mono ? n_large : n_small;
          nb = std::max<int64_t>(1, (int64_t)std::llround(frac * (double)N));
          nb = std::min(nb, qb - qf);
          f0 = qf;
          qf += nb;
        }
        // one attempt at the current eps: K+1 nearest among all points
        // (itself included), the query's own id dropped afterwards
        const int32_t* bids = dqueue.p + f0;
        QA.reserve((size_t)nb * n);
        QX.reserve((size_t)nb * n);
        i1.reserve((size_t)nb * (K + 1));
        d1.reserve((size_t)nb * (K + 1));
        unsolved.reserve(nb);
        uids.reserve(nb);
        flags.reserve(nb);
        k_gather_queries<<<grid_of(nb), kBlock, 0, s>>>(idx->XA.p, n, bids, nb, QA.p, QX.p);
        KNN_LAUNCHED();
        JoinQueries jq;
        jq.QA = QA.p;
        jq.QX = QX.p;
        jq.NQ = nb;
        for (int j = 0; j < n; ++j) {
          jq.lo[j] = idx->lo[j];
          jq.hi[j] = idx->hi[j];
        }
        knn_join_opts o{};
        o.cell_width = eps;
        o.tail_pairs = -1;
        o.zorder = zorder;
        JoinLimit lim;
        lim.max_levels = 1;
        lim.unsolved = unsolved.p;
        lim.reuse_level0 = true;
        self_join(*idx, gc, K + 1, i1.p, d1.p, o, s, nullptr, nullptr, &jq, &lim);
        const int64_t nf = lim.n_unsolved;
        launch_zero(flags.p, (size_t)nb, s);
        if (nf > 0) {
          k_mark_rows<<<grid_of(nf), kBlock, 0, s>>>(unsolved.p, nf, flags.p);
          KNN_LAUNCHED();
          k_take_ids<<<grid_of(nf), kBlock, 0, s>>>(unsolved.p, nf, bids, uids.p);
          KNN_LAUNCHED();
        }
        k_drop_self<<<grid_of(nb), kBlock, 0, s>>>(i1.p, d1.p, bids, flags.p, nb, K, g_ids.p,
                                                    g_d.p, g_solved.p);
        KNN_LAUNCHED();
        h_uids.reserve(std::max<int64_t>(nf, 1));
        if (nf > 0) {
          KNN_HIP(hipMemcpyAsync(h_uids.p, uids.p, (size_t)nf * 4, hipMemcpyDeviceToHost, s));
          // failures go back to the front of the queue: positions
          // [f0 + nb - nf, f0 + nb), which this batch consumed
          KNN_HIP(hipMemcpyAsync(dqueue.p + f0 + nb - nf, uids.p, (size_t)nf * 4,
                                 hipMemcpyDeviceToDevice, s));
        }
        KNN_HIP(hipStreamSynchronize(s));
        hs.gpu_batches += 1;
        hs.gpu_attempts += nb;
        if (mono) hs.monolithic_batches += 1;
        {
          std::lock_guard<std::mutex> lk(mu);
          if (nf > 0) {
            std::memcpy(hqueue.data() + f0 + nb - nf, h_uids.p, (size_t)nf * 4);
            qf -= nf;
          }
          done_g += nb - nf;
          // re-index when more than a quarter of the batch failed (Alg. 1)
          if ((double)nf > 0.25 * (double)nb) {
            eps += 0.5 * eps_min;
            hs.reindexes += 1;
          }
          if (mono) {
            const double gp = (double)done_g / (double)N, cp = (double)done_c / (double)N;
            n_large = std::min(0.5 * n_large, std::max(0.0, 1.0 - gp - cp - n_cwin));
            if (n_large * (double)N < 1.0) {
              n_large = 0;
              n_cwin = 0;
            }
          }
          if (!halved && done_g + done_c >= (int64_t)std::ceil(0.95 * (double)N)) {
            halved = true;
            n_small = sch.n_small / 2;
            n_cpu = sch.n_cpu / 2;
          }
          t_gpu_end = ms_since(t0);
        }
        cv.notify_all();
      }
    } catch (...) {
      {
        std::lock_guard<std::mutex> lk(mu);
        abort = true;
        gpu_active = false;
      }
      cv.notify_all();
      if (cpu_launcher.joinable()) cpu_launcher.join();
      throw;
    }
    {
      std::lock_guard<std::mutex> lk(mu);
      gpu_active = false;
    }
    cv.notify_all();
    if (cpu_launcher.joinable()) cpu_launcher.join();
    KNN_CHECK(cpu_error.empty(), KNN_EINTERNAL, "CPU component failed: " + cpu_error);
    KNN_CHECK(done_g + done_c == N, KNN_EINTERNAL, "the work queue lost queries");
    // the GPU's rows into the host outputs: their ids in increasing order
    // (a list from the solved flags), gathered into consecutive rows and
    // copied in chunks (two in flight: the next chunk's copy overlaps the host
    // threads writing this one), so the host writes move through the outputs
    // in order
    if (done_g > 0) {
      const auto tm = Clock::now();
      DevBuf<int32_t> glist(N);
      DevBuf<uint32_t> gcount(1);
      launch_active_list(g_solved.p, 1, nullptr, N, glist.p, gcount.p, gc.scan_state.p,
                         (int64_t)gc.scan_state.n, s);
      const int64_t chunk =
          std::min<int64_t>(done_g, std::max<int64_t>(1, (64ll << 20) / (12 * (int64_t)K)));
      std::vector<int32_t> hlist(done_g);
      KNN_HIP(hipMemcpyAsync(hlist.data(), glist.p, done_g * sizeof(int32_t), hipMemcpyDeviceToHost, s));
      uint32_t listed = 0;
      KNN_HIP(hipMemcpyAsync(&listed, gcount.p, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
      KNN_HIP(hipStreamSynchronize(s));
      KNN_CHECK((int64_t)listed == done_g, KNN_EINTERNAL, "GPU rows: flags and counts differ");
      DevBuf<int32_t> ci[2];
      DevBuf<double> cd[2];
      HostBuf<int32_t> hi_[2];
      HostBuf<double> hd_[2];
      hipEvent_t ev[2] = {nullptr, nullptr};
      struct EvGuard {
        hipEvent_t* e;
        ~EvGuard() {
          for (int i = 0; i < 2; ++i)
            if (e[i]) (void)hipEventDestroy(e[i]);
        }
      } eg{ev};
      for (int i = 0; i < 2; ++i) {
        ci[i].reserve((size_t)chunk * K);
        cd[i].reserve((size_t)chunk * K);
        hi_[i].reserve((size_t)chunk * K);
        hd_[i].reserve((size_t)chunk * K);
        KNN_HIP(hipEventCreateWithFlags(&ev[i], hipEventDisableTiming));
      }
      const int64_t nchunks = ceil_div(done_g, chunk);
      auto issue = [&](int64_t c) {
        const int i = (int)(c & 1);
        const int64_t r0 = c * chunk, nr = std::min(chunk, done_g - r0);
        k_gather_rows<<<grid_of(nr * K), kBlock, 0, s>>>(glist.p + r0, nr, K, g_ids.p, g_d.p,
                                                         ci[i].p, cd[i].p);
        KNN_LAUNCHED();
        KNN_HIP(hipMemcpyAsync(hi_[i].p, ci[i].p, (size_t)nr * K * 4, hipMemcpyDeviceToHost, s));
        KNN_HIP(hipMemcpyAsync(hd_[i].p, cd[i].p, (size_t)nr * K * 8, hipMemcpyDeviceToHost, s));
        KNN_HIP(hipEventRecord(ev[i], s));
      };
      const int nt = std::max(1, std::min(sch.threads > 0 ? sch.threads : 8, 16));
      issue(0);
      for (int64_t c = 0; c < nchunks; ++c) {
        const int i = (int)(c & 1);
        KNN_HIP(hipEventSynchronize(ev[i]));
        if (c + 1 < nchunks) issue(c + 1);
        const int64_t r0 = c * chunk, nr = std::min(chunk, done_g - r0);
        auto part = [&](int t) {
          for (int64_t r = nr * t / nt; r < nr * (t + 1) / nt; ++r) {
            const int32_t id = hlist[r0 + r];
            std::memcpy(ids + (size_t)id * K, hi_[i].p + (size_t)r * K, (size_t)K * 4);
            std::memcpy(dists + (size_t)id * K, hd_[i].p + (size_t)r * K, (size_t)K * 8);
          }
        };
        std::vector<std::thread> th;
        for (int t = 1; t < nt; ++t) th.emplace_back(part, t);
        part(0);
        for (auto& x : th) x.join();
      }
      hs.ms_merge = ms_since(tm);
    }
    hs.ms_total = ms_since(t0);
    hs.ms_gpu = t_gpu_end;
    hs.ms_cpu = sch.threads > 0 ? t_cpu_end : 0;
    hs.load_imbalance = sch.threads > 0 ? std::fabs(hs.ms_cpu - hs.ms_gpu) / hs.ms_total : 0;
    hs.gpu_queries = done_g;
    hs.cpu_queries = done_c;
    hs.eps_final = eps;
    if (stats) *stats = hs;
  });
}

}  // extern "C"
