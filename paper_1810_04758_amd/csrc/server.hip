// server.hip -- continuous-batching request loop over resident indexes.
//
// Requests (dataset, K, host output arrays) wait in a FIFO queue.  Worker
// slots (max_inflight, each with its own HIP stream and join scratch) admit
// the oldest pending request whose device footprint fits the free memory
// budget, so requests that arrive while others run are admitted as slots and
// memory free up, and their kernels overlap on the device.  Each join is a
// pure function of (index, K), so a result is the same alone and in the mix.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <thread>
#include <unordered_map>
#include <vector>

#include "index.hpp"

namespace knn {
namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  int64_t ticket;
  int32_t ds;
  int32_t K;
  int32_t* ids;
  double* dists;
  uint64_t footprint;
  Clock::time_point t_submit;
  bool done = false;
  int status = KNN_OK;
};

}  // namespace
}  // namespace knn

struct knn_server {
  knn_server_opts opts{};
  std::vector<knn_index*> datasets;
  std::mutex mu;
  std::condition_variable cv_work;  // workers wait for admissible work
  std::condition_variable cv_done;  // waiters wait for completions
  std::deque<std::shared_ptr<knn::Request>> pending;
  std::unordered_map<int64_t, std::shared_ptr<knn::Request>> all;
  int64_t next_ticket = 1;
  uint64_t used_bytes = 0;
  int inflight = 0;
  bool stop = false;
  std::vector<std::thread> workers;
  // statistics
  int64_t submitted = 0, completed = 0, failed = 0, queries_done = 0;
  std::vector<double> lat_ms;
  uint64_t peak_bytes = 0;
  int peak_inflight = 0;
  knn::Clock::time_point t_first{}, t_last{};
  bool any = false;
};

namespace knn {
namespace {

void worker_main(knn_server* srv) {
  try {
    KNN_HIP(hipSetDevice(srv->opts.device));
  } catch (...) {
  }
  hipStream_t s = nullptr;
  (void)hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  HostStage stage;  // pinned staging of this worker's host-destination results
  for (;;) {
    std::shared_ptr<Request> rq;
    {
      std::unique_lock<std::mutex> lk(srv->mu);
      for (;;) {
        if (srv->stop && srv->pending.empty()) {
          (void)hipStreamDestroy(s);
          return;
        }
        // admit the oldest pending request that fits the free budget
        auto it = srv->pending.begin();
        for (; it != srv->pending.end(); ++it)
          if (srv->used_bytes + (*it)->footprint <= srv->opts.mem_budget_bytes) break;
        if (it != srv->pending.end()) {
          rq = *it;
          srv->pending.erase(it);
          srv->used_bytes += rq->footprint;
          srv->inflight += 1;
          srv->peak_bytes = std::max(srv->peak_bytes, srv->used_bytes);
          srv->peak_inflight = std::max(srv->peak_inflight, srv->inflight);
          break;
        }
        srv->cv_work.wait(lk);
      }
    }
    int status = KNN_OK;
    try {
      knn_index* idx = srv->datasets[rq->ds];
      JoinContext ctx;  // scratch freed when the request ends (budget stays exact)
      ctx.device = idx->device;
      const size_t NK = (size_t)idx->N * rq->K;
      ctx.out_ids.reserve(NK);
      ctx.out_d.reserve(NK);
      knn_join_opts o{};
      self_join(*idx, ctx, rq->K, ctx.out_ids.p, ctx.out_d.p, o, s);
      if (rq->ids) {  // NULL outputs: a latency-only request, results discarded
        copy_to_host(stage, rq->ids, ctx.out_ids.p, NK * sizeof(int32_t), s);
        copy_to_host(stage, rq->dists, ctx.out_d.p, NK * sizeof(double), s);
      }
      KNN_HIP(hipStreamSynchronize(s));
    } catch (const Error& e) {
      status = e.code;
      set_last_error(e.what());
      (void)hipStreamSynchronize(s);
    } catch (...) {
      status = KNN_EINTERNAL;
      (void)hipStreamSynchronize(s);
    }
    auto t_end = Clock::now();
    {
      std::lock_guard<std::mutex> lk(srv->mu);
      srv->used_bytes -= rq->footprint;
      srv->inflight -= 1;
      rq->status = status;
      rq->done = true;
      if (status == KNN_OK) {
        srv->completed += 1;
        srv->queries_done += srv->datasets[rq->ds]->N;
        srv->lat_ms.push_back(
            std::chrono::duration<double, std::milli>(t_end - rq->t_submit).count());
      } else {
        srv->failed += 1;
      }
      srv->t_last = t_end;
    }
    srv->cv_done.notify_all();
    srv->cv_work.notify_all();
  }
}

double percentile(std::vector<double> v, double p) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  double pos = p * (double)(v.size() - 1);
  size_t i = (size_t)pos;
  double f = pos - (double)i;
  if (i + 1 < v.size()) return v[i] * (1 - f) + v[i + 1] * f;
  return v[i];
}

}  // namespace
}  // namespace knn

using namespace knn;

extern "C" {

int knn_server_create(const knn_server_opts* opts, knn_server** out) {
  return guarded([&] {
    KNN_CHECK(out != nullptr, KNN_EINVAL, "NULL pointer");
    auto* srv = new knn_server();
    if (opts) srv->opts = *opts;
    if (srv->opts.mem_budget_bytes == 0) srv->opts.mem_budget_bytes = 8ull << 30;
    if (srv->opts.max_inflight <= 0) srv->opts.max_inflight = 4;
    if (srv->opts.max_queue <= 0) srv->opts.max_queue = 4096;
    if (srv->opts.device < 0) {
      int d = 0;
      KNN_HIP(hipGetDevice(&d));
      srv->opts.device = d;
    }
    for (int i = 0; i < srv->opts.max_inflight; ++i) srv->workers.emplace_back(worker_main, srv);
    *out = srv;
  });
}

int knn_server_add_dataset(knn_server* srv, knn_index* idx, int32_t* dataset_id) {
  return guarded([&] {
    KNN_CHECK(srv && idx && dataset_id, KNN_EINVAL, "NULL pointer");
    KNN_CHECK(idx->device == srv->opts.device, KNN_EINVAL, "index lives on another device");
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->datasets.push_back(idx);
    *dataset_id = (int32_t)srv->datasets.size() - 1;
  });
}

int knn_server_submit(knn_server* srv, int32_t dataset_id, int32_t K, int32_t* ids, double* dists,
                      int64_t* ticket) {
  return guarded([&] {
    KNN_CHECK(srv && ticket, KNN_EINVAL, "NULL pointer");
    KNN_CHECK((ids == nullptr) == (dists == nullptr), KNN_EINVAL,
              "ids and dists must both be given or both be NULL");
    std::unique_lock<std::mutex> lk(srv->mu);
    KNN_CHECK(dataset_id >= 0 && dataset_id < (int32_t)srv->datasets.size(), KNN_EINVAL,
              "unknown dataset");
    knn_index* idx = srv->datasets[dataset_id];
    validate_join(idx, K);
    uint64_t fp = join_footprint(*idx, K, true);
    KNN_CHECK(fp <= srv->opts.mem_budget_bytes, KNN_EINVAL,
              "request footprint exceeds the whole memory budget");
    KNN_CHECK((int32_t)srv->pending.size() < srv->opts.max_queue, KNN_EBUSY, "request queue full");
    auto rq = std::make_shared<Request>();
    rq->ticket = srv->next_ticket++;
    rq->ds = dataset_id;
    rq->K = K;
    rq->ids = ids;
    rq->dists = dists;
    rq->footprint = fp;
    rq->t_submit = Clock::now();
    if (!srv->any) {
      srv->any = true;
      srv->t_first = rq->t_submit;
    }
    srv->pending.push_back(rq);
    srv->all[rq->ticket] = rq;
    srv->submitted += 1;
    *ticket = rq->ticket;
    lk.unlock();
    srv->cv_work.notify_all();
  });
}

int knn_server_wait(knn_server* srv, int64_t ticket, int64_t timeout_us) {
  try {
    KNN_CHECK(srv != nullptr, KNN_EINVAL, "NULL pointer");
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->all.find(ticket);
    KNN_CHECK(it != srv->all.end(), KNN_EINVAL, "unknown ticket");
    auto rq = it->second;
    auto pred = [&] { return rq->done; };
    if (timeout_us < 0) {
      srv->cv_done.wait(lk, pred);
    } else if (!srv->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), pred)) {
      return KNN_ETIMEOUT;
    }
    srv->all.erase(ticket);
    if (rq->status != KNN_OK) set_last_error("request failed");
    return rq->status;
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  } catch (...) {
    set_last_error("unknown error");
    return KNN_EINTERNAL;
  }
}

int knn_server_stats_get(knn_server* srv, knn_server_stats* out) {
  return guarded([&] {
    KNN_CHECK(srv && out, KNN_EINVAL, "NULL pointer");
    std::lock_guard<std::mutex> lk(srv->mu);
    std::memset(out, 0, sizeof(*out));
    out->submitted = srv->submitted;
    out->completed = srv->completed;
    out->failed = srv->failed;
    out->p50_ms = percentile(srv->lat_ms, 0.50);
    out->p99_ms = percentile(srv->lat_ms, 0.99);
    double sum = 0, mx = 0;
    for (double v : srv->lat_ms) {
      sum += v;
      mx = std::max(mx, v);
    }
    out->mean_ms = srv->lat_ms.empty() ? 0.0 : sum / (double)srv->lat_ms.size();
    out->max_ms = mx;
    double wall = srv->any ? std::chrono::duration<double>(srv->t_last - srv->t_first).count() : 0;
    out->queries_per_s = wall > 0 ? (double)srv->queries_done / wall : 0.0;
    out->requests_per_s = wall > 0 ? (double)srv->completed / wall : 0.0;
    out->peak_bytes = srv->peak_bytes;
    out->peak_inflight = srv->peak_inflight;
  });
}

void knn_server_destroy(knn_server* srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
  }
  srv->cv_work.notify_all();
  for (auto& t : srv->workers)
    if (t.joinable()) t.join();
  delete srv;
}

}  // extern "C"
