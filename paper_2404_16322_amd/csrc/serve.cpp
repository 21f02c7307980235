// Continuous-batching search server.
//
// A scheduler thread owns n_streams slots (one HIP stream each, with preallocated device and
// pinned host buffers for max_batch queries).  Whenever a slot is free it forms a micro-batch
// from the front of the request queue -- requests keep their own K and N_probe per query --
// as long as the device bytes of all batches in flight stay within the HBM budget, and queues
// upload -> search -> download on the slot's stream.  Batches on different streams overlap on
// the GPU; requests that arrive while others run are admitted as soon as a slot and budget
// free up.  A query's result does not depend on the batch it lands in: every step of the
// search is computed per query (per-query rotation row, probe list, threshold schedule).
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <thread>
#include <unordered_map>

#include "runtime.h"

using namespace ddc;
using Clock = std::chrono::steady_clock;

namespace {

uint64_t now_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             Clock::now().time_since_epoch()).count();
}

struct Request {
  uint64_t ticket = 0;
  int nq = 0;
  int64_t nres = 0;                  // sum of k
  std::vector<float> q;
  std::vector<int32_t> k, np;
  uint64_t t_submit = 0, t_done = 0;
  std::vector<int64_t> ids;
  std::vector<float> d;
  int state = 0;                     // 0 queued, 1 running, 2 done, 3 failed
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  DevBuf d_q, d_k, d_np, d_off, d_ids, d_d;
  float *h_q = nullptr;
  int32_t *h_k = nullptr, *h_np = nullptr;
  int64_t *h_off = nullptr, *h_ids = nullptr;
  float *h_d = nullptr;
  std::vector<std::shared_ptr<Request>> reqs;
  std::vector<int64_t> res_off;      // first result of every request in the batch
  int64_t bytes = 0;
  bool busy = false;
};

}  // namespace

struct ddc_server {
  ddc_index *ix = nullptr;
  ddc_server_params p{};
  std::mutex mtx;
  std::condition_variable cv;
  std::deque<std::shared_ptr<Request>> queue;
  std::unordered_map<uint64_t, std::shared_ptr<Request>> by_ticket;
  std::vector<Slot> slots;
  std::thread th;
  bool stop = false;
  uint64_t next_ticket = 1;
  int64_t in_flight_bytes = 0, peak_bytes = 0;
  int running = 0, max_running = 0;
  std::vector<double> lat_ms;
  int64_t done_requests = 0, done_queries = 0, rejected = 0;
  uint64_t t_first = 0, t_last = 0;
  std::string thread_error;

  int64_t batch_bytes(int64_t nq, int64_t nres, int np_max) const {
    return nq * (ix->D * 4 + 16) + nres * 12 + (int64_t)search_scratch_bytes(ix, nq, np_max);
  }
};

// pinned host buffer of n bytes (counted like the device allocations)
template <class T> static void host_alloc(T **p, size_t n) {
  fault_check_alloc();
  HIPC(hipHostMalloc((void **)p, n, 0));
  alloc_track(1, 0);   // counted, not in the device bytes
}
template <class T> static void host_free(T *&p) {
  if (!p) return;
  (void)hipHostFree(p);
  alloc_track(-1, 0);
  p = nullptr;
}

static void release_slot(Slot &sl) {
  host_free(sl.h_q);
  host_free(sl.h_k);
  host_free(sl.h_np);
  host_free(sl.h_off);
  host_free(sl.h_ids);
  host_free(sl.h_d);
  if (sl.done) (void)hipEventDestroy(sl.done);
  if (sl.stream) (void)hipStreamDestroy(sl.stream);
  sl.d_q.release(); sl.d_k.release(); sl.d_np.release();
  sl.d_off.release(); sl.d_ids.release(); sl.d_d.release();
  sl.h_q = nullptr; sl.h_k = sl.h_np = nullptr; sl.h_off = sl.h_ids = nullptr; sl.h_d = nullptr;
  sl.done = nullptr; sl.stream = nullptr;
}

// Collect finished batches: results to their requests, budget back.
static bool reap(ddc_server *s) {
  bool any = false;
  for (auto &sl : s->slots) {
    if (!sl.busy) continue;
    const hipError_t e = hipEventQuery(sl.done);
    if (e == hipErrorNotReady) continue;
    const uint64_t t = now_ns();
    std::lock_guard<std::mutex> lk(s->mtx);
    for (size_t r = 0; r < sl.reqs.size(); ++r) {
      Request &rq = *sl.reqs[r];
      if (e == hipSuccess) {
        rq.ids.assign(sl.h_ids + sl.res_off[r], sl.h_ids + sl.res_off[r] + rq.nres);
        rq.d.assign(sl.h_d + sl.res_off[r], sl.h_d + sl.res_off[r] + rq.nres);
        rq.state = 2;
        rq.t_done = t;
        s->lat_ms.push_back((double)(t - rq.t_submit) * 1e-6);
        s->done_requests += 1;
        s->done_queries += rq.nq;
        s->t_last = t;
      } else {
        rq.state = 3;
        s->thread_error = hipGetErrorString(e);
      }
    }
    sl.reqs.clear();
    sl.busy = false;
    s->in_flight_bytes -= sl.bytes;
    s->running -= 1;
    any = true;
  }
  if (any) s->cv.notify_all();
  return any;
}

// Form and launch one batch on a free slot; false if nothing could be admitted.
static bool admit(ddc_server *s, Slot &sl) {
  std::vector<std::shared_ptr<Request>> take;
  int64_t nq = 0, nres = 0, bytes = 0;
  int np_max = 1, k_max = 1;
  {
    std::lock_guard<std::mutex> lk(s->mtx);
    while (!s->queue.empty()) {
      const auto &r = s->queue.front();
      int npm = np_max, km = k_max;
      for (int i = 0; i < r->nq; ++i) { npm = std::max(npm, r->np[i]); km = std::max(km, r->k[i]); }
      if (nq + r->nq > s->p.max_batch) break;
      const int64_t b = s->batch_bytes(nq + r->nq, nres + r->nres, npm);
      if (s->in_flight_bytes + b > s->p.hbm_budget_bytes) break;
      nq += r->nq; nres += r->nres; np_max = npm; k_max = km; bytes = b;
      r->state = 1;
      take.push_back(r);
      s->queue.pop_front();
    }
    if (take.empty()) return false;
    s->in_flight_bytes += bytes;
    s->peak_bytes = std::max(s->peak_bytes, s->in_flight_bytes);
    s->running += 1;
    s->max_running = std::max(s->max_running, s->running);
  }
  const int D = s->ix->D;
  int64_t qo = 0, ro = 0;
  sl.res_off.clear();
  sl.h_off[0] = 0;
  for (auto &r : take) {
    std::memcpy(sl.h_q + qo * D, r->q.data(), (size_t)r->nq * D * 4);
    sl.res_off.push_back(ro);
    for (int i = 0; i < r->nq; ++i) {
      sl.h_k[qo + i] = r->k[i];
      sl.h_np[qo + i] = r->np[i];
      sl.h_off[qo + i + 1] = sl.h_off[qo + i] + r->k[i];
    }
    qo += r->nq;
    ro += r->nres;
  }
  sl.reqs = std::move(take);
  sl.bytes = bytes;
  sl.busy = true;
  hipStream_t st = sl.stream;
  HIPC(hipMemcpyAsync(sl.d_q.p, sl.h_q, (size_t)nq * D * 4, hipMemcpyHostToDevice, st));
  HIPC(hipMemcpyAsync(sl.d_k.p, sl.h_k, (size_t)nq * 4, hipMemcpyHostToDevice, st));
  HIPC(hipMemcpyAsync(sl.d_np.p, sl.h_np, (size_t)nq * 4, hipMemcpyHostToDevice, st));
  HIPC(hipMemcpyAsync(sl.d_off.p, sl.h_off, (size_t)(nq + 1) * 8, hipMemcpyHostToDevice, st));
  search_device(s->ix, sl.d_q.as<float>(), nq, sl.d_k.as<int32_t>(), 0, k_max, sl.d_np.as<int32_t>(),
                0, np_max, s->p.significance, s->p.mode, sl.d_off.as<int64_t>(),
                sl.d_ids.as<int64_t>(), sl.d_d.as<float>(), nullptr, st, nullptr, nullptr,
                /*may_tune=*/false);
  HIPC(hipMemcpyAsync(sl.h_ids, sl.d_ids.p, (size_t)nres * 8, hipMemcpyDeviceToHost, st));
  HIPC(hipMemcpyAsync(sl.h_d, sl.d_d.p, (size_t)nres * 4, hipMemcpyDeviceToHost, st));
  HIPC(hipEventRecord(sl.done, st));
  return true;
}

static void run_loop(ddc_server *s) {
  (void)hipSetDevice(s->ix->device);
  try {
    for (;;) {
      bool progress = reap(s);
      for (auto &sl : s->slots) {
        if (sl.busy) continue;
        if (!admit(s, sl)) break;
        progress = true;
      }
      std::unique_lock<std::mutex> lk(s->mtx);
      if (s->stop && s->queue.empty() && s->running == 0) break;
      if (!progress) {
        if (s->running > 0) {
          lk.unlock();
          std::this_thread::sleep_for(std::chrono::microseconds(20));
        } else {
          s->cv.wait_for(lk, std::chrono::milliseconds(20));
        }
      }
    }
  } catch (const std::exception &e) {
    std::lock_guard<std::mutex> lk(s->mtx);
    s->thread_error = e.what();
    for (auto &r : s->queue) r->state = 3;
    for (auto &sl : s->slots)
      for (auto &r : sl.reqs) r->state = 3;
    s->queue.clear();
    s->cv.notify_all();
  }
}

extern "C" {

ddc_status ddc_server_create(const ddc_index *ixc, const ddc_server_params *p, ddc_server **out) {
  if (!out) return set_err(DDC_EINVAL, "out is NULL");
  *out = nullptr;
  if (!ixc || !p) return set_err(DDC_EINVAL, "NULL index or params");
  if (p->n_streams < 1 || p->n_streams > 16) return set_err(DDC_EINVAL, "n_streams must be in [1, 16]");
  if (p->max_batch < 1 || p->max_batch > 65536) return set_err(DDC_EINVAL, "max_batch must be in [1, 65536]");
  if (!(p->significance >= 0.0 && p->significance < 1.0)) return set_err(DDC_EINVAL, "significance must be in [0, 1)");
  if (p->mode != DDC_CORR_LEARNED && p->mode != DDC_CORR_LOSSLESS && p->mode != DDC_CORR_NONE &&
      p->mode != DDC_CORR_ADS && p->mode != DDC_CORR_BSAR)
    return set_err(DDC_EINVAL, "unknown correction mode");
  if (p->mode == DDC_CORR_LEARNED && p->significance > 0 && ixc->Tt() > 0 && ixc->tables.empty())
    return set_err(DDC_EINVAL, "index has no calibrated correction table");
  ddc_index *ix = const_cast<ddc_index *>(ixc);
  std::unique_ptr<ddc_server> s(new ddc_server);
  s->ix = ix;
  s->p = *p;
  if (s->batch_bytes(1, kMaxK, 1) > p->hbm_budget_bytes)
    return set_err(DDC_EINVAL, "hbm_budget_bytes cannot hold a single query");
  try {
    DeviceGuard dg(ix->device);
    s->slots.resize(p->n_streams);
    const int64_t mb = p->max_batch;
    for (auto &sl : s->slots) {
      HIPC(hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking));
      HIPC(hipEventCreateWithFlags(&sl.done, hipEventDisableTiming));
      sl.d_q.alloc(mb * ix->D * 4);
      sl.d_k.alloc(mb * 4);
      sl.d_np.alloc(mb * 4);
      sl.d_off.alloc((mb + 1) * 8);
      sl.d_ids.alloc(mb * kMaxK * 8);
      sl.d_d.alloc(mb * kMaxK * 4);
      host_alloc(&sl.h_q, mb * ix->D * 4);
      host_alloc(&sl.h_k, mb * 4);
      host_alloc(&sl.h_np, mb * 4);
      host_alloc(&sl.h_off, (mb + 1) * 8);
      host_alloc(&sl.h_ids, mb * kMaxK * 8);
      host_alloc(&sl.h_d, mb * kMaxK * 4);
    }
    {
      // grow the stream-ordered pool once for n_streams batches of max_batch queries (it keeps
      // what it reserved), so the first requests do not pay for mapping new memory
      std::vector<AsyncBuf> warm;
      for (auto &sl : s->slots)
        warm.emplace_back(search_scratch_bytes(ix, mb, std::min(ix->nlist, 4096)), sl.stream);
      for (auto &sl : s->slots) HIPC(hipStreamSynchronize(sl.stream));
    }
    for (auto &sl : s->slots) HIPC(hipStreamSynchronize(sl.stream));
    // one small search per stream with the server's significance and test, so the first
    // requests find the correction rows uploaded, the kernels they launch loaded and the pool
    // grown for a batch of that shape (zero queries: finite, valid input)
    {
      const int wq = (int)std::min<int64_t>(mb, 256);
      const int wnp = std::min(ix->nlist, 16), wk = 10;
      for (auto &sl : s->slots) {
        HIPC(hipMemsetAsync(sl.d_q.p, 0, (size_t)wq * ix->D * 4, sl.stream));
        std::vector<int32_t> hk(wq, wk), hn(wq, wnp);
        std::vector<int64_t> ho(wq + 1);
        for (int i = 0; i <= wq; ++i) ho[i] = (int64_t)i * wk;
        HIPC(hipMemcpyAsync(sl.d_k.p, hk.data(), (size_t)wq * 4, hipMemcpyHostToDevice, sl.stream));
        HIPC(hipMemcpyAsync(sl.d_np.p, hn.data(), (size_t)wq * 4, hipMemcpyHostToDevice, sl.stream));
        HIPC(hipMemcpyAsync(sl.d_off.p, ho.data(), (size_t)(wq + 1) * 8, hipMemcpyHostToDevice, sl.stream));
        for (int nq : {wq, 1})
          search_device(ix, sl.d_q.as<float>(), nq, sl.d_k.as<int32_t>(), 0, wk, sl.d_np.as<int32_t>(), 0,
                        wnp, p->significance, p->mode, sl.d_off.as<int64_t>(), sl.d_ids.as<int64_t>(),
                        sl.d_d.as<float>(), nullptr, sl.stream, nullptr, nullptr, /*may_tune=*/false);
        HIPC(hipStreamSynchronize(sl.stream));   // the pageable staging above stays alive until here
      }
    }
  } catch (const DdcError &e) {
    for (auto &sl : s->slots) release_slot(sl);
    return set_err(e.st, "%s", e.what());
  } catch (const std::exception &e) {
    for (auto &sl : s->slots) release_slot(sl);
    return set_err(DDC_EDEVICE, "%s", e.what());
  }
  s->th = std::thread(run_loop, s.get());
  *out = s.release();
  return DDC_OK;
}

ddc_status ddc_server_submit(ddc_server *s, const float *queries, int32_t nq, const int32_t *k,
                             const int32_t *nprobe, uint64_t *ticket) {
  if (!s || !queries || !k || !nprobe || !ticket) return set_err(DDC_EINVAL, "NULL argument");
  if (nq < 1 || nq > s->p.max_batch) return set_err(DDC_EINVAL, "nq must be in [1, max_batch=%d]", s->p.max_batch);
  const ddc_index *ix = s->ix;
  auto r = std::make_shared<Request>();
  r->nq = nq;
  int npm = 1;
  for (int i = 0; i < nq; ++i) {
    if (k[i] < 1 || k[i] > kMaxK) return set_err(DDC_EINVAL, "k must be in [1, %d]", kMaxK);
    if (nprobe[i] < 1 || nprobe[i] > std::min(ix->nlist, 4096))
      return set_err(DDC_EINVAL, "nprobe must be in [1, min(nlist, 4096)]");
    r->nres += k[i];
    npm = std::max(npm, nprobe[i]);
  }
  for (int64_t i = 0; i < (int64_t)nq * ix->D; ++i)
    if (!std::isfinite(queries[i])) return set_err(DDC_EINVAL, "non-finite query values");
  if (s->batch_bytes(nq, r->nres, npm) > s->p.hbm_budget_bytes) {
    std::lock_guard<std::mutex> lk(s->mtx);
    s->rejected += 1;
    return set_err(DDC_EBUSY, "request needs more device memory than the HBM budget");
  }
  r->q.assign(queries, queries + (size_t)nq * ix->D);
  r->k.assign(k, k + nq);
  r->np.assign(nprobe, nprobe + nq);
  r->t_submit = now_ns();
  std::lock_guard<std::mutex> lk(s->mtx);
  if (!s->thread_error.empty()) return set_err(DDC_EDEVICE, "server stopped: %s", s->thread_error.c_str());
  r->ticket = s->next_ticket++;
  if (s->t_first == 0) s->t_first = r->t_submit;
  s->by_ticket[r->ticket] = r;
  s->queue.push_back(r);
  *ticket = r->ticket;
  s->cv.notify_all();
  return DDC_OK;
}

ddc_status ddc_server_poll(ddc_server *s, uint64_t ticket, int64_t *ids, float *dists, int *done,
                           uint64_t *t_done_ns) {
  if (!s || !done) return set_err(DDC_EINVAL, "NULL argument");
  std::shared_ptr<Request> r;
  {
    std::lock_guard<std::mutex> lk(s->mtx);
    auto it = s->by_ticket.find(ticket);
    if (it == s->by_ticket.end()) return set_err(DDC_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    r = it->second;
    if (r->state == 3) {
      s->by_ticket.erase(it);
      return set_err(DDC_EDEVICE, "request failed: %s", s->thread_error.c_str());
    }
    if (r->state != 2) { *done = 0; return DDC_OK; }
    s->by_ticket.erase(it);
  }
  if (ids) std::copy(r->ids.begin(), r->ids.end(), ids);
  if (dists) std::copy(r->d.begin(), r->d.end(), dists);
  if (t_done_ns) *t_done_ns = r->t_done;
  *done = 1;
  return DDC_OK;
}

ddc_status ddc_server_get_stats(ddc_server *s, ddc_server_stats *st) {
  if (!s || !st) return set_err(DDC_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mtx);
  std::memset(st, 0, sizeof *st);
  st->requests_done = s->done_requests;
  st->queries_done = s->done_queries;
  st->rejected = s->rejected;
  if (s->t_last > s->t_first) st->qps = (double)s->done_queries / ((double)(s->t_last - s->t_first) * 1e-9);
  std::vector<double> l = s->lat_ms;
  if (!l.empty()) {
    std::sort(l.begin(), l.end());
    auto q = [&](double f) { return l[std::min(l.size() - 1, (size_t)std::floor(f * (l.size() - 1) + 0.5))]; };
    st->p50_ms = q(0.50);
    st->p99_ms = q(0.99);
    st->max_ms = l.back();
  }
  st->budget_peak_bytes = s->peak_bytes;
  st->max_concurrent = s->max_running;
  return DDC_OK;
}

void ddc_server_destroy(ddc_server *s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mtx);
    s->stop = true;
    s->cv.notify_all();
  }
  if (s->th.joinable()) s->th.join();
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(s->ix->device);
  for (auto &sl : s->slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    release_slot(sl);
  }
  (void)hipSetDevice(prev);
  delete s;
}

}  // extern "C"
