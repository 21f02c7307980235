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

#include <algorithm>
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

// A batch's inputs (queries, K, nprobe, result offsets) and outputs (ids, distances) each travel
// as one packed block, so a batch costs one host-to-device and one device-to-host copy: with
// four copies per batch, one of them now and then waited milliseconds for other streams' work.
struct InLayout {
  size_t k, np, off, bytes;   // byte offsets of K, nprobe and the offsets; total (queries at 0)
};
static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }
static InLayout in_layout(int64_t nq, int D) {
  InLayout l;
  l.k = align256((size_t)nq * D * 4);
  l.np = l.k + align256((size_t)nq * 4);
  l.off = l.np + align256((size_t)nq * 4);
  l.bytes = l.off + (size_t)(nq + 1) * 8;
  return l;
}
static size_t out_d_offset(int64_t nres) { return align256((size_t)nres * 8); }   // ids at 0

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  DevBuf d_in, d_out;
  DevBuf ws;   // the batch's correction rows and search scratch (sized for max_batch at creation)
  char *h_in = nullptr, *h_out = nullptr;
  size_t out_d = 0;                  // the current batch's distances in h_out / d_out
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
template <class T> static void host_alloc(T **p, size_t n, unsigned flags = 0) {
  fault_check_alloc();
  HIPC(hipHostMalloc((void **)p, n, flags));
  alloc_track(1, 0);   // counted, not in the device bytes
}

// A batch's packed inputs and outputs are moved by this kernel on the batch's stream, reading
// or writing the pinned host block (coherent, so never cached stale on the device) over PCIe:
// the runtime's copy commands now and then blocked the submitting thread for milliseconds while
// other streams ran.  A write to the host ends with a system-scope fence, so the host sees the
// results once the batch's completion event has fired.  n16: 16-byte words (the blocks are
// sized in whole words).
template <bool TO_HOST>
__global__ __launch_bounds__(256) void stage_kernel(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                    int64_t n16) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += (int64_t)gridDim.x * 256)
    dst[i] = src[i];
  if (TO_HOST) __threadfence_system();
}
template <bool TO_HOST> static void stage(const char *src, char *dst, size_t bytes, hipStream_t st) {
  const int64_t n16 = (int64_t)((bytes + 15) / 16);
  if (n16 == 0) return;
  const unsigned grid = (unsigned)std::min<int64_t>((n16 + 255) / 256, 1024);
  hipLaunchKernelGGL(stage_kernel<TO_HOST>, dim3(grid), dim3(256), 0, st,
                     reinterpret_cast<const uint4 *>(src), reinterpret_cast<uint4 *>(dst), n16);
  HIPC(hipGetLastError());
}
template <class T> static void host_free(T *&p) {
  if (!p) return;
  (void)hipHostFree(p);
  alloc_track(-1, 0);
  p = nullptr;
}

static void release_slot(Slot &sl) {
  host_free(sl.h_in);
  host_free(sl.h_out);
  if (sl.done) (void)hipEventDestroy(sl.done);
  if (sl.stream) (void)hipStreamDestroy(sl.stream);
  sl.d_in.release(); sl.d_out.release(); sl.ws.release();
  sl.h_in = sl.h_out = nullptr;
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
        const int64_t *h_ids = reinterpret_cast<const int64_t *>(sl.h_out);
        const float *h_d = reinterpret_cast<const float *>(sl.h_out + sl.out_d);
        rq.ids.assign(h_ids + sl.res_off[r], h_ids + sl.res_off[r] + rq.nres);
        rq.d.assign(h_d + sl.res_off[r], h_d + sl.res_off[r] + rq.nres);
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
  const InLayout L = in_layout(nq, D);
  float *h_q = reinterpret_cast<float *>(sl.h_in);
  int32_t *h_k = reinterpret_cast<int32_t *>(sl.h_in + L.k);
  int32_t *h_np = reinterpret_cast<int32_t *>(sl.h_in + L.np);
  int64_t *h_off = reinterpret_cast<int64_t *>(sl.h_in + L.off);
  int64_t qo = 0, ro = 0;
  sl.res_off.clear();
  h_off[0] = 0;
  for (auto &r : take) {
    std::memcpy(h_q + qo * D, r->q.data(), (size_t)r->nq * D * 4);
    sl.res_off.push_back(ro);
    for (int i = 0; i < r->nq; ++i) {
      h_k[qo + i] = r->k[i];
      h_np[qo + i] = r->np[i];
      h_off[qo + i + 1] = h_off[qo + i] + r->k[i];
    }
    qo += r->nq;
    ro += r->nres;
  }
  sl.reqs = std::move(take);
  sl.bytes = bytes;
  sl.busy = true;
  hipStream_t st = sl.stream;
  char *d_in = sl.d_in.as<char>();
  stage<false>(sl.h_in, d_in, L.bytes, st);
  sl.out_d = out_d_offset(nres);
  char *d_out = sl.d_out.as<char>();
  const Workspace w{sl.ws.p, sl.ws.bytes, /*cached_tables=*/true};
  search_device(s->ix, reinterpret_cast<const float *>(d_in), nq, reinterpret_cast<const int32_t *>(d_in + L.k),
                0, k_max, reinterpret_cast<const int32_t *>(d_in + L.np), 0, np_max, s->p.significance,
                s->p.mode, reinterpret_cast<const int64_t *>(d_in + L.off), reinterpret_cast<int64_t *>(d_out),
                reinterpret_cast<float *>(d_out + sl.out_d), nullptr, st, nullptr, nullptr,
                /*may_tune=*/false, nullptr, false, &w);
  stage<true>(d_out, sl.h_out, sl.out_d + (size_t)nres * 4, st);
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
          // the queue is checked under the lock before sleeping: a request submitted after
          // admit() saw the queue empty (its notify found no waiter) is not left waiting
          s->cv.wait_for(lk, std::chrono::milliseconds(20), [s] { return !s->queue.empty() || s->stop; });
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
      p->mode != DDC_CORR_ADS && p->mode != DDC_CORR_BSAR && p->mode != DDC_CORR_BSAO)
    return set_err(DDC_EINVAL, "unknown correction mode");
  if (p->mode == DDC_CORR_BSAO && !ixc->pq_tables())
    return set_err(DDC_EINVAL, "the BSA-O test needs an index with pq_m > 0 and its calibrated tables");
  if (p->mode == DDC_CORR_BSAR && (int)ixc->lam.size() != ixc->D)
    return set_err(DDC_EINVAL, "the residual test needs the rotation's eigenvalues (lam)");
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
      const size_t in_b = (in_layout(mb, ix->D).bytes + 15) & ~(size_t)15;   // whole 16-byte words
      const size_t out_b = (out_d_offset(mb * kMaxK) + (size_t)mb * kMaxK * 4 + 15) & ~(size_t)15;
      sl.d_in.alloc(in_b);
      sl.d_out.alloc(out_b);
      host_alloc(&sl.h_in, in_b, hipHostMallocCoherent);
      host_alloc(&sl.h_out, out_b, hipHostMallocCoherent);
      // every batch's scratch comes from this one buffer, so serving maps no device memory:
      // an allocation the stream-ordered pool cannot serve from a freed block maps new memory,
      // which stalled every stream of the device for several milliseconds
      sl.ws.alloc(Workspace::kTableBytes + search_scratch_bytes(ix, mb, std::min(ix->nlist, 4096)));
    }
    for (auto &sl : s->slots) HIPC(hipStreamSynchronize(sl.stream));
    // one small search per stream with the server's significance and test, so the first
    // requests find the correction rows computed and the kernels they launch loaded (zero
    // queries: finite, valid input)
    {
      const int wq = (int)std::min<int64_t>(mb, 256);
      const int wnp = std::min(ix->nlist, 16), wk = 10;
      for (auto &sl : s->slots) {
        const Workspace w{sl.ws.p, sl.ws.bytes, /*cached_tables=*/true};
        for (int nq : {wq, 1}) {
          // the batch path as admit() runs it: one packed input copy, the search, one output copy
          const InLayout L = in_layout(nq, ix->D);
          std::memset(sl.h_in, 0, (size_t)nq * ix->D * 4);
          int32_t *h_k = reinterpret_cast<int32_t *>(sl.h_in + L.k);
          int32_t *h_np = reinterpret_cast<int32_t *>(sl.h_in + L.np);
          int64_t *h_off = reinterpret_cast<int64_t *>(sl.h_in + L.off);
          for (int i = 0; i < nq; ++i) { h_k[i] = wk; h_np[i] = wnp; }
          for (int i = 0; i <= nq; ++i) h_off[i] = (int64_t)i * wk;
          char *d_in = sl.d_in.as<char>(), *d_out = sl.d_out.as<char>();
          const size_t od = out_d_offset((int64_t)nq * wk);
          stage<false>(sl.h_in, d_in, L.bytes, sl.stream);
          search_device(ix, reinterpret_cast<const float *>(d_in), nq, reinterpret_cast<const int32_t *>(d_in + L.k),
                        0, wk, reinterpret_cast<const int32_t *>(d_in + L.np), 0, wnp, p->significance,
                        p->mode, reinterpret_cast<const int64_t *>(d_in + L.off), reinterpret_cast<int64_t *>(d_out),
                        reinterpret_cast<float *>(d_out + od), nullptr, sl.stream, nullptr, nullptr,
                        /*may_tune=*/false, nullptr, false, &w);
          stage<true>(d_out, sl.h_out, od + (size_t)nq * wk * 4, sl.stream);
          HIPC(hipStreamSynchronize(sl.stream));   // h_in is rewritten for the next shape
        }
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
