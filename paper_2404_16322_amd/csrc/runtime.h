// Host runtime types shared by the C-ABI implementation files (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <limits>
#include <array>
#include <map>
#include <tuple>
#include <memory>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "ddc.h"
#include "ddc_internal.h"

namespace ddc {

ddc_status set_err(ddc_status st, const char *fmt, ...);

// ---------------------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------------------

struct DdcError : std::runtime_error {
  ddc_status st;
  DdcError(ddc_status s, const std::string &m) : std::runtime_error(m), st(s) {}
};

#define HIPC(expr)                                                                          \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      throw DdcError(e_ == hipErrorOutOfMemory ? DDC_ENOMEM : DDC_EDEVICE,                  \
                     std::string(#expr) + ": " + hipGetErrorString(e_));                    \
  } while (0)

#define GUARD_BEGIN try {
#define GUARD_END                                                        \
  }                                                                      \
  catch (const DdcError &e) { return set_err(e.st, "%s", e.what()); }   \
  catch (const std::bad_alloc &) { return set_err(DDC_ENOMEM, "host allocation failed"); } \
  catch (const std::exception &e) { return set_err(DDC_EDEVICE, "%s", e.what()); }

// ---------------------------------------------------------------------------------------
// device memory
// ---------------------------------------------------------------------------------------
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  explicit DevBuf(size_t b) { alloc(b); }
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  DevBuf(DevBuf &&o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
  void alloc(size_t b) {
    release();
    if (b) {
      fault_check_alloc();
      HIPC(hipMalloc(&p, b));
      alloc_track(1, (int64_t)b);
    }
    bytes = b;
  }
  void release() {
    if (p) {
      (void)hipFree(p);
      alloc_track(-1, -(int64_t)bytes);
    }
    p = nullptr;
    bytes = 0;
  }
  ~DevBuf() { release(); }
  template <class T> T *as() const { return reinterpret_cast<T *>(p); }
};

struct DeviceGuard {
  int prev = 0;
  explicit DeviceGuard(int dev) {
    (void)hipGetDevice(&prev);
    if (prev != dev) HIPC(hipSetDevice(dev));
  }
  ~DeviceGuard() { (void)hipSetDevice(prev); }
};

struct StreamHolder {
  hipStream_t s = nullptr;
  StreamHolder() { HIPC(hipStreamCreateWithFlags(&s, hipStreamNonBlocking)); }
  ~StreamHolder() {
    if (s) (void)hipStreamDestroy(s);
  }
};

inline void set_pool_retain(int dev) {
  static std::mutex mtx;
  static std::vector<int> done;
  std::lock_guard<std::mutex> lk(mtx);
  if (std::find(done.begin(), done.end(), dev) != done.end()) return;
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
    uint64_t thr = std::numeric_limits<uint64_t>::max();
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
  }
  done.push_back(dev);
}

// stream-ordered scratch (returned to the pool when the stream reaches the free)
struct AsyncBuf {
  void *p = nullptr;
  hipStream_t s = nullptr;
  size_t n = 0;
  AsyncBuf(size_t bytes, hipStream_t st) : s(st) {
    if (bytes) {
      fault_check_alloc();
      HIPC(hipMallocAsync(&p, bytes, st));
      n = bytes;
      alloc_track(1, (int64_t)n);
    }
  }
  AsyncBuf(const AsyncBuf &) = delete;
  AsyncBuf &operator=(AsyncBuf &&o) noexcept {
    if (this != &o) {
      drop();
      p = o.p; s = o.s; n = o.n; o.p = nullptr; o.n = 0;
    }
    return *this;
  }
  AsyncBuf(AsyncBuf &&o) noexcept : p(o.p), s(o.s), n(o.n) { o.p = nullptr; o.n = 0; }
  ~AsyncBuf() { drop(); }
  void drop() {
    if (p) {
      (void)hipFreeAsync(p, s);
      alloc_track(-1, -(int64_t)n);
    }
    p = nullptr;
    n = 0;
  }
  template <class T> T *as() const { return reinterpret_cast<T *>(p); }
};

}  // namespace ddc

// ---------------------------------------------------------------------------------------
// index
// ---------------------------------------------------------------------------------------
struct ddc_index {
  int device = 0;
  int64_t n = 0;
  int D = 0, Dp = 0, NB = 0, nlist = 0, delta_d = 32, S = 0, St = 0, B = 256, L = 0;
  ddc_dtype storage = DDC_F32;
  ddc_rot rot = DDC_ROT_F32;
  std::vector<double> mu, R, lam;
  std::vector<float> cent;          // nlist x D
  std::vector<int32_t> assign;      // n
  std::vector<int32_t> list_len, tile_off;
  std::vector<int64_t> id_to_slot;  // n
  int64_t total_tiles = 0;
  std::vector<int64_t> len_desc_prefix;   // [nlist + 1] sums of the longest lists' lengths
  // correction tables, ascending calibration K_c; a search with K uses the last with
  // kc <= K (the first when none): m [Tt], resid [n0 x Tt] (label-0 residuals)
  // pq: the BSA-O classifier m1 dis' + m3 err + beta > tau of the same label-0/1 pairs, with
  // the label-0 residuals tau - m1 dis' - m3 err (empty: no BSA-O table)
  struct Table {
    int kc = 1;
    std::vector<double> m, resid;
    int64_t n0 = 0;
    double pq_m1 = 1.0, pq_m3 = 0.0;
    std::vector<double> pq_resid;
  };
  std::vector<Table> tables;
  int64_t n0_total() const {
    int64_t t = 0;
    for (auto &x : tables) t += x.n0;
    return t;
  }
  std::mutex beta_mtx;
  std::map<std::tuple<double, int, int>, std::vector<double>> beta_cache;   // (alpha, mode, table)
  std::map<std::pair<double, int>, std::shared_ptr<ddc::DevBuf>> tab_cache; // device tables
  std::map<std::pair<double, int>, std::shared_ptr<const std::vector<float>>> tab_host;  // their rows
  ddc::DevBuf d_R32, d_mu32, d_cent, d_cnorm, d_tile_off, d_list_len, d_ids, d_base, d_R64, d_mu64;
  ddc::DevBuf d_tile_list;          // [total_tiles] list of each tile
  int fp8 = 0;                      // FP8 pre-stage lead dims (0 or 64)
  double ads_eps0 = 2.1;            // eps0 of the ADSampling test
  double bsar_m = 8.0;              // multiplier of the residual test (<= 0: from the significance)
  ddc::DevBuf d_xnorm, d_lam32;     // ||y||^2 per stored slot; eigenvalues (Dp, zero padded)
  ddc::DevBuf d_base8, d_scale8;    // its codes (tiles x 64 x 64 B) and per-tile scales
  // quantization estimate (BSA-O): OPQ subspaces of the rotated axes, 256 codewords each
  int pq_m = 0, pq_dsub = 0;
  std::vector<int32_t> pq_perm;     // [D] axes of subspace j at [j * dsub, (j + 1) * dsub)
  std::vector<float> pq_books;      // [M x 256 x dsub]
  ddc::DevBuf d_pq_perm, d_pq_books, d_pq_codes, d_pq_err;   // codes [tiles x 64 x M], err [tiles x 64]
  bool pq_tables() const { return pq_m > 0 && !tables.empty() && !tables[0].pq_resid.empty(); }
  int P() const { return fp8 ? 1 : 0; }
  int Tt() const { return St + P(); }   // columns of the correction table
  // optional per-kernel event timing
  bool timing = false;
  std::mutex timing_mtx;
  struct Mark { int kernel; hipEvent_t a, b; };
  std::vector<Mark> marks;
  ~ddc_index() {
    for (auto &m : marks) { (void)hipEventDestroy(m.a); (void)hipEventDestroy(m.b); }
  }

  // search scratch per stream: grow-only, reused by the next call on the same stream
  std::mutex scratch_mtx;
  std::map<hipStream_t, std::unique_ptr<ddc::DevBuf>> scratch;

  // result-invariant launch knobs of the scan (0 / -1 = tuned per size class)
  int waves_per_query = 0, lookahead = -1, query_order = 1, xcd_swizzle = 1, persistent = -1;
  int two_phase = -1;
  int full_d_matrix = 0;            // NONE-mode scans: distances list by list on the matrix cores
  int stage1_matrix = 0;            // two-phase first phase (stored values) on the matrix cores
  int waves_per_simd = 0;           // register budget of the one-wave pruned kernel (0 = tuned)
  std::mutex tune_mtx;
  // class -> (waves per query, look-ahead, persistent, two-phase)
  std::map<std::array<int, 4>, std::array<int, 5>> tuned;   // size class -> launch shape
  int store() const {
    return storage == DDC_F32 ? ddc::ST_F32 : storage == DDC_F16 ? ddc::ST_F16 : ddc::ST_BF16;
  }
  int esize() const { return storage == DDC_F32 ? 4 : 2; }
};


namespace ddc {

// Estimate-only scan: rank candidates by an estimate over the leading nb dim blocks.
struct EstimateSpec {
  int nb;        // dim blocks read
  int residual;  // 0: scale * partial distance; 1: residual estimate (Alg. 1, C1 - C2)
  float scale;
};

// A caller-provided device workspace for one search: the correction tables at its start
// (kTableBytes), then the scratch of search_scratch_bytes.
struct Workspace {
  void *p;
  size_t bytes;
  // the correction rows from the index's device cache (made on first use, then reused) instead
  // of a copy from their host rows into the workspace on every call: for callers that may
  // allocate once but not per call (the server), since a copy from pageable host memory can
  // stall the device
  bool cached_tables = false;
  static constexpr size_t kTableBytes = 16384;
};

// The search pipeline on device buffers (rotation -> coarse -> select -> scan), queued on s.
// est (nullable): rank by that estimate instead (mode and alpha are then ignored).
// stream_scratch: take the scratch from s's grow-only workspace in the index (callers whose
// streams live on; calls on one stream must not overlap), else from the stream-ordered pool.
// ws (nullable): take tables and scratch from this workspace instead, allocate nothing (with
// ws->cached_tables the tables come from the index's device cache, which allocates on the first
// use of a (significance, test) pair), time nothing and never tune (the caller has checked that
// the workspace is large enough).
void search_device(ddc_index *ix, const float *d_q, int64_t nq, const int32_t *d_k, int k_all,
                   int k_max, const int32_t *d_np, int np_all, int np_max, double alpha,
                   ddc_corr mode, const int64_t *d_off, int64_t *d_ids, float *d_d,
                   int64_t *d_ctr, hipStream_t s, float *qrot_out = nullptr,
                   int32_t *probes_out = nullptr, bool may_tune = true,
                   const EstimateSpec *est = nullptr, bool stream_scratch = false,
                   const Workspace *ws = nullptr);
// Argument checks of a search on device buffers (no device call).
ddc_status check_device_search(const ddc_index *ix, const float *d_queries, int64_t nq,
                               const int32_t *d_k, int32_t k_all, int32_t k_max,
                               const int32_t *d_nprobe, int32_t nprobe_all, int32_t nprobe_max,
                               double significance, ddc_corr mode, const int64_t *d_out_offsets,
                               int64_t *d_ids, float *d_dists);
// Device bytes of one search's scratch for nq queries (from the stream-ordered pool, the
// stream's workspace, or a Workspace after its table bytes).
size_t search_scratch_bytes(const ddc_index *ix, int64_t nq, int np_max, bool two_phase = false);

}  // namespace ddc
