// Host runtime behind include/ddc.h: index construction (GPU fit or import), the search
// pipeline (rotation GEMM -> coarse GEMM -> probe selection -> pruned scan), calibration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <atomic>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <numeric>
#include <stdexcept>
#include <string>
#include <vector>

#include "ddc.h"
#include "ddc_internal.h"
#include "host_math.h"
#include "runtime.h"

using namespace ddc;

// ---- scan launch shape: fixed rule, or timed once per size class --------------------
static int ceil_log2(int64_t v) {
  int r = 0;
  while ((int64_t(1) << r) < v) ++r;
  return r;
}

static std::array<int, 4> tune_class(int64_t nq, int np_max, int k_max, int kind) {
  return {ceil_log2(std::max<int64_t>(nq, 1)), ceil_log2(std::max(np_max, 1)),
          ceil_log2(std::max(k_max, 1)), kind};
}

// kernel family of a launch: pruned or not, FP8 pre-stage, residual test, estimate only
// Whether a launch can run two-phase: the learned or fixed-table stage tests (no residual or
// quantization test, no estimate-only scan) whose first test is the FP8 pre-stage, or follows
// dim block 0 with more blocks after it.
static bool two_phase_eligible(const ddc_index *ix, const ScanArgs &a) {
  if (!a.prune || a.res || a.pq_m != 0 || a.est_nb != 0 || ix->d_tile_list.p == nullptr) return false;
  if (a.pre) return true;
  return ix->NB > 1 && ix->St > 0 && ix->delta_d == kBlockDims;
}

static int scan_kind(const ScanArgs &a) {
  return a.prune + 2 * a.pre + 4 * a.res + 8 * (a.est_nb > 0 ? 1 : 0) + 16 * (a.pq_m > 0 ? 1 : 0);
}

// Launch shape of the scan: waves per query (1 or 4), look-ahead (0 or 1), persistent (0 or 1),
// two-phase (0 or 1: stage-1 sums computed list by list first), and the register budget of the
// one-wave lag-free kernel of the plain stage tests (0: four waves per SIMD, 1: five).
using Variant = std::array<int, 5>;

// Without measurements: a workgroup per query while the batch leaves the chip's wave slots
// mostly empty, multi-block loads once vectors span eight or more dim blocks, one pass, and the
// two-phase scan once a list is probed by four or more queries on average.
static Variant fixed_variant(const ddc_index *ix, int64_t nq, int prune, int np_max, bool two_ok) {
  const bool reuse = two_ok && (double)nq * np_max >= 4.0 * ix->nlist;
  return {nq < 4096 ? 4 : 1, prune && ix->NB >= 8 ? 1 : 0, 0, reuse ? 1 : 0, 0};
}

static Variant forced_or(const ddc_index *ix, Variant v, int kind, bool two_ok) {
  if (ix->waves_per_query) v[0] = ix->waves_per_query;
  // two waves per query only as the lag-parallel scan (a pruned search on an index with L >= 1)
  if (v[0] == 2 && !((kind & 1) && ix->L >= 1)) v[0] = 1;
  if (ix->lookahead >= 0) v[1] = ix->lookahead;
  if (ix->persistent >= 0) v[2] = ix->persistent;
  if (ix->two_phase >= 0) v[3] = ix->two_phase;
  if (!(kind & 1) || (kind & 4)) v[1] = 0;   // look-ahead only for the learned/fixed-table tests
  if (!two_ok) v[3] = 0;
  if (ix->waves_per_simd) v[4] = ix->waves_per_simd == 5 ? 1 : 0;
  // the five-wave build exists only there: the plain stage tests, with or without the pre-stage
  if (!((kind == 1 || kind == 3) && ix->L == 0 && v[0] == 1)) v[4] = 0;
  return v;
}

// Query orders a launch may use: grouped by first probed list (one pass per workgroup), and
// longest first with a slot counter (persistent), the latter made on first use (rebuild = true
// makes it again: the tuner charges a persistent candidate for its order kernels).
// stage1 (set when the launch may run two-phase) queues the first phase, made on first use
// like longest_first, and returns the stage-1 sums and the per-query offsets into them.
struct LaunchOrders {
  const int32_t *group = nullptr;
  std::function<std::pair<const int32_t *, int32_t *>(bool rebuild)> longest_first;
  std::function<std::pair<const float *, const int64_t *>(bool rebuild)> stage1;
  int64_t e1_cap = 0;
  float e1_tol = 0.f;   // stage1's sums in the expanded form: their error bound (ScanArgs::e1_tol)
  // the list-major full-D scan: its distances, computed before the launch shape is chosen, so
  // the tuner times the merge scan that reads them
  const float *lm_e1 = nullptr;
  const int64_t *lm_qoff = nullptr;
};

static void apply_variant(ScanArgs &a, const Variant &v, LaunchOrders &o) {
  a.waves_per_query = v[0];
  a.lookahead = v[1];
  a.occ5 = v[4];
  if (v[2]) {
    const auto pq = o.longest_first(false);
    a.order = pq.first;
    a.queue = pq.second;
  } else {
    a.order = o.group;
    a.queue = nullptr;
  }
  if (v[3] && o.stage1) {
    const auto e = o.stage1(false);
    a.e1 = e.first;
    a.e1_qoff = e.second;
    a.e1_cap = o.e1_cap;
    a.e1_tol = o.e1_tol;
  } else if (o.lm_e1) {
    a.e1 = o.lm_e1;
    a.e1_qoff = o.lm_qoff;
    a.e1_cap = o.e1_cap;
    a.e1_tol = 0.f;
  } else {
    a.e1 = nullptr;
    a.e1_qoff = nullptr;
    a.e1_cap = 0;
    a.e1_tol = 0.f;
  }
}

// Sets the launch shape of a.  An untuned class is timed on this very launch (each candidate
// three times, counters off; every candidate writes the same results), then cached; callers that
// must not stall (the server) pass may_tune = false and get the fixed rule.
static void choose_variant(ddc_index *ix, ScanArgs &a, int np_max, hipStream_t s, bool may_tune,
                           LaunchOrders &orders) {
  const int kind = scan_kind(a);
  const bool two_ok = static_cast<bool>(orders.stage1);
  const auto key = tune_class(a.nq, np_max, a.k_max, kind + (two_ok ? 32 : 0) + (orders.lm_e1 ? 64 : 0));
  Variant v = fixed_variant(ix, a.nq, a.prune, np_max, two_ok);
  if (scan_lds_request(a, v[0]) > kMaxLds) v[0] = 4;   // e.g. four lookup tables of BSA-O
  const bool need_w = ix->waves_per_query == 0, need_l = a.prune && !a.res && ix->lookahead < 0;
  const bool need_p = ix->persistent < 0, need_t = two_ok && ix->two_phase < 0;
  if (need_w || need_l || need_p || need_t) {
    std::lock_guard<std::mutex> lk(ix->tune_mtx);
    auto it = ix->tuned.find(key);
    if (it != ix->tuned.end()) {
      v = it->second;
    } else {
      hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
      HIPC(hipStreamIsCapturing(s, &cs));
      if (may_tune && cs == hipStreamCaptureStatusNone) {
        std::vector<Variant> cand;   // simplest shapes first; shapes whose LDS does not fit skipped
        for (int t2 : {0, 1})
          for (int p : {0, 1})
            for (int w : {1, 2, 4})
              for (int l : {0, 1})
                for (int o : {0, 1}) {
                  auto c = forced_or(ix, {w, l, p, t2, o}, kind, two_ok);
                  if (scan_lds_request(a, c[0]) > kMaxLds) continue;
                  if (std::find(cand.begin(), cand.end(), c) == cand.end()) cand.push_back(c);
                }
        if (cand.empty()) cand.push_back(v);
        hipEvent_t e0, e1;
        HIPC(hipEventCreate(&e0));
        HIPC(hipEventCreate(&e1));
        ScanArgs t = a;
        t.counters = nullptr;
        std::vector<float> tbest(cand.size(), INFINITY);
        for (size_t ci = 0; ci < cand.size(); ++ci) {
          apply_variant(t, cand[ci], orders);
          for (int rep = 0; rep < 3; ++rep) {
            HIPC(hipEventRecord(e0, s));
            if (cand[ci][2]) orders.longest_first(true);   // the persistent launch's own order kernels
            if (cand[ci][3]) orders.stage1(true);          // the two-phase launch's first phase
            launch_scan(t, ix->store(), s);
            HIPC(hipEventRecord(e1, s));
            HIPC(hipEventSynchronize(e1));
            float ms = 0.f;
            HIPC(hipEventElapsedTime(&ms, e0, e1));
            tbest[ci] = std::min(tbest[ci], ms);
          }
        }
        // the first candidate (simplest shape first) within 3% of the fastest: timing noise
        // does not flip the choice between near-equal shapes
        const float fastest = *std::min_element(tbest.begin(), tbest.end());
        for (size_t ci = 0; ci < cand.size(); ++ci)
          if (tbest[ci] <= fastest * 1.03f) { v = cand[ci]; break; }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        ix->tuned[key] = v;
      }
    }
  }
  v = forced_or(ix, v, kind, two_ok);
  apply_variant(a, v, orders);
}

// Phi^-1(p) by bisection on Phi(x) = erfc(-x / sqrt 2) / 2 (monotone), to double precision.
static double normal_quantile(double p) {
  double lo = -40.0, hi = 40.0;
  for (int i = 0; i < 200; ++i) {
    const double mid = 0.5 * (lo + hi);
    if (0.5 * std::erfc(-mid / std::sqrt(2.0)) < p) lo = mid; else hi = mid;
  }
  return 0.5 * (lo + hi);
}

static thread_local std::string g_err;

// ---- allocation fault injection -------------------------------------------------------
namespace {
std::atomic<int64_t> g_fault_at{0};     // the allocation that fails (1-based), 0 = none
std::atomic<int64_t> g_fault_seen{0};   // allocations checked since it was set
std::once_flag g_fault_env;

bool parse_fault(const char *spec, int64_t *n) {
  if (!spec) return false;
  if (std::strncmp(spec, "alloc:", 6) != 0) return false;
  char *end = nullptr;
  const long long v = std::strtoll(spec + 6, &end, 10);
  if (end == spec + 6 || *end != '\0' || v < 0) return false;
  *n = v;
  return true;
}
}  // namespace

std::atomic<int64_t> g_live_count{0}, g_live_bytes{0};

// the environment's setting, read once (before the first check or the first ddc_set_fault)
void fault_env_once() {
  std::call_once(g_fault_env, [] {
    int64_t n = 0;
    if (parse_fault(std::getenv("DDC_FAULT"), &n)) { g_fault_seen = 0; g_fault_at = n; }
  });
}

void ddc::alloc_track(int64_t count, int64_t bytes) {
  g_live_count += count;
  g_live_bytes += bytes;
}

void ddc::fault_check_alloc() {
  fault_env_once();
  const int64_t at = g_fault_at.load();
  if (at > 0 && ++g_fault_seen == at)
    throw DdcError(DDC_ENOMEM, "allocation failed (injected fault: allocation " + std::to_string(at) + ")");
}

ddc_status ddc::set_err(ddc_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

static int stage_count(int D, int dd) { return (D + dd - 1) / dd; }

// Lists keep ids ascending; list j occupies ceil(len_j / 64) tiles starting at tile_off[j].
static void build_lists(ddc_index *ix, std::vector<int64_t> &slot_row) {
  const int nl = ix->nlist;
  ix->list_len.assign(nl, 0);
  for (int64_t i = 0; i < ix->n; ++i) ix->list_len[ix->assign[i]]++;
  ix->tile_off.assign(nl + 1, 0);
  for (int j = 0; j < nl; ++j) ix->tile_off[j + 1] = ix->tile_off[j] + (ix->list_len[j] + kTile - 1) / kTile;
  ix->total_tiles = ix->tile_off[nl];
  slot_row.assign((size_t)ix->total_tiles * kTile, -1);
  ix->id_to_slot.assign(ix->n, -1);
  std::vector<int32_t> fill(nl, 0);
  for (int64_t i = 0; i < ix->n; ++i) {
    const int j = ix->assign[i];
    const int64_t slot = (int64_t)ix->tile_off[j] * kTile + fill[j]++;
    slot_row[slot] = i;
    ix->id_to_slot[i] = slot;
  }
}

// Upload rotation, centroids, list tables and pack the rotated base Y (device, n x Dp).
static void upload_index(ddc_index *ix, const float *d_Y, hipStream_t s) {
  const int D = ix->D, Dp = ix->Dp;
  std::vector<float> R32((size_t)Dp * Dp, 0.f), mu32(Dp, 0.f);
  for (int i = 0; i < D; ++i) {
    mu32[i] = (float)ix->mu[i];
    for (int j = 0; j < D; ++j) R32[(size_t)i * Dp + j] = (float)ix->R[(size_t)i * D + j];
  }
  ix->d_R32.alloc(R32.size() * 4);
  ix->d_mu32.alloc(mu32.size() * 4);
  HIPC(hipMemcpy(ix->d_R32.p, R32.data(), R32.size() * 4, hipMemcpyHostToDevice));
  HIPC(hipMemcpy(ix->d_mu32.p, mu32.data(), mu32.size() * 4, hipMemcpyHostToDevice));
  ix->d_R64.alloc((size_t)D * D * 8);
  ix->d_mu64.alloc((size_t)D * 8);
  HIPC(hipMemcpy(ix->d_R64.p, ix->R.data(), (size_t)D * D * 8, hipMemcpyHostToDevice));
  HIPC(hipMemcpy(ix->d_mu64.p, ix->mu.data(), (size_t)D * 8, hipMemcpyHostToDevice));

  std::vector<float> cp((size_t)ix->nlist * Dp, 0.f), cn(ix->nlist);
  for (int j = 0; j < ix->nlist; ++j) {
    double s2 = 0.0;
    for (int d = 0; d < D; ++d) {
      const float v = ix->cent[(size_t)j * D + d];
      cp[(size_t)j * Dp + d] = v;
      s2 += (double)v * v;
    }
    cn[j] = (float)s2;
  }
  ix->d_cent.alloc(cp.size() * 4);
  ix->d_cnorm.alloc(cn.size() * 4);
  HIPC(hipMemcpy(ix->d_cent.p, cp.data(), cp.size() * 4, hipMemcpyHostToDevice));
  HIPC(hipMemcpy(ix->d_cnorm.p, cn.data(), cn.size() * 4, hipMemcpyHostToDevice));

  std::vector<int64_t> slot_row;
  build_lists(ix, slot_row);
  std::vector<int32_t> ids(slot_row.size());
  for (size_t i = 0; i < slot_row.size(); ++i) ids[i] = (int32_t)slot_row[i];
  ix->d_tile_off.alloc(ix->tile_off.size() * 4);
  ix->d_list_len.alloc(ix->list_len.size() * 4);
  ix->d_ids.alloc(std::max<size_t>(ids.size(), 1) * 4);
  HIPC(hipMemcpy(ix->d_tile_off.p, ix->tile_off.data(), ix->tile_off.size() * 4, hipMemcpyHostToDevice));
  HIPC(hipMemcpy(ix->d_list_len.p, ix->list_len.data(), ix->list_len.size() * 4, hipMemcpyHostToDevice));
  if (!ids.empty()) HIPC(hipMemcpy(ix->d_ids.p, ids.data(), ids.size() * 4, hipMemcpyHostToDevice));
  {
    // list of every tile (the two-phase scan's first phase runs a workgroup per tile), and the
    // list lengths in descending order, summed (a bound on any query's candidate count)
    std::vector<int32_t> tl(std::max<int64_t>(ix->total_tiles, 1), -1);
    for (int j = 0; j < ix->nlist; ++j)
      for (int t = ix->tile_off[j]; t < ix->tile_off[j + 1]; ++t) tl[t] = j;
    ix->d_tile_list.alloc(tl.size() * 4);
    HIPC(hipMemcpy(ix->d_tile_list.p, tl.data(), tl.size() * 4, hipMemcpyHostToDevice));
    std::vector<int64_t> ls(ix->list_len.begin(), ix->list_len.end());
    std::sort(ls.begin(), ls.end(), std::greater<int64_t>());
    ix->len_desc_prefix.assign(ls.size() + 1, 0);
    for (size_t i = 0; i < ls.size(); ++i) ix->len_desc_prefix[i + 1] = ix->len_desc_prefix[i] + ls[i];
  }
  DevBuf d_slot(std::max<size_t>(slot_row.size(), 1) * 8);
  if (!slot_row.empty())
    HIPC(hipMemcpy(d_slot.p, slot_row.data(), slot_row.size() * 8, hipMemcpyHostToDevice));
  const size_t packed = (size_t)ix->total_tiles * ix->NB * kTile * kBlockDims * ix->esize();
  ix->d_base.alloc(std::max<size_t>(packed, 16));
  launch_pack(d_Y, Dp, D, ix->NB, d_slot.as<int64_t>(), ix->total_tiles, ix->d_base.p, ix->store(), s);
  ix->d_xnorm.alloc(std::max<size_t>((size_t)ix->total_tiles * kTile * 4, 16));
  launch_slot_sqnorm(ix->d_base.p, ix->store(), ix->NB, ix->total_tiles, ix->d_xnorm.as<float>(), s);
  {
    std::vector<float> lam32(Dp, 0.f);
    for (int i = 0; i < D && i < (int)ix->lam.size(); ++i) lam32[i] = (float)ix->lam[i];
    ix->d_lam32.alloc(lam32.size() * 4);
    HIPC(hipMemcpy(ix->d_lam32.p, lam32.data(), lam32.size() * 4, hipMemcpyHostToDevice));
  }
  if (ix->fp8) {
    ix->d_base8.alloc(std::max<size_t>((size_t)ix->total_tiles * kTile * kFp8Lead, 16));
    ix->d_scale8.alloc(std::max<size_t>((size_t)ix->total_tiles * 4, 16));
    launch_encode_fp8(ix->d_base.p, ix->store(), ix->NB, ix->total_tiles, ix->d_base8.as<uint8_t>(),
                      ix->d_scale8.as<float>(), s);
  }
  HIPC(hipGetLastError());
  HIPC(hipStreamSynchronize(s));
}

static void pq_upload_encode(ddc_index *ix, hipStream_t s);

static bool all_finite(const float *x, int64_t cnt) {
  for (int64_t i = 0; i < cnt; ++i)
    if (!std::isfinite(x[i])) return false;
  return true;
}

// ---------------------------------------------------------------------------------------
// calibration (Sec. V-A): label 0 = the calib_k nearest stored vectors of every training
// query (tau = K_c-th distance), label 1 = candidates met by an unpruned canonical IVF search
// with a finite tau_b and dis > tau_b (<= max_neg per query, smallest SplitMix64 keys).
// Per test stage a logistic regression on (e_s, tau) gives m_s; the residuals
// g_s = tau - m_s e_s of the label-0 pairs are kept for the target-recall adjustment.
// ---------------------------------------------------------------------------------------
static ddc_index::Table run_calibration(ddc_index *ix, const float *calib, int64_t nc, int kc,
                                        int nprobe_c, int max_neg, uint64_t seed, hipStream_t s) {
  const int D = ix->D, Dp = ix->Dp, St = ix->St;
  DevBuf d_c((size_t)nc * D * 4);
  HIPC(hipMemcpyAsync(d_c.p, calib, (size_t)nc * D * 4, hipMemcpyHostToDevice, s));
  DevBuf d_q64((size_t)nc * D * 8);
  launch_rotate64(d_c.as<float>(), nc, D, ix->d_mu64.as<double>(), ix->d_R64.as<double>(),
                  d_q64.as<double>(), s);

  // -- exact K_c-NN: FP32 unpruned scan over all lists for a candidate superset, FP64 refine
  const int kp = std::min(kMaxK, std::max(4 * kc, kc + 32));
  DevBuf d_q32((size_t)nc * Dp * 4);
  {
    GemmArgs g{};
    g.A = d_c.as<float>(); g.lda = D; g.mu = ix->d_mu32.as<float>();
    g.B = ix->d_R32.as<float>(); g.ldb = Dp; g.C = d_q32.as<float>(); g.ldc = Dp;
    g.M = nc; g.N = Dp; g.K = D; g.mode = 0; g.prec = 0;
    launch_gemm(g, s);
  }
  std::vector<int32_t> iota((size_t)nc * ix->nlist);
  for (int64_t q = 0; q < nc; ++q)
    for (int j = 0; j < ix->nlist; ++j) iota[(size_t)q * ix->nlist + j] = j;
  DevBuf d_all((size_t)nc * ix->nlist * 4);
  HIPC(hipMemcpyAsync(d_all.p, iota.data(), iota.size() * 4, hipMemcpyHostToDevice, s));
  DevBuf d_cid((size_t)nc * kp * 8), d_cd((size_t)nc * kp * 4);
  {
    ScanArgs a{};
    a.qrot = d_q32.as<float>(); a.q_stride = Dp;
    a.probes = d_all.as<int32_t>(); a.p_stride = ix->nlist; a.nprobe_all = ix->nlist;
    a.k_all = kp; a.tile_off = ix->d_tile_off.as<int32_t>(); a.list_len = ix->d_list_len.as<int32_t>();
    a.base = ix->d_base.p; a.ids = ix->d_ids.as<int32_t>();
    a.out_ids = d_cid.as<int64_t>(); a.out_d = d_cd.as<float>();
    a.nq = (int32_t)nc; a.nblocks = ix->NB; a.block_b = ix->B; a.prune = 0; a.nlist = ix->nlist;
    a.k_max = kp;
    a.waves_per_query = fixed_variant(ix, nc, 0, ix->nlist, false)[0];
    launch_scan(a, ix->store(), s);
  }
  std::vector<int64_t> cid((size_t)nc * kp);
  std::vector<float> cd((size_t)nc * kp);
  HIPC(hipMemcpyAsync(cid.data(), d_cid.p, cid.size() * 8, hipMemcpyDeviceToHost, s));
  HIPC(hipMemcpyAsync(cd.data(), d_cd.p, cd.size() * 4, hipMemcpyDeviceToHost, s));
  HIPC(hipStreamSynchronize(s));
  std::vector<int64_t> cslot(cid.size());
  for (size_t i = 0; i < cid.size(); ++i) cslot[i] = cid[i] >= 0 ? ix->id_to_slot[cid[i]] : -1;
  DevBuf d_cs(cslot.size() * 8), d_c64(cslot.size() * 8);
  HIPC(hipMemcpyAsync(d_cs.p, cslot.data(), cslot.size() * 8, hipMemcpyHostToDevice, s));
  launch_refine64(d_q64.as<double>(), D, ix->d_base.p, ix->store(), ix->NB, d_cs.as<int64_t>(), kp,
                  nc, d_c64.as<double>(), s);
  std::vector<double> c64(cslot.size());
  HIPC(hipMemcpyAsync(c64.data(), d_c64.p, c64.size() * 8, hipMemcpyDeviceToHost, s));
  std::vector<double> q64((size_t)nc * D);
  HIPC(hipMemcpyAsync(q64.data(), d_q64.p, q64.size() * 8, hipMemcpyDeviceToHost, s));
  HIPC(hipStreamSynchronize(s));

  std::vector<int32_t> pair_q;
  std::vector<int64_t> pair_slot;
  std::vector<double> pair_tau;
  std::vector<int64_t> all_slots;  // for the rare full-FP64 fallback
  for (int64_t q = 0; q < nc; ++q) {
    std::vector<std::pair<double, int64_t>> c;  // (d64, id)
    for (int t = 0; t < kp; ++t)
      if (cid[q * kp + t] >= 0) c.push_back({c64[q * kp + t], cid[q * kp + t]});
    std::sort(c.begin(), c.end());
    const int got = (int)c.size();
    bool exact = got >= kc;
    if (exact && got == kp) {
      // any vector outside the FP32 superset has FP32 distance >= the last one kept
      double qn = 0;
      for (int d = 0; d < D; ++d) qn += q64[q * D + d] * q64[q * D + d];
      const double last32 = cd[q * kp + kp - 1];
      exact = c[kc - 1].first * (1.0 + 1e-3) + 1e-6 * qn < last32;
    }
    if (!exact && got < std::min<int64_t>(kc, ix->n)) exact = got == ix->n;
    if (!exact) {
      // FP64 over every stored vector for this query
      if (all_slots.empty())
        for (int64_t i = 0; i < ix->n; ++i) all_slots.push_back(ix->id_to_slot[i]);
      DevBuf d_as(all_slots.size() * 8), d_ad(all_slots.size() * 8);
      HIPC(hipMemcpyAsync(d_as.p, all_slots.data(), all_slots.size() * 8, hipMemcpyHostToDevice, s));
      launch_refine64(d_q64.as<double>() + q * D, D, ix->d_base.p, ix->store(), ix->NB,
                      d_as.as<int64_t>(), (int32_t)all_slots.size(), 1, d_ad.as<double>(), s);
      std::vector<double> ad(all_slots.size());
      HIPC(hipMemcpyAsync(ad.data(), d_ad.p, ad.size() * 8, hipMemcpyDeviceToHost, s));
      HIPC(hipStreamSynchronize(s));
      c.clear();
      for (int64_t i = 0; i < ix->n; ++i) c.push_back({ad[i], i});
      std::partial_sort(c.begin(), c.begin() + std::min<int64_t>(kc, ix->n), c.end());
    }
    const int take = std::min<int>(kc, (int)c.size());
    if (take < kc) throw DdcError(DDC_EINVAL, "calibration needs at least calib_k base vectors");
    const double tau = c[kc - 1].first;
    for (int t = 0; t < kc; ++t) {
      pair_q.push_back((int32_t)q);
      pair_slot.push_back(ix->id_to_slot[c[t].second]);
      pair_tau.push_back(tau);
    }
  }
  const int64_t n0 = (int64_t)pair_q.size();

  // -- label 1: probes (FP64 centroid distances, ascending by (d, list)), FP64 canonical search
  DevBuf d_cd64((size_t)nc * ix->nlist * 8);
  launch_cdist64(d_q64.as<double>(), nc, D, ix->d_cent.as<float>(), Dp, ix->nlist, d_cd64.as<double>(), s);
  std::vector<double> cd64((size_t)nc * ix->nlist);
  HIPC(hipMemcpyAsync(cd64.data(), d_cd64.p, cd64.size() * 8, hipMemcpyDeviceToHost, s));
  HIPC(hipStreamSynchronize(s));
  std::vector<int32_t> probes((size_t)nc * nprobe_c);
  {
    std::vector<int32_t> ord(ix->nlist);
    for (int64_t q = 0; q < nc; ++q) {
      std::iota(ord.begin(), ord.end(), 0);
      const double *row = &cd64[(size_t)q * ix->nlist];
      std::partial_sort(ord.begin(), ord.begin() + nprobe_c, ord.end(), [&](int a, int b) {
        return row[a] < row[b] || (row[a] == row[b] && a < b);
      });
      for (int p = 0; p < nprobe_c; ++p) probes[(size_t)q * nprobe_c + p] = ord[p];
    }
  }
  DevBuf d_pr(probes.size() * 4), d_ns((size_t)nc * max_neg * 8), d_nt((size_t)nc * max_neg * 8);
  HIPC(hipMemcpyAsync(d_pr.p, probes.data(), probes.size() * 4, hipMemcpyHostToDevice, s));
  {
    NegArgs a{};
    a.qrot = d_q64.as<double>(); a.D = D; a.probes = d_pr.as<int32_t>(); a.nprobe = nprobe_c;
    a.tile_off = ix->d_tile_off.as<int32_t>(); a.list_len = ix->d_list_len.as<int32_t>();
    a.base = ix->d_base.p; a.store = ix->store(); a.nblocks = ix->NB; a.ids = ix->d_ids.as<int32_t>();
    a.k = kc; a.block_b = ix->B; a.max_neg = max_neg; a.lag = ix->L;
    a.key_base = splitmix64(seed + TAG_NEG); a.nq = nc;
    a.neg_slot = d_ns.as<int64_t>(); a.neg_tau = d_nt.as<double>();
    launch_negatives64(a, s);
  }
  std::vector<int64_t> ns((size_t)nc * max_neg);
  std::vector<double> nt((size_t)nc * max_neg);
  HIPC(hipMemcpyAsync(ns.data(), d_ns.p, ns.size() * 8, hipMemcpyDeviceToHost, s));
  HIPC(hipMemcpyAsync(nt.data(), d_nt.p, nt.size() * 8, hipMemcpyDeviceToHost, s));
  HIPC(hipStreamSynchronize(s));
  for (int64_t q = 0; q < nc; ++q)
    for (int t = 0; t < max_neg; ++t) {
      const int64_t sl = ns[q * max_neg + t];
      if (sl < 0) continue;
      pair_q.push_back((int32_t)q);
      pair_slot.push_back(sl);
      pair_tau.push_back(nt[q * max_neg + t]);
    }
  const int64_t npairs = (int64_t)pair_q.size();
  const int64_t n1 = npairs - n0;

  // -- features e_s at every test stage (FP64); with FP8 codes column 0 is the pre-stage's
  // e_0 over the decoded lead dims, then the stored-precision stages
  const int P = ix->P(), Tt = ix->Tt();
  std::vector<int32_t> send(std::max(St, 1));
  for (int t = 0; t < St; ++t) send[t] = ((t + 1) * ix->delta_d) / kBlockDims;
  std::vector<double> feat((size_t)npairs * std::max(Tt, 1));
  if (Tt > 0) {
    DevBuf d_pq(npairs * 4), d_ps(npairs * 8), d_se(std::max(St, 1) * 4),
        d_f((size_t)npairs * Tt * 8), d_f8(P ? (size_t)npairs * 8 : 8);
    HIPC(hipMemcpyAsync(d_pq.p, pair_q.data(), npairs * 4, hipMemcpyHostToDevice, s));
    HIPC(hipMemcpyAsync(d_ps.p, pair_slot.data(), npairs * 8, hipMemcpyHostToDevice, s));
    HIPC(hipMemcpyAsync(d_se.p, send.data(), std::max(St, 1) * 4, hipMemcpyHostToDevice, s));
    if (St > 0)
      launch_features64(d_q64.as<double>(), D, ix->d_base.p, ix->store(), ix->NB, d_pq.as<int32_t>(),
                        d_ps.as<int64_t>(), npairs, d_se.as<int32_t>(), St, d_f.as<double>(), s);
    std::vector<double> f8(P ? npairs : 0);
    if (P) {
      launch_features8(d_q64.as<double>(), D, ix->d_base8.as<uint8_t>(), ix->d_scale8.as<float>(),
                       d_pq.as<int32_t>(), d_ps.as<int64_t>(), npairs, d_f8.as<double>(), 1, s);
      HIPC(hipMemcpyAsync(f8.data(), d_f8.p, (size_t)npairs * 8, hipMemcpyDeviceToHost, s));
    }
    std::vector<double> fs((size_t)npairs * St);
    if (St > 0)
      HIPC(hipMemcpyAsync(fs.data(), d_f.p, (size_t)npairs * St * 8, hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    for (int64_t p = 0; p < npairs; ++p) {
      if (P) feat[(size_t)p * Tt] = f8[p];
      for (int t = 0; t < St; ++t) feat[(size_t)p * Tt + P + t] = fs[(size_t)p * St + t];
    }
  }
  HIPC(hipGetLastError());

  // -- per stage logistic regression -> m_s ; residuals of label 0
  std::vector<double> m(Tt, 1.0);
  for (int t = 0; t < Tt && n1 > 0; ++t) {
    std::vector<double> F((size_t)npairs * 2), y(npairs);
    for (int64_t p = 0; p < npairs; ++p) {
      F[2 * p] = feat[(size_t)p * Tt + t];
      F[2 * p + 1] = pair_tau[p];
      y[p] = p < n0 ? 0.0 : 1.0;
    }
    double b, w1, w2;
    logistic_fit(F, y, b, w1, w2);
    if (w2 < 0 && -w1 / w2 > 0) m[t] = -w1 / w2;
  }
  std::vector<double> G((size_t)n0 * Tt);
  for (int64_t j = 0; j < n0; ++j)
    for (int t = 0; t < Tt; ++t) G[(size_t)j * Tt + t] = pair_tau[j] - m[t] * feat[(size_t)j * Tt + t];
  ddc_index::Table tab;
  tab.kc = kc;
  tab.m = m;
  tab.resid = G;
  tab.n0 = n0;

  // -- BSA-O: features (asymmetric distance, quantization error, tau) of the same pairs, FP64;
  // one logistic regression, then the label-0 residuals of its test
  if (ix->pq_m > 0) {
    DevBuf d_pq_q(npairs * 4), d_pq_s(npairs * 8), d_adc(npairs * 8), d_err(npairs * 8);
    HIPC(hipMemcpyAsync(d_pq_q.p, pair_q.data(), npairs * 4, hipMemcpyHostToDevice, s));
    HIPC(hipMemcpyAsync(d_pq_s.p, pair_slot.data(), npairs * 8, hipMemcpyHostToDevice, s));
    launch_pq_features64(d_q64.as<double>(), D, ix->d_base.p, ix->store(), ix->NB,
                         ix->d_pq_perm.as<int32_t>(), ix->d_pq_books.as<float>(), ix->pq_m, ix->pq_dsub,
                         ix->d_pq_codes.as<uint8_t>(), d_pq_q.as<int32_t>(), d_pq_s.as<int64_t>(), npairs,
                         d_adc.as<double>(), d_err.as<double>(), s);
    std::vector<double> adc(npairs), err(npairs);
    HIPC(hipMemcpyAsync(adc.data(), d_adc.p, npairs * 8, hipMemcpyDeviceToHost, s));
    HIPC(hipMemcpyAsync(err.data(), d_err.p, npairs * 8, hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    HIPC(hipGetLastError());
    if (n1 > 0) {
      std::vector<double> F((size_t)npairs * 3), y(npairs), w;
      for (int64_t p = 0; p < npairs; ++p) {
        F[3 * p] = adc[p];
        F[3 * p + 1] = err[p];
        F[3 * p + 2] = pair_tau[p];
        y[p] = p < n0 ? 0.0 : 1.0;
      }
      double b;
      logistic_fit_p(F, 3, y, b, w);
      // sign(w1 dis' + w3 err + w2 tau + b) > 0  <=>  m1 dis' + m3 err + beta > tau (w2 < 0)
      if (w[2] < 0 && -w[0] / w[2] > 0) {
        tab.pq_m1 = -w[0] / w[2];
        tab.pq_m3 = -w[1] / w[2];
      }
    }
    tab.pq_resid.resize(n0);
    for (int64_t j = 0; j < n0; ++j) tab.pq_resid[j] = pair_tau[j] - tab.pq_m1 * adc[j] - tab.pq_m3 * err[j];
  }
  return tab;
}

static void set_tables(ddc_index *ix, std::vector<ddc_index::Table> t) {
  std::sort(t.begin(), t.end(), [](const ddc_index::Table &a, const ddc_index::Table &b) { return a.kc < b.kc; });
  std::lock_guard<std::mutex> lk(ix->beta_mtx);
  ix->tables = std::move(t);
  ix->beta_cache.clear();
  ix->tab_cache.clear();
  ix->tab_host.clear();
}

// The table a search with K uses: the last (largest K_c) with K_c <= K, else the first.
static int table_for_k(const ddc_index *ix, int k) {
  int t = 0;
  for (int i = 1; i < (int)ix->tables.size(); ++i)
    if (ix->tables[i].kc <= k) t = i;
  return t;
}

static std::vector<double> beta_locked(ddc_index *ix, double alpha, int mode, int t) {
  auto key = std::make_tuple(alpha, mode, t);
  auto it = ix->beta_cache.find(key);
  if (it != ix->beta_cache.end()) return it->second;
  const auto &tb = ix->tables[t];
  auto b = beta_for_alpha(tb.resid, tb.n0, ix->Tt(), alpha, mode);
  ix->beta_cache[key] = b;
  return b;
}

static std::vector<double> get_beta(ddc_index *ix, double alpha, int mode, int t) {
  std::lock_guard<std::mutex> lk(ix->beta_mtx);
  return beta_locked(ix, alpha, mode, t);
}

// Every table for one (alpha, correction mode) as the scan reads it: [ntab][NB + 1][2] (m, beta)
// per dim block (beta = -inf where no test follows; entry NB = the FP8 pre-stage).  Host rows,
// cached per key (beta_mtx held).
static std::shared_ptr<const std::vector<float>> host_tables_locked(ddc_index *ix, double alpha,
                                                                    ddc_corr mode, int *ntab) {
  const bool ads = mode == DDC_CORR_ADS;
  const bool lossless = mode == DDC_CORR_LOSSLESS || ads;   // one fixed table, no pre-stage
  const auto key = std::make_pair(ads ? ix->ads_eps0 : lossless ? -1.0 : alpha, (int)mode);
  const int nt = lossless ? 1 : (int)ix->tables.size();
  *ntab = nt;
  auto it = ix->tab_host.find(key);
  if (it != ix->tab_host.end()) return it->second;
  const int NB = ix->NB, P = ix->P();
  auto hp = std::make_shared<std::vector<float>>((size_t)nt * (NB + 1) * 2);
  std::vector<float> &h = *hp;
  for (int t = 0; t < nt; ++t) {
    float *row = &h[(size_t)t * (NB + 1) * 2];
    for (int b = 0; b <= NB; ++b) { row[2 * b] = 0.f; row[2 * b + 1] = -INFINITY; }
    std::vector<double> mm(ix->Tt(), 1.0), bb(ix->Tt(), 0.0);
    if (ads) {
      // (D / d) e > (1 + eps0 / sqrt(d))^2 tau  <=>  m e > tau
      for (int j = 0; j < ix->St; ++j) {
        const double d = std::min((j + 1) * ix->delta_d, ix->D);
        const double g = 1.0 + ix->ads_eps0 / std::sqrt(d);
        mm[P + j] = ((double)ix->D / d) / (g * g);
      }
    } else if (!lossless) {
      mm = ix->tables[t].m;
      bb = beta_locked(ix, alpha, DDC_CALIB_JOINT, t);
    }
    for (int j = 0; j < ix->St; ++j) {
      const int b = ((j + 1) * ix->delta_d) / kBlockDims - 1;
      row[2 * b] = (float)mm[P + j];
      row[2 * b + 1] = (float)bb[P + j];
    }
    if (P && !lossless) { row[2 * NB] = (float)mm[0]; row[2 * NB + 1] = (float)bb[0]; }
  }
  ix->tab_host[key] = hp;
  return hp;
}

// Device copy of host_tables_locked's rows, cached per key.
static std::shared_ptr<DevBuf> device_tables(ddc_index *ix, double alpha, ddc_corr mode, int *ntab) {
  std::lock_guard<std::mutex> lk(ix->beta_mtx);
  const bool ads = mode == DDC_CORR_ADS;
  const bool lossless = mode == DDC_CORR_LOSSLESS || ads;
  const auto key = std::make_pair(ads ? ix->ads_eps0 : lossless ? -1.0 : alpha, (int)mode);
  const auto h = host_tables_locked(ix, alpha, mode, ntab);
  auto it = ix->tab_cache.find(key);
  if (it != ix->tab_cache.end()) return it->second;
  auto buf = std::make_shared<DevBuf>(h->size() * 4);
  HIPC(hipMemcpy(buf->p, h->data(), h->size() * 4, hipMemcpyHostToDevice));
  ix->tab_cache[key] = buf;
  return buf;
}

// Device tables of a BSA-O search: [ntab][NB + 1][2] lossless stage rows (m = 1, beta = 0 where
// a test follows: refinement only prunes candidates whose partial distance already exceeds
// tau), then [ntab][4] = (m1, m3, beta(alpha), 0) of each table's quantization test.
static std::shared_ptr<const std::vector<float>> host_pq_tables_locked(ddc_index *ix, double alpha,
                                                                       int *ntab) {
  const auto key = std::make_pair(alpha, (int)DDC_CORR_BSAO);
  const int nt = (int)ix->tables.size();
  *ntab = nt;
  auto it = ix->tab_host.find(key);
  if (it != ix->tab_host.end()) return it->second;
  const int NB = ix->NB;
  auto hp = std::make_shared<std::vector<float>>((size_t)nt * (NB + 1) * 2 + (size_t)nt * 4);
  std::vector<float> &h = *hp;
  for (int t = 0; t < nt; ++t) {
    float *row = &h[(size_t)t * (NB + 1) * 2];
    for (int b = 0; b <= NB; ++b) { row[2 * b] = 0.f; row[2 * b + 1] = -INFINITY; }
    for (int j = 0; j < ix->St; ++j) {
      const int b = ((j + 1) * ix->delta_d) / kBlockDims - 1;
      row[2 * b] = 1.f;
      row[2 * b + 1] = 0.f;
    }
    const auto &tb = ix->tables[t];
    const double beta = beta_for_alpha(tb.pq_resid, tb.n0, 1, alpha, 0)[0];
    float *pq = &h[(size_t)nt * (NB + 1) * 2 + (size_t)t * 4];
    pq[0] = (float)tb.pq_m1;
    pq[1] = (float)tb.pq_m3;
    pq[2] = (float)beta;
    pq[3] = 0.f;
  }
  ix->tab_host[key] = hp;
  return hp;
}

static std::shared_ptr<DevBuf> device_pq_tables(ddc_index *ix, double alpha, int *ntab) {
  std::lock_guard<std::mutex> lk(ix->beta_mtx);
  const auto key = std::make_pair(alpha, (int)DDC_CORR_BSAO);
  const auto h = host_pq_tables_locked(ix, alpha, ntab);
  auto it = ix->tab_cache.find(key);
  if (it != ix->tab_cache.end()) return it->second;
  auto buf = std::make_shared<DevBuf>(h->size() * 4);
  HIPC(hipMemcpy(buf->p, h->data(), h->size() * 4, hipMemcpyHostToDevice));
  ix->tab_cache[key] = buf;
  return buf;
}

// ---------------------------------------------------------------------------------------
// search pipeline
// ---------------------------------------------------------------------------------------
template <class F> static void timed(ddc_index *ix, int kernel, hipStream_t s, F &&launch,
                                     bool off = false) {
  if (!ix->timing || off) { launch(); return; }
  ddc_index::Mark m{kernel, nullptr, nullptr};
  HIPC(hipEventCreate(&m.a));
  HIPC(hipEventCreate(&m.b));
  HIPC(hipEventRecord(m.a, s));
  launch();
  HIPC(hipEventRecord(m.b, s));
  std::lock_guard<std::mutex> lk(ix->timing_mtx);
  ix->marks.push_back(m);
}

// A piece of a search's scratch buffer.
struct ScratchPart {
  void *p;
  template <class T> T *as() const { return reinterpret_cast<T *>(p); }
};

// The stream's search workspace, grown to at least `bytes` (a grown one replaces the old after
// the stream's queued work is done with it).
static void *stream_workspace(ddc_index *ix, hipStream_t s, size_t bytes) {
  std::lock_guard<std::mutex> lk(ix->scratch_mtx);
  auto &w = ix->scratch[s];
  if (!w) w = std::make_unique<DevBuf>();
  if (w->bytes < bytes) {
    if (w->p) HIPC(hipStreamSynchronize(s));
    w->alloc(bytes);
  }
  return w->p;
}

// Queries per scratch chunk, and the scratch pieces of one chunk of cmax queries: rotated
// queries, coarse distances, probes, then the query orders' keys, histograms and ranks and the
// persistent launch's slot counter; with two_phase (or the list-major full-D scan) the first
// phase's list counts and starts, pair ranks, pairs by list, pair offsets, query counts and
// offsets, its sums (a bound on the batch's candidates: cmax times the summed lengths of the
// np_max longest lists, each padded to whole 128-byte lines) and the queries' squared norms;
// each piece 256-byte aligned.
constexpr int64_t kChunk = 32768;
// Error bound of the expanded-form stage-1 sums against the scan's own, relative to
// 3 ||q'_1||^2 + 2 |e1|: about 85 units in the last place cover the norms' and inner product's
// FP32 sums over 32 terms, the final two roundings and the direct sum's rounding (||y_1||^2 <=
// 2 ||q'_1||^2 + 2 e1); 2^-12 leaves a factor of about 48 on top.
constexpr float kE1Tol = 1.0f / 4096.0f;
constexpr int kParts = 20;
static int64_t e1_bound(const ddc_index *ix, int64_t cmax, int np_max) {
  // every (query, list) segment is padded to a multiple of 32 sums
  const int np = std::min<int>(std::max(np_max, 0), (int)ix->len_desc_prefix.size() - 1);
  return np > 0 ? cmax * (ix->len_desc_prefix[np] + 31 * (int64_t)np) : 0;
}
static void scratch_sizes(const ddc_index *ix, int64_t cmax, int np_max, bool two_phase,
                          size_t (&sizes)[kParts]) {
  const size_t pairs = (size_t)cmax * np_max, t = two_phase ? 1 : 0;
  const size_t v[kParts] = {(size_t)cmax * ix->Dp * 4, (size_t)cmax * ix->nlist * 4,
                            (size_t)cmax * np_max * 4, (size_t)(ix->nlist + 1) * 4, (size_t)cmax * 4,
                            (size_t)cmax * 4, (size_t)cmax * 4, (size_t)257 * 4, (size_t)cmax * 4,
                            (size_t)cmax * 4, 256,
                            t * (ix->nlist + 1) * 4, t * (ix->nlist + 1) * 4, t * pairs * 4, t * pairs * 4,
                            t * pairs * 8, t * cmax * 8, t * (cmax + 1) * 8,
                            t * (size_t)e1_bound(ix, cmax, np_max) * 4, t * cmax * 4};
  for (int i = 0; i < kParts; ++i) sizes[i] = v[i];
}

// Queries per chunk: kChunk, fewer when the two-phase sums of a chunk could pass 16 GiB.
static int64_t chunk_queries(const ddc_index *ix, int np_max, bool two_phase) {
  if (!two_phase) return kChunk;
  const int64_t per = std::max<int64_t>(1, e1_bound(ix, 1, np_max));
  return std::max<int64_t>(1, std::min<int64_t>(kChunk, ((int64_t)1 << 32) / per));
}

size_t ddc::search_scratch_bytes(const ddc_index *ix, int64_t nq, int np_max, bool two_phase) {
  size_t sizes[kParts], total = 0;
  scratch_sizes(ix, std::min(chunk_queries(ix, np_max, two_phase), nq), np_max, two_phase, sizes);
  for (size_t b : sizes) total += (b + 255) & ~(size_t)255;
  return total;
}

void ddc::search_device(ddc_index *ix, const float *d_q, int64_t nq, const int32_t *d_k, int k_all,
                        int k_max, const int32_t *d_np, int np_all, int np_max, double alpha,
                        ddc_corr mode, const int64_t *d_off, int64_t *d_ids, float *d_d,
                        int64_t *d_ctr, hipStream_t s, float *qrot_out, int32_t *probes_out,
                        bool may_tune, const EstimateSpec *est, bool stream_scratch,
                        const Workspace *ws_ext) {
  const int Dp = ix->Dp, D = ix->D;
  const bool fixed_ws = ws_ext != nullptr;
  if (fixed_ws) may_tune = false;
  // correction rows: from the device cache, or (fixed workspace) copied from their host rows into
  // the workspace's start on s (the host rows live in the index, so the copy's source outlives it)
  auto take_tables = [&](std::shared_ptr<const std::vector<float>> h) -> float * {
    if (h->size() * 4 > Workspace::kTableBytes) throw DdcError(DDC_EINVAL, "correction tables exceed the workspace");
    HIPC(hipMemcpyAsync(ws_ext->p, h->data(), h->size() * 4, hipMemcpyHostToDevice, s));
    return reinterpret_cast<float *>(ws_ext->p);
  };
  ScanArgs a{};
  a.prune = 0;
  std::shared_ptr<DevBuf> tabs;   // keeps the device tables alive for this call
  if (est) {
    mode = DDC_CORR_NONE;
    a.est_nb = est->nb;
    a.est_res = est->residual;
    a.est_scale = est->scale;
    a.xnorm = ix->d_xnorm.as<float>();
  }
  const bool learned = mode == DDC_CORR_LEARNED && alpha > 0 && ix->Tt() > 0;
  // LOSSLESS tests e_s > tau with the stored values only: the FP8 estimate is no lower bound;
  // ADS is a fixed table on the stored values too
  const bool lossless = (mode == DDC_CORR_LOSSLESS || mode == DDC_CORR_ADS) && ix->St > 0;
  const bool copy_tables = fixed_ws && !ws_ext->cached_tables;
  if (mode == DDC_CORR_BSAO) {
    a.prune = 1;
    if (copy_tables) {
      std::shared_ptr<const std::vector<float>> h;
      {
        std::lock_guard<std::mutex> lk(ix->beta_mtx);
        h = host_pq_tables_locked(ix, alpha, &a.ntab);
      }
      a.tab = take_tables(h);
    } else {
      tabs = device_pq_tables(ix, alpha, &a.ntab);
      a.tab = tabs->as<float>();
    }
    a.pq_tab = a.tab + (size_t)a.ntab * (ix->NB + 1) * 2;
    for (int t = 0; t < a.ntab; ++t) a.tab_k[t] = ix->tables[t].kc;
    for (int j = 0; j < ix->St; ++j) a.test_after[((j + 1) * ix->delta_d) / kBlockDims - 1] = 1;
    a.pq_m = ix->pq_m;
    a.pq_dsub = ix->pq_dsub;
    a.pq_codes = ix->d_pq_codes.as<uint8_t>();
    a.pq_err = ix->d_pq_err.as<float>();
    a.pq_books = ix->d_pq_books.as<float>();
    a.pq_perm = ix->d_pq_perm.as<int32_t>();
  } else if (mode == DDC_CORR_BSAR && ix->St > 0) {
    a.prune = 1;
    a.res = 1;
    a.xnorm = ix->d_xnorm.as<float>();
    a.lam = ix->d_lam32.as<float>();
    a.bsar_m = (float)(ix->bsar_m > 0 ? ix->bsar_m : normal_quantile(1.0 - alpha));
    for (int j = 0; j < ix->St; ++j) a.test_after[((j + 1) * ix->delta_d) / kBlockDims - 1] = 1;
  } else if (learned || lossless) {
    a.prune = 1;
    if (copy_tables) {
      std::shared_ptr<const std::vector<float>> h;
      {
        std::lock_guard<std::mutex> lk(ix->beta_mtx);
        h = host_tables_locked(ix, alpha, mode, &a.ntab);
      }
      a.tab = take_tables(h);
    } else {
      tabs = device_tables(ix, alpha, mode, &a.ntab);
      a.tab = tabs->as<float>();
    }
    for (int t = 0; t < a.ntab; ++t) a.tab_k[t] = lossless ? 1 : ix->tables[t].kc;
    for (int j = 0; j < ix->St; ++j) a.test_after[((j + 1) * ix->delta_d) / kBlockDims - 1] = 1;
    if (learned && ix->P()) {
      a.pre = 1;
      a.base8 = ix->d_base8.as<uint8_t>();
      a.scale8 = ix->d_scale8.as<float>();
    }
  }
  // Scratch of a chunk (rotated queries, coarse distances, probes, query orders), carved from
  // one buffer: a caller's fixed workspace after its table bytes; with stream_scratch and
  // outside graph capture the stream's grow-only workspace, reused call after call (stream
  // order keeps a call's kernels from overlapping the next call's use of it; per-call
  // stream-ordered allocations left the GPU idle about 30 us at every call); else one
  // stream-ordered allocation (which a captured graph records).
  // the two-phase scan may run (its scratch is then part of the buffer)
  ScanArgs elig{};
  elig.prune = a.prune; elig.res = a.res; elig.pre = a.pre; elig.pq_m = a.pq_m; elig.est_nb = a.est_nb;
  // (not for the fixed workspace, which has no room for the stage-1 sums, nor for callers that
  // neither tune nor keep a stream workspace: the server sizes its admission budget without them)
  const bool two_ok = !fixed_ws && !qrot_out && (may_tune || stream_scratch) && ix->two_phase != 0 &&
                      two_phase_eligible(ix, elig);
  // the list-major full-D scan (no test; opted into with full_d_matrix)
  const bool lm_full = !fixed_ws && !qrot_out && !a.prune && !est && ix->full_d_matrix == 1 &&
                       ix->d_tile_list.p != nullptr;
  const int64_t chunk = chunk_queries(ix, np_max, two_ok || lm_full);
  const int64_t cmax = std::min(chunk, nq);
  size_t sizes[kParts];
  scratch_sizes(ix, cmax, np_max, two_ok || lm_full, sizes);
  size_t total = 0;
  for (size_t b : sizes) total += (b + 255) & ~(size_t)255;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  HIPC(hipStreamIsCapturing(s, &cap));
  if (fixed_ws && Workspace::kTableBytes + total > ws_ext->bytes)
    throw DdcError(DDC_EINVAL, "search scratch exceeds the workspace");
  const bool reuse = !fixed_ws && stream_scratch && cap == hipStreamCaptureStatusNone;
  AsyncBuf pooled(reuse || fixed_ws ? 0 : total, s);
  char *const ws = fixed_ws ? reinterpret_cast<char *>(ws_ext->p) + Workspace::kTableBytes
                   : reuse  ? reinterpret_cast<char *>(stream_workspace(ix, s, total))
                            : pooled.as<char>();
  void *part[kParts];
  {
    size_t off = 0;
    for (int i = 0; i < kParts; ++i) {
      part[i] = ws + off;
      off += (sizes[i] + 255) & ~(size_t)255;
    }
  }
  const ScratchPart qrot{part[0]}, cdist{part[1]}, probes{part[2]}, ord_hist{part[3]}, ord_rank{part[4]},
      ord{part[5]}, lpt_key{part[6]}, lpt_hist{part[7]}, lpt_rank{part[8]}, lpt{part[9]}, queue{part[10]},
      s1_lcnt{part[11]}, s1_lstart{part[12]}, s1_rank{part[13]}, s1_lpair{part[14]}, s1_poff{part[15]},
      s1_qcnt{part[16]}, s1_qoff{part[17]}, s1_e1{part[18]}, s1_qnorm{part[19]};
  const int64_t e1_cap = two_ok || lm_full ? e1_bound(ix, cmax, np_max) : 0;
  for (int64_t q0 = 0; q0 < nq; q0 += chunk) {
    const int64_t nqc = std::min(chunk, nq - q0);
    GemmArgs g{};
    g.A = d_q + q0 * D; g.lda = D; g.mu = ix->d_mu32.as<float>();
    g.B = ix->d_R32.as<float>(); g.ldb = Dp; g.C = qrot.as<float>(); g.ldc = Dp;
    g.M = nqc; g.N = Dp; g.K = D; g.mode = 0; g.prec = ix->rot == DDC_ROT_BF16 ? 1 : 0;
    timed(ix, 0, s, [&] { launch_gemm(g, s); }, fixed_ws);
    GemmArgs c{};
    c.A = qrot.as<float>(); c.lda = Dp; c.mu = nullptr; c.B = ix->d_cent.as<float>(); c.ldb = Dp;
    c.bias = ix->d_cnorm.as<float>(); c.C = cdist.as<float>(); c.ldc = ix->nlist;
    c.M = nqc; c.N = ix->nlist; c.K = Dp; c.mode = 1; c.prec = 0;
    timed(ix, 1, s, [&] { launch_gemm(c, s); }, fixed_ws);
    timed(ix, 2, s, [&] {
      launch_select(cdist.as<float>(), ix->nlist, ix->nlist, d_np ? d_np + q0 : nullptr, np_all,
                    np_max, probes.as<int32_t>(), np_max, nqc, s);
    }, fixed_ws);
    if (qrot_out) {
      HIPC(hipMemcpy2DAsync(qrot_out + q0 * D, D * 4, qrot.p, Dp * 4, D * 4, nqc,
                            hipMemcpyDeviceToHost, s));
      HIPC(hipMemcpyAsync(probes_out + q0 * np_max, probes.p, (size_t)nqc * np_max * 4,
                          hipMemcpyDeviceToHost, s));
      HIPC(hipStreamSynchronize(s));
      continue;
    }
    a.qrot = qrot.as<float>(); a.q_stride = Dp;
    a.probes = probes.as<int32_t>(); a.p_stride = np_max;
    a.nprobe = d_np ? d_np + q0 : nullptr; a.nprobe_all = np_all;
    a.k = d_k ? d_k + q0 : nullptr; a.k_all = k_all;
    a.out_off = d_off ? d_off + q0 : nullptr;
    a.tile_off = ix->d_tile_off.as<int32_t>(); a.list_len = ix->d_list_len.as<int32_t>();
    a.base = ix->d_base.p; a.ids = ix->d_ids.as<int32_t>();
    a.out_ids = d_off ? d_ids : d_ids + q0 * k_all;
    a.out_d = d_off ? d_d : d_d + q0 * k_all;
    a.counters = d_ctr;
    LaunchOrders orders;
    if (ix->query_order) {
      launch_query_order(probes.as<int32_t>(), np_max, nqc, ix->nlist, ord_hist.as<int32_t>(),
                         ord_rank.as<int32_t>(), ord.as<int32_t>(), s);
      orders.group = ord.as<int32_t>();
    }
    bool lpt_made = false;
    orders.longest_first = [&](bool rebuild) -> std::pair<const int32_t *, int32_t *> {
      const bool first = !lpt_made;
      lpt_made = true;
      if (first || rebuild) {
        launch_work_order(probes.as<int32_t>(), np_max, d_np ? d_np + q0 : nullptr, np_all,
                          ix->d_list_len.as<int32_t>(), ix->nlist, nqc, lpt_key.as<int32_t>(),
                          lpt_hist.as<int32_t>(), lpt_rank.as<int32_t>(), lpt.as<int32_t>(), s);
      }
      return {lpt.as<int32_t>(), queue.as<int32_t>()};
    };
    bool s1_made = false;
    auto stage1_args = [&]() {
      Stage1Args s1{};
      s1.probes = probes.as<int32_t>(); s1.p_stride = np_max;
      s1.nprobe = d_np ? d_np + q0 : nullptr; s1.nprobe_all = np_all;
      s1.list_len = ix->d_list_len.as<int32_t>(); s1.tile_off = ix->d_tile_off.as<int32_t>();
      s1.tile_list = ix->d_tile_list.as<int32_t>(); s1.nlist = ix->nlist;
      s1.total_tiles = ix->total_tiles; s1.nq = nqc;
      s1.qrot = qrot.as<float>(); s1.q_stride = Dp; s1.base = ix->d_base.p; s1.nblocks = ix->NB;
      s1.pre = a.pre; s1.base8 = a.base8; s1.scale8 = a.scale8;
      s1.lcnt = s1_lcnt.as<int32_t>(); s1.lstart = s1_lstart.as<int32_t>();
      s1.rank = s1_rank.as<int32_t>(); s1.lpair = s1_lpair.as<int32_t>();
      s1.poff = s1_poff.as<int64_t>(); s1.qcnt = s1_qcnt.as<int64_t>(); s1.qoff = s1_qoff.as<int64_t>();
      s1.e1 = s1_e1.as<float>(); s1.e1_cap = e1_cap;
      return s1;
    };
    if (two_ok) {
      orders.e1_cap = e1_cap;
      // stage1_matrix 1: expanded-form sums behind their error bound (dim block 0 only; the FP8
      // pre-stage keeps the scan's arithmetic); 2: taken as they are (also the pre-stage's)
      const bool matrix = ix->stage1_matrix == 2 || (ix->stage1_matrix == 1 && !a.pre);
      orders.e1_tol = ix->stage1_matrix == 1 && !a.pre ? kE1Tol : 0.f;
      orders.stage1 = [&, matrix](bool rebuild) -> std::pair<const float *, const int64_t *> {
        const bool first = !s1_made;
        s1_made = true;
        if (first || rebuild) {
          const Stage1Args s1 = stage1_args();
          timed(ix, 4, s, [&] { launch_stage1_lists(s1, ix->store(), s, matrix); }, fixed_ws);
        }
        return {s1_e1.as<float>(), s1_qoff.as<int64_t>()};
      };
    }
    a.xcd_swizzle = ix->xcd_swizzle;
    a.nq = (int32_t)nqc; a.nblocks = ix->NB; a.block_b = ix->B; a.nlist = ix->nlist;
    a.k_max = k_max; a.lag = ix->L;
    if (lm_full) {
      const Stage1Args s1 = stage1_args();
      timed(ix, 4, s, [&] {
        launch_full_lists(s1, ix->d_xnorm.as<float>(), s1_qnorm.as<float>(), ix->store(), s);
      }, fixed_ws);
      orders.lm_e1 = s1_e1.as<float>();
      orders.lm_qoff = s1_qoff.as<int64_t>();
      orders.e1_cap = e1_cap;
    }
    choose_variant(ix, a, np_max, s, may_tune, orders);
    // callers with a fixed workspace (the allocation-free entry point, the server) keep the
    // four-wave build: the five-wave one spills to a private segment the runtime provides
    if (fixed_ws) a.occ5 = 0;
    timed(ix, 3, s, [&] { launch_scan(a, ix->store(), s); }, fixed_ws);
  }
  HIPC(hipGetLastError());
}

static void stats_from_counters(const ddc_index *ix, const int64_t *c, ddc_search_stats *st) {
  std::memset(st, 0, sizeof *st);
  st->candidates = c[0];
  st->refined = c[1];
  st->stage_slices = c[2];
  st->bytes_touched = c[2] * (int64_t)kBlockDims * ix->esize() + c[kCtrPreReads] * kFp8Lead;
  for (int i = 0; i < 64; ++i) st->stage_stop[i] = c[4 + i];
  st->prestage_reads = c[kCtrPreReads];
  st->prestage_pruned = c[kCtrPrePruned];
  st->two_phase_sums = c[3];
  st->two_phase_slices = c[kCtrSlicesSummed];
}

// ---------------------------------------------------------------------------------------
// validation helpers
// ---------------------------------------------------------------------------------------
static ddc_status check_search_args(const ddc_index *ix, int64_t nq, double alpha, ddc_corr mode) {
  if (!ix) return set_err(DDC_EINVAL, "index is NULL");
  if (nq < 0) return set_err(DDC_EINVAL, "nq must be >= 0");
  if (!(alpha >= 0.0 && alpha < 1.0)) return set_err(DDC_EINVAL, "significance must be in [0, 1)");
  if (mode != DDC_CORR_LEARNED && mode != DDC_CORR_LOSSLESS && mode != DDC_CORR_NONE &&
      mode != DDC_CORR_ADS && mode != DDC_CORR_BSAR && mode != DDC_CORR_BSAO)
    return set_err(DDC_EINVAL, "unknown correction mode %d", (int)mode);
  if (mode == DDC_CORR_BSAO && !ix->pq_tables())
    return set_err(DDC_EINVAL, "the BSA-O test needs an index with pq_m > 0 and its calibrated tables");
  if (mode == DDC_CORR_BSAR && (int)ix->lam.size() != ix->D)
    return set_err(DDC_EINVAL, "the residual test needs the rotation's eigenvalues (lam)");
  if (mode == DDC_CORR_BSAR && ix->bsar_m <= 0 && !(alpha > 0))
    return set_err(DDC_EINVAL, "the residual test with m from the significance needs significance > 0");
  if (mode == DDC_CORR_LEARNED && alpha > 0 && ix->Tt() > 0 && ix->tables.empty())
    return set_err(DDC_EINVAL, "index has no calibrated correction table (use LOSSLESS/NONE or calibrate)");
  return DDC_OK;
}

static ddc_status check_k_np(const ddc_index *ix, int k, int np) {
  if (k < 1 || k > kMaxK) return set_err(DDC_EINVAL, "k must be in [1, %d], got %d", kMaxK, k);
  if (np < 1 || np > ix->nlist) return set_err(DDC_EINVAL, "nprobe must be in [1, nlist=%d], got %d", ix->nlist, np);
  if (np > 4096) return set_err(DDC_EUNSUP, "nprobe > 4096 is not supported");
  return DDC_OK;
}

static ddc_status check_pq_shape(int M, int dim) {
  if (M < 8 || M > 128 || M % 8 || dim % M || dim / M > 32)
    return set_err(DDC_EINVAL, "pq_m must be a multiple of 8 in [8, 128] dividing dim with dim/pq_m <= 32");
  return DDC_OK;
}

static ddc_status check_params(const ddc_fit_params *p, int64_t n, int dim) {
  if (!p) return set_err(DDC_EINVAL, "params is NULL");
  if (dim < 1 || dim > kMaxBlocks * kBlockDims) return set_err(DDC_EINVAL, "dim must be in [1, 4096]");
  if (p->nlist < 1 || p->nlist > 65536) return set_err(DDC_EINVAL, "nlist must be in [1, 65536]");
  if (n < p->nlist) return set_err(DDC_EINVAL, "need n >= nlist");
  if (p->delta_d < kBlockDims || p->delta_d % kBlockDims) return set_err(DDC_EINVAL, "delta_d must be a positive multiple of 32");
  if (p->block_b < 64 || p->block_b > 1024 || p->block_b % 64) return set_err(DDC_EINVAL, "block_b must be a multiple of 64 in [64, 1024]");
  if (p->lag_l < 0 || p->lag_l > kMaxLag) return set_err(DDC_EINVAL, "lag_l must be in [0, 64]");
  if (p->kmeans_iters < 0 || p->kmeans_train_per_list < 1) return set_err(DDC_EINVAL, "bad k-means parameters");
  if (p->calib_k < 1 || p->calib_k > kMaxK) return set_err(DDC_EINVAL, "calib_k must be in [1, 256]");
  for (int i = 0, prev = p->calib_k; i < kMaxTables - 1; ++i) {
    const int e = p->calib_k_extra[i];
    if (e == 0) continue;
    if (e <= prev || e > kMaxK) return set_err(DDC_EINVAL, "calib_k_extra must ascend above calib_k, <= 256");
    if (i > 0 && p->calib_k_extra[i - 1] == 0) return set_err(DDC_EINVAL, "calib_k_extra: zeros only at the end");
    prev = e;
  }
  if (p->calib_nprobe < 0 || p->calib_nprobe > p->nlist) return set_err(DDC_EINVAL, "calib_nprobe must be in [0, nlist]");
  if (p->calib_max_neg < 1 || p->calib_max_neg > 256) return set_err(DDC_EINVAL, "calib_max_neg must be in [1, 256]");
  if (p->storage != DDC_F32 && p->storage != DDC_F16 && p->storage != DDC_BF16) return set_err(DDC_EINVAL, "bad storage");
  if (p->rotation != DDC_ROT_F32 && p->rotation != DDC_ROT_BF16) return set_err(DDC_EINVAL, "bad rotation");
  if (p->pca_sample < 2) return set_err(DDC_EINVAL, "pca_sample must be >= 2");
  if (p->projection != DDC_PROJ_PCA && p->projection != DDC_PROJ_HAAR) return set_err(DDC_EINVAL, "bad projection");
  if (p->fp8_lead_dims != 0 && p->fp8_lead_dims != kFp8Lead) return set_err(DDC_EINVAL, "fp8_lead_dims must be 0 or 64");
  if (p->fp8_lead_dims && dim < kFp8Lead) return set_err(DDC_EINVAL, "the FP8 pre-stage needs dim >= 64");
  if (p->pq_m != 0) {
    ddc_status st = check_pq_shape(p->pq_m, dim);
    if (st != DDC_OK) return st;
    if (p->projection != DDC_PROJ_PCA) return set_err(DDC_EINVAL, "the OPQ allocation needs the PCA rotation");
    if (p->pq_iters < 0 || p->pq_train < 256) return set_err(DDC_EINVAL, "pq_iters >= 0 and pq_train >= 256");
    if (n < 256) return set_err(DDC_EINVAL, "the quantization estimate needs n >= 256");
  }
  return DDC_OK;
}

static void init_sizes(ddc_index *ix, int64_t n, int D, int nlist, int dd, int B, int L, ddc_dtype st,
                       ddc_rot rot, int fp8) {
  ix->n = n; ix->D = D; ix->nlist = nlist; ix->delta_d = dd; ix->B = B; ix->L = L;
  ix->storage = st; ix->rot = rot; ix->fp8 = fp8;
  ix->NB = (D + kBlockDims - 1) / kBlockDims;
  ix->Dp = ix->NB * kBlockDims;
  ix->S = stage_count(D, dd);
  ix->St = ix->S - 1;
  (void)hipGetDevice(&ix->device);
  set_pool_retain(ix->device);
}

// ---------------------------------------------------------------------------------------
// ABI
// ---------------------------------------------------------------------------------------
// ---- index file: "DDCINDEX", version, sizes, then the artifact arrays (little-endian, as
// in memory), then a 64-bit FNV-1a checksum of everything before it --------------------------
namespace {
constexpr char kMagic[8] = {'D', 'D', 'C', 'I', 'N', 'D', 'E', 'X'};
constexpr uint32_t kFileVersion = 2;   // 2: the quantization estimate's section (1 still loads)

struct Fnv {
  uint64_t h = 1469598103934665603ull;
  void add(const void *p, size_t n) {
    const unsigned char *c = static_cast<const unsigned char *>(p);
    for (size_t i = 0; i < n; ++i) { h ^= c[i]; h *= 1099511628211ull; }
  }
};

struct Writer {
  FILE *f;
  Fnv sum;
  void put(const void *p, size_t n) {
    if (n && fwrite(p, 1, n, f) != n) throw DdcError(DDC_EIO, "write failed");
    sum.add(p, n);
  }
  template <class T> void val(T v) { put(&v, sizeof v); }
};

struct Reader {
  FILE *f;
  Fnv sum;
  void get(void *p, size_t n) {
    if (n && fread(p, 1, n, f) != n) throw DdcError(DDC_EIO, "file truncated");
    sum.add(p, n);
  }
  template <class T> T val() { T v; get(&v, sizeof v); return v; }
};

struct FileCloser { FILE *f; ~FileCloser() { if (f) fclose(f); } };
}  // namespace

extern "C" {

const char *ddc_last_error(void) { return g_err.c_str(); }

ddc_status ddc_fit_params_default(ddc_fit_params *p) {
  if (!p) return set_err(DDC_EINVAL, "params is NULL");
  std::memset(p, 0, sizeof *p);
  p->nlist = 4096; p->delta_d = 32; p->block_b = 256; p->lag_l = 0;
  p->kmeans_iters = 25; p->kmeans_train_per_list = 256;
  p->calib_k = 10; p->calib_nprobe = 0; p->calib_max_neg = 50;
  p->storage = DDC_F32; p->rotation = DDC_ROT_F32;
  p->pca_sample = 1000000; p->seed = 0;
  p->pq_m = 0; p->pq_iters = 25; p->pq_train = 65536;
  return DDC_OK;
}

void ddc_free(ddc_index *ix) {
  if (!ix) return;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(ix->device);
  delete ix;
  (void)hipSetDevice(prev);
}

ddc_status ddc_index_get_info(const ddc_index *ix, ddc_index_info *info) {
  if (!ix || !info) return set_err(DDC_EINVAL, "NULL argument");
  std::memset(info, 0, sizeof *info);
  info->n = ix->n; info->dim = ix->D; info->dim_padded = ix->Dp; info->nlist = ix->nlist;
  info->delta_d = ix->delta_d; info->n_stages = ix->S; info->n_test_stages = ix->Tt();
  info->fp8_lead_dims = ix->fp8;
  info->block_b = ix->B; info->lag_l = ix->L; info->storage = ix->storage; info->rotation = ix->rot;
  info->n0 = ix->n0_total(); info->packed_bytes = (int64_t)ix->d_base.bytes; info->total_tiles = ix->total_tiles;
  info->n_tables = (int32_t)ix->tables.size();
  for (size_t t = 0; t < ix->tables.size(); ++t) info->table_k[t] = ix->tables[t].kc;
  info->pq_m = ix->pq_m;
  info->pq_tables = ix->pq_tables() ? 1 : 0;
  return DDC_OK;
}

ddc_status ddc_import(const ddc_artifacts *a, ddc_index **out) {
  if (!out) return set_err(DDC_EINVAL, "out is NULL");
  *out = nullptr;
  if (!a) return set_err(DDC_EINVAL, "artifacts is NULL");
  if (a->n < 1 || a->dim < 1 || a->dim > kMaxBlocks * kBlockDims) return set_err(DDC_EINVAL, "bad n/dim");
  if (a->nlist < 1 || a->nlist > 65536) return set_err(DDC_EINVAL, "nlist must be in [1, 65536]");
  if (a->delta_d < kBlockDims || a->delta_d % kBlockDims) return set_err(DDC_EINVAL, "delta_d must be a positive multiple of 32");
  if (a->block_b < 64 || a->block_b > 1024 || a->block_b % 64) return set_err(DDC_EINVAL, "block_b must be a multiple of 64 in [64, 1024]");
  if (a->lag_l < 0 || a->lag_l > kMaxLag) return set_err(DDC_EINVAL, "lag_l must be in [0, 64]");
  if (a->storage != DDC_F32 && a->storage != DDC_F16 && a->storage != DDC_BF16) return set_err(DDC_EINVAL, "bad storage");
  if (a->rotation != DDC_ROT_F32 && a->rotation != DDC_ROT_BF16) return set_err(DDC_EINVAL, "bad rotation");
  if (!a->mu || !a->rot || !a->centroids || !a->assign || !a->y) return set_err(DDC_EINVAL, "missing artifact array");
  if (a->fp8_lead_dims != 0 && a->fp8_lead_dims != kFp8Lead) return set_err(DDC_EINVAL, "fp8_lead_dims must be 0 or 64");
  if (a->fp8_lead_dims && a->dim < kFp8Lead) return set_err(DDC_EINVAL, "the FP8 pre-stage needs dim >= 64");
  const int D = a->dim;
  const int Tt = stage_count(D, a->delta_d) - 1 + (a->fp8_lead_dims ? 1 : 0);
  if (a->n_tables < 0 || a->n_tables > kMaxTables) return set_err(DDC_EINVAL, "n_tables must be in [0, 4]");
  for (int t = 0; t < a->n_tables; ++t) {
    if (a->table_n0[t] < 1 || a->table_k[t] < 1 || (t > 0 && a->table_k[t] <= a->table_k[t - 1]))
      return set_err(DDC_EINVAL, "bad correction table %d (n0 >= 1, K_c ascending)", t);
  }
  if (a->n_tables > 0 && (!a->m || !a->resid)) return set_err(DDC_EINVAL, "missing m/resid");
  if (a->pq_m != 0) {
    ddc_status st = check_pq_shape(a->pq_m, a->dim);
    if (st != DDC_OK) return st;
    if (!a->pq_perm || !a->pq_books) return set_err(DDC_EINVAL, "missing pq_perm/pq_books");
    std::vector<int> seen(a->dim, 0);
    for (int i = 0; i < a->dim; ++i) {
      const int v = a->pq_perm[i];
      if (v < 0 || v >= a->dim || seen[v]++) return set_err(DDC_EINVAL, "pq_perm is not a permutation of the axes");
    }
    if (!all_finite(a->pq_books, (int64_t)a->pq_m * 256 * (a->dim / a->pq_m)))
      return set_err(DDC_EINVAL, "non-finite codewords");
    if (a->n_tables > 0 && (!a->pq_m1) != (!a->pq_resid)) return set_err(DDC_EINVAL, "pq_m1/pq_m3/pq_resid: all or none");
    if (a->pq_m1 && !a->pq_m3) return set_err(DDC_EINVAL, "pq_m1/pq_m3/pq_resid: all or none");
  }
  for (int64_t i = 0; i < a->n; ++i)
    if (a->assign[i] < 0 || a->assign[i] >= a->nlist) return set_err(DDC_EINVAL, "assign out of range at %lld", (long long)i);
  if (!all_finite(a->y, a->n * D) || !all_finite(a->centroids, (int64_t)a->nlist * D))
    return set_err(DDC_EINVAL, "non-finite values in y or centroids");
  GUARD_BEGIN
  std::unique_ptr<ddc_index> ix(new ddc_index);
  init_sizes(ix.get(), a->n, D, a->nlist, a->delta_d, a->block_b, a->lag_l, a->storage, a->rotation,
             a->fp8_lead_dims);
  ix->mu.assign(a->mu, a->mu + D);
  ix->R.assign(a->rot, a->rot + (size_t)D * D);
  if (a->lam) ix->lam.assign(a->lam, a->lam + D);
  ix->cent.assign(a->centroids, a->centroids + (size_t)a->nlist * D);
  ix->assign.assign(a->assign, a->assign + a->n);
  {
    std::vector<ddc_index::Table> tabs(a->n_tables);
    size_t roff = 0;
    for (int t = 0; t < a->n_tables; ++t) {
      tabs[t].kc = a->table_k[t];
      tabs[t].n0 = a->table_n0[t];
      tabs[t].m.assign(a->m + (size_t)t * Tt, a->m + (size_t)(t + 1) * Tt);
      tabs[t].resid.assign(a->resid + roff * Tt, a->resid + (roff + a->table_n0[t]) * Tt);
      if (a->pq_m && a->pq_m1) {
        tabs[t].pq_m1 = a->pq_m1[t];
        tabs[t].pq_m3 = a->pq_m3[t];
        tabs[t].pq_resid.assign(a->pq_resid + roff, a->pq_resid + roff + a->table_n0[t]);
      }
      roff += a->table_n0[t];
    }
    set_tables(ix.get(), std::move(tabs));
  }
  if (a->pq_m) {
    ix->pq_m = a->pq_m;
    ix->pq_dsub = D / a->pq_m;
    ix->pq_perm.assign(a->pq_perm, a->pq_perm + D);
    ix->pq_books.assign(a->pq_books, a->pq_books + (size_t)a->pq_m * 256 * ix->pq_dsub);
  }
  StreamHolder sh;
  DevBuf d_Y((size_t)a->n * ix->Dp * 4);
  HIPC(hipMemset2DAsync(d_Y.p, ix->Dp * 4, 0, ix->Dp * 4, a->n, sh.s));
  HIPC(hipMemcpy2DAsync(d_Y.p, ix->Dp * 4, a->y, D * 4, D * 4, a->n, hipMemcpyHostToDevice, sh.s));
  launch_round_storage(d_Y.as<float>(), a->n * ix->Dp, ix->store(), sh.s);
  upload_index(ix.get(), d_Y.as<float>(), sh.s);
  if (ix->pq_m) pq_upload_encode(ix.get(), sh.s);
  *out = ix.release();
  return DDC_OK;
  GUARD_END
}

ddc_status ddc_export(const ddc_index *ixc, ddc_artifacts *a) {
  if (!ixc || !a) return set_err(DDC_EINVAL, "NULL argument");
  ddc_index *ix = const_cast<ddc_index *>(ixc);
  if (!a->mu || !a->rot || !a->centroids || !a->assign) return set_err(DDC_EINVAL, "missing output array");
  if (!ix->tables.empty() && (!a->m || !a->resid)) return set_err(DDC_EINVAL, "missing m/resid output");
  GUARD_BEGIN
  DeviceGuard dg(ix->device);
  const int D = ix->D;
  a->n = ix->n; a->dim = D; a->nlist = ix->nlist; a->delta_d = ix->delta_d; a->block_b = ix->B;
  a->lag_l = ix->L; a->storage = ix->storage; a->rotation = ix->rot;
  a->n_tables = (int32_t)ix->tables.size();
  a->fp8_lead_dims = ix->fp8;
  if (ix->fp8 && (a->codes8 || a->scale8)) {
    std::vector<uint8_t> c8((size_t)ix->total_tiles * kTile * kFp8Lead);
    std::vector<float> s8(ix->total_tiles);
    HIPC(hipMemcpy(c8.data(), ix->d_base8.p, c8.size(), hipMemcpyDeviceToHost));
    HIPC(hipMemcpy(s8.data(), ix->d_scale8.p, s8.size() * 4, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < ix->n; ++i) {
      const int64_t slot = ix->id_to_slot[i];
      if (a->codes8) std::memcpy(a->codes8 + (size_t)i * kFp8Lead, &c8[(size_t)slot * kFp8Lead], kFp8Lead);
      if (a->scale8) a->scale8[i] = s8[slot / kTile];
    }
  }
  a->pq_m = ix->pq_m;
  if (ix->pq_m) {
    if (a->pq_perm) std::copy(ix->pq_perm.begin(), ix->pq_perm.end(), a->pq_perm);
    if (a->pq_books) std::copy(ix->pq_books.begin(), ix->pq_books.end(), a->pq_books);
    if (a->pq_codes) {
      const int M = ix->pq_m;
      std::vector<uint8_t> c((size_t)ix->total_tiles * kTile * M);
      HIPC(hipMemcpy(c.data(), ix->d_pq_codes.p, c.size(), hipMemcpyDeviceToHost));
      for (int64_t i = 0; i < ix->n; ++i)
        std::memcpy(a->pq_codes + (size_t)i * M, &c[(size_t)ix->id_to_slot[i] * M], M);
    }
    if (ix->pq_tables() && a->pq_m1 && a->pq_m3 && a->pq_resid) {
      size_t roff = 0;
      for (size_t t = 0; t < ix->tables.size(); ++t) {
        const auto &tb = ix->tables[t];
        a->pq_m1[t] = tb.pq_m1;
        a->pq_m3[t] = tb.pq_m3;
        std::copy(tb.pq_resid.begin(), tb.pq_resid.end(), a->pq_resid + roff);
        roff += (size_t)tb.n0;
      }
    }
  }
  std::copy(ix->mu.begin(), ix->mu.end(), a->mu);
  std::copy(ix->R.begin(), ix->R.end(), a->rot);
  if (a->lam && !ix->lam.empty()) std::copy(ix->lam.begin(), ix->lam.end(), a->lam);
  std::copy(ix->cent.begin(), ix->cent.end(), a->centroids);
  std::copy(ix->assign.begin(), ix->assign.end(), a->assign);
  {
    size_t roff = 0;
    for (size_t t = 0; t < ix->tables.size(); ++t) {
      const auto &tb = ix->tables[t];
      a->table_k[t] = tb.kc;
      a->table_n0[t] = tb.n0;
      std::copy(tb.m.begin(), tb.m.end(), a->m + t * ix->Tt());
      std::copy(tb.resid.begin(), tb.resid.end(), a->resid + roff * ix->Tt());
      roff += (size_t)tb.n0;
    }
  }
  if (a->y) {
    const size_t per = (size_t)ix->NB * kTile * kBlockDims;
    std::vector<unsigned char> packed(ix->d_base.bytes);
    HIPC(hipMemcpy(packed.data(), ix->d_base.p, packed.size(), hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < ix->n; ++i) {
      const int64_t slot = ix->id_to_slot[i];
      const int64_t tile = slot / kTile;
      const int v = (int)(slot % kTile);
      for (int d = 0; d < D; ++d) {
        const size_t idx = tile * per + ((size_t)(d / kBlockDims) * kTile + v) * kBlockDims + d % kBlockDims;
        float x;
        if (ix->storage == DDC_F32) {
          std::memcpy(&x, &packed[idx * 4], 4);
        } else {
          uint16_t h;
          std::memcpy(&h, &packed[idx * 2], 2);
          if (ix->storage == DDC_BF16) {
            const uint32_t u = (uint32_t)h << 16;
            std::memcpy(&x, &u, 4);
          } else {
            // IEEE binary16 -> binary32
            const uint32_t sgn = (uint32_t)(h >> 15) << 31, ex = (h >> 10) & 31, man = h & 1023;
            uint32_t u;
            if (ex == 0) {
              if (man == 0) u = sgn;
              else {
                int e = -1;
                uint32_t mm = man;
                do { ++e; mm <<= 1; } while (!(mm & 1024));
                u = sgn | ((uint32_t)(127 - 15 - e) << 23) | ((mm & 1023) << 13);
              }
            } else if (ex == 31) u = sgn | 0x7F800000u | (man << 13);
            else u = sgn | ((ex + 112) << 23) | (man << 13);
            std::memcpy(&x, &u, 4);
          }
        }
        a->y[(size_t)i * D + d] = x;
      }
    }
  }
  return DDC_OK;
  GUARD_END
}


ddc_status ddc_save(const ddc_index *ixc, const char *path) {
  if (!ixc || !path) return set_err(DDC_EINVAL, "NULL argument");
  GUARD_BEGIN
  ddc_index *ix = const_cast<ddc_index *>(ixc);
  const int D = ix->D, T = ix->Tt();
  const int64_t n = ix->n, n0 = ix->n0_total();
  const int nt = (int)ix->tables.size();
  std::vector<double> mu(D), R((size_t)D * D), lam(D), m((size_t)std::max(nt, 1) * T), resid((size_t)n0 * T);
  std::vector<float> cent((size_t)ix->nlist * D), y((size_t)n * D);
  std::vector<int32_t> assign(n);
  ddc_artifacts a{};
  a.mu = mu.data(); a.rot = R.data(); a.lam = lam.data(); a.centroids = cent.data();
  a.assign = assign.data(); a.y = y.data(); a.m = m.data(); a.resid = resid.data();
  const ddc_status st = ddc_export(ixc, &a);
  if (st != DDC_OK) return st;
  FileCloser fc{fopen(path, "wb")};
  if (!fc.f) return set_err(DDC_EIO, "cannot open %s for writing", path);
  Writer w{fc.f};
  w.put(kMagic, 8);
  w.val<uint32_t>(kFileVersion);
  w.val<int64_t>(n);
  for (int32_t v : {D, ix->nlist, ix->delta_d, ix->B, ix->L, (int32_t)ix->storage, (int32_t)ix->rot, ix->fp8, nt})
    w.val<int32_t>(v);
  for (int t = 0; t < kMaxTables; ++t) w.val<int32_t>(t < nt ? a.table_k[t] : 0);
  for (int t = 0; t < kMaxTables; ++t) w.val<int64_t>(t < nt ? a.table_n0[t] : 0);
  const uint8_t has_lam = ix->lam.empty() ? 0 : 1;
  w.val<uint8_t>(has_lam);
  w.put(mu.data(), mu.size() * 8);
  w.put(R.data(), R.size() * 8);
  if (has_lam) w.put(lam.data(), lam.size() * 8);
  w.put(cent.data(), cent.size() * 4);
  w.put(assign.data(), assign.size() * 4);
  w.put(y.data(), y.size() * 4);
  w.put(m.data(), (size_t)nt * T * 8);
  w.put(resid.data(), resid.size() * 8);
  // quantization estimate: M, then axes, codewords and (when calibrated) each table's classifier
  w.val<int32_t>(ix->pq_m);
  if (ix->pq_m) {
    const uint8_t has_pq_tab = ix->pq_tables() ? 1 : 0;
    w.val<uint8_t>(has_pq_tab);
    w.put(ix->pq_perm.data(), ix->pq_perm.size() * 4);
    w.put(ix->pq_books.data(), ix->pq_books.size() * 4);
    if (has_pq_tab)
      for (const auto &tb : ix->tables) {
        w.val<double>(tb.pq_m1);
        w.val<double>(tb.pq_m3);
        w.put(tb.pq_resid.data(), tb.pq_resid.size() * 8);
      }
  }
  const uint64_t h = w.sum.h;
  if (fwrite(&h, 1, 8, fc.f) != 8) throw DdcError(DDC_EIO, "write failed");
  if (fflush(fc.f) != 0) throw DdcError(DDC_EIO, "write failed");
  return DDC_OK;
  GUARD_END
}

ddc_status ddc_load(const char *path, ddc_index **out) {
  if (!out) return set_err(DDC_EINVAL, "out is NULL");
  *out = nullptr;
  if (!path) return set_err(DDC_EINVAL, "path is NULL");
  GUARD_BEGIN
  FileCloser fc{fopen(path, "rb")};
  if (!fc.f) return set_err(DDC_EIO, "cannot open %s", path);
  Reader r{fc.f};
  char magic[8];
  r.get(magic, 8);
  if (std::memcmp(magic, kMagic, 8) != 0) return set_err(DDC_EIO, "%s is not an index file", path);
  const uint32_t version = r.val<uint32_t>();
  if (version != 1 && version != kFileVersion) return set_err(DDC_EIO, "unsupported index file version");
  ddc_artifacts a{};
  a.n = r.val<int64_t>();
  a.dim = r.val<int32_t>(); a.nlist = r.val<int32_t>(); a.delta_d = r.val<int32_t>();
  a.block_b = r.val<int32_t>(); a.lag_l = r.val<int32_t>();
  a.storage = (ddc_dtype)r.val<int32_t>(); a.rotation = (ddc_rot)r.val<int32_t>();
  a.fp8_lead_dims = r.val<int32_t>(); a.n_tables = r.val<int32_t>();
  for (int t = 0; t < kMaxTables; ++t) a.table_k[t] = r.val<int32_t>();
  int64_t n0 = 0;
  for (int t = 0; t < kMaxTables; ++t) { a.table_n0[t] = r.val<int64_t>(); n0 += a.table_n0[t]; }
  // sizes are checked before any allocation they decide
  if (a.n < 1 || a.n > (int64_t(1) << 40) || a.dim < 1 || a.dim > kMaxBlocks * kBlockDims ||
      a.nlist < 1 || a.nlist > 65536 || a.delta_d < kBlockDims || a.n_tables < 0 ||
      a.n_tables > kMaxTables || n0 < 0 || n0 > (int64_t(1) << 36))
    return set_err(DDC_EIO, "corrupt index file header");
  const int D = a.dim;
  const int T = (D + a.delta_d - 1) / a.delta_d - 1 + (a.fp8_lead_dims ? 1 : 0);
  const uint8_t has_lam = r.val<uint8_t>();
  std::vector<double> mu(D), R((size_t)D * D), lam(has_lam ? D : 0), m((size_t)a.n_tables * T),
      resid((size_t)n0 * T);
  std::vector<float> cent((size_t)a.nlist * D), y((size_t)a.n * D);
  std::vector<int32_t> assign(a.n);
  r.get(mu.data(), mu.size() * 8);
  r.get(R.data(), R.size() * 8);
  if (has_lam) r.get(lam.data(), lam.size() * 8);
  r.get(cent.data(), cent.size() * 4);
  r.get(assign.data(), assign.size() * 4);
  r.get(y.data(), y.size() * 4);
  r.get(m.data(), m.size() * 8);
  r.get(resid.data(), resid.size() * 8);
  std::vector<int32_t> pq_perm;
  std::vector<float> pq_books;
  std::vector<double> pq_m1, pq_m3, pq_resid;
  if (version >= 2) {
    a.pq_m = r.val<int32_t>();
    if (a.pq_m) {
      if (a.pq_m < 1 || a.pq_m > 128 || D % a.pq_m) return set_err(DDC_EIO, "corrupt index file (pq section)");
      const uint8_t has_pq_tab = r.val<uint8_t>();
      pq_perm.resize(D);
      pq_books.resize((size_t)a.pq_m * 256 * (D / a.pq_m));
      r.get(pq_perm.data(), pq_perm.size() * 4);
      r.get(pq_books.data(), pq_books.size() * 4);
      if (has_pq_tab) {
        pq_m1.resize(a.n_tables);
        pq_m3.resize(a.n_tables);
        pq_resid.resize(n0);
        size_t roff = 0;
        for (int t = 0; t < a.n_tables; ++t) {
          pq_m1[t] = r.val<double>();
          pq_m3[t] = r.val<double>();
          r.get(pq_resid.data() + roff, (size_t)a.table_n0[t] * 8);
          roff += (size_t)a.table_n0[t];
        }
        a.pq_m1 = pq_m1.data(); a.pq_m3 = pq_m3.data(); a.pq_resid = pq_resid.data();
      }
      a.pq_perm = pq_perm.data(); a.pq_books = pq_books.data();
    }
  }
  const uint64_t want = r.sum.h;
  uint64_t got = 0;
  if (fread(&got, 1, 8, fc.f) != 8 || got != want) return set_err(DDC_EIO, "index file checksum mismatch");
  a.mu = mu.data(); a.rot = R.data(); a.lam = has_lam ? lam.data() : nullptr; a.centroids = cent.data();
  a.assign = assign.data(); a.y = y.data(); a.m = m.data(); a.resid = resid.data();
  return ddc_import(&a, out);
  GUARD_END
}

ddc_status ddc_correction_pq(const ddc_index *ixc, int32_t k, double alpha, double *m1, double *m3,
                             double *beta) {
  if (!ixc || !m1 || !m3 || !beta) return set_err(DDC_EINVAL, "NULL argument");
  if (!(alpha >= 0.0 && alpha < 1.0)) return set_err(DDC_EINVAL, "significance must be in [0, 1)");
  if (k < 1 || k > kMaxK) return set_err(DDC_EINVAL, "k must be in [1, %d]", kMaxK);
  if (!ixc->pq_tables()) return set_err(DDC_EINVAL, "index has no BSA-O table");
  GUARD_BEGIN
  const auto &tb = ixc->tables[table_for_k(ixc, k)];
  *m1 = tb.pq_m1;
  *m3 = tb.pq_m3;
  *beta = beta_for_alpha(tb.pq_resid, tb.n0, 1, alpha, 0)[0];
  return DDC_OK;
  GUARD_END
}

ddc_status ddc_correction(const ddc_index *ixc, int32_t k, double alpha, ddc_calib_mode mode,
                          double *m_out, double *beta_out) {
  if (!ixc || !m_out || !beta_out) return set_err(DDC_EINVAL, "NULL argument");
  if (!(alpha >= 0.0 && alpha < 1.0)) return set_err(DDC_EINVAL, "significance must be in [0, 1)");
  if (mode != DDC_CALIB_JOINT && mode != DDC_CALIB_BONFERRONI) return set_err(DDC_EINVAL, "bad calibration mode");
  if (k < 1 || k > kMaxK) return set_err(DDC_EINVAL, "k must be in [1, %d]", kMaxK);
  if (ixc->tables.empty()) return set_err(DDC_EINVAL, "index has no correction table");
  GUARD_BEGIN
  ddc_index *ix = const_cast<ddc_index *>(ixc);
  const int t = table_for_k(ix, k);
  auto b = get_beta(ix, alpha, mode, t);
  for (int j = 0; j < ix->Tt(); ++j) { m_out[j] = ix->tables[t].m[j]; beta_out[j] = b[j]; }
  return DDC_OK;
  GUARD_END
}

ddc_status ddc_search_device(const ddc_index *ixc, const float *d_queries, int64_t nq,
                             const int32_t *d_k, int32_t k_all, int32_t k_max,
                             const int32_t *d_nprobe, int32_t nprobe_all, int32_t nprobe_max,
                             double significance, ddc_corr mode, const int64_t *d_out_offsets,
                             int64_t *d_ids, float *d_dists, int64_t *d_counters, void *hip_stream) {
  ddc_status st = check_device_search(ixc, d_queries, nq, d_k, k_all, k_max, d_nprobe, nprobe_all,
                                      nprobe_max, significance, mode, d_out_offsets, d_ids, d_dists);
  if (st != DDC_OK) return st;
  if (nq == 0) return DDC_OK;
  GUARD_BEGIN
  ddc_index *ix = const_cast<ddc_index *>(ixc);
  DeviceGuard dg(ix->device);
  search_device(ix, d_queries, nq, d_k, k_all, d_k ? k_max : k_all, d_nprobe, nprobe_all,
                d_nprobe ? nprobe_max : nprobe_all, significance, mode, d_out_offsets, d_ids,
                d_dists, d_counters, reinterpret_cast<hipStream_t>(hip_stream), nullptr, nullptr,
                true, nullptr, /*stream_scratch=*/true);
  return DDC_OK;
  GUARD_END
}

static ddc_status search_host(const ddc_index *ixc, const float *queries, int64_t nq,
                              const int32_t *k, int32_t k_all, const int32_t *np, int32_t np_all,
                              double alpha, ddc_corr mode, const int64_t *offs, int64_t *ids,
                              float *dists, ddc_search_stats *stats) {
  ddc_index *ix = const_cast<ddc_index *>(ixc);
  int kmax = k_all, npmax = np_all;
  int64_t total = nq * (int64_t)k_all;
  if (k) {
    kmax = 0;
    npmax = 0;
    for (int64_t i = 0; i < nq; ++i) {
      ddc_status st = check_k_np(ix, k[i], np[i]);
      if (st != DDC_OK) return st;
      if (offs[i + 1] - offs[i] < k[i] || offs[i] < 0) return set_err(DDC_EINVAL, "out_offsets too small for k at %lld", (long long)i);
      kmax = std::max(kmax, k[i]);
      npmax = std::max(npmax, np[i]);
    }
    total = offs[nq];
  }
  if (!all_finite(queries, nq * ix->D)) return set_err(DDC_EINVAL, "non-finite query values");
  if (nq == 0) {
    if (stats) std::memset(stats, 0, sizeof *stats);
    return DDC_OK;
  }
  GUARD_BEGIN
  DeviceGuard dg(ix->device);
  StreamHolder sh;
  DevBuf d_q((size_t)nq * ix->D * 4), d_ids(total * 8), d_d(total * 4), d_ctr(kMaxCounters * 8);
  DevBuf d_k, d_np, d_off;
  HIPC(hipMemcpyAsync(d_q.p, queries, (size_t)nq * ix->D * 4, hipMemcpyHostToDevice, sh.s));
  HIPC(hipMemsetAsync(d_ctr.p, 0, kMaxCounters * 8, sh.s));
  if (k) {
    d_k.alloc(nq * 4); d_np.alloc(nq * 4); d_off.alloc((nq + 1) * 8);
    HIPC(hipMemcpyAsync(d_k.p, k, nq * 4, hipMemcpyHostToDevice, sh.s));
    HIPC(hipMemcpyAsync(d_np.p, np, nq * 4, hipMemcpyHostToDevice, sh.s));
    HIPC(hipMemcpyAsync(d_off.p, offs, (nq + 1) * 8, hipMemcpyHostToDevice, sh.s));
  }
  // slots of the CSR not covered by any query's k keep the padding values
  if (k) {
    std::vector<int64_t> pad_i(total, -1);
    std::vector<float> pad_d(total, INFINITY);
    HIPC(hipMemcpyAsync(d_ids.p, pad_i.data(), total * 8, hipMemcpyHostToDevice, sh.s));
    HIPC(hipMemcpyAsync(d_d.p, pad_d.data(), total * 4, hipMemcpyHostToDevice, sh.s));
    HIPC(hipStreamSynchronize(sh.s));
  }
  search_device(ix, d_q.as<float>(), nq, k ? d_k.as<int32_t>() : nullptr, k_all, kmax,
                k ? d_np.as<int32_t>() : nullptr, np_all, npmax, alpha, mode,
                k ? d_off.as<int64_t>() : nullptr, d_ids.as<int64_t>(), d_d.as<float>(),
                d_ctr.as<int64_t>(), sh.s);
  HIPC(hipMemcpyAsync(ids, d_ids.p, total * 8, hipMemcpyDeviceToHost, sh.s));
  HIPC(hipMemcpyAsync(dists, d_d.p, total * 4, hipMemcpyDeviceToHost, sh.s));
  int64_t ctr[kMaxCounters];
  HIPC(hipMemcpyAsync(ctr, d_ctr.p, sizeof ctr, hipMemcpyDeviceToHost, sh.s));
  HIPC(hipStreamSynchronize(sh.s));
  if (stats) stats_from_counters(ix, ctr, stats);
  return DDC_OK;
  GUARD_END
}

ddc_status ddc_search(const ddc_index *ix, const float *queries, int64_t nq, int32_t k, int32_t nprobe,
                      double significance, ddc_corr mode, int64_t *ids, float *dists,
                      ddc_search_stats *stats) {
  ddc_status st = check_search_args(ix, nq, significance, mode);
  if (st != DDC_OK) return st;
  if ((st = check_k_np(ix, k, nprobe)) != DDC_OK) return st;
  if (nq > 0 && (!queries || !ids || !dists)) return set_err(DDC_EINVAL, "NULL buffer");
  return search_host(ix, queries, nq, nullptr, k, nullptr, nprobe, significance, mode, nullptr, ids,
                     dists, stats);
}

ddc_status ddc_search_estimate(const ddc_index *ixc, const float *queries, int64_t nq, int32_t k,
                               int32_t nprobe, int32_t dims, ddc_estimator estimator, int64_t *ids,
                               float *dists) {
  if (!ixc) return set_err(DDC_EINVAL, "index is NULL");
  ddc_status st = check_k_np(ixc, k, nprobe);
  if (st != DDC_OK) return st;
  if (dims < kBlockDims || dims % kBlockDims || dims > ixc->Dp)
    return set_err(DDC_EINVAL, "dims must be a multiple of 32 in [32, %d], got %d", ixc->Dp, dims);
  if (estimator != DDC_EST_PARTIAL && estimator != DDC_EST_RESIDUAL)
    return set_err(DDC_EINVAL, "unknown estimator %d", (int)estimator);
  if (nq < 0 || (nq > 0 && (!queries || !ids || !dists))) return set_err(DDC_EINVAL, "bad buffers");
  if (!all_finite(queries, nq * ixc->D)) return set_err(DDC_EINVAL, "non-finite query values");
  if (nq == 0) return DDC_OK;
  GUARD_BEGIN
  ddc_index *ix = const_cast<ddc_index *>(ixc);
  DeviceGuard dg(ix->device);
  StreamHolder sh;
  EstimateSpec es{dims / kBlockDims, estimator == DDC_EST_RESIDUAL ? 1 : 0,
                  (float)((double)ix->D / std::min(dims, ix->D))};
  DevBuf d_q((size_t)nq * ix->D * 4), d_ids((size_t)nq * k * 8), d_d((size_t)nq * k * 4);
  HIPC(hipMemcpyAsync(d_q.p, queries, (size_t)nq * ix->D * 4, hipMemcpyHostToDevice, sh.s));
  search_device(ix, d_q.as<float>(), nq, nullptr, k, k, nullptr, nprobe, nprobe, 0.0, DDC_CORR_NONE,
                nullptr, d_ids.as<int64_t>(), d_d.as<float>(), nullptr, sh.s, nullptr, nullptr, true,
                &es);
  HIPC(hipMemcpyAsync(ids, d_ids.p, (size_t)nq * k * 8, hipMemcpyDeviceToHost, sh.s));
  HIPC(hipMemcpyAsync(dists, d_d.p, (size_t)nq * k * 4, hipMemcpyDeviceToHost, sh.s));
  HIPC(hipStreamSynchronize(sh.s));
  return DDC_OK;
  GUARD_END
}

ddc_status ddc_search_var(const ddc_index *ix, const float *queries, int64_t nq, const int32_t *k,
                          const int32_t *nprobe, double significance, ddc_corr mode,
                          const int64_t *out_offsets, int64_t *ids, float *dists,
                          ddc_search_stats *stats) {
  ddc_status st = check_search_args(ix, nq, significance, mode);
  if (st != DDC_OK) return st;
  if (nq > 0 && (!queries || !k || !nprobe || !out_offsets || !ids || !dists))
    return set_err(DDC_EINVAL, "NULL buffer");
  return search_host(ix, queries, nq, k, 0, nprobe, 0, significance, mode, out_offsets, ids, dists,
                     stats);
}

ddc_status ddc_debug_intermediates(const ddc_index *ixc, const float *queries, int64_t nq,
                                   int32_t nprobe, float *q_rot, int32_t *probes) {
  if (!ixc) return set_err(DDC_EINVAL, "index is NULL");
  ddc_status st = check_k_np(ixc, 1, nprobe);
  if (st != DDC_OK) return st;
  if (nq < 0 || (nq > 0 && (!queries || !q_rot || !probes))) return set_err(DDC_EINVAL, "bad buffers");
  if (!all_finite(queries, nq * ixc->D)) return set_err(DDC_EINVAL, "non-finite query values");
  if (nq == 0) return DDC_OK;
  GUARD_BEGIN
  ddc_index *ix = const_cast<ddc_index *>(ixc);
  DeviceGuard dg(ix->device);
  StreamHolder sh;
  DevBuf d_q((size_t)nq * ix->D * 4);
  HIPC(hipMemcpyAsync(d_q.p, queries, (size_t)nq * ix->D * 4, hipMemcpyHostToDevice, sh.s));
  search_device(ix, d_q.as<float>(), nq, nullptr, 1, 1, nullptr, nprobe, nprobe, 0.0, DDC_CORR_NONE,
                nullptr, nullptr, nullptr, nullptr, sh.s, q_rot, probes);
  HIPC(hipStreamSynchronize(sh.s));
  return DDC_OK;
  GUARD_END
}

ddc_status ddc_live_allocations(int64_t *count, int64_t *bytes) {
  if (!count || !bytes) return set_err(DDC_EINVAL, "NULL argument");
  *count = g_live_count.load();
  *bytes = g_live_bytes.load();
  return DDC_OK;
}

ddc_status ddc_set_fault(const char *spec) {
  int64_t n = 0;
  if (!parse_fault(spec, &n)) return set_err(DDC_EINVAL, "fault spec must be \"alloc:<n>\" with n >= 0");
  fault_env_once();
  g_fault_at = 0;
  g_fault_seen = 0;
  g_fault_at = n;
  return DDC_OK;
}

ddc_status ddc_set_kernel_timing(ddc_index *ix, int enable) {
  if (!ix) return set_err(DDC_EINVAL, "index is NULL");
  std::lock_guard<std::mutex> lk(ix->timing_mtx);
  ix->timing = enable != 0;
  return DDC_OK;
}

ddc_status ddc_get_kernel_timing(ddc_index *ix, double *ms_total, int64_t *launches, int reset) {
  if (!ix || !ms_total || !launches) return set_err(DDC_EINVAL, "NULL argument");
  GUARD_BEGIN
  DeviceGuard dg(ix->device);
  std::lock_guard<std::mutex> lk(ix->timing_mtx);
  for (int i = 0; i < 5; ++i) { ms_total[i] = 0.0; launches[i] = 0; }
  for (auto &m : ix->marks) {
    HIPC(hipEventSynchronize(m.b));
    float ms = 0.f;
    HIPC(hipEventElapsedTime(&ms, m.a, m.b));
    ms_total[m.kernel] += ms;
    launches[m.kernel] += 1;
  }
  if (reset) {
    for (auto &m : ix->marks) { (void)hipEventDestroy(m.a); (void)hipEventDestroy(m.b); }
    ix->marks.clear();
  }
  return DDC_OK;
  GUARD_END
}

ddc_status ddc_set_bsar_multiplier(ddc_index *ix, double m) {
  if (!ix) return set_err(DDC_EINVAL, "index is NULL");
  if (!std::isfinite(m)) return set_err(DDC_EINVAL, "m must be finite");
  ix->bsar_m = m;
  return DDC_OK;
}

ddc_status ddc_set_ads_epsilon(ddc_index *ix, double eps0) {
  if (!ix) return set_err(DDC_EINVAL, "index is NULL");
  if (!(eps0 > 0.0) || !std::isfinite(eps0)) return set_err(DDC_EINVAL, "eps0 must be > 0");
  std::lock_guard<std::mutex> lk(ix->beta_mtx);
  ix->ads_eps0 = eps0;
  return DDC_OK;
}

ddc_status ddc_set_launch(ddc_index *ix, const ddc_launch_params *p) {
  if (!ix || !p) return set_err(DDC_EINVAL, "NULL argument");
  if (p->waves_per_query != 0 && p->waves_per_query != 1 && p->waves_per_query != 2 &&
      p->waves_per_query != 4)
    return set_err(DDC_EINVAL, "waves_per_query must be 0, 1, 2 or 4");
  if (p->lookahead < -1 || p->lookahead > 1) return set_err(DDC_EINVAL, "lookahead must be -1, 0 or 1");
  if ((p->query_order != 0 && p->query_order != 1) || (p->xcd_swizzle != 0 && p->xcd_swizzle != 1))
    return set_err(DDC_EINVAL, "query_order and xcd_swizzle must be 0 or 1");
  if (p->persistent < -1 || p->persistent > 1) return set_err(DDC_EINVAL, "persistent must be -1, 0 or 1");
  if (p->two_phase < -1 || p->two_phase > 1) return set_err(DDC_EINVAL, "two_phase must be -1, 0 or 1");
  if (p->full_d_matrix != 0 && p->full_d_matrix != 1) return set_err(DDC_EINVAL, "full_d_matrix must be 0 or 1");
  if (p->stage1_matrix < 0 || p->stage1_matrix > 2) return set_err(DDC_EINVAL, "stage1_matrix must be 0, 1 or 2");
  if (p->waves_per_simd != 0 && p->waves_per_simd != 4 && p->waves_per_simd != 5)
    return set_err(DDC_EINVAL, "waves_per_simd must be 0, 4 or 5");
  std::lock_guard<std::mutex> lk(ix->tune_mtx);
  ix->tuned.clear();   // a choice tuned under other forced knobs may not be the best now
  ix->waves_per_query = p->waves_per_query;
  ix->lookahead = p->lookahead;
  ix->query_order = p->query_order;
  ix->xcd_swizzle = p->xcd_swizzle;
  ix->persistent = p->persistent;
  ix->two_phase = p->two_phase;
  ix->full_d_matrix = p->full_d_matrix;
  ix->stage1_matrix = p->stage1_matrix;
  ix->waves_per_simd = p->waves_per_simd;
  return DDC_OK;
}

ddc_status ddc_get_launch(const ddc_index *ix, ddc_launch_params *p) {
  if (!ix || !p) return set_err(DDC_EINVAL, "NULL argument");
  p->waves_per_query = ix->waves_per_query;
  p->lookahead = ix->lookahead;
  p->query_order = ix->query_order;
  p->xcd_swizzle = ix->xcd_swizzle;
  p->persistent = ix->persistent;
  p->two_phase = ix->two_phase;
  p->full_d_matrix = ix->full_d_matrix;
  p->stage1_matrix = ix->stage1_matrix;
  p->waves_per_simd = ix->waves_per_simd;
  return DDC_OK;
}

ddc_status ddc_scan_variant(ddc_index *ix, int64_t nq, int32_t k_max, int32_t nprobe_max,
                            ddc_corr mode, int32_t *waves, int32_t *lookahead, int32_t *persistent,
                            int32_t *two_phase, int32_t *waves_per_simd) {
  if (!ix || !waves || !lookahead) return set_err(DDC_EINVAL, "NULL argument");
  if (nq < 1 || k_max < 1 || nprobe_max < 1) return set_err(DDC_EINVAL, "sizes must be >= 1");
  // the kernel family a search in this mode launches (significance > 0 assumed for LEARNED)
  const int prune = mode == DDC_CORR_BSAO ? 1 :
                    mode == DDC_CORR_LEARNED ? ix->Tt() > 0 : (mode != DDC_CORR_NONE && ix->St > 0);
  const int kind = prune + 2 * (mode == DDC_CORR_LEARNED && ix->P() ? 1 : 0) +
                   4 * (mode == DDC_CORR_BSAR && prune ? 1 : 0) + 16 * (mode == DDC_CORR_BSAO ? 1 : 0);
  const int64_t nqc = std::min<int64_t>(nq, 32768);
  ScanArgs la{};
  la.nblocks = ix->NB; la.k_max = k_max; la.block_b = ix->B; la.res = mode == DDC_CORR_BSAR;
  la.pq_m = mode == DDC_CORR_BSAO ? ix->pq_m : 0;
  la.pre = (kind & 2) ? 1 : 0; la.prune = prune;
  la.p_stride = nprobe_max; la.lag = ix->L;   // as the search sets them
  const bool two_ok = two_phase_eligible(ix, la);
  Variant v = fixed_variant(ix, nqc, prune, nprobe_max, two_ok);
  if (scan_lds_request(la, v[0]) > kMaxLds) v[0] = 4;
  {
    std::lock_guard<std::mutex> lk(ix->tune_mtx);
    const bool lm = !prune && ix->full_d_matrix == 1 && ix->d_tile_list.p != nullptr;
    auto it = ix->tuned.find(tune_class(nqc, nprobe_max, k_max, kind + (two_ok ? 32 : 0) + (lm ? 64 : 0)));
    if (it != ix->tuned.end()) v = it->second;
  }
  v = forced_or(ix, v, kind, two_ok);
  *waves = v[0];
  *lookahead = v[1];
  if (persistent) *persistent = v[2];
  if (two_phase) *two_phase = v[3];
  if (waves_per_simd) *waves_per_simd = v[4] ? 5 : 4;
  return DDC_OK;
}

ddc_status ddc_calibrate(ddc_index *ix, const float *calib, int64_t n_calib, int32_t calib_k,
                         int32_t calib_nprobe, int32_t calib_max_neg, uint64_t seed) {
  if (!ix || !calib) return set_err(DDC_EINVAL, "NULL argument");
  if (n_calib < 1) return set_err(DDC_EINVAL, "n_calib must be >= 1");
  if (calib_k < 0 || calib_k > kMaxK || calib_k > ix->n) return set_err(DDC_EINVAL, "calib_k must be in [0, min(256, n)]");
  if (calib_k == 0 && ix->tables.empty()) return set_err(DDC_EINVAL, "calib_k = 0 needs existing tables");
  if (calib_nprobe < 0 || calib_nprobe > ix->nlist) return set_err(DDC_EINVAL, "calib_nprobe must be in [0, nlist]");
  if (calib_max_neg < 1 || calib_max_neg > 256) return set_err(DDC_EINVAL, "calib_max_neg must be in [1, 256]");
  if (!all_finite(calib, n_calib * ix->D)) return set_err(DDC_EINVAL, "non-finite calibration values");
  const int npc = calib_nprobe ? calib_nprobe : std::min(std::max(1, ix->nlist / 8), 64);
  GUARD_BEGIN
  DeviceGuard dg(ix->device);
  StreamHolder sh;
  std::vector<int> kcs;
  if (calib_k) kcs.push_back(calib_k);
  else for (auto &t : ix->tables) kcs.push_back(t.kc);
  std::vector<ddc_index::Table> tabs;
  for (int kc : kcs) tabs.push_back(run_calibration(ix, calib, n_calib, kc, npc, calib_max_neg, seed, sh.s));
  set_tables(ix, std::move(tabs));
  return DDC_OK;
  GUARD_END
}

}  // extern "C"

ddc_status ddc::check_device_search(const ddc_index *ixc, const float *d_queries, int64_t nq,
                                     const int32_t *d_k, int32_t k_all, int32_t k_max,
                                     const int32_t *d_nprobe, int32_t nprobe_all, int32_t nprobe_max,
                                     double significance, ddc_corr mode, const int64_t *d_out_offsets,
                                     int64_t *d_ids, float *d_dists) {
  ddc_status st = check_search_args(ixc, nq, significance, mode);
  if (st != DDC_OK) return st;
  if (nq > 0 && (!d_queries || !d_ids || !d_dists)) return set_err(DDC_EINVAL, "NULL buffer");
  if (!d_k && (st = check_k_np(ixc, k_all, 1)) != DDC_OK) return st;
  if (d_k && (k_max < 1 || k_max > kMaxK)) return set_err(DDC_EINVAL, "k_max must be in [1, %d]", kMaxK);
  if (d_k && !d_out_offsets) return set_err(DDC_EINVAL, "per-query k needs out_offsets");
  return check_k_np(ixc, 1, d_nprobe ? nprobe_max : nprobe_all);
}


// ---------------------------------------------------------------------------------------
// fit
// ---------------------------------------------------------------------------------------
static void gather_rows(const float *src, int64_t ld, const std::vector<int64_t> &rows, int cols,
                        float *dst, int64_t ldd, hipStream_t s) {
  if (rows.empty()) return;
  DevBuf d_r(rows.size() * 8);
  HIPC(hipMemcpyAsync(d_r.p, rows.data(), rows.size() * 8, hipMemcpyHostToDevice, s));
  launch_gather_rows(src, ld, d_r.as<int64_t>(), (int64_t)rows.size(), cols, dst, ldd, s);
  HIPC(hipStreamSynchronize(s));
}

static void kmeans_assign(const float *d_Y, int64_t n, int Dp, const float *d_C, int nlist,
                          float *d_cn, unsigned long long *d_key, int32_t *d_assign, hipStream_t s) {
  launch_row_norms(d_C, Dp, nlist, Dp, d_cn, s);
  HIPC(hipMemsetAsync(d_key, 0xFF, n * 8, s));
  GemmArgs g{};
  g.A = d_Y; g.lda = Dp; g.mu = nullptr; g.B = d_C; g.ldb = Dp; g.bias = d_cn; g.key64 = d_key;
  g.M = n; g.N = nlist; g.K = Dp; g.mode = 2; g.prec = 0;
  launch_gemm(g, s);
  launch_decode_argmin(d_key, n, d_assign, s);
}

// Upload the quantizer (axes, codebooks) and encode every packed slot on the GPU.
static void pq_upload_encode(ddc_index *ix, hipStream_t s) {
  const int M = ix->pq_m;
  ix->d_pq_perm.alloc(ix->pq_perm.size() * 4);
  ix->d_pq_books.alloc(ix->pq_books.size() * 4);
  HIPC(hipMemcpyAsync(ix->d_pq_perm.p, ix->pq_perm.data(), ix->pq_perm.size() * 4, hipMemcpyHostToDevice, s));
  HIPC(hipMemcpyAsync(ix->d_pq_books.p, ix->pq_books.data(), ix->pq_books.size() * 4, hipMemcpyHostToDevice, s));
  ix->d_pq_codes.alloc(std::max<size_t>((size_t)ix->total_tiles * kTile * M, 16));
  ix->d_pq_err.alloc(std::max<size_t>((size_t)ix->total_tiles * kTile * 4, 16));
  launch_pq_encode(ix->d_base.p, ix->store(), ix->NB, ix->total_tiles, ix->d_pq_perm.as<int32_t>(),
                   ix->d_pq_books.as<float>(), M, ix->pq_dsub, ix->d_pq_codes.as<uint8_t>(),
                   ix->d_pq_err.as<float>(), s);
  HIPC(hipGetLastError());
  HIPC(hipStreamSynchronize(s));
}

// Codebooks of the quantization estimate: OPQ eigenvalue allocation of the PCA axes, then
// Lloyd k-means with 256 codewords in every subspace over the same key-sampled stored rows
// (initial codewords: the training rows with the smallest keys).
static void pq_train(ddc_index *ix, const float *d_Y, int M, int iters, int64_t ntrain, uint64_t seed,
                     hipStream_t s) {
  const int ds = ix->D / M;
  constexpr int K = 256;
  ix->pq_m = M;
  ix->pq_dsub = ds;
  ix->pq_perm = opq_allocation(ix->lam, M);
  const std::vector<int64_t> rows = select_by_key(ix->n, std::min<int64_t>(ix->n, ntrain), seed, TAG_PQ_SAMPLE);
  const int64_t ntr = (int64_t)rows.size();
  const std::vector<int64_t> init = select_by_key(ntr, K, seed, TAG_KMEANS_INIT);
  DevBuf d_rows(ntr * 8), d_cols((size_t)ds * 4), d_T((size_t)ntr * ds * 4), d_C((size_t)K * ds * 4),
      d_cn(K * 4), d_key(ntr * 8), d_as(ntr * 4), d_off((K + 1) * 4), d_mem(ntr * 4);
  HIPC(hipMemcpyAsync(d_rows.p, rows.data(), ntr * 8, hipMemcpyHostToDevice, s));
  std::vector<int32_t> asg(ntr), off(K + 1), mem(ntr), fill(K);
  ix->pq_books.assign((size_t)M * K * ds, 0.f);
  for (int j = 0; j < M; ++j) {
    HIPC(hipMemcpyAsync(d_cols.p, &ix->pq_perm[(size_t)j * ds], (size_t)ds * 4, hipMemcpyHostToDevice, s));
    launch_gather_cols(d_Y, ix->Dp, d_rows.as<int64_t>(), ntr, d_cols.as<int32_t>(), ds, d_T.as<float>(), s);
    gather_rows(d_T.as<float>(), ds, init, ds, d_C.as<float>(), ds, s);
    for (int it = 0; it < iters; ++it) {
      kmeans_assign(d_T.as<float>(), ntr, ds, d_C.as<float>(), K, d_cn.as<float>(),
                    d_key.as<unsigned long long>(), d_as.as<int32_t>(), s);
      HIPC(hipMemcpyAsync(asg.data(), d_as.p, ntr * 4, hipMemcpyDeviceToHost, s));
      HIPC(hipStreamSynchronize(s));
      std::fill(off.begin(), off.end(), 0);
      for (int64_t i = 0; i < ntr; ++i) off[asg[i] + 1]++;
      for (int c = 0; c < K; ++c) off[c + 1] += off[c];
      for (int c = 0; c < K; ++c) fill[c] = off[c];
      for (int64_t i = 0; i < ntr; ++i) mem[fill[asg[i]]++] = (int32_t)i;
      HIPC(hipMemcpyAsync(d_off.p, off.data(), off.size() * 4, hipMemcpyHostToDevice, s));
      HIPC(hipMemcpyAsync(d_mem.p, mem.data(), ntr * 4, hipMemcpyHostToDevice, s));
      launch_centroid_update(d_T.as<float>(), ds, ds, d_off.as<int32_t>(), d_mem.as<int32_t>(), K,
                             d_C.as<float>(), ds, s);
    }
    HIPC(hipMemcpyAsync(&ix->pq_books[(size_t)j * K * ds], d_C.p, (size_t)K * ds * 4, hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
  }
  HIPC(hipGetLastError());
}

extern "C" ddc_status ddc_fit(const float *base, int64_t n, int32_t dim, const float *calib,
                              int64_t n_calib, const ddc_fit_params *p, ddc_index **out) {
  if (!out) return set_err(DDC_EINVAL, "out is NULL");
  *out = nullptr;
  if (!base || !calib) return set_err(DDC_EINVAL, "NULL base or calib");
  ddc_status st = check_params(p, n, dim);
  if (st != DDC_OK) return st;
  if (n_calib < 1) return set_err(DDC_EINVAL, "n_calib must be >= 1");
  if (p->calib_k > n) return set_err(DDC_EINVAL, "calib_k > n");
  for (int i = 0; i < kMaxTables - 1; ++i)
    if (p->calib_k_extra[i] > n) return set_err(DDC_EINVAL, "calib_k_extra > n");
  if (!all_finite(base, n * dim) || !all_finite(calib, n_calib * dim))
    return set_err(DDC_EINVAL, "non-finite input values");
  GUARD_BEGIN
  std::unique_ptr<ddc_index> ix(new ddc_index);
  init_sizes(ix.get(), n, dim, p->nlist, p->delta_d, p->block_b, p->lag_l, p->storage, p->rotation,
             p->fp8_lead_dims);
  const int D = dim, Dp = ix->Dp, nlist = p->nlist;
  StreamHolder sh;
  hipStream_t s = sh.s;
  DevBuf d_X((size_t)n * D * 4);
  HIPC(hipMemcpyAsync(d_X.p, base, (size_t)n * D * 4, hipMemcpyHostToDevice, s));

  // F1: FP64 mean and covariance of the PCA sample
  std::vector<int64_t> rows;
  int64_t nrows = n;
  DevBuf d_rows;
  if (n > p->pca_sample) {
    rows = select_by_key(n, p->pca_sample, p->seed, TAG_PCA);
    nrows = (int64_t)rows.size();
    d_rows.alloc(rows.size() * 8);
    HIPC(hipMemcpyAsync(d_rows.p, rows.data(), rows.size() * 8, hipMemcpyHostToDevice, s));
  }
  const int nparts_m = (int)std::min<int64_t>(256, std::max<int64_t>(1, nrows / 1024));
  DevBuf d_mpart((size_t)nparts_m * D * 8), d_mu64((size_t)D * 8);
  launch_mean64(d_X.as<float>(), n, D, d_rows.as<int64_t>(), nrows, d_mpart.as<double>(), nparts_m,
                d_mu64.as<double>(), s);
  const int ntile = (D + 63) / 64;
  const int tiles = ntile * (ntile + 1) / 2;
  int nparts_c = (int)std::max<int64_t>(1, std::min<int64_t>(nrows / 256, 2048 / std::max(1, tiles)));
  nparts_c = std::max(1, std::min(nparts_c, (int)std::max<int64_t>(1, (int64_t)(1u << 30) / ((int64_t)ntile * ntile * 64 * 64 * 8))));
  DevBuf d_cpart((size_t)nparts_c * ntile * ntile * 64 * 64 * 8), d_cov((size_t)D * D * 8);
  launch_cov64(d_X.as<float>(), n, D, d_rows.as<int64_t>(), nrows, d_mu64.as<double>(),
               d_cpart.as<double>(), nparts_c, d_cov.as<double>(), s);
  std::vector<double> cov((size_t)D * D);
  ix->mu.resize(D);
  HIPC(hipMemcpyAsync(cov.data(), d_cov.p, cov.size() * 8, hipMemcpyDeviceToHost, s));
  HIPC(hipMemcpyAsync(ix->mu.data(), d_mu64.p, (size_t)D * 8, hipMemcpyDeviceToHost, s));
  HIPC(hipStreamSynchronize(s));
  HIPC(hipGetLastError());
  d_cpart.release();

  // F2: eigenvectors (rows of R, largest eigenvalue first)
  if (p->projection == DDC_PROJ_HAAR) {
    // a random rotation instead of PCA; lam = the variance along each rotated axis
    haar_rotation(D, p->seed, ix->R);
    ix->lam.assign(D, 0.0);
    for (int i = 0; i < D; ++i) {
      double v = 0.0;
      for (int a = 0; a < D; ++a) {
        double t = 0.0;
        for (int b = 0; b < D; ++b) t += cov[(size_t)a * D + b] * ix->R[(size_t)i * D + b];
        v += ix->R[(size_t)i * D + a] * t;
      }
      ix->lam[i] = v;
    }
  } else if (!sym_eig_desc(cov, D, ix->lam, ix->R)) {
    throw DdcError(DDC_EDEVICE, "eigen-decomposition did not converge");
  }

  // F3: rotate the base on the matrix cores, round to the storage format
  std::vector<float> R32((size_t)Dp * Dp, 0.f), mu32(Dp, 0.f);
  for (int i = 0; i < D; ++i) {
    mu32[i] = (float)ix->mu[i];
    for (int j = 0; j < D; ++j) R32[(size_t)i * Dp + j] = (float)ix->R[(size_t)i * D + j];
  }
  DevBuf d_R(R32.size() * 4), d_m32(mu32.size() * 4);
  HIPC(hipMemcpyAsync(d_R.p, R32.data(), R32.size() * 4, hipMemcpyHostToDevice, s));
  HIPC(hipMemcpyAsync(d_m32.p, mu32.data(), mu32.size() * 4, hipMemcpyHostToDevice, s));
  DevBuf d_Y((size_t)n * Dp * 4);
  {
    GemmArgs g{};
    g.A = d_X.as<float>(); g.lda = D; g.mu = d_m32.as<float>(); g.B = d_R.as<float>(); g.ldb = Dp;
    g.C = d_Y.as<float>(); g.ldc = Dp; g.M = n; g.N = Dp; g.K = D; g.mode = 0; g.prec = 0;
    launch_gemm(g, s);
  }
  launch_round_storage(d_Y.as<float>(), n * Dp, ix->store(), s);
  d_X.release();

  // F4: k-means (Lloyd) on the stored values
  const int64_t cap = (int64_t)p->kmeans_train_per_list * nlist;
  std::vector<int64_t> trows;
  const float *d_T = d_Y.as<float>();
  int64_t ntr = n;
  DevBuf d_train;
  if (n > cap) {
    trows = select_by_key(n, cap, p->seed, TAG_KMEANS_SAMPLE);
    ntr = (int64_t)trows.size();
    d_train.alloc((size_t)ntr * Dp * 4);
    gather_rows(d_Y.as<float>(), Dp, trows, Dp, d_train.as<float>(), Dp, s);
    d_T = d_train.as<float>();
  }
  const std::vector<int64_t> init = select_by_key(ntr, nlist, p->seed, TAG_KMEANS_INIT);
  DevBuf d_C((size_t)nlist * Dp * 4), d_cn((size_t)nlist * 4), d_key((size_t)n * 8),
      d_as((size_t)n * 4), d_off((size_t)(nlist + 1) * 4), d_mem((size_t)ntr * 4);
  gather_rows(d_T, Dp, init, Dp, d_C.as<float>(), Dp, s);
  std::vector<int32_t> asg(ntr), off(nlist + 1), mem(ntr), fill(nlist);
  for (int it = 0; it < p->kmeans_iters; ++it) {
    kmeans_assign(d_T, ntr, Dp, d_C.as<float>(), nlist, d_cn.as<float>(),
                  d_key.as<unsigned long long>(), d_as.as<int32_t>(), s);
    HIPC(hipMemcpyAsync(asg.data(), d_as.p, ntr * 4, hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    std::fill(off.begin(), off.end(), 0);
    for (int64_t i = 0; i < ntr; ++i) off[asg[i] + 1]++;
    for (int j = 0; j < nlist; ++j) off[j + 1] += off[j];
    for (int j = 0; j < nlist; ++j) fill[j] = off[j];
    for (int64_t i = 0; i < ntr; ++i) mem[fill[asg[i]]++] = (int32_t)i;
    HIPC(hipMemcpyAsync(d_off.p, off.data(), off.size() * 4, hipMemcpyHostToDevice, s));
    HIPC(hipMemcpyAsync(d_mem.p, mem.data(), ntr * 4, hipMemcpyHostToDevice, s));
    launch_centroid_update(d_T, Dp, D, d_off.as<int32_t>(), d_mem.as<int32_t>(), nlist,
                           d_C.as<float>(), Dp, s);
  }
  d_train.release();
  kmeans_assign(d_Y.as<float>(), n, Dp, d_C.as<float>(), nlist, d_cn.as<float>(),
                d_key.as<unsigned long long>(), d_as.as<int32_t>(), s);
  ix->assign.resize(n);
  std::vector<float> cpad((size_t)nlist * Dp);
  HIPC(hipMemcpyAsync(ix->assign.data(), d_as.p, n * 4, hipMemcpyDeviceToHost, s));
  HIPC(hipMemcpyAsync(cpad.data(), d_C.p, cpad.size() * 4, hipMemcpyDeviceToHost, s));
  HIPC(hipStreamSynchronize(s));
  HIPC(hipGetLastError());
  ix->cent.resize((size_t)nlist * D);
  for (int j = 0; j < nlist; ++j)
    for (int d = 0; d < D; ++d) ix->cent[(size_t)j * D + d] = cpad[(size_t)j * Dp + d];
  d_key.release();

  upload_index(ix.get(), d_Y.as<float>(), s);
  if (p->pq_m) {
    pq_train(ix.get(), d_Y.as<float>(), p->pq_m, p->pq_iters, p->pq_train, p->seed, s);
    pq_upload_encode(ix.get(), s);
  }
  d_Y.release();

  // F5: calibration of the correction table
  const int npc = p->calib_nprobe ? p->calib_nprobe : std::min(std::max(1, nlist / 8), 64);
  std::vector<ddc_index::Table> tabs;
  tabs.push_back(run_calibration(ix.get(), calib, n_calib, p->calib_k, npc, p->calib_max_neg, p->seed, s));
  for (int i = 0; i < kMaxTables - 1 && p->calib_k_extra[i]; ++i)
    tabs.push_back(run_calibration(ix.get(), calib, n_calib, p->calib_k_extra[i], npc, p->calib_max_neg,
                                   p->seed, s));
  set_tables(ix.get(), std::move(tabs));
  *out = ix.release();
  return DDC_OK;
  GUARD_END
}
