// Pruned candidate scan, top-K merge and finalize for IVF search on gfx950.
//
// Method (one wavefront, or a workgroup of four, per query):
//  * candidates are taken list by list in probe order, each list in blocks of B
//    stored positions; all candidates of a block are tested against the same
//    threshold tau_b, the K-th distance of the result queue after the previous block
//    (the paper refreshes tau after every candidate, Sec. I; B = 1 is that rule);
//  * a candidate's distance is accumulated 32 rotated dimensions at a time from a
//    dimension-blocked tile layout; after every stage of Delta_d dimensions the
//    data-driven test  m_s * e_s + beta_s > tau_b  (Sec. V-A linear classifier,
//    applied per stage as in Sec. V-B "Incremental Correction") prunes it, so a pruned
//    candidate never loads its remaining dimensions;
//  * survivors of the last stage carry their exact distance (Eq. (1): the full
//    rotated sum equals ||x - q||^2) into the block's survivor list; after the block
//    the queue becomes the K smallest (dis, id) of queue and survivors.
//
// Memory layout: tile t of 64 vectors, 32-dim block b -> 64 x 32 elements with each
// vector's 32-element slice contiguous (128 B in FP32, 64 B in FP16/BF16).  G lanes
// (8 for FP32, 4 for 16-bit) read one slice with 16-byte loads, so a wavefront reads 8
// or 16 slices per instruction, fully coalesced, and only for candidates still alive.
#include "ddc_internal.h"

#include <hip/hip_fp16.h>
#include <math.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <stdexcept>
#include <tuple>

namespace ddc {

namespace {

// ---- 16-byte payload -> EPL floats ----------------------------------------------
template <int ST> struct Store;
template <> struct Store<ST_F32> {
  static constexpr int kBytes = 4;
  __device__ static inline void unpack(const uint4 &v, float *f) {
    f[0] = __uint_as_float(v.x); f[1] = __uint_as_float(v.y);
    f[2] = __uint_as_float(v.z); f[3] = __uint_as_float(v.w);
  }
};
template <> struct Store<ST_F16> {
  static constexpr int kBytes = 2;
  __device__ static inline void unpack(const uint4 &v, float *f) {
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      __half2 h = *reinterpret_cast<const __half2 *>(&w[i]);
      float2 t = __half22float2(h);
      f[2 * i] = t.x; f[2 * i + 1] = t.y;
    }
  }
};
template <> struct Store<ST_BF16> {
  static constexpr int kBytes = 2;
  __device__ static inline void unpack(const uint4 &v, float *f) {
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      f[2 * i] = __uint_as_float(w[i] << 16);
      f[2 * i + 1] = __uint_as_float(w[i] & 0xFFFF0000u);
    }
  }
};

// Lane exchanges inside aligned groups of 8 lanes (DPP, no LDS traffic).
__device__ inline float dpp_xor1(float v) {  // quad_perm [1,0,3,2]
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));
}
__device__ inline float dpp_xor2(float v) {  // quad_perm [2,3,0,1]
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false));
}
__device__ inline float dpp_xor4(float v) {  // row_shl:4 into banks 0,2 and row_shr:4 into banks 1,3
  const int x = __float_as_int(v);
  int r = __builtin_amdgcn_update_dpp(x, x, 0x104, 0xF, 0x5, false);
  r = __builtin_amdgcn_update_dpp(r, x, 0x114, 0xF, 0xA, false);
  return __int_as_float(r);
}

// Transposed group reduction: lane j of every aligned group of G lanes (G = 4 or 8) holds
// G partial sums p[0..G-1]; on return it holds the group-wide sum of p[j].  Each halving
// step keeps the half of the values selected by one bit of j and adds the partner's copy.
template <int G> __device__ inline float transpose_sum(const float (&p)[G], int j) {
  float q[4];
  if constexpr (G == 8) {
    const bool hi = (j & 4) != 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float send = hi ? p[i] : p[i + 4];
      const float keep = hi ? p[i + 4] : p[i];
      q[i] = keep + dpp_xor4(send);
    }
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i) q[i] = p[i];
  }
  float r[2];
  const bool h1 = (j & 2) != 0;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const float send = h1 ? q[i] : q[i + 2];
    const float keep = h1 ? q[i + 2] : q[i];
    r[i] = keep + dpp_xor2(send);
  }
  const bool h0 = (j & 1) != 0;
  const float send = h0 ? r[0] : r[1];
  const float keep = h0 ? r[1] : r[0];
  return keep + dpp_xor1(send);
}

// Four FP8 E4M3 codes (byte k of w = element k) -> four floats, exact (gfx950 converts
// the OCP E4M3 format in hardware, two codes per instruction).
__device__ inline void e4m3x4_to_f32(uint32_t w, float *f) {
  const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)w, false);
  const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)w, true);
  f[0] = lo[0]; f[1] = lo[1]; f[2] = hi[0]; f[3] = hi[1];
}

// One term of the FP8 pre-stage: the decoded value is the code's value times the tile's scale
// rounded to FP32, and its difference to the query coordinate is rounded again.  Contraction
// into one fused multiply-add is off here, so every kernel forms the same sum (a fused form in
// one kernel and a separately rounded product in another once decided 1 pre-stage test of
// 3e8 differently).
__device__ inline float fp8_term(float code_value, float scale, float q) {
#pragma clang fp contract(off)
  const float decoded = code_value * scale;
  return decoded - q;
}

__device__ inline bool lex_less(float d, int32_t id, float td, int32_t tid) {
  return d < td || (d == td && id < tid);
}

__device__ inline unsigned long long lane_mask_lt() {
  const int lane = __lane_id();
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

}  // namespace

// LDS: per query (shared by its W waves) the rotated query, two result queues (double
// buffer), the block's survivors and two survivor counters; per wave two alive lists of the
// staged scan and the per-dim-block test table (m, beta; beta = -inf where no test follows).
// probe lists of a query staged in LDS (list id, length, first tile) when nprobe_max <= this
constexpr int kMetaCap = 256;

struct Lds {
  size_t q, td, ti, sd, si, cnt, lut, meta, query_bytes;
  size_t ac, ae, ap, mb, pr, th, wave_bytes;
};
__host__ __device__ inline size_t align16(size_t b) { return (b + 15) & ~(size_t)15; }
// res: the alive lists also carry each survivor's running sum of squared coordinates;
// lut_floats: the query's quantization lookup table (BSA-O), 0 when unused
// lag: the wave keeps the taus after its query's last lag + 1 blocks (lag > 0)
// lp: lag-parallel (each of the W waves scans a whole block; one survivor list per wave)
__host__ __device__ inline Lds lds_layout(int Dp, int kmax, int block_b, int W, bool res,
                                          int lut_floats, int p_stride, int lag, bool lp = false) {
  Lds l;
  size_t o = 0;
  l.q = o; o += align16((size_t)Dp * 4);
  l.lut = o; o += align16((size_t)lut_floats * 4);
  l.meta = o; o += p_stride <= kMetaCap ? align16((size_t)3 * p_stride * 4) : 0;
  l.td = o; o += align16((size_t)2 * kmax * 4);
  l.ti = o; o += align16((size_t)2 * kmax * 4);
  const int lists = lp ? W : 1;
  l.sd = o; o += align16((size_t)lists * block_b * 4);
  l.si = o; o += align16((size_t)lists * block_b * 4);
  l.cnt = o; o += lp ? 32 : 16;   // lp: the four waves' survivor counts after the first four
  l.query_bytes = o;
  const int seg = (W == 1 || lp) ? block_b : kTile;   // candidates one wave scans per segment
  o = 0;
  l.ac = o; o += align16((size_t)2 * seg * 2);
  l.ae = o; o += align16((size_t)2 * seg * 4);
  l.ap = o; o += res ? align16((size_t)2 * seg * 4) : 0;
  l.mb = o; o += align16((size_t)2 * (Dp / kBlockDims + 1) * 4);
  l.pr = o; o += 64 * 4;   // per-pair stage sums of a deep look-ahead round
  l.th = o; o += lag > 0 ? align16((size_t)(lag + 1) * 4) : 0;
  l.wave_bytes = o;
  return l;
}
__host__ __device__ inline size_t scan_lds_bytes(int Dp, int kmax, int block_b, int W, bool res,
                                                  int lut_floats, int p_stride, int lag,
                                                  bool lp = false) {
  const Lds l = lds_layout(Dp, kmax, block_b, W, res, lut_floats, p_stride, lag, lp);
  // lp: a workgroup of W waves for one query; otherwise four waves for 4 / W queries
  return lp ? l.query_bytes + (size_t)W * l.wave_bytes : (size_t)(4 / W) * l.query_bytes + 4 * l.wave_bytes;
}

// W waves per query (W = 1: four queries per workgroup, no workgroup barrier at all; W = 4:
// one query per workgroup, each block's tiles split over the four waves, survivors merged
// by the workgroup between two barriers).  LOOK enables the multi-stage look-ahead; PRE the
// FP8 pre-stage over the leading 64 dims before the first stage; RES the residual-estimate
// test of Alg. 2 instead of the learned one (one stage per load).  EST (with PRUNE off): rank
// every candidate by an estimate over the leading est_nb dim blocks instead of its distance
// (no refinement): est_scale * e_d, or with est_res the residual estimate of Alg. 1
// e_d + ||x_r||^2 + ||q'_r||^2 (C1 - C2).  PQ: the quantization test of BSA-O (asymmetric
// distance from the query's lookup table in LDS and the candidate's codes, with its
// quantization error as second feature) before the stages, whose tests are then lossless.
// LP (lag-parallel, W = 2 or 4 with LAG and lag >= W - 1; a workgroup of W waves runs one
// query): the blocks of a query go to its W waves in turn, each wave scanning a whole block
// (every block of a group of W consecutive blocks is tested against a tau from before the group,
// which the lag provides); the group's survivor lists are then merged into the queue in block
// order, recording every block's tau, so the results are those of the one-wave lagged scan bit
// for bit.
// OCC: the register budget, in waves per SIMD (4; 5 for the one-wave lag-free kernels' second
// build, a launch shape the tuner may pick: same code and results, fewer registers)
template <int ST, bool PRUNE, bool LOOK, int W, bool PRE, bool RES, bool EST = false, bool PQ = false,
          bool LAG = false, bool LM = false, bool LP = false, int OCC = 4>
__global__ __launch_bounds__(kScanThreads) __attribute__((amdgpu_waves_per_eu(OCC, 8))) void scan_kernel(ScanArgs a) {
  using S = Store<ST>;
  constexpr int EPL = 16 / S::kBytes;          // elements per lane load
  constexpr int G = kBlockDims / EPL;          // lanes per vector slice
  constexpr int CPW = 64 / G;                  // slices per wavefront load
  constexpr int MAXCH = 64 / CPW;              // loads per group: one 64-vector tile
  constexpr int GROUP = CPW * MAXCH;           // candidates per load group (64)
  constexpr int SLICE = kBlockDims * S::kBytes;            // bytes per vector slice
  constexpr int64_t BLOCK_BYTES = (int64_t)kTile * SLICE;  // bytes per tile dim-block
  constexpr int QPW = LP ? 1 : 4 / W;          // queries per workgroup (LP: W waves, one query)

  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int qs = wave / W, wsub = wave % W;    // query slot in the workgroup, wave within query
  int wg = blockIdx.x;
  if (a.xcd_swizzle) {
    // consecutive workgroups land on XCDs 0..7 in turn: give each XCD a contiguous range
    const int n = gridDim.x, x = wg % 8, r = wg / 8;
    const int per = n / 8, rem = n % 8;
    wg = x * per + min(x, rem) + r;
  }
  const int g = lane % G;
  const int sub = lane / G;
  const int nb = a.nblocks;
  const int Dp = nb * kBlockDims;
  const int B = a.block_b;
  const int KM = a.k_max;
  static_assert(!LP || ((W == 2 || W == 4) && LAG), "lag-parallel scans need two or four waves and a lag");
  constexpr int GM = W - 1;                  // LP: block index mod the group size
  constexpr bool WHOLE = W == 1 || LP;       // a wave scans whole blocks
  const int SEG = WHOLE ? B : kTile;
  const Lds L = lds_layout(Dp, KM, B, W, RES, PQ ? a.pq_m * 256 + Dp : 0, a.p_stride, LAG ? a.lag : 0, LP);
  unsigned char *ql = smem + (size_t)qs * L.query_bytes;
  unsigned char *wl = smem + (size_t)QPW * L.query_bytes + (size_t)wave * L.wave_bytes;
  float *s_q = reinterpret_cast<float *>(ql + L.q);
  float *s_td = reinterpret_cast<float *>(ql + L.td);
  int32_t *s_ti = reinterpret_cast<int32_t *>(ql + L.ti);
  float *s_sd = reinterpret_cast<float *>(ql + L.sd);
  int32_t *s_si = reinterpret_cast<int32_t *>(ql + L.si);
  int32_t *s_cnt = reinterpret_cast<int32_t *>(ql + L.cnt);
  uint16_t *s_ac = reinterpret_cast<uint16_t *>(wl + L.ac);
  float *s_ae = reinterpret_cast<float *>(wl + L.ae);
  float *s_ap = reinterpret_cast<float *>(wl + L.ap);
  float *s_mb = reinterpret_cast<float *>(wl + L.mb);
  float *s_pr = reinterpret_cast<float *>(wl + L.pr);
  float *s_th = reinterpret_cast<float *>(wl + L.th);   // taus after the last lag + 1 blocks
  float *s_lut = reinterpret_cast<float *>(ql + L.lut);
  const bool meta_lds = a.p_stride <= kMetaCap;
  int32_t *s_ml = reinterpret_cast<int32_t *>(ql + L.meta);   // list ids, lengths, first tiles

  // statistics (wave-uniform, flushed once when counters are requested)
  int64_t st_cand = 0, st_ref = 0, st_slices = 0, st_pre = 0, st_pre_pruned = 0, st_e1 = 0, st_e1_sl = 0;
  unsigned long long *ctr = reinterpret_cast<unsigned long long *>(a.counters);
  // stop-stage histogram, lane i counting stage i (one atomic per lane at the end)
  uint32_t st_stop = 0;
  auto stop_add = [&](int stage, uint32_t cnt) {
    if (lane == min(stage, 63)) st_stop += cnt;
  };

  // One query per pass.  Persistent launch (a.queue set): the workgroup stays resident and
  // takes the next slot from a device counter until none is left (the counter only grows, so
  // every wave reaches the exit); otherwise the slot is fixed by the workgroup index and there
  // is one pass.
  for (int pass = 0;; ++pass) {
  int slot;
  if (a.queue) {
    if (W == 1) {
      int v = 0;
      if (lane == 0) v = atomicAdd(a.queue, 1);
      slot = __builtin_amdgcn_readfirstlane(__shfl(v, 0));
    } else {
      if (threadIdx.x == 0) s_cnt[2] = atomicAdd(a.queue, 1);
      __syncthreads();
      slot = __builtin_amdgcn_readfirstlane(s_cnt[2]);
      __syncthreads();
    }
  } else {
    if (pass) break;
    slot = wg * QPW + qs;
  }
  if (slot >= a.nq) break;    // W = 4: the whole workgroup leaves together
  __builtin_amdgcn_wave_barrier();
  const int q = a.order ? a.order[slot] : slot;

  // per-query K and nprobe clamped to [1, k_max] and [1, p_stride]: the result queues and the
  // probe row are sized by those bounds
  const int K = __builtin_amdgcn_readfirstlane(min(max(a.k ? a.k[q] : a.k_all, 1), KM));
  const int np = min(max(a.nprobe ? a.nprobe[q] : a.nprobe_all, 1), a.p_stride);
  const float *qg = a.qrot + (int64_t)q * a.q_stride;
  const int qt = wsub * 64 + lane;             // thread index within the query's waves
  for (int i = qt; i < Dp; i += 64 * W) s_q[i] = qg[i];
  if (meta_lds) {
    // the query's probed lists and their lengths / first tiles, gathered once, so the list
    // loop below reads them from LDS instead of two dependent trips to memory per list
    for (int i = qt; i < np; i += 64 * W) {
      const int l = a.probes[(int64_t)q * a.p_stride + i];
      const bool ok = l >= 0 && l < a.nlist;
      s_ml[i] = ok ? l : -1;
      s_ml[a.p_stride + i] = ok ? a.list_len[l] : 0;
      s_ml[2 * a.p_stride + i] = ok ? a.tile_off[l] : 0;
    }
  }
  if (qt < 2) s_cnt[qt] = 0;
  float pq_m1 = 0.f, pq_m3 = 0.f, pq_beta = -INFINITY;
  if (PRUNE && !RES) {
    // this query's correction table (by its K) into the wave's LDS
    int tsel = 0;
    for (int t = 1; t < a.ntab; ++t)
      if (K >= a.tab_k[t]) tsel = t;
    const float *tq = a.tab + (size_t)tsel * (nb + 1) * 2;
    for (int i = lane; i < 2 * (nb + 1); i += 64) s_mb[i] = tq[i];
    if (PQ) {
      pq_m1 = a.pq_tab[4 * tsel];
      pq_m3 = a.pq_tab[4 * tsel + 1];
      pq_beta = a.pq_tab[4 * tsel + 2];
    }
  }
  if (W > 1) __syncthreads(); else __builtin_amdgcn_wave_barrier();
  if (PQ) {
    // lookup table lut[j][c] = ||q'_j - C_j[c]||^2 over the axes of subspace j: first the
    // query's coordinates in subspace order (after the table in LDS), then every entry from
    // its codeword (contiguous, coalesced across threads; four entries' loads in flight)
    const int ds = a.pq_dsub, M = a.pq_m;
    float *s_qp = s_lut + M * 256;
    for (int i = qt; i < M * ds; i += 64 * W) s_qp[i] = s_q[a.pq_perm[i]];
    if (W > 1) __syncthreads(); else __builtin_amdgcn_wave_barrier();
    const int nent = M * 256, step = 64 * W;
    for (int e0 = qt; e0 < nent; e0 += 4 * step) {
      float acc[4] = {0.f, 0.f, 0.f, 0.f};
      for (int t = 0; t < ds; ++t) {
        float cv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int e = min(e0 + u * step, nent - 1);
          cv[u] = a.pq_books[(int64_t)e * ds + t];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int e = min(e0 + u * step, nent - 1);
          const float d = s_qp[(e >> 8) * ds + t] - cv[u];
          acc[u] = fmaf(d, d, acc[u]);
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (e0 + u * step < nent) s_lut[e0 + u * step] = acc[u];
    }
    if (W > 1) __syncthreads(); else __builtin_amdgcn_wave_barrier();
  }
  // ||q'_1||^2 over dim block 0 (the expanded-form sums' error bound; any order will do)
  float qn1 = 0.f;
  if (!PQ && !PRE && !RES && PRUNE && a.e1_tol > 0.f) {
    const float v = lane < kBlockDims ? s_q[lane] : 0.f;
    qn1 = v * v;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) qn1 += __shfl_xor(qn1, o);
  }
  const int nbe = EST ? a.est_nb : nb;           // dim blocks the no-test path reads
  float qres = 0.f;                              // EST: ||q'_r||^2 beyond the leading blocks
  if (EST) {
    for (int i = nbe * kBlockDims + lane; i < Dp; i += 64) qres = fmaf(s_q[i], s_q[i], qres);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) qres += __shfl_xor(qres, o);
  }
  if (RES) {
    // per dim block b: ||q'_r||^2 - m sigma over the residual dims >= 32 (b + 1), with
    // sigma = sqrt(4 sum q'_i^2 lam_i) (Eq. (2)); block sums first, then suffix sums
    for (int b = lane; b < nb; b += 64) {
      float s2 = 0.f, sl = 0.f;
      for (int e = 0; e < kBlockDims; ++e) {
        const float v = s_q[b * kBlockDims + e];
        s2 = fmaf(v, v, s2);
        sl = fmaf(v * v, a.lam[b * kBlockDims + e], sl);
      }
      s_mb[2 * b] = s2;
      s_mb[2 * b + 1] = sl;
    }
    __builtin_amdgcn_wave_barrier();
    if (lane == 0) {
      float c2 = 0.f, cl = 0.f;
      for (int b = nb - 1; b >= 0; --b) {
        const float s2 = s_mb[2 * b], sl = s_mb[2 * b + 1];
        s_mb[2 * b] = c2 - a.bsar_m * 2.f * sqrtf(fmaxf(cl, 0.f));
        c2 += s2;
        cl += sl;
      }
    }
    __builtin_amdgcn_wave_barrier();
  }

  int tin = 0, tn = 0, par = 0;
  float tau = INFINITY;
  int32_t tau_id = 0x7FFFFFFF;
  int bidx = 0;   // blocks of this query done (the lagged tau's index)
  const unsigned long long lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  int ns = 0;   // W = 1 and LP: the wave's survivors of the current block (wave-uniform)
  // LP: each wave's survivors go to a list of its own
  float *sdw = LP ? s_sd + wsub * B : s_sd;
  int32_t *siw = LP ? s_si + wsub * B : s_si;

  // append the lanes with `take` to the block's survivor list
  auto append = [&](bool take, float ev, int32_t id) {
    const unsigned long long bal = __ballot(take);
    const int cnt = __popcll(bal);
    if (cnt == 0) return;
    int base;
    if (WHOLE) {
      base = ns;
      ns += cnt;
    } else {
      int b0 = 0;
      if (lane == 0) b0 = atomicAdd(&s_cnt[par], cnt);
      base = __shfl(b0, 0);
    }
    if (take) {
      const int pos = base + __popcll(bal & lt);
      sdw[pos] = ev;
      siw[pos] = id;
    }
  };

  // LP: merge the survivor lists of the group's n blocks (wave j scanned block g0 + j) into
  // the queue in block order, recording the tau after each block in the ring; a candidate's
  // rank is its place in the queue plus the survivors before it by (dis, id)
  auto lp_merge = [&](int n) {
    __syncthreads();                         // every wave's list and count are in LDS
    const int g0 = (bidx - 1) & ~GM;         // the group's first block
    for (int j = 0; j < n; ++j) {
      const int nsj = __builtin_amdgcn_readfirstlane(s_cnt[4 + j]);
      if (nsj > 0) {
        const float *sd = s_sd + j * B;
        const int32_t *si = s_si + j * B;
        const float *td = s_td + tin * KM;
        const int32_t *ti = s_ti + tin * KM;
        float *od = s_td + (tin ^ 1) * KM;
        int32_t *oi = s_ti + (tin ^ 1) * KM;
        for (int i = qt; i < tn + nsj; i += 64 * W) {
          float d;
          int32_t id;
          int rank;
          if (i < tn) {
            d = td[i]; id = ti[i]; rank = i;
          } else {
            d = sd[i - tn]; id = si[i - tn];
            int lo = 0, hi = tn;
            while (lo < hi) {
              const int mid = (lo + hi) >> 1;
              if (lex_less(td[mid], ti[mid], d, id)) lo = mid + 1; else hi = mid;
            }
            rank = lo;
          }
          for (int k2 = 0; k2 < nsj; ++k2) rank += lex_less(sd[k2], si[k2], d, id) ? 1 : 0;
          if (rank < K) { od[rank] = d; oi[rank] = id; }
        }
        __syncthreads();
        tin ^= 1;
        tn = min(K, tn + nsj);
        if (tn == K) {
          tau = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(s_td[tin * KM + K - 1])));
          tau_id = __builtin_amdgcn_readfirstlane(s_ti[tin * KM + K - 1]);
        }
      }
      if (lane == 0) s_th[(g0 + j) % (a.lag + 1)] = tn == K ? tau : INFINITY;
    }
    __builtin_amdgcn_wave_barrier();
    __syncthreads();                         // the lists are free for the next group
  };

  // two-phase scan: the first e1 entry of the current list (its candidates follow in order)
  int64_t e1_at = a.e1 ? a.e1_qoff[q] : 0;
  for (int p = 0; p < np; ++p) {
    int lst, len, toff;
    if (meta_lds) {
      lst = __builtin_amdgcn_readfirstlane(s_ml[p]);
      len = __builtin_amdgcn_readfirstlane(s_ml[a.p_stride + p]);
      toff = __builtin_amdgcn_readfirstlane(s_ml[2 * a.p_stride + p]);
    } else {
      lst = a.probes[(int64_t)q * a.p_stride + p];
      len = (lst >= 0 && lst < a.nlist) ? a.list_len[lst] : 0;
      toff = (lst >= 0 && lst < a.nlist) ? a.tile_off[lst] : 0;
    }
    const int64_t e1_list = e1_at;
    e1_at += (lst >= 0 && lst < a.nlist) ? e1_padded(len) : 0;
    if (lst < 0 || lst >= a.nlist) continue;  // never follow an invalid list id
    const unsigned char *lbase = reinterpret_cast<const unsigned char *>(a.base) +
                                 (int64_t)toff * nb * BLOCK_BYTES;  // wave-uniform
    const int32_t *lids = a.ids + (int64_t)toff * kTile;
    for (int bs = 0; bs < len; bs += B) {
      const int blen = min(B, len - bs);
      ns = 0;
      // the stage tests' threshold: the tau after block bidx - 1 - lag (+inf before it exists
      // or while that queue held fewer than K); the merge below is exact against the queue
      // (LAG: lag > 0; otherwise the current tau, +inf while the queue holds fewer than K)
      float tau_t = tau;
      if constexpr (LAG) {
        const int j = bidx - 1 - a.lag;
        tau_t = j >= 0 ? s_th[j % (a.lag + 1)] : INFINITY;
        tau_t = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, tau_t)));
      }
      // LP: the block belongs to wave bidx % 4; the other waves skip it
      const bool mine = !LP || (bidx & GM) == wsub;
      for (int s0 = (WHOLE ? (mine ? 0 : blen) : wsub * kTile); s0 < blen; s0 += (WHOLE ? blen : W * kTile)) {
      const int slen = WHOLE ? blen : min(kTile, blen - s0);
      const unsigned char *bbase = lbase + (int64_t)((bs + s0) / kTile) * nb * BLOCK_BYTES;
      const int32_t *bids = lids + bs + s0;
      const float *xnorm_seg = (RES || EST) ? a.xnorm + (int64_t)toff * kTile + bs + s0 : nullptr;
      // In a load group, chunk c, lane (sub, g) reads dims [g*EPL, g*EPL+EPL) of candidate
      // t0 + c*CPW + sub; after transpose_sum the lane owns candidate t0 + g*CPW + sub.
      if (LM) {
        // ---- list-major full-D scan: every candidate's distance was computed beforehand on
        // the matrix cores (launch_full_lists); one 4-byte load per candidate, four in flight ----
        const int64_t e0 = e1_list + bs + s0;
        for (int c0 = 0; c0 < slen; c0 += 256) {
          float ds[4];
          int32_t is[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int idx = c0 + u * 64 + lane;
            ds[u] = (idx < slen && e0 + idx < a.e1_cap) ? a.e1[e0 + idx] : 0.f;
            is[u] = bids[min(idx, slen - 1)];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int idx = c0 + u * 64 + lane;
            const bool valid = idx < slen && e0 + idx < a.e1_cap;
            append(valid && (tn < K || lex_less(ds[u], is[u], tau, tau_id)), ds[u], is[u]);
          }
        }
        st_cand += slen; st_ref += slen; st_slices += (int64_t)slen * nb;
        st_e1 += slen; st_e1_sl += (int64_t)slen * nb;
        if (ctr) stop_add(nb - 1, (uint32_t)slen);
      } else if (!PRUNE || (LAG ? !(tau_t < INFINITY) : tn < K)) {
        // ---- no test can prune: every candidate, every dim block ----
        // Slots past slen inside the last tile are zero padding: loads stay in bounds.
        for (int t0 = 0; t0 < slen; t0 += GROUP) {
          float acc[MAXCH], accp[MAXCH];
#pragma unroll
          for (int c = 0; c < MAXCH; ++c) acc[c] = accp[c] = 0.f;
          const uint32_t tile_off = (uint32_t)(t0 / kTile) * nb * (uint32_t)BLOCK_BYTES;
          const int sl = t0 + g * CPW + sub;      // the candidate this lane owns after the reduction
          const int32_t id_pre = bids[min(sl, slen - 1)];
          // full-D kernels: dim block b + 1 is loaded while block b is summed (a second register
          // set; the pruned kernels, whose full path is only a query's first block, keep their
          // registers for the staged scan, and the FP32 estimate kernels have none to spare)
          constexpr bool PIPE = !PRUNE && (S::kBytes == 2 || !EST);
          const unsigned char *tp = bbase + tile_off + g * 16;
          auto load_blk = [&](uint4 (&dst)[MAXCH], int b) {
#pragma unroll
            for (int c = 0; c < MAXCH; ++c)
              dst[c] = *reinterpret_cast<const uint4 *>(tp + b * BLOCK_BYTES + (uint32_t)((c * CPW + sub) * SLICE));
          };
          uint4 vn[MAXCH];
          if (PIPE) load_blk(vn, 0);
          for (int b = 0; b < nbe; ++b) {
            float qv[EPL];
#pragma unroll
            for (int e = 0; e < EPL; ++e) qv[e] = s_q[b * kBlockDims + g * EPL + e];
            uint4 v[MAXCH];
            if (PIPE) {
#pragma unroll
              for (int c = 0; c < MAXCH; ++c) v[c] = vn[c];
              if (b + 1 < nbe) load_blk(vn, b + 1);
            } else {
              load_blk(v, b);
            }
#pragma unroll
            for (int c = 0; c < MAXCH; ++c) {
              float f[EPL];
              S::unpack(v[c], f);
#pragma unroll
              for (int e = 0; e < EPL; ++e) {
                const float d = f[e] - qv[e];
                acc[c] = fmaf(d, d, acc[c]);
                if (EST) accp[c] = fmaf(f[e], f[e], accp[c]);
              }
            }
          }
          float dis = transpose_sum<G>(acc, g);
          if (EST) {
            const float xr = transpose_sum<G>(accp, g);   // ||x_d||^2 of the leading blocks
            dis = a.est_res ? dis + ((sl < slen ? xnorm_seg[sl] : 0.f) - xr) + qres : a.est_scale * dis;
          }
          bool keep = false;
          int32_t id = 0;
          if (sl < slen) {
            id = id_pre;
            keep = tn < K || lex_less(dis, id, tau, tau_id);
          }
          append(keep, dis, id);
        }
        st_cand += slen; st_ref += slen; st_slices += (int64_t)slen * nbe;
        if (ctr) stop_add(nbe - 1, (uint32_t)slen);
      } else if (PRUNE) {
        // ---- staged scan: test after every stage, compact the survivors ----
        // Lanes past the live count read the group's first live candidate (same cache
        // line, always in bounds) and are masked out of every decision.
        int cur = 0;
        int nalive = slen;
        st_cand += slen;
        bool listed = false;   // the alive list holds pre-stage survivors (partial sums restart at 0)
        if (PQ) {
          // ---- quantization test (BSA-O): lane = candidate; its code bytes (8 per load) index
          // the lookup table, the sum over subspaces is the asymmetric distance; prune iff
          // m1 dis' + m3 err + beta > tau; survivors go to the alive list ----
          const int tile0 = toff + (bs + s0) / kTile;   // wave-uniform
          const int M = a.pq_m;
          int nn = 0;
          for (int t0 = 0; t0 < slen; t0 += kTile) {
            const int idx = t0 + lane;
            const int64_t slot = (int64_t)(tile0 + t0 / kTile) * kTile + lane;   // in the tile: in bounds
            const uint2 *cp = reinterpret_cast<const uint2 *>(a.pq_codes + slot * M);
            float adc = 0.f;
            for (int c8 = 0; c8 < M / 8; ++c8) {
              const uint2 w = cp[c8];
              const int j0 = c8 * 8 * 256;
#pragma unroll
              for (int e = 0; e < 4; ++e) adc += s_lut[j0 + e * 256 + ((w.x >> (8 * e)) & 255u)];
#pragma unroll
              for (int e = 0; e < 4; ++e) adc += s_lut[j0 + (4 + e) * 256 + ((w.y >> (8 * e)) & 255u)];
            }
            const float er = a.pq_err[slot];
            const bool valid = idx < slen;
            const bool prune = valid && fmaf(pq_m1, adc, fmaf(pq_m3, er, pq_beta)) > tau_t;
            const bool keep = valid && !prune;
            const unsigned long long bal = __ballot(keep);
            if (keep) {
              const int pos = nn + __popcll(bal & lt);
              s_ac[pos] = (uint16_t)idx;
              s_ae[pos] = 0.f;
            }
            nn += __popcll(bal);
            st_pre_pruned += __popcll(__ballot(prune));
          }
          st_pre += slen;
          __builtin_amdgcn_wave_barrier();
          nalive = nn;
          listed = true;
        }
        if (PRE && a.e1) {
          // ---- FP8 pre-stage of the two-phase scan: the segment's pre-stage sums come from e1
          // (one 4-byte load per candidate instead of its 64 code bytes); same test, same
          // alive list contents ----
          const float mb = s_mb[2 * nb], bb = s_mb[2 * nb + 1];
          const int64_t e0 = e1_list + bs + s0;
          int nn = 0;
          for (int c0 = 0; c0 < slen; c0 += 256) {
            float evs[4];   // four loads in flight, then the tests
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int idx = c0 + u * 64 + lane;
              evs[u] = (idx < slen && e0 + idx < a.e1_cap) ? a.e1[e0 + idx] : 0.f;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int idx = c0 + u * 64 + lane;
              const bool valid = idx < slen && e0 + idx < a.e1_cap;
              const bool prune = valid && fmaf(mb, evs[u], bb) > tau_t;
              const bool keep = valid && !prune;
              const unsigned long long bal = __ballot(keep);
              if (keep) {
                const int pos = nn + __popcll(bal & lt);
                s_ac[pos] = (uint16_t)idx;
                s_ae[pos] = 0.f;
              }
              nn += __popcll(bal);
              st_pre_pruned += __popcll(__ballot(prune));
            }
          }
          st_pre += slen;
          st_e1 += slen;
          __builtin_amdgcn_wave_barrier();
          nalive = nn;
          listed = true;
        } else if (PRE) {
          // ---- FP8 pre-stage: one 64-byte code slice per candidate, decoded with the tile's
          // scale; survivors go to the alive list and the stages start over at dim 0 ----
          constexpr int G8 = 4, CPW8 = 16, CH8 = 4;   // 16 codes per lane, 16 candidates per load
          const int g8 = lane & 3, sub8 = lane >> 2;
          float q8[16];
#pragma unroll
          for (int e = 0; e < 16; ++e) q8[e] = s_q[g8 * 16 + e];
          const int tile0 = toff + (bs + s0) / kTile;   // wave-uniform
          const int last_tile = tile0 + (slen - 1) / kTile;
          int nn = 0;
          // two tiles per round trip: their loads are issued together; a second tile past the
          // segment re-reads the last one (in bounds) and every lane of it is masked out
          constexpr int NT8 = 2;
          for (int t0 = 0; t0 < slen; t0 += NT8 * kTile) {
            uint4 v[NT8][CH8];
            float sc[NT8];
#pragma unroll
            for (int u = 0; u < NT8; ++u) {
              const int tile = min(tile0 + t0 / kTile + u, last_tile);
              sc[u] = a.scale8[tile];
              const unsigned char *p8 = a.base8 + (int64_t)tile * (kTile * kFp8Lead) + g8 * 16;
#pragma unroll
              for (int c = 0; c < CH8; ++c)
                v[u][c] = *reinterpret_cast<const uint4 *>(p8 + (c * CPW8 + sub8) * 64);
            }
#pragma unroll
            for (int u = 0; u < NT8; ++u) {
              float part[CH8];
#pragma unroll
              for (int c = 0; c < CH8; ++c) {
                const uint32_t w[4] = {v[u][c].x, v[u][c].y, v[u][c].z, v[u][c].w};
                float acc = 0.f;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                  float f[4];
                  e4m3x4_to_f32(w[i], f);
#pragma unroll
                  for (int e = 0; e < 4; ++e) {
                    const float d = fp8_term(f[e], sc[u], q8[4 * i + e]);
                    acc = fmaf(d, d, acc);
                  }
                }
                part[c] = acc;
              }
              const float e0 = transpose_sum<G8>(part, g8);
              const int idx = t0 + u * kTile + g8 * CPW8 + sub8;
              const bool valid = idx < slen;
              const bool prune = valid && fmaf(s_mb[2 * nb], e0, s_mb[2 * nb + 1]) > tau_t;
              const bool keep = valid && !prune;
              const unsigned long long bal = __ballot(keep);
              if (keep) {
                const int pos = nn + __popcll(bal & lt);
                s_ac[pos] = (uint16_t)idx;
                s_ae[pos] = 0.f;
              }
              nn += __popcll(bal);
              st_pre_pruned += __popcll(__ballot(prune));
            }
          }
          st_pre += slen;
          __builtin_amdgcn_wave_barrier();
          nalive = nn;
          listed = true;
        }
        int b = 0;
        if (!PQ && !PRE && !RES && a.e1) {
          // ---- two-phase scan: the stage-1 sums of the segment come from e1 (one 4-byte load
          // per candidate instead of its dim block 0); the test after block 0 as the one-stage
          // path takes it; survivors go to the alive list and the stages continue at block 1.
          // Expanded-form sums (e1_tol > 0): a candidate is pruned here only if the test prunes
          // every value within the sum's error bound (the test is monotone in the sum); the
          // others restart at block 0 and are tested on the sum of the scan's own arithmetic ----
          const float mb = s_mb[0], bb = s_mb[1];
          const int64_t e0 = e1_list + bs + s0;
          const bool bounded = a.e1_tol > 0.f;
          const float tq = a.e1_tol * 3.f * qn1;
          const float t2 = a.e1_tol * 2.f;
          int nn = 0, pruned = 0;
          for (int c0 = 0; c0 < slen; c0 += 256) {
            float evs[4];   // four loads in flight, then the tests
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int idx = c0 + u * 64 + lane;
              evs[u] = (idx < slen && e0 + idx < a.e1_cap) ? a.e1[e0 + idx] : 0.f;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int idx = c0 + u * 64 + lane;
              const bool valid = idx < slen && e0 + idx < a.e1_cap;
              float ev = evs[u];
              if (bounded) {
                // the end of the bound interval where the test value is smallest
                const float w = fmaf(t2, fabsf(ev), tq) + 1e-30f;
                ev = mb >= 0.f ? ev - w : ev + w;
              }
              const bool prune = valid && fmaf(mb, ev, bb) > tau_t;
              const bool keep = valid && !prune;
              const unsigned long long bal = __ballot(keep);
              if (keep) {
                const int pos = nn + __popcll(bal & lt);
                s_ac[pos] = (uint16_t)idx;
                s_ae[pos] = bounded ? 0.f : ev;
              }
              nn += __popcll(bal);
              pruned += __popcll(__ballot(prune));
            }
          }
          // slices: block 0 of every candidate once (the re-read of the rechecked ones is
          // counted by the stages below, so they are taken off here)
          st_slices += bounded ? slen - nn : slen;
          st_e1 += slen;
          st_e1_sl += bounded ? slen - nn : slen;
          if (ctr) stop_add(0, (uint32_t)pruned);
          __builtin_amdgcn_wave_barrier();
          nalive = nn;
          listed = true;
          b = bounded ? 0 : 1;
        }
        while (b < nb && nalive > 0) {
          if (LOOK && nalive <= 8 && 64 / (nalive <= 1 ? 1 : nalive <= 2 ? 2 : nalive <= 4 ? 4 : 8) > G &&
              nb - b > G) {
            // ---- deep look-ahead: at most 8 live candidates; the 64 load slots of one round
            // hold Lr = 64 / 2^ceil(log2 nalive) consecutive stages of every one of them, so a
            // candidate walks up to 64 stages per memory round trip.  Slot p = c * CPW + sub
            // loads (candidate p / Lr, stage b + p % Lr); after the transposed reduction lane
            // (g, sub) holds slot g * CPW + sub, whose sum goes to LDS; lane i < nalive then
            // adds its candidate's stage sums in stage order and takes every test as the
            // one-stage path does, so results and counters are bit-identical to it.
            const int P2 = nalive <= 1 ? 1 : nalive <= 2 ? 2 : nalive <= 4 ? 4 : 8;
            const int Lr = 64 / P2;
            const int lgLr = Lr == 64 ? 6 : Lr == 32 ? 5 : Lr == 16 ? 4 : 3;
            const int Le = min(Lr, nb - b);
            const uint16_t *alive = s_ac + cur * SEG;
            const float *alive_e = s_ae + cur * SEG;
            const bool direct = b == 0 && !listed;
            const int first = direct ? 0 : (int)alive[0];
            uint4 v[MAXCH];
#pragma unroll
            for (int c = 0; c < MAXCH; ++c) {
              const int pp = c * CPW + sub;
              const int ci = pp >> lgLr;
              const int cd = ci < nalive ? (direct ? ci : (int)alive[ci]) : first;
              const int bb = min(b + (pp & (Lr - 1)), nb - 1);
              const uint32_t off = (uint32_t)((cd / kTile) * nb + bb) * (uint32_t)BLOCK_BYTES +
                                   (uint32_t)((cd % kTile) * SLICE + g * 16);
              v[c] = *reinterpret_cast<const uint4 *>(bbase + off);
            }
            const bool mine = lane < nalive;
            const int cand = mine ? (direct ? lane : (int)alive[lane]) : 0;
            // a window that ends the scan fetches its candidates' ids with the data
            int32_t id_pre = 0;
            if (b + Le == nb) id_pre = bids[cand];
            float part[MAXCH];
#pragma unroll
            for (int c = 0; c < MAXCH; ++c) {
              const int bb = min(b + ((c * CPW + sub) & (Lr - 1)), nb - 1);
              float f[EPL];
              S::unpack(v[c], f);
              float acc = 0.f;
#pragma unroll
              for (int e = 0; e < EPL; ++e) {
                const float d = f[e] - s_q[bb * kBlockDims + g * EPL + e];
                acc = fmaf(d, d, acc);
              }
              part[c] = acc;
            }
            const float tot = transpose_sum<G>(part, g);
            s_pr[g * CPW + sub] = tot;
            __builtin_amdgcn_wave_barrier();
            float ev = mine ? (direct ? 0.f : alive_e[lane]) : 0.f;
            int stop = Le;          // first pruning stage in the window (Le: none)
            if (mine) {
              for (int st = 0; st < Le; ++st) {
                ev += s_pr[lane * Lr + st];
                const int bb = b + st;
                if (fmaf(s_mb[2 * bb], ev, s_mb[2 * bb + 1]) > tau_t) { stop = st; break; }
              }
            }
            const bool survive = mine && stop == Le;
            // slices read up to each candidate's stopping stage
            {
              int cnt = mine ? (stop < Le ? stop + 1 : Le) : 0;
#pragma unroll
              for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o);
              st_slices += cnt;
            }
            if (ctr)
              for (int st = 0; st < Le; ++st)
                stop_add(b + st, (uint32_t)__popcll(__ballot(mine && stop == st)));
            __builtin_amdgcn_wave_barrier();
            if (b + Le == nb) {
              const int nsurv = __popcll(__ballot(survive));
              if (ctr) stop_add(nb - 1, (uint32_t)nsurv);
              st_ref += nsurv;
              int32_t id = 0;
              bool take = false;
              if (survive) {
                id = id_pre;
                take = lex_less(ev, id, tau, tau_id);
              }
              append(take, ev, id);
              __builtin_amdgcn_wave_barrier();
              nalive = 0;
            } else {
              const unsigned long long bal = __ballot(survive);
              if (survive) {
                const int pos = __popcll(bal & lt);
                s_ac[(cur ^ 1) * SEG + pos] = (uint16_t)cand;
                s_ae[(cur ^ 1) * SEG + pos] = ev;
              }
              __builtin_amdgcn_wave_barrier();
              nalive = __popcll(bal);
              cur ^= 1;
            }
            b += Le;
            continue;
          }
          int L = 1;
          if (LOOK && nb - b > 1) {
            // Look-ahead: when the live candidates fit in MAXCH / L load slots, every slot
            // loads one (candidate, stage) pair of L consecutive stages, so L dependent loads
            // become one.  Decisions are still taken stage by stage; bytes past a
            // candidate's stopping stage are read but not counted as algorithmic.
            const int ch = (nalive + CPW - 1) / CPW;
            if (ch * 8 <= MAXCH) L = 8;
            else if (ch * 4 <= MAXCH) L = 4;
            else if (ch * 2 <= MAXCH) L = 2;
          }
          if (LOOK && L > 1) {
            const int Le = min(L, nb - b);
            const int lgL = L == 8 ? 3 : (L == 4 ? 2 : 1);
            const uint16_t *alive = s_ac + cur * SEG;
            const float *alive_e = s_ae + cur * SEG;
            const bool direct = b == 0 && !listed;
            const int first = direct ? 0 : (int)alive[0];
            uint4 v[MAXCH];
#pragma unroll
            for (int c = 0; c < MAXCH; ++c) {
              const int idx = (c >> lgL) * CPW + sub;
              const int cd = idx < nalive ? (direct ? idx : (int)alive[idx]) : first;
              const int bb = min(b + (c & (L - 1)), nb - 1);
              const uint32_t off = (uint32_t)((cd / kTile) * nb + bb) * (uint32_t)BLOCK_BYTES +
                                   (uint32_t)((cd % kTile) * SLICE + g * 16);
              v[c] = *reinterpret_cast<const uint4 *>(bbase + off);
            }
            // lane (g, sub) owns slot g = (candidate g >> lgL, stage g & (L-1)) after the reduction
            const int my_cc = g >> lgL, my_ss = g & (L - 1);
            const int idx = my_cc * CPW + sub;
            const bool valid = idx < nalive;
            const int ci = min(idx, SEG - 1);
            const int cand = direct ? idx : (int)alive[ci];
            int32_t id_pre = 0;
            if (b + Le == nb) id_pre = bids[valid ? cand : first];
            float part[MAXCH];
#pragma unroll
            for (int c = 0; c < MAXCH; ++c) {
              const int bb = min(b + (c & (L - 1)), nb - 1);
              float f[EPL];
              S::unpack(v[c], f);
              float acc = 0.f;
#pragma unroll
              for (int e = 0; e < EPL; ++e) {
                const float d = f[e] - s_q[bb * kBlockDims + g * EPL + e];
                acc = fmaf(d, d, acc);
              }
              part[c] = acc;
            }
            const float tot = transpose_sum<G>(part, g);
            // running partial distance, added one stage at a time in stage order: the same
            // rounding as the one-stage path, so the variant changes no result bit
            float ev = my_ss == 0 ? (direct ? tot : alive_e[ci] + tot) : tot;
            for (int j = 1; j < L; ++j) {
              const float prev = __shfl_up(ev, 1);
              if (my_ss == j) ev = prev + ev;
            }
            bool prune = false;
            if (valid && my_ss < Le) {
              const int bb = b + my_ss;
              prune = fmaf(s_mb[2 * bb], ev, s_mb[2 * bb + 1]) > tau_t;
            }
            const unsigned long long pm = __ballot(prune);
            const uint32_t bits = (uint32_t)(pm >> (sub * G + my_cc * L)) & ((1u << L) - 1u);
            const int firstp = bits ? __builtin_ctz(bits) : Le;
            st_slices += __popcll(__ballot(valid && my_ss < Le && my_ss <= firstp));
            const bool writer = valid && my_ss == Le - 1;
            const bool survive = writer && bits == 0;
            if (ctr)
              for (int s2 = 0; s2 < Le; ++s2)
                stop_add(b + s2, (uint32_t)__popcll(__ballot(writer && bits && firstp == s2)));
            if (b + Le == nb) {
              // the window reached the last stage: survivors carry their exact distance
              const int nsurv = __popcll(__ballot(survive));
              if (ctr) stop_add(nb - 1, (uint32_t)nsurv);
              st_ref += nsurv;
              int32_t id = 0;
              bool take = false;
              if (survive) {
                id = id_pre;
                take = lex_less(ev, id, tau, tau_id);
              }
              append(take, ev, id);
              __builtin_amdgcn_wave_barrier();
              nalive = 0;
            } else {
              const unsigned long long bal = __ballot(survive);
              if (survive) {
                const int pos = __popcll(bal & lt);
                s_ac[(cur ^ 1) * SEG + pos] = (uint16_t)cand;
                s_ae[(cur ^ 1) * SEG + pos] = ev;
              }
              __builtin_amdgcn_wave_barrier();
              nalive = __popcll(bal);
              cur ^= 1;
            }
            b += Le;
            continue;
          }
          const bool last = b == nb - 1;
          const bool test = a.test_after[b] != 0;
          const float mb = s_mb[2 * b], bb = s_mb[2 * b + 1];
          float qv[EPL];
#pragma unroll
          for (int e = 0; e < EPL; ++e) qv[e] = s_q[b * kBlockDims + g * EPL + e];
          const unsigned char *bp = bbase + b * BLOCK_BYTES + g * 16;
          const uint16_t *alive = s_ac + cur * SEG;
          const float *alive_e = s_ae + cur * SEG;
          const float *alive_p = s_ap + cur * SEG;
          const bool direct = b == 0 && !listed;
          int nnext = 0;
          int pruned = 0;
          for (int t0 = 0; t0 < nalive; t0 += GROUP) {
            const int first = direct ? t0 : (int)alive[t0];
            uint4 v[MAXCH];
#pragma unroll
            for (int c = 0; c < MAXCH; ++c) {
              const int idx = t0 + c * CPW + sub;
              const int cd = idx < nalive ? (direct ? idx : (int)alive[idx]) : first;
              const uint32_t off = (uint32_t)(cd / kTile) * nb * (uint32_t)BLOCK_BYTES +
                                   (uint32_t)((cd % kTile) * SLICE);
              v[c] = *reinterpret_cast<const uint4 *>(bp + off);
            }
            const int idx = t0 + g * CPW + sub;   // the candidate this lane owns after the reduction
            const bool valid = idx < nalive;
            const int ci = min(idx, SEG - 1);
            const int cand = direct ? idx : (int)alive[ci];
            int32_t id_pre = 0;
            if (last) id_pre = bids[valid ? cand : first];
            float part[MAXCH], partp[MAXCH];
#pragma unroll
            for (int c = 0; c < MAXCH; ++c) {
              float f[EPL];
              S::unpack(v[c], f);
              float acc = 0.f, accp = 0.f;
#pragma unroll
              for (int e = 0; e < EPL; ++e) {
                const float d = f[e] - qv[e];
                acc = fmaf(d, d, acc);
                if (RES) accp = fmaf(f[e], f[e], accp);
              }
              part[c] = acc;
              partp[c] = accp;
            }
            const float tot = transpose_sum<G>(part, g);
            const float ev = direct ? tot : alive_e[ci] + tot;
            float pv = 0.f;   // RES: sum of the candidate's squared coordinates so far
            if (RES) {
              const float totp = transpose_sum<G>(partp, g);
              pv = direct ? totp : alive_p[ci] + totp;
            }
            bool keep = valid;
            if (test) {
              if (RES) {
                // dis' = e_s + ||x_r||^2 + ||q'_r||^2 (C1 - C2 of Alg. 1); prune iff
                // dis' - m sigma > tau (Alg. 2)
                const float xn = valid ? xnorm_seg[cand] : 0.f;
                keep = keep && !(ev + (xn - pv) + mb > tau_t);
              } else {
                keep = keep && !(fmaf(mb, ev, bb) > tau_t);
              }
            }
            if (last) {
              int32_t id = 0;
              bool take = false;
              if (keep) {
                id = id_pre;
                take = lex_less(ev, id, tau, tau_id);
              }
              append(take, ev, id);
            } else {
              const unsigned long long bal = __ballot(keep);
              if (keep) {
                const int pos = nnext + __popcll(bal & lt);
                s_ac[(cur ^ 1) * SEG + pos] = (uint16_t)cand;
                s_ae[(cur ^ 1) * SEG + pos] = ev;
                if (RES) s_ap[(cur ^ 1) * SEG + pos] = pv;
              }
              nnext += __popcll(bal);
            }
            pruned += __popcll(__ballot(valid && !keep));
          }
          st_slices += nalive;
          if (last) st_ref += nalive - pruned;
          if (ctr) stop_add(b, (uint32_t)(last ? nalive : pruned));   // last block: all stop here
          __builtin_amdgcn_wave_barrier();
          if (!last) { nalive = nnext; cur ^= 1; }
          b += 1;
        }
      }
      }  // segments
      if constexpr (LP) {
        // the block's survivor count for the group merge, which follows the group's last block
        if (mine && lane == 0) s_cnt[4 + wsub] = ns;
        ++bidx;
        if ((bidx & GM) == 0) lp_merge(W);
        continue;
      }
      // ---- merge: queue (sorted, tn) + survivors (ns) -> K smallest by (dis, id) ----
      int mt, mstep;
      if (W == 1) {
        __builtin_amdgcn_wave_barrier();
        mt = lane; mstep = 64;
      } else {
        __syncthreads();                       // every wave's survivors are in LDS
        ns = s_cnt[par];
        mt = qt; mstep = 64 * W;
      }
      // many survivors (a query's first blocks, where no test prunes): sort them first with a
      // bitonic network in LDS, so every element's rank is two binary searches instead of a
      // count over all survivors (one wave; the padding sorts last)
      int np2 = 64;
      while (np2 < ns) np2 <<= 1;
      const bool sorted = W == 1 && ns > 64 && np2 <= B;
      if (sorted) {
        for (int i = ns + lane; i < np2; i += 64) { s_sd[i] = INFINITY; s_si[i] = 0x7FFFFFFF; }
        __builtin_amdgcn_wave_barrier();
        for (int kk = 2; kk <= np2; kk <<= 1) {
          for (int jj = kk >> 1; jj > 0; jj >>= 1) {
            for (int t = lane; t < (np2 >> 1); t += 64) {
              const int i0 = ((t & ~(jj - 1)) << 1) | (t & (jj - 1));
              const int i1 = i0 + jj;
              const float d0 = s_sd[i0], d1 = s_sd[i1];
              const int32_t x0 = s_si[i0], x1 = s_si[i1];
              const bool up = (i0 & kk) == 0;
              if (up ? lex_less(d1, x1, d0, x0) : lex_less(d0, x0, d1, x1)) {
                s_sd[i0] = d1; s_sd[i1] = d0; s_si[i0] = x1; s_si[i1] = x0;
              }
            }
            __builtin_amdgcn_wave_barrier();
          }
        }
      }
      if (ns > 0) {
        const float *td = s_td + tin * KM;
        const int32_t *ti = s_ti + tin * KM;
        float *od = s_td + (tin ^ 1) * KM;
        int32_t *oi = s_ti + (tin ^ 1) * KM;
        if (sorted) {
          // rank = place in its own sorted list + elements of the other list before it
          for (int i = mt; i < tn + ns && i < tn + K; i += mstep) {
            const bool inq = i < tn;
            const int own = inq ? i : i - tn;
            const float d = inq ? td[i] : s_sd[own];
            const int32_t id = inq ? ti[i] : s_si[own];
            int lo = 0, hi = inq ? ns : tn;
            while (lo < hi) {
              const int mid = (lo + hi) >> 1;
              const bool lt_ = inq ? lex_less(s_sd[mid], s_si[mid], d, id) : lex_less(td[mid], ti[mid], d, id);
              if (lt_) lo = mid + 1; else hi = mid;
            }
            const int rank = own + lo;
            if (rank < K) { od[rank] = d; oi[rank] = id; }
          }
        } else
        for (int i = mt; i < tn + ns; i += mstep) {
          float d;
          int32_t id;
          int rank;
          if (i < tn) {
            d = td[i]; id = ti[i]; rank = i;
          } else {
            d = s_sd[i - tn]; id = s_si[i - tn];
            int lo = 0, hi = tn;
            while (lo < hi) {
              const int mid = (lo + hi) >> 1;
              if (lex_less(td[mid], ti[mid], d, id)) lo = mid + 1; else hi = mid;
            }
            rank = lo;
          }
          for (int j = 0; j < ns; ++j) rank += lex_less(s_sd[j], s_si[j], d, id) ? 1 : 0;
          if (rank < K) { od[rank] = d; oi[rank] = id; }
        }
      }
      if (W == 1) {
        __builtin_amdgcn_wave_barrier();
      } else {
        if (qt == 0) s_cnt[par ^ 1] = 0;       // the next block's counter (unused until then)
        __syncthreads();
        par ^= 1;
      }
      if (ns > 0) {
        tin ^= 1;
        tn = min(K, tn + ns);
        if (tn == K) {
          tau = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(s_td[tin * KM + K - 1])));
          tau_id = __builtin_amdgcn_readfirstlane(s_ti[tin * KM + K - 1]);
        }
      }
      if constexpr (LAG) {
        // this block's tau into the wave's ring (every wave of the query keeps the same ring)
        if (lane == 0) s_th[bidx % (a.lag + 1)] = tn == K ? tau : INFINITY;
        __builtin_amdgcn_wave_barrier();
        ++bidx;
      }
    }
  }
  if (LP && (bidx & GM) != 0) lp_merge(bidx & GM);   // a last, incomplete group

  // ---- finalize: ascending (dis, id), original ids, padding ----
  const int64_t off = a.out_off ? a.out_off[q] : (int64_t)q * a.k_all;
  for (int i = qt; i < K; i += 64 * W) {
    const bool have = i < tn;
    a.out_ids[off + i] = have ? (int64_t)s_ti[tin * KM + i] : (int64_t)-1;
    a.out_d[off + i] = have ? s_td[tin * KM + i] : INFINITY;
  }
  }  // passes
  if (ctr && st_stop) atomicAdd(&ctr[4 + lane], (unsigned long long)st_stop);
  if (ctr && lane == 0 && st_cand) {
    atomicAdd(&ctr[0], (unsigned long long)st_cand);
    atomicAdd(&ctr[1], (unsigned long long)st_ref);
    atomicAdd(&ctr[2], (unsigned long long)st_slices);
    if (st_e1) atomicAdd(&ctr[3], (unsigned long long)st_e1);
    if (st_e1_sl) atomicAdd(&ctr[kCtrSlicesSummed], (unsigned long long)st_e1_sl);
    if (PRE || PQ) {
      atomicAdd(&ctr[kCtrPreReads], (unsigned long long)st_pre);
      atomicAdd(&ctr[kCtrPrePruned], (unsigned long long)st_pre_pruned);
    }
  }
}

__global__ void fill_i32_kernel(int32_t *p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void order_hist_kernel(const int32_t *probes, int32_t p_stride, int64_t nq, int32_t *hist,
                                  int32_t *rank) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < nq) rank[q] = atomicAdd(&hist[probes[q * p_stride] + 1], 1);
}

__global__ void order_scan_kernel(int32_t *hist, int32_t nlist) {
  // exclusive prefix over hist[1..nlist] in place (hist[0] = 0), one workgroup
  __shared__ int32_t part[256];
  const int t = threadIdx.x;
  const int chunk = (nlist + 255) / 256;
  const int b = 1 + t * chunk, e = min(nlist + 1, b + chunk);
  int s = 0;
  for (int i = b; i < e; ++i) s += hist[i];
  part[t] = s;
  __syncthreads();
  if (t == 0) {
    int c = 0;
    for (int i = 0; i < 256; ++i) { const int v = part[i]; part[i] = c; c += v; }
  }
  __syncthreads();
  int c = part[t];
  for (int i = b; i < e; ++i) { const int v = hist[i]; hist[i] = c; c += v; }
}

__global__ void order_scatter_kernel(const int32_t *probes, int32_t p_stride, int64_t nq,
                                     const int32_t *hist, const int32_t *rank, int32_t *order) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < nq) order[hist[probes[q * p_stride] + 1] + rank[q]] = (int32_t)q;
}

// Counting sort of the queries by key (keys[q * stride] in [0, nbins); anything else counts as
// one more key below all of them) in one workgroup: histogram in LDS, exclusive prefix, scatter.
// rank[q] (global scratch) is the query's place among equal keys, in the order the atomics
// took them; the scan gives the same results for any order of the queries.
constexpr int kOrderThreads = 1024;
__global__ __launch_bounds__(kOrderThreads) void order_fused_kernel(const int32_t *keys, int32_t stride,
                                                                   int64_t nq, int32_t nbins,
                                                                   int32_t *rank, int32_t *order) {
  extern __shared__ int32_t hist_lds[];      // nbins + 1 counters
  __shared__ int32_t wsum[kOrderThreads / 64];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int nb1 = nbins + 1;
  for (int i = t; i < nb1; i += kOrderThreads) hist_lds[i] = 0;
  __syncthreads();
  for (int64_t q = t; q < nq; q += kOrderThreads) {
    const int k = keys[q * stride];
    rank[q] = atomicAdd(&hist_lds[(k >= 0 && k < nbins) ? k + 1 : 0], 1);
  }
  __syncthreads();
  // exclusive prefix: every thread a contiguous chunk of counters, then a scan of the chunk sums
  const int chunk = (nb1 + kOrderThreads - 1) / kOrderThreads;
  const int b0 = min(nb1, t * chunk), b1 = min(nb1, b0 + chunk);
  int sum = 0;
  for (int i = b0; i < b1; ++i) sum += hist_lds[i];
  int inc = sum;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int v = __shfl_up(inc, o);
    if (lane >= o) inc += v;
  }
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  if (t == 0) {
    int c = 0;
    for (int i = 0; i < kOrderThreads / 64; ++i) { const int v = wsum[i]; wsum[i] = c; c += v; }
  }
  __syncthreads();
  int c = wsum[w] + inc - sum;
  for (int i = b0; i < b1; ++i) { const int v = hist_lds[i]; hist_lds[i] = c; c += v; }
  __syncthreads();
  for (int64_t q = t; q < nq; q += kOrderThreads) {
    const int k = keys[q * stride];
    order[hist_lds[(k >= 0 && k < nbins) ? k + 1 : 0] + rank[q]] = (int32_t)q;
  }
}

// up to this many keys the one-workgroup sort (its counters in LDS) is used
constexpr int kOrderMaxBins = 32767;

void launch_query_order(const int32_t *probes, int32_t p_stride, int64_t nq, int32_t nlist,
                        int32_t *hist, int32_t *rank, int32_t *order, hipStream_t s) {
  if (nq <= 0) return;
  if (nlist <= kOrderMaxBins) {
    hipLaunchKernelGGL(order_fused_kernel, dim3(1), dim3(kOrderThreads), (size_t)(nlist + 1) * 4, s,
                       probes, p_stride, nq, nlist, rank, order);
    return;
  }
  hipLaunchKernelGGL(fill_i32_kernel, dim3((nlist + 256) / 256), dim3(256), 0, s, hist,
                     (int64_t)nlist + 1, 0);
  const unsigned g = (unsigned)((nq + 255) / 256);
  hipLaunchKernelGGL(order_hist_kernel, dim3(g), dim3(256), 0, s, probes, p_stride, nq, hist, rank);
  hipLaunchKernelGGL(order_scan_kernel, dim3(1), dim3(256), 0, s, hist, nlist);
  hipLaunchKernelGGL(order_scatter_kernel, dim3(g), dim3(256), 0, s, probes, p_stride, nq, hist, rank,
                     order);
}

// One wavefront per query: the lanes add the lengths of its probed lists, and the key is 255
// minus the log2 of that candidate count in eighths (longest first).
__global__ __launch_bounds__(256) void work_key_kernel(const int32_t *probes, int32_t p_stride,
                                                       const int32_t *nprobe, int32_t nprobe_all,
                                                       const int32_t *list_len, int32_t nlist, int64_t nq,
                                                       int32_t *key) {
  const int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (q >= nq) return;
  const int np = min(max(nprobe ? nprobe[q] : nprobe_all, 1), p_stride);
  long long work = 0;
  for (int p = lane; p < np; p += 64) {
    const int l = probes[q * p_stride + p];
    if (l >= 0 && l < nlist) work += list_len[l];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) work += __shfl_xor(work, o);
  if (lane == 0) {
    const int bucket = work > 0 ? min(255, (int)(log2f((float)work) * 8.f)) : 0;
    key[q] = 255 - bucket;
  }
}

void launch_work_order(const int32_t *probes, int32_t p_stride, const int32_t *nprobe,
                       int32_t nprobe_all, const int32_t *list_len, int32_t nlist, int64_t nq,
                       int32_t *key, int32_t *hist, int32_t *rank, int32_t *order, hipStream_t s) {
  if (nq <= 0) return;
  hipLaunchKernelGGL(work_key_kernel, dim3((unsigned)((nq + 3) / 4)), dim3(256), 0, s, probes,
                     p_stride, nprobe, nprobe_all, list_len, nlist, nq, key);
  launch_query_order(key, 1, nq, 256, hist, rank, order, s);
}

// ---- two-phase scan, first phase: stage-1 partial distances list by list ----------------

// Exclusive prefix sum in one workgroup: start[i] = cnt[0] + ... + cnt[i-1], start[n] = total.
constexpr int kScanPrefixThreads = 1024;
template <class T>
__global__ __launch_bounds__(kScanPrefixThreads) void excl_prefix_kernel(const T *cnt, int64_t n, T *start) {
  __shared__ T wsum[kScanPrefixThreads / 64];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int64_t chunk = (n + kScanPrefixThreads - 1) / kScanPrefixThreads;
  const int64_t b0 = min(n, t * chunk), b1 = min(n, b0 + chunk);
  T sum = 0;
  for (int64_t i = b0; i < b1; ++i) sum += cnt[i];
  T inc = sum;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const T v = __shfl_up(inc, o);
    if (lane >= o) inc += v;
  }
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  if (t == 0) {
    T c = 0;
    for (int i = 0; i < kScanPrefixThreads / 64; ++i) { const T v = wsum[i]; wsum[i] = c; c += v; }
    start[n] = c;
  }
  __syncthreads();
  T c = wsum[w] + inc - sum;
  for (int64_t i = b0; i < b1; ++i) { const T v = cnt[i]; start[i] = c; c += v; }
}

// One wavefront per query: offset of each probed list's first candidate among the query's
// candidates (lengths of the lists before it, in probe order) and the query's total.
__global__ __launch_bounds__(256) void pair_offsets_kernel(const int32_t *probes, int32_t p_stride,
                                                           const int32_t *nprobe, int32_t nprobe_all,
                                                           const int32_t *list_len, int32_t nlist,
                                                           int64_t nq, int64_t *poff, int64_t *qcnt) {
  const int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (q >= nq) return;
  const int np = min(max(nprobe ? nprobe[q] : nprobe_all, 1), p_stride);
  int64_t carry = 0;
  for (int p0 = 0; p0 < np; p0 += 64) {
    const int p = p0 + lane;
    int64_t len = 0;   // the pair's e1 segment: the list's length, padded to whole cache lines
    if (p < np) {
      const int l = probes[q * p_stride + p];
      len = (l >= 0 && l < nlist) ? e1_padded(list_len[l]) : 0;
    }
    int64_t inc = len;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int64_t v = __shfl_up(inc, o);
      if (lane >= o) inc += v;
    }
    if (p < np) poff[q * p_stride + p] = carry + inc - len;
    carry += __shfl(inc, 63);
  }
  if (lane == 0) qcnt[q] = carry;
}

// Tile of a list-major workgroup: consecutive workgroups go to the eight XCDs in turn, so XCD x
// takes the x-th contiguous eighth of the tiles; a list's tiles then share one XCD's L2, which
// fetches the slices of the queries probing the list once for all of them.
__device__ inline int64_t xcd_tile() {
  const int64_t n = gridDim.x, wg = blockIdx.x, x = wg % 8, r = wg / 8;
  const int64_t per = n / 8, rem = n % 8;
  return x * per + min(x, rem) + r;
}

// Probed (query, list) pairs grouped by list: count, then scatter after the prefix sum.
__global__ __launch_bounds__(256) void pair_count_kernel(const int32_t *probes, int32_t p_stride,
                                                         const int32_t *nprobe, int32_t nprobe_all,
                                                         int32_t nlist, int64_t nq, int32_t *lcnt,
                                                         int32_t *rank) {
  const int64_t pidx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pidx >= nq * p_stride) return;
  const int64_t q = pidx / p_stride;
  const int p = (int)(pidx - q * p_stride);
  if (p >= min(max(nprobe ? nprobe[q] : nprobe_all, 1), p_stride)) return;
  const int l = probes[pidx];
  if (l >= 0 && l < nlist) rank[pidx] = atomicAdd(&lcnt[l], 1);
}

__global__ __launch_bounds__(256) void pair_scatter_kernel(const int32_t *probes, int32_t p_stride,
                                                           const int32_t *nprobe, int32_t nprobe_all,
                                                           int32_t nlist, int64_t nq, const int32_t *lstart,
                                                           const int32_t *rank, int32_t *lpair) {
  const int64_t pidx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pidx >= nq * p_stride) return;
  const int64_t q = pidx / p_stride;
  const int p = (int)(pidx - q * p_stride);
  if (p >= min(max(nprobe ? nprobe[q] : nprobe_all, 1), p_stride)) return;
  const int l = probes[pidx];
  if (l >= 0 && l < nlist) lpair[lstart[l] + rank[pidx]] = (int32_t)pidx;
}

// In-lane copies of the scan's sums.  The scan spreads a vector's 32-dim slice over G lanes
// (lane j holding dims [j EPL, j EPL + EPL); with the FP8 pre-stage G = 4 lanes of 16 codes) and
// adds the G lane partials with the transposed reduction, whose tree pairs lanes differing in
// bit 2 (G = 8), then in bit 1, then in bit 0: for every vector the sum is
// ((P0 + P4) + (P2 + P6)) + ((P1 + P5) + (P3 + P7)) for G = 8 and (P0 + P2) + (P1 + P3) for
// G = 4 (each addition commutes).  A lane holding the whole slice forms the same partials (the
// same FMA chains in the same order) and adds them in the same tree, so its sum equals the
// scan's bit for bit.
template <int G> __device__ inline float tree_sum(const float (&P)[G]) {
  if constexpr (G == 8) return ((P[0] + P[4]) + (P[2] + P[6])) + ((P[1] + P[5]) + (P[3] + P[7]));
  else return (P[0] + P[2]) + (P[1] + P[3]);
}

// One workgroup per stored tile; lane = stored vector, which stays in registers (dim block 0, or
// with PRE the FP8 codes of the leading 64 dims) while the workgroup takes the (query, list)
// pairs of its list in chunks: first every pair's destination and query slice are staged in LDS
// (independent loads), then the four waves take the chunk's pairs in turn, reading the query
// slice as LDS broadcasts and adding each vector's partials in the scan's tree (no cross-lane
// reduction).
constexpr int kS1Threads = 256;
template <int ST, bool PRE>
__global__ __launch_bounds__(kS1Threads) void stage1_lists_kernel(Stage1Args a) {
  using S = Store<ST>;
  constexpr int EPL = 16 / S::kBytes;
  constexpr int G = PRE ? 4 : kBlockDims / EPL;             // the scan's lanes per slice
  constexpr int NP = PRE ? 16 : EPL;                        // values per lane partial
  constexpr int SLICE = kBlockDims * S::kBytes;
  constexpr int64_t BLOCK_BYTES = (int64_t)kTile * SLICE;
  constexpr int QD = PRE ? kFp8Lead : kBlockDims;           // query dims per pair
  constexpr int CHUNK = PRE ? 32 : 64;                      // pairs staged at once (8 KiB of LDS)
  __shared__ __align__(16) float s_qv[CHUNK * QD];
  __shared__ int64_t s_dst[CHUNK];
  const int64_t t = xcd_tile();
  if (t >= a.total_tiles) return;
  const int l = a.tile_list[t];
  if (l < 0 || l >= a.nlist) return;
  const int pb = a.lstart[l], pe = a.lstart[l + 1];
  if (pb >= pe) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tl = (int)(t - a.tile_off[l]);                 // tile within its list
  const int cnt = min(kTile, a.list_len[l] - tl * kTile);  // stored vectors in this tile
  float f[G][NP];
  float sc = 1.f;
  if constexpr (PRE) {
    sc = a.scale8[t];
    const uint4 *p8 = reinterpret_cast<const uint4 *>(a.base8 + t * (kTile * kFp8Lead) + lane * kFp8Lead);
#pragma unroll
    for (int k = 0; k < G; ++k) {
      const uint4 v = p8[k];
      const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int i = 0; i < 4; ++i) e4m3x4_to_f32(w[i], &f[k][4 * i]);
    }
  } else {
    const uint4 *tp = reinterpret_cast<const uint4 *>(reinterpret_cast<const unsigned char *>(a.base) +
                                                      t * a.nblocks * BLOCK_BYTES + lane * SLICE);
#pragma unroll
    for (int k = 0; k < G; ++k) S::unpack(tp[k], f[k]);
  }
  for (int c0 = pb; c0 < pe; c0 += CHUNK) {
    const int n = min(CHUNK, pe - c0);
    __syncthreads();                 // the previous chunk's slices are no longer read
    for (int j = tid; j < n; j += kS1Threads) {
      const int pidx = a.lpair[c0 + j];
      const int64_t q = pidx / a.p_stride;
      s_dst[j] = a.qoff[q] + a.poff[pidx] + (int64_t)tl * kTile;
    }
    for (int j4 = tid; j4 < n * (QD / 4); j4 += kS1Threads) {
      const int j = j4 / (QD / 4), k4 = j4 % (QD / 4);
      const int64_t q = a.lpair[c0 + j] / a.p_stride;
      reinterpret_cast<float4 *>(s_qv)[j4] = reinterpret_cast<const float4 *>(a.qrot + q * a.q_stride)[k4];
    }
    __syncthreads();
    for (int j = wave; j < n; j += kS1Threads / 64) {
      const float *qs = s_qv + j * QD;
      float P[G];
#pragma unroll
      for (int k = 0; k < G; ++k) {
        float qk[NP];
#pragma unroll
        for (int e4 = 0; e4 < NP / 4; ++e4) {
          const float4 x = *reinterpret_cast<const float4 *>(qs + k * NP + 4 * e4);
          qk[4 * e4] = x.x; qk[4 * e4 + 1] = x.y; qk[4 * e4 + 2] = x.z; qk[4 * e4 + 3] = x.w;
        }
        float acc = 0.f;
#pragma unroll
        for (int e = 0; e < NP; ++e) {
          const float d = PRE ? fp8_term(f[k][e], sc, qk[e]) : f[k][e] - qk[e];
          acc = fmaf(d, d, acc);
        }
        P[k] = acc;
      }
      const float tot = tree_sum<G>(P);
      const int64_t o = s_dst[j] + lane;
      if (lane < cnt && o < a.e1_cap) a.e1[o] = tot;
    }
  }
}

// Pair grouping of both list-major first phases: per-query offsets, then pairs by list.
static void launch_pair_groups(const Stage1Args &a, hipStream_t s) {
  const int64_t npair = a.nq * a.p_stride;
  const unsigned gp = (unsigned)((npair + 255) / 256);
  hipLaunchKernelGGL(fill_i32_kernel, dim3((a.nlist + 256) / 256), dim3(256), 0, s, a.lcnt,
                     (int64_t)a.nlist + 1, 0);
  hipLaunchKernelGGL(pair_offsets_kernel, dim3((unsigned)((a.nq + 3) / 4)), dim3(256), 0, s, a.probes,
                     a.p_stride, a.nprobe, a.nprobe_all, a.list_len, a.nlist, a.nq, a.poff, a.qcnt);
  hipLaunchKernelGGL(excl_prefix_kernel<int64_t>, dim3(1), dim3(kScanPrefixThreads), 0, s, a.qcnt, a.nq,
                     a.qoff);
  hipLaunchKernelGGL(pair_count_kernel, dim3(gp), dim3(256), 0, s, a.probes, a.p_stride, a.nprobe,
                     a.nprobe_all, a.nlist, a.nq, a.lcnt, a.rank);
  hipLaunchKernelGGL(excl_prefix_kernel<int32_t>, dim3(1), dim3(kScanPrefixThreads), 0, s, a.lcnt,
                     (int64_t)a.nlist, a.lstart);
  hipLaunchKernelGGL(pair_scatter_kernel, dim3(gp), dim3(256), 0, s, a.probes, a.p_stride, a.nprobe,
                     a.nprobe_all, a.nlist, a.nq, a.lstart, a.rank, a.lpair);
}

// ---- list-major full-D scan: distances on the matrix cores ----------------------------------

typedef float lm_floatx4 __attribute__((ext_vector_type(4)));

// ||q'||^2 of every rotated query (FP32, dims in order; zero padding beyond D adds nothing)
__global__ __launch_bounds__(256) void qnorm_kernel(const float *qrot, int64_t q_stride, int32_t Dp,
                                                    int64_t nq, float *qnorm) {
  const int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (q >= nq) return;
  float s = 0.f;
  for (int i = lane; i < Dp; i += 64) s = fmaf(qrot[q * q_stride + i], qrot[q * q_stride + i], s);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) qnorm[q] = s;
}

// One workgroup per stored tile: a 64-query x 64-vector block of inner products per chunk of the
// list's pairs, K stepping one 32-dim block at a time through LDS (the tile's block b is a
// row-major 64 x 32 matrix in the packed layout).  Four waves own 32 x 32 quarters, 2 x 2 MFMA
// 16x16 blocks each (A[i][k] at lane i + 16 k, B[k][j] at lane j + 16 k; result lane l, register
// r holds C[4 (l / 16) + r][l % 16]).
constexpr int kLmLd = 36;   // padded LDS row (floats)
template <int ST>
__global__ __launch_bounds__(256) void full_lists_kernel(Stage1Args a, const float *xnorm, const float *qnorm) {
  using S = Store<ST>;
  constexpr int EPL = 16 / S::kBytes;                        // elements per 16-byte load
  constexpr int SLICE = kBlockDims * S::kBytes;
  constexpr int64_t BLOCK_BYTES = (int64_t)kTile * SLICE;
  constexpr int YLOADS = (kTile * kBlockDims / EPL) / 256;  // 16-byte loads per thread per block
  __shared__ __align__(16) float Ys[kTile * kLmLd];
  __shared__ __align__(16) float Qs[kTile * kLmLd];
  __shared__ int64_t s_dst[kTile];
  __shared__ int64_t s_q[kTile];
  __shared__ float s_qn[kTile], s_yn[kTile];
  const int64_t t = xcd_tile();
  if (t >= a.total_tiles) return;
  const int l = a.tile_list[t];
  if (l < 0 || l >= a.nlist) return;
  const int pb = a.lstart[l], pe = a.lstart[l + 1];
  if (pb >= pe) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int tl = (int)(t - a.tile_off[l]);
  const int cnt = min(kTile, a.list_len[l] - tl * kTile);
  const unsigned char *tp = reinterpret_cast<const unsigned char *>(a.base) + t * a.nblocks * BLOCK_BYTES;
  if (tid < kTile) s_yn[tid] = xnorm[t * kTile + tid];
  for (int c0 = pb; c0 < pe; c0 += kTile) {
    const int n = min(kTile, pe - c0);
    __syncthreads();
    if (tid < kTile) {
      int64_t q = 0, dst = 0;
      float qn = 0.f;
      if (tid < n) {
        const int pidx = a.lpair[c0 + tid];
        q = pidx / a.p_stride;
        dst = a.qoff[q] + a.poff[pidx] + (int64_t)tl * kTile;
        qn = qnorm[q];
      }
      s_q[tid] = q;
      s_dst[tid] = dst;
      s_qn[tid] = qn;
    }
    __syncthreads();
    lm_floatx4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = lm_floatx4{0.f, 0.f, 0.f, 0.f};
    for (int b = 0; b < a.nblocks; ++b) {
      // stage the tile's dim block b (as FP32) and the chunk's query slices
#pragma unroll
      for (int it = 0; it < YLOADS; ++it) {
        const int e = (tid + it * 256) * EPL;          // element of the 64 x 32 block
        const int r = e / kBlockDims, c = e % kBlockDims;
        const uint4 v = *reinterpret_cast<const uint4 *>(tp + b * BLOCK_BYTES + (int64_t)e * S::kBytes);
        float f[EPL];
        S::unpack(v, f);
#pragma unroll
        for (int u = 0; u < EPL; u += 4)
          *reinterpret_cast<float4 *>(&Ys[r * kLmLd + c + u]) = make_float4(f[u], f[u + 1], f[u + 2], f[u + 3]);
      }
#pragma unroll
      for (int it = 0; it < 2; ++it) {
        const int e = (tid + it * 256) * 4;
        const int r = e / kBlockDims, c = e % kBlockDims;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (r < n) v = *reinterpret_cast<const float4 *>(a.qrot + s_q[r] * a.q_stride + b * kBlockDims + c);
        *reinterpret_cast<float4 *>(&Qs[r * kLmLd + c]) = v;
      }
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < kBlockDims; kk += 4) {
        float af[2], bf[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) af[i] = Qs[(wr * 32 + i * 16 + (lane & 15)) * kLmLd + kk + (lane >> 4)];
#pragma unroll
        for (int j = 0; j < 2; ++j) bf[j] = Ys[(wc * 32 + j * 16 + (lane & 15)) * kLmLd + kk + (lane >> 4)];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i], bf[j], acc[i][j], 0, 0, 0);
      }
      __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int col = wc * 32 + j * 16 + (lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = wr * 32 + i * 16 + 4 * (lane >> 4) + r;
          if (row < n && col < cnt) {
            const float d = fmaxf(s_qn[row] + s_yn[col] - 2.f * acc[i][j][r], 0.f);
            const int64_t o = s_dst[row] + col;
            if (o < a.e1_cap) a.e1[o] = d;
          }
        }
      }
  }
}

void launch_full_lists(const Stage1Args &a, const float *xnorm, float *qnorm, int store, hipStream_t s) {
  if (a.nq <= 0 || a.total_tiles <= 0) return;
  launch_pair_groups(a, s);
  hipLaunchKernelGGL(qnorm_kernel, dim3((unsigned)((a.nq + 3) / 4)), dim3(256), 0, s, a.qrot, a.q_stride,
                     a.nblocks * kBlockDims, a.nq, qnorm);
  const dim3 grid((unsigned)a.total_tiles), blk(256);
  switch (store) {
    case ST_F32: hipLaunchKernelGGL(full_lists_kernel<ST_F32>, grid, blk, 0, s, a, xnorm, qnorm); break;
    case ST_F16: hipLaunchKernelGGL(full_lists_kernel<ST_F16>, grid, blk, 0, s, a, xnorm, qnorm); break;
    default: hipLaunchKernelGGL(full_lists_kernel<ST_BF16>, grid, blk, 0, s, a, xnorm, qnorm); break;
  }
}

// Stage-1 sums on the matrix cores, in the expanded form (the scan prunes on them only where their
// error bound decides its own test, ScanArgs::e1_tol): one workgroup per stored tile.  The tile's dim block 0 is staged once through LDS with each
// vector's ||y_1||^2 and every wave keeps the MFMA B operand of all 64 vectors in registers;
// the waves then take the list's (query, list) pairs 16 at a time each, with no workgroup
// barrier: a 16 x 64 block of inner products from 4 v_mfma_f32_16x16x4_f32 blocks over 8 K
// steps, and e1 = max(||q'_1||^2 + ||y_1||^2 - 2 <q'_1, y_1>, 0) per pair and vector.  The K
// order is permuted so each lane reads 8 contiguous dims: at step s the lane of K slot k4
// holds dim 8 k4 + s of its row (A: query, B: vector), which leaves every sum unchanged in
// content (A[i][k] at lane i + 16 k, B[k][j] at lane j + 16 k; result lane l, register r holds
// C[4 (l / 16) + r][l % 16]).
// PRE: the FP8 pre-stage's sums over the leading 64 dims instead, from the tile's codes decoded
// as the scan decodes them (code value times the tile's scale, rounded to FP32), 16 K steps.
template <int ST, bool PRE>
__global__ __launch_bounds__(256) void stage1_matrix_kernel(Stage1Args a) {
  using S = Store<ST>;
  constexpr int EPL = 16 / S::kBytes;
  constexpr int YLOADS = (kTile * kBlockDims / EPL) / 256;
  constexpr int SLICE = kBlockDims * S::kBytes;
  constexpr int RW = 16;                          // pairs per wave per round
  constexpr int KD = PRE ? kFp8Lead : kBlockDims; // dims of the first test
  constexpr int KS = KD / 4;                      // K steps; a lane holds KS contiguous dims
  constexpr int LD = PRE ? KD + 4 : kLmLd;        // padded LDS row (floats)
  __shared__ __align__(16) float Ys[kTile * LD];
  __shared__ float s_yn[kTile];
  __shared__ int64_t s_dst[4][RW];
  __shared__ float s_qn[4][RW];
  const int64_t t = xcd_tile();
  if (t >= a.total_tiles) return;
  const int l = a.tile_list[t];
  if (l < 0 || l >= a.nlist) return;
  const int pb = a.lstart[l], pe = a.lstart[l + 1];
  if (pb >= pe) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r16 = lane & 15, k4 = lane >> 4;
  const int tl = (int)(t - a.tile_off[l]);
  const int cnt = min(kTile, a.list_len[l] - tl * kTile);
  if constexpr (PRE) {
    // thread tid decodes codes 16 (tid % 4) .. + 15 of vector tid / 4
    const float sc = a.scale8[t];
    const uint4 v = *reinterpret_cast<const uint4 *>(a.base8 + t * (kTile * kFp8Lead) + tid * 16);
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
    const int r = tid >> 2, c = 16 * (tid & 3);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float f[4];
      e4m3x4_to_f32(w[i], f);
      *reinterpret_cast<float4 *>(&Ys[r * LD + c + 4 * i]) = make_float4(f[0] * sc, f[1] * sc, f[2] * sc, f[3] * sc);
    }
  } else {
    const unsigned char *tp = reinterpret_cast<const unsigned char *>(a.base) +
                              t * a.nblocks * ((int64_t)kTile * SLICE);   // dim block 0 of the tile
#pragma unroll
    for (int it = 0; it < YLOADS; ++it) {
      const int e = (tid + it * 256) * EPL;
      const int r = e / kBlockDims, c = e % kBlockDims;
      const uint4 v = *reinterpret_cast<const uint4 *>(tp + (int64_t)e * S::kBytes);
      float f[EPL];
      S::unpack(v, f);
#pragma unroll
      for (int u = 0; u < EPL; u += 4)
        *reinterpret_cast<float4 *>(&Ys[r * LD + c + u]) = make_float4(f[u], f[u + 1], f[u + 2], f[u + 3]);
    }
  }
  __syncthreads();
  if (tid < kTile) {
    float sq = 0.f;
    for (int k = 0; k < KD; ++k) sq = fmaf(Ys[tid * LD + k], Ys[tid * LD + k], sq);
    s_yn[tid] = sq;
  }
  float bf[KS][4];   // B operand: vector 16 j + r16, dims KS k4 .. KS k4 + KS - 1
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int s8 = 0; s8 < KS; ++s8) bf[s8][j] = Ys[(16 * j + r16) * LD + KS * k4 + s8];
  __syncthreads();
  float yn[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) yn[j] = s_yn[16 * j + r16];
  int64_t *wdst = s_dst[wave];
  float *wqn = s_qn[wave];
  for (int r0 = pb + RW * wave; r0 < pe; r0 += 4 * RW) {
    const int n = min(RW, pe - r0);
    float af[RW / 16][KS];
#pragma unroll
    for (int i = 0; i < RW / 16; ++i) {
      const int row = 16 * i + r16;
      int pidx = 0;
      int64_t q = 0;
      if (row < n) {
        pidx = a.lpair[r0 + row];
        q = pidx / a.p_stride;
      }
      const float4 *qp = reinterpret_cast<const float4 *>(a.qrot + q * a.q_stride + KS * k4);
#pragma unroll
      for (int v4 = 0; v4 < KS / 4; ++v4) {
        const float4 x = row < n ? qp[v4] : make_float4(0.f, 0.f, 0.f, 0.f);
        af[i][4 * v4] = x.x; af[i][4 * v4 + 1] = x.y; af[i][4 * v4 + 2] = x.z; af[i][4 * v4 + 3] = x.w;
      }
      float sq = 0.f;
#pragma unroll
      for (int s8 = 0; s8 < KS; ++s8) sq = fmaf(af[i][s8], af[i][s8], sq);
      sq += __shfl_xor(sq, 16);
      sq += __shfl_xor(sq, 32);
      if (k4 == 0 && row < n) {
        wqn[row] = sq;
        wdst[row] = a.qoff[q] + a.poff[pidx] + (int64_t)tl * kTile;
      }
    }
    __builtin_amdgcn_wave_barrier();
    lm_floatx4 acc[RW / 16][4];
#pragma unroll
    for (int i = 0; i < RW / 16; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = lm_floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s8 = 0; s8 < KS; ++s8)
#pragma unroll
      for (int i = 0; i < RW / 16; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i][s8], bf[s8][j], acc[i][j], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < RW / 16; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * i + 4 * k4 + r;
        if (row < n) {
          const float qn = wqn[row];
          const int64_t o0 = wdst[row];
          const int lim = (int)min<int64_t>(cnt, a.e1_cap - o0);   // vectors of the row to write
          float *rp = a.e1 + o0 + r16;
#pragma unroll
          for (int j = 0; j < 4; ++j)
            if (16 * j + r16 < lim) rp[16 * j] = fmaxf(qn + yn[j] - 2.f * acc[i][j][r], 0.f);
        }
      }
    __builtin_amdgcn_wave_barrier();   // this round's rows are read before the next round's writes
  }
}

void launch_stage1_lists(const Stage1Args &a, int store, hipStream_t s, bool matrix) {
  if (a.nq <= 0 || a.total_tiles <= 0) return;
  launch_pair_groups(a, s);
  const dim3 grid((unsigned)a.total_tiles), blk(kS1Threads);
  if (a.pre) {   // the FP8 codes do not depend on the storage type
    if (matrix)
      hipLaunchKernelGGL((stage1_matrix_kernel<ST_F32, true>), grid, blk, 0, s, a);
    else
      hipLaunchKernelGGL((stage1_lists_kernel<ST_F32, true>), grid, blk, 0, s, a);
    return;
  }
  if (matrix) {
    switch (store) {
      case ST_F32: hipLaunchKernelGGL((stage1_matrix_kernel<ST_F32, false>), grid, blk, 0, s, a); break;
      case ST_F16: hipLaunchKernelGGL((stage1_matrix_kernel<ST_F16, false>), grid, blk, 0, s, a); break;
      default: hipLaunchKernelGGL((stage1_matrix_kernel<ST_BF16, false>), grid, blk, 0, s, a); break;
    }
    return;
  }
  switch (store) {
    case ST_F32: hipLaunchKernelGGL((stage1_lists_kernel<ST_F32, false>), grid, blk, 0, s, a); break;
    case ST_F16: hipLaunchKernelGGL((stage1_lists_kernel<ST_F16, false>), grid, blk, 0, s, a); break;
    default: hipLaunchKernelGGL((stage1_lists_kernel<ST_BF16, false>), grid, blk, 0, s, a); break;
  }
}

// Workgroups of this kernel that fit on the device at once (occupancy x compute units).
static int resident_workgroups(const void *kern, size_t smem, int threads = kScanThreads) {
  static std::mutex mtx;
  static std::map<std::tuple<const void *, size_t, int>, int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) throw std::runtime_error("scan: hipGetDevice failed");
  std::lock_guard<std::mutex> lk(mtx);
  const auto key = std::make_tuple(kern, smem, dev);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, smem) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    throw std::runtime_error("scan: occupancy query failed");
  const int r = std::max(1, per_cu) * std::max(1, cus);
  cache[key] = r;
  return r;
}

size_t scan_lds_request(const ScanArgs &a, int W) {
  return scan_lds_bytes(a.nblocks * kBlockDims, a.k_max, a.block_b, W, a.res != 0,
                        a.pq_m > 0 ? a.pq_m * 256 + a.nblocks * kBlockDims : 0, a.p_stride, a.lag,
                        lag_parallel(a, W));
}

template <int ST, bool P, bool LK, int W, bool PRE = false, bool RES = false, bool EST = false,
          bool PQ = false, bool LG = false, bool LM = false, bool LP = false, int OCC = 4>
static void launch_variant(const ScanArgs &a, hipStream_t s) {
  const size_t smem = scan_lds_bytes(a.nblocks * kBlockDims, a.k_max, a.block_b, W, RES,
                                     PQ ? a.pq_m * 256 + a.nblocks * kBlockDims : 0, a.p_stride,
                                     LG ? a.lag : 0, LP);
  if (smem > kMaxLds) throw std::runtime_error("scan: LDS request exceeds 160 KiB");
  const int qpw = LP ? 1 : 4 / W;
  const int threads = LP ? 64 * W : kScanThreads;   // LP: the query's W waves alone
  const void *kern = reinterpret_cast<const void *>(&scan_kernel<ST, P, LK, W, PRE, RES, EST, PQ, LG, LM, LP, OCC>);
  int64_t grid = (a.nq + qpw - 1) / qpw;
  if (a.queue) {
    // W = 1: each wave takes its own slots, so the grid covers ceil(nq / 4) workgroups at most
    grid = std::min<int64_t>(grid, resident_workgroups(kern, smem, threads));
    hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(64), 0, s, a.queue, (int64_t)1, 0);
  }
  hipLaunchKernelGGL((scan_kernel<ST, P, LK, W, PRE, RES, EST, PQ, LG, LM, LP, OCC>), dim3((unsigned)grid),
                     dim3(threads), smem, s, a);
}

// one pruned kernel; with a lag of at least W - 1 blocks, W = 2 or 4 waves per query scan
// consecutive blocks in parallel (lag-parallel); W = 4 with a shorter lag splits each block's
// tiles instead
template <int ST, bool LK, int W, bool PRE, bool RES, bool PQ, bool LG>
static void launch_pruned_w(const ScanArgs &a, hipStream_t s) {
  if constexpr (LG && W > 1) {
    if (lag_parallel(a, W)) {
      launch_variant<ST, true, LK, W, PRE, RES, false, PQ, true, false, true>(a, s);
      return;
    }
  }
  if constexpr (W == 2) {
    throw std::runtime_error("scan: two waves per query need a lagged threshold");
  } else if constexpr (W == 1 && !RES && !PQ && !LG) {
    if (a.occ5) launch_variant<ST, true, LK, 1, PRE, false, false, false, false, false, false, 5>(a, s);
    else launch_variant<ST, true, LK, 1, PRE, false, false, false, false>(a, s);
  } else {
    launch_variant<ST, true, LK, W, PRE, RES, false, PQ, LG>(a, s);
  }
}

template <int ST, bool LK, bool PRE, bool RES, bool PQ, bool LG>
static void launch_pruned_lk(const ScanArgs &a, hipStream_t s) {
  if (a.waves_per_query == 4) launch_pruned_w<ST, LK, 4, PRE, RES, PQ, LG>(a, s);
  else if (LG && a.waves_per_query == 2) launch_pruned_w<ST, LK, 2, PRE, RES, PQ, LG>(a, s);
  else launch_pruned_w<ST, LK, 1, PRE, RES, PQ, LG>(a, s);
}

// LG: the pruned kernels with a lagged threshold (lag > 0), a separate instantiation so that
// the lag-free kernels carry none of its bookkeeping
template <int ST, bool LG> static void launch_pruned(const ScanArgs &a, hipStream_t s) {
  if (a.pq_m > 0) {
    if (a.lookahead) launch_pruned_lk<ST, true, false, false, true, LG>(a, s);
    else launch_pruned_lk<ST, false, false, false, true, LG>(a, s);
  } else if (a.res) {
    launch_pruned_lk<ST, false, false, true, false, LG>(a, s);
  } else if (a.pre) {
    if (a.lookahead) launch_pruned_lk<ST, true, true, false, false, LG>(a, s);
    else launch_pruned_lk<ST, false, true, false, false, LG>(a, s);
  } else if (a.lookahead) {
    launch_pruned_lk<ST, true, false, false, false, LG>(a, s);
  } else {
    launch_pruned_lk<ST, false, false, false, false, LG>(a, s);
  }
}

template <int ST> static void launch_store(const ScanArgs &a, hipStream_t s) {
  const bool w4 = a.waves_per_query == 4;
  if (a.est_nb > 0) {
    if (w4) launch_variant<ST, false, false, 4, false, false, true>(a, s);
    else launch_variant<ST, false, false, 1, false, false, true>(a, s);
  } else if (!a.prune && a.e1) {
    // the list-major full-D scan's merge: a kernel without the base-reading paths
    if (w4) launch_variant<ST, false, false, 4, false, false, false, false, false, true>(a, s);
    else launch_variant<ST, false, false, 1, false, false, false, false, false, true>(a, s);
  } else if (!a.prune) {
    if (w4) launch_variant<ST, false, false, 4>(a, s); else launch_variant<ST, false, false, 1>(a, s);
  } else if (a.lag > 0) {
    launch_pruned<ST, true>(a, s);
  } else {
    launch_pruned<ST, false>(a, s);
  }
}

void launch_scan(const ScanArgs &a, int store, hipStream_t s) {
  if (a.nq <= 0) return;
  switch (store) {
    case ST_F32: launch_store<ST_F32>(a, s); break;
    case ST_F16: launch_store<ST_F16>(a, s); break;
    default: launch_store<ST_BF16>(a, s); break;
  }
}

}  // namespace ddc
