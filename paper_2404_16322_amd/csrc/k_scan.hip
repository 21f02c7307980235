// Pruned candidate scan, top-K merge and finalize for IVF search on gfx950.
//
// Method (one workgroup of 4 wavefronts per query):
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

// Sum over aligned groups of G lanes with DPP moves (every lane of the group gets the sum).
__device__ inline float dpp_xor1(float v) {  // quad_perm [1,0,3,2]
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));
}
__device__ inline float dpp_xor2(float v) {  // quad_perm [2,3,0,1]
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false));
}
__device__ inline float dpp_half_mirror(float v) {  // lane i <- lane 7-i within 8
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x141, 0xF, 0xF, false));
}
template <int G> __device__ inline float group_sum(float v) {
  v += dpp_xor1(v);
  v += dpp_xor2(v);
  if (G == 8) v += dpp_half_mirror(v);
  return v;
}

__device__ inline bool lex_less(float d, int32_t id, float td, int32_t tid) {
  return d < td || (d == td && id < tid);
}

__device__ inline unsigned long long lane_mask_lt() {
  const int lane = __lane_id();
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

}  // namespace

template <int ST>
__global__ __launch_bounds__(kScanThreads) void scan_kernel(ScanArgs a) {
  using S = Store<ST>;
  constexpr int EPL = 16 / S::kBytes;          // elements per lane load
  constexpr int G = kBlockDims / EPL;          // lanes per vector slice
  constexpr int CPW = 64 / G;                  // slices per wavefront load
  constexpr int MAXCH = kTile / CPW;           // loads to cover a tile
  constexpr int SLICE = kBlockDims * S::kBytes;          // bytes per vector slice
  constexpr int64_t BLOCK_BYTES = (int64_t)kTile * SLICE;  // bytes per tile block

  extern __shared__ __align__(16) unsigned char smem[];
  const int q = blockIdx.x;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int g = lane % G;
  const int sub = lane / G;
  const int nb = a.nblocks;
  const int Dp = nb * kBlockDims;

  // LDS carve-up
  float *s_q = reinterpret_cast<float *>(smem);                       // [Dp]
  float *s_td = s_q + Dp;                                             // [2][kMaxK]
  int32_t *s_ti = reinterpret_cast<int32_t *>(s_td + 2 * kMaxK);      // [2][kMaxK]
  float *s_sd = reinterpret_cast<float *>(s_ti + 2 * kMaxK);          // [block_b]
  int32_t *s_si = reinterpret_cast<int32_t *>(s_sd + a.block_b);      // [block_b]
  uint16_t *s_ac = reinterpret_cast<uint16_t *>(s_si + a.block_b);    // [4][2][64] alive cand
  float *s_ae = reinterpret_cast<float *>(s_ac + 4 * 2 * 64);         // [4][2][64] alive e
  int32_t *s_ctr = reinterpret_cast<int32_t *>(s_ae + 4 * 2 * 64);    // [2] survivor counts
  int32_t *s_stat = s_ctr + 2;                                        // [3 + 64]

  const int K = a.k ? a.k[q] : a.k_all;
  const int np = a.nprobe ? a.nprobe[q] : a.nprobe_all;
  const float *qg = a.qrot + (int64_t)q * a.q_stride;
  for (int i = tid; i < Dp; i += kScanThreads) s_q[i] = qg[i];
  if (tid < 2) s_ctr[tid] = 0;
  for (int i = tid; i < 3 + 64; i += kScanThreads) s_stat[i] = 0;
  __syncthreads();

  // queried lane-private stats
  int st_cand = 0, st_ref = 0, st_slices = 0;

  int tin = 0;         // active queue buffer
  int tn = 0;          // queue size
  float tau = INFINITY;
  int32_t tau_id = 0x7FFFFFFF;
  int par = 0;         // survivor-counter parity
  const bool prune = a.prune != 0;
  const uint16_t *no16 = nullptr;
  (void)no16;

  for (int p = 0; p < np; ++p) {
    const int lst = a.probes[(int64_t)q * a.p_stride + p];
    if (lst < 0 || lst >= a.nlist) continue;  // never follow an invalid list id
    const int len = a.list_len[lst];
    const int64_t tile0 = a.tile_off[lst];
    for (int bs = 0; bs < len; bs += a.block_b) {
      const int blen = min(a.block_b, len - bs);
      const int ntiles = (blen + kTile - 1) / kTile;
      const bool finite = tn == K;   // tau_b < inf
      for (int t = wave; t < ntiles; t += 4) {
        const int64_t tile = tile0 + (bs / kTile) + t;
        const int cnt = min(kTile, blen - t * kTile);
        const unsigned char *tb = reinterpret_cast<const unsigned char *>(a.base) +
                                  tile * (int64_t)nb * BLOCK_BYTES;
        if (!prune || !finite) {
          // ---- every candidate of the tile, every block (no test can prune) ----
          float acc[MAXCH];
#pragma unroll
          for (int c = 0; c < MAXCH; ++c) acc[c] = 0.f;
          const int nch = (cnt + CPW - 1) / CPW;
          for (int b = 0; b < nb; ++b) {
            float qv[EPL];
#pragma unroll
            for (int e = 0; e < EPL; ++e) qv[e] = s_q[b * kBlockDims + g * EPL + e];
            uint4 v[MAXCH];
#pragma unroll
            for (int c = 0; c < MAXCH; ++c)
              if (c < nch)
                v[c] = *reinterpret_cast<const uint4 *>(tb + b * BLOCK_BYTES +
                                                        (c * CPW + sub) * SLICE + g * 16);
#pragma unroll
            for (int c = 0; c < MAXCH; ++c) {
              if (c < nch) {
                float f[EPL];
                S::unpack(v[c], f);
#pragma unroll
                for (int e = 0; e < EPL; ++e) {
                  const float d = f[e] - qv[e];
                  acc[c] = fmaf(d, d, acc[c]);
                }
              }
            }
          }
#pragma unroll
          for (int c = 0; c < MAXCH; ++c) {
            if (c < nch) {
              const float dis = group_sum<G>(acc[c]);
              const int slot = c * CPW + sub;
              if (g == 0 && slot < cnt) {
                const int32_t id = a.ids[tile * kTile + slot];
                if (tn < K || lex_less(dis, id, tau, tau_id)) {
                  const int pos = atomicAdd(&s_ctr[par], 1);
                  s_sd[pos] = dis;
                  s_si[pos] = id;
                }
              }
            }
          }
          if (lane == 0) {
            st_cand += cnt; st_ref += cnt; st_slices += cnt * nb;
            atomicAdd(&s_stat[3 + min(nb - 1, 63)], cnt);
          }
        } else {
          // ---- staged scan with per-stage tests and wavefront compaction ----
          uint16_t *ac = s_ac + wave * 128;
          float *ae = s_ae + wave * 128;
          int cur = 0;
          int nalive = cnt;
          if (lane == 0) st_cand += cnt;
          for (int b = 0; b < nb && nalive > 0; ++b) {
            const bool last = b == nb - 1;
            const bool test = a.test_after[b] != 0;
            const float mb = a.m[b], bb = a.beta[b];
            float qv[EPL];
#pragma unroll
            for (int e = 0; e < EPL; ++e) qv[e] = s_q[b * kBlockDims + g * EPL + e];
            const int nch = (nalive + CPW - 1) / CPW;
            uint4 v[MAXCH];
            int cand[MAXCH];
#pragma unroll
            for (int c = 0; c < MAXCH; ++c) {
              if (c < nch) {
                const int slot = c * CPW + sub;
                const int cd = slot < nalive ? (b == 0 ? slot : (int)ac[cur * 64 + slot]) : 0;
                cand[c] = cd;
                v[c] = *reinterpret_cast<const uint4 *>(tb + b * BLOCK_BYTES + cd * SLICE + g * 16);
              }
            }
            int nnext = 0;
            int pruned_here = 0;
#pragma unroll
            for (int c = 0; c < MAXCH; ++c) {
              if (c < nch) {
                float f[EPL];
                S::unpack(v[c], f);
                float part = 0.f;
#pragma unroll
                for (int e = 0; e < EPL; ++e) {
                  const float d = f[e] - qv[e];
                  part = fmaf(d, d, part);
                }
                part = group_sum<G>(part);
                const int slot = c * CPW + sub;
                const bool valid = slot < nalive;
                const float eprev = (b == 0 || !valid) ? 0.f : ae[cur * 64 + slot];
                const float ev = eprev + part;
                bool keep = valid;
                if (test && valid) keep = !(fmaf(mb, ev, bb) > tau);
                const bool leader = g == 0;
                if (last) {
                  if (leader && keep) {
                    const int32_t id = a.ids[tile * kTile + cand[c]];
                    if (lex_less(ev, id, tau, tau_id)) {
                      const int pos = atomicAdd(&s_ctr[par], 1);
                      s_sd[pos] = ev;
                      s_si[pos] = id;
                    }
                  }
                } else {
                  const unsigned long long bal = __ballot(leader && keep);
                  const int pos = nnext + __popcll(bal & lane_mask_lt());
                  if (leader && keep) {
                    ac[(cur ^ 1) * 64 + pos] = (uint16_t)cand[c];
                    ae[(cur ^ 1) * 64 + pos] = ev;
                  }
                  nnext += __popcll(bal);
                }
                pruned_here += __popcll(__ballot(leader && valid && !keep));
              }
            }
            if (lane == 0) {
              st_slices += nalive;
              if (last) {
                st_ref += nalive - pruned_here;
                atomicAdd(&s_stat[3 + min(b, 63)], nalive - pruned_here);
              }
              if (pruned_here) atomicAdd(&s_stat[3 + min(b, 63)], pruned_here);
            }
            __builtin_amdgcn_wave_barrier();
            if (!last) {
              nalive = nnext;
              cur ^= 1;
            }
          }
        }
      }
      __syncthreads();  // survivors of the block complete
      const int ns = s_ctr[par];
      if (ns > 0) {
        // ---- merge: queue (sorted, tn) + survivors (ns, unsorted) -> K smallest ----
        const float *td = s_td + tin * kMaxK;
        const int32_t *ti = s_ti + tin * kMaxK;
        float *od = s_td + (tin ^ 1) * kMaxK;
        int32_t *oi = s_ti + (tin ^ 1) * kMaxK;
        for (int i = tid; i < tn + ns; i += kScanThreads) {
          float d;
          int32_t id;
          int rank;
          if (i < tn) {
            d = td[i]; id = ti[i];
            rank = i;
          } else {
            d = s_sd[i - tn]; id = s_si[i - tn];
            int lo = 0, hi = tn;           // queue entries smaller than (d, id)
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
      if (tid == 0) s_ctr[par ^ 1] = 0;
      __syncthreads();  // merge complete
      if (ns > 0) {
        tin ^= 1;
        tn = min(K, tn + ns);
      }
      if (tn == K) {
        tau = s_td[tin * kMaxK + K - 1];
        tau_id = s_ti[tin * kMaxK + K - 1];
      }
      par ^= 1;
    }
  }

  // ---- finalize: ascending (dis, id), original ids, padding ----
  const int64_t off = a.out_off ? a.out_off[q] : (int64_t)q * a.k_all;
  for (int i = tid; i < K; i += kScanThreads) {
    const bool have = i < tn;
    a.out_ids[off + i] = have ? (int64_t)s_ti[tin * kMaxK + i] : (int64_t)-1;
    a.out_d[off + i] = have ? s_td[tin * kMaxK + i] : INFINITY;
  }
  if (a.counters) {
    if (lane == 0) {
      atomicAdd(&s_stat[0], st_cand);
      atomicAdd(&s_stat[1], st_ref);
      atomicAdd(&s_stat[2], st_slices);
    }
    __syncthreads();
    for (int i = tid; i < 3 + 64; i += kScanThreads) {
      const int v = s_stat[i];
      if (v) atomicAdd(reinterpret_cast<unsigned long long *>(&a.counters[i < 3 ? i : i + 1]),
                       (unsigned long long)v);
    }
  }
}

size_t scan_smem_bytes(int nblocks, int block_b) {
  const size_t Dp = (size_t)nblocks * kBlockDims;
  return Dp * 4 + 2 * kMaxK * 8 + (size_t)block_b * 8 + 4 * 2 * 64 * 2 + 4 * 2 * 64 * 4 +
         (2 + 3 + 64) * 4;
}

void launch_scan(const ScanArgs &a, int store, hipStream_t s) {
  if (a.nq <= 0) return;
  const size_t smem = scan_smem_bytes(a.nblocks, a.block_b);
  dim3 grid((unsigned)a.nq), block(kScanThreads);
  switch (store) {
    case ST_F32: hipLaunchKernelGGL(scan_kernel<ST_F32>, grid, block, smem, s, a); break;
    case ST_F16: hipLaunchKernelGGL(scan_kernel<ST_F16>, grid, block, smem, s, a); break;
    default: hipLaunchKernelGGL(scan_kernel<ST_BF16>, grid, block, smem, s, a); break;
  }
}

}  // namespace ddc
