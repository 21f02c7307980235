// FP64 kernels of the correction calibration (Sec. V-A: label-0 pairs are the KNN of
// training queries, label-1 pairs are met in a query process; features (dis', tau)).
// FP64 here keeps the calibration's order statistics independent of FP32 rounding.
#include "ddc_internal.h"

#include <hip/hip_fp16.h>

namespace ddc {

namespace {

__device__ inline double elem(const void *base, int store, int64_t idx) {
  if (store == ST_F32) return (double)reinterpret_cast<const float *>(base)[idx];
  const unsigned short h = reinterpret_cast<const unsigned short *>(base)[idx];
  if (store == ST_F16) return (double)__half2float(__ushort_as_half(h));
  return (double)__uint_as_float((uint32_t)h << 16);
}

// element (dim) of the vector in packed slot `slot`
__device__ inline int64_t packed_index(int64_t slot, int nblocks, int dim) {
  const int64_t tile = slot / kTile;
  const int v = (int)(slot % kTile);
  const int b = dim / kBlockDims, d = dim % kBlockDims;
  return ((tile * nblocks + b) * kTile + v) * kBlockDims + d;
}

__device__ inline unsigned long long splitmix64(unsigned long long x) {
  unsigned long long z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ inline bool lex_less64(double d, int32_t id, double td, int32_t tid) {
  return d < td || (d == td && id < tid);
}

}  // namespace

// out[q][i] = sum_j R[i][j] (Q[q][j] - mu[j]), FP64
__global__ void rotate64_kernel(const float *Q, int32_t D, const double *mu, const double *R,
                                double *out) {
  const int64_t q = blockIdx.x;
  for (int i = threadIdx.x; i < D; i += blockDim.x) {
    double s = 0.0;
    for (int j = 0; j < D; ++j) s = fma(R[(int64_t)i * D + j], (double)Q[q * D + j] - mu[j], s);
    out[q * D + i] = s;
  }
}

void launch_rotate64(const float *Q, int64_t nq, int32_t D, const double *mu, const double *R,
                     double *out, hipStream_t s) {
  if (nq <= 0) return;
  hipLaunchKernelGGL(rotate64_kernel, dim3((unsigned)nq), dim3(256), 0, s, Q, D, mu, R, out);
}

// out[q][c] = ||q' - y_slot||^2 in FP64 for slot = slots[q][c] (>= 0)
__global__ void refine64_kernel(const double *qrot, int32_t D, const void *base, int store,
                                int32_t nblocks, const int64_t *slots, int32_t nc, int64_t nq,
                                double *out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nq * nc) return;
  const int64_t q = e / nc;
  const int64_t slot = slots[e];
  if (slot < 0) { out[e] = INFINITY; return; }
  double s = 0.0;
  for (int i = 0; i < D; ++i) {
    const double t = qrot[q * D + i] - elem(base, store, packed_index(slot, nblocks, i));
    s = fma(t, t, s);
  }
  out[e] = s;
}

void launch_refine64(const double *qrot, int32_t D, const void *base, int store, int32_t nblocks,
                     const int64_t *slots, int32_t nc, int64_t nq, double *out, hipStream_t s) {
  const int64_t tot = nq * nc;
  if (tot <= 0) return;
  hipLaunchKernelGGL(refine64_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, qrot, D,
                     base, store, nblocks, slots, nc, nq, out);
}

// out[p][s] = sum_{i < 32 * stage_end_block[s]} (q'_i - y_i)^2 for pair p, FP64
__global__ void features64_kernel(const double *qrot, int32_t D, const void *base, int store,
                                  int32_t nblocks, const int32_t *pair_q, const int64_t *pair_slot,
                                  int64_t npairs, const int32_t *stage_end_block, int32_t n_test,
                                  double *out) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npairs) return;
  const int64_t q = pair_q[p];
  const int64_t slot = pair_slot[p];
  double s = 0.0;
  int i = 0;
  for (int t = 0; t < n_test; ++t) {
    const int end = min(D, stage_end_block[t] * kBlockDims);
    for (; i < end; ++i) {
      const double d = qrot[q * D + i] - elem(base, store, packed_index(slot, nblocks, i));
      s = fma(d, d, s);
    }
    out[p * n_test + t] = s;
  }
}

void launch_features64(const double *qrot, int32_t D, const void *base, int store, int32_t nblocks,
                       const int32_t *pair_q, const int64_t *pair_slot, int64_t npairs,
                       const int32_t *stage_end_block, int32_t n_test, double *out, hipStream_t s) {
  if (npairs <= 0 || n_test <= 0) return;
  hipLaunchKernelGGL(features64_kernel, dim3((unsigned)((npairs + 255) / 256)), dim3(256), 0, s, qrot,
                     D, base, store, nblocks, pair_q, pair_slot, npairs, stage_end_block, n_test, out);
}

__global__ void cdist64_kernel(const double *qrot, int64_t nq, int32_t D, const float *cent,
                               int64_t ldc, int32_t nlist, double *out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nq * nlist) return;
  const int64_t q = e / nlist;
  const int j = (int)(e % nlist);
  double s = 0.0;
  for (int i = 0; i < D; ++i) {
    const double t = qrot[q * D + i] - (double)cent[(int64_t)j * ldc + i];
    s = fma(t, t, s);
  }
  out[e] = s;
}

void launch_cdist64(const double *qrot, int64_t nq, int32_t D, const float *cent, int64_t ldc,
                    int32_t nlist, double *out, hipStream_t s) {
  const int64_t tot = nq * nlist;
  if (tot <= 0) return;
  hipLaunchKernelGGL(cdist64_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, qrot, nq, D,
                     cent, ldc, nlist, out);
}

// One workgroup per calibration query: the unpruned canonical block-synchronous IVF
// search (tau_b = K-th distance after block b - 1 - lag) in FP64.  Every candidate met
// with a finite tau_b and dis > tau_b is label-1 eligible; the max_neg with the smallest
// (SplitMix64 key, id) are kept.
constexpr int kNegThreads = 256;
__global__ __launch_bounds__(kNegThreads) void negatives64_kernel(NegArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int64_t q = blockIdx.x;
  const int tid = threadIdx.x;
  const int D = a.D, K = a.k, B = a.block_b, MN = a.max_neg;
  size_t off = 0;
  auto carve = [&](size_t bytes) {
    unsigned char *p = smem + off;
    off = (off + bytes + 7) & ~(size_t)7;
    return p;
  };
  double *s_q = reinterpret_cast<double *>(carve((size_t)D * 8));                    // [D]
  double *s_td = reinterpret_cast<double *>(carve((size_t)2 * K * 8));               // [2][K]
  int32_t *s_ti = reinterpret_cast<int32_t *>(carve((size_t)2 * K * 4));             // [2][K]
  double *s_bd = reinterpret_cast<double *>(carve((size_t)B * 8));                   // [B]
  int32_t *s_bi = reinterpret_cast<int32_t *>(carve((size_t)B * 4));                 // [B]
  unsigned long long *s_pk = reinterpret_cast<unsigned long long *>(carve((size_t)2 * MN * 8));
  int64_t *s_ps = reinterpret_cast<int64_t *>(carve((size_t)2 * MN * 8));            // slot
  double *s_pt = reinterpret_cast<double *>(carve((size_t)2 * MN * 8));              // tau_b
  int32_t *s_pi = reinterpret_cast<int32_t *>(carve((size_t)2 * MN * 4));            // id
  unsigned long long *s_ek = reinterpret_cast<unsigned long long *>(carve((size_t)B * 8));
  int64_t *s_es = reinterpret_cast<int64_t *>(carve((size_t)B * 8));
  int32_t *s_ei = reinterpret_cast<int32_t *>(carve((size_t)B * 4));
  int32_t *s_ctr = reinterpret_cast<int32_t *>(carve(8));                            // [2]
  double *s_th = reinterpret_cast<double *>(carve((size_t)(a.lag + 1) * 8));         // taus of the last lag + 1 blocks

  for (int i = tid; i < D; i += kNegThreads) s_q[i] = a.qrot[q * D + i];
  if (tid < 2) s_ctr[tid] = 0;
  __syncthreads();

  int tin = 0, tn = 0, pin = 0, pn = 0, bidx = 0;
  double tau = INFINITY;
  for (int p = 0; p < a.nprobe; ++p) {
    const int lst = a.probes[q * a.nprobe + p];
    const int len = a.list_len[lst];
    const int64_t slot0 = (int64_t)a.tile_off[lst] * kTile;
    for (int bs = 0; bs < len; bs += B) {
      const int blen = min(B, len - bs);
      const bool finite = tn == K;
      const double tkd = finite ? s_td[tin * K + K - 1] : INFINITY;
      const int32_t tki = finite ? s_ti[tin * K + K - 1] : 0x7FFFFFFF;
      // tau_b: the tau after block bidx - 1 - lag (+inf before it or while that queue held < K)
      double tau_b = tau;
      if (a.lag > 0) {
        const int j = bidx - 1 - a.lag;
        tau_b = j >= 0 ? s_th[j % (a.lag + 1)] : INFINITY;
      }
      const bool fin_b = tau_b < INFINITY;
      const bool pfull = pn == MN;
      const unsigned long long pkk = pfull ? s_pk[pin * MN + MN - 1] : ~0ull;
      const int32_t pki = pfull ? s_pi[pin * MN + MN - 1] : 0x7FFFFFFF;
      for (int v = tid; v < blen; v += kNegThreads) {
        const int64_t slot = slot0 + bs + v;
        double s = 0.0;
        for (int i = 0; i < D; ++i) {
          const double t = s_q[i] - elem(a.base, a.store, packed_index(slot, a.nblocks, i));
          s = fma(t, t, s);
        }
        const int32_t id = a.ids[slot];
        if (!finite || lex_less64(s, id, tkd, tki)) {
          const int pos = atomicAdd(&s_ctr[0], 1);
          s_bd[pos] = s; s_bi[pos] = id;
        }
        if (fin_b && s > tau_b) {
          const unsigned long long key =
              splitmix64(a.key_base + (((unsigned long long)q << 32) + (unsigned long long)(uint32_t)id));
          if (!pfull || key < pkk || (key == pkk && id < pki)) {
            const int pos = atomicAdd(&s_ctr[1], 1);
            s_ek[pos] = key; s_es[pos] = slot; s_ei[pos] = id;
          }
        }
      }
      __syncthreads();
      const int nb = s_ctr[0], ne = s_ctr[1];
      // queue merge by (dis, id)
      for (int i = tid; i < tn + nb; i += kNegThreads) {
        double d; int32_t id; int r;
        if (i < tn) { d = s_td[tin * K + i]; id = s_ti[tin * K + i]; r = i; }
        else {
          d = s_bd[i - tn]; id = s_bi[i - tn]; r = 0;
          for (int t = 0; t < tn; ++t) r += lex_less64(s_td[tin * K + t], s_ti[tin * K + t], d, id);
        }
        for (int t = 0; t < nb; ++t) r += lex_less64(s_bd[t], s_bi[t], d, id);
        if (r < K) { s_td[(tin ^ 1) * K + r] = d; s_ti[(tin ^ 1) * K + r] = id; }
      }
      // label-1 pool merge by (key, id)
      for (int i = tid; i < pn + ne; i += kNegThreads) {
        unsigned long long k; int64_t sl; int32_t id; double tb; int r;
        if (i < pn) {
          k = s_pk[pin * MN + i]; sl = s_ps[pin * MN + i]; id = s_pi[pin * MN + i];
          tb = s_pt[pin * MN + i]; r = i;
        } else {
          k = s_ek[i - pn]; sl = s_es[i - pn]; id = s_ei[i - pn]; tb = tau_b; r = 0;
          for (int t = 0; t < pn; ++t) {
            const unsigned long long o = s_pk[pin * MN + t];
            r += o < k || (o == k && s_pi[pin * MN + t] < id);
          }
        }
        for (int t = 0; t < ne; ++t) r += s_ek[t] < k || (s_ek[t] == k && s_ei[t] < id);
        if (r < MN) {
          s_pk[(pin ^ 1) * MN + r] = k; s_ps[(pin ^ 1) * MN + r] = sl;
          s_pi[(pin ^ 1) * MN + r] = id; s_pt[(pin ^ 1) * MN + r] = tb;
        }
      }
      __syncthreads();
      if (nb > 0) { tin ^= 1; tn = min(K, tn + nb); }
      if (ne > 0) { pin ^= 1; pn = min(MN, pn + ne); }
      if (tn == K) tau = s_td[tin * K + K - 1];
      if (tid == 0) {
        s_ctr[0] = 0; s_ctr[1] = 0;
        if (a.lag > 0) s_th[bidx % (a.lag + 1)] = tn == K ? tau : INFINITY;
      }
      ++bidx;
      __syncthreads();
    }
  }
  for (int i = tid; i < MN; i += kNegThreads) {
    a.neg_slot[q * MN + i] = i < pn ? s_ps[pin * MN + i] : -1;
    a.neg_tau[q * MN + i] = i < pn ? s_pt[pin * MN + i] : 0.0;
  }
}

size_t negatives_smem(int D, int K, int B, int MN, int lag) {
  auto r8 = [](size_t b) { return (b + 7) & ~(size_t)7; };
  return r8((size_t)D * 8) + r8((size_t)2 * K * 8) + r8((size_t)2 * K * 4) + r8((size_t)B * 8) +
         r8((size_t)B * 4) + 3 * r8((size_t)2 * MN * 8) + r8((size_t)2 * MN * 4) +
         2 * r8((size_t)B * 8) + r8((size_t)B * 4) + 8 + r8((size_t)(lag + 1) * 8);
}

void launch_negatives64(const NegArgs &a, hipStream_t s) {
  if (a.nq <= 0) return;
  const size_t smem = negatives_smem(a.D, a.k, a.block_b, a.max_neg, a.lag);
  hipLaunchKernelGGL(negatives64_kernel, dim3((unsigned)a.nq), dim3(kNegThreads), smem, s, a);
}

}  // namespace ddc
