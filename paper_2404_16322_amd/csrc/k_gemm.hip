// Dense products on the gfx950 matrix cores.
//
// The query rotation q' = R (q - mu) (Sec. IV-B; Eq. (1) rotates both sides) is a
// GEMM  Q' = (Q - mu) R^T  with FP32 accumulation.  The same kernel computes the
// coarse distances of the IVF probe step (Sec. II-A, IVF: nearest centroids first)
// as  ||c_j||^2 - 2 <q', c_j>  (the per-query constant ||q'||^2 does not change the
// order) and, for k-means, the per-row argmin of that quantity.
//
// Tiling: 64 x 64 output tile per workgroup of 4 wavefronts, each wavefront owns a
// 32 x 32 quarter = 2 x 2 MFMA 16x16 blocks; K advances 32 at a time through LDS.
//   FP32: v_mfma_f32_16x16x4_f32  (A[i][k] at lane i + 16 k; B[k][j] at lane j + 16 k)
//   BF16: v_mfma_f32_16x16x32_bf16 (8 consecutive k per lane, lane groups of 16 by k/8)
//   result: lane l, register r holds C[4 (l / 16) + r][l % 16].
#include "ddc_internal.h"

namespace ddc {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int BM = 64, BN = 64, BK = 32;
constexpr int LDA = BK + 4;  // padded LDS row (floats)

__device__ inline uint32_t f32_order_key(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ inline unsigned short bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

}  // namespace

__global__ __launch_bounds__(256) void gemm_nt_kernel(GemmArgs g) {
  __shared__ __align__(16) float As[BM * LDA];
  __shared__ __align__(16) float Bs[BN * LDA];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int64_t m0 = (int64_t)blockIdx.y * BM;
  const int n0 = blockIdx.x * BN;

  floatx4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  for (int k0 = 0; k0 < g.K; k0 += BK) {
    // stage A (minus mu) and B tiles: 64 rows x 32 k, 8 elements per thread each
    const bool vec = (g.lda % 4 == 0) && (g.ldb % 4 == 0) && (k0 + BK <= g.K);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      const int e = tid + it * 256;       // 0..511 -> (row, k4)
      const int r = e >> 3;
      const int kc = (e & 7) * 4;
      const int64_t gm = m0 + r;
      const int gn = n0 + r;
      float4 av = make_float4(0.f, 0.f, 0.f, 0.f), bv = av;
      if (vec) {
        if (gm < g.M) {
          av = *reinterpret_cast<const float4 *>(g.A + gm * g.lda + k0 + kc);
          if (g.mu) {
            const float4 mv = *reinterpret_cast<const float4 *>(g.mu + k0 + kc);
            av.x -= mv.x; av.y -= mv.y; av.z -= mv.z; av.w -= mv.w;
          }
        }
        if (gn < g.N) bv = *reinterpret_cast<const float4 *>(g.B + (int64_t)gn * g.ldb + k0 + kc);
      } else {
        float ta[4], tb[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int k = k0 + kc + t;
          float x = 0.f, y = 0.f;
          if (k < g.K) {
            if (gm < g.M) x = g.A[gm * g.lda + k] - (g.mu ? g.mu[k] : 0.f);
            if (gn < g.N) y = g.B[(int64_t)gn * g.ldb + k];
          }
          ta[t] = x; tb[t] = y;
        }
        av = make_float4(ta[0], ta[1], ta[2], ta[3]);
        bv = make_float4(tb[0], tb[1], tb[2], tb[3]);
      }
      *reinterpret_cast<float4 *>(&As[r * LDA + kc]) = av;
      *reinterpret_cast<float4 *>(&Bs[r * LDA + kc]) = bv;
    }
    __syncthreads();
    if (g.prec == 0) {
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        float af[2], bf[2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
          af[i] = As[(wr * 32 + i * 16 + (lane & 15)) * LDA + kk + (lane >> 4)];
#pragma unroll
        for (int j = 0; j < 2; ++j)
          bf[j] = Bs[(wc * 32 + j * 16 + (lane & 15)) * LDA + kk + (lane >> 4)];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i], bf[j], acc[i][j], 0, 0, 0);
      }
    } else {
      bf16x8 af[2], bf[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const float *src = &As[(wr * 32 + i * 16 + (lane & 15)) * LDA + 8 * (lane >> 4)];
        unsigned short h[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) h[t] = bf16_rne(src[t]);
        af[i] = *reinterpret_cast<const bf16x8 *>(h);
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const float *src = &Bs[(wc * 32 + j * 16 + (lane & 15)) * LDA + 8 * (lane >> 4)];
        unsigned short h[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) h[t] = bf16_rne(src[t]);
        bf[j] = *reinterpret_cast<const bf16x8 *>(h);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }

  // epilogue
#pragma unroll
  for (int i = 0; i < 2; ++i) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = n0 + wc * 32 + j * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = m0 + wr * 32 + i * 16 + 4 * (lane >> 4) + r;
        const float v = acc[i][j][r];
        if (g.mode == 2) {
          // row-wise argmin of bias[n] - 2 v, ties to the lower column
          float d = INFINITY;
          if (row < g.M && col < g.N) d = g.bias[col] - 2.f * v;
          unsigned long long key = ((unsigned long long)f32_order_key(d) << 32) | (uint32_t)col;
          // reduce over the 16 columns held by lanes of the same row group
#pragma unroll
          for (int off = 1; off < 16; off <<= 1) {
            const unsigned long long o = __shfl_xor(key, off);
            key = o < key ? o : key;
          }
          if ((lane & 15) == 0 && row < g.M) atomicMin(&g.key64[row], key);
        } else if (row < g.M && col < g.N) {
          g.C[row * g.ldc + col] = g.mode == 1 ? g.bias[col] - 2.f * v : v;
        }
      }
    }
  }
}

void launch_gemm(const GemmArgs &g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return;
  dim3 grid((g.N + BN - 1) / BN, (unsigned)((g.M + BM - 1) / BM));
  hipLaunchKernelGGL(gemm_nt_kernel, grid, dim3(256), 0, s, g);
}

// ------------------------------------------------------------------------------------
// Probe selection: radix select of the nprobe-th smallest (value, index) key, ordered
// gather, then a rank sort of the selected items.  One workgroup per query.
// ------------------------------------------------------------------------------------
constexpr int kSelThreads = 256;

__device__ inline int wave_incl_scan(int v) {
  const int lane = __lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(v, o);
    if (lane >= o) v += t;
  }
  return v;
}

// Exclusive prefix of one int per thread over the workgroup, in thread order; also the total.
__device__ inline int block_excl_scan(int v, int *wsum, int &total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int inc = wave_incl_scan(v);
  if (lane == 63) wsum[wave] = inc;
  __syncthreads();
  int before = 0;
  total = 0;
#pragma unroll
  for (int w = 0; w < kSelThreads / 64; ++w) {
    const int x = wsum[w];
    if (w < wave) before += x;
    total += x;
  }
  __syncthreads();
  return before + inc - v;
}

__global__ __launch_bounds__(kSelThreads) void select_kernel(const float *dist, int64_t ld,
                                                             int32_t nlist, const int32_t *nprobe,
                                                             int32_t nprobe_all, int32_t *probes,
                                                             int32_t p_stride) {
  extern __shared__ __align__(16) unsigned char smem[];
  int32_t *hist = reinterpret_cast<int32_t *>(smem);           // [256]
  int32_t *wsum = hist + 256;                                    // [4]
  int32_t *sh = wsum + 4;                                        // [4]
  uint32_t *sel_k = reinterpret_cast<uint32_t *>(sh + 4);        // [p_stride]
  int32_t *sel_j = reinterpret_cast<int32_t *>(sel_k + p_stride);  // [p_stride]

  const int64_t q = blockIdx.x;
  const int tid = threadIdx.x;
  const int np = nprobe ? nprobe[q] : nprobe_all;
  const float *row = dist + q * ld;

  // radix select (8 bits per pass, most significant first) of the np-th smallest key
  uint32_t prefix = 0, mask = 0;
  int kk = np;
  for (int shift = 24; shift >= 0; shift -= 8) {
    hist[tid] = 0;
    __syncthreads();
    for (int j = tid; j < nlist; j += kSelThreads) {
      const uint32_t u = f32_order_key(row[j]);
      if ((u & mask) == prefix) atomicAdd(&hist[(u >> shift) & 255], 1);
    }
    __syncthreads();
    if (tid < 64) {   // one wavefront finds the bucket holding rank kk
      const int h0 = hist[4 * tid], h1 = hist[4 * tid + 1], h2 = hist[4 * tid + 2], h3 = hist[4 * tid + 3];
      const int inc = wave_incl_scan(h0 + h1 + h2 + h3);
      const int exc = inc - (h0 + h1 + h2 + h3);
      if (exc < kk && kk <= inc) {
        int c = exc, d = 4 * tid;
        if (c + h0 < kk) { c += h0; ++d;
          if (c + h1 < kk) { c += h1; ++d;
            if (c + h2 < kk) { c += h2; ++d; } } }
        sh[0] = d;
        sh[1] = kk - c;
      }
    }
    __syncthreads();
    prefix |= (uint32_t)sh[0] << shift;
    mask |= 255u << shift;
    kk = sh[1];
    __syncthreads();
  }
  // prefix = threshold key; take every key < prefix and the first kk (by index) == prefix,
  // in index order via exclusive scans over contiguous per-thread index ranges.
  const int chunk = (nlist + kSelThreads - 1) / kSelThreads;
  const int jb = tid * chunk, je = min(nlist, jb + chunk);
  int nless = 0, neq = 0;
  for (int j = jb; j < je; ++j) {
    const uint32_t u = f32_order_key(row[j]);
    nless += u < prefix;
    neq += u == prefix;
  }
  int total_less;
  int pl = block_excl_scan(nless, wsum, total_less);
  int total_eq;
  int pe = block_excl_scan(neq, wsum, total_eq);
  for (int j = jb; j < je; ++j) {
    const uint32_t u = f32_order_key(row[j]);
    if (u < prefix) {
      sel_k[pl] = u; sel_j[pl] = j; ++pl;
    } else if (u == prefix) {
      if (pe < kk) { sel_k[total_less + pe] = u; sel_j[total_less + pe] = j; }
      ++pe;
    }
  }
  __syncthreads();
  // rank sort of the np selected by (key, index)
  for (int i = tid; i < np; i += kSelThreads) {
    const uint32_t u = sel_k[i];
    const int j = sel_j[i];
    int r = 0;
    for (int t = 0; t < np; ++t) {
      const uint32_t v = sel_k[t];
      r += (v < u) || (v == u && sel_j[t] < j);
    }
    probes[q * p_stride + r] = j;
  }
}

void launch_select(const float *dist, int64_t ld, int32_t nlist, const int32_t *nprobe,
                   int32_t nprobe_all, int32_t nprobe_max, int32_t *probes, int32_t p_stride,
                   int64_t nq, hipStream_t s) {
  if (nq <= 0) return;
  const size_t smem = (256 + 4 + 4) * 4 + (size_t)p_stride * 8;
  hipLaunchKernelGGL(select_kernel, dim3((unsigned)nq), dim3(kSelThreads), smem, s, dist, ld, nlist,
                     nprobe, nprobe_all, probes, p_stride);
  (void)nprobe_max;
}

}  // namespace ddc
