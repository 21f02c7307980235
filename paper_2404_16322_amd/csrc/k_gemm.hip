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

#include <cstdint>
#include <map>
#include <mutex>
#include <stdexcept>

namespace ddc {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int BK = 32;
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

// PD: K steps whose global loads are in flight at once (PD register sets).  Tile t is stored to
// LDS stage t & 1 while the loads of tiles t + 1 .. t + PD are in flight, so one barrier per K
// step suffices (stage t & 1 was last read in step t - 2).  PD = 1 for grids that fill the chip;
// a grid of at most one workgroup per compute unit walks its K steps one after another, and PD =
// 3 keeps three steps' loads in flight.  The products and their order do not depend on PD.
// VEC: every K step is a full 32-wide tile of 16-byte aligned rows (the host checks lda, ldb, K
// and the base pointers), so each thread's loads are four float4 loads with only a row mask;
// otherwise every element is loaded on its own with a K mask.
// WT: MFMA 16x16 blocks per wave in each dimension; the workgroup's four waves (2 x 2) cover a
// TB x TB output tile, TB = 32 WT (64 for WT = 2; 128 for WT = 4, half the global and LDS
// traffic per product, taken for FP32 products with K >= 512 and at least two workgroups per
// compute unit: measured 11% faster at K = 768, equal at K = 256, 13% slower at K = 128).
// GEN: any operands (A - mu when g.mu is set, BF16 products when g.prec = 1); false: the host
// guarantees g.mu == NULL and g.prec == 0, and neither costs registers.
template <int PD, bool VEC, int WT, bool GEN>
__global__ __launch_bounds__(256) void gemm_nt_kernel(GemmArgs g) {
  constexpr int TB = 32 * WT;        // output tile rows = columns
  constexpr int NIT = TB / 32;       // float4 loads per thread per operand and K step
  extern __shared__ __align__(16) float gemm_lds[];   // As[2][TB * LDA], Bs[2][TB * LDA]
  float *const As0 = gemm_lds, *const Bs0 = gemm_lds + 2 * TB * LDA;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int64_t m0 = (int64_t)blockIdx.y * TB;
  const int n0 = blockIdx.x * TB;

  floatx4 acc[WT][WT];
#pragma unroll
  for (int i = 0; i < WT; ++i)
#pragma unroll
    for (int j = 0; j < WT; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  // A, mu and B tiles: TB rows x 32 k each, TB / 8 elements per thread each.  The loads only
  // fill registers; A - mu is formed when the tile is stored to LDS, so no load is waited for
  // before its tile's turn
  float4 ra[PD][NIT], rm[PD][NIT], rb[PD][NIT];
  auto load_tile = [&](float4 (&ra_)[NIT], float4 (&rm_)[NIT], float4 (&rb_)[NIT], int k0) {
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int e = tid + it * 256;       // 0..511 -> (row, k4)
      const int r = e >> 3;
      const int kc = (e & 7) * 4;
      const int64_t gm = m0 + r;
      const int gn = n0 + r;
      float4 av = make_float4(0.f, 0.f, 0.f, 0.f), mv = av, bv = av;
      if (VEC) {
        if (gm < g.M) {
          av = *reinterpret_cast<const float4 *>(g.A + gm * g.lda + k0 + kc);
          if (GEN && g.mu) mv = *reinterpret_cast<const float4 *>(g.mu + k0 + kc);
        }
        if (gn < g.N) bv = *reinterpret_cast<const float4 *>(g.B + (int64_t)gn * g.ldb + k0 + kc);
      } else {
        float ta[4], tm[4], tb[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int k = k0 + kc + t;
          float x = 0.f, m = 0.f, y = 0.f;
          if (k < g.K) {
            if (gm < g.M) {
              x = g.A[gm * g.lda + k];
              if (GEN && g.mu) m = g.mu[k];
            }
            if (gn < g.N) y = g.B[(int64_t)gn * g.ldb + k];
          }
          ta[t] = x; tm[t] = m; tb[t] = y;
        }
        av = make_float4(ta[0], ta[1], ta[2], ta[3]);
        mv = make_float4(tm[0], tm[1], tm[2], tm[3]);
        bv = make_float4(tb[0], tb[1], tb[2], tb[3]);
      }
      ra_[it] = av;
      rm_[it] = mv;
      rb_[it] = bv;
    }
  };

#pragma unroll
  for (int u = 0; u < PD; ++u)
    if (u * BK < g.K) load_tile(ra[u], rm[u], rb[u], u * BK);
  // register set u holds tile t with t % PD == u: the inner loop is unrolled, so every set is
  // addressed statically and stays in registers
  for (int kb = 0; kb < g.K; kb += PD * BK) {
#pragma unroll
  for (int u = 0; u < PD; ++u) {
    const int k0 = kb + u * BK;
    if (k0 >= g.K) break;
    const int stage = (k0 / BK) & 1;
    float *as = As0 + stage * TB * LDA;
    float *bs = Bs0 + stage * TB * LDA;
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int e = tid + it * 256;
      const int r = e >> 3;
      const int kc = (e & 7) * 4;
      float4 av = ra[u][it];
      if (GEN && g.mu) {
        const float4 mv = rm[u][it];
        av.x -= mv.x; av.y -= mv.y; av.z -= mv.z; av.w -= mv.w;
      }
      *reinterpret_cast<float4 *>(&as[r * LDA + kc]) = av;
      *reinterpret_cast<float4 *>(&bs[r * LDA + kc]) = rb[u][it];
    }
    __syncthreads();
    // tile t + PD's loads overlap the products of tiles t .. t + PD - 1
    if (k0 + PD * BK < g.K) load_tile(ra[u], rm[u], rb[u], k0 + PD * BK);
    if (!GEN || g.prec == 0) {
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        float af[WT], bf[WT];
#pragma unroll
        for (int i = 0; i < WT; ++i)
          af[i] = as[(wr * 16 * WT + i * 16 + (lane & 15)) * LDA + kk + (lane >> 4)];
#pragma unroll
        for (int j = 0; j < WT; ++j)
          bf[j] = bs[(wc * 16 * WT + j * 16 + (lane & 15)) * LDA + kk + (lane >> 4)];
#pragma unroll
        for (int i = 0; i < WT; ++i)
#pragma unroll
          for (int j = 0; j < WT; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i], bf[j], acc[i][j], 0, 0, 0);
      }
    } else if constexpr (GEN) {
      bf16x8 af[WT], bf[WT];
#pragma unroll
      for (int i = 0; i < WT; ++i) {
        const float *src = &as[(wr * 16 * WT + i * 16 + (lane & 15)) * LDA + 8 * (lane >> 4)];
        unsigned short h[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) h[t] = bf16_rne(src[t]);
        af[i] = *reinterpret_cast<const bf16x8 *>(h);
      }
#pragma unroll
      for (int j = 0; j < WT; ++j) {
        const float *src = &bs[(wc * 16 * WT + j * 16 + (lane & 15)) * LDA + 8 * (lane >> 4)];
        unsigned short h[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) h[t] = bf16_rne(src[t]);
        bf[j] = *reinterpret_cast<const bf16x8 *>(h);
      }
#pragma unroll
      for (int i = 0; i < WT; ++i)
#pragma unroll
        for (int j = 0; j < WT; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
  }
  }

  // epilogue
#pragma unroll
  for (int i = 0; i < WT; ++i) {
#pragma unroll
    for (int j = 0; j < WT; ++j) {
      const int col = n0 + wc * 16 * WT + j * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = m0 + wr * 16 * WT + i * 16 + 4 * (lane >> 4) + r;
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

// compute units of the current device (cached per device)
static int device_cus() {
  static std::mutex mtx;
  static std::map<int, int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) throw std::runtime_error("gemm: hipGetDevice failed");
  std::lock_guard<std::mutex> lk(mtx);
  auto it = cache.find(dev);
  if (it != cache.end()) return it->second;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    throw std::runtime_error("gemm: device query failed");
  cache[dev] = cus;
  return cus;
}

void launch_gemm(const GemmArgs &g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return;
  auto grid_for = [&](int tb) { return dim3((g.N + tb - 1) / tb, (unsigned)((g.M + tb - 1) / tb)); };
  auto lds = [](int tb) { return (size_t)4 * 2 * 2 * tb * LDA; };
  auto al16 = [](const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
  const bool vec = g.lda % 4 == 0 && g.ldb % 4 == 0 && g.K % BK == 0 && al16(g.A) && al16(g.B) &&
                   (g.mu == nullptr || al16(g.mu));
  const dim3 g64 = grid_for(64), g128 = grid_for(128);
  const int cus = device_cus();
  if (!vec)
    hipLaunchKernelGGL((gemm_nt_kernel<1, false, 2, true>), g64, dim3(256), lds(64), s, g);
  else if ((int64_t)g64.x * g64.y <= cus)
    hipLaunchKernelGGL((gemm_nt_kernel<3, true, 2, true>), g64, dim3(256), lds(64), s, g);
  else if (g.mu == nullptr && g.prec == 0 && g.K >= 512 && (int64_t)g128.x * g128.y >= 2 * cus)
    hipLaunchKernelGGL((gemm_nt_kernel<1, true, 4, false>), g128, dim3(256), lds(128), s, g);
  else
    hipLaunchKernelGGL((gemm_nt_kernel<1, true, 2, true>), g64, dim3(256), lds(64), s, g);
}

// ------------------------------------------------------------------------------------
// Probe selection: the nprobe smallest (distance, list) pairs of a query, ascending.
// One wavefront per query (four per workgroup).  A threshold from the lanes' smallest keys
// gathers the candidates in one pass when few enough pass it; otherwise a radix select on
// the order-preserving 32-bit key of the distance, whose first 8-bit digit starts at the highest bit where the
// row's smallest and largest keys differ (so the first histogram is spread over the whole
// range); passes stop once the bucket holding the remaining rank has at most kExtra keys,
// or on the last digit (then every key in it is equal and index order decides).  The
// chosen keys are rank-sorted by (key, index).
// ------------------------------------------------------------------------------------
constexpr int kSelThreads = 256;
constexpr int kExtra = 64;

__device__ inline int wave_incl_scan(int v) {
  const int lane = __lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(v, o);
    if (lane >= o) v += t;
  }
  return v;
}

__device__ inline uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, o));
  return v;
}
__device__ inline uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o));
  return v;
}

__host__ __device__ inline size_t select_wave_lds(int p_stride) { return 256 * 4 + (size_t)(p_stride + kExtra) * 8; }

// The np-th smallest (np <= 64 RR) of the union of every lane's RR smallest keys: the lanes'
// keys are passed through `each`, the RR smallest kept sorted in v, then the 64 RR kept keys
// (key r * 64 + lane in register r of that lane) are bitonic-sorted across the wavefront.
template <int RR, typename Each>
__device__ inline uint32_t lane_union_threshold(Each &&each, int np) {
  uint32_t v[RR];
#pragma unroll
  for (int r = 0; r < RR; ++r) v[r] = 0xFFFFFFFFu;
  each([&](int, uint32_t x) {
#pragma unroll
    for (int m = 0; m < RR; ++m) {
      const uint32_t lo = min(v[m], x);
      x = max(v[m], x);
      v[m] = lo;
    }
  });
  const int lane = __lane_id();
#pragma unroll
  for (int size = 2; size <= 64 * RR; size <<= 1) {
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      if (stride >= 64) {
        const int rs = stride >> 6;
#pragma unroll
        for (int r = 0; r < RR; ++r) {
          if (r & rs) continue;
          const bool up = ((r * 64) & size) == 0;
          const uint32_t lo = min(v[r], v[r | rs]), hi = max(v[r], v[r | rs]);
          v[r] = up ? lo : hi;
          v[r | rs] = up ? hi : lo;
        }
      } else {
#pragma unroll
        for (int r = 0; r < RR; ++r) {
          const uint32_t o = (uint32_t)__shfl_xor((int)v[r], stride);
          const bool up = ((r * 64 + lane) & size) == 0;
          const bool lower = (lane & stride) == 0;
          v[r] = (lower == up) ? min(v[r], o) : max(v[r], o);
        }
      }
    }
  }
  const int e = np - 1, er = e >> 6;
  uint32_t pick = v[0];
#pragma unroll
  for (int r = 1; r < RR; ++r)
    if (er == r) pick = v[r];
  return (uint32_t)__shfl((int)pick, e & 63);
}

// NR > 0: the row's keys stay in registers (key j in register j / 64 of lane j % 64), read
// from memory once; NR = 0: every pass re-reads the row (any nlist).
template <int NR>
__global__ __launch_bounds__(kSelThreads) void select_kernel(const float *dist, int64_t ld,
                                                             int32_t nlist, const int32_t *nprobe,
                                                             int32_t nprobe_all, int32_t *probes,
                                                             int32_t p_stride, int64_t nq) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t q = (int64_t)blockIdx.x * (kSelThreads / 64) + wave;
  if (q >= nq) return;
  unsigned char *wl = smem + (size_t)wave * select_wave_lds(p_stride);
  int32_t *hist = reinterpret_cast<int32_t *>(wl);
  // selected (key, index) pairs packed as key << 32 | index: one 64-bit compare orders them
  unsigned long long *sel = reinterpret_cast<unsigned long long *>(wl + 256 * 4);
  // a per-query count outside [1, min(p_stride, nlist)] is clamped to it (device arrays are
  // the caller's: an entry past the probe row would write past it)
  const int np = min(max(nprobe ? nprobe[q] : nprobe_all, 1), min(p_stride, nlist));
  const float *row = dist + q * ld;
  const unsigned long long lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));

  constexpr int R = NR > 0 ? NR : 1;
  uint32_t ureg[R];
  if constexpr (NR > 0) {
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int j = lane + 64 * i;
      ureg[i] = j < nlist ? f32_order_key(row[j]) : 0xFFFFFFFFu;
    }
  }
  // f(j, key) for this lane's keys
  auto each = [&](auto &&f) {
    if constexpr (NR > 0) {
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const int j = lane + 64 * i;
        if (j < nlist) f(j, ureg[i]);
      }
    } else {
      // 16 loads in flight per lane before any of them is used
      for (int j0 = lane; j0 < nlist; j0 += 64 * 16) {
        float v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) v[u] = j0 + 64 * u < nlist ? row[j0 + 64 * u] : 0.f;
#pragma unroll
        for (int u = 0; u < 16; ++u)
          if (j0 + 64 * u < nlist) f(j0 + 64 * u, f32_order_key(v[u]));
      }
    }
  };
  // f(j, key, valid) for every group of 64 consecutive keys, all lanes together
  auto each_group = [&](auto &&f) {
    if constexpr (NR > 0) {
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const int j = lane + 64 * i;
        f(j, ureg[i], j < nlist);
      }
    } else {
      for (int g0 = 0; g0 < nlist; g0 += 64 * 16) {
        float v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int j = g0 + 64 * u + lane;
          v[u] = j < nlist ? row[j] : 0.f;
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int j = g0 + 64 * u + lane;
          if (g0 + 64 * u < nlist) f(j, j < nlist ? f32_order_key(v[u]) : 0xFFFFFFFFu, j < nlist);
        }
      }
    }
  };

  const int cap = p_stride + kExtra;   // LDS slots for selected keys
  int nsel = 0;
  bool fast = false;
  {
    // Threshold from the lanes' RR smallest keys (RR = 1 for np <= 16, 2 for np <= 64, else 4):
    // t = the np-th smallest of these 64 RR keys.  At least np keys
    // are <= t (those np of them), so the np smallest keys are all <= t; keys <= t are gathered
    // in one pass.  A lane rarely holds more than RR of the np smallest keys, so few more than np
    // are gathered; when more than `cap` are, the radix selection below runs.
    if (np <= 256) {
      uint32_t t;
      if (np <= 16) t = lane_union_threshold<1>(each, np);
      else if (np <= 64) t = lane_union_threshold<2>(each, np);
      else t = lane_union_threshold<4>(each, np);
      each_group([&](int j, uint32_t u, bool valid) {
        const bool take = valid && u <= t;
        const unsigned long long bt = __ballot(take);
        const int pos = nsel + __popcll(bt & lt);
        if (take && pos < cap) sel[pos] = ((unsigned long long)u << 32) | (uint32_t)j;
        nsel += __popcll(bt);
      });
      fast = nsel <= cap;
      if (!fast) nsel = 0;
    }
  }

  if (!fast) {
    uint32_t kmin = 0xFFFFFFFFu, kmax = 0u;
    each([&](int, uint32_t u) {
      kmin = min(kmin, u);
      kmax = max(kmax, u);
    });
    kmin = wave_min_u32(kmin);
    kmax = wave_max_u32(kmax);
    // keys share the bits above `top`; digits are taken below it
    int top = kmin == kmax ? -1 : 31 - __clz((int)(kmin ^ kmax));
    uint32_t prefix = top >= 31 ? 0u : (kmin & ~((2u << top) - 1u));
    uint32_t mask = top >= 31 ? 0u : ~((2u << top) - 1u);
    if (top < 0) { prefix = kmin; mask = 0xFFFFFFFFu; }
    int kk = np;          // rank still to place inside the current region
    int shift = top - 7;  // low bit of the current digit (may go negative: clamp below)
    bool boundary_ties = top < 0;  // the region holds a single key value
    while (top >= 0) {
      const int sh = max(shift, 0);
      const int width = top - sh + 1;   // <= 8 bits
      const uint32_t dmask = (1u << width) - 1u;
      for (int i = lane; i < 256; i += 64) hist[i] = 0;
      __builtin_amdgcn_wave_barrier();
      each([&](int, uint32_t u) {
        if ((u & mask) == prefix) atomicAdd(&hist[(u >> sh) & dmask], 1);
      });
      __builtin_amdgcn_wave_barrier();
      const int h0 = hist[4 * lane], h1 = hist[4 * lane + 1], h2 = hist[4 * lane + 2], h3 = hist[4 * lane + 3];
      const int inc = wave_incl_scan(h0 + h1 + h2 + h3);
      const int exc = inc - (h0 + h1 + h2 + h3);
      int d = 0, before = 0, inb = 0;
      if (exc < kk && kk <= inc) {
        int c = exc, dd = 4 * lane;
        int hv = h0;
        if (c + h0 < kk) { c += h0; ++dd; hv = h1;
          if (c + h1 < kk) { c += h1; ++dd; hv = h2;
            if (c + h2 < kk) { c += h2; ++dd; hv = h3; } } }
        d = dd; before = c; inb = hv;
      }
      const unsigned long long owner = __ballot(exc < kk && kk <= inc);
      const int src = __ffsll((long long)owner) - 1;
      d = __shfl(d, src); before = __shfl(before, src); inb = __shfl(inb, src);
      // narrow the region to the bucket holding the remaining rank
      const uint32_t region_lo = prefix | ((uint32_t)d << sh);
      if (sh == 0) {
        prefix = region_lo;
        mask = 0xFFFFFFFFu;
        kk -= before;
        boundary_ties = true;
        break;
      }
      if (inb <= kExtra) {
        // finalize with the bucket's keys as extra candidates: region = [region_lo, +2^sh)
        prefix = region_lo;
        mask |= dmask << sh;
        kk -= before;
        break;
      }
      prefix = region_lo;
      mask |= dmask << sh;
      kk -= before;
      top = sh - 1;
      shift = top - 7;
    }
    // gather: every key below the region, then the region's keys (all of them when it is a
    // small bucket; the first kk in index order when it is a single value)
    const uint32_t region_lo = prefix;
    each_group([&](int j, uint32_t u, bool valid) {
      const bool below = valid && u < region_lo;
      const bool inreg = valid && (u & mask) == prefix;
      bool take = below;
      if (!boundary_ties) take = take || inreg;
      const unsigned long long bt = __ballot(take);
      if (take) {
        const int pos = nsel + __popcll(bt & lt);
        sel[pos] = ((unsigned long long)u << 32) | (uint32_t)j;
      }
      nsel += __popcll(bt);
    });
    if (boundary_ties) {
      // the first kk keys equal to the boundary value, in index order
      int taken = 0;
      each_group([&](int j, uint32_t u, bool valid) {
        const bool inreg = valid && u == prefix;
        const unsigned long long bt = __ballot(inreg);
        const int r = __popcll(bt & lt);
        if (inreg && taken + r < kk) {
          sel[nsel + taken + r] = ((unsigned long long)u << 32) | (uint32_t)j;
        }
        taken = min(kk, taken + __popcll(bt));
      });
      nsel += taken;
    }
  }
  __builtin_amdgcn_wave_barrier();
  // rank sort by (key, index); the first np ranks are the probes
  for (int i = lane; i < nsel; i += 64) {
    const unsigned long long u = sel[i];
    int r = 0;
#pragma unroll 8
    for (int t = 0; t < nsel; ++t) r += sel[t] < u ? 1 : 0;
    if (r < np) probes[q * p_stride + r] = (int32_t)(uint32_t)u;
  }
}

void launch_select(const float *dist, int64_t ld, int32_t nlist, const int32_t *nprobe,
                   int32_t nprobe_all, int32_t nprobe_max, int32_t *probes, int32_t p_stride,
                   int64_t nq, hipStream_t s) {
  if (nq <= 0) return;
  const size_t smem = 4 * select_wave_lds(p_stride);
  const dim3 grid((unsigned)((nq + 3) / 4));
  // the row's keys in registers when they fit (64 per lane at most) and the batch is small
  // (64 keys per lane allow 3 waves per SIMD; a 10,000-query batch measured faster re-reading
  // its rows with 8 waves per SIMD), else re-read per pass
  if (nlist <= 256)
    hipLaunchKernelGGL(select_kernel<4>, grid, dim3(kSelThreads), smem, s, dist, ld, nlist, nprobe,
                       nprobe_all, probes, p_stride, nq);
  else if (nlist <= 1024)
    hipLaunchKernelGGL(select_kernel<16>, grid, dim3(kSelThreads), smem, s, dist, ld, nlist, nprobe,
                       nprobe_all, probes, p_stride, nq);
  else if (nlist <= 4096 && nq <= 4096)
    hipLaunchKernelGGL(select_kernel<64>, grid, dim3(kSelThreads), smem, s, dist, ld, nlist, nprobe,
                       nprobe_all, probes, p_stride, nq);
  else
    hipLaunchKernelGGL(select_kernel<0>, grid, dim3(kSelThreads), smem, s, dist, ld, nlist, nprobe,
                       nprobe_all, probes, p_stride, nq);
  (void)nprobe_max;
}

}  // namespace ddc
