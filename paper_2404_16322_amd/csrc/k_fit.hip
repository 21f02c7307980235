// Fit-side kernels: FP64 mean and covariance of the PCA sample (Sec. IV-B: data centred,
// the projection is the covariance's eigenbasis, Thm. 1), storage rounding, the k-means
// centroid update of the IVF lists (Sec. II-A), and packing of the rotated base into the
// dimension-blocked tile layout the scan reads.
#include "ddc_internal.h"

#include <hip/hip_fp16.h>

namespace ddc {

namespace {

__device__ inline unsigned short bf16_rne_bits(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

__device__ inline int64_t row_of(const int64_t *rows, int64_t i) { return rows ? rows[i] : i; }

}  // namespace

// partial[p][d] = sum over rows of part p of X[row][d]   (FP64, fixed order)
__global__ void mean_partial_kernel(const float *X, int32_t D, const int64_t *rows, int64_t nrows,
                                    int32_t nparts, double *partial) {
  const int p = blockIdx.x;
  const int64_t chunk = (nrows + nparts - 1) / nparts;
  const int64_t r0 = p * chunk, r1 = min(nrows, r0 + chunk);
  for (int d = threadIdx.x; d < D; d += blockDim.x) {
    double s = 0.0;
    for (int64_t r = r0; r < r1; ++r) s += (double)X[row_of(rows, r) * D + d];
    partial[(int64_t)p * D + d] = s;
  }
}

__global__ void mean_final_kernel(const double *partial, int32_t D, int32_t nparts, int64_t nrows,
                                  double *mu) {
  const int d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= D) return;
  double s = 0.0;
  for (int p = 0; p < nparts; ++p) s += partial[(int64_t)p * D + d];
  mu[d] = s / (double)nrows;
}

void launch_mean64(const float *X, int64_t n, int32_t D, const int64_t *rows, int64_t nrows,
                   double *partial, int32_t nparts, double *mu, hipStream_t s) {
  (void)n;
  hipLaunchKernelGGL(mean_partial_kernel, dim3(nparts), dim3(256), 0, s, X, D, rows, nrows, nparts,
                     partial);
  hipLaunchKernelGGL(mean_final_kernel, dim3((D + 255) / 256), dim3(256), 0, s, partial, D, nparts,
                     nrows, mu);
}

// Covariance tiles: workgroup (ti, tj, part) accumulates the 64x64 tile (ti <= tj) of
// sum (x - mu)(x - mu)^T over the rows of `part`, 32 rows at a time through LDS, FP64.
constexpr int CT = 64, CR = 32;
__global__ __launch_bounds__(256) void cov_partial_kernel(const float *X, int32_t D,
                                                          const int64_t *rows, int64_t nrows,
                                                          const double *mu, int32_t nparts,
                                                          double *partial) {
  const int ti = blockIdx.x, tj = blockIdx.y, p = blockIdx.z;
  if (ti > tj) return;
  __shared__ double As[CR][CT + 1];
  __shared__ double Bs[CR][CT + 1];
  const int tid = threadIdx.x;
  const int tr = tid / 16, tc = tid % 16;  // 4x4 outputs each: rows tr*4.., cols tc*4..
  double acc[4][4] = {};
  const int64_t chunk = (nrows + nparts - 1) / nparts;
  const int64_t r0 = p * chunk, r1 = min(nrows, r0 + chunk);
  const int i0 = ti * CT, j0 = tj * CT;
  for (int64_t rb = r0; rb < r1; rb += CR) {
    for (int e = tid; e < CR * CT; e += 256) {
      const int rr = e / CT, cc = e % CT;
      const int64_t r = rb + rr;
      double a = 0.0, b = 0.0;
      if (r < r1) {
        const int64_t row = row_of(rows, r);
        if (i0 + cc < D) a = (double)X[row * D + i0 + cc] - mu[i0 + cc];
        if (j0 + cc < D) b = (double)X[row * D + j0 + cc] - mu[j0 + cc];
      }
      As[rr][cc] = a;
      Bs[rr][cc] = b;
    }
    __syncthreads();
    for (int rr = 0; rr < CR; ++rr) {
      double av[4], bv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) { av[u] = As[rr][tr * 4 + u]; bv[u] = Bs[rr][tc * 4 + u]; }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fma(av[u], bv[v], acc[u][v]);
    }
    __syncthreads();
  }
  const int ntile = (D + CT - 1) / CT;
  double *out = partial + (((int64_t)p * ntile + ti) * ntile + tj) * CT * CT;
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) out[(tr * 4 + u) * CT + tc * 4 + v] = acc[u][v];
}

__global__ void cov_final_kernel(const double *partial, int32_t D, int32_t nparts, int64_t nrows,
                                 double *cov) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)D * D) return;
  int i = (int)(e / D), j = (int)(e % D);
  if (i > j) { const int t = i; i = j; j = t; }
  const int ntile = (D + CT - 1) / CT;
  const int ti = i / CT, tj = j / CT;
  double s = 0.0;
  for (int p = 0; p < nparts; ++p)
    s += partial[(((int64_t)p * ntile + ti) * ntile + tj) * CT * CT + (i % CT) * CT + (j % CT)];
  cov[e] = s / (double)nrows;
}

void launch_cov64(const float *X, int64_t n, int32_t D, const int64_t *rows, int64_t nrows,
                  const double *mu, double *partial, int32_t nparts, double *cov, hipStream_t s) {
  (void)n;
  const int ntile = (D + CT - 1) / CT;
  hipLaunchKernelGGL(cov_partial_kernel, dim3(ntile, ntile, nparts), dim3(256), 0, s, X, D, rows,
                     nrows, mu, nparts, partial);
  const int64_t tot = (int64_t)D * D;
  hipLaunchKernelGGL(cov_final_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, partial,
                     D, nparts, nrows, cov);
}

__global__ void round_storage_kernel(float *Y, int64_t count, int store) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float v = Y[i];
  if (store == ST_F16) {
    Y[i] = __half2float(__float2half_rn(v));
  } else if (store == ST_BF16) {
    Y[i] = __uint_as_float((uint32_t)bf16_rne_bits(v) << 16);
  }
}

void launch_round_storage(float *Y, int64_t count, int store, hipStream_t s) {
  if (store == ST_F32 || count <= 0) return;
  hipLaunchKernelGGL(round_storage_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, Y,
                     count, store);
}

// Centroid j = FP64 mean of its members (in member order); an empty list keeps its centroid.
__global__ void centroid_update_kernel(const float *Y, int64_t ldy, int32_t D, const int32_t *off,
                                       const int32_t *members, float *C, int64_t ldc) {
  const int j = blockIdx.x;
  const int b = off[j], e = off[j + 1];
  if (b == e) return;
  for (int d = threadIdx.x; d < D; d += blockDim.x) {
    double s = 0.0;
    for (int t = b; t < e; ++t) s += (double)Y[(int64_t)members[t] * ldy + d];
    C[(int64_t)j * ldc + d] = (float)(s / (double)(e - b));
  }
}

void launch_centroid_update(const float *Y, int64_t ldy, int32_t D, const int32_t *off,
                            const int32_t *members, int32_t nlist, float *C, int64_t ldc,
                            hipStream_t s) {
  hipLaunchKernelGGL(centroid_update_kernel, dim3(nlist), dim3(128), 0, s, Y, ldy, D, off, members,
                     C, ldc);
}

__global__ void row_norms_kernel(const float *C, int64_t ldc, int32_t rows, int32_t D, float *out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  double s = 0.0;
  for (int d = 0; d < D; ++d) {
    const double v = C[(int64_t)r * ldc + d];
    s += v * v;
  }
  out[r] = (float)s;
}

void launch_row_norms(const float *C, int64_t ldc, int32_t rows, int32_t D, float *out,
                      hipStream_t s) {
  hipLaunchKernelGGL(row_norms_kernel, dim3((rows + 255) / 256), dim3(256), 0, s, C, ldc, rows, D,
                     out);
}

__global__ void gather_rows_kernel(const float *src, int64_t ld, const int64_t *rows, int32_t cols,
                                   float *dst, int64_t ldd) {
  const int64_t r = blockIdx.x;
  const int64_t sr = rows[r];
  for (int c = threadIdx.x; c < cols; c += blockDim.x) dst[r * ldd + c] = src[sr * ld + c];
}

void launch_gather_rows(const float *src, int64_t ld, const int64_t *rows, int64_t nrows, int32_t cols,
                        float *dst, int64_t ldd, hipStream_t s) {
  if (nrows <= 0) return;
  hipLaunchKernelGGL(gather_rows_kernel, dim3((unsigned)nrows), dim3(128), 0, s, src, ld, rows, cols, dst,
                     ldd);
}

__global__ void decode_argmin_kernel(const unsigned long long *key64, int64_t n, int32_t *assign) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) assign[i] = (int32_t)(key64[i] & 0xFFFFFFFFull);
}

void launch_decode_argmin(const unsigned long long *key64, int64_t n, int32_t *assign,
                          hipStream_t s) {
  hipLaunchKernelGGL(decode_argmin_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, key64,
                     n, assign);
}

// tile t, block b: 64 vectors x 32 dims, vector-major; one workgroup per (tile, block).
__global__ void pack_kernel(const float *Y, int64_t ldy, int32_t D, int32_t nblocks,
                            const int64_t *slot_row, void *base, int store) {
  const int64_t t = blockIdx.x;
  const int b = blockIdx.y;
  for (int e = threadIdx.x; e < kTile * kBlockDims; e += blockDim.x) {
    const int v = e / kBlockDims, d = e % kBlockDims;
    const int64_t row = slot_row[t * kTile + v];
    const int dim = b * kBlockDims + d;
    const float x = (row >= 0 && dim < D) ? Y[row * ldy + dim] : 0.f;
    const int64_t idx = ((t * nblocks + b) * kTile + v) * kBlockDims + d;
    if (store == ST_F32) {
      reinterpret_cast<float *>(base)[idx] = x;
    } else if (store == ST_F16) {
      reinterpret_cast<__half *>(base)[idx] = __float2half_rn(x);
    } else {
      reinterpret_cast<unsigned short *>(base)[idx] = bf16_rne_bits(x);
    }
  }
}

void launch_pack(const float *Y, int64_t ldy, int32_t D, int32_t nblocks, const int64_t *slot_row,
                 int64_t total_tiles, void *base, int store, hipStream_t s) {
  if (total_tiles <= 0) return;
  hipLaunchKernelGGL(pack_kernel, dim3((unsigned)total_tiles, nblocks), dim3(256), 0, s, Y, ldy, D,
                     nblocks, slot_row, base, store);
}

// ---- FP8 E4M3 (OCP OFP8 v1.0: bias 7, no infinities, largest finite 448) ----------
// Round to nearest, ties to even mantissa, saturating at +-448; sign from the sign bit.
__device__ inline uint32_t e4m3_rne_sat(float v) {
  const uint32_t sign = (__float_as_uint(v) >> 24) & 0x80u;
  const float a = fabsf(v);
  uint32_t code;
  if (!(a < 464.f)) {
    code = 0x7Eu;                                   // beyond halfway to 480: clamp to 448
  } else if (a < 0.015625f) {
    code = (uint32_t)rintf(a * 512.f);              // below 2^-6: subnormal steps of 2^-9
  } else {
    const int e = (int)((__float_as_uint(a) >> 23) & 0xFFu) - 127;   // a in [2^e, 2^(e+1))
    const uint32_t n = (uint32_t)rintf(ldexpf(a, 3 - e));           // 8 .. 16
    code = (uint32_t)(e + 7) * 8u + n - 8u;                          // 16 carries into e + 1
  }
  return min(code, 0x7Eu) | sign;
}

__device__ inline float packed_value(const void *base, int store, int32_t nblocks, int64_t tile,
                                     int v, int dim) {
  const int64_t idx = ((tile * nblocks + dim / kBlockDims) * kTile + v) * kBlockDims + dim % kBlockDims;
  if (store == ST_F32) return reinterpret_cast<const float *>(base)[idx];
  if (store == ST_F16) return __half2float(reinterpret_cast<const __half *>(base)[idx]);
  return __uint_as_float((uint32_t)reinterpret_cast<const unsigned short *>(base)[idx] << 16);
}

// One wavefront per tile, lane = vector slot (padding slots hold zeros).
__global__ void encode_fp8_kernel(const void *base, int store, int32_t nblocks, uint8_t *codes,
                                  float *scale) {
  const int64_t t = blockIdx.x;
  const int v = threadIdx.x;
  float amax = 0.f;
  for (int d = 0; d < kFp8Lead; ++d) amax = fmaxf(amax, fabsf(packed_value(base, store, nblocks, t, v, d)));
  for (int o = 32; o > 0; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o));
  const float sc = amax > 0.f ? amax / 448.f : 1.f;
  uint32_t *out = reinterpret_cast<uint32_t *>(codes + (t * kTile + v) * kFp8Lead);
  for (int d = 0; d < kFp8Lead; d += 4) {
    uint32_t w = 0;
    for (int e = 0; e < 4; ++e)
      w |= e4m3_rne_sat(packed_value(base, store, nblocks, t, v, d + e) / sc) << (8 * e);
    out[d / 4] = w;
  }
  if (v == 0) scale[t] = sc;
}

void launch_encode_fp8(const void *base, int store, int32_t nblocks, int64_t total_tiles,
                       uint8_t *codes, float *scale, hipStream_t s) {
  if (total_tiles <= 0) return;
  hipLaunchKernelGGL(encode_fp8_kernel, dim3((unsigned)total_tiles), dim3(kTile), 0, s, base, store,
                     nblocks, codes, scale);
}

// Value of an E4M3 code from the format's fields (exact in FP32).
__device__ inline float e4m3_value(uint32_t c) {
  const float sgn = (c & 0x80u) ? -1.f : 1.f;
  const uint32_t e = (c >> 3) & 0xFu, m = c & 7u;
  if (e == 0) return sgn * (float)m * 0.001953125f;            // m * 2^-9
  return sgn * ldexpf(1.f + (float)m * 0.125f, (int)e - 7);
}

__global__ void features8_kernel(const double *qrot, int32_t D, const uint8_t *codes,
                                 const float *scale, const int32_t *pair_q, const int64_t *pair_slot,
                                 int64_t npairs, double *out, int64_t out_stride) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npairs) return;
  const int64_t slot = pair_slot[p];
  const double *q = qrot + (int64_t)pair_q[p] * D;
  const float sc = scale[slot / kTile];
  const uint8_t *c = codes + slot * kFp8Lead;
  double acc = 0.0;
  for (int i = 0; i < kFp8Lead; ++i) {
    const float dec = e4m3_value(c[i]) * sc;
    const double d = q[i] - (double)dec;
    acc += d * d;
  }
  out[p * out_stride] = acc;
}

void launch_features8(const double *qrot, int32_t D, const uint8_t *codes, const float *scale,
                      const int32_t *pair_q, const int64_t *pair_slot, int64_t npairs, double *out,
                      int64_t out_stride, hipStream_t s) {
  if (npairs <= 0) return;
  hipLaunchKernelGGL(features8_kernel, dim3((unsigned)((npairs + 255) / 256)), dim3(256), 0, s, qrot,
                     D, codes, scale, pair_q, pair_slot, npairs, out, out_stride);
}

// ||y||^2 of every stored slot of the packed base (FP64 sum, stored as float).
__global__ void slot_sqnorm_kernel(const void *base, int store, int32_t nblocks, float *out) {
  const int64_t t = blockIdx.x;
  const int v = threadIdx.x;
  double acc = 0.0;
  for (int d = 0; d < nblocks * kBlockDims; ++d) {
    const double x = packed_value(base, store, nblocks, t, v, d);
    acc += x * x;
  }
  out[t * kTile + v] = (float)acc;
}

void launch_slot_sqnorm(const void *base, int store, int32_t nblocks, int64_t total_tiles, float *out,
                        hipStream_t s) {
  if (total_tiles <= 0) return;
  hipLaunchKernelGGL(slot_sqnorm_kernel, dim3((unsigned)total_tiles), dim3(kTile), 0, s, base, store,
                     nblocks, out);
}

}  // namespace ddc
