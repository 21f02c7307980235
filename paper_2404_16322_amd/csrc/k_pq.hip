// Kernels of the quantization estimate (BSA-O, Sec. V-B "Approximate Distances"): the base is
// product-quantised over OPQ subspaces of the PCA axes (M subspaces of D/M axes, 256 codewords
// each, Sec. VII-A), the query's asymmetric distance to a point's codewords is the estimate,
// and the point's distance to its own codewords is one more classifier feature.
//
// The encode decides an integer, so its arithmetic is fixed: differences, squares and sums
// are FP32 operations rounded one at a time (no fused multiply-add), summed in axis order,
// lowest codeword on ties.  The FP64 feature kernel serves the calibration.
#include "ddc_internal.h"

#include <hip/hip_fp16.h>

#include <stdexcept>

namespace ddc {

namespace {

__device__ inline float stored_value(const void *base, int store, int32_t nblocks, int64_t tile, int v,
                                     int dim) {
  const int64_t idx = ((tile * nblocks + dim / kBlockDims) * kTile + v) * kBlockDims + dim % kBlockDims;
  if (store == ST_F32) return reinterpret_cast<const float *>(base)[idx];
  if (store == ST_F16) return __half2float(reinterpret_cast<const __half *>(base)[idx]);
  return __uint_as_float((uint32_t)reinterpret_cast<const unsigned short *>(base)[idx] << 16);
}

constexpr int kCodewords = 256;
constexpr int kMaxDsub = 32;

}  // namespace

__global__ void gather_cols_kernel(const float *Y, int64_t ldy, const int64_t *rows, int64_t nrows,
                                   const int32_t *cols, int32_t ncols, float *out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrows * ncols) return;
  const int64_t r = i / ncols;
  const int t = (int)(i % ncols);
  out[i] = Y[rows[r] * ldy + cols[t]];
}

void launch_gather_cols(const float *Y, int64_t ldy, const int64_t *rows, int64_t nrows,
                        const int32_t *cols, int32_t ncols, float *out, hipStream_t s) {
  const int64_t total = nrows * ncols;
  if (total <= 0) return;
  hipLaunchKernelGGL(gather_cols_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, Y, ldy,
                     rows, nrows, cols, ncols, out);
}

// grid (tiles, M): one workgroup of 64 lanes per (tile, subspace), lane = slot in the tile; the
// subspace's codebook is staged in LDS (every lane reads the same codeword: broadcast).
__global__ __launch_bounds__(kTile) void pq_encode_kernel(const void *base, int store, int32_t nblocks,
                                                         const int32_t *perm, const float *books,
                                                         int32_t M, int32_t dsub, uint8_t *codes,
                                                         float *dmin) {
  __shared__ float cb[kCodewords * kMaxDsub];
  const int64_t tile = blockIdx.x;
  const int j = blockIdx.y;
  const int v = threadIdx.x;
  for (int e = v; e < kCodewords * dsub; e += kTile) cb[e] = books[(int64_t)j * kCodewords * dsub + e];
  float y[kMaxDsub];
  for (int t = 0; t < dsub; ++t) y[t] = stored_value(base, store, nblocks, tile, v, perm[j * dsub + t]);
  __syncthreads();
  float best = INFINITY;
  int arg = 0;
  for (int c = 0; c < kCodewords; ++c) {
    // every operation rounded on its own: no contraction into fused multiply-adds
#pragma clang fp contract(off)
    float acc = 0.f;
    for (int t = 0; t < dsub; ++t) {
      const float d = y[t] - cb[c * dsub + t];
      acc = acc + d * d;
    }
    if (acc < best) { best = acc; arg = c; }
  }
  const int64_t slot = tile * kTile + v;
  codes[slot * M + j] = (uint8_t)arg;
  dmin[slot * M + j] = best;
}

// err[slot] = sum over subspaces of the minimum, in subspace order (FP32)
__global__ void pq_err_kernel(const float *dmin, int64_t nslots, int32_t M, float *err) {
  const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= nslots) return;
  float acc = 0.f;
  for (int j = 0; j < M; ++j) acc += dmin[slot * M + j];
  err[slot] = acc;
}

void launch_pq_encode(const void *base, int store, int32_t nblocks, int64_t total_tiles,
                      const int32_t *perm, const float *books, int32_t M, int32_t dsub,
                      uint8_t *codes, float *err, hipStream_t s) {
  if (total_tiles <= 0) return;
  if (dsub < 1 || dsub > kMaxDsub || M < 1 || M > 65535) throw std::invalid_argument("pq: bad M / dsub");
  const int64_t nslots = total_tiles * kTile;
  float *dmin = nullptr;
  fault_check_alloc();
  if (hipMallocAsync(reinterpret_cast<void **>(&dmin), (size_t)nslots * M * 4, s) != hipSuccess)
    throw std::runtime_error("pq: scratch allocation failed");
  alloc_track(1, (int64_t)nslots * M * 4);
  hipLaunchKernelGGL(pq_encode_kernel, dim3((unsigned)total_tiles, (unsigned)M), dim3(kTile), 0, s, base,
                     store, nblocks, perm, books, M, dsub, codes, dmin);
  hipLaunchKernelGGL(pq_err_kernel, dim3((unsigned)((nslots + 255) / 256)), dim3(256), 0, s, dmin, nslots, M,
                     err);
  (void)hipFreeAsync(dmin, s);
  alloc_track(-1, -(int64_t)nslots * M * 4);
}

__global__ void pq_features64_kernel(const double *qrot, int32_t D, const void *base, int store,
                                     int32_t nblocks, const int32_t *perm, const float *books, int32_t M,
                                     int32_t dsub, const uint8_t *codes, const int32_t *pair_q,
                                     const int64_t *pair_slot, int64_t npairs, double *adc, double *err) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npairs) return;
  const int64_t slot = pair_slot[p];
  const double *q = qrot + (int64_t)pair_q[p] * D;
  const int64_t tile = slot / kTile;
  const int v = (int)(slot % kTile);
  double a = 0.0, e = 0.0;
  for (int j = 0; j < M; ++j) {
    const float *cw = books + ((int64_t)j * kCodewords + codes[slot * M + j]) * dsub;
    for (int t = 0; t < dsub; ++t) {
      const int ax = perm[j * dsub + t];
      const double c = (double)cw[t];
      const double dq = q[ax] - c;
      const double dy = (double)stored_value(base, store, nblocks, tile, v, ax) - c;
      a += dq * dq;
      e += dy * dy;
    }
  }
  adc[p] = a;
  err[p] = e;
}

void launch_pq_features64(const double *qrot, int32_t D, const void *base, int store,
                          int32_t nblocks, const int32_t *perm, const float *books, int32_t M,
                          int32_t dsub, const uint8_t *codes, const int32_t *pair_q,
                          const int64_t *pair_slot, int64_t npairs, double *adc, double *err,
                          hipStream_t s) {
  if (npairs <= 0) return;
  hipLaunchKernelGGL(pq_features64_kernel, dim3((unsigned)((npairs + 255) / 256)), dim3(256), 0, s, qrot, D,
                     base, store, nblocks, perm, books, M, dsub, codes, pair_q, pair_slot, npairs, adc, err);
}

}  // namespace ddc
