// Internal declarations shared by the HIP kernel files and the host runtime.
// Not part of the public ABI (include/ddc.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ddc {

// Dimension blocks of the packed base are 32 wide; a stage (Delta_d) is a whole
// number of blocks.  Vectors are grouped in tiles of 64 (one wavefront).
constexpr int kBlockDims = 32;
constexpr int kTile = 64;
constexpr int kMaxBlocks = 128;      // D <= 4096
constexpr int kMaxLag = 64;          // tau lag L in blocks
constexpr int kMaxK = 256;
constexpr int kScanThreads = 256;    // 4 wavefronts per query
// counters: candidates, refined, stage_slices, two-phase sums read, stop[64], pre-stage reads,
// pre-stage prunes, dim-block slices the two-phase sums stood in for
constexpr int kCtrPreReads = 4 + 64, kCtrPrePruned = 4 + 64 + 1, kCtrSlicesSummed = 4 + 64 + 2;
constexpr int kMaxCounters = 4 + 64 + 3;
constexpr int kFp8Lead = 64;          // dims covered by the FP8 pre-stage
constexpr int kMaxTables = 4;         // correction tables (calibration K_c values) per index
constexpr size_t kMaxLds = 160 * 1024;  // LDS per workgroup on gfx950

enum StoreType : int { ST_F32 = 0, ST_F16 = 1, ST_BF16 = 2 };

// Allocation fault injection (tests): DDC_FAULT=alloc:<n> in the environment, or
// ddc_set_fault("alloc:<n>"), makes the n-th device or pinned-host allocation from then on fail
// as out of memory before the runtime is called (0 / unset: never).  Called before every such
// allocation; throws the library's out-of-memory error on the injected one.
void fault_check_alloc();
// Live device / pinned-host allocations of the library (count, bytes): every successful
// allocation adds, every release subtracts (tests check that failed calls leave nothing behind).
void alloc_track(int64_t count, int64_t bytes);

// Arguments of the pruned scan (A3) + top-K merge (A4) + finalize (A5) kernel.
struct ScanArgs {
  const float *qrot;       // [nq x q_stride] rotated queries, zero beyond D
  int64_t q_stride;
  const int32_t *probes;   // [nq x p_stride] list ids in probe order
  int32_t p_stride;
  const int32_t *nprobe;   // per query, or NULL -> nprobe_all
  int32_t nprobe_all;
  const int32_t *k;        // per query, or NULL -> k_all
  int32_t k_all;
  const int64_t *out_off;  // CSR result offsets, or NULL -> q * k_all
  const int32_t *tile_off; // [nlist + 1] first tile of each list
  const int32_t *list_len; // [nlist]
  const void *base;        // packed tiles: [tile][block][64 vectors][32 dims]
  const int32_t *ids;      // [tiles * 64] original id of each stored slot (-1 = padding)
  int64_t *out_ids;
  float *out_d;
  int64_t *counters;       // NULL or [kMaxCounters] (added to)
  const int32_t *order;    // NULL or [nq]: wave slot -> query (results do not depend on it)
  int32_t *queue;          // NULL: one workgroup per slot group; else a device counter: the
                           // grid is sized to the resident capacity and workgroups take slots
                           // from it until none is left (launch_scan zeroes it first)
  int32_t xcd_swizzle;     // 1: workgroup w runs slot range of XCD (w mod 8), contiguous per XCD
  const uint8_t *base8;    // FP8 pre-stage codes: per tile 64 vectors x 64 B (NULL if none)
  const float *scale8;     // per tile decode scale
  int32_t pre;             // 1: run the FP8 pre-stage test first
  int32_t res;             // 1: residual-estimate test (needs xnorm, lam, bsar_m; one stage per load)
  const float *xnorm;      // [tiles * 64] ||y||^2 of every stored slot
  const float *lam;        // [nblocks * 32] variance along every rotated axis (0 beyond D)
  float bsar_m;            // multiplier m of m sigma
  // quantization test of BSA-O before the stages (pq_m > 0): codes [tiles * 64][pq_m] bytes,
  // per-slot quantization error, codebooks [pq_m][256][pq_dsub], subspace axes [pq_m * pq_dsub],
  // per-table (m1, m3, beta, unused) at pq_tab[4 t]
  const uint8_t *pq_codes;
  const float *pq_err;
  const float *pq_books;
  const int32_t *pq_perm;
  const float *pq_tab;
  int32_t pq_m, pq_dsub;
  int32_t est_nb;          // > 0 (with prune = 0): rank by an estimate over the leading est_nb
                           // dim blocks, no refinement (needs xnorm when est_res)
  int32_t est_res;         // estimate: 0 = est_scale * partial distance, 1 = residual (Alg. 1)
  float est_scale;
  int32_t waves_per_query; // 1 or 4 (result-invariant)
  int32_t lookahead;       // 0 or 1: multi-stage loads when few candidates survive (result-invariant)
  int32_t occ5;            // 1: the one-wave lag-free pruned kernel built for five waves per SIMD
                           // (no residual or quantization test; result-invariant)
  int32_t nq, nblocks, block_b, prune, nlist, k_max;
  int32_t lag;           // tau lag L in blocks: block b is tested against the tau after block b - 1 - L
  // Correction tables [ntab][nblocks + 1][2] = (m, beta) of the test after dim block b
  // (beta = -inf, m = 0 where none follows); entry nblocks is the FP8 pre-stage.  A query
  // with K uses the last table t with tab_k[t] <= K (table 0 when none).
  const float *tab;
  int32_t ntab;
  int32_t tab_k[kMaxTables];
  int8_t test_after[kMaxBlocks]; // 1 if a stage test follows block b
  // Two-phase scan: when e1 is set, the partial distance after dim block 0 (with pre: the FP8
  // pre-stage's) of every candidate of every probed list was computed beforehand list by list
  // (launch_stage1_lists): query q's candidates start at e1[e1_qoff[q]], its lists' in probe
  // order, each list's in stored order and its segment padded to e1_padded(length) entries.
  // The first test then reads these instead of the base (bit-identical sums).
  const float *e1;
  const int64_t *e1_qoff;
  int64_t e1_cap;          // entries of e1 (no read at or past it)
  // e1_tol > 0: e1 holds stage-1 sums in the expanded form (launch_stage1_lists with matrix),
  // each within e1_tol (3 ||q'_1||^2 + 2 |e1|) of the scan's own sum; the scan prunes on them
  // only where the bound decides its own test, and the candidates left re-read dim block 0 and
  // take the first test in the scan's own arithmetic (results and counters as with exact sums)
  float e1_tol;
  // (prune = 0 with e1 set: e1 holds every candidate's full distance, from launch_full_lists)
};

void launch_scan(const ScanArgs &a, int store, hipStream_t s);

// First phase of the two-phase scan: the partial distance over dim block 0 (pre: the FP8
// pre-stage's over the leading 64 dims) of every candidate of every probed list, computed list
// by list so each stored tile is read once for all the queries that probe its list, with the
// arithmetic (and rounding) of the scan's own first test.  Probes of query q: probes[q * p_stride + p], p < clamp(nprobe[q], 1, p_stride), every
// list at most once per query.  Scratch (caller's): lcnt, lstart [nlist + 1]; rank, lpair
// [nq * p_stride] int32; poff [nq * p_stride], qcnt [nq], qoff [nq + 1] int64; e1 [e1_cap].
struct Stage1Args {
  const int32_t *probes; int32_t p_stride;
  const int32_t *nprobe; int32_t nprobe_all;
  const int32_t *list_len, *tile_off, *tile_list;   // tile_list: [total_tiles] list of each tile
  int32_t nlist; int64_t total_tiles; int64_t nq;
  const float *qrot; int64_t q_stride;
  const void *base; int32_t nblocks;
  int32_t pre;                      // 1: the FP8 pre-stage sums over the leading 64 dims instead
  const uint8_t *base8; const float *scale8;
  int32_t *lcnt, *lstart, *rank, *lpair;
  int64_t *poff, *qcnt, *qoff;
  float *e1; int64_t e1_cap;
};
// matrix (stored values only, not with pre): the sums are formed instead as
// ||q'_1||^2 + ||y_1||^2 - 2 <q'_1, y_1> on the matrix cores (FP32 products), clamped at 0: the
// scan's own sums up to the bound ScanArgs::e1_tol describes, not their bits.
void launch_stage1_lists(const Stage1Args &a, int store, hipStream_t s, bool matrix = false);

// Full-dimension distances list by list on the matrix cores (the list-major full-D scan):
// the pair grouping of launch_stage1_lists, then for every stored tile and every query that
// probes its list  ||q'||^2 + ||y||^2 - 2 <q', y>  (FP32 products, v_mfma_f32_16x16x4_f32; the
// norms ||y||^2 of the stored values from xnorm, ||q'||^2 in FP32), clamped at 0, written to
// e1 in the layout of launch_stage1_lists.  qnorm: [nq] scratch.
void launch_full_lists(const Stage1Args &a, const float *xnorm, float *qnorm, int store, hipStream_t s);
// e1 (the list-major phases' per-candidate sums): every (query, list) segment starts at a
// multiple of this many floats (128 B), so the first phase's 64-sum rows are whole cache lines
__host__ __device__ inline int64_t e1_padded(int64_t len) { return (len + 31) & ~(int64_t)31; }
// Lag-parallel scan: with a lag of at least W - 1 blocks, every block of a group of W
// consecutive blocks is tested against a tau known before the group starts, so with W = 2 or 4
// waves per query each wave scans one block of the group at once and the group's survivors are
// merged in block order afterwards (results and counters equal the one-wave lagged scan's).
inline bool lag_parallel(const ScanArgs &a, int W) {
  return a.prune && ((W == 4 && a.lag >= 3) || (W == 2 && a.lag >= 1));
}
// LDS bytes one workgroup of the scan needs with W waves per query (> kMaxLds: not launchable).
size_t scan_lds_request(const ScanArgs &a, int W);

// Query order for cache locality: queries grouped by their first probed list (counting sort,
// order within a group arbitrary).  hist: [nlist + 1] scratch, rank: [nq] scratch.
void launch_query_order(const int32_t *probes, int32_t p_stride, int64_t nq, int32_t nlist,
                        int32_t *hist, int32_t *rank, int32_t *order, hipStream_t s);
// Longest-first query order for the persistent launch: key[q] = 255 - bucket of the query's
// candidate count (sum of its probed list lengths; 8 buckets per octave), then the counting
// sort above over the 256 keys.  key, rank: [nq] scratch; hist: [257] scratch.
void launch_work_order(const int32_t *probes, int32_t p_stride, const int32_t *nprobe,
                       int32_t nprobe_all, const int32_t *list_len, int32_t nlist, int64_t nq,
                       int32_t *key, int32_t *hist, int32_t *rank, int32_t *order, hipStream_t s);

// C[M x N] = (A - mu)[M x K] * B[N x K]^T on MFMA, FP32 accumulation.
//   mode 0: out[m][n] = acc                      (query / base rotation)
//   mode 1: out[m][n] = bias[n] - 2 acc          (coarse: ||c||^2 - 2 <q', c>)
//   mode 2: argmin over n of bias[n] - 2 acc per row -> atomicMin into key64[m]
// A, B row-major with leading dims lda, ldb (elements); K is padded by zero-filling.
// prec 0 = FP32 MFMA, 1 = BF16 MFMA (inputs rounded to nearest even bfloat16).
struct GemmArgs {
  const float *A; int64_t lda;
  const float *mu;        // [K] or NULL
  const float *B; int64_t ldb;
  const float *bias;      // [N] (modes 1, 2)
  float *C; int64_t ldc;  // modes 0, 1
  unsigned long long *key64; // mode 2
  int64_t M; int32_t N, K;
  int32_t mode, prec;
};
void launch_gemm(const GemmArgs &g, hipStream_t s);

// Probe selection (A2): the nprobe smallest of dist[q][0..nlist) by (value, index),
// ascending, written to probes[q][0..nprobe).
void launch_select(const float *dist, int64_t ld, int32_t nlist, const int32_t *nprobe,
                   int32_t nprobe_all, int32_t nprobe_max, int32_t *probes, int32_t p_stride,
                   int64_t nq, hipStream_t s);

// ---- fit-side kernels (k_fit.hip) ----
// FP64 column means of X[rows] (rows = NULL -> all n): out mu[D].
void launch_mean64(const float *X, int64_t n, int32_t D, const int64_t *rows, int64_t nrows,
                   double *partial, int32_t nparts, double *mu, hipStream_t s);
// FP64 covariance (1/nrows) sum (x-mu)(x-mu)^T, deterministic (fixed partial order).
void launch_cov64(const float *X, int64_t n, int32_t D, const int64_t *rows, int64_t nrows,
                  const double *mu, double *partial, int32_t nparts, double *cov, hipStream_t s);
// Round FP32 rows to the storage format and back (values become exactly representable).
void launch_round_storage(float *Y, int64_t count, int store, hipStream_t s);
// Per-cluster FP64 means in a fixed order: members[off[j]..off[j+1]) of Y rows.
void launch_centroid_update(const float *Y, int64_t ldy, int32_t D, const int32_t *off,
                            const int32_t *members, int32_t nlist, float *C, int64_t ldc,
                            hipStream_t s);
void launch_row_norms(const float *C, int64_t ldc, int32_t rows, int32_t D, float *out,
                      hipStream_t s);
// dst[r] = src[rows[r]] (row copies, `cols` floats each)
void launch_gather_rows(const float *src, int64_t ld, const int64_t *rows, int64_t nrows, int32_t cols,
                        float *dst, int64_t ldd, hipStream_t s);
void launch_decode_argmin(const unsigned long long *key64, int64_t n, int32_t *assign,
                          hipStream_t s);
// Pack rotated rows into [tile][block][64][32] storage tiles; slot_row[t*64+v] = row or -1.
void launch_pack(const float *Y, int64_t ldy, int32_t D, int32_t nblocks, const int64_t *slot_row,
                 int64_t total_tiles, void *base, int store, hipStream_t s);

// ---- calibration kernels (k_calib.hip), FP64 ----
void launch_rotate64(const float *Q, int64_t nq, int32_t D, const double *mu, const double *R,
                     double *out, hipStream_t s);
// Exact FP64 squared distances of rows `cand[q][0..nc)` of the packed base to q'.
void launch_refine64(const double *qrot, int32_t D, const void *base, int store, int32_t nblocks,
                     const int64_t *slots, int32_t nc, int64_t nq, double *out, hipStream_t s);
// FP64 partial distances e_s after every test stage for (query, slot) pairs.
// FP8 E4M3 codes of the leading 64 dims of every packed tile, one scale per tile
// (max |y| / 448); codes: [tiles x 64 vectors x 64] bytes, scale: [tiles].
void launch_encode_fp8(const void *base, int store, int32_t nblocks, int64_t total_tiles,
                       uint8_t *codes, float *scale, hipStream_t s);
// ||y||^2 of every stored slot: out [tiles x 64].
void launch_slot_sqnorm(const void *base, int store, int32_t nblocks, int64_t total_tiles, float *out,
                        hipStream_t s);
// FP64 pre-stage feature e_0 = sum_{i<64} (q_i - dec_i)^2 of (query, packed slot) pairs,
// dec = fp32(value(code) * scale).
void launch_features8(const double *qrot, int32_t D, const uint8_t *codes, const float *scale,
                      const int32_t *pair_q, const int64_t *pair_slot, int64_t npairs, double *out,
                      int64_t out_stride, hipStream_t s);
void launch_features64(const double *qrot, int32_t D, const void *base, int store, int32_t nblocks,
                       const int32_t *pair_q, const int64_t *pair_slot, int64_t npairs,
                       const int32_t *stage_end_block, int32_t n_test, double *out, hipStream_t s);
// ---- OPQ / PQ kernels of the quantization estimate (k_pq.hip) ----
// out[r][t] = Y[rows[r]][cols[t]]  (t < ncols)
void launch_gather_cols(const float *Y, int64_t ldy, const int64_t *rows, int64_t nrows,
                        const int32_t *cols, int32_t ncols, float *out, hipStream_t s);
// Codes of every packed slot: codes[slot][j] = argmin_c ||y_j - books[j][c]||^2 in FP32 with
// every operation rounded separately (differences, squares, sums in axis order; lowest c on
// ties); err[slot] = FP32 sum over j of the minima.
void launch_pq_encode(const void *base, int store, int32_t nblocks, int64_t total_tiles,
                      const int32_t *perm, const float *books, int32_t M, int32_t dsub,
                      uint8_t *codes, float *err, hipStream_t s);
// FP64 features of (query, slot) pairs: adc = sum_j ||q'_j - books[j][code_j]||^2 and
// err = sum_j ||y_j - books[j][code_j]||^2 (y from the packed base).
void launch_pq_features64(const double *qrot, int32_t D, const void *base, int store,
                          int32_t nblocks, const int32_t *perm, const float *books, int32_t M,
                          int32_t dsub, const uint8_t *codes, const int32_t *pair_q,
                          const int64_t *pair_slot, int64_t npairs, double *adc, double *err,
                          hipStream_t s);
// FP64 centroid distances for probe ordering of calibration queries.
void launch_cdist64(const double *qrot, int64_t nq, int32_t D, const float *cent, int64_t ldc,
                    int32_t nlist, double *out, hipStream_t s);
// Unpruned canonical IVF search in FP64 collecting label-1 candidates (dis > tau_b, tau_b finite),
// keeping the max_neg with the smallest SplitMix64 keys per query.
struct NegArgs {
  const double *qrot; int32_t D;
  const int32_t *probes; int32_t nprobe;
  const int32_t *tile_off; const int32_t *list_len;
  const void *base; int store; int32_t nblocks;
  const int32_t *ids;
  int32_t k, block_b, max_neg, lag;
  unsigned long long key_base;   // splitmix64(seed + tag)
  int64_t nq;
  int64_t *neg_slot;   // [nq x max_neg] stored slot or -1
  double *neg_tau;     // [nq x max_neg]
};
void launch_negatives64(const NegArgs &a, hipStream_t s);

}  // namespace ddc
