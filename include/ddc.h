/*
 * ddc.h -- C ABI of the MI355X (gfx950) library for data-driven, PCA-based,
 * incrementally pruned distance comparison inside an IVF nearest-neighbour
 * search ("Effective and General Distance Computation for Approximate Nearest
 * Neighbor Search").
 *
 * Problem (Sec. II-A): a set S of n points in R^D, a query q, the K points of S
 * with the smallest squared Euclidean distance dis(p, q) = ||p - q||^2.  Candidates
 * come from an inverted file (IVF, Sec. II-A): k-means lists, the N_probe lists
 * whose centroids are nearest to q are scanned.  Each candidate is compared with
 * the running K-th distance tau of the result queue (Sec. I) through the
 * data-driven correction of Sec. V-A applied incrementally (Sec. V-B): after every
 * block of Delta_d PCA-rotated dimensions (Sec. IV-B, Thm. 1; Alg. 2's loop) the
 * partial distance e_s is tested with  m_s * e_s + beta_s > tau  and the candidate
 * is pruned, otherwise refined to its exact distance.
 *
 * Conventions shared by every call:
 *  - Pointers are plain host or device addresses as stated per argument; no
 *    call keeps a caller pointer after it returns (device entry points keep them
 *    until the work queued on the given stream has finished).
 *  - Matrices are row-major, float32 unless stated.  Distances are squared L2
 *    in the caller's original coordinates (rotation invariance, Eq. (1)).
 *  - Results are ascending by (dist, id); a query with fewer than k candidates
 *    is padded with id -1 and dist +INFINITY.
 *  - Errors: every entry point returns a ddc_status; argument validation happens
 *    before the first HIP call; on error the output buffers are unspecified and
 *    ddc_last_error() describes the failure (thread-local text, valid until the
 *    next call on the same thread).  No C++ exception crosses this boundary.
 *  - Threads: an index is immutable after fit/import, except ddc_calibrate,
 *    which replaces the correction table and must not overlap searches on the
 *    same index.  Concurrent searches on one index are allowed.
 */
#ifndef DDC_H
#define DDC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ddc_index ddc_index; /* opaque, library-owned; freed only by ddc_free */

typedef enum {
  DDC_OK = 0,
  DDC_EINVAL = -1,  /* bad argument (checked before any device call) */
  DDC_ENOMEM = -2,  /* device or host allocation failed */
  DDC_EDEVICE = -3, /* a HIP call failed */
  DDC_EIO = -4,     /* file error in save/load */
  DDC_EBUSY = -5,
  DDC_EUNSUP = -6   /* valid request the library does not implement */
} ddc_status;

/* Storage format of the rotated base vectors (the paper stores FP32, Sec. VII-A). */
typedef enum { DDC_F32 = 0, DDC_F16 = 1, DDC_BF16 = 2 } ddc_dtype;

/* Input precision of the query-rotation matrix product (FP32 accumulation either way). */
typedef enum { DDC_ROT_F32 = 0, DDC_ROT_BF16 = 1 } ddc_rot;

/* Distance correction used by the stage tests.
 *  LEARNED : m_s * e_s + beta_s(alpha) > tau with the calibrated table (Sec. V-A, V-B)
 *  LOSSLESS: m_s = 1, beta_s = 0 -- e_s <= dis always (sums of squares, Eq. (1)), so
 *            the result equals NONE exactly (classic partial-distance early exit)
 *  NONE    : no test; every candidate is refined (full-D scan)
 *  ADS     : the random-projection test of ADSampling (Sec. III): prune iff
 *            (D / d_s) e_s > (1 + eps0 / sqrt(d_s))^2 tau, eps0 set by ddc_set_ads_epsilon
 *            (2.1 by default); meant for a DDC_PROJ_HAAR index; significance is ignored
 *  BSAR    : the residual estimate of Alg. 1/2: prune iff e_s + ||x_r||^2 + ||q'_r||^2 -
 *            m sigma_s > tau with sigma_s = sqrt(4 sum_{i > d_s} q'_i^2 lambda_i) (Eq. (2));
 *            m from ddc_set_bsar_multiplier (8 by default), or Phi^-1(1 - significance)
 *            when that is set <= 0; needs the eigenvalues (fit, or lam on import)           */
typedef enum { DDC_CORR_LEARNED = 0, DDC_CORR_LOSSLESS = 1, DDC_CORR_NONE = 2, DDC_CORR_ADS = 3,
               DDC_CORR_BSAR = 4, DDC_CORR_BSAO = 5 } ddc_corr;
/*  BSAO    : the quantization estimate of Sec. V-B ("BSA-O"): before any dimension is read, a
 *            candidate is pruned iff m1 dis' + m3 err + beta(alpha) > tau, with dis' the
 *            asymmetric distance from the query to the candidate's OPQ codewords, err the
 *            candidate's distance to its own codewords and (m1, m3, beta) the calibrated
 *            classifier of the table the search's K selects; survivors are refined to their
 *            exact distance (stage tests there are lossless, so they prune without changing
 *            the result).  Needs an index fitted or imported with pq_m > 0 and its tables.   */

/* Rotation learned by the fit: PCA (Sec. IV-B, Thm. 1) or, for the ablation of Sec. III /
 * IV-B, a Haar-distributed random rotation drawn from the fit seed. */
typedef enum { DDC_PROJ_PCA = 0, DDC_PROJ_HAAR = 1 } ddc_proj;

/* How the target recall r = 1 - alpha of label 0 (true neighbours) is split over
 * the test stages (Sec. V-A "Adaptive Adjustment"):
 *  JOINT      : alpha bounds the probability that a true neighbour is pruned at ANY stage
 *  BONFERRONI : every stage gets alpha / S_t (per-stage target r_i = 1-(1-r)/(D/Delta_d)) */
typedef enum { DDC_CALIB_JOINT = 0, DDC_CALIB_BONFERRONI = 1 } ddc_calib_mode;

typedef struct {
  int32_t nlist;          /* IVF lists (k-means centroids); paper: 4096 (Sec. VII-A) */
  int32_t delta_d;        /* dims per stage, Delta_d (Alg. 2); 32; must be a multiple of 32 */
  int32_t block_b;        /* tau refresh block B, candidates; multiple of 64, 64..1024; 256 */
  int32_t lag_l;          /* tau lag L in blocks, 0..64: the candidates of block b are tested
                             against the tau in force after block b - 1 - L (+inf before it);
                             the calibration replays the same schedule; 0 */
  int32_t kmeans_iters;   /* Lloyd iterations; 25 */
  int32_t kmeans_train_per_list; /* k-means trains on <= this * nlist rows; 256 */
  int32_t calib_k;        /* K_c of the label-0 pairs (KNN of each calibration query), 1..256; 10 */
  int32_t calib_nprobe;   /* N_probe of the label-1 query process; 0 = min(max(1,nlist/8),64) */
  int32_t calib_max_neg;  /* label-1 pairs kept per calibration query; 50 */
  int32_t calib_k_extra[3]; /* further K_c values, ascending above calib_k, 0 = unused: one
                             correction table per K_c; a search with K uses the table of the
                             largest K_c <= K (calib_k's when K is smaller); {0, 0, 0} */
  ddc_dtype storage;      /* base storage format; DDC_F32 */
  ddc_rot rotation;       /* query rotation precision; DDC_ROT_F32 */
  ddc_proj projection;    /* DDC_PROJ_PCA */
  int32_t fp8_lead_dims;  /* 0, or 64: FP8 E4M3 codes of the leading 64 rotated dims (one scale
                             per list tile of 64 vectors) give a first test stage over 64 dims
                             before the stored-precision stages (needs dim >= 64); 0 */
  int64_t pca_sample;     /* PCA rows: all if n <= this, else a SplitMix64 sample; 1,000,000 */
  uint64_t seed;          /* SplitMix64 seed of every random choice in fit; 0 */
  int32_t pq_m;           /* 0, or M subspaces of the quantization estimate (DDC_CORR_BSAO): OPQ
                             eigenvalue allocation of the PCA axes into M subspaces of dim/M axes
                             with 256 codewords each (Sec. VII-A: M = dim/4, dim/8 for GIST);
                             M divides dim, M % 8 == 0, dim/M <= 32, M <= 128; needs PCA; 0 */
  int32_t pq_iters;       /* k-means iterations of every subspace codebook; 25 */
  int64_t pq_train;       /* codebook training rows (SplitMix64 sample); 65,536 (Sec. VII-A) */
} ddc_fit_params;

/* Artifacts of a fitted index, host memory, for ddc_import / ddc_export.
 * Sizes: D = dim, S = ceil(D / delta_d) stages, T = S - 1 test stages, plus one (first in
 * m and resid) when fp8_lead_dims = 64. */
typedef struct {
  int64_t n;              /* base vectors */
  int32_t dim;            /* D */
  int32_t nlist;
  int32_t delta_d;
  int32_t block_b;        /* as ddc_params.block_b */
  int32_t lag_l;          /* as ddc_params.lag_l, 0..64 */
  ddc_dtype storage;
  ddc_rot rotation;
  int32_t fp8_lead_dims;  /* 0 or 64 (import encodes the codes from y) */
  double *mu;             /* [D]        centring mean (Sec. IV-B footnote) */
  double *rot;            /* [D x D]    R, rows = eigenvectors, largest eigenvalue first */
  double *lam;            /* [D]        eigenvalues (export only; may be NULL on import) */
  float *centroids;       /* [nlist x D] IVF centroids in the rotated frame */
  int32_t *assign;        /* [n]        list of every base vector; lists keep ids ascending */
  float *y;               /* [n x D]    stored rotated base: values exactly representable in
                                         `storage` (import rounds anything else to nearest even) */
  int32_t n_tables;       /* correction tables, 0..4 (0: none) */
  int32_t table_k[4];     /* their calibration K_c, ascending */
  int64_t table_n0[4];    /* their label-0 pairs */
  double *m;              /* [n_tables x T] per-stage slope m_s (Sec. V-A: m = -w1/w2) */
  double *resid;          /* [sum n0 x T] residuals g_s(j) = tau_j - m_s e_s(j) of the label-0
                             pairs, table after table */
  uint8_t *codes8;        /* [n x 64]   export only, may be NULL: FP8 codes of vector i (by id) */
  float *scale8;          /* [n]        export only, may be NULL: decode scale of vector i's tile */
  int32_t pq_m;           /* 0, or M: the quantization estimate's subspaces (as in ddc_fit_params) */
  int32_t *pq_perm;       /* [D]        rotated axes of subspace j at [j D/M, (j+1) D/M) */
  float *pq_books;        /* [M x 256 x D/M] codewords */
  uint8_t *pq_codes;      /* [n x M]    export only, may be NULL: codes of vector i (by id); import
                                         encodes them from y and pq_books */
  double *pq_m1, *pq_m3;  /* [n_tables] the BSA-O classifier of each table (NULL on import: none) */
  double *pq_resid;       /* [sum n0]   its label-0 residuals tau_j - m1 dis'_j - m3 err_j, table
                                         after table (NULL on import: none) */
} ddc_artifacts;

typedef struct {
  int64_t n;
  int32_t dim, dim_padded, nlist, delta_d, n_stages, n_test_stages, block_b, lag_l;
  ddc_dtype storage;
  ddc_rot rotation;
  int64_t n0;             /* label-0 pairs over all correction tables */
  int64_t packed_bytes;   /* device bytes of the packed base */
  int64_t total_tiles;    /* 64-vector tiles over all lists */
  int32_t fp8_lead_dims;  /* 0 or 64; n_test_stages counts the FP8 pre-stage when 64 */
  int32_t n_tables;       /* correction tables and their calibration K_c */
  int32_t table_k[4];
  int32_t pq_m;           /* subspaces of the quantization estimate, 0 = none */
  int32_t pq_tables;      /* 1 if the tables hold the BSA-O classifier */
} ddc_index_info;

/* Per-call counters of the scan (sums over all queries of the call). */
typedef struct {
  int64_t candidates;        /* candidates met in probed lists */
  int64_t refined;           /* candidates that reached the last stage (exact distance) */
  int64_t stage_slices;      /* sum over candidates of stages read (one stage = Delta_d dims) */
  int64_t bytes_touched;     /* algorithmic bytes of base data read by the scan */
  int64_t stage_stop[64];    /* candidates whose last stage read was s (0-based; S-1 = refined) */
  int64_t prestage_reads;    /* candidates whose 64-byte FP8 slice was read (tested) */
  int64_t prestage_pruned;   /* candidates the FP8 pre-stage pruned (not in stage_stop) */
  int64_t two_phase_sums;    /* candidates whose first test (dim block 0, or the FP8 pre-stage)
                                read a sum the two-phase scan's first phase computed list by
                                list, or whose full distance the list-major full-D scan
                                computed, instead of the base (see ddc_launch_params) */
  int64_t two_phase_slices;  /* dim-block slices those sums stood in for */
} ddc_search_stats;

/* Fills *p with the defaults listed above. */
ddc_status ddc_fit_params_default(ddc_fit_params *p);

/* Fit an index on the GPU (Sec. IV-B PCA, Sec. II-A IVF, Sec. V-A/V-B calibration).
 *  base  : host [n x dim] float32, finite.   calib: host [n_calib x dim] float32 training
 *  queries held out from base (Sec. VII-A: training queries are removed from the data).
 *  Requires n >= nlist, 1 <= dim <= 4096, n_calib >= 1.  *out = NULL on failure. */
ddc_status ddc_fit(const float *base, int64_t n, int32_t dim, const float *calib,
                   int64_t n_calib, const ddc_fit_params *p, ddc_index **out);

/* Build an index from artifacts (e.g. another implementation's fit).  Every array
 * in `a` is read, none is kept.  resid/m may be NULL with n_tables = 0 (then only LOSSLESS
 * and NONE searches, or a later ddc_calibrate, are possible). */
ddc_status ddc_import(const ddc_artifacts *a, ddc_index **out);

/* Copy the artifacts out.  The caller allocates every array of `a` with the sizes from
 * ddc_index_info (y may be NULL to skip the base).  lam is filled when known. */
ddc_status ddc_export(const ddc_index *ix, ddc_artifacts *a);

ddc_status ddc_index_get_info(const ddc_index *ix, ddc_index_info *info);

/* Write the index to a file (its artifacts: rotation, centroids, lists, stored base,
 * correction tables; FP8 codes are re-encoded on load) / build an index from such a file.
 * DDC_EIO on any file error, a foreign or truncated file, or a checksum mismatch. */
ddc_status ddc_save(const ddc_index *ix, const char *path);
ddc_status ddc_load(const char *path, ddc_index **out);

/* Re-run the calibration of Sec. V-A on new training queries (e.g. ~100 out-of-distribution
 * queries, Sec. V-C) and replace the index's correction tables: one table at K_c = calib_k,
 * or, with calib_k = 0, one at every K_c the index has now.  calib: host [n_calib x dim].
 * The label-1 candidates come from an unpruned search with the index's block_b and lag_l. */
ddc_status ddc_calibrate(ddc_index *ix, const float *calib, int64_t n_calib, int32_t calib_k,
                         int32_t calib_nprobe, int32_t calib_max_neg, uint64_t seed);

/* The correction a search with K uses for a significance alpha = 1 - r (target recall r of
 * label 0): m_out[T] = m_s, beta_out[T] = beta_s(alpha) (FP64, -INFINITY when alpha = 0); T as
 * in ddc_index_info.n_test_stages (the FP8 pre-stage first when present). */
ddc_status ddc_correction(const ddc_index *ix, int32_t k, double significance, ddc_calib_mode mode,
                          double *m_out, double *beta_out);

/* The BSA-O classifier a search with K uses at significance alpha: *m1, *m3 and *beta of
 * m1 dis' + m3 err + beta > tau (beta = -INFINITY when alpha = 0).  EINVAL without BSA-O
 * tables. */
ddc_status ddc_correction_pq(const ddc_index *ix, int32_t k, double significance, double *m1,
                             double *m3, double *beta);

/* Search, host buffers: for every query the k stored vectors nearest in squared Euclidean
 * distance among the nprobe lists whose centroids are nearest (the AKNN problem and the IVF
 * probe step of Sec. II-A), each candidate tested stage by stage with the data-driven
 * correction (Sec. V-A, V-B) at significance = 1 - the target recall r of Sec. V-A "Adaptive
 * Adjustment", survivors refined to their exact distance.  queries: [nq x dim] FP32 row-major;
 * ids (int64, original row ids) / dists (FP32 squared distances in the original coordinates,
 * Eq. (1)): [nq x k], ascending by (dist, id), padded with (-1, +inf).
 * 1 <= k <= 256, 1 <= nprobe <= nlist, 0 <= significance < 1 (0: no learned pruning);
 * otherwise EINVAL before any GPU work.  Inputs are copied; outputs are the caller's. */
ddc_status ddc_search(const ddc_index *ix, const float *queries, int64_t nq, int32_t k,
                      int32_t nprobe, double significance, ddc_corr mode, int64_t *ids,
                      float *dists, ddc_search_stats *stats);

/* Search with a K and an N_probe per query (host buffers): the search of ddc_search (Sec.
 * II-A, V-A, V-B) where every query carries its own K and N_probe.  k[nq], nprobe[nq], each
 * within the bounds of ddc_search (EINVAL otherwise, before any GPU work); results of query i
 * at out_offsets[i] .. out_offsets[i] + k[i] (caller-built CSR with
 * out_offsets[i+1] - out_offsets[i] >= k[i]); ids/dists sized out_offsets[nq]. */
ddc_status ddc_search_var(const ddc_index *ix, const float *queries, int64_t nq, const int32_t *k,
                          const int32_t *nprobe, double significance, ddc_corr mode,
                          const int64_t *out_offsets, int64_t *ids, float *dists,
                          ddc_search_stats *stats);

/* Search on device buffers (the search of ddc_search / ddc_search_var: Sec. II-A, V-A,
 * V-B), queued on `hip_stream` (a hipStream_t; NULL = default stream), no host
 * synchronisation.  d_queries [nq x dim]; d_k / d_nprobe: per-query arrays or NULL
 * to use k_all / nprobe_all; k_max / nprobe_max bound them (the host checks the bounds
 * themselves; the device clamps a per-query entry outside [1, k_max] or [1, nprobe_max]
 * into that range rather than trusting it); d_out_offsets: CSR as in
 * ddc_search_var or NULL for dense [nq x k_all]; d_ids int64 / d_dists float32 outputs;
 * d_counters: NULL or device int64[4 + 64 + 3] (added to): candidates, refined, stage
 * slices, two-phase sums read, stage_stop[64], prestage_reads, prestage_pruned, dim-block slices
 * the two-phase sums stood in for (read by the first phase instead of the query's scan).
 * Scratch: the index keeps one grow-only device workspace per stream (rotated queries, coarse
 * distances, probes; about nq x (dim + nlist + nprobe_max) x 4 bytes for nq <= 32,768), made on
 * the stream's first call and reused by the next ones, freed with the index; calls on one
 * stream from several host threads must therefore not overlap.  Under graph capture the
 * scratch comes from the stream-ordered pool instead. */
ddc_status ddc_search_device(const ddc_index *ix, const float *d_queries, int64_t nq,
                             const int32_t *d_k, int32_t k_all, int32_t k_max,
                             const int32_t *d_nprobe, int32_t nprobe_all, int32_t nprobe_max,
                             double significance, ddc_corr mode, const int64_t *d_out_offsets,
                             int64_t *d_ids, float *d_dists, int64_t *d_counters,
                             void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the search of ddc_search_device, same arguments,
 * same kernels, same results, but its correction rows and scratch (rotated queries, coarse
 * distances, probes, query orders) come from one fixed device array of
 * ddc_search_device_noalloc_bytes() bytes (64 MiB) inside the library, which each device it
 * runs on holds until the process ends.  The call allocates and frees no device memory, never
 * times or tunes a launch shape (an untuned size class takes the fixed rule), and queues a
 * copy of the correction rows (host memory held by the index) and the kernels on `hip_stream`.
 * Size limit: the scratch of one chunk of min(nq, 32768) queries, about
 * (dim rounded up to 32 + nlist + nprobe_max + 5) x 4 bytes per query, plus 16 KiB of tables
 * and (nlist + 1) x 4 bytes, must fit, else
 * EINVAL before any device work, with the largest query count that fits in the message
 * (e.g. nlist 4096, dim 128, nprobe_max 48: about 3,900 queries).
 * Every call on one device shares that device's array and leaves its contents behind (the
 * kernels clear what must start at zero): calls that overlap on one device, from any stream or
 * thread, race and give wrong results; serialise them (one stream, or events).  Other errors as
 * ddc_search_device. */
ddc_status ddc_search_device_noalloc(const ddc_index *ix, const float *d_queries, int64_t nq,
                                     const int32_t *d_k, int32_t k_all, int32_t k_max,
                                     const int32_t *d_nprobe, int32_t nprobe_all, int32_t nprobe_max,
                                     double significance, ddc_corr mode,
                                     const int64_t *d_out_offsets, int64_t *d_ids, float *d_dists,
                                     int64_t *d_counters, void *hip_stream);
size_t ddc_search_device_noalloc_bytes(void);

/* Approximation accuracy of a distance estimate alone (the direct scan of the paper's
 * approximation-accuracy experiment, Sec. VII Exp-7 and its Table III): for every query, the
 * k candidates of the nprobe nearest lists (nprobe = nlist: the whole base) with the smallest
 * estimated squared distance over the leading `dims` rotated dimensions, with no correction and
 * no refinement.  Estimators:
 *   DDC_EST_PARTIAL  (dim / min(dims, dim)) * sum_{i < dims} (q'_i - y_i)^2: the projection
 *                    estimate (on a PCA index the paper's "PCA" column, on a Haar index its
 *                    random-projection "Rand" column, unbiased there);
 *   DDC_EST_RESIDUAL sum_{i < dims} (q'_i - y_i)^2 + ||y_r||^2 + ||q'_r||^2 = C1 - C2 of
 *                    Alg. 1 (the residual decomposition behind the paper's third column).
 * dims: a multiple of 32 in [32, dim rounded up to 32]; dims >= dim gives exact distances.
 * ids/dists: host [nq x k], ascending by (estimate, id), dists = the estimates, padding
 * (-1, +inf).  Errors: EINVAL for bad sizes, k, nprobe, dims or estimator (before any GPU
 * work). */
typedef enum { DDC_EST_PARTIAL = 0, DDC_EST_RESIDUAL = 1 } ddc_estimator;
ddc_status ddc_search_estimate(const ddc_index *ix, const float *queries, int64_t nq, int32_t k,
                               int32_t nprobe, int32_t dims, ddc_estimator estimator, int64_t *ids,
                               float *dists);

/* Intermediates of the first two hot-path steps for parity checks (host buffers):
 * q_rot [nq x dim] = R (q - mu) as the search computes it; probes [nq x nprobe] in probe
 * order (ascending centroid distance, then list id). */
ddc_status ddc_debug_intermediates(const ddc_index *ix, const float *queries, int64_t nq,
                                   int32_t nprobe, float *q_rot, int32_t *probes);

/* Allocation failure injection, for tests of the error paths: spec "alloc:<n>" makes the n-th
 * device or pinned-host allocation the library makes from now on (any thread, any call) fail
 * before the runtime is asked, so that call returns DDC_ENOMEM having released what it had
 * allocated (a failed fit / import / load leaves *out = NULL; a failed search leaves the index
 * as it was); "alloc:0" turns it off.  The environment variable DDC_FAULT=alloc:<n>, read once
 * when the library first allocates, has the same effect.  EINVAL for another spec. */
ddc_status ddc_set_fault(const char *spec);
/* Device and pinned-host allocations the library holds right now (count; bytes = the device
 * ones), for leak checks after failed calls.  EINVAL on a NULL argument. */
ddc_status ddc_live_allocations(int64_t *count, int64_t *bytes);

/* Per-kernel timing of the search pipeline with HIP events recorded on the launch stream
 * around every kernel of every later search on this index (enable = 1) or none (0).
 * Kernels: 0 query rotation (A1), 1 coarse centroid distances (A2), 2 probe selection (A2),
 * 3 pruned scan + top-K merge + finalize (A3-A5), 4 the two-phase scan's first phase (its
 * list grouping and stage-1 sums).  ddc_get_kernel_timing waits for the
 * recorded events, adds their elapsed times to ms_total[5] and counts to launches[5]
 * (both caller arrays, overwritten), and clears the record when reset != 0. */
ddc_status ddc_set_kernel_timing(ddc_index *ix, int enable);
ddc_status ddc_get_kernel_timing(ddc_index *ix, double *ms_total, int64_t *launches, int reset);

/* eps0 of the DDC_CORR_ADS test (> 0; 2.1 by default, the value the paper uses for it). */
ddc_status ddc_set_ads_epsilon(ddc_index *ix, double eps0);
/* Multiplier m of the DDC_CORR_BSAR test (8 by default, the paper's value for SIFT, GIST and
 * DEEP; m <= 0: m = Phi^-1(1 - significance) per search). */
ddc_status ddc_set_bsar_multiplier(ddc_index *ix, double m);

/* Launch shape of the pruned scan (A3-A5).  None of these changes any result bit (every
 * candidate's partial distances are summed in the same order in every variant); they only
 * trade occupancy, latency and bytes read.  waves_per_query: 1 (one wavefront runs a query's
 * whole scan, four queries per workgroup), 4 (a workgroup per query, the tiles of every
 * candidate block split over its four wavefronts; on an index with lag_l >= 3 instead the
 * lag-parallel scan below) or 2 (the lag-parallel scan with two wavefronts, on an index with
 * lag_l >= 1; elsewhere, and in unpruned searches, as 1), 0 = tuned.  Lag-parallel scan with W
 * wavefronts: wavefront j scans the blocks b with b mod W = j, W blocks at once, each tested
 * against the lagged tau that is already known when its group of W starts, and the group's
 * survivors are merged in block order, so results and counters equal those of
 * waves_per_query = 1.  lookahead: 0 (one dim block
 * per dependent load), 1 (when few candidates are alive, one load covers up to 8 consecutive
 * dim blocks of each), -1 = tuned.  query_order: group queries with the same first list;
 * xcd_swizzle: give each XCD a contiguous query range (0 or 1 each).  Tuned values are picked
 * per (queries, N_probe, K, pruned or not) size class on the first search of that class by
 * timing each candidate on the actual launch (that search synchronises its stream once); a
 * stream that is capturing a graph, and the server (which must not stall), get a fixed rule
 * for classes not tuned yet.  persistent: 0 (one workgroup per query group, the grid covers
 * the batch), 1 (the grid holds only the workgroups the device keeps resident at once; each
 * takes the next query from a device counter until none is left, queries ordered by
 * decreasing candidate count so long scans start first; query_order does not apply), -1 =
 * tuned.  two_phase: 0 (every candidate's first test reads its data in its query's scan), 1
 * (for the learned and fixed-table tests whose first test follows dim block 0 with Delta_d = 32,
 * or is the FP8 pre-stage: first that test's partial distance of every candidate of every
 * probed list is computed list by list, each stored tile read once for all the queries that
 * probe its list, in the scan's own arithmetic (or on the matrix cores: stage1_matrix below);
 * the scan then tests those sums and reads the survivors' remaining dims only; its scratch
 * holds one float per candidate of the batch), -1 = tuned (fixed rule: on once a list is
 * probed by four or more queries on average).
 * full_d_matrix (not result-invariant, never tuned; 0 or 1): with 1, scans without a test
 * (DDC_CORR_NONE, or significance 0 in the learned mode) run list by list: for every stored
 * tile and every query probing its list the distance ||q'||^2 + ||y||^2 - 2 <q', y> is formed
 * on the matrix cores (FP32 products; each tile read once for all those queries), clamped at 0,
 * and the per-query scan merges these distances.  The result is the exact full-D search up to
 * FP32 rounding of that expanded form (its ids and distances can differ from the default scan's
 * in the last bits and at near ties).  stage1_matrix (0, 1 or 2; 0 and 1 result-invariant): with
 * 1, the first phase of a two-phase scan whose first test follows dim block 0 (not the FP8
 * pre-stage) forms
 * each candidate's stage-1 distance as ||q'_1||^2 + ||y_1||^2 - 2 <q'_1, y_1> over that block on
 * the matrix cores (FP32 products, each stored tile's block 0 read once and kept in registers for
 * all the queries probing its list), clamped at 0.  The scan prunes on such a sum only where the
 * first test prunes every value within its proven FP32 error bound (2^-12 (3 ||q'_1||^2 + 2 e1),
 * about 48 times the worst case); every other candidate re-reads dim block 0 and takes the test
 * on the sum in the scan's own arithmetic, so ids, distances and counters equal the one-phase
 * scan's bit for bit.  With 2 (not result-invariant) the scan takes the expanded-form sums as
 * they are: its results equal the one-phase scan's up to FP32 rounding of the first block's
 * partial distance (ids can differ at near-threshold decisions and near ties), and no candidate
 * re-reads dim block 0; with the FP8 pre-stage, mode 2 also forms the pre-stage's sums over the
 * leading 64 dims this way (from the decoded codes; the pre-stage's decisions then hold up to
 * FP32 rounding, and its survivors' distances are exact as ever).  0 keeps the first phase in
 * the scan's own arithmetic.  waves_per_simd (result-invariant; 0 = tuned, 4 or 5): the
 * register budget of the one-wave kernel of the lag-free learned and fixed-table tests (a
 * second build for five waves per SIMD spills a few registers to a private segment the HIP
 * runtime provides, to trade them for occupancy; searches with a fixed workspace,
 * ddc_search_device_noalloc and the server, always use the four-wave build); other kernels
 * ignore it.  Defaults: 0, -1, 1, 1, -1, -1, 0, 0, 0. */
typedef struct {
  int32_t waves_per_query, lookahead, query_order, xcd_swizzle, persistent, two_phase;
  int32_t full_d_matrix, stage1_matrix, waves_per_simd;
} ddc_launch_params;
ddc_status ddc_set_launch(ddc_index *ix, const ddc_launch_params *p);
ddc_status ddc_get_launch(const ddc_index *ix, ddc_launch_params *p);
/* The scan variant a search of nq queries with this K, N_probe and mode runs: waves (1 or 4),
 * lookahead (0 or 1), persistent (0 or 1; nullable), two_phase (0 or 1; nullable) and
 * waves_per_simd (4 or 5, the register budget of the kernel; nullable).  A size class not tuned
 * yet reports the fixed rule's choice. */
ddc_status ddc_scan_variant(ddc_index *ix, int64_t nq, int32_t k_max, int32_t nprobe_max,
                            ddc_corr mode, int32_t *waves, int32_t *lookahead, int32_t *persistent,
                            int32_t *two_phase, int32_t *waves_per_simd);

/* ---- continuous-batching server --------------------------------------------------------
 * A scheduler thread admits queued requests into micro-batches on n_streams HIP streams while
 * the device bytes of all batches in flight (queries, results, search scratch) stay within
 * hbm_budget_bytes; batches on different streams overlap on the GPU and a request arriving
 * while others run starts as soon as a stream and budget are free.  Every query keeps its own
 * K and N_probe; its result is the same as searching it alone (ddc_search_var).  The index
 * must outlive the server.  Slot buffers for max_batch queries, each stream's search scratch
 * included, are allocated at creation: serving itself allocates no device memory. */
typedef struct ddc_server ddc_server;
typedef struct {
  int32_t n_streams;        /* concurrent micro-batches, 1..16 */
  int32_t max_batch;        /* queries per micro-batch and per request, 1..65536 */
  int64_t hbm_budget_bytes; /* device bytes all in-flight batches may use */
  double significance;      /* alpha of every request, [0, 1) */
  ddc_corr mode;            /* the test of every request, any of ddc_search's under its conditions
                               (DDC_CORR_BSAO: an index with pq_m > 0 and its tables; DDC_CORR_BSAR:
                               the rotation's eigenvalues); EINVAL at creation otherwise */
} ddc_server_params;
typedef struct {
  int64_t requests_done, queries_done, rejected;
  double qps;               /* queries_done / (last completion - first submission), s^-1 */
  double p50_ms, p99_ms, max_ms; /* request latency: submission -> results on the host */
  int64_t budget_peak_bytes;     /* most device bytes in flight at once */
  int32_t max_concurrent;        /* most batches in flight at once */
} ddc_server_stats;

ddc_status ddc_server_create(const ddc_index *ix, const ddc_server_params *p, ddc_server **out);
/* Queue nq queries (host [nq x dim], copied) with per-query k[nq] (1..256) and nprobe[nq]
 * (1..min(nlist, 4096)); returns at once with a ticket.  DDC_EBUSY when the request alone needs
 * more device memory than the budget (it is never admitted). */
ddc_status ddc_server_submit(ddc_server *s, const float *queries, int32_t nq, const int32_t *k,
                             const int32_t *nprobe, uint64_t *ticket);
/* *done = 1 and results copied (ids/dists sized sum(k), query-major, each query ascending,
 * padded) once the request finished, else *done = 0.  t_done_ns (nullable): CLOCK_MONOTONIC
 * time at which the server saw the results on the host.  A finished ticket is forgotten. */
ddc_status ddc_server_poll(ddc_server *s, uint64_t ticket, int64_t *ids, float *dists, int *done,
                           uint64_t *t_done_ns);
ddc_status ddc_server_get_stats(ddc_server *s, ddc_server_stats *st);
/* Finishes every queued request, then frees the server. */
void ddc_server_destroy(ddc_server *s);

void ddc_free(ddc_index *ix);
const char *ddc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DDC_H */
