"""FP64 reference implementation (oracle) of the method of "Effective and General
Distance Computation for Approximate Nearest Neighbor Search".

TEST INFRASTRUCTURE ONLY -- see the package docstring.  Plain, slow and written
to be checked against the paper by eye.  Every floating-point step is FP64
unless the step *is* a rounding to a storage format.

What is computed (paper section in brackets):

* exact KNN under the squared Euclidean distance            [Sec. II-A]
* PCA rotation: centring, covariance, eigenvectors as rows  [Sec. IV-B, Thm. 1]
* IVF lists by k-means, probe the N_probe nearest centroids [Sec. II-A, IVF]
* the pruned refinement: per block of candidates, per stage of Delta_d
  dimensions, the partial (PCA-projected) squared distance dis'_s is tested
  with the learned linear classifier  m_s * dis'_s + beta_s > tau  and the
  candidate is pruned, else refined; the result queue keeps the K best and tau
  is its K-th distance                                       [Sec. V-A, V-B; Alg. 2 loop]
* calibration: logistic regression per stage on (dis', tau) features with
  KNN pairs as label 0 and pairs met in a query process as label 1, then the
  bias is moved to reach a target recall of label 0          [Sec. V-A "Parameter
  Learning", "Adaptive Adjustment"; Sec. VII-A implementation details]

Readings of points the paper leaves open are listed in the design notes; the
ones that change results are repeated next to the code that takes them.

Parity status: every function here is pinned by tests under ``tests/`` that
check it against closed forms, invariants, brute force or library routines
(never against its own formula retyped).  Values printed in the paper's figures
and tables cannot be reproduced (their datasets are absent): those are parity
unpinned and no function here claims them.
"""
from __future__ import annotations

import heapq
import math

import numpy as np

# --------------------------------------------------------------------------------------
# Counter-based random keys (SplitMix64, Steele, Lea & Flood, OOPSLA 2014).  Random
# choices the method makes during fit (PCA sample, k-means init/sample, the label-1
# subsample, the calibration sample) are "the m items with the smallest keys", keys
# being SplitMix64 outputs of a counter.  The GPU library implements the same
# published generator on its own.
# --------------------------------------------------------------------------------------
_M64 = (1 << 64) - 1
TAG_PCA, TAG_KMEANS_INIT, TAG_KMEANS_SAMPLE, TAG_NEG, TAG_CALIB, TAG_HAAR = 1, 2, 3, 4, 5, 6
TAG_PQ_SAMPLE = 7


def splitmix64(x):
    """SplitMix64 output for state ``x`` (uint64 array): add the golden gamma, then the
    two xor-shift-multiply rounds and a final xor-shift."""
    x = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = x + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def ctr_key(seed: int, tag: int, idx) -> np.ndarray:
    """key = splitmix64(splitmix64(seed + tag) + idx)  (all mod 2^64)."""
    base = splitmix64(np.uint64((seed + tag) & _M64))
    with np.errstate(over="ignore"):
        return splitmix64(base + np.asarray(idx, dtype=np.uint64))


def select_by_key(n: int, m: int, seed: int, tag: int) -> np.ndarray:
    """Indices of the ``m`` smallest keys among 0..n-1 (ties by index), ascending index order."""
    if m >= n:
        return np.arange(n, dtype=np.int64)
    keys = ctr_key(seed, tag, np.arange(n, dtype=np.uint64))
    order = np.lexsort((np.arange(n), keys))
    return np.sort(order[:m]).astype(np.int64)


# --------------------------------------------------------------------------------------
# Exact KNN  [Sec. II-A]: K smallest dis(p, q) = ||p - q||^2, ties by id.
# --------------------------------------------------------------------------------------

def sq_dist_direct(X: np.ndarray, q: np.ndarray) -> np.ndarray:
    """||x - q||^2 for each row x of X, summed term by term in FP64."""
    d = np.asarray(X, dtype=np.float64) - np.asarray(q, dtype=np.float64)[None, :]
    return np.einsum("ij,ij->i", d, d)


def topk_lex(dist: np.ndarray, ids: np.ndarray, k: int):
    """The k smallest (dist, id) pairs in lexicographic order."""
    order = np.lexsort((ids, dist))[:k]
    return ids[order], dist[order]


def bruteforce_knn(X: np.ndarray, Q: np.ndarray, k: int, chunk: int = 256):
    """Exact K nearest neighbours of every query row, FP64.

    Distances are screened with the algebraic expansion ||x||^2 + ||q||^2 - 2<x,q>
    (one matrix product), then every point whose screened distance lies within a
    safe margin of the screened K-th distance is recomputed term by term, and the
    answer is taken from the recomputed values.  The margin (1e-10 of the norms'
    scale) is orders of magnitude above the FP64 error of the expansion for D<=4096,
    so the result equals the term-by-term definition.

    Returns ids (nq, k) int64 padded with -1 and dists (nq, k) float64 padded with inf.
    """
    X = np.asarray(X, dtype=np.float64)
    Q = np.asarray(Q, dtype=np.float64)
    n = X.shape[0]
    nq = Q.shape[0]
    kk = min(k, n)
    ids_out = np.full((nq, k), -1, dtype=np.int64)
    d_out = np.full((nq, k), np.inf)
    xn = np.einsum("ij,ij->i", X, X)
    all_ids = np.arange(n, dtype=np.int64)
    for s in range(0, nq, chunk):
        Qc = Q[s:s + chunk]
        qn = np.einsum("ij,ij->i", Qc, Qc)
        approx = Qc @ X.T                  # screened ||x||^2 + ||q||^2 - 2 <x, q>, in place
        approx *= -2.0
        approx += xn[None, :]
        approx += qn[:, None]
        for r in range(Qc.shape[0]):
            a = approx[r]
            if kk == 0:
                continue
            kth = np.partition(a, kk - 1)[kk - 1]
            margin = 1e-10 * (xn.max() + qn[r]) + 1e-300
            cand = np.nonzero(a <= kth + margin)[0]
            exact = sq_dist_direct(X[cand], Qc[r])
            i, d = topk_lex(exact, all_ids[cand], kk)
            ids_out[s + r, :kk] = i
            d_out[s + r, :kk] = d
    return ids_out, d_out


# --------------------------------------------------------------------------------------
# PCA rotation  [Sec. IV-B Thm. 1 and its Remark; centring per the footnote of Sec. IV-B]
# --------------------------------------------------------------------------------------

def pca_fit(X: np.ndarray, pca_sample: int = 1_000_000, seed: int = 0) -> dict:
    """mu = mean of the PCA sample, C = (1/#P) sum (x-mu)(x-mu)^T, and R whose rows are the
    eigenvectors of C ordered by eigenvalue, largest first.

    Readings: the sample P is all rows when n <= pca_sample, otherwise the pca_sample rows
    with the smallest SplitMix64 keys; eigenvalue ties keep the solver's index order; each
    eigenvector is signed so that its largest-magnitude component is positive (first such
    component on ties).  The eigen-decomposition itself is a library routine (LAPACK syevd).
    """
    X = np.asarray(X)
    n, D = X.shape
    rows = select_by_key(n, pca_sample, seed, TAG_PCA) if n > pca_sample else None
    P = np.asarray(X if rows is None else X[rows], dtype=np.float64)
    mu = P.mean(axis=0)
    Pc = P - mu[None, :]
    C = (Pc.T @ Pc) / P.shape[0]
    lam, V = np.linalg.eigh(C)                 # ascending
    order = np.lexsort((np.arange(D), -lam))   # descending, index tie-break
    lam, V = lam[order], V[:, order]
    for j in range(D):
        v = V[:, j]
        i = int(np.argmax(np.abs(v)))          # first index of the largest magnitude
        if v[i] < 0:
            V[:, j] = -v
    return dict(mu=mu, cov=C, lam=lam, R=np.ascontiguousarray(V.T))


def gaussian_by_key(count: int, seed: int, tag: int) -> np.ndarray:
    """``count`` standard normals by the Box-Muller transform (Box & Muller 1958) of pairs of
    SplitMix64 counter keys: u1 = (key(2i) >> 11 + 1) 2^-53 in (0, 1], u2 = (key(2i+1) >> 11)
    2^-53 in [0, 1); z(2i) = r cos(2 pi u2), z(2i+1) = r sin(2 pi u2), r = sqrt(-2 ln u1)."""
    npair = (count + 1) // 2
    k = ctr_key(seed, tag, np.arange(2 * npair, dtype=np.uint64))
    u1 = ((k[0::2] >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0 ** -53
    u2 = (k[1::2] >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    r = np.sqrt(-2.0 * np.log(u1))
    z = np.empty(2 * npair)
    z[0::2] = r * np.cos(2.0 * math.pi * u2)
    z[1::2] = r * np.sin(2.0 * math.pi * u2)
    return z[:count]


def haar_rotation(D: int, seed: int) -> np.ndarray:
    """A Haar-distributed random rotation (the random projection of the ablation against
    PCA, Sec. III / IV-B): Q of the QR factorisation of a D x D matrix of standard normals
    (row-major from ``gaussian_by_key``), each column's sign flipped so that the triangular
    factor has a positive diagonal (Mezzadri 2007).  Returned with the rotated axes as rows."""
    Z = gaussian_by_key(D * D, seed, TAG_HAAR).reshape(D, D)
    Q, T = np.linalg.qr(Z)
    Q = Q * np.where(np.diag(T) < 0, -1.0, 1.0)[None, :]
    return np.ascontiguousarray(Q.T)


def rotate(X: np.ndarray, mu: np.ndarray, R: np.ndarray) -> np.ndarray:
    """x_D = R (x - mu)  [Eq. (1): the rotation preserves ||x - q||^2]."""
    return (np.asarray(X, dtype=np.float64) - mu[None, :]) @ R.T


# --------------------------------------------------------------------------------------
# Storage formats.  The paper stores FP32 (Sec. VII-A); lower-precision storage is a
# deployment choice.  Reading: a stored value is the FP64 rotated value rounded to FP32
# (round to nearest even), then, for FP16/BF16, rounded again (nearest even) to the
# narrow format.  Every distance "exact" for a stored vector is exact for its stored value.
# --------------------------------------------------------------------------------------

def _bf16_round_f32(a32: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (nearest, ties to even) and widen back to float32."""
    u = a32.astype(np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    return u.astype(np.uint32).view(np.float32)


def round_storage(y: np.ndarray, dtype: str) -> np.ndarray:
    """Stored value of FP64 ``y`` for storage ``dtype`` in {'f32', 'f16', 'bf16'}, as FP64."""
    y32 = np.asarray(y, dtype=np.float64).astype(np.float32)
    if dtype == "f32":
        out = y32
    elif dtype == "f16":
        out = y32.astype(np.float16).astype(np.float32)
    elif dtype == "bf16":
        out = _bf16_round_f32(y32)
    else:
        raise ValueError(dtype)
    return out.astype(np.float64)


def rotate_bf16(X: np.ndarray, mu: np.ndarray, R: np.ndarray) -> np.ndarray:
    """x_D = R (x - mu) [Eq. (1)] with both operands of the product rounded to bfloat16.

    Reading for a query rotation on BF16 matrix units (the paper rotates in FP32): the
    query and the mean are FP32 values, the centred query is their FP32 difference
    (correctly rounded), then rounded to bfloat16 (nearest, ties to even); every entry of R
    is rounded to FP32 and then to bfloat16 the same way (the storage rule of
    ``round_storage``).  The product of the two rounded operands is then taken exactly up
    to FP64 rounding, so this reading fixes the operands and leaves only the summation
    order of an FP32 accumulation open."""
    x32 = np.asarray(X, dtype=np.float32)
    mu32 = np.asarray(mu, dtype=np.float64).astype(np.float32)
    c = _bf16_round_f32((x32 - mu32[None, :]).astype(np.float32)).astype(np.float64)
    Rb = _bf16_round_f32(np.asarray(R, dtype=np.float64).astype(np.float32)).astype(np.float64)
    return c @ Rb.T


def rotate_as(X: np.ndarray, mu: np.ndarray, R: np.ndarray, rotation: str = "f32") -> np.ndarray:
    """The query rotation a search takes: ``rotate`` (FP64, the paper's FP32 reading within
    rounding) for rotation 'f32', ``rotate_bf16`` for 'bf16'."""
    if rotation == "f32":
        return rotate(X, mu, R)
    if rotation == "bf16":
        return rotate_bf16(X, mu, R)
    raise ValueError(rotation)


# --------------------------------------------------------------------------------------
# FP8 pre-stage codes.  Not in the paper (it stores FP32 only, Sec. VII-A); the paper's
# argument that the learned correction absorbs whatever error the estimate carries
# (Sec. V-A, V-B) is what makes a coarser first test usable.  Format: OCP 8-bit floating
# point E4M3 (OFP8 spec v1.0): sign, 4 exponent bits with bias 7, 3 mantissa bits,
# subnormals, no infinities, S.1111.111 = NaN, largest finite 448.  The leading `lead`
# rotated dims of every stored vector are coded with one scale per (list, tile of 64
# consecutive list positions): s = max |y| over the tile / 448 in FP32 (1 if the tile is all
# zero), code = E4M3 round-to-nearest-even of fp32(y / s) with saturation to +-448, decoded
# value = fp32(value(code) * s).  Reading: the code is an integer decided by FP32 values,
# so every step that decides it is taken in FP32 (division and product correctly rounded).
# --------------------------------------------------------------------------------------
FP8_MAX = 448.0
FP8_TILE = 64


def fp8_e4m3_value(code: int) -> float:
    """Value of one E4M3 code by the format's definition (NaN for S.1111.111)."""
    code = int(code) & 0xFF
    sign = -1.0 if code & 0x80 else 1.0
    e = (code >> 3) & 0xF
    m = code & 0x7
    if e == 0xF and m == 0x7:
        return math.nan
    if e == 0:
        return sign * m * 2.0 ** -9              # subnormal: m/8 * 2^(1-7)
    return sign * (1.0 + m / 8.0) * 2.0 ** (e - 7)


FP8_TABLE = np.array([fp8_e4m3_value(c) for c in range(256)], dtype=np.float64)


def fp8_e4m3_encode(v: np.ndarray) -> np.ndarray:
    """E4M3 code of every FP32 value: nearest finite value, ties to the even mantissa,
    magnitudes beyond 448 saturate to 448; the sign bit is the sign bit of v."""
    v = np.asarray(v, dtype=np.float32).astype(np.float64)   # exact
    a = np.abs(v)
    code = np.zeros(v.shape, dtype=np.int64)
    sub = a < 2.0 ** -6
    # subnormal range: grid 2^-9, code = number of grid steps (8 steps = smallest normal)
    code[sub] = np.rint(a[sub] / 2.0 ** -9).astype(np.int64)
    nrm = ~sub
    if nrm.any():
        _, ex = np.frexp(a[nrm])                  # a = f * 2^ex, f in [0.5, 1)
        e = ex.astype(np.int64) - 1                # a in [2^e, 2^(e+1))
        e = np.minimum(e, 8)
        n = np.rint(a[nrm] / np.ldexp(1.0, e - 3)).astype(np.int64)   # in [8, 16]
        code[nrm] = ((e + 7) << 3) + (n - 8)       # n = 16 carries into the next exponent
    code = np.minimum(code, 0x7E)                  # saturate (0x7F would be NaN)
    code |= np.where(np.signbit(v), 0x80, 0)
    return code.astype(np.uint8)


def fp8_encode_lead(Y: np.ndarray, list_off: np.ndarray, list_ids: np.ndarray, lead: int = 64):
    """Codes of the leading ``lead`` dims of every stored vector (rows of Y by id), with
    one scale per (list, 64-position tile).  Returns dict(lead, codes (n, lead) uint8,
    scale (n,) float32 = the scale of the vector's tile, dec (n, lead) FP64 decoded)."""
    Y = np.asarray(Y, dtype=np.float64)
    n = Y.shape[0]
    codes = np.zeros((n, lead), dtype=np.uint8)
    scale = np.ones(n, dtype=np.float32)
    dec = np.zeros((n, lead), dtype=np.float64)
    for j in range(list_off.shape[0] - 1):
        lo, hi = int(list_off[j]), int(list_off[j + 1])
        for t0 in range(lo, hi, FP8_TILE):
            ids = list_ids[t0:min(t0 + FP8_TILE, hi)]
            a = Y[ids, :lead].astype(np.float32)
            amax = np.float32(np.abs(a).max())
            s = np.float32(amax / np.float32(FP8_MAX)) if amax > 0 else np.float32(1.0)
            c = fp8_e4m3_encode(a / s)                                # FP32 division
            codes[ids] = c
            scale[ids] = s
            dec[ids] = (FP8_TABLE[c].astype(np.float32) * s).astype(np.float64)  # FP32 product
    return dict(lead=lead, codes=codes, scale=scale, dec=dec)


# --------------------------------------------------------------------------------------
# IVF  [Sec. II-A "Inverted File-Based"]: k-means buckets, probe the nearest centroids.
# --------------------------------------------------------------------------------------

def nearest_centroid(Y: np.ndarray, C: np.ndarray, chunk: int = 8192) -> np.ndarray:
    """argmin_j ||y - c_j||^2 per row (ties to the lower j).  Screened through the
    expansion, then every centroid within a safe margin of the screened minimum is
    recomputed term by term (same argument as in ``bruteforce_knn``)."""
    Y = np.asarray(Y, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    cn = np.einsum("ij,ij->i", C, C)
    out = np.empty(Y.shape[0], dtype=np.int64)
    jj = np.arange(C.shape[0])
    for s in range(0, Y.shape[0], chunk):
        Yc = Y[s:s + chunk]
        yn = np.einsum("ij,ij->i", Yc, Yc)
        a = Yc @ C.T                      # screened ||y||^2 + ||c||^2 - 2 <y, c>, in place
        a *= -2.0
        a += cn[None, :]
        a += yn[:, None]
        amin = a.min(axis=1)
        margin = 1e-10 * (cn.max() + yn) + 1e-300
        close = a <= (amin + margin)[:, None]
        out[s:s + Yc.shape[0]] = np.argmax(close, axis=1)      # single close centroid
        for r in np.nonzero(close.sum(axis=1) > 1)[0]:         # several: recompute exactly
            cand = np.nonzero(close[r])[0]
            ex = sq_dist_direct(C[cand], Yc[r])
            best = np.lexsort((jj[cand], ex))[0]
            out[s + r] = cand[best]
    return out


def kmeans(Y: np.ndarray, nlist: int, iters: int = 25, seed: int = 0, train_per_list: int = 256):
    """Lloyd's k-means.  Readings: training set = all rows if n <= train_per_list * nlist,
    else that many rows with the smallest SplitMix64 keys; initial centroids = the nlist
    training rows with the smallest keys (in ascending row order); assignment ties go to
    the lower centroid index; an empty cluster keeps its previous centroid; after the
    iterations every row of Y is assigned once more."""
    Y = np.asarray(Y, dtype=np.float64)
    n = Y.shape[0]
    cap = train_per_list * nlist
    train = Y if n <= cap else Y[select_by_key(n, cap, seed, TAG_KMEANS_SAMPLE)]
    init = select_by_key(train.shape[0], nlist, seed, TAG_KMEANS_INIT)
    C = train[init].copy()
    for _ in range(iters):
        a = nearest_centroid(train, C)
        for j in range(nlist):
            members = train[a == j]
            if members.shape[0]:
                C[j] = members.mean(axis=0)
    return C, nearest_centroid(Y, C)


def build_lists(assign: np.ndarray, nlist: int):
    """List j holds the ids assigned to centroid j in ascending id order.
    Returns (offsets[nlist+1], ids in list order)."""
    assign = np.asarray(assign, dtype=np.int64)
    ids = np.lexsort((np.arange(assign.shape[0]), assign)).astype(np.int64)
    counts = np.bincount(assign, minlength=nlist)
    off = np.zeros(nlist + 1, dtype=np.int64)
    off[1:] = np.cumsum(counts)
    return off, ids


def probe_order(qrot: np.ndarray, C: np.ndarray, nprobe: int):
    """The nprobe centroids nearest to the rotated query, ascending by (distance, list id).
    Also returns the smallest relative gap between consecutive distances among the first
    nprobe+1 (a near tie there can reorder or swap probed lists under other rounding)."""
    d = sq_dist_direct(C, qrot)
    order = np.lexsort((np.arange(C.shape[0]), d))
    top = order[:nprobe]
    ds = d[order[:min(nprobe + 1, C.shape[0])]]
    if ds.shape[0] > 1:
        gap = np.abs(np.diff(ds)) / np.maximum(np.abs(ds[1:]), 1e-300)
        margin = float(gap.min())
    else:
        margin = math.inf
    return top.astype(np.int64), d[top], margin


# --------------------------------------------------------------------------------------
# Quantization estimate (BSA-O)  [Sec. V-B "Approximate Distances": the asymmetric distance
# from the query to the point's OPQ codewords is dis', the point's distance to its own
# reconstruction is one more classifier feature; Sec. VI-B (M subspaces of 2^nbits
# codewords, O(D 2^nbits) lookup-table build); Sec. VII-A (M = D/4, D/8 for GIST; nbits = 8;
# OPQ trained on 65,536 sampled points)]
# --------------------------------------------------------------------------------------

def opq_allocation(lam: np.ndarray, M: int) -> np.ndarray:
    """OPQ's parametric solution (eigenvalue allocation, Ge et al.): the PCA axes, largest
    eigenvalue first, are dealt to M subspaces of D/M axes each, every axis to the subspace
    whose product of eigenvalues so far is smallest among those not full (lowest index on
    ties), which balances the subspaces' variance products.  The OPQ rotation is then the PCA
    rotation with its rows permuted.  Reading: the eigenvalues are first divided by their
    geometric mean (eigenvalues below 1e-12 of the largest count as 1e-12 of it), so an empty
    subspace's product 1 sits in the middle of the spectrum and the rule does not depend on
    the data's scale (with raw eigenvalues all below 1 it would fill one subspace at a time).
    Returns perm (M, D/M): the axes of subspace j, ascending."""
    lam = np.asarray(lam, dtype=np.float64)
    D = lam.shape[0]
    if M < 1 or D % M:
        raise ValueError("M must divide D")
    dsub = D // M
    ll = np.log(np.maximum(lam, lam.max() * 1e-12 if lam.max() > 0 else 1e-300))
    ll = ll - ll.mean()
    logp = np.zeros(M)
    members = [[] for _ in range(M)]
    for i in np.argsort(-lam, kind="stable"):
        best = -1
        for j in range(M):
            if len(members[j]) < dsub and (best < 0 or logp[j] < logp[best]):
                best = j
        members[best].append(int(i))
        logp[best] += ll[i]
    return np.array([sorted(m) for m in members], dtype=np.int64)


def pq_train(Y: np.ndarray, perm: np.ndarray, ksub: int = 256, iters: int = 25, seed: int = 0,
             train: int = 65536) -> np.ndarray:
    """Codebooks: ``kmeans`` with ksub centroids in every subspace over the same <= ``train``
    stored rows (the smallest SplitMix64 keys); centroids rounded to FP32, as stored.
    Returns books (M, ksub, dsub), FP64 holding FP32 values."""
    n = Y.shape[0]
    rows = select_by_key(n, min(n, train), seed, TAG_PQ_SAMPLE)
    T = np.asarray(Y, dtype=np.float64)[rows]
    if T.shape[0] < ksub:
        raise ValueError("fewer training rows than codewords")
    books = []
    for j in range(perm.shape[0]):
        C, _ = kmeans(T[:, perm[j]], ksub, iters, seed, train_per_list=max(1, -(-T.shape[0] // ksub)))
        books.append(C.astype(np.float32).astype(np.float64))
    return np.stack(books)


def pq_encode(Y: np.ndarray, perm: np.ndarray, books: np.ndarray) -> np.ndarray:
    """codes[x, j] = argmin_c ||y_j - C_j[c]||^2 (lowest c on ties).  The argmin decides an
    integer, so it is taken in FP32 as the GPU takes it: differences rounded to FP32,
    squared and rounded, added in subspace-axis order, each operation rounded separately."""
    Y32 = np.asarray(Y, dtype=np.float32)
    M, ksub, dsub = books.shape
    B32 = books.astype(np.float32)
    codes = np.empty((Y32.shape[0], M), dtype=np.uint8)
    for j in range(M):
        acc = np.zeros((Y32.shape[0], ksub), dtype=np.float32)
        for t in range(dsub):
            dlt = Y32[:, perm[j, t]][:, None] - B32[j, :, t][None, :]
            acc = acc + dlt * dlt
        codes[:, j] = np.argmin(acc, axis=1)
    return codes


def pq_error(Y: np.ndarray, perm: np.ndarray, books: np.ndarray, codes: np.ndarray) -> np.ndarray:
    """||u - c(u)||^2: squared distance of every stored row to its own codewords (FP64)."""
    Y = np.asarray(Y, dtype=np.float64)
    out = np.zeros(Y.shape[0])
    for j in range(perm.shape[0]):
        out += np.sum((Y[:, perm[j]] - books[j][codes[:, j]]) ** 2, axis=1)
    return out


def pq_lut(qrot: np.ndarray, perm: np.ndarray, books: np.ndarray) -> np.ndarray:
    """lut[j, c] = ||q'_j - C_j[c]||^2 for one rotated query (FP64)."""
    q = np.asarray(qrot, dtype=np.float64)
    return np.stack([np.sum((q[perm[j]][None, :] - books[j]) ** 2, axis=1)
                     for j in range(perm.shape[0])])


def pq_adc(lut: np.ndarray, codes: np.ndarray) -> np.ndarray:
    """Asymmetric distance dis' = sum_j lut[j, codes[x, j]] for the given code rows."""
    return lut[np.arange(lut.shape[0])[None, :], codes.astype(np.int64)].sum(axis=1)


# --------------------------------------------------------------------------------------
# Stages  [Sec. IV-D Alg. 2: dimensions are added Delta_d at a time; Sec. V-B
# "Incremental Correction": one classifier per stage until d = D]
# --------------------------------------------------------------------------------------

def stage_bounds(D: int, delta_d: int = 32) -> np.ndarray:
    """d_s = min(s * Delta_d, D) for s = 1..S, S = ceil(D / Delta_d).  Stages 1..S-1 are
    tested; at stage S all D dimensions are summed, so the value is the exact distance."""
    S = -(-D // delta_d)
    return np.minimum(np.arange(1, S + 1) * delta_d, D).astype(np.int64)


def partial_dists(Yc: np.ndarray, qrot: np.ndarray, bounds: np.ndarray) -> np.ndarray:
    """e_s = sum_{i < d_s} (q'_i - y_i)^2 for every row and stage (FP64): the PCA
    partial distance dis' over the first d_s projected dimensions [Sec. V-B]."""
    diff = np.asarray(Yc, dtype=np.float64) - qrot[None, :]
    sq = diff * diff
    cs = np.cumsum(sq, axis=1)
    return cs[:, bounds - 1]


def bsar_terms(qrot: np.ndarray, lam: np.ndarray, bounds: np.ndarray):
    """Per test stage s (residual dims i >= d_s): ||q'_r||^2 and sigma_s = the standard
    deviation of the omitted cross term -2 <q'_r, x_r>, sqrt(4 sum_i q'_i^2 lam_i), when x is
    distributed with variance lam_i along rotated axis i [Eq. (2); the sigma of Alg. 1]."""
    q = np.asarray(qrot, dtype=np.float64)
    qr = np.array([np.sum(q[d:] ** 2) for d in bounds[:-1]])
    sig = np.array([math.sqrt(4.0 * np.sum(q[d:] ** 2 * lam[d:])) for d in bounds[:-1]])
    return qr, sig


def residual_norms(Yc: np.ndarray, bounds: np.ndarray) -> np.ndarray:
    """||x_r||^2 = sum over the residual dims i >= d_s of x_i^2, per row and test stage."""
    Yc = np.asarray(Yc, dtype=np.float64)
    return np.column_stack([np.sum(Yc[:, d:] ** 2, axis=1) for d in bounds[:-1]]) \
        if bounds.shape[0] > 1 else np.zeros((Yc.shape[0], 0))


def _rel(a, b, c):
    return np.abs(a) + np.abs(b) + np.abs(c) + 1e-300


def search_one(qrot, Y, list_off, list_ids, probes, k, m, beta, bounds, B=256, L=0,
               prune=True, collect_neg=None, pre=None, res=None, pq=None, log=None, flip=(),
               near_tol=1e-4):
    """Canonical block-synchronous pruned refinement for one rotated query.

    The paper's refinement updates tau after every candidate [Sec. I: result queue Q with
    threshold tau].  Reading for parallel hardware: candidates are taken in probe order,
    each list in blocks of B consecutive stored positions (blocks never span lists); every
    candidate of block b is tested against tau_b = the tau in force after block b-1-L
    (+inf if there is none or the queue held fewer than K).  B = 1, L = 0 is the paper's
    sequential rule.  A candidate is pruned at the first tested stage s with
    tau_b < inf and m_s * e_s + beta_s > tau_b (strict, Sec. V-A classifier), otherwise its
    exact distance e_S joins the block's survivors; after the block the queue becomes the
    K smallest (dis, id) of queue and survivors, and tau its K-th distance.

    Returns (ids, dists, stop_counts, margin):
      stop_counts[s] = candidates whose last scanned stage is s (0-based, S-1 = refined);
      margin = smallest relative distance of any decision quantity to its threshold.
    If ``collect_neg`` is a list, (id, tau_b, e_1..e_S) of every candidate with tau_b
    finite and dis > tau_b is appended to it (label-1 pool of the calibration).
    ``pre`` = (dec, m0, beta0) adds the FP8 pre-stage: before stage 1 every tested
    candidate's e_0 = sum over the coded lead dims of (q'_i - dec_i)^2 is tested with
    m0 e_0 + beta0 > tau_b; survivors restart at dim 0 on the stored values.  Then
    stop_counts has S + 1 entries, entry 0 counting the candidates the pre-stage pruned.
    ``res`` = (qr, msig) replaces the stage test by the residual-estimate test of Alg. 2
    (incremental): dis'_s = e_s + ||x_r||^2 + ||q'_r||^2 (equal to C1 - C2 of Alg. 1, the
    exact distance without the cross term of the residual dims), pruned iff
    dis'_s - m sigma_s > tau_b, with qr = ||q'_r||^2 and msig = m sigma_s per test stage.
    ``pq`` = (lut, codes, err, m1, m3, beta) adds the quantization test of BSA-O before the
    stages: every tested candidate with m1 dis' + m3 err + beta > tau_b is pruned (dis' =
    ``pq_adc``, err = its ``pq_error``), entry 0 of stop_counts counting them; survivors are
    refined over all dims (with m = 1, beta = -inf no stage test fires: the paper's BSA-O is
    one classifier, not incremental).

    Near-threshold log (parity with other rounding): if ``log`` is a dict it receives
      'stage': ids with an evaluated test whose decision quantity lies within ``near_tol``
               (relative) of tau_b,
      'near':  those ids plus every id whose distance lies within ``near_tol`` of the K-th
               distance of a merge that cut the queue, or of a neighbour in the final order.
    ``flip`` (ids): for each listed candidate the outcome of its first evaluated test within
    ``near_tol`` of its threshold is inverted (a pass becomes a prune and the other way
    round); its walk through the later tests continues as usual.  This replays the search
    as hardware whose rounding took that one decision the other way.
    """
    S = bounds.shape[0]
    T_d = np.zeros(0)
    T_i = np.zeros(0, dtype=np.int64)
    tau_hist = []
    P = 1 if (pre is not None or pq is not None) else 0
    stop_counts = np.zeros(S + P, dtype=np.int64)
    margin = math.inf
    flip = set(int(x) for x in flip)
    near_stage, near_all = set(), set()
    b = 0
    for lst in probes:
        lo, hi = int(list_off[lst]), int(list_off[lst + 1])
        for s0 in range(lo, hi, B):
            ids = list_ids[s0:min(s0 + B, hi)]
            j = b - 1 - L
            tau_b = tau_hist[j] if j >= 0 else math.inf
            e = partial_dists(Y[ids], qrot, bounds)          # (nb, S)
            # every test this block can take, in test order: (prune outcome, relative margin)
            hits, rels = [], []
            if prune and pre is not None and math.isfinite(tau_b):
                dec, m0, beta0 = pre
                lead = dec.shape[1]
                e0 = partial_dists(dec[ids], qrot[:lead], np.array([lead]))[:, 0]
                lhs0 = m0 * e0 + beta0
                hits.append(lhs0 > tau_b)
                rels.append(np.abs(lhs0 - tau_b) / _rel(m0 * e0, np.full_like(e0, beta0), tau_b))
            if prune and pq is not None and math.isfinite(tau_b):
                lut, codes, err, m1, m3, beta0 = pq
                adc = pq_adc(lut, codes[ids])
                lhs0 = m1 * adc + m3 * err[ids] + beta0
                hits.append(lhs0 > tau_b)
                rels.append(np.abs(lhs0 - tau_b) / (np.abs(m1 * adc) + np.abs(m3 * err[ids]) + abs(beta0)
                                                    + abs(tau_b) + 1e-300))
            P_b = len(hits)                                  # 1 if the pre-test ran on this block
            if prune and math.isfinite(tau_b) and S > 1 and (res is not None or np.isfinite(beta).any()):
                if res is None:
                    lhs = e[:, :S - 1] * m[None, :] + beta[None, :]   # (nb, S-1)
                    scale = _rel(e[:, :S - 1] * m[None, :], beta[None, :], tau_b)
                else:
                    qr, msig = res
                    xr = residual_norms(Y[ids], bounds)
                    lhs = e[:, :S - 1] + xr + qr[None, :] - msig[None, :]
                    scale = np.abs(e[:, :S - 1]) + xr + qr[None, :] + msig[None, :] + abs(tau_b)
                for st in range(S - 1):
                    hits.append(lhs[:, st] > tau_b)
                    with np.errstate(invalid="ignore"):
                        rels.append(np.abs(lhs[:, st] - tau_b) / scale[:, st])
            nt = len(hits)
            if nt:
                H = np.column_stack(hits)
                Rl = np.nan_to_num(np.column_stack(rels), nan=math.inf)
                first = np.where(H.any(axis=1), H.argmax(axis=1), nt)   # nt: no test prunes
                for r in range(ids.shape[0]):
                    if int(ids[r]) in flip:
                        first[r] = nt
                        flipped = False
                        for t in range(nt):
                            h = bool(H[r, t])
                            if not flipped and Rl[r, t] < near_tol:
                                h, flipped = not h, True
                            if h:
                                first[r] = t
                                break
                evaluated = np.arange(nt)[None, :] <= first[:, None]
                if evaluated.any():
                    margin = min(margin, float(Rl[evaluated].min()))
                close = (evaluated & (Rl < near_tol)).any(axis=1)
                for x in ids[close]:
                    near_stage.add(int(x))
            else:
                first = np.zeros(ids.shape[0], dtype=np.int64)
            pre_hit = (first == 0) if P_b else np.zeros(ids.shape[0], dtype=bool)
            stop = np.where(first >= nt, S - 1, first - P_b) if nt else np.full(ids.shape[0], S - 1)
            np.add.at(stop_counts, stop[~pre_hit] + P, 1)
            if P:
                stop_counts[0] += int(pre_hit.sum())
            surv = (stop == S - 1) & ~pre_hit
            sd = e[surv, S - 1]
            si = ids[surv]
            if collect_neg is not None and math.isfinite(tau_b):
                neg = sd > tau_b
                es = e[surv]
                for r in np.nonzero(neg)[0]:
                    collect_neg.append((int(si[r]), tau_b, es[r]))
            # merge: K smallest of queue and survivors by (dis, id)
            all_d = np.concatenate([T_d, sd])
            all_i = np.concatenate([T_i, si])
            order = np.lexsort((all_i, all_d))
            if order.shape[0] > k:
                dk, dk1 = all_d[order[k - 1]], all_d[order[k]]
                margin = min(margin, float(abs(dk1 - dk) / max(abs(dk1), 1e-300)))
                close = np.abs(all_d - dk) <= near_tol * max(abs(dk), 1e-300)
                if close.sum() > 1:
                    near_all.update(int(x) for x in all_i[close])
            order = order[:k]
            T_d, T_i = all_d[order], all_i[order]
            tau_hist.append(float(T_d[k - 1]) if T_d.shape[0] == k else math.inf)
            b += 1
    if T_d.shape[0] > 1:
        gaps = np.abs(np.diff(T_d)) / np.maximum(np.abs(T_d[1:]), 1e-300)
        margin = min(margin, float(gaps.min()))
        for i in np.nonzero(gaps < near_tol)[0]:
            near_all.update((int(T_i[i]), int(T_i[i + 1])))
    if log is not None:
        log["stage"] = sorted(near_stage)
        log["near"] = near_all | near_stage
    ids_out = np.full(k, -1, dtype=np.int64)
    d_out = np.full(k, np.inf)
    ids_out[:T_i.shape[0]] = T_i
    d_out[:T_d.shape[0]] = T_d
    return ids_out, d_out, stop_counts, margin


def search_sequential(qrot, Y, list_off, list_ids, probes, k, m, beta, bounds, pre=None, res=None,
                      pq=None):
    """The paper's per-candidate refinement, coded separately: a binary max-heap Q of the
    K best (dis, id); tau = its root once it holds K entries; each candidate walks the
    stages and is pruned at the first stage with m_s e_s + beta_s > tau, otherwise enters
    Q when (dis, id) is smaller than the root [Sec. I refinement; Alg. 2 stage loop;
    Sec. V-A classifier].  Equals ``search_one`` with B = 1, L = 0 (``pre``, ``pq`` as
    there; the quantization estimate is summed codeword by codeword here)."""
    heap = []   # entries (-dis, -id): the root is the largest (dis, id)
    q = np.asarray(qrot, dtype=np.float64)
    S = bounds.shape[0]
    for lst in probes:
        for pos in range(int(list_off[lst]), int(list_off[lst + 1])):
            x = int(list_ids[pos])
            tau = -heap[0][0] if len(heap) == k else math.inf
            if pre is not None and tau != math.inf:
                dec, m0, beta0 = pre
                e0 = 0.0
                for i in range(dec.shape[1]):
                    t = q[i] - dec[x, i]
                    e0 += t * t
                if m0 * e0 + beta0 > tau:
                    continue
            if pq is not None and tau != math.inf:
                lut, codes, err, m1, m3, beta0 = pq
                adc = 0.0
                for j in range(lut.shape[0]):
                    adc += lut[j, int(codes[x, j])]
                if m1 * adc + m3 * err[x] + beta0 > tau:
                    continue
            acc = 0.0
            lo = 0
            pruned = False
            for s in range(S):
                hi = int(bounds[s])
                for i in range(lo, hi):
                    t = q[i] - Y[x, i]
                    acc += t * t
                lo = hi
                if s < S - 1 and tau != math.inf:
                    if res is None:
                        test = m[s] * acc + beta[s] > tau
                    else:       # C1 - C2 - m sigma > tau, C1 - C2 = acc + ||x_r||^2 + ||q_r||^2
                        xr = 0.0
                        for i in range(hi, Y.shape[1]):
                            xr += Y[x, i] * Y[x, i]
                        test = acc + xr + res[0][s] - res[1][s] > tau
                    if test:
                        pruned = True
                        break
            if pruned:
                continue
            item = (-acc, -x)
            if len(heap) < k:
                heapq.heappush(heap, item)
            elif (acc, x) < (-heap[0][0], -heap[0][1]):
                heapq.heapreplace(heap, item)
    res = sorted((-a, -b) for a, b in heap)
    ids = np.full(k, -1, dtype=np.int64)
    ds = np.full(k, np.inf)
    for i, (d, x) in enumerate(res):
        ids[i], ds[i] = x, d
    return ids, ds


# --------------------------------------------------------------------------------------
# Logistic regression  [Sec. V-A "Parameter Learning": linear classifier on (dis', tau),
# cross-entropy loss].  Reading: the paper trains with SGD and reports that other linear
# models give similar outcomes; the oracle takes the exact minimiser of the same
# cross-entropy (plus a 1e-8 ridge) by Newton's method (IRLS).
# --------------------------------------------------------------------------------------

def irls_logistic(F: np.ndarray, y: np.ndarray, ridge: float = 1e-8, max_iter: int = 100,
                  tol: float = 1e-12):
    """Minimise mean BCE(sigmoid(w0 + w.f), y) + ridge/2 * |w|^2 (w without intercept) on
    standardised features; returns (b, w) in the original feature units."""
    F = np.asarray(F, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    mean = F.mean(axis=0)
    std = F.std(axis=0)
    std[std == 0] = 1.0
    Z = np.hstack([np.ones((F.shape[0], 1)), (F - mean) / std])
    n, p = Z.shape
    w = np.zeros(p)
    reg = np.full(p, ridge)
    reg[0] = 0.0
    for _ in range(max_iter):
        t = Z @ w
        pr = 0.5 * (1.0 + np.tanh(0.5 * t))          # sigmoid, overflow-free
        g = Z.T @ (pr - y) / n + reg * w
        W = pr * (1.0 - pr)
        H = (Z * W[:, None]).T @ Z / n + np.diag(reg) + 1e-300 * np.eye(p)
        step = np.linalg.solve(H, g)
        w = w - step
        if np.max(np.abs(step)) < tol:
            break
    wf = w[1:] / std
    b = w[0] - float(np.dot(w[1:], mean / std))
    return b, wf


def classifier_to_correction(b: float, w1: float, w2: float):
    """sign(w1 dis' + w2 tau + b) > 0  <=>  m dis' + beta > tau  with m = -w1/w2,
    beta = -b/w2 when w2 < 0 [Sec. V-A, linear model].  Reading: if w2 >= 0 or m <= 0 the
    classifier has no usable orientation and m falls back to 1."""
    if w2 < 0:
        m = -w1 / w2
        if m > 0:
            return m, -b / w2
    return 1.0, 0.0


def classifier3_to_correction(b: float, w1: float, w3: float, w2: float):
    """The BSA-O classifier sign(w1 dis' + w3 err + w2 tau + b) > 0 as the test
    m1 dis' + m3 err + beta > tau: m1 = -w1/w2, m3 = -w3/w2, beta = -b/w2 when w2 < 0
    [Sec. V-A linear model with the extra feature of Sec. V-B].  Same fallback as
    ``classifier_to_correction``: m1 = 1, m3 = 0 without a usable orientation."""
    if w2 < 0:
        m1 = -w1 / w2
        if m1 > 0:
            return m1, -w3 / w2, -b / w2
    return 1.0, 0.0, 0.0


# --------------------------------------------------------------------------------------
# Target-recall adjustment  [Sec. V-A "Adaptive Adjustment": move beta to beta' so that the
# recall of label 0 reaches r].  Reading: alpha = 1 - r is the probability that a true
# neighbour is pruned at ANY stage (joint), so beta_s = the (k*+1)-th smallest residual
# g_s = tau - m_s e_s of stage s, with k* the largest k whose joint false-prune fraction
# F(k) = (1/n0) #{ j : exists s, g_s(j) < g_s^(k+1) } is <= alpha.  The binary search the
# paper mentions is exact here because F is monotone in k.  Per-stage (Bonferroni) mode
# gives every test stage alpha / S_t instead.
# --------------------------------------------------------------------------------------

def joint_false_prune(G: np.ndarray, Gs: np.ndarray, k: int) -> float:
    """F(k) for residual matrix G (n0, S_t) and its column-sorted copy Gs."""
    thr = Gs[k, :]
    return float(np.mean((G < thr[None, :]).any(axis=1)))


def beta_for_alpha(G: np.ndarray, alpha: float, mode: str = "joint") -> np.ndarray:
    G = np.asarray(G, dtype=np.float64)
    n0, St = G.shape
    if alpha <= 0.0 or n0 == 0:
        return np.full(St, -np.inf)
    Gs = np.sort(G, axis=0)
    if mode == "bonferroni":
        k = min(int(math.floor(alpha * n0 / St)), n0 - 1)
        return Gs[k, :].copy()
    lo, hi = 0, n0 - 1                    # F(0) = 0 <= alpha always
    while lo < hi:
        mid = (lo + hi + 1) // 2
        if joint_false_prune(G, Gs, mid) <= alpha:
            lo = mid
        else:
            hi = mid - 1
    return Gs[lo, :].copy()


# --------------------------------------------------------------------------------------
# Calibration  [Sec. V-A; Sec. VII-A implementation details: training queries, their KNN as
# label 0, items met "through a query process" as label 1, BCE training, target recall]
# --------------------------------------------------------------------------------------

def calibrate(Y, list_off, list_ids, centroids, mu, R, calib, bounds, calib_k=10, calib_nprobe=8,
              B=256, L=0, seed=0, max_neg=50, pre_dec=None):
    """Per test stage: m_s from logistic regression on label 0 = (e_s, tau_q) of the K_c
    true neighbours of every calibration query (tau_q = its K_c-th distance) and label 1 =
    up to ``max_neg`` (e_s, tau_b) per query drawn (smallest SplitMix64 keys of
    query_index * 2^32 + id) from the candidates of an unpruned canonical IVF search
    (calib_nprobe, B, L) whose exact distance exceeds the block's finite tau_b.
    Returns dict(m, G) with G the (n0, S_t) residual matrix g_s(j) = tau_j - m_s e_s(j).
    With ``pre_dec`` (decoded FP8 lead dims, rows by id) the pre-stage is one more test
    stage, first in m and G, whose feature e_0 is taken over the decoded values."""
    Y = np.asarray(Y, dtype=np.float64)
    S = bounds.shape[0]
    P = 1 if pre_dec is not None else 0
    St = S - 1
    Qr = rotate(calib, mu, R)
    knn_ids, knn_d = bruteforce_knn(Y, Qr, calib_k)
    pos_e, pos_tau, neg_e, neg_tau, neg_q, neg_id = [], [], [], [], [], []
    zeros_m = np.zeros(St)
    for qi in range(Qr.shape[0]):
        tau_q = knn_d[qi, calib_k - 1]
        e = partial_dists(Y[knn_ids[qi]], Qr[qi], bounds)
        if pre_dec is not None:
            lead = pre_dec.shape[1]
            e0 = partial_dists(pre_dec[knn_ids[qi]], Qr[qi][:lead], np.array([lead]))
            e = np.hstack([e0, e])
        pos_e.append(e[:, :St + P])
        pos_tau.append(np.full(calib_k, tau_q))
        probes, _, _ = probe_order(Qr[qi], centroids, calib_nprobe)
        pool = []
        search_one(Qr[qi], Y, list_off, list_ids, probes, calib_k, zeros_m, zeros_m, bounds,
                   B=B, L=L, prune=False, collect_neg=pool)
        if pool:
            idx = np.array([p[0] for p in pool], dtype=np.uint64)
            keys = ctr_key(seed, TAG_NEG, (np.uint64(qi) << np.uint64(32)) + idx)
            take = np.lexsort((idx, keys))[:max_neg]
            for t in take:
                en = pool[t][2][:St]
                if pre_dec is not None:
                    lead = pre_dec.shape[1]
                    e0 = partial_dists(pre_dec[[pool[t][0]]], Qr[qi][:lead], np.array([lead]))[0]
                    en = np.concatenate([e0, en])
                neg_e.append(en)
                neg_tau.append(pool[t][1])
                neg_q.append(qi)
                neg_id.append(pool[t][0])
    pos_e = np.vstack(pos_e)
    pos_tau = np.concatenate(pos_tau)
    neg_e = np.vstack(neg_e) if neg_e else np.zeros((0, St + P))
    neg_tau = np.asarray(neg_tau, dtype=np.float64)
    m = np.ones(St + P)
    lr = []
    for s in range(St + P):
        F = np.vstack([np.column_stack([pos_e[:, s], pos_tau]), np.column_stack([neg_e[:, s], neg_tau])])
        lab = np.concatenate([np.zeros(pos_e.shape[0]), np.ones(neg_e.shape[0])])
        if neg_e.shape[0] == 0:
            lr.append((0.0, 0.0, 0.0))
            continue
        b, w = irls_logistic(F, lab)
        m[s], _ = classifier_to_correction(b, w[0], w[1])
        lr.append((b, w[0], w[1]))
    G = pos_tau[:, None] - pos_e * m[None, :]
    return dict(m=m, G=G, pos_e=pos_e, pos_tau=pos_tau, neg_e=neg_e, neg_tau=neg_tau, lr=lr,
                knn_ids=knn_ids, knn_d=knn_d, neg_q=np.asarray(neg_q, dtype=np.int64),
                neg_id=np.asarray(neg_id, dtype=np.int64), qrot=Qr)


def calibrate_pq(cal: dict, pq: dict) -> dict:
    """The BSA-O classifier on the calibration pairs ``calibrate`` collected (label 0 = the
    K_c nearest stored vectors with tau = the K_c-th distance, label 1 = the sampled pairs of
    the unpruned query process with their tau_b): features (dis' = ADC, err = the point's
    quantization error, tau) [Sec. V-B], logistic regression by ``irls_logistic``, then the
    residuals g(j) = tau_j - m1 dis'_j - m3 err_j of label 0 for the target-recall shift
    (``beta_for_alpha`` on the one test).  Returns dict(m1, m3, G (n0, 1), lr)."""
    Qr, perm, books, codes, err = cal["qrot"], pq["perm"], pq["books"], pq["codes"], pq["err"]
    luts = [pq_lut(q, perm, books) for q in Qr]
    kc = cal["knn_ids"].shape[1]
    pos_adc = np.concatenate([pq_adc(luts[qi], codes[cal["knn_ids"][qi]]) for qi in range(Qr.shape[0])])
    pos_err = err[cal["knn_ids"].reshape(-1)]
    pos_tau = cal["pos_tau"]
    assert pos_adc.shape[0] == pos_tau.shape[0] == Qr.shape[0] * kc
    neg_adc = np.array([pq_adc(luts[q], codes[[x]])[0] for q, x in zip(cal["neg_q"], cal["neg_id"])])
    neg_err = err[cal["neg_id"]] if cal["neg_id"].size else np.zeros(0)
    if neg_adc.size == 0:
        m1, m3, lr = 1.0, 0.0, (0.0, np.zeros(3))
    else:
        F = np.vstack([np.column_stack([pos_adc, pos_err, pos_tau]),
                       np.column_stack([neg_adc, neg_err, cal["neg_tau"]])])
        lab = np.concatenate([np.zeros(pos_adc.shape[0]), np.ones(neg_adc.shape[0])])
        b, w = irls_logistic(F, lab)
        m1, m3, _ = classifier3_to_correction(b, w[0], w[1], w[2])
        lr = (b, w)
    G = (pos_tau - m1 * pos_adc - m3 * pos_err)[:, None]
    return dict(m1=m1, m3=m3, G=G, lr=lr, pos_adc=pos_adc, pos_err=pos_err, neg_adc=neg_adc,
                neg_err=neg_err)


# --------------------------------------------------------------------------------------
# End-to-end fit and search
# --------------------------------------------------------------------------------------

def ads_table(bounds: np.ndarray, D: int, eps0: float = 2.1):
    """The random-projection test of ADSampling (Sec. III "Distance Correction") in this
    code's test form.  With a random rotation, dis' = (D / d) e_d estimates dis; the test
    dis' > (1 + eps)^2 tau (squared distances) with eps = eps0 / sqrt(d) (reading: the
    failure bound 2 exp(-c0 d eps^2) of its lemma held at the level 2 exp(-c0 eps0^2)) is
    m_s e_s + beta_s > tau with m_s = (D / d_s) / (1 + eps0 / sqrt(d_s))^2, beta_s = 0."""
    d = np.asarray(bounds[:-1], dtype=np.float64)
    m = (D / d) / (1.0 + eps0 / np.sqrt(d)) ** 2
    return m, np.zeros_like(m)


def fit(base, calib, nlist, delta_d=32, storage="f32", kmeans_iters=25, calib_k=10,
        calib_nprobe=None, B=256, L=0, seed=0, pca_sample=1_000_000, max_neg=50, fp8_lead=0,
        calib_k_extra=(), projection="pca", pq_m=0, pq_iters=25, pq_train_rows=65536):
    """Projection + IVF lists + calibrated correction table for ``base``; ``fp8_lead`` = 64
    adds the FP8 pre-stage over the leading 64 rotated dims.  ``calib_k_extra`` adds one
    table per further K_c (see ``table_for_k``).  ``projection`` = "haar" replaces the PCA
    rotation by ``haar_rotation(D, seed)`` (centring and everything after it unchanged).
    ``pq_m`` > 0 adds the BSA-O quantization estimate: OPQ (``opq_allocation`` of the PCA
    axes into pq_m subspaces, 256 codewords each, ``pq_train`` on pq_train_rows rows) and one
    BSA-O classifier per table (``calibrate_pq``)."""
    base = np.asarray(base)
    D = base.shape[1]
    pca = pca_fit(base, pca_sample, seed)
    if projection == "haar":
        Rh = haar_rotation(D, seed)
        pca = dict(mu=pca["mu"], cov=pca["cov"], R=Rh,
                   lam=np.einsum("ij,jk,ik->i", Rh, pca["cov"], Rh))   # variance along each axis
    elif projection != "pca":
        raise ValueError(projection)
    Y = round_storage(rotate(base, pca["mu"], pca["R"]), storage)
    C, assign = kmeans(Y, nlist, kmeans_iters, seed)
    off, ids = build_lists(assign, nlist)
    bounds = stage_bounds(D, delta_d)
    if calib_nprobe is None:
        calib_nprobe = int(min(max(1, nlist // 8), 64))
    pre = fp8_encode_lead(Y, off, ids, fp8_lead) if fp8_lead else None
    pq = None
    if pq_m:
        if projection != "pca":
            raise ValueError("the OPQ allocation needs the PCA rotation")
        perm = opq_allocation(pca["lam"], pq_m)
        books = pq_train(Y, perm, 256, pq_iters, seed, pq_train_rows)
        codes = pq_encode(Y, perm, books)
        pq = dict(m=pq_m, perm=perm, books=books, codes=codes, err=pq_error(Y, perm, books, codes))
    tables = []
    for kc in [calib_k, *calib_k_extra]:
        cal = calibrate(Y, off, ids, C, pca["mu"], pca["R"], calib, bounds, kc, calib_nprobe,
                        B, L, seed, max_neg, pre_dec=pre["dec"] if pre else None)
        tables.append(dict(kc=kc, m=cal["m"], G=cal["G"], calib=cal,
                           pq=calibrate_pq(cal, pq) if pq else None))
    cal = tables[0]["calib"]
    return dict(mu=pca["mu"], R=pca["R"], lam=pca["lam"], cov=pca["cov"], Y=Y, centroids=C,
                assign=assign, list_off=off, list_ids=ids, bounds=bounds, m=cal["m"], G=cal["G"],
                calib=cal, storage=storage, delta_d=delta_d, B=B, L=L, pre=pre,
                tables=tables if len(tables) > 1 else None, pq=pq, pq_tab=tables[0]["pq"])


def pq_table_for_k(index, k):
    """The BSA-O classifier (m1, m3, G) a search with K uses (same K_c rule as ``table_for_k``)."""
    tabs = index.get("tables")
    if not tabs:
        t = index["pq_tab"]
    else:
        best = tabs[0]
        for c in tabs:
            if c["kc"] <= k and c["kc"] >= best["kc"]:
                best = c
        t = best["pq"]
    return t["m1"], t["m3"], t["G"]


def table_for_k(index, k):
    """(m, G) of the correction table a search with K uses.  Reading: the paper trains with
    the K nearest neighbours as label 0 and its threshold tau is the K-th distance; an index
    calibrated at several K_c applies the table of the largest K_c <= K (the smallest K_c's
    table when K is below all of them), so the label-0 semantics match the search's K."""
    tabs = index.get("tables")
    if not tabs:
        return index["m"], index["G"]
    best = tabs[0]
    for t in tabs:
        if t["kc"] <= k and t["kc"] >= best["kc"]:
            best = t
    return best["m"], best["G"]


def search(index, queries, k, nprobe, alpha, mode="learned", B=None, L=None, calib_mode="joint",
           flip=None, probe_swap=None, near_tol=1e-4):
    """Search every query; mode in {'learned', 'lossless', 'none', 'ads', 'bsar', 'bsao'}
    ('ads': the ADSampling test of ``ads_table`` with index["ads_eps0"], default 2.1; 'bsar':
    the residual-estimate test with multiplier index["bsar_m"], default 8, or Phi^-1(1 - alpha)
    when that is <= 0; 'bsao': the OPQ estimate with its learned classifier, index fitted
    with pq_m > 0).  The queries are rotated as index["rotation"] says ('f32' default,
    'bf16': ``rotate_bf16``).
    Returns ids (nq, k), dists (nq, k), stop_counts (nq, S), margin (nq,), and per query the
    near-threshold log of ``search_one`` ('near', 'stage_near') plus 'probe_near': the
    positions i < nprobe whose ranked centroid distances i and i + 1 lie within ``near_tol``
    (relative) of each other.
    Replays under other rounding: ``flip`` = {query: ids} passes those ids to ``search_one``;
    ``probe_swap`` = {query: i} exchanges the lists ranked i and i + 1 (i + 1 = nprobe brings
    in the next list in place of the last probed one)."""
    B = index["B"] if B is None else B
    L = index["L"] if L is None else L
    bounds = index["bounds"]
    St = bounds.shape[0] - 1
    pre_ix = index.get("pre")
    pre = None
    if mode == "learned":
        m, G = table_for_k(index, k)
        beta = beta_for_alpha(G, alpha, calib_mode)
        prune = alpha > 0
        if pre_ix is not None:     # the pre-stage is the first test stage of the table
            pre = (pre_ix["dec"], float(m[0]), float(beta[0]))
            m, beta = m[1:], beta[1:]
    elif mode == "lossless":
        # the FP8 estimate is not a lower bound of the stored-value distance: no pre-stage
        m, beta, prune = np.ones(St), np.zeros(St), True
    elif mode == "ads":
        m, beta = ads_table(bounds, index["Y"].shape[1], index.get("ads_eps0", 2.1))
        prune = True
    elif mode == "bsar":
        m, beta, prune = np.ones(St), np.zeros(St), True
        mult = bsar_multiplier(alpha, index.get("bsar_m", 8.0))
    elif mode == "none":
        m, beta, prune = np.ones(St), np.zeros(St), False
    elif mode == "bsao":
        # one quantization test, then survivors refined over all dims (no stage test)
        m1, m3, Gq = pq_table_for_k(index, k)
        beta_q = float(beta_for_alpha(Gq, alpha, calib_mode)[0])
        m, beta, prune = np.ones(St), np.full(St, -np.inf), alpha > 0
    else:
        raise ValueError(mode)
    Qr = rotate_as(queries, index["mu"], index["R"], index.get("rotation", "f32"))
    nq = Qr.shape[0]
    ids = np.full((nq, k), -1, dtype=np.int64)
    ds = np.full((nq, k), np.inf)
    stops = np.zeros((nq, bounds.shape[0] + (1 if (pre is not None or mode == "bsao") and prune else 0)),
                     dtype=np.int64)
    margins = np.full(nq, math.inf)
    probes_all = np.zeros((nq, nprobe), dtype=np.int64)
    near, stage_near, probe_near = [], [], []
    nl = index["centroids"].shape[0]
    for qi in range(nq):
        ranked, rd, pm = probe_order(Qr[qi], index["centroids"], min(nprobe + 1, nl))
        gaps = np.abs(np.diff(rd)) / np.maximum(np.abs(rd[1:]), 1e-300)
        probe_near.append([int(i) for i in np.nonzero(gaps < near_tol)[0] if i < nprobe])
        probes = ranked[:nprobe].copy()
        pm = float(gaps.min()) if gaps.size else math.inf
        if probe_swap and qi in probe_swap:
            i = probe_swap[qi]
            if i + 1 < nprobe:
                probes[i], probes[i + 1] = probes[i + 1], probes[i]
            elif i + 1 == nprobe and ranked.shape[0] > nprobe:
                probes[i] = ranked[nprobe]
        probes_all[qi] = probes
        res = None
        if mode == "bsar":
            qr, sig = bsar_terms(Qr[qi], index["lam"], bounds)
            res = (qr, mult * sig)
        pqa = None
        if mode == "bsao" and prune:
            pqix = index["pq"]
            pqa = (pq_lut(Qr[qi], pqix["perm"], pqix["books"]), pqix["codes"], pqix["err"], m1, m3,
                   beta_q)
        lg = {}
        i, d, st, mg = search_one(Qr[qi], index["Y"], index["list_off"], index["list_ids"], probes,
                                  k, m, beta, bounds, B, L, prune, pre=pre if prune else None, res=res,
                                  pq=pqa, log=lg, flip=(flip or {}).get(qi, ()), near_tol=near_tol)
        ids[qi], ds[qi], stops[qi], margins[qi] = i, d, st, min(mg, pm)
        near.append(lg["near"])
        stage_near.append(lg["stage"])
    return dict(ids=ids, dists=ds, stops=stops, margin=margins, probes=probes_all, qrot=Qr, m=m,
                beta=beta, near=near, stage_near=stage_near, probe_near=probe_near,
                queries=np.asarray(queries),
                args=dict(k=k, nprobe=nprobe, alpha=alpha, mode=mode, B=B, L=L, calib_mode=calib_mode,
                          near_tol=near_tol))


# --------------------------------------------------------------------------------------
# Approximation accuracy of an estimate alone  [Sec. VII Exp-7, Table III: the estimate
# ranks the points directly, with no AKNN index logic, correction or refinement]
# --------------------------------------------------------------------------------------

def estimate_values(Y, qrot, ids, dims, estimator="partial"):
    """The estimate of ``estimate_scan`` for the stored rows ``ids`` and one rotated query."""
    D = Y.shape[1]
    d = min(int(dims), D)
    Yc = np.asarray(Y[ids], dtype=np.float64)
    q = np.asarray(qrot, dtype=np.float64)
    e = np.sum((Yc[:, :d] - q[None, :d]) ** 2, axis=1)
    if estimator == "partial":
        return (D / d) * e
    if estimator == "residual":
        return e + np.sum(Yc[:, d:] ** 2, axis=1) + float(np.sum(q[d:] ** 2))
    raise ValueError(estimator)


def estimate_scan(index, queries, k, nprobe, dims, estimator="partial"):
    """Top-k of the candidates of the nprobe nearest lists (nprobe = nlist: every point) by
    an estimated squared distance over the leading d = min(dims, D) rotated dimensions:

      'partial':  (D / d) * sum_{i<d} (q'_i - y_i)^2  -- the projection estimate; under a
                  random rotation its expectation is the distance (Sec. III, Lemma 1's
                  scaling); on the PCA rotation it ranks like the plain projected distance;
      'residual': sum_{i<d} (q'_i - y_i)^2 + ||y_r||^2 + ||q'_r||^2 = C1 - C2 of Alg. 1,
                  i.e. Eq. (1) with the cross term of the residual dims i >= d dropped.

    Ranked by (estimate, id), padded with (-1, inf).  Returns ids (nq, k), estimates (nq, k)
    and margin (nq,): the smallest relative gap at the k-th / (k+1)-th estimate and in the
    probe order, where other rounding may swap candidates."""
    Qr = rotate_as(queries, index["mu"], index["R"], index.get("rotation", "f32"))
    nq = Qr.shape[0]
    ids = np.full((nq, k), -1, dtype=np.int64)
    est = np.full((nq, k), np.inf)
    margin = np.full(nq, math.inf)
    off, lids = index["list_off"], index["list_ids"]
    for qi in range(nq):
        probes, _, pm = probe_order(Qr[qi], index["centroids"], nprobe)
        cand = np.concatenate([lids[off[l]:off[l + 1]] for l in probes]) if len(probes) else \
            np.zeros(0, np.int64)
        if cand.size == 0:
            continue
        v = estimate_values(index["Y"], Qr[qi], cand, dims, estimator)
        order = np.lexsort((cand, v))
        top = order[:k]
        ids[qi, :top.size] = cand[top]
        est[qi, :top.size] = v[top]
        mg = pm
        if order.size > k:
            a_, b_ = v[order[k - 1]], v[order[k]]
            mg = min(mg, abs(b_ - a_) / max(abs(b_), 1e-300))
        margin[qi] = mg
    return dict(ids=ids, est=est, margin=margin, qrot=Qr)


def bsar_multiplier(alpha: float, m: float) -> float:
    """The multiplier of the residual test: m itself when m > 0 (the paper fixes m per data
    set, Sec. VII-A), else the one-sided Gaussian quantile Phi^-1(1 - alpha) of the error
    model of Eq. (2) (Lemma 2: the quantile shrinks with the variance)."""
    if m > 0:
        return float(m)
    from statistics import NormalDist
    return NormalDist().inv_cdf(1.0 - alpha)


def recall_at(ids: np.ndarray, gt: np.ndarray, k: int = 10) -> float:
    """recall@k = |T ∩ G| / k averaged over queries [Sec. VII-A evaluation metrics]."""
    hits = 0
    for a, g in zip(ids[:, :k], gt[:, :k]):
        hits += len(set(a.tolist()) & set(g.tolist()))
    return hits / (k * ids.shape[0])


def false_prune_rate(index, queries, k, alpha, calib_mode="joint", mode="learned"):
    """Held-out check of the calibration: the fraction of (query, true K-NN) pairs that the
    stage tests (mode 'bsao': the quantization test) would prune at the query's final tau
    (its K-th true distance), i.e. the label-0 miss rate the target recall r = 1 - alpha
    bounds [Sec. V-A].  Also returns the per-query miss counts for a query-level bootstrap."""
    if mode == "bsao":
        m1, m3, Gq = pq_table_for_k(index, k)
        bq = float(beta_for_alpha(Gq, alpha, calib_mode)[0])
        pq = index["pq"]
        Qr = rotate(queries, index["mu"], index["R"])
        knn_ids, knn_d = bruteforce_knn(index["Y"], Qr, k)
        per_q = np.zeros(Qr.shape[0])
        for qi in range(Qr.shape[0]):
            adc = pq_adc(pq_lut(Qr[qi], pq["perm"], pq["books"]), pq["codes"][knn_ids[qi]])
            per_q[qi] = np.count_nonzero(m1 * adc + m3 * pq["err"][knn_ids[qi]] + bq > knn_d[qi, k - 1])
        return float(per_q.sum() / (k * Qr.shape[0])), per_q
    bounds = index["bounds"]
    St = bounds.shape[0] - 1
    m, G = table_for_k(index, k)
    beta = beta_for_alpha(G, alpha, calib_mode)
    pre = index.get("pre")
    Qr = rotate(queries, index["mu"], index["R"])
    knn_ids, knn_d = bruteforce_knn(index["Y"], Qr, k)
    per_q = np.zeros(Qr.shape[0])
    for qi in range(Qr.shape[0]):
        tau = knn_d[qi, k - 1]
        e = partial_dists(index["Y"][knn_ids[qi]], Qr[qi], bounds)[:, :St]
        if pre is not None:
            lead = pre["lead"]
            e0 = partial_dists(pre["dec"][knn_ids[qi]], Qr[qi][:lead], np.array([lead]))
            e = np.hstack([e0, e])
        per_q[qi] = np.count_nonzero((e * m[None, :] + beta[None, :] > tau).any(axis=1))
    return float(per_q.sum() / (k * Qr.shape[0])), per_q
