"""Pins of the FP64 oracle against what the paper and the mathematics fix (CPU only).

Each test checks an oracle function against something other than itself: a closed
form, a published value, an invariant, a library routine or brute force on a tiny
input.  Paper references are to sections, equations, theorems and algorithms.
"""
import heapq
import math
import os

import numpy as np
import pytest
import scipy.optimize
import scipy.spatial.distance as ssd

import oracle as O
import synthdata

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------------------- generator

def test_splitmix64_published_outputs():
    """SplitMix64 (Steele, Lea, Flood 2014) first outputs for seed 0."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "splitmix64.txt")) if l.strip() and l[0] != "#"]
    gamma = 0x9E3779B97F4A7C15
    for idx, hexv in rows:
        state = (int(idx) * gamma) % (1 << 64)
        assert int(O.splitmix64(np.uint64(state))) == int(hexv, 16)


def test_select_by_key_is_smallest_keys():
    keys = O.ctr_key(5, O.TAG_PCA, np.arange(1000, dtype=np.uint64))
    sel = O.select_by_key(1000, 37, 5, O.TAG_PCA)
    brute = sorted(range(1000), key=lambda i: (int(keys[i]), i))[:37]
    assert sorted(brute) == sel.tolist()


# ----------------------------------------------------------------------------- exact KNN

def test_bruteforce_matches_library_distance_sort():
    """Exact KNN [Sec. II-A] vs scipy's squared-Euclidean distance matrix + a full sort."""
    rng = np.random.default_rng(1)
    X = rng.standard_normal((700, 24)).astype(np.float32)
    Q = rng.standard_normal((9, 24)).astype(np.float32)
    X[5] = X[3]                                # an exact duplicate: tie broken by id
    Q[0] = X[3]
    ids, d = O.bruteforce_knn(X, Q, 12)
    Dm = ssd.cdist(Q.astype(np.float64), X.astype(np.float64), "sqeuclidean")
    for r in range(Q.shape[0]):
        ref = sorted(range(X.shape[0]), key=lambda i: (Dm[r, i], i))[:12]
        assert ids[r].tolist() == ref
        np.testing.assert_allclose(d[r], Dm[r, ref], rtol=1e-12, atol=1e-12)
    assert ids[0, 0] == 3 and ids[0, 1] == 5 and d[0, 0] == 0.0


def test_bruteforce_pads_when_k_exceeds_n():
    X = np.eye(3, dtype=np.float32)
    ids, d = O.bruteforce_knn(X, np.zeros((1, 3), np.float32), 5)
    assert ids[0, 3:].tolist() == [-1, -1] and np.isinf(d[0, 3:]).all()
    assert ids[0, :3].tolist() == [0, 1, 2]


# ----------------------------------------------------------------------------- PCA (Thm. 1)

def test_pca_closed_form_2d():
    """Covariance [[2,1],[1,2]] -> eigenvalues 3, 1 and eigenvectors (1,1)/sqrt2, (1,-1)/sqrt2."""
    lines = [l for l in open(os.path.join(GOLDEN, "pca_2d.txt")) if l.strip() and l[0] != "#"]
    P = np.array([[float(v) for v in l.split()] for l in lines])
    p = O.pca_fit(P)
    s = 1 / math.sqrt(2)
    np.testing.assert_allclose(p["mu"], [10, -5], atol=1e-14)
    np.testing.assert_allclose(p["lam"], [3, 1], atol=1e-13)
    np.testing.assert_allclose(p["R"], [[s, s], [s, -s]], atol=1e-13)


def test_pca_covariance_matches_library(small_workload):
    """C = (1/n) sum (x-mu)(x-mu)^T  (population covariance of the centred data)."""
    X = small_workload["base"][:2000]
    p = O.pca_fit(X)
    np.testing.assert_allclose(p["cov"], np.cov(X.astype(np.float64).T, bias=True), rtol=1e-10,
                               atol=1e-13)


def test_pca_rotation_orthogonal_and_diagonalising(small_workload):
    p = O.pca_fit(small_workload["base"])
    R, C, lam = p["R"], p["cov"], p["lam"]
    assert np.abs(R @ R.T - np.eye(R.shape[0])).max() <= 1e-12
    RC = R @ C @ R.T
    off = RC - np.diag(np.diag(RC))
    assert np.abs(off).max() <= 1e-10 * lam[0]
    np.testing.assert_allclose(np.diag(RC), lam, rtol=1e-9, atol=1e-12)
    assert np.all(np.diff(lam) <= 0)
    # sign rule: the largest-magnitude component of every row is positive
    assert np.all(R[np.arange(R.shape[0]), np.abs(R).argmax(axis=1)] > 0)


def test_pca_recovers_generating_spectrum(small_workload):
    """Data are Q diag(sqrt(1/i)) z: sample eigenvalues ~ 1/i and leading eigenvectors ~ the
    columns of Q (closed form of the generating covariance)."""
    w = small_workload
    p = O.pca_fit(w["base"])
    n = w["base"].shape[0]
    rel = np.abs(p["lam"][:16] - w["lam"][:16]) / w["lam"][:16]
    assert rel.max() <= 3 * math.sqrt(2 / n) * 3
    for i in range(3):
        assert abs(float(p["R"][i] @ w["rot"][:, i])) >= 0.99


def test_theorem1_pca_minimises_residual_variance(small_workload):
    """Thm. 1 (Ky Fan): for every d, the variance left in dims d+1..D after the PCA rotation
    is no larger than after any other orthogonal rotation (20 Haar draws)."""
    X = small_workload["base"][:3000].astype(np.float64)
    p = O.pca_fit(X)
    Xc = X - p["mu"]
    tail_pca = np.cumsum(np.var(Xc @ p["R"].T, axis=0)[::-1])[::-1]
    rng = np.random.default_rng(11)
    for _ in range(20):
        Rr = synthdata.haar_rotation(X.shape[1], rng)
        tail_r = np.cumsum(np.var(Xc @ Rr, axis=0)[::-1])[::-1]
        assert np.all(tail_pca <= tail_r * (1 + 1e-9) + 1e-12)


# ----------------------------------------------------------------------------- Eq. (1)

def test_eq1_rotation_invariance_full_stage(small_workload):
    """Eq. (1): ||x - q||^2 = ||R x - R q||^2, so the last stage's partial distance e_S of the
    rotated vectors is the exact distance in the original coordinates."""
    w = small_workload
    p = O.pca_fit(w["base"])
    Y = O.rotate(w["base"][:500], p["mu"], p["R"])
    bounds = O.stage_bounds(128, 32)
    for qi in range(5):
        q = w["queries"][qi]
        e = O.partial_dists(Y, O.rotate(q[None], p["mu"], p["R"])[0], bounds)
        exact = O.sq_dist_direct(w["base"][:500], q)
        np.testing.assert_allclose(e[:, -1], exact, rtol=1e-12)
        # partial distances of squares never decrease and never exceed the exact one
        assert np.all(np.diff(e, axis=1) >= 0)


def test_stage_bounds_ragged():
    assert O.stage_bounds(128, 32).tolist() == [32, 64, 96, 128]
    assert O.stage_bounds(100, 32).tolist() == [32, 64, 96, 100]
    assert O.stage_bounds(20, 32).tolist() == [20]


# ----------------------------------------------------------------------------- storage rounding

def test_storage_rounding_matches_library_and_definition():
    import torch
    rng = np.random.default_rng(3)
    y = rng.standard_normal(5000) * 10
    y32 = y.astype(np.float32)
    np.testing.assert_array_equal(O.round_storage(y, "f32"), y32.astype(np.float64))
    np.testing.assert_array_equal(O.round_storage(y, "f16"),
                                  torch.from_numpy(y32).to(torch.float16).double().numpy())
    np.testing.assert_array_equal(O.round_storage(y, "bf16"),
                                  torch.from_numpy(y32).to(torch.bfloat16).double().numpy())
    # ties to even on the bfloat16 grid near 1 (spacing 2^-7)
    assert O.round_storage(np.array([1 + 2 ** -8]), "bf16")[0] == 1.0
    assert O.round_storage(np.array([1 + 3 * 2 ** -8]), "bf16")[0] == 1 + 2 ** -6


def test_rotate_bf16_is_the_exact_product_of_the_rounded_operands():
    """BF16 query rotation reading: the centred query is the FP32 difference of the FP32
    query and the FP32 mean, rounded to bfloat16; R is rounded to FP32 and then bfloat16;
    the product is exact up to FP64 rounding.  Checked entry by entry against a product of
    the operands rounded by torch's bfloat16 conversion and summed in exact rational
    arithmetic, with inputs that sit on bfloat16 rounding ties."""
    import fractions

    import torch
    rng = np.random.default_rng(11)
    D = 6
    R = np.linalg.qr(rng.standard_normal((D, D)))[0]
    mu = rng.integers(-4, 5, D).astype(np.float64)     # integers: the tie rows centre exactly
    X = (rng.standard_normal((5, D)) * 3).astype(np.float32)
    mu32 = mu.astype(np.float32)
    X[0] = mu32 + np.float32(1 + 2 ** -8)          # tie: rounds to 1 (even)
    X[1] = mu32 + np.float32(1 + 3 * 2 ** -8)      # tie: rounds up to 1 + 2^-6 (even)
    got = O.rotate_bf16(X, mu, R)
    c = torch.from_numpy(X - mu32[None, :]).to(torch.bfloat16).double().numpy()
    assert np.all(c[0] == 1.0) and np.all(c[1] == 1 + 2 ** -6)
    Rb = torch.from_numpy(R.astype(np.float32)).to(torch.bfloat16).double().numpy()
    for qi in range(X.shape[0]):
        for i in range(D):
            exact = sum(fractions.Fraction(float(Rb[i, j])) * fractions.Fraction(float(c[qi, j]))
                        for j in range(D))
            bound = 1e-15 * sum(abs(Rb[i, j] * c[qi, j]) for j in range(D))
            assert abs(got[qi, i] - float(exact)) <= bound, (qi, i)
    # rows 0 and 1 are the tie values times the row sums of the rounded R
    np.testing.assert_allclose(got[0], Rb.sum(axis=1), rtol=1e-15)
    np.testing.assert_allclose(got[1], (1 + 2 ** -6) * Rb.sum(axis=1), rtol=1e-15)


def test_rotate_bf16_within_the_rounding_bound_of_the_fp64_rotation(small_workload, small_index):
    """Both operands are rounded with relative error <= 2^-9 (plus one FP32 rounding of the
    centred query), so |q'_bf16 - q'_64| <= (2^-8 + 2^-16) sum_j |R_ij| |q_j - mu_j| + tiny,
    and the reading really differs from the FP64 rotation."""
    ix = small_index
    Q = small_workload["queries"]
    a = O.rotate_bf16(Q, ix["mu"], ix["R"])
    b = O.rotate(Q, ix["mu"], ix["R"])
    bound = (2.0 ** -8 + 2.0 ** -16) * (np.abs(Q.astype(np.float64) - ix["mu"]) @ np.abs(ix["R"]).T)
    assert np.all(np.abs(a - b) <= bound * (1 + 1e-6) + 1e-12)
    assert np.abs(a - b).max() > 1e-4 * np.abs(b).max()
    np.testing.assert_array_equal(O.rotate_as(Q, ix["mu"], ix["R"], "bf16"), a)
    np.testing.assert_array_equal(O.rotate_as(Q, ix["mu"], ix["R"], "f32"), b)


# ----------------------------------------------------------------------------- IVF

def test_kmeans_two_clumps_closed_form():
    rng = np.random.default_rng(2)
    a = rng.standard_normal((50, 4)) * 0.01 + 10
    b = rng.standard_normal((70, 4)) * 0.01 - 10
    Y = np.vstack([a, b])
    C, assign = O.kmeans(Y, 2, iters=5, seed=1)
    got = sorted(map(tuple, np.round(C, 9)))
    want = sorted(map(tuple, np.round([a.mean(0), b.mean(0)], 9)))
    np.testing.assert_allclose(got, want, atol=1e-9)
    assert len(set(assign[:50])) == 1 and len(set(assign[50:])) == 1


def test_kmeans_assignment_is_nearest(small_index):
    ix = small_index
    Dm = ssd.cdist(ix["Y"][:2000], ix["centroids"], "sqeuclidean")
    ref = np.array([min(range(Dm.shape[1]), key=lambda j: (Dm[i, j], j)) for i in range(2000)])
    np.testing.assert_array_equal(ix["assign"][:2000], ref)
    off, ids = ix["list_off"], ix["list_ids"]
    assert off[-1] == ix["Y"].shape[0]
    for j in range(0, 64, 7):
        mem = ids[off[j]:off[j + 1]]
        assert np.all(np.diff(mem) > 0) and np.all(ix["assign"][mem] == j)


def test_probe_order_matches_library(small_index, small_workload):
    ix = small_index
    qr = O.rotate(small_workload["queries"][:4], ix["mu"], ix["R"])
    for q in qr:
        top, d, _ = O.probe_order(q, ix["centroids"], 8)
        Dm = ssd.cdist(q[None], ix["centroids"], "sqeuclidean")[0]
        ref = sorted(range(64), key=lambda j: (Dm[j], j))[:8]
        assert top.tolist() == ref


# ----------------------------------------------------------------------------- search semantics

def _probed_bruteforce(ix, qr, probes, k):
    cand = np.concatenate([ix["list_ids"][ix["list_off"][p]:ix["list_off"][p + 1]] for p in probes])
    d = ssd.cdist(qr[None], ix["Y"][cand], "sqeuclidean")[0]
    order = sorted(range(cand.shape[0]), key=lambda i: (d[i], cand[i]))[:k]
    return cand[order], d[order]


@pytest.mark.parametrize("mode", ["none", "lossless"])
def test_zero_pruning_and_lossless_reproduce_bruteforce(small_index, small_workload, mode):
    """No pruning, and the lossless partial-distance exit (m=1, beta=0: e_s <= dis, so
    e_s > tau implies dis > tau by Eq. (1)), both equal exact KNN over the probed lists."""
    ix = small_index
    r = O.search(ix, small_workload["queries"][:20], 10, 8, 0.0, mode=mode)
    for qi in range(20):
        ids, d = _probed_bruteforce(ix, r["qrot"][qi], r["probes"][qi], 10)
        assert r["ids"][qi].tolist() == ids.tolist()
        np.testing.assert_allclose(r["dists"][qi], d, rtol=1e-12)


def test_alpha_zero_and_all_lists_is_exact_knn(small_index, small_workload):
    ix = small_index
    Q = small_workload["queries"][:10]
    r = O.search(ix, Q, 10, 64, 0.0, mode="learned")
    gt, gd = O.bruteforce_knn(ix["Y"], r["qrot"], 10)
    np.testing.assert_array_equal(r["ids"], gt)
    np.testing.assert_allclose(r["dists"], gd, rtol=1e-12)


def test_lossless_prunes_something(small_index, small_workload):
    r = O.search(small_index, small_workload["queries"][:10], 10, 8, 0.0, mode="lossless")
    assert r["stops"][:, :-1].sum() > 0


def test_block_of_one_equals_sequential_heap(small_index, small_workload):
    """B = 1, L = 0 block-synchronous search == the paper's per-candidate refinement with a
    binary max-heap (coded separately), on a learned table that prunes."""
    ix = small_index
    beta = O.beta_for_alpha(ix["G"], 0.1)
    qr = O.rotate(small_workload["queries"][:6], ix["mu"], ix["R"])
    for q in qr:
        probes, _, _ = O.probe_order(q, ix["centroids"], 3)
        a_ids, a_d, stops, _ = O.search_one(q, ix["Y"], ix["list_off"], ix["list_ids"], probes, 10,
                                            ix["m"], beta, ix["bounds"], B=1, L=0)
        b_ids, b_d = O.search_sequential(q, ix["Y"], ix["list_off"], ix["list_ids"], probes, 10,
                                         ix["m"], beta, ix["bounds"])
        assert stops[:-1].sum() > 0
        assert a_ids.tolist() == b_ids.tolist()
        np.testing.assert_allclose(a_d, b_d, rtol=1e-12)


def test_lag_beyond_block_count_disables_pruning(small_index, small_workload):
    """tau_b is +inf when block b-1-L does not exist, so a lag longer than the whole scan
    reproduces the unpruned result."""
    ix = small_index
    r1 = O.search(ix, small_workload["queries"][:8], 10, 8, 0.2, L=10_000)
    r0 = O.search(ix, small_workload["queries"][:8], 10, 8, 0.0, mode="none")
    np.testing.assert_array_equal(r1["ids"], r0["ids"])
    assert r1["stops"][:, :-1].sum() == 0


def _lagged_heap_search(q, Y, off, ids, probes, k, m, beta, bounds, lag, B=1, invert_first=(),
                        pool=None):
    """Block-synchronous refinement with a lagged threshold, coded with heapq in this test:
    each list is cut into blocks of B consecutive positions; every candidate of block b is
    tested against the tau in force after block b-1-lag (+inf before it exists or while the
    queue held fewer than k); the block's survivors then enter the queue one by one.
    Candidates in ``invert_first`` take their first stage test the other way round.  With
    ``pool`` a list, (id, tau_b, dis) of every survivor with a finite tau_b below its
    distance is appended to it."""
    heap, taus = [], []   # heap of (-dis, -id); taus[b] = tau after block b
    stops = [0] * len(bounds)
    q = np.asarray(q, np.float64)
    b = 0
    for lst in probes:
        lo_l, hi_l = int(off[lst]), int(off[lst + 1])
        for start in range(lo_l, hi_l, B):
            j = b - 1 - lag
            tau = taus[j] if j >= 0 else math.inf
            survivors = []
            for pos in range(start, min(start + B, hi_l)):
                x = int(ids[pos])
                diff = q - Y[x]
                pruned = False
                if tau != math.inf:
                    for s in range(len(bounds) - 1):
                        e = float(np.sum(diff[:bounds[s]] ** 2))
                        test = m[s] * e + beta[s] > tau
                        if s == 0 and x in invert_first:
                            test = not test
                        if test:
                            pruned = True
                            stops[s] += 1
                            break
                if not pruned:
                    stops[-1] += 1
                    dis = float(np.sum(diff ** 2))
                    survivors.append((dis, x))
                    if pool is not None and tau != math.inf and dis > tau:
                        pool.append((x, tau, dis))
            for d, x in survivors:
                if len(heap) < k:
                    heapq.heappush(heap, (-d, -x))
                elif (d, x) < (-heap[0][0], -heap[0][1]):
                    heapq.heapreplace(heap, (-d, -x))
            taus.append(-heap[0][0] if len(heap) == k else math.inf)
            b += 1
    best = sorted((-a, -c) for a, c in heap)
    return [c for _, c in best], [a for a, _ in best], stops


@pytest.mark.parametrize("B,lag", [(1, 1), (1, 3), (16, 1), (64, 1), (64, 3)])
def test_lagged_blocks_equal_heap_loop(small_index, small_workload, B, lag):
    """Block b is tested against the tau after block b-1-L; the oracle's block-synchronous
    search equals a separately coded heap loop keeping every block's tau (ids, distances and
    the stage each candidate stopped at), and the lag changes what is pruned."""
    ix = small_index
    beta = O.beta_for_alpha(ix["G"], 0.1)
    qr = O.rotate(small_workload["queries"][:6], ix["mu"], ix["R"])
    pruned_lag = pruned0 = 0
    for q in qr:
        probes, _, _ = O.probe_order(q, ix["centroids"], 3)
        a_ids, a_d, stops, _ = O.search_one(q, ix["Y"], ix["list_off"], ix["list_ids"], probes, 10,
                                            ix["m"], beta, ix["bounds"], B=B, L=lag)
        b_ids, b_d, b_st = _lagged_heap_search(q, ix["Y"], ix["list_off"], ix["list_ids"], probes, 10,
                                               ix["m"], beta, ix["bounds"], lag, B)
        assert a_ids.tolist() == b_ids
        np.testing.assert_allclose(a_d, b_d, rtol=1e-12)
        assert stops.tolist() == b_st   # the same candidates pruned at the same stages
        _, _, st0, _ = O.search_one(q, ix["Y"], ix["list_off"], ix["list_ids"], probes, 10,
                                    ix["m"], beta, ix["bounds"], B=B, L=0)
        pruned_lag += int(stops[:-1].sum())
        pruned0 += int(st0[:-1].sum())
    assert 0 < pruned_lag != pruned0


def test_returned_distances_are_exact_for_stored_vectors(small_index, small_workload):
    ix = small_index
    r = O.search(ix, small_workload["queries"][:20], 10, 8, 0.1)
    for qi in range(20):
        exact = O.sq_dist_direct(ix["Y"][r["ids"][qi]], r["qrot"][qi])
        np.testing.assert_allclose(r["dists"][qi], exact, rtol=1e-12)
        assert np.all(np.diff(r["dists"][qi]) >= 0)


def test_topk_merge_matches_full_sort(small_index, small_workload):
    """With B larger than every list the queue is one merge of all survivors: a full sort."""
    ix = small_index
    q = O.rotate(small_workload["queries"][:1], ix["mu"], ix["R"])[0]
    probes, _, _ = O.probe_order(q, ix["centroids"], 1)
    ids, d, _, _ = O.search_one(q, ix["Y"], ix["list_off"], ix["list_ids"], probes, 25,
                                ix["m"], ix["m"] * 0, ix["bounds"], B=1 << 20, prune=False)
    ref_ids, ref_d = _probed_bruteforce(ix, q, probes, 25)
    assert ids.tolist() == ref_ids.tolist()


def test_empty_lists_and_short_candidate_sets_pad():
    Y = np.array([[0.0, 0.0], [1.0, 0.0]])
    off = np.array([0, 0, 2])
    lids = np.array([0, 1])
    ids, d, _, _ = O.search_one(np.zeros(2), Y, off, lids, np.array([0, 1]), 4, np.ones(0),
                                np.zeros(0), np.array([2]), B=256)
    assert ids.tolist() == [0, 1, -1, -1] and np.isinf(d[2:]).all()


# ----------------------------------------------------------------------------- calibration

def test_irls_matches_library_optimiser():
    """IRLS (Newton) minimiser == scipy BFGS minimiser of the same penalised cross-entropy."""
    rng = np.random.default_rng(4)
    F = rng.standard_normal((400, 2)) * [3.0, 1.0] + [5.0, 2.0]
    logit = 0.8 * F[:, 0] - 1.5 * F[:, 1] + 0.3
    y = (rng.random(400) < 1 / (1 + np.exp(-logit))).astype(float)
    b, w = O.irls_logistic(F, y)

    def loss(v):
        t = v[0] + F @ v[1:]
        return np.mean(np.logaddexp(0, t) - y * t) + 0.5e-8 * np.sum((v[1:] * F.std(0)) ** 2)

    ref = scipy.optimize.minimize(loss, np.zeros(3), method="BFGS", options=dict(gtol=1e-12)).x
    np.testing.assert_allclose([b, *w], ref, rtol=2e-5, atol=2e-5)
    # stationarity by central finite differences of the loss
    h = 1e-6
    g = [(loss(np.array([b, *w]) + h * e) - loss(np.array([b, *w]) - h * e)) / (2 * h) for e in np.eye(3)]
    assert np.max(np.abs(g)) < 1e-7


def test_classifier_to_correction_is_the_same_decision():
    """sign(w1 e + w2 tau + b) == [m e + beta > tau] on a grid (Sec. V-A linear model)."""
    b, w1, w2 = 0.7, 1.3, -2.1
    m, beta = O.classifier_to_correction(b, w1, w2)
    for e in np.linspace(0, 5, 21):
        for tau in np.linspace(0.1, 5, 17):
            assert (w1 * e + w2 * tau + b > 0) == (m * e + beta > tau)
    assert O.classifier_to_correction(0.0, 1.0, 0.5) == (1.0, 0.0)


def test_beta_single_stage_is_plain_quantile():
    """One test stage: the joint rule reduces to the (floor(alpha n0)+1)-th smallest residual."""
    g = np.random.default_rng(5).standard_normal((1000, 1))
    for a in [0.001, 0.005, 0.05, 0.1, 0.37]:
        assert O.beta_for_alpha(g, a)[0] == np.sort(g[:, 0])[int(math.floor(a * 1000))]


def test_beta_joint_bruteforce_small():
    """k* by enumerating every k on n0 <= 50, and F(k*) <= alpha < F(k*+1)."""
    rng = np.random.default_rng(6)
    for trial in range(20):
        n0, St = int(rng.integers(5, 50)), int(rng.integers(1, 5))
        G = rng.standard_normal((n0, St))
        for a in [0.01, 0.05, 0.1, 0.3]:
            beta = O.beta_for_alpha(G, a)

            def frac(k):
                thr = [sorted(G[:, s])[k] for s in range(St)]
                return sum(any(G[j, s] < thr[s] for s in range(St)) for j in range(n0)) / n0
            ks = [k for k in range(n0) if frac(k) <= a]
            kstar = max(ks)
            assert beta.tolist() == [sorted(G[:, s])[kstar] for s in range(St)]
            # with these betas the calibration set's joint false-prune fraction is frac(k*)
            pruned = (G < beta[None, :]).any(axis=1).mean()
            assert pruned == frac(kstar) <= a
            if kstar + 1 < n0:
                assert frac(kstar + 1) > a
    assert np.all(np.isneginf(O.beta_for_alpha(G, 0.0)))


def test_bonferroni_split():
    """Per-stage target r_i = 1 - (1-r)/(D/Delta_d) -> each stage gets alpha/S_t."""
    G = np.random.default_rng(8).standard_normal((2000, 4))
    beta = O.beta_for_alpha(G, 0.1, "bonferroni")
    k = int(math.floor(0.1 * 2000 / 4))
    assert beta.tolist() == np.sort(G, axis=0)[k].tolist()


def test_calibration_labels(small_index):
    cal = small_index["calib"]
    # label 0: the K_c true neighbours of each calibration query, tau = their K_c-th distance
    assert cal["pos_e"].shape == (1000 * 10, 3)
    np.testing.assert_array_equal(cal["pos_tau"].reshape(1000, 10), np.repeat(cal["knn_d"][:, 9:10], 10, 1))
    # label 1: at most 50 per query, every one met with a finite tau_b and dis > tau_b
    assert 0 < cal["neg_e"].shape[0] <= 50 * 1000
    assert np.all(np.isfinite(cal["neg_tau"]))
    m = small_index["m"]
    assert np.all(m > 0)


_M64 = (1 << 64) - 1


def _splitmix64_int(x):
    """SplitMix64 on Python integers (Steele, Lea & Flood 2014), written here on its own."""
    z = (x + 0x9E3779B97F4A7C15) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def test_splitmix64_int_matches_published_outputs():
    want = [int(line.split()[1], 16) for line in open(os.path.join(GOLDEN, "splitmix64.txt"))
            if line.strip() and not line.startswith("#")]
    state, got = 0, []
    for _ in range(len(want)):
        got.append(_splitmix64_int(state))
        state = (state + 0x9E3779B97F4A7C15) & _M64
    assert got == want


@pytest.mark.parametrize("B,lag", [(64, 0), (64, 1), (64, 3)])
def test_label_one_pool_is_smallest_keys_of_eligible_pairs(small_index, small_workload, B, lag):
    """Label 1 of the calibration [Sec. V-A "Parameter Learning"; Sec. VII-A: pairs met in a
    query process]: per training query, the unpruned canonical search (calib_nprobe lists,
    blocks of B, threshold lag L, K = K_c) is replayed with a heap loop written in this test;
    the eligible pairs are the candidates whose exact distance exceeds the finite tau_b of
    their block (the tau after block b-1-L, not the query's final tau); the kept pairs are
    the <= 50 with the smallest SplitMix64 keys of (query index << 32) + id.  The oracle's
    pairs, their tau_b and their stage features must be exactly these."""
    ix = small_index
    calib = small_workload["calib"][:40]
    seed, kc, nprobe_c, max_neg = 7, 10, 8, 50
    cal = O.calibrate(ix["Y"], ix["list_off"], ix["list_ids"], ix["centroids"], ix["mu"], ix["R"], calib,
                      ix["bounds"], calib_k=kc, calib_nprobe=nprobe_c, B=B, L=lag, seed=seed,
                      max_neg=max_neg)
    S = ix["bounds"].shape[0]
    base_key = _splitmix64_int((seed + O.TAG_NEG) & _M64)
    qr = (calib.astype(np.float64) - ix["mu"][None, :]) @ ix["R"].T
    total_pool = capped = 0
    for qi in range(calib.shape[0]):
        dc = ssd.cdist(qr[qi][None], ix["centroids"], "sqeuclidean")[0]
        probes = sorted(range(dc.shape[0]), key=lambda j: (dc[j], j))[:nprobe_c]
        pool = []
        _lagged_heap_search(qr[qi], ix["Y"], ix["list_off"], ix["list_ids"], probes, kc,
                            np.zeros(S - 1), np.full(S - 1, -np.inf), ix["bounds"], lag, B, pool=pool)
        total_pool += len(pool)
        capped += len(pool) > max_neg
        for x, tau_b, dis in pool:
            assert math.isfinite(tau_b) and dis > tau_b
        keyed = sorted(pool, key=lambda p: (_splitmix64_int((base_key + (qi << 32) + p[0]) & _M64), p[0]))
        want = sorted((x, t) for x, t, _ in keyed[:max_neg])
        sel = np.nonzero(cal["neg_q"] == qi)[0]
        got = sorted((int(cal["neg_id"][i]), float(cal["neg_tau"][i])) for i in sel)
        assert [g[0] for g in got] == [w_[0] for w_ in want], qi
        np.testing.assert_allclose([g[1] for g in got], [w_[1] for w_ in want], rtol=1e-12)
        for i in sel:   # stage features: the partial distances over the leading d_s dims
            y = ix["Y"][cal["neg_id"][i]]
            e = [float(np.sum((qr[qi][:d] - y[:d]) ** 2)) for d in ix["bounds"][:-1]]
            np.testing.assert_allclose(cal["neg_e"][i], e, rtol=1e-12)
    assert total_pool > 0 and capped > 0    # the key selection really chose among more pairs


def test_near_log_and_flip_replay(small_index, small_workload):
    """The near-threshold log holds exactly the candidates with an evaluated test within the
    tolerance of tau_b (recomputed here from the stage features), and a replay that inverts
    one candidate's first test equals the separately coded heap loop with that test
    inverted (ids, distances and stopping stages)."""
    ix = small_index
    beta = O.beta_for_alpha(ix["G"], 0.1)
    q = O.rotate(small_workload["queries"][:1], ix["mu"], ix["R"])[0]
    probes, _, _ = O.probe_order(q, ix["centroids"], 4)
    tol = 0.02
    lg = {}
    ids0, d0, st0, _ = O.search_one(q, ix["Y"], ix["list_off"], ix["list_ids"], probes, 10, ix["m"], beta,
                                    ix["bounds"], B=1, L=0, log=lg, near_tol=tol)
    # recompute: walk the sequential search keeping tau, note every test within tol
    heap, want = [], set()
    for lst in probes:
        for pos in range(int(ix["list_off"][lst]), int(ix["list_off"][lst + 1])):
            x = int(ix["list_ids"][pos])
            tau = -heap[0][0] if len(heap) == 10 else math.inf
            diff = q - ix["Y"][x]
            pruned = False
            if tau != math.inf:
                for s_, d in enumerate(ix["bounds"][:-1]):
                    lhs = ix["m"][s_] * float(np.sum(diff[:d] ** 2)) + beta[s_]
                    if abs(lhs - tau) / (abs(lhs - beta[s_]) + abs(beta[s_]) + abs(tau)) < tol:
                        want.add(x)
                    if lhs > tau:
                        pruned = True
                        break
            if not pruned:
                dis = float(np.sum(diff ** 2))
                if len(heap) < 10:
                    heapq.heappush(heap, (-dis, -x))
                elif (dis, x) < (-heap[0][0], -heap[0][1]):
                    heapq.heapreplace(heap, (-dis, -x))
    assert set(lg["stage"]) == want and len(want) > 0
    assert set(lg["stage"]) <= lg["near"]
    # invert the first test of candidates whose first test decided (huge tolerance: every
    # evaluated test counts as near, so "first near" is the first test)
    pruned_at_0 = [x for x in want][:3]
    for x in pruned_at_0:
        a_ids, a_d, a_st, _ = O.search_one(q, ix["Y"], ix["list_off"], ix["list_ids"], probes, 10, ix["m"],
                                           beta, ix["bounds"], B=1, L=0, flip=[x], near_tol=1e300)
        b_ids, b_d, b_st = _lagged_heap_search(q, ix["Y"], ix["list_off"], ix["list_ids"], probes, 10,
                                               ix["m"], beta, ix["bounds"], 0, 1, invert_first={x})
        assert a_ids.tolist() == b_ids and a_st.tolist() == b_st
        np.testing.assert_allclose(a_d, b_d, rtol=1e-12)
    # flipping a candidate with no test near its threshold changes nothing
    far = [int(x) for x in ids0 if int(x) not in lg["near"]][:1]
    r_ids, r_d, r_st, _ = O.search_one(q, ix["Y"], ix["list_off"], ix["list_ids"], probes, 10, ix["m"], beta,
                                       ix["bounds"], B=1, L=0, flip=far, near_tol=tol)
    assert r_ids.tolist() == ids0.tolist() and r_st.tolist() == st0.tolist()


def test_heldout_false_prune_rate_matches_significance(small_index, small_workload):
    """On fresh validation queries the fraction of true neighbours the stage tests would prune
    (at the query's final tau) matches alpha [Sec. V-A target recall r = 1 - alpha]: alpha lies
    in a 99% query-level bootstrap interval, widened by sqrt(2) because calibration and
    validation are two independent query samples of the same size."""
    rng = np.random.default_rng(9)
    for a in [0.05, 0.1]:
        rate, per_q = O.false_prune_rate(small_index, small_workload["val"], 10, a)
        boots = np.array([per_q[rng.integers(0, per_q.shape[0], per_q.shape[0])].mean() / 10
                          for _ in range(2000)])
        lo, hi = np.quantile(boots, [0.005, 0.995])
        half = (hi - lo) / 2 * math.sqrt(2)
        assert abs(rate - a) <= half, (a, rate, half)


def test_learned_pruning_scans_fewer_dims_and_keeps_recall(small_index, small_workload):
    ix = small_index
    Q = small_workload["queries"]
    r0 = O.search(ix, Q, 10, 8, 0.0, mode="none")
    r1 = O.search(ix, Q, 10, 8, 0.1)
    S = r1["stops"].shape[1]
    scanned = (r1["stops"] * np.arange(1, S + 1)).sum() / (r1["stops"].sum() * S)
    assert scanned < 0.6
    same = np.mean([len(set(a) & set(b)) / 10 for a, b in zip(r0["ids"], r1["ids"])])
    assert same >= 0.9


def test_rotate_orientation_gives_principal_coordinates(small_workload):
    """y = R (x - mu): the rotated coordinates are uncorrelated and their variances are the
    eigenvalues, largest first (a transposed R would still preserve distances but not this)."""
    X = small_workload["base"]
    p = O.pca_fit(X)
    Y = O.rotate(X, p["mu"], p["R"])
    cov = np.cov(Y.T, bias=True)
    np.testing.assert_allclose(np.diag(cov), p["lam"], rtol=1e-9, atol=1e-12)
    assert np.abs(cov - np.diag(np.diag(cov))).max() <= 1e-9 * p["lam"][0]
    np.testing.assert_allclose(Y.mean(axis=0), 0, atol=1e-9)


# ----------------------------------------------------------------------------- FP8 pre-stage

def _finite_codes():
    return [c for c in range(256) if not math.isnan(O.fp8_e4m3_value(c))]


def test_fp8_e4m3_published_values():
    """Code values against the OFP8 specification's E4M3 table (golden fixture)."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "fp8_e4m3.txt")) if l.strip() and l[0] != "#"]
    for hexc, val in rows:
        v = O.fp8_e4m3_value(int(hexc, 16))
        if val == "nan":
            assert math.isnan(v)
        else:
            assert v == float(val) and math.copysign(1, v) == math.copysign(1, float(val))
    fin = [O.fp8_e4m3_value(c) for c in _finite_codes()]
    assert len(fin) == 254 and max(fin) == 448.0 and min(fin) == -448.0
    pos = sorted({v for v in fin if v > 0})
    assert len(pos) == 126 and pos[0] == 2.0 ** -9       # strictly increasing magnitudes


def test_fp8_encode_is_nearest_ties_to_even_with_saturation():
    """Brute force over all finite codes: nearest value, ties to the even code (even
    mantissa), magnitudes beyond 448 clamp to 448."""
    codes = np.array(_finite_codes())
    vals = np.array([O.fp8_e4m3_value(c) for c in codes])
    rng = np.random.default_rng(5)
    v = np.concatenate([
        rng.standard_normal(3000) * 10.0 ** rng.uniform(-4, 3, 3000),
        # exact midpoints between neighbouring positive values (ties)
        (np.sort(vals[vals > 0])[:-1] + np.sort(vals[vals > 0])[1:]) / 2,
        -(np.sort(vals[vals > 0])[:-1] + np.sort(vals[vals > 0])[1:]) / 2,
        [0.0, -0.0, 448.0, 463.9, 464.0, 465.0, 1e6, -1e6, 2.0 ** -10, 2.0 ** -10 * 3, 2.0 ** -6],
    ]).astype(np.float32)
    got = O.fp8_e4m3_encode(v)
    for x, c in zip(v.astype(np.float64), got):
        xc = min(max(x, -448.0), 448.0)
        err = np.abs(vals - xc)
        best = err.min()
        cands = codes[err == best]
        if len(cands) > 1:
            cands = [c2 for c2 in cands if c2 % 2 == 0 or (c2 & 0x7F) == 0]
        if xc == 0.0:
            assert c in (0x00, 0x80) and (c == 0x80) == bool(np.signbit(x))
            continue
        assert int(c) in [int(t) for t in cands], (x, c, cands)


def test_fp8_lead_codes_per_list_tile(small_index):
    """Every (list, 64-position tile) has scale max|y|/448 (FP32); its largest element codes
    to +-448; decoded values are within half an E4M3 step of the stored values."""
    ix = small_index
    pre = O.fp8_encode_lead(ix["Y"], ix["list_off"], ix["list_ids"], 64)
    Y = ix["Y"][:, :64]
    for j in range(ix["list_off"].shape[0] - 1):
        lo, hi = int(ix["list_off"][j]), int(ix["list_off"][j + 1])
        for t0 in range(lo, hi, 64):
            ids = ix["list_ids"][t0:min(t0 + 64, hi)]
            s = pre["scale"][ids]
            assert np.all(s == s[0])
            amax = np.abs(Y[ids]).max()
            assert abs(float(s[0]) - amax / 448) <= 2.0 ** -23 * amax / 448
            assert np.any((pre["codes"][ids] & 0x7F) == 0x7E)
    v = Y / pre["scale"][:, None].astype(np.float64)
    a = np.abs(v)
    step = np.where(a < 2.0 ** -6, 2.0 ** -9, 2.0 ** (np.floor(np.log2(np.maximum(a, 1e-300))) - 3))
    decv = pre["dec"] / pre["scale"][:, None].astype(np.float64)
    assert np.all(np.abs(decv - v) <= step / 2 * (1 + 1e-6) + 1e-12)


@pytest.fixture(scope="module")
def fp8_index(small_workload):
    w = small_workload
    return O.fit(w["base"], w["calib"], nlist=64, kmeans_iters=25, calib_k=10, calib_nprobe=8,
                 seed=7, fp8_lead=64)


def test_fp8_prestage_block_of_one_equals_sequential(fp8_index, small_workload):
    ix = fp8_index
    St = ix["bounds"].shape[0] - 1
    assert ix["m"].shape == (St + 1,) and ix["G"].shape[1] == St + 1
    beta = O.beta_for_alpha(ix["G"], 0.1)
    pre = (ix["pre"]["dec"], ix["m"][0], beta[0])
    for qv in small_workload["queries"][:12]:
        qr = O.rotate(qv[None], ix["mu"], ix["R"])[0]
        probes, _, _ = O.probe_order(qr, ix["centroids"], 8)
        a = O.search_one(qr, ix["Y"], ix["list_off"], ix["list_ids"], probes, 10, ix["m"][1:],
                         beta[1:], ix["bounds"], B=1, L=0, pre=pre)
        b = O.search_sequential(qr, ix["Y"], ix["list_off"], ix["list_ids"], probes, 10, ix["m"][1:],
                                beta[1:], ix["bounds"], pre=pre)
        assert a[0].tolist() == b[0].tolist()
        np.testing.assert_array_equal(a[1], b[1])


def test_fp8_prestage_prunes_and_lossless_ignores_it(fp8_index, small_index, small_workload):
    Q = small_workload["queries"]
    r = O.search(fp8_index, Q, 10, 8, 0.1)
    assert r["stops"].shape[1] == fp8_index["bounds"].shape[0] + 1
    assert r["stops"][:, 0].sum() > 0                   # the pre-stage prunes candidates
    # lossless / none never use the FP8 estimate: identical to the index without codes
    for mode in ("lossless", "none"):
        a = O.search(fp8_index, Q, 10, 8, 0.0, mode=mode)
        b = O.search(small_index, Q, 10, 8, 0.0, mode=mode)
        assert a["ids"].tolist() == b["ids"].tolist()
    # every returned distance is the exact distance of the stored (not FP8) vector
    for qi in range(20):
        ok = r["ids"][qi] >= 0
        ex = O.sq_dist_direct(fp8_index["Y"][r["ids"][qi][ok]], r["qrot"][qi])
        np.testing.assert_allclose(r["dists"][qi][ok], ex, rtol=1e-12)


def test_fp8_heldout_false_prune_rate_matches_significance(fp8_index, small_workload):
    """The joint calibration covers the pre-stage too: held-out miss rate matches alpha."""
    rng = np.random.default_rng(9)
    for a in [0.05, 0.1]:
        rate, per_q = O.false_prune_rate(fp8_index, small_workload["val"], 10, a)
        boots = np.array([per_q[rng.integers(0, per_q.shape[0], per_q.shape[0])].mean() / 10
                          for _ in range(2000)])
        lo, hi = np.quantile(boots, [0.005, 0.995])
        half = (hi - lo) / 2 * math.sqrt(2)
        assert abs(rate - a) <= half, (a, rate, half)


# ----------------------------------------------------------------------------- tables per K_c

@pytest.fixture(scope="module")
def multi_k_index(small_workload):
    w = small_workload
    return O.fit(w["base"], w["calib"], nlist=64, kmeans_iters=25, calib_k=10, calib_nprobe=8,
                 seed=7, calib_k_extra=(50,))


def test_table_for_k_picks_largest_calibrated_k_not_above(multi_k_index):
    ix = multi_k_index
    t10, t50 = ix["tables"]
    assert t10["kc"] == 10 and t50["kc"] == 50
    assert t10["G"].shape[0] == 1000 * 10 and t50["G"].shape[0] == 1000 * 50
    for k, want in [(1, t10), (10, t10), (49, t10), (50, t50), (100, t50)]:
        m, G = O.table_for_k(ix, k)
        assert m is want["m"] and G is want["G"]


def test_table_at_k50_holds_significance_at_k50(multi_k_index, small_workload):
    """Label 0 = the K nearest with tau = the K-th distance: the K_c = 50 table reaches alpha
    for K = 50 searches on held-out queries (99% bootstrap interval, widened by sqrt 2)."""
    rng = np.random.default_rng(11)
    for a in [0.05, 0.1]:
        rate, per_q = O.false_prune_rate(multi_k_index, small_workload["val"], 50, a)
        boots = np.array([per_q[rng.integers(0, per_q.shape[0], per_q.shape[0])].mean() / 50
                          for _ in range(2000)])
        lo, hi = np.quantile(boots, [0.005, 0.995])
        assert abs(rate - a) <= (hi - lo) / 2 * math.sqrt(2), (a, rate)


# ----------------------------------------------------------------------------- random-rotation ablation

def test_gaussian_by_key_is_standard_normal():
    import scipy.stats as st
    z = O.gaussian_by_key(20000, 3, O.TAG_HAAR)
    assert st.kstest(z, "norm").pvalue > 0.01
    assert abs(z.mean()) < 0.03 and abs(z.std() - 1) < 0.03


def test_haar_rotation_orthogonal_and_sign_symmetric():
    """Orthogonal to rounding; with the sign fix every entry is symmetric about zero (QR
    without it leaves the first entry of the first column of one sign)."""
    R = O.haar_rotation(64, 5)
    assert np.abs(R @ R.T - np.eye(64)).max() < 1e-12
    r00 = np.array([O.haar_rotation(4, s)[0, 0] for s in range(2000)])
    assert 0.45 < (r00 > 0).mean() < 0.55 and abs(r00.mean()) < 0.03
    # E[R_ij^2] = 1/D for a uniformly random rotation
    sq = np.mean([O.haar_rotation(8, s) ** 2 for s in range(400)], axis=0)
    assert np.abs(sq - 1 / 8).max() < 0.03


def test_scaled_partial_distance_unbiased_under_random_rotation():
    """Isotropic data, random rotation: (D/d) e_d estimates the distance without bias (the
    premise of the ADSampling test), per stage within 2%."""
    rng = np.random.default_rng(0)
    X = rng.standard_normal((1000, 128))
    Q = rng.standard_normal((400, 128))
    R = O.haar_rotation(128, 7)
    Y, Qr = X @ R.T, Q @ R.T
    b = O.stage_bounds(128, 32)
    e = np.concatenate([O.partial_dists(Y, q, b) for q in Qr])
    est = (e[:, :-1] * (128 / b[:-1])[None, :]).mean(axis=0)
    assert np.all(np.abs(est / e[:, -1].mean() - 1) < 0.02)


def test_ads_test_is_safe_on_isotropic_data_and_exact_for_large_eps(small_workload):
    rng = np.random.default_rng(1)
    X = rng.standard_normal((6000, 128)).astype(np.float32)
    C = rng.standard_normal((12000, 128)).astype(np.float32)
    ix = O.fit(X, C[:200], nlist=16, kmeans_iters=5, calib_k=10, calib_nprobe=4, seed=3,
               projection="haar")
    Q = C[1000:1040]
    a = O.search(ix, Q, 10, 16, 0.0, mode="ads")
    n = O.search(ix, Q, 10, 16, 0.0, mode="none")
    assert a["stops"][:, :-1].sum() > 0                         # it prunes
    miss = np.mean([len(set(x) - set(y)) for x, y in zip(n["ids"], a["ids"])]) / 10
    assert miss < 0.01                                          # and rarely wrongly
    big = dict(ix, ads_eps0=1e6)
    b = O.search(big, Q, 10, 16, 0.0, mode="ads")
    assert b["ids"].tolist() == n["ids"].tolist() and b["stops"][:, :-1].sum() == 0


# ----------------------------------------------------------------------------- residual estimate (Alg. 1/2)

def test_eq2_residual_cross_term_is_gaussian_with_predicted_variance(small_workload):
    """Eq. (2): for a fixed query, 2 <q'_r, x_r> over the data is N(0, 4 sum_{i>d} q_i^2 lam_i)
    on the Gaussian workload (KS test against N(0, 1) after dividing by sigma)."""
    import scipy.stats as st
    p = O.pca_fit(small_workload["base"])
    Y = O.rotate(small_workload["base"], p["mu"], p["R"])
    Qr = O.rotate(small_workload["val"][:3], p["mu"], p["R"])
    b = O.stage_bounds(128, 32)
    for q in Qr:
        _, sig = O.bsar_terms(q, p["lam"], b)
        for s, d in enumerate(b[:-1]):
            z = 2 * (Y[:, d:] @ q[d:]) / sig[s]
            assert st.kstest(z, "norm").pvalue > 0.01
            assert abs(z.std() - 1) < 0.02 and abs(z.mean()) < 0.05


def test_residual_estimate_plus_cross_term_is_the_distance(small_workload):
    """C1 - C2 - C3 = dis (Alg. 1): e_s + ||x_r||^2 + ||q_r||^2 - 2 <q_r, x_r> == ||x - q||^2."""
    p = O.pca_fit(small_workload["base"])
    Y = O.rotate(small_workload["base"][:500], p["mu"], p["R"])
    q = O.rotate(small_workload["val"][:1], p["mu"], p["R"])[0]
    b = O.stage_bounds(128, 32)
    e = O.partial_dists(Y, q, b)
    xr = O.residual_norms(Y, b)
    qr, _ = O.bsar_terms(q, p["lam"], b)
    for s, d in enumerate(b[:-1]):
        est = e[:, s] + xr[:, s] + qr[s] - 2 * (Y[:, d:] @ q[d:])
        np.testing.assert_allclose(est, e[:, -1], rtol=1e-11)


def test_residual_test_block_of_one_equals_sequential(small_index, small_workload):
    ix = small_index
    b = ix["bounds"]
    for qv in small_workload["queries"][:10]:
        qr_, sig = O.bsar_terms(O.rotate(qv[None], ix["mu"], ix["R"])[0], ix["lam"], b)
        q = O.rotate(qv[None], ix["mu"], ix["R"])[0]
        probes, _, _ = O.probe_order(q, ix["centroids"], 8)
        res = (qr_, 2.0 * sig)
        one = np.ones(b.shape[0] - 1)
        a = O.search_one(q, ix["Y"], ix["list_off"], ix["list_ids"], probes, 10, one, 0 * one, b,
                         B=1, L=0, res=res)
        c = O.search_sequential(q, ix["Y"], ix["list_off"], ix["list_ids"], probes, 10, one, 0 * one,
                                b, res=res)
        assert a[0].tolist() == c[0].tolist()
        np.testing.assert_array_equal(a[1], c[1])


def test_residual_test_prunes_and_huge_multiplier_is_exact(small_index, small_workload):
    Q = small_workload["queries"]
    n = O.search(small_index, Q, 10, 8, 0.0, mode="none")
    r = O.search(dict(small_index, bsar_m=3.0), Q, 10, 8, 0.0, mode="bsar")
    assert r["stops"][:, :-1].sum() > 0.3 * r["stops"].sum()
    same = np.mean([len(set(x) & set(y)) / 10 for x, y in zip(n["ids"], r["ids"])])
    assert same > 0.98
    h = O.search(dict(small_index, bsar_m=1e12), Q, 10, 8, 0.0, mode="bsar")
    assert h["ids"].tolist() == n["ids"].tolist() and h["stops"][:, :-1].sum() == 0
    assert abs(O.bsar_multiplier(0.05, 0.0) - 1.6448536269514722) < 1e-9


# ----------------------------------------------------------------------------- out-of-distribution queries

def test_recalibration_on_100_ood_queries_restores_significance(small_index):
    """Sec. V-C: queries from a shifted distribution move the held-out false-prune rate away
    from alpha; recalibrating on about 100 such queries brings it back (99% bootstrap interval
    of the validation rate, widened by sqrt(1 + 1000/100) for the ten times smaller
    calibration sample)."""
    ix = small_index
    val = synthdata.ood_queries("gauss128", 1000, stream=13)
    cal = synthdata.ood_queries("gauss128", 100, stream=12)
    before, _ = O.false_prune_rate(ix, val, 10, 0.1)
    assert abs(before - 0.1) > 0.03                       # the in-distribution table misses alpha
    c2 = O.calibrate(ix["Y"], ix["list_off"], ix["list_ids"], ix["centroids"], ix["mu"], ix["R"], cal,
                     ix["bounds"], 10, 8, 256, 0, 7, 50)
    ix2 = dict(ix, m=c2["m"], G=c2["G"])
    rng = np.random.default_rng(5)
    for a in [0.05, 0.1]:
        rate, per_q = O.false_prune_rate(ix2, val, 10, a)
        boots = np.array([per_q[rng.integers(0, 1000, 1000)].mean() / 10 for _ in range(2000)])
        lo, hi = np.quantile(boots, [0.005, 0.995])
        assert abs(rate - a) <= (hi - lo) / 2 * math.sqrt(11), (a, rate)


# ----------------------------------------------------------------------------- estimate-only scan (Exp-7)

def _flat_index(Y, R=None, mu=None):
    """An index dict with one list holding every row (nprobe = 1 scans everything)."""
    n, D = Y.shape
    return dict(Y=np.asarray(Y, np.float64), R=np.eye(D) if R is None else R,
                mu=np.zeros(D) if mu is None else mu, centroids=np.zeros((1, D)),
                list_off=np.array([0, n]), list_ids=np.arange(n))


def test_estimate_scan_worked_example():
    """By hand, D = 2, d = 1, R = I, q' = (1, 2):
    x0 = (0, 0): partial 2 * 1^2 = 2; residual 1 + 0 + 4 = 5; exact 5
    x1 = (3, 1): partial 2 * 2^2 = 8; residual 4 + 1 + 4 = 9; exact 5
    x2 = (1,-1): partial 0;           residual 0 + 1 + 4 = 5; exact 9
    so partial ranks x2, x0, x1; residual ranks x0, x2 (tie 5, lower id first), x1."""
    ix = _flat_index(np.array([[0.0, 0.0], [3.0, 1.0], [1.0, -1.0]]))
    q = np.array([[1.0, 2.0]])
    p = O.estimate_scan(ix, q, 3, 1, 1, "partial")
    assert p["ids"][0].tolist() == [2, 0, 1] and p["est"][0].tolist() == [0.0, 2.0, 8.0]
    r = O.estimate_scan(ix, q, 3, 1, 1, "residual")
    assert r["ids"][0].tolist() == [0, 2, 1] and r["est"][0].tolist() == [5.0, 5.0, 9.0]
    assert r["margin"][0] == math.inf                  # k = n: no (k+1)-th candidate
    full = O.estimate_scan(ix, q, 2, 1, 2, "residual")  # d = D: exact distances
    assert full["ids"][0].tolist() == [0, 1] and full["est"][0].tolist() == [5.0, 5.0]
    pad = O.estimate_scan(ix, q, 5, 1, 1, "partial")
    assert pad["ids"][0, 3:].tolist() == [-1, -1] and np.all(np.isinf(pad["est"][0, 3:]))


def test_estimate_scan_full_dims_is_brute_force(small_index, small_workload):
    """d >= D: both estimates are the exact distance, so all lists give the exact KNN."""
    Q = small_workload["queries"][:20]
    Qr = O.rotate(Q, small_index["mu"], small_index["R"])
    gi, gd = O.bruteforce_knn(small_index["Y"], Qr, 10)
    for est in ("partial", "residual"):
        r = O.estimate_scan(small_index, Q, 10, 64, 128, est)
        assert r["ids"].tolist() == gi.tolist()
        np.testing.assert_allclose(r["est"], gd, rtol=1e-12)


def test_estimates_match_the_projector_form_in_original_coordinates(small_index, small_workload):
    """Written with the projector P_d = R_d^T R_d onto the leading d axes, in the original
    coordinates:  partial = (D/d) ||P_d (q - x)||^2  and  residual = ||q - x||^2 +
    2 (q - mu)^T (I - P_d) (x - mu)  (the dropped cross term of the residual dims, sign
    included)."""
    X = small_workload["base"][:300].astype(np.float64)
    q = small_workload["queries"][3].astype(np.float64)
    mu, R, Y = small_index["mu"], small_index["R"], small_index["Y"]
    qr = O.rotate(q[None, :], mu, R)[0]
    for d in (32, 64, 96):
        Pd = R[:d].T @ R[:d]
        diff = q[None, :] - X
        part = (128 / d) * np.einsum("ij,jk,ik->i", diff, Pd, diff)
        res = np.sum(diff ** 2, axis=1) + 2 * ((q - mu) @ (np.eye(128) - Pd) @ (X - mu).T)
        # the oracle works on the stored (rotated, FP32-rounded) rows of the same points
        ids = np.arange(300)
        np.testing.assert_allclose(O.estimate_values(Y, qr, ids, d, "partial"), part, rtol=1e-5)
        np.testing.assert_allclose(O.estimate_values(Y, qr, ids, d, "residual"), res, rtol=1e-5)


def test_partial_estimate_unbiased_over_random_rotations():
    """Averaged over Haar rotations, the partial estimate of a fixed pair is its distance
    (the (D/d) scale of the random-projection column); a wrong scale is off by >= 25%."""
    rng = np.random.default_rng(4)
    X = rng.standard_normal((4, 16))
    q = rng.standard_normal((1, 16))
    exact = np.sum((X - q) ** 2, axis=1)
    acc = np.zeros(4)
    reps = 600
    for s in range(reps):
        R = O.haar_rotation(16, 100 + s)
        r = O.estimate_scan(_flat_index(X @ R.T, R=R), q, 4, 1, 4, "partial")
        acc[r["ids"][0]] += r["est"][0]
    np.testing.assert_allclose(acc / reps, exact, rtol=0.12)


# ----------------------------------------------------------------------------- quantization estimate (BSA-O)

@pytest.fixture(scope="module")
def pq_index(small_workload):
    w = small_workload
    return O.fit(w["base"], w["calib"], nlist=64, kmeans_iters=10, calib_k=10, calib_nprobe=8, seed=7,
                 pq_m=32, pq_iters=8)


def test_opq_allocation_worked_examples():
    """By hand, eigenvalues over their geometric mean g: [8, 4, 2, 1] (g = 2 sqrt 2) into 2
    subspaces: 8 -> s0 (ties: lowest), 4 -> s1 (empty product 1 < 8/g), 2 -> s1 (4/g < 8/g),
    1 -> s0 (s1 full); products 8 and 8.  [16, 8, 4, 2, 1, 1] (g = 1024^(1/6)) into 3:
    16 -> s0, 8 -> s1, 4 -> s2 (empty subspaces first: 1 < 8/g), 2 -> s2 (4/g smallest),
    1 -> s1 (8/g < 16/g), 1 -> s0; products 16, 8, 8.  Scaling the eigenvalues changes
    nothing."""
    assert O.opq_allocation(np.array([8.0, 4, 2, 1]), 2).tolist() == [[0, 3], [1, 2]]
    assert O.opq_allocation(np.array([16.0, 8, 4, 2, 1, 1]), 3).tolist() == [[0, 5], [1, 4], [2, 3]]
    # unsorted input: axes are dealt by eigenvalue, not by index
    assert O.opq_allocation(np.array([1.0, 8, 2, 4]), 2).tolist() == [[0, 1], [2, 3]]
    for c in (1e-6, 1e6):
        assert O.opq_allocation(c * np.array([16.0, 8, 4, 2, 1, 1]), 3).tolist() == \
            [[0, 5], [1, 4], [2, 3]]


def test_opq_allocation_is_a_balanced_partition():
    lam = 1.0 / np.arange(1, 129)
    perm = O.opq_allocation(lam, 32)
    assert sorted(perm.reshape(-1).tolist()) == list(range(128)) and perm.shape == (32, 4)
    logp = np.log(lam)[perm].sum(axis=1)
    contiguous = np.log(lam).reshape(32, 4).sum(axis=1)
    assert np.ptp(logp) < 0.2 * np.ptp(contiguous)


def test_pq_encode_is_the_nearest_codeword(pq_index):
    """Every code of every stored row and subspace is the nearest codeword: the FP32 argmin
    equals the FP64 argmin over the same operands (the stored values and the codewords as the
    FP32 values the encoder reads), except where the two FP64 distances are so close that the
    encoder's FP32 rounding can order them either way.  Bound: each of the dsub terms is a
    rounded difference, rounded square and rounded running sum of nonnegative terms, so the
    FP32 distance is within (dsub + 2) u (1 + o(1)) of the exact one (u = 2^-24); two distances
    can swap only if they differ by less than (dsub + 3) u times their sum.  A wrong axis, a
    dropped or transposed term or a wrong tie rule moves codes far outside this bound."""
    pq = pq_index["pq"]
    Y = pq_index["Y"].astype(np.float32).astype(np.float64)
    codes = pq["codes"].astype(np.int64)
    M, ksub, dsub = pq["books"].shape
    u = 2.0 ** -24
    flips = 0
    for j in range(M):
        C = pq["books"][j].astype(np.float32).astype(np.float64)            # [ksub, dsub]
        d = ((Y[:, pq["perm"][j]][:, None, :] - C[None, :, :]) ** 2).sum(-1)  # FP64
        best = d.argmin(axis=1)
        got = codes[:, j]
        diff = np.nonzero(got != best)[0]
        if diff.size:
            dg, db = d[diff, got[diff]], d[diff, best[diff]]
            assert np.all(dg - db <= (dsub + 3) * u * (dg + db)), (j, float((dg - db).max()))
            flips += diff.size
    assert flips <= 1e-4 * codes.size, flips     # near ties are rare
    # exact ties (none in the data above): duplicated codewords, the lowest index wins
    rng = np.random.default_rng(4)
    books = rng.standard_normal((2, 8, 2))
    books[0, 5] = books[0, 2]                      # codeword 2 repeated at 5
    books[1, 7] = books[1, 1]                      # codeword 1 repeated at 7
    perm = np.array([[0, 2], [1, 3]])
    Yt = np.zeros((2, 4))
    Yt[0, [0, 2]] = books[0, 2]
    Yt[0, [1, 3]] = books[1, 1]
    Yt[1, [0, 2]] = books[0, 5] + 1e-3
    Yt[1, [1, 3]] = books[1, 7] - 1e-3
    np.testing.assert_array_equal(O.pq_encode(Yt, perm, books), [[2, 1], [2, 1]])


def test_pq_error_and_adc_equal_distances_to_the_reconstruction(pq_index, small_workload):
    """err(x) = ||y - recon(y)||^2 and dis' = ||q' - recon(y)||^2, with recon(y) assembled by
    writing every codeword back to its subspace's axes."""
    pq = pq_index["pq"]
    ids = np.arange(0, 10000, 37)
    rec = np.zeros((ids.size, 128))
    for j in range(32):
        rec[:, pq["perm"][j]] = pq["books"][j][pq["codes"][ids, j]]
    Y = pq_index["Y"][ids]
    np.testing.assert_allclose(pq["err"][ids], ((Y - rec) ** 2).sum(1), rtol=1e-12)
    q = O.rotate(small_workload["queries"][:1], pq_index["mu"], pq_index["R"])[0]
    adc = O.pq_adc(O.pq_lut(q, pq["perm"], pq["books"]), pq["codes"][ids])
    np.testing.assert_allclose(adc, ((q[None, :] - rec) ** 2).sum(1), rtol=1e-12)


def test_classifier3_to_correction_is_the_same_decision():
    rng = np.random.default_rng(2)
    for _ in range(50):
        b, w1, w3 = rng.normal(size=3)
        w2 = -abs(rng.normal())
        w1 = abs(w1)
        m1, m3, beta = O.classifier3_to_correction(b, w1, w3, w2)
        F = rng.normal(size=(200, 3)) * 3
        lhs = (w1 * F[:, 0] + w3 * F[:, 1] + w2 * F[:, 2] + b) > 0
        rhs = m1 * F[:, 0] + m3 * F[:, 1] + beta > F[:, 2]
        close = np.abs(w1 * F[:, 0] + w3 * F[:, 1] + w2 * F[:, 2] + b) < 1e-9
        assert np.array_equal(lhs[~close], rhs[~close])
    assert O.classifier3_to_correction(0.3, 1.0, 0.5, 0.2) == (1.0, 0.0, 0.0)


def test_pq_classifier_is_the_logistic_optimum(pq_index):
    """The BSA-O weights are a stationary point of the penalised cross-entropy (3 features)."""
    t = pq_index["pq_tab"]
    cal = pq_index["calib"]
    F = np.vstack([np.column_stack([t["pos_adc"], t["pos_err"], cal["pos_tau"]]),
                   np.column_stack([t["neg_adc"], t["neg_err"], cal["neg_tau"]])])
    y = np.concatenate([np.zeros(t["pos_adc"].size), np.ones(t["neg_adc"].size)])
    b, w = t["lr"]
    mean, std = F.mean(0), F.std(0)
    Z = (F - mean) / std
    ws = w * std
    b0 = b + float(np.dot(w, mean))
    p = 1.0 / (1.0 + np.exp(-(Z @ ws + b0)))
    g = np.concatenate([[np.mean(p - y)], Z.T @ (p - y) / y.size + 1e-8 * ws])
    assert np.abs(g).max() < 1e-9
    m1, m3, _ = O.classifier3_to_correction(b, w[0], w[1], w[2])
    assert (t["m1"], t["m3"]) == (m1, m3) and t["m1"] > 0


def test_bsao_zero_significance_is_the_unpruned_search(pq_index, small_workload):
    Q = small_workload["queries"][:30]
    a = O.search(pq_index, Q, 10, 8, 0.0, mode="bsao")
    n = O.search(pq_index, Q, 10, 8, 0.0, mode="none")
    assert a["ids"].tolist() == n["ids"].tolist()


def test_bsao_block_of_one_equals_sequential(pq_index, small_workload):
    Q = small_workload["queries"][:12]
    r = O.search(pq_index, Q, 10, 8, 0.2, mode="bsao", B=1)
    m1, m3, Gq = O.pq_table_for_k(pq_index, 10)
    bq = float(O.beta_for_alpha(Gq, 0.2)[0])
    pq = pq_index["pq"]
    St = pq_index["bounds"].shape[0] - 1
    pruned = r["stops"][:, 0].sum()
    assert pruned > 0
    for qi in range(Q.shape[0]):
        qr = r["qrot"][qi]
        arg = (O.pq_lut(qr, pq["perm"], pq["books"]), pq["codes"], pq["err"], m1, m3, bq)
        ids, ds = O.search_sequential(qr, pq_index["Y"], pq_index["list_off"], pq_index["list_ids"],
                                      r["probes"][qi], 10, np.ones(St), np.full(St, -np.inf),
                                      pq_index["bounds"], pq=arg)
        assert ids.tolist() == r["ids"][qi].tolist()
        np.testing.assert_allclose(ds, r["dists"][qi], rtol=1e-12)


def test_bsao_heldout_false_prune_rate_matches_significance(pq_index, small_workload):
    rng = np.random.default_rng(11)
    for a in (0.05, 0.2):
        rate, per_q = O.false_prune_rate(pq_index, small_workload["val"], 10, a, mode="bsao")
        boots = np.array([per_q[rng.integers(0, per_q.shape[0], per_q.shape[0])].mean() / 10
                          for _ in range(2000)])
        lo, hi = np.quantile(boots, [0.005, 0.995])
        assert abs(rate - a) <= (hi - lo) / 2 * math.sqrt(2), (a, rate)


def test_lag_beyond_every_training_scan_leaves_label_one_empty():
    """With a lag longer than any training query's block count no candidate meets a finite
    tau_b: the label-1 pool is empty, no classifier is fitted (m_s = 1), and the label-0
    residuals are tau - e_s, non-negative since e_s <= dis <= tau (Eq. (1))."""
    w = synthdata.make_workload("gauss128", n_calib=60)
    ix = O.fit(w["base"], w["calib"], nlist=64, kmeans_iters=5, calib_k=10, calib_nprobe=8,
               seed=7, B=1024, L=64)
    cal = ix["calib"]
    assert cal["neg_e"].shape[0] == 0
    np.testing.assert_array_equal(ix["m"], np.ones_like(ix["m"]))
    np.testing.assert_allclose(ix["G"], cal["pos_tau"][:, None] - cal["pos_e"], rtol=0, atol=0)
    assert np.all(ix["G"] >= 0)
