"""GPU (HIP, gfx950) vs FP64 oracle parity, through the C ABI.

Bar (from the method's contract): ids identical except where the oracle logged a decision
quantity within 1e-4 (relative) of its threshold; every returned FP32 distance within 1e-4
(relative) of the FP64 distance of the stored vector; padding and ordering exact.
"""
import numpy as np
import pytest

import oracle as O
from parity_util import TOL, artifacts, check_search, oracle_index, workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_2404_16322_amd as P
    P.load_library()
    return P


def _gpu_index(ix, with_table=True):
    from paper_2404_16322_amd import Index
    return Index.from_artifacts(artifacts(ix, with_table))


def _assert_ok(res, max_excused_frac=0.05):
    print(f"parity: {res['same']}/{res['nq']} identical, {res['excused']} excused near-threshold")
    assert not res["bad"], res["bad"][:5]
    assert res["excused"] <= max_excused_frac * res["nq"] + 1


# ------------------------------------------------------------------------------ A1, A2

def test_rotation_and_probes_match_oracle():
    ix = oracle_index()
    w = workload("gauss128")
    g = _gpu_index(ix)
    Q = np.vstack([w["queries"], w["val"][:400]])
    qr, probes = g.debug_intermediates(Q, 8)
    ref = O.rotate(Q, ix["mu"], ix["R"])
    scale = np.linalg.norm(Q.astype(np.float64) - ix["mu"], axis=1)
    assert np.all(np.abs(qr - ref) <= 1e-5 * scale[:, None])
    differ = 0
    for qi in range(Q.shape[0]):
        top, _, margin = O.probe_order(ref[qi], ix["centroids"], 8)
        if probes[qi].tolist() != top.tolist():
            differ += 1
            assert margin < TOL, (qi, probes[qi], top)
    assert differ <= 2


def test_rotation_bf16_matrix_cores_within_bf16_bound():
    ix = oracle_index()
    w = workload("gauss128")
    from paper_2404_16322_amd import Index
    art = artifacts(ix)
    art["rotation"] = "bf16"
    g = Index.from_artifacts(art)
    qr, _ = g.debug_intermediates(w["queries"], 8)
    ref = O.rotate(w["queries"], ix["mu"], ix["R"])
    # both operands rounded to bfloat16 (relative 2^-9 each), FP32 accumulation
    bound = 2.0 ** -7 * (np.abs(w["queries"].astype(np.float64) - ix["mu"]) @ np.abs(ix["R"]).T)
    assert np.all(np.abs(qr - ref) <= bound + 1e-6)
    assert np.abs(qr - ref).max() > 1e-7   # really went through bf16


# ------------------------------------------------------------------------------ A3-A5

@pytest.mark.parametrize("alpha", [0.05, 0.1, 0.3])
@pytest.mark.parametrize("k,nprobe", [(10, 8), (1, 3), (100, 16)])
def test_learned_search_matches_oracle(alpha, k, nprobe):
    ix = oracle_index()
    w = workload("gauss128")
    Q = np.vstack([w["queries"], w["val"][:300]])
    g = _gpu_index(ix)
    ids, d, st = g.search(Q, k, nprobe, alpha)
    ora = O.search(ix, Q, k, nprobe, alpha)
    _assert_ok(check_search(ids, d, ora, ix))
    # work counters: the same candidates, pruning close to the oracle's
    assert st["candidates"] == int(ora["stops"].sum())
    assert abs(st["refined"] - int(ora["stops"][:, -1].sum())) <= 0.01 * st["candidates"] + 5


@pytest.mark.parametrize("mode", ["lossless", "none"])
def test_lossless_and_none_equal_exact_over_probed_lists(mode):
    ix = oracle_index()
    w = workload("gauss128")
    g = _gpu_index(ix)
    ids, d, st = g.search(w["queries"], 10, 8, 0.0, mode=mode)
    ora = O.search(ix, w["queries"], 10, 8, 0.0, mode="none")
    _assert_ok(check_search(ids, d, ora, ix), 0.02)
    if mode == "none":
        assert st["refined"] == st["candidates"]
    else:
        assert st["refined"] < st["candidates"]


def test_zero_significance_all_lists_is_bruteforce():
    ix = oracle_index()
    w = workload("gauss128")
    g = _gpu_index(ix)
    ids, d, _ = g.search(w["queries"], 20, 64, 0.0)
    qr = O.rotate(w["queries"], ix["mu"], ix["R"])
    gt, gd = O.bruteforce_knn(ix["Y"], qr, 20)
    diff = (ids != gt).any(axis=1)
    for qi in np.nonzero(diff)[0]:   # only exact-distance near ties may swap
        rel = np.abs(np.diff(gd[qi])) / gd[qi][1:]
        assert rel.min() < TOL, qi
    assert diff.sum() <= 2
    np.testing.assert_allclose(np.sort(d, axis=1), d)


def test_padding_when_fewer_candidates_than_k():
    ix = oracle_index()
    w = workload("gauss128")
    g = _gpu_index(ix)
    ids, d, _ = g.search(w["queries"][:10], 256, 1, 0.1)
    ora = O.search(ix, w["queries"][:10], 256, 1, 0.1)
    _assert_ok(check_search(ids, d, ora, ix), 0.2)
    assert (ids == -1).any() and np.isinf(d[ids == -1]).all()


@pytest.mark.parametrize("B", [64, 512])
def test_block_size_variants(B):
    ix = oracle_index(B=B, n_calib=300)
    w = workload("gauss128")
    g = _gpu_index(ix)
    ids, d, _ = g.search(w["queries"], 10, 8, 0.1)
    ora = O.search(ix, w["queries"], 10, 8, 0.1)
    _assert_ok(check_search(ids, d, ora, ix))


def test_ragged_dimension_and_wide_stages():
    # D = 100 (not a multiple of 32) with Delta_d = 64: stages end at 64 and 100
    ix = oracle_index(D=100, delta_d=64, n_calib=300)
    w = workload("gauss128", D=100)
    g = _gpu_index(ix)
    assert g.info()["n_test_stages"] == 1
    ids, d, _ = g.search(w["queries"], 10, 8, 0.1)
    ora = O.search(ix, w["queries"], 10, 8, 0.1)
    _assert_ok(check_search(ids, d, ora, ix))


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_half_precision_storage(storage):
    ix = oracle_index(storage=storage, n_calib=300)
    w = workload("gauss128")
    g = _gpu_index(ix)
    exp = g.export()
    np.testing.assert_array_equal(exp["y"], ix["Y"].astype(np.float32))
    ids, d, _ = g.search(w["queries"], 10, 8, 0.1)
    ora = O.search(ix, w["queries"], 10, 8, 0.1)
    _assert_ok(check_search(ids, d, ora, ix))


def test_per_query_k_and_nprobe():
    ix = oracle_index()
    w = workload("gauss128")
    g = _gpu_index(ix)
    rng = np.random.default_rng(5)
    Q = w["queries"][:60]
    ks = rng.choice([1, 10, 50, 100], size=60).astype(np.int32)
    nps = rng.integers(1, 33, size=60).astype(np.int32)
    ids, d, off, _ = g.search_var(Q, ks, nps, 0.1)
    for qi in range(60):
        ora = O.search(ix, Q[qi:qi + 1], int(ks[qi]), int(nps[qi]), 0.1)
        res = check_search(ids[off[qi]:off[qi + 1]][None], d[off[qi]:off[qi + 1]][None], ora, ix)
        assert not res["bad"], (qi, res["bad"])


def test_empty_lists_and_single_vector_lists():
    ix = dict(oracle_index())
    # move every member of lists 3 and 5 into list 4; list 7 keeps only its first member
    assign = ix["assign"].copy()
    assign[np.isin(assign, [3, 5])] = 4
    seven = np.nonzero(assign == 7)[0]
    assign[seven[1:]] = 6
    ix["assign"] = assign
    ix["list_off"], ix["list_ids"] = O.build_lists(assign, 64)
    w = workload("gauss128")
    g = _gpu_index(ix)
    ids, d, _ = g.search(w["queries"], 10, 12, 0.1)
    ora = O.search(ix, w["queries"], 10, 12, 0.1)
    _assert_ok(check_search(ids, d, ora, ix))


# ------------------------------------------------------------------------------ correction table

def test_target_recall_bias_equals_oracle_order_statistic():
    ix = oracle_index()
    g = _gpu_index(ix)
    for a in [0.0, 0.001, 0.01, 0.1, 0.5]:
        for mode in ["joint", "bonferroni"]:
            m, b = g.correction(a, mode)
            np.testing.assert_array_equal(m, ix["m"])
            np.testing.assert_array_equal(b, O.beta_for_alpha(ix["G"], a, mode))


def test_gpu_calibration_equals_oracle_on_identical_inputs():
    """Calibration (FP64 on the GPU) from the oracle's rotation, lists and stored base: the
    label-0/label-1 sets are identical, so m_s and beta_s(alpha) agree to FP64 rounding."""
    ix = oracle_index()
    w = workload("gauss128")
    g = _gpu_index(ix, with_table=False)
    g.calibrate(w["calib"], calib_k=10, calib_nprobe=8, max_neg=50, seed=7)
    info = g.info()
    assert info["n0"] == ix["G"].shape[0]
    for a in [0.01, 0.1]:
        m, b = g.correction(a)
        np.testing.assert_allclose(m, ix["m"], rtol=1e-6)
        ref = O.beta_for_alpha(ix["G"], a)
        np.testing.assert_allclose(b, ref, rtol=1e-6, atol=1e-9 * np.abs(ref).max())


def test_export_roundtrip():
    ix = oracle_index()
    g = _gpu_index(ix)
    e = g.export()
    np.testing.assert_array_equal(e["y"], ix["Y"].astype(np.float32))
    np.testing.assert_array_equal(e["assign"], ix["assign"])
    np.testing.assert_array_equal(e["R"], ix["R"])
    np.testing.assert_array_equal(e["resid"], ix["G"])


# ------------------------------------------------------------------------------ fit on the GPU

def test_gpu_fit_pca_and_index_against_oracle():
    """GPU fit: FP64 covariance + host eigensolver vs the oracle's PCA (L0), and a search of
    the GPU-fitted index against the oracle searching the exported artifacts."""
    from paper_2404_16322_amd import Index
    w = workload("gauss128")
    g = Index.fit(w["base"], w["calib"], nlist=64, kmeans_iters=25, calib_k=10, calib_nprobe=8,
                  seed=7)
    e = g.export()
    p = O.pca_fit(w["base"])
    np.testing.assert_allclose(e["mu"], p["mu"], rtol=1e-12, atol=1e-12)
    lam = p["lam"]
    np.testing.assert_allclose(e["lam"], lam, rtol=1e-9, atol=1e-12 * lam[0])
    gaps = np.minimum(np.r_[np.inf, -np.diff(lam)], np.r_[-np.diff(lam), np.inf]) / lam[0]
    sep = gaps > 1e-6
    dots = np.abs(np.sum(e["R"] * p["R"], axis=1))
    assert np.all(dots[sep] >= 1 - 1e-8)
    assert np.abs(e["R"] @ e["R"].T - np.eye(128)).max() < 1e-12
    # the GPU's own index: search it and the oracle on the same (exported) artifacts
    ix = dict(mu=e["mu"], R=e["R"], Y=e["y"].astype(np.float64), centroids=e["centroids"].astype(np.float64),
              assign=e["assign"], bounds=O.stage_bounds(128, 32), m=e["m"], G=e["resid"], B=256, L=0)
    ix["list_off"], ix["list_ids"] = O.build_lists(e["assign"], 64)
    # stored values = FP32 rounding of the FP64 rotation within FP32 GEMM error
    ref_y = O.rotate(w["base"][:1000], e["mu"], e["R"])
    assert np.abs(e["y"][:1000] - ref_y).max() <= 1e-5 * np.abs(ref_y).max()
    # nearest-centroid assignment of the stored values (ties within FP32 error excused)
    dc = ((ix["Y"][:2000, None, :] - ix["centroids"][None]) ** 2).sum(-1)
    best = dc.min(axis=1)
    assert np.all(dc[np.arange(2000), e["assign"][:2000]] <= best * (1 + 1e-5) + 1e-9)
    ids, d, _ = g.search(w["queries"], 10, 8, 0.1)
    ora = O.search(ix, w["queries"], 10, 8, 0.1)
    _assert_ok(check_search(ids, d, ora, ix))


# ------------------------------------------------------------------------------ probe selection edges

def _probe_index(centroids, D=32, n=200, seed=0):
    """An index whose lists hold a few random vectors, for probe-selection checks."""
    from paper_2404_16322_amd import Index
    rng = np.random.default_rng(seed)
    nl = centroids.shape[0]
    y = rng.standard_normal((n, D)).astype(np.float32)
    assign = rng.integers(0, nl, size=n).astype(np.int32)
    return Index.from_artifacts(dict(mu=np.zeros(D), R=np.eye(D), centroids=centroids.astype(np.float32),
                                     assign=assign, y=y))


def _oracle_probes(q, C, nprobe):
    d = O.sq_dist_direct(C, q)
    return np.lexsort((np.arange(C.shape[0]), d))[:nprobe], d


@pytest.mark.parametrize("nl,nprobe", [(64, 8), (64, 64), (5000, 100), (5000, 4096), (300, 1),
                                       (1024, 1024), (1025, 37), (4096, 48), (4096, 4096), (3000, 129)])
def test_probe_selection_ties_and_sizes(nl, nprobe):
    rng = np.random.default_rng(nl + nprobe)
    C = rng.standard_normal((nl, 32)).astype(np.float32)
    C[10:20] = C[3]          # exact duplicates: equal distances, ordered by list id
    C[40] = C[3]
    g = _probe_index(C)
    Q = rng.standard_normal((50, 32)).astype(np.float32)
    Q[0] = C[3]              # the duplicated centroid itself: distance 0 ten times over
    _, probes = g.debug_intermediates(Q, nprobe)
    C64 = C.astype(np.float64)
    for qi in range(Q.shape[0]):
        ref, d = _oracle_probes(Q[qi].astype(np.float64), C64, nprobe)
        if probes[qi].tolist() == ref.tolist():
            continue
        # only near ties between different centroids may reorder
        ds = np.sort(d)[:nprobe + 1]
        gaps = np.abs(np.diff(ds)) / np.maximum(ds[1:], 1e-30)
        gaps = gaps[gaps > 0]
        assert gaps.size and gaps.min() < TOL, (qi, probes[qi][:12], ref[:12])
        assert sorted(probes[qi].tolist()) == sorted(set(probes[qi].tolist()))
    dup = [j for j in probes[0].tolist() if j in {3, 40} | set(range(10, 20))]
    assert dup == sorted(dup) and dup[:min(12, nprobe)] == [3, *range(10, 20), 40][:min(12, nprobe)]


@pytest.mark.parametrize("nl", [300, 4096, 5000])
def test_probe_selection_all_equal_distances(nl):
    C = np.ones((nl, 32), np.float32)
    g = _probe_index(C)
    _, probes = g.debug_intermediates(np.zeros((3, 32), np.float32), 70)
    for row in probes:
        assert row.tolist() == list(range(70))


@pytest.mark.parametrize("D,nl,nq", [(512, 4096, 2048), (768, 4096, 1100)])
def test_probe_selection_wide_gemm_tiles(D, nl, nq):
    """Coarse distances of large batches with long vectors (the 128 x 128 GEMM tile when the grid
    has at least two such tiles per compute unit, the 64 x 64 tile otherwise): the rotated
    queries and the probes match FP64."""
    rng = np.random.default_rng(D + nl)
    C = rng.standard_normal((nl, D)).astype(np.float32)
    g = _probe_index(C, D=D)
    Q = rng.standard_normal((nq, D)).astype(np.float32)
    qrot, probes = g.debug_intermediates(Q, 20)
    np.testing.assert_allclose(qrot, Q, rtol=0, atol=0)   # identity rotation, zero mean
    C64 = C.astype(np.float64)
    for qi in range(0, nq, 7):
        ref, d = _oracle_probes(Q[qi].astype(np.float64), C64, 20)
        if probes[qi].tolist() == ref.tolist():
            continue
        ds = np.sort(d)[:21]
        gaps = np.abs(np.diff(ds)) / np.maximum(ds[1:], 1e-30)
        gaps = gaps[gaps > 0]
        assert gaps.size and gaps.min() < TOL, (qi, probes[qi][:12], ref[:12])
