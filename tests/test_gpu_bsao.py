"""The quantization estimate with its learned correction (BSA-O, Sec. V-B) on the GPU against
the FP64 oracle: codes bit-identical, calibration, searches, launch shapes, per-query K, the
GPU fit and the index file."""
import numpy as np
import pytest

import oracle as O
from parity_util import artifacts, check_search, oracle_index, workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"


@pytest.fixture(scope="module")
def pq():
    return oracle_index(pq_m=32, n_calib=400)


@pytest.fixture(scope="module")
def pq_multi():
    return oracle_index(pq_m=16, n_calib=300, calib_k_extra=(50,))


def _index(ix, with_table=True):
    from paper_2404_16322_amd import Index
    return Index.from_artifacts(artifacts(ix, with_table))


def _ok(r, frac=0.05):
    print(f"parity: {r['same']}/{r['nq']} identical, {r['excused']} excused")
    assert not r["bad"], r["bad"][:5]
    assert r["excused"] <= frac * r["nq"] + 1


def test_codes_bit_identical_and_tables_exported(pq):
    g = _index(pq)
    inf = g.info()
    assert inf["pq_m"] == 32 and inf["pq_tables"] == 1
    e = g.export()
    np.testing.assert_array_equal(e["pq_codes"], pq["pq"]["codes"])
    np.testing.assert_array_equal(e["pq_perm"], pq["pq"]["perm"])
    t = e["tables"][0]
    assert t["pq_m1"] == pq["pq_tab"]["m1"] and t["pq_m3"] == pq["pq_tab"]["m3"]
    np.testing.assert_array_equal(t["pq_resid"], pq["pq_tab"]["G"][:, 0])
    for a in (0.0, 0.05, 0.3):
        m1, m3, b = g.correction_pq(a)
        assert (m1, m3) == (pq["pq_tab"]["m1"], pq["pq_tab"]["m3"])
        assert b == O.beta_for_alpha(pq["pq_tab"]["G"], a)[0]


@pytest.mark.parametrize("alpha", [0.05, 0.2])
@pytest.mark.parametrize("k,nprobe", [(10, 8), (1, 3), (100, 16)])
def test_bsao_search_matches_oracle(pq, alpha, k, nprobe):
    w = workload("gauss128")
    Q = np.vstack([w["queries"], w["val"][:150]])
    g = _index(pq)
    ids, d, st = g.search(Q, k, nprobe, alpha, mode="bsao")
    ora = O.search(pq, Q, k, nprobe, alpha, mode="bsao")
    _ok(check_search(ids, d, ora, pq))
    assert 0 < st["prestage_pruned"] <= st["prestage_reads"] <= st["candidates"]
    # pruned by the quantization test: close to the oracle's count (decisions differ only at ties)
    assert abs(st["prestage_pruned"] - int(ora["stops"][:, 0].sum())) <= 0.01 * st["candidates"] + 5


def test_bsao_zero_significance_is_exact(pq):
    w = workload("gauss128")
    g = _index(pq)
    a = g.search(w["queries"], 10, 8, 0.0, mode="bsao")
    n = g.search(w["queries"], 10, 8, 0.0, mode="none")
    np.testing.assert_array_equal(a[0], n[0])
    # the staged and the full-D kernels sum a distance's terms in different orders
    np.testing.assert_allclose(a[1], n[1], rtol=1e-6)
    assert a[2]["prestage_pruned"] == 0


def test_bsao_launch_variants_bitwise_identical(pq):
    w = workload("gauss128")
    g = _index(pq)
    res = []
    for wv, la, p in [(w_, l_, p_) for p_ in (0, 1) for w_ in (1, 4) for l_ in (0, 1)]:
        g.set_launch(waves_per_query=wv, lookahead=la, persistent=p)
        res.append(g.search(w["queries"], 10, 8, 0.1, mode="bsao"))
    g.set_launch(waves_per_query=0, lookahead=-1, persistent=-1)
    for r in res[1:]:
        np.testing.assert_array_equal(r[0], res[0][0])
        np.testing.assert_array_equal(r[1], res[0][1])
        assert r[2]["prestage_pruned"] == res[0][2]["prestage_pruned"]


def test_bsao_per_query_k_uses_each_querys_table(pq_multi):
    w = workload("gauss128")
    g = _index(pq_multi)
    Q = w["queries"][:100]
    rng = np.random.default_rng(6)
    ks = rng.choice([10, 30, 50, 100], Q.shape[0]).astype(np.int32)
    nps = rng.integers(3, 20, Q.shape[0]).astype(np.int32)
    ids, d, off, _ = g.search_var(Q, ks, nps, 0.1, mode="bsao")
    bad = []
    for qi in range(Q.shape[0]):
        ora = O.search(pq_multi, Q[qi:qi + 1], int(ks[qi]), int(nps[qi]), 0.1, mode="bsao")
        r = check_search(ids[off[qi]:off[qi + 1]][None], d[off[qi]:off[qi + 1]][None], ora, pq_multi)
        bad += r["bad"]
    assert not bad, bad[:5]


def test_gpu_calibration_of_the_bsao_classifier_equals_oracle(pq_multi):
    w = workload("gauss128", n_calib=300)
    g = _index(pq_multi, with_table=False)
    g.calibrate(w["calib"], calib_k=10, calib_nprobe=8, max_neg=50, seed=7)
    g.calibrate(w["calib"], calib_k=0, calib_nprobe=8, max_neg=50, seed=7)   # no-op without tables
    # tables at K_c = 10 only (calib_k = 10): compare with the oracle's first table
    t = pq_multi["tables"][0]["pq"]
    m1, m3, b = g.correction_pq(0.05, k=10)
    np.testing.assert_allclose([m1, m3], [t["m1"], t["m3"]], rtol=1e-6)
    ref = O.beta_for_alpha(t["G"], 0.05)[0]
    np.testing.assert_allclose(b, ref, rtol=1e-6, atol=1e-9 * abs(ref))


def test_gpu_fit_with_quantizer_encodes_its_own_codebooks():
    """GPU-fitted codebooks: the GPU's codes are exactly the FP32 nearest codewords of its
    exported codebooks, and a BSA-O search of the GPU index matches the oracle on the
    exported artifacts."""
    from paper_2404_16322_amd import Index
    w = workload("gauss128")
    g = Index.fit(w["base"], w["calib"][:400], nlist=64, seed=7, calib_nprobe=8, pq_m=32, pq_iters=8)
    inf = g.info()
    assert inf["pq_m"] == 32 and inf["pq_tables"] == 1
    e = g.export()
    Y = e["y"].astype(np.float64)
    perm = e["pq_perm"].astype(np.int64)
    books = e["pq_books"].astype(np.float64)
    np.testing.assert_array_equal(e["pq_codes"], O.pq_encode(Y, perm, books))
    assert sorted(perm.reshape(-1).tolist()) == list(range(128))
    np.testing.assert_array_equal(perm, O.opq_allocation(e["lam"], 32))
    # oracle index on the exported artifacts
    ix = dict(mu=e["mu"], R=e["R"], Y=Y, centroids=e["centroids"].astype(np.float64), B=256, L=0,
              bounds=O.stage_bounds(128, 32), m=e["m"], G=e["resid"], lam=e["lam"])
    ix["list_off"], ix["list_ids"] = O.build_lists(e["assign"], 64)
    codes = e["pq_codes"]
    ix["pq"] = dict(perm=perm, books=books, codes=codes, err=O.pq_error(Y, perm, books, codes))
    t = e["tables"][0]
    ix["pq_tab"] = dict(m1=t["pq_m1"], m3=t["pq_m3"], G=t["pq_resid"][:, None])
    Q = w["queries"]
    ids, d, _ = g.search(Q, 10, 8, 0.1, mode="bsao")
    _ok(check_search(ids, d, O.search(ix, Q, 10, 8, 0.1, mode="bsao"), ix))


def test_bsao_index_file_round_trip(pq, tmp_path):
    from paper_2404_16322_amd import Index
    w = workload("gauss128")
    g = _index(pq)
    path = str(tmp_path / "pq.ddc")
    g.save(path)
    h = Index.load(path)
    assert h.info() == g.info()
    a, b = g.export(), h.export()
    for key in ("pq_perm", "pq_books", "pq_codes"):
        np.testing.assert_array_equal(a[key], b[key])
    np.testing.assert_array_equal(a["tables"][0]["pq_resid"], b["tables"][0]["pq_resid"])
    r1, r2 = g.search(w["queries"], 10, 8, 0.1, mode="bsao"), h.search(w["queries"], 10, 8, 0.1, mode="bsao")
    np.testing.assert_array_equal(r1[0], r2[0])
    np.testing.assert_array_equal(r1[1], r2[1])


def test_bsao_rejected_without_quantizer():
    from paper_2404_16322_amd.binding import DdcError
    ix = oracle_index()
    g = _index(ix)
    with pytest.raises(DdcError, match="BSA-O"):
        g.search(workload("gauss128")["queries"][:2], 10, 8, 0.1, mode="bsao")
