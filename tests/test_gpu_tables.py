"""Correction tables per calibration K_c (a search with K uses the largest K_c <= K) and the
index file: GPU vs oracle parity, GPU recalibration of every table, save/load round trip."""
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
def multi():
    w = workload("gauss128")
    ix = O.fit(w["base"], w["calib"], nlist=64, kmeans_iters=25, calib_k=10, calib_nprobe=8,
               seed=7, calib_k_extra=(50,), fp8_lead=64)
    ix["centroids"] = ix["centroids"].astype(np.float32).astype(np.float64)
    return w, ix


def _index(ix, with_table=True):
    from paper_2404_16322_amd import Index
    return Index.from_artifacts(artifacts(ix, with_table))


def _ok(r):
    print(f"parity: {r['same']}/{r['nq']} identical, {r['excused']} excused")
    assert not r["bad"], r["bad"][:5]
    assert r["excused"] <= 0.05 * r["nq"] + 1


def test_tables_exported_and_selected_by_k(multi):
    w, ix = multi
    g = _index(ix)
    inf = g.info()
    assert inf["n_tables"] == 2 and inf["table_k"] == [10, 50]
    e = g.export()
    for t, te in zip(ix["tables"], e["tables"]):
        assert te["kc"] == t["kc"]
        np.testing.assert_array_equal(te["m"], t["m"])
        np.testing.assert_array_equal(te["resid"], t["G"])
    for k, want in [(1, 0), (10, 0), (49, 0), (50, 1), (100, 1)]:
        m, b = g.correction(0.1, k=k)
        np.testing.assert_array_equal(m, ix["tables"][want]["m"])
        np.testing.assert_array_equal(b, O.beta_for_alpha(ix["tables"][want]["G"], 0.1))


@pytest.mark.parametrize("k", [10, 50, 100])
def test_search_uses_the_table_of_its_k(multi, k):
    w, ix = multi
    g = _index(ix)
    Q = np.vstack([w["queries"], w["val"][:200]])
    ids, d, _ = g.search(Q, k, 12, 0.1)
    ora = O.search(ix, Q, k, 12, 0.1)
    _ok(check_search(ids, d, ora, ix))


def test_mixed_k_per_query_uses_each_querys_table(multi):
    w, ix = multi
    g = _index(ix)
    Q = w["queries"][:120]
    rng = np.random.default_rng(4)
    ks = rng.choice([10, 30, 50, 100], Q.shape[0]).astype(np.int32)
    nps = rng.integers(4, 20, Q.shape[0]).astype(np.int32)
    ids, d, off, _ = g.search_var(Q, ks, nps, 0.1)
    for qi in range(Q.shape[0]):
        ora = O.search(ix, Q[qi:qi + 1], int(ks[qi]), int(nps[qi]), 0.1)
        r = check_search(ids[off[qi]:off[qi + 1]][None], d[off[qi]:off[qi + 1]][None], ora, ix)
        assert not r["bad"], (qi, r["bad"])


def test_gpu_recalibrates_every_table(multi):
    w, ix = multi
    g = _index(ix)
    g.calibrate(w["calib"], calib_k=0, calib_nprobe=8, max_neg=50, seed=7)
    for t, k in zip(ix["tables"], (10, 50)):
        m, b = g.correction(0.05, k=k)
        np.testing.assert_allclose(m, t["m"], rtol=1e-6)
        ref = O.beta_for_alpha(t["G"], 0.05)
        np.testing.assert_allclose(b, ref, rtol=1e-6, atol=1e-9 * np.abs(ref).max())


def test_save_load_round_trip(multi, tmp_path):
    from paper_2404_16322_amd import Index
    w, ix = multi
    g = _index(ix)
    path = str(tmp_path / "index.ddc")
    g.save(path)
    h = Index.load(path)
    assert h.info() == g.info()
    a, b = g.export(), h.export()
    for key in ("mu", "R", "centroids", "assign", "y", "m", "resid", "codes8", "scale8"):
        np.testing.assert_array_equal(a[key], b[key])
    for k in (10, 100):
        r1, r2 = g.search(w["queries"], k, 8, 0.1), h.search(w["queries"], k, 8, 0.1)
        np.testing.assert_array_equal(r1[0], r2[0])
        np.testing.assert_array_equal(r1[1], r2[1])
    # a damaged file is refused
    raw = bytearray(open(path, "rb").read())
    raw[len(raw) // 2] ^= 0xFF
    open(path, "wb").write(bytes(raw))
    with pytest.raises(Exception, match="checksum"):
        Index.load(path)
