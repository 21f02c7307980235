"""Threshold lag L > 0 on the GPU.  The refinement of Sec. I keeps a result queue whose K-th
distance tau is the pruning threshold; read for block-synchronous hardware, the candidates of
block b are tested against the tau in force after block b - 1 - L (+inf before it exists),
while the merge stays exact against the current queue.  The GPU search and the GPU
calibration (label-1 pool of Sec. V-B) follow that schedule; both are compared with the
oracle on the same artifacts, and every launch shape returns bit-identical results."""
import numpy as np
import pytest

import oracle as O
from parity_util import artifacts, check_search, oracle_index, workload

pytestmark = pytest.mark.gpu

VARIANTS = [(w, la, p, t) for t in (0, 1) for p in (0, 1) for w in (1, 2, 4) for la in (0, 1)]


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"


def _index(ix, with_table=True):
    from paper_2404_16322_amd import Index
    return Index.from_artifacts(artifacts(ix, with_table))


def _all_variants(g, run):
    out = []
    for w, la, p, t in VARIANTS:
        g.set_launch(waves_per_query=w, lookahead=la, persistent=p, two_phase=t)
        out.append(run())
    g.set_launch(waves_per_query=0, lookahead=-1, persistent=-1, two_phase=-1)
    return out


@pytest.mark.parametrize("L", [1, 3])
@pytest.mark.parametrize("storage,fp8", [("f32", 0), ("bf16", 0), ("f32", 64)])
def test_lagged_search_matches_oracle_in_every_launch_shape(L, storage, fp8):
    # B = 64: a 64-list index of 20k vectors gives ~5 blocks per list, so lags of 1 and 3
    # change which tau a block sees
    ix = oracle_index(storage=storage, B=64, L=L, n_calib=300, fp8_lead=fp8)
    assert ix["L"] == L and ix["B"] == 64
    w = workload("gauss128")
    g = _index(ix)
    assert g.info()["lag_l"] == L
    Q = w["queries"]
    res = _all_variants(g, lambda: g.search(Q, 10, 8, 0.1))
    for r in res[1:]:
        np.testing.assert_array_equal(res[0][0], r[0])
        np.testing.assert_array_equal(res[0][1], r[1])
        assert r[2]["candidates"] == res[0][2]["candidates"]
        assert r[2]["refined"] == res[0][2]["refined"]
    ids, d, st = res[0]
    ora = O.search(ix, Q, 10, 8, 0.1)
    r = check_search(ids, d, ora, ix)
    print(f"L={L} {storage} fp8={fp8}: {r['same']}/{r['nq']} identical, {r['excused']} excused")
    assert not r["bad"], r["bad"][:5]
    assert r["excused"] <= 0.05 * r["nq"] + 1
    assert st["candidates"] == int(ora["stops"].sum())
    assert abs(st["refined"] - int(ora["stops"][:, -1].sum())) <= 0.01 * st["candidates"] + 5


def test_lossless_lag_prunes_no_more_than_no_lag():
    """With the lossless test (partial distance > tau) every queue is the exact top-K of the
    candidates merged so far, and tau only shrinks as candidates join (Sec. I), so the tau a
    lagged block sees is never below the L = 0 one: the lagged scan refines at least as many
    candidates and returns the same distances."""
    ix0 = oracle_index(B=64, L=0, n_calib=300)
    ix3 = dict(ix0)
    ix3["L"] = 3
    w = workload("gauss128")
    g0, g3 = _index(ix0), _index(ix3)
    _, e0, s0 = g0.search(w["queries"], 10, 8, 0.0, mode="lossless")
    _, e3, s3 = g3.search(w["queries"], 10, 8, 0.0, mode="lossless")
    assert s3["candidates"] == s0["candidates"]
    assert s0["refined"] <= s3["refined"] < s3["candidates"]
    np.testing.assert_allclose(e0, e3, rtol=1e-5)


def test_lag_beyond_every_list_refines_everything():
    """L larger than any query's block count: no block ever sees a finite threshold."""
    ix = dict(oracle_index(B=64, L=0, n_calib=300))
    ix["L"] = 64
    w = workload("gauss128")
    g = _index(ix)
    _, _, st = g.search(w["queries"], 10, 8, 0.1)
    assert st["refined"] == st["candidates"]


@pytest.mark.parametrize("L", [1, 3])
def test_gpu_calibration_with_lag_equals_oracle(L):
    """The GPU calibration replays the lagged schedule: its label-1 pool and therefore
    m_s and beta_s(alpha) equal the oracle's fit with the same B and L."""
    ix = oracle_index(B=64, L=L, n_calib=300)
    w = workload("gauss128", n_calib=300)
    g = _index(ix, with_table=False)
    g.calibrate(w["calib"], calib_k=10, calib_nprobe=8, max_neg=50, seed=7)
    assert g.info()["n0"] == ix["G"].shape[0]
    for a in [0.01, 0.1]:
        m, b = g.correction(a)
        np.testing.assert_allclose(m, ix["m"], rtol=1e-6)
        ref = O.beta_for_alpha(ix["G"], a)
        np.testing.assert_allclose(b, ref, rtol=1e-6, atol=1e-9 * np.abs(ref).max())


def test_lagged_residual_test_matches_oracle():
    """The residual-estimate test (Alg. 2, incremental) under a lagged threshold, in every
    launch shape that runs it."""
    ix = oracle_index(B=64, L=2, n_calib=300)
    w = workload("gauss128")
    g = _index(ix)
    g.set_bsar_multiplier(3.0)
    Q = w["queries"]
    res = []
    for wv in (1, 2, 4):
        for p in (0, 1):
            g.set_launch(waves_per_query=wv, lookahead=0, persistent=p)
            res.append(g.search(Q, 10, 8, 0.0, mode="bsar"))
    g.set_launch(waves_per_query=0, lookahead=-1, persistent=-1)
    for r in res[1:]:
        np.testing.assert_array_equal(res[0][0], r[0])
        np.testing.assert_array_equal(res[0][1], r[1])
    ids, d, st = res[0]
    ora = O.search(dict(ix, bsar_m=3.0), Q, 10, 8, 0.0, mode="bsar")
    r = check_search(ids, d, ora, ix)
    assert not r["bad"], r["bad"][:5]
    assert r["excused"] <= 0.05 * r["nq"] + 1
    assert st["candidates"] == int(ora["stops"].sum())
    assert abs(st["refined"] - int(ora["stops"][:, -1].sum())) <= 0.01 * st["candidates"] + 5


def test_lagged_quantization_test_matches_oracle():
    """BSA-O's quantization test before the refinement, under a lagged threshold, in every
    launch shape."""
    ix = oracle_index(B=64, L=2, pq_m=32, n_calib=400)
    w = workload("gauss128")
    g = _index(ix)
    Q = w["queries"]
    res = _all_variants(g, lambda: g.search(Q, 10, 8, 0.1, mode="bsao"))
    for r in res[1:]:
        np.testing.assert_array_equal(res[0][0], r[0])
        np.testing.assert_array_equal(res[0][1], r[1])
        assert r[2]["prestage_pruned"] == res[0][2]["prestage_pruned"]
    ids, d, st = res[0]
    ora = O.search(ix, Q, 10, 8, 0.1, mode="bsao")
    r = check_search(ids, d, ora, ix)
    assert not r["bad"], r["bad"][:5]
    assert r["excused"] <= 0.05 * r["nq"] + 1
    assert 0 < st["prestage_pruned"]
    assert abs(st["prestage_pruned"] - int(ora["stops"][:, 0].sum())) <= 0.01 * st["candidates"] + 5
