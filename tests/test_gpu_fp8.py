"""FP8 E4M3 pre-stage over the leading 64 rotated dims: codes and scales bit-identical to the
oracle's, searches and calibration in parity with the oracle, every launch variant
bit-identical, LOSSLESS unaffected."""
import numpy as np
import pytest

import oracle as O
from parity_util import artifacts, check_search, oracle_index, workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"


def _index(ix, with_table=True):
    from paper_2404_16322_amd import Index
    return Index.from_artifacts(artifacts(ix, with_table))


def _ok(r, frac=0.05):
    print(f"fp8 parity: {r['same']}/{r['nq']} identical, {r['excused']} excused")
    assert not r["bad"], r["bad"][:5]
    assert r["excused"] <= frac * r["nq"] + 1


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_codes_and_scales_bit_identical(storage):
    ix = oracle_index(storage=storage, n_calib=300, fp8_lead=64)
    g = _index(ix)
    assert g.info()["fp8_lead_dims"] == 64
    e = g.export()
    np.testing.assert_array_equal(e["codes8"], ix["pre"]["codes"])
    np.testing.assert_array_equal(e["scale8"], ix["pre"]["scale"])
    np.testing.assert_array_equal(e["m"], ix["m"])


@pytest.mark.parametrize("storage", ["f32", "f16"])
@pytest.mark.parametrize("k,nprobe,alpha", [(10, 8, 0.05), (10, 8, 0.2), (100, 16, 0.1), (1, 3, 0.1)])
def test_search_with_prestage_matches_oracle(storage, k, nprobe, alpha):
    ix = oracle_index(storage=storage, n_calib=300, fp8_lead=64)
    w = workload("gauss128")
    Q = np.vstack([w["queries"], w["val"][:200]])
    g = _index(ix)
    ids, d, st = g.search(Q, k, nprobe, alpha)
    ora = O.search(ix, Q, k, nprobe, alpha)
    _ok(check_search(ids, d, ora, ix))
    assert st["candidates"] == int(ora["stops"].sum())
    pre_ora = int(ora["stops"][:, 0].sum())
    assert st["prestage_pruned"] > 0
    assert abs(st["prestage_pruned"] - pre_ora) <= 0.01 * st["candidates"] + 5
    assert st["prestage_pruned"] + sum(st["stage_stop"]) == st["candidates"]


def test_lossless_and_none_ignore_the_prestage():
    ix = oracle_index(n_calib=300, fp8_lead=64)
    w = workload("gauss128")
    g = _index(ix)
    for mode in ("lossless", "none"):
        ids, d, st = g.search(w["queries"], 10, 8, 0.0, mode=mode)
        ora = O.search(ix, w["queries"], 10, 8, 0.0, mode="none")
        _ok(check_search(ids, d, ora, ix), 0.02)
        assert st["prestage_reads"] == 0


def test_prestage_variants_bitwise_identical():
    ix = oracle_index(storage="f16", n_calib=300, fp8_lead=64)
    w = workload("gauss128")
    g = _index(ix)
    res = []
    for wv, la, p, t in [(w_, l_, p_, t_) for t_ in (0, 1) for p_ in (0, 1) for w_ in (1, 4) for l_ in (0, 1)]:
        g.set_launch(waves_per_query=wv, lookahead=la, persistent=p, two_phase=t)
        res.append(g.search(w["queries"], 10, 8, 0.1))
    g.set_launch(waves_per_query=0, lookahead=-1, persistent=-1, two_phase=-1)
    for r in res[1:]:
        np.testing.assert_array_equal(r[0], res[0][0])
        np.testing.assert_array_equal(r[1], res[0][1])
        for key in ("prestage_reads", "prestage_pruned", "candidates", "refined", "stage_slices"):
            assert r[2][key] == res[0][2][key], key
    # the two-phase launches took every pre-stage sum from the first phase
    assert res[-1][2]["two_phase_sums"] == res[-1][2]["prestage_reads"] > 0
    assert res[0][2]["two_phase_sums"] == 0


def test_gpu_calibration_with_prestage_equals_oracle():
    ix = oracle_index(n_calib=300, fp8_lead=64)
    w = workload("gauss128", n_calib=300)
    g = _index(ix, with_table=False)
    g.calibrate(w["calib"], calib_k=10, calib_nprobe=8, max_neg=50, seed=7)
    assert g.info()["n_test_stages"] == ix["m"].shape[0] == ix["bounds"].shape[0]
    for a in [0.01, 0.1]:
        m, b = g.correction(a)
        np.testing.assert_allclose(m, ix["m"], rtol=1e-6)
        ref = O.beta_for_alpha(ix["G"], a)
        np.testing.assert_allclose(b, ref, rtol=1e-6, atol=1e-9 * np.abs(ref).max())


def test_gpu_fit_with_prestage():
    from paper_2404_16322_amd import Index
    w = workload("gauss128")
    g = Index.fit(w["base"], w["calib"], nlist=64, kmeans_iters=10, calib_k=10, calib_nprobe=8,
                  seed=7, storage="f16", fp8_lead_dims=64)
    e = g.export()
    off, lids = O.build_lists(e["assign"], 64)
    pre = O.fp8_encode_lead(e["y"].astype(np.float64), off, lids, 64)
    np.testing.assert_array_equal(e["codes8"], pre["codes"])
    np.testing.assert_array_equal(e["scale8"], pre["scale"])
    ix = dict(mu=e["mu"], R=e["R"], Y=e["y"].astype(np.float64),
              centroids=e["centroids"].astype(np.float64), assign=e["assign"], list_off=off,
              list_ids=lids, bounds=O.stage_bounds(128, 32), m=e["m"], G=e["resid"], B=256, L=0,
              pre=pre)
    ids, d, st = g.search(w["queries"], 10, 8, 0.1)
    ora = O.search(ix, w["queries"], 10, 8, 0.1)
    _ok(check_search(ids, d, ora, ix))
    assert st["prestage_pruned"] > 0
