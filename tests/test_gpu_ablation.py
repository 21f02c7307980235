"""Random-rotation ablation on the GPU: the Haar rotation of the fit equals the oracle's, and
the ADSampling test (DDC_CORR_ADS) matches the oracle's decisions."""
import numpy as np
import pytest

import oracle as O
from parity_util import artifacts, check_search, workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"


@pytest.fixture(scope="module")
def haar_oracle():
    w = workload("gauss128")
    ix = O.fit(w["base"], w["calib"], nlist=64, kmeans_iters=25, calib_k=10, calib_nprobe=8,
               seed=7, projection="haar")
    ix["centroids"] = ix["centroids"].astype(np.float32).astype(np.float64)
    return w, ix


def _ok(r):
    print(f"parity: {r['same']}/{r['nq']} identical, {r['excused']} excused")
    assert not r["bad"], r["bad"][:5]
    assert r["excused"] <= 0.05 * r["nq"] + 1


def test_gpu_fit_haar_rotation_equals_oracle():
    from paper_2404_16322_amd import Index
    w = workload("gauss128")
    g = Index.fit(w["base"], w["calib"], nlist=64, kmeans_iters=5, calib_k=10, calib_nprobe=8,
                  seed=7, projection="haar")
    e = g.export()
    Rh = O.haar_rotation(128, 7)
    assert np.abs(e["R"] - Rh).max() < 1e-12
    p = O.pca_fit(w["base"])
    np.testing.assert_allclose(e["lam"], np.einsum("ij,jk,ik->i", Rh, p["cov"], Rh), rtol=1e-9)
    # the GPU-fitted index searched against the oracle on its exported artifacts
    ix = dict(mu=e["mu"], R=e["R"], Y=e["y"].astype(np.float64), centroids=e["centroids"].astype(np.float64),
              assign=e["assign"], bounds=O.stage_bounds(128, 32), m=e["m"], G=e["resid"], B=256, L=0)
    ix["list_off"], ix["list_ids"] = O.build_lists(e["assign"], 64)
    ids, d, _ = g.search(w["queries"], 10, 8, 0.1)
    _ok(check_search(ids, d, O.search(ix, w["queries"], 10, 8, 0.1), ix))


@pytest.mark.parametrize("eps0", [1.0, 2.1, 4.0])
def test_ads_mode_matches_oracle(haar_oracle, eps0):
    from paper_2404_16322_amd import Index
    w, ix = haar_oracle
    g = Index.from_artifacts(artifacts(ix))
    g.set_ads_epsilon(eps0)
    Q = np.vstack([w["queries"], w["val"][:200]])
    ids, d, st = g.search(Q, 10, 8, 0.0, mode="ads")
    ora = O.search(dict(ix, ads_eps0=eps0), Q, 10, 8, 0.0, mode="ads")
    _ok(check_search(ids, d, ora, ix))
    assert st["candidates"] == int(ora["stops"].sum())
    assert abs(st["refined"] - int(ora["stops"][:, -1].sum())) <= 0.01 * st["candidates"] + 5


def test_ads_with_huge_eps_is_the_full_scan(haar_oracle):
    from paper_2404_16322_amd import Index
    w, ix = haar_oracle
    g = Index.from_artifacts(artifacts(ix))
    g.set_ads_epsilon(1e6)
    a = g.search(w["queries"], 10, 8, 0.0, mode="ads")
    n = g.search(w["queries"], 10, 8, 0.0, mode="none")
    np.testing.assert_array_equal(a[0], n[0])
    assert a[2]["refined"] == a[2]["candidates"]


# ------------------------------------------------------------------ residual estimate (Alg. 1/2)

@pytest.mark.parametrize("storage", ["f32", "f16"])
@pytest.mark.parametrize("m,alpha", [(8.0, 0.0), (3.0, 0.0), (0.0, 0.05), (0.0, 0.2)])
def test_residual_test_matches_oracle(storage, m, alpha):
    from paper_2404_16322_amd import Index
    from parity_util import oracle_index
    ix = oracle_index(storage=storage, n_calib=300)
    w = workload("gauss128")
    g = Index.from_artifacts(artifacts(ix))
    g.set_bsar_multiplier(m)
    Q = np.vstack([w["queries"], w["val"][:200]])
    ids, d, st = g.search(Q, 10, 8, alpha, mode="bsar")
    ora = O.search(dict(ix, bsar_m=m), Q, 10, 8, alpha, mode="bsar")
    _ok(check_search(ids, d, ora, ix))
    assert st["candidates"] == int(ora["stops"].sum())
    assert abs(st["refined"] - int(ora["stops"][:, -1].sum())) <= 0.01 * st["candidates"] + 5
    assert st["refined"] < st["candidates"]


def test_residual_test_variants_identical_and_huge_m_is_exact():
    from paper_2404_16322_amd import Index
    from parity_util import oracle_index
    ix = oracle_index()
    w = workload("gauss128")
    g = Index.from_artifacts(artifacts(ix))
    g.set_bsar_multiplier(4.0)
    res = []
    for wv in (1, 4):
        for p in (0, 1):
            # look-ahead does not apply to this test
            g.set_launch(waves_per_query=wv, lookahead=1, persistent=p)
            res.append(g.search(w["queries"], 10, 8, 0.0, mode="bsar"))
    for r in res[1:]:
        np.testing.assert_array_equal(res[0][0], r[0])
        np.testing.assert_array_equal(res[0][1], r[1])
    g.set_launch(waves_per_query=0, lookahead=-1, persistent=-1)
    g.set_bsar_multiplier(1e12)
    a = g.search(w["queries"], 10, 8, 0.0, mode="bsar")
    n = g.search(w["queries"], 10, 8, 0.0, mode="none")
    np.testing.assert_array_equal(a[0], n[0])
    assert a[2]["refined"] == a[2]["candidates"]
