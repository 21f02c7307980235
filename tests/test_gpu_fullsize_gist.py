"""Parity at the 960-d configuration's full size and launch configuration: 1,000,000 x 960
GIST-shaped base stored in BF16, IVF with 4,096 lists, queries rotated on the BF16 matrix
cores, all 1,000 queries in one search at K = 100, nprobe 64, alpha 0.3, in the launch shape
the tuner picks.  The oracle fits its own index (PCA on the full base, BF16 storage rounding,
centroids = key-sampled rows with one exact nearest-centroid pass, a K_c = 100 correction
table from 200 held-out queries), the GPU imports it, and sampled queries are compared one by
one with the oracle searching from its BF16 rotation reading."""
import numpy as np
import pytest

import oracle as O
import synthdata
from parity_util import check_search

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def full_gist():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_2404_16322_amd import Index
    print("[fullsize-gist] oracle fit of 1M x 960", flush=True)
    w = synthdata.make_workload("gist1m", n_calib=200, n_val=0)
    p = O.pca_fit(w["base"])
    Y = O.round_storage(O.rotate(w["base"], p["mu"], p["R"]), "bf16")
    C, assign = O.kmeans(Y, 4096, iters=0, seed=2)
    C = C.astype(np.float32).astype(np.float64)
    off, ids = O.build_lists(assign, 4096)
    bounds = O.stage_bounds(960, 32)
    cal = O.calibrate(Y, off, ids, C, p["mu"], p["R"], w["calib"], bounds, calib_k=100,
                      calib_nprobe=16, B=256, L=0, seed=2, max_neg=50)
    ix = dict(mu=p["mu"], R=p["R"], Y=Y, centroids=C, assign=assign, list_off=off, list_ids=ids,
              bounds=bounds, m=cal["m"], G=cal["G"], B=256, L=0, rotation="bf16", storage="bf16")
    print("[fullsize-gist] GPU import", flush=True)
    g = Index.from_artifacts(dict(mu=p["mu"], R=p["R"], centroids=C.astype(np.float32),
                                  assign=assign.astype(np.int32), y=Y.astype(np.float32),
                                  m=cal["m"], resid=cal["G"], storage="bf16", rotation="bf16"))
    return w, ix, g


def test_full_size_960d_sampled_queries_match_oracle(full_gist):
    w, ix, g = full_gist
    Q = w["queries"]
    assert Q.shape == (1_000, 960)
    ids, d, st = g.search(Q, 100, 64, 0.3)
    print(f"[fullsize-gist] launch shape {g.scan_variant(Q.shape[0], 100, 64)}", flush=True)
    sample = np.random.default_rng(7).choice(Q.shape[0], 24, replace=False)
    ora = O.search(ix, Q[sample], 100, 64, 0.3)
    res = check_search(ids[sample], d[sample], ora, ix)
    print(f"full size 960-d: {res['same']}/{res['nq']} identical, {res['excused']} excused")
    assert not res["bad"], res["bad"][:5]
    assert res["excused"] <= 2
    assert st["refined"] < 0.1 * st["candidates"]
    # at any size: ascending, valid ids, every distance exact for the stored vector it names
    assert np.all(np.diff(d, axis=1) >= 0)
    assert np.all((ids >= 0) & (ids < 1_000_000))
    qr = O.rotate_bf16(Q[:64], ix["mu"], ix["R"])
    for qi in range(64):
        np.testing.assert_allclose(d[qi], O.sq_dist_direct(ix["Y"][ids[qi]], qr[qi]), rtol=1e-4)
