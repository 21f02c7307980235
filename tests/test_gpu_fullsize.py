"""Parity at the benchmark's full size and launch configuration: 1,000,000 x 128 SIFT-like
base, IVF with 4,096 lists, all 10,000 queries in one search (nprobe 48, alpha 0.05, K 10).
The oracle fits its own index (PCA on the full base, centroids = key-sampled rows with one
exact nearest-centroid pass, calibration on 200 held-out queries), the GPU imports it, and
sampled queries are compared one by one; properties that hold at any size are checked on
all 10,000."""
import numpy as np
import pytest

import oracle as O
import synthdata
from parity_util import check_search

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def full():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_2404_16322_amd import Index
    w = synthdata.make_workload("sift1m", n_calib=200, n_val=0)
    p = O.pca_fit(w["base"])
    Y = O.round_storage(O.rotate(w["base"], p["mu"], p["R"]), "f32")
    C, assign = O.kmeans(Y, 4096, iters=0, seed=2)
    C = C.astype(np.float32).astype(np.float64)
    off, ids = O.build_lists(assign, 4096)
    bounds = O.stage_bounds(128, 32)
    cal = O.calibrate(Y, off, ids, C, p["mu"], p["R"], w["calib"], bounds, calib_k=10,
                      calib_nprobe=16, B=256, L=0, seed=2, max_neg=50)
    ix = dict(mu=p["mu"], R=p["R"], Y=Y, centroids=C, assign=assign, list_off=off, list_ids=ids,
              bounds=bounds, m=cal["m"], G=cal["G"], B=256, L=0)
    g = Index.from_artifacts(dict(mu=p["mu"], R=p["R"], centroids=C.astype(np.float32),
                                  assign=assign.astype(np.int32), y=Y.astype(np.float32),
                                  m=cal["m"], resid=cal["G"]))
    return w, ix, g


@pytest.fixture(scope="module")
def sampled(full):
    w, ix, _ = full
    sample = np.random.default_rng(7).choice(w["queries"].shape[0], 64, replace=False)
    return sample, O.search(ix, w["queries"][sample], 10, 48, 0.05)


def test_full_size_sampled_queries_match_oracle(full, sampled):
    w, ix, g = full
    Q = w["queries"]
    assert Q.shape == (10_000, 128)
    ids, d, st = g.search(Q, 10, 48, 0.05)
    sample, ora = sampled
    res = check_search(ids[sample], d[sample], ora, ix)
    print(f"full size: {res['same']}/{res['nq']} identical, {res['excused']} excused")
    assert not res["bad"], res["bad"][:5]
    assert res["excused"] <= 4
    assert st["refined"] < 0.2 * st["candidates"]


def test_full_size_properties_on_every_query(full):
    w, ix, g = full
    Q = w["queries"]
    a_ids, a_d, _ = g.search(Q, 10, 48, 0.0, mode="lossless")
    n_ids, n_d, n_st = g.search(Q, 10, 48, 0.0, mode="none")
    # lossless partial-distance pruning never changes the exact result over the probed lists:
    # the K distances agree; ids may differ only by a swap of near-equal distances (the two
    # modes sum the 128 terms in different orders in FP32)
    np.testing.assert_allclose(a_d, n_d, rtol=1e-4)
    same = (a_ids == n_ids).all(axis=1)
    for qi in np.nonzero(~same)[0]:
        for j in np.nonzero(a_ids[qi] != n_ids[qi])[0]:
            assert abs(a_d[qi, j] - n_d[qi, j]) <= 1e-4 * n_d[qi, j]
    assert same.mean() > 0.99   # integer data: exact ties in the original space are common
    ids, d, _ = g.search(Q, 10, 48, 0.05)
    assert np.all(np.diff(d, axis=1) >= 0)
    assert np.all((ids >= 0) & (ids < 1_000_000))
    # returned distances are exact for the stored vectors (FP64 recomputation, 1e-4)
    qr = O.rotate(Q[:500], ix["mu"], ix["R"])
    for qi in range(500):
        ex = O.sq_dist_direct(ix["Y"][ids[qi]], qr[qi])
        np.testing.assert_allclose(d[qi], ex, rtol=1e-4)


def test_full_size_first_phase_forms_bit_identical(full, sampled):
    """The two-phase scan with its stage-1 sums from the matrix cores (expanded form, pruning on
    them only where their error bound decides the test) and from the direct first phase, and
    the one-phase scan, in the benchmark's launch configuration: ids, distances and counters
    bit-identical, and the sampled queries match the oracle."""
    w, ix, g = full
    Q = w["queries"]
    out = {}
    for name, t2, m in (("matrix", 1, 1), ("direct", 1, 0), ("one-phase", 0, 0), ("expanded", 1, 2)):
        g.set_launch(two_phase=t2, stage1_matrix=m)
        out[name] = g.search(Q, 10, 48, 0.05)
        print(f"[fullsize] {name}: launch shape {g.scan_variant(Q.shape[0], 10, 48)}", flush=True)
    g.set_launch(two_phase=-1, stage1_matrix=0)
    ids, d, st = out["matrix"]
    assert 0 < st["two_phase_sums"] <= st["candidates"]   # a query's first block runs untested
    for name in ("direct", "one-phase"):
        i2, d2, s2 = out[name]
        np.testing.assert_array_equal(ids, i2)
        np.testing.assert_array_equal(d, d2)
        for key in ("candidates", "refined", "stage_slices"):
            assert st[key] == s2[key], (name, key)
    sample, ora = sampled
    res = check_search(ids[sample], d[sample], ora, ix)
    assert not res["bad"], res["bad"][:5]
    # the expanded-form sums taken as they are: the oracle's bar, and the bit-identical form's
    # results up to FP32 rounding
    ie, de, se = out["expanded"]
    res = check_search(ie[sample], de[sample], ora, ix)
    print(f"full size, expanded sums: {res['same']}/{res['nq']} identical, {res['excused']} excused")
    assert not res["bad"], res["bad"][:5]
    assert res["excused"] <= 4
    same = (ie == ids).all(axis=1)
    assert same.mean() > 0.99
    np.testing.assert_allclose(de[same], d[same], rtol=1e-4)
