"""Lag-parallel scan on the GPU.  With a threshold lag L (candidates of block b tested against
the tau after block b - 1 - L) of at least W - 1 blocks, every block of a group of W consecutive
blocks sees a tau that is known before the group starts.  W = 2 (L >= 1) or 4 (L >= 3)
wavefronts of a workgroup then scan the W blocks of a group at once and merge their survivors
into the queue in block order; the merge is exact, so results and every work counter must equal
those of the one-wavefront lagged scan bit for bit, and both match the oracle run with the same
B and L."""
import numpy as np
import pytest

import oracle as O
from parity_util import artifacts, check_search, oracle_index, workload

pytestmark = pytest.mark.gpu

ONE_WAVE = [(1, la, p, t) for t in (0, 1) for p in (0, 1) for la in (0, 1)]
# two waves per query: lag-parallel from L = 1; four: lag-parallel from L = 3 (below that the
# four waves split each block's tiles, which equals the one-wave scan as well)
LAG_PARALLEL = [(w, la, p, t) for w in (2, 4) for t in (0, 1) for p in (0, 1) for la in (0, 1)]


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"


def _index(ix):
    from paper_2404_16322_amd import Index
    return Index.from_artifacts(artifacts(ix))


def _run(g, shapes, run):
    out = []
    for w, la, p, t in shapes:
        g.set_launch(waves_per_query=w, lookahead=la, persistent=p, two_phase=t)
        out.append(run())
    g.set_launch(waves_per_query=0, lookahead=-1, persistent=-1, two_phase=-1)
    return out


def _assert_same(ref, other):
    for a, b in zip(ref, other):
        if isinstance(a, np.ndarray):
            np.testing.assert_array_equal(a, b)
        elif isinstance(a, dict):
            for key in a:
                if key in ("two_phase_sums", "two_phase_slices"):
                    continue   # these depend on the two-phase choice, compared per choice below
                assert a[key] == b[key], key


@pytest.mark.parametrize("L", [1, 2, 3, 4, 7])
@pytest.mark.parametrize("storage,mode,alpha", [("f32", "learned", 0.1), ("bf16", "learned", 0.1),
                                                ("f32", "lossless", 0.0)])
def test_lag_parallel_equals_one_wave_scan(L, storage, mode, alpha):
    # B = 64 over 64 lists of ~312 vectors: ~5 blocks per list, so queries end on every
    # position of a group of four (incomplete last groups included) and the lag matters
    ix = oracle_index(storage=storage, B=64, L=L, n_calib=300)
    w = workload("gauss128")
    g = _index(ix)
    Q = w["queries"][:160]
    rng = np.random.default_rng(11 + L)
    ks = rng.integers(1, 100, Q.shape[0]).astype(np.int32)
    nps = rng.integers(1, 24, Q.shape[0]).astype(np.int32)
    run = lambda: g.search_var(Q, ks, nps, alpha, mode=mode)
    ref = _run(g, ONE_WAVE, run)
    lp = _run(g, LAG_PARALLEL, run)
    for r in ref[1:] + lp:
        _assert_same(ref[0], r)
    for i in range(len(lp)):
        # same two-phase choice: the two-phase counters agree too
        assert lp[i][3]["two_phase_sums"] == ref[i % len(ref)][3]["two_phase_sums"]
    ids, d, off, st = lp[0]
    for qi in range(0, Q.shape[0], 8):   # every 8th query against the oracle, one at a time
        ora = O.search(ix, Q[qi:qi + 1], int(ks[qi]), int(nps[qi]), alpha, mode=mode)
        r = check_search(ids[off[qi]:off[qi + 1]][None], d[off[qi]:off[qi + 1]][None], ora, ix)
        assert not r["bad"], (qi, r["bad"])


@pytest.mark.parametrize("L,W", [(1, 2), (2, 2), (3, 4), (5, 4), (5, 2)])
def test_lag_parallel_matches_oracle_d128(L, W):
    ix = oracle_index(B=64, L=L, n_calib=300)
    w = workload("gauss128")
    g = _index(ix)
    Q = w["queries"]
    g.set_launch(waves_per_query=W, lookahead=1, persistent=0, two_phase=0)
    ids, d, st = g.search(Q, 10, 8, 0.1)
    g.set_launch(waves_per_query=0, lookahead=-1, persistent=-1, two_phase=-1)
    ora = O.search(ix, Q, 10, 8, 0.1)
    r = check_search(ids, d, ora, ix)
    print(f"L={L} W={W}: {r['same']}/{r['nq']} identical, {r['excused']} excused")
    assert not r["bad"], r["bad"][:5]
    assert r["excused"] <= 0.05 * r["nq"] + 1
    assert st["candidates"] == int(ora["stops"].sum())
    assert abs(st["refined"] - int(ora["stops"][:, -1].sum())) <= 0.01 * st["candidates"] + 5


@pytest.fixture(scope="module")
def wide_lag3():
    # 960-d, the 256-vector blocks of the full-size configurations, L = 3
    w = workload("gist1m", n=16000, nq=96, n_calib=200, n_val=0)
    ix = O.fit(w["base"], w["calib"], nlist=16, delta_d=32, storage="bf16", kmeans_iters=8,
               calib_k=10, calib_nprobe=6, B=256, L=3, seed=7)
    ix["centroids"] = ix["centroids"].astype(np.float32).astype(np.float64)
    return w, ix


@pytest.mark.parametrize("k,nprobe", [(10, 6), (100, 4)])
def test_lag_parallel_d960_block256(wide_lag3, k, nprobe):
    w, ix = wide_lag3
    g = _index(ix)
    Q = w["queries"]
    run = lambda: g.search(Q, k, nprobe, 0.1)
    ref = _run(g, ONE_WAVE[:2], run)
    lp = _run(g, LAG_PARALLEL, run)
    for r in ref[1:] + lp:
        _assert_same(ref[0], r)
    ora = O.search(ix, Q, k, nprobe, 0.1)
    r = check_search(lp[0][0], lp[0][1], ora, ix)
    print(f"d960 L=3: {r['same']}/{r['nq']} identical, {r['excused']} excused")
    assert not r["bad"], r["bad"][:5]
    assert r["excused"] <= 0.05 * r["nq"] + 1


def test_lag_parallel_residual_and_quantization_tests():
    """The residual-estimate test (Alg. 2) and BSA-O's quantization test under the
    lag-parallel schedule equal their one-wavefront scans."""
    ix = oracle_index(B=64, L=3, pq_m=32, n_calib=400)
    w = workload("gauss128")
    g = _index(ix)
    Q = w["queries"]
    run = lambda: g.search(Q, 10, 8, 0.1, mode="bsao")
    ref = _run(g, [(1, 0, 0, 0), (1, 1, 1, 0)], run)
    lp = _run(g, [(4, 0, 0, 0), (4, 1, 1, 0), (2, 0, 0, 0), (2, 1, 1, 0)], run)
    for r in ref[1:] + lp:
        _assert_same(ref[0], r)
    ora = O.search(ix, Q, 10, 8, 0.1, mode="bsao")
    r = check_search(lp[0][0], lp[0][1], ora, ix)
    assert not r["bad"], r["bad"][:5]
    g.set_bsar_multiplier(3.0)
    run = lambda: g.search(Q, 10, 8, 0.0, mode="bsar")
    ref = _run(g, [(1, 0, 0, 0), (1, 0, 1, 0)], run)
    lp = _run(g, [(4, 0, 0, 0), (4, 0, 1, 0), (2, 0, 0, 0), (2, 0, 1, 0)], run)
    for r in ref[1:] + lp:
        _assert_same(ref[0], r)
    ora = O.search(dict(ix, bsar_m=3.0), Q, 10, 8, 0.0, mode="bsar")
    r = check_search(lp[0][0], lp[0][1], ora, ix)
    assert not r["bad"], r["bad"][:5]


def test_two_waves_without_lag_run_as_one():
    """waves_per_query = 2 on an index without lag, or in an unpruned search, is the one-wave
    scan (the tuner's and scan_variant's answer say so)."""
    ix = oracle_index(B=64, L=0, n_calib=300)
    w = workload("gauss128")
    g = _index(ix)
    Q = w["queries"]
    g.set_launch(waves_per_query=2, lookahead=0, persistent=0, two_phase=0)
    assert g.scan_variant(Q.shape[0], 10, 8)[0] == 1
    a = g.search(Q, 10, 8, 0.1)
    g.set_launch(waves_per_query=1)
    b = g.search(Q, 10, 8, 0.1)
    _assert_same(a, b)
    g.set_launch(waves_per_query=0, lookahead=-1, persistent=-1, two_phase=-1)
    ix3 = oracle_index(B=64, L=3, n_calib=300)
    g3 = _index(ix3)
    g3.set_launch(waves_per_query=2)
    assert g3.scan_variant(Q.shape[0], 10, 8)[0] == 2
    assert g3.scan_variant(Q.shape[0], 10, 8, mode="none")[0] == 1


def test_lag_parallel_persistent_grid_smaller_than_batch():
    """Many more queries than resident workgroups: the persistent lag-parallel launch runs
    queries in turn and equals the one-pass launches bit for bit."""
    ix = oracle_index(B=64, L=3, n_calib=300)
    w = workload("gauss128")
    g = _index(ix)
    Q = np.tile(w["queries"], (60, 1))             # 6,000 queries
    rng = np.random.default_rng(5)
    ks = np.tile(rng.integers(1, 64, 100), 60).astype(np.int32)
    nps = np.tile(rng.integers(1, 33, 100), 60).astype(np.int32)
    run = lambda: g.search_var(Q, ks, nps, 0.1)
    res = _run(g, [(1, 0, 0, 0), (4, 0, 1, 0), (4, 0, 0, 1), (4, 0, 1, 1), (2, 0, 1, 0), (2, 0, 1, 1)], run)
    for r in res[1:]:
        _assert_same(res[0], r)
