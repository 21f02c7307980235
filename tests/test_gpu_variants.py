"""Launch-shape variants of the scan (one wavefront or a workgroup of four per query, with and
without multi-block look-ahead loads, one pass per workgroup or a persistent grid taking queries
longest first from a counter, with or without the stage-1 sums computed list by list first)
return bit-identical results, which match the oracle; the tuner picks one of them per size
class."""
import numpy as np
import pytest

import oracle as O
from parity_util import artifacts, check_search, oracle_index, workload

pytestmark = pytest.mark.gpu

VARIANTS = [(w, la, p, t) for t in (0, 1) for p in (0, 1) for w in (1, 4) for la in (0, 1)]


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"


def _index(ix):
    from paper_2404_16322_amd import Index
    return Index.from_artifacts(artifacts(ix))


def _all_variants(g, run):
    out = []
    for w, la, p, t in VARIANTS:
        g.set_launch(waves_per_query=w, lookahead=la, persistent=p, two_phase=t)
        out.append(run())
    g.set_launch(waves_per_query=0, lookahead=-1, persistent=-1, two_phase=-1)
    return out


def _assert_identical(results):
    first = results[0]
    for r in results[1:]:
        for a, b in zip(first, r):
            if isinstance(a, np.ndarray):
                np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("storage", ["f32", "bf16"])
@pytest.mark.parametrize("mode,alpha", [("learned", 0.1), ("lossless", 0.0), ("none", 0.0)])
def test_variants_bitwise_identical_d128(storage, mode, alpha):
    ix = oracle_index(storage=storage, n_calib=300)
    w = workload("gauss128")
    g = _index(ix)
    Q = w["queries"]
    res = _all_variants(g, lambda: g.search(Q, 10, 8, alpha, mode=mode)[:2])
    _assert_identical(res)
    ora = O.search(ix, Q, 10, 8, alpha, mode=mode)
    r = check_search(res[0][0], res[0][1], ora, ix)
    assert not r["bad"], r["bad"][:5]


@pytest.fixture(scope="module")
def wide():
    # 960-d: 30 dim blocks, so look-ahead windows of 8 blocks occur
    w = workload("gist1m", n=12000, nq=120, n_calib=200, n_val=0)
    ix = O.fit(w["base"], w["calib"], nlist=32, delta_d=32, storage="bf16", kmeans_iters=10,
               calib_k=10, calib_nprobe=6, B=256, seed=7)
    ix["centroids"] = ix["centroids"].astype(np.float32).astype(np.float64)
    return w, ix


@pytest.mark.parametrize("k,nprobe", [(10, 6), (100, 4)])
def test_variants_bitwise_identical_d960(wide, k, nprobe):
    w, ix = wide
    g = _index(ix)
    Q = w["queries"]
    res = _all_variants(g, lambda: g.search(Q, k, nprobe, 0.1)[:2])
    _assert_identical(res)
    ora = O.search(ix, Q, k, nprobe, 0.1)
    r = check_search(res[0][0], res[0][1], ora, ix)
    print(f"d960: {r['same']}/{r['nq']} identical, {r['excused']} excused")
    assert not r["bad"], r["bad"][:5]
    assert r["excused"] <= 0.05 * r["nq"] + 1


def test_variants_per_query_k_nprobe_and_counters():
    ix = oracle_index()
    w = workload("gauss128")
    g = _index(ix)
    Q = w["queries"][:150]
    rng = np.random.default_rng(3)
    ks = rng.integers(1, 120, Q.shape[0]).astype(np.int32)
    nps = rng.integers(1, 20, Q.shape[0]).astype(np.int32)
    res = _all_variants(g, lambda: g.search_var(Q, ks, nps, 0.2))
    _assert_identical([r[:3] for r in res])
    # work counters describe the algorithm, not the launch: identical in every variant
    for r in res[1:]:
        for key in ("candidates", "refined", "stage_slices"):
            assert r[3][key] == res[0][3][key], key


@pytest.mark.parametrize("storage,fp8", [("f32", 0), ("bf16", 0), ("f16", 0), ("f16", 64), ("f32", 64)])
def test_five_wave_build_bitwise_identical(storage, fp8):
    """The one-wave kernel's second build for five waves per SIMD (waves_per_simd = 5; it
    spills a few registers) returns the four-wave build's ids, distances and counters in every
    one-wave shape, one- and two-phase, with and without the FP8 pre-stage; kernels without
    that build ignore the knob."""
    ix = oracle_index(storage=storage, n_calib=300, fp8_lead=fp8)
    w = workload("gauss128")
    g = _index(ix)
    Q = np.concatenate([w["queries"], w["val"][:200]])
    for mode, alpha, k in (("learned", 0.1, 10), ("learned", 0.3, 100), ("lossless", 0.0, 10)):
        ref = None
        for la in (0, 1):
            for p in (0, 1):
                for t in (0, 1):
                    for ws in (4, 5):
                        g.set_launch(waves_per_query=1, lookahead=la, persistent=p, two_phase=t,
                                     waves_per_simd=ws)
                        r = g.search(Q, k, 8, alpha, mode=mode)
                        if ref is None:
                            ref = r
                            continue
                        for a, b in zip(ref, r):
                            if isinstance(a, np.ndarray):
                                np.testing.assert_array_equal(a, b)
                            else:
                                for key in ("candidates", "refined", "stage_slices"):
                                    assert a[key] == b[key], key
    g.set_launch(waves_per_query=0, lookahead=-1, persistent=-1, two_phase=-1, waves_per_simd=0)
    with pytest.raises(Exception):
        g.set_launch(waves_per_simd=6)


def test_tuner_picks_a_variant_and_caches_it():
    ix = oracle_index()
    w = workload("gauss128")
    g = _index(ix)
    assert g.launch() == dict(waves_per_query=0, lookahead=-1, query_order=1, xcd_swizzle=1,
                              persistent=-1, two_phase=-1, full_d_matrix=0, stage1_matrix=0,
                              waves_per_simd=0)
    ids0, d0, _ = g.search(w["queries"], 10, 8, 0.1)
    v = g.scan_variant(w["queries"].shape[0], 10, 8)
    assert v in VARIANTS
    ids1, d1, _ = g.search(w["queries"], 10, 8, 0.1)
    np.testing.assert_array_equal(ids0, ids1)
    np.testing.assert_array_equal(d0, d1)
    g.set_launch(waves_per_query=4, lookahead=0, query_order=0, xcd_swizzle=0, persistent=1,
                 two_phase=1)
    assert g.scan_variant(1000, 10, 8) == (4, 0, 1, 1)
    assert g.scan_variant(1000, 10, 8, mode="none") == (4, 0, 1, 0)   # no test: one phase
    ids2, d2, _ = g.search(w["queries"], 10, 8, 0.1)
    np.testing.assert_array_equal(ids0, ids2)
    np.testing.assert_array_equal(d0, d2)


def test_persistent_grid_smaller_than_batch():
    """A batch far larger than the resident grid: every workgroup of the persistent launch
    runs many queries in turn; results equal the one-pass launch bit for bit."""
    ix = oracle_index()
    w = workload("gauss128")
    g = _index(ix)
    Q = np.tile(w["queries"], (120, 1))            # 12,000 queries
    rng = np.random.default_rng(5)
    ks = np.tile(rng.integers(1, 64, 100), 120).astype(np.int32)
    nps = np.tile(rng.integers(1, 33, 100), 120).astype(np.int32)
    res = []
    for t in (0, 1):
        for wv in (1, 4):
            for p in (0, 1):
                g.set_launch(waves_per_query=wv, lookahead=0, persistent=p, two_phase=t)
                res.append(g.search_var(Q, ks, nps, 0.1))
    g.set_launch(waves_per_query=0, lookahead=-1, persistent=-1, two_phase=-1)
    _assert_identical([r[:3] for r in res])
    for r in res[1:]:
        for key in ("candidates", "refined", "stage_slices"):
            assert r[3][key] == res[0][3][key], key
    # every copy of a query returns that query's result, wherever the launch placed it
    ids, d, off = res[-1][:3]
    for i in range(100, Q.shape[0]):
        j = i % 100
        np.testing.assert_array_equal(ids[off[i]:off[i + 1]], ids[off[j]:off[j + 1]])
        np.testing.assert_array_equal(d[off[i]:off[i + 1]], d[off[j]:off[j + 1]])
