"""The two-phase scan with the stage-1 sums on the matrix cores (launch knob stage1_matrix = 1): for every stored tile and every query probing its list, the partial distance over
dim block 0 is formed as ||q'_1||^2 + ||y_1||^2 - 2 <q'_1, y_1> (FP32 products), clamped at 0.
The scan prunes on such a sum only where the first test prunes every value within the sum's
FP32 error bound, and takes the test on its own sum for the rest, so ids, distances and work
counters equal the one-phase scan's and the direct first phase's bit for bit in every launch
shape, and match the oracle.  With stage1_matrix = 2 the scan takes the expanded-form sums as
they are (results within FP32 rounding, matching the oracle)."""
import numpy as np
import pytest

import oracle as O
from parity_util import artifacts, check_search, oracle_index, workload

pytestmark = pytest.mark.gpu

SHAPES = [(w, la, p) for p in (0, 1) for w in (1, 4) for la in (0, 1)]
COUNTERS = ("candidates", "refined", "stage_slices")


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"


def _index(ix):
    from paper_2404_16322_amd import Index
    return Index.from_artifacts(artifacts(ix))


def _same(r0, r1):
    for a, b in zip(r0, r1):
        if isinstance(a, np.ndarray):
            np.testing.assert_array_equal(a, b)
        elif isinstance(a, dict):
            for key in COUNTERS:
                assert a[key] == b[key], key


def _all_forms(g, run):
    """Every launch shape with the matrix first phase, the direct first phase and one phase:
    all bit-identical.  Returns the matrix form's first result."""
    g.set_launch(waves_per_query=1, lookahead=1, persistent=0, two_phase=0)
    ref = run()
    out = None
    for w, la, p in SHAPES:
        for m in (1, 0):
            g.set_launch(waves_per_query=w, lookahead=la, persistent=p, two_phase=1, stage1_matrix=m)
            r = run()
            _same(ref, r)
            if m == 1 and out is None:
                out = r
    g.set_launch(waves_per_query=0, lookahead=-1, persistent=-1, two_phase=-1, stage1_matrix=0)
    return out


@pytest.mark.parametrize("storage", ["f32", "bf16", "f16"])
@pytest.mark.parametrize("mode,alpha,k,nprobe", [("learned", 0.1, 10, 8), ("learned", 0.3, 100, 20),
                                                 ("lossless", 0.0, 10, 8)])
def test_stage1_matrix_bit_identical_and_matches_oracle(storage, mode, alpha, k, nprobe):
    ix = oracle_index(storage=storage, n_calib=300)
    w = workload("gauss128")
    g = _index(ix)
    # more queries than a wave's 16-pair round per list: 1,200 queries x nprobe over 64 lists
    Q = np.concatenate([w["queries"], w["val"][:200]])
    ids, d, st = _all_forms(g, lambda: g.search(Q, k, nprobe, alpha, mode=mode))
    assert 0 < st["two_phase_sums"] <= st["candidates"]   # a query's first block runs untested
    ora = O.search(ix, Q, k, nprobe, alpha, mode=mode)
    r = check_search(ids, d, ora, ix)
    print(f"{storage} {mode} k={k} nprobe={nprobe}: {r['same']}/{r['nq']} identical, "
          f"{r['excused']} excused")
    assert not r["bad"], r["bad"][:5]


def test_stage1_matrix_ragged_lists_and_per_query():
    """Short lists (partial tiles), per-query K and nprobe, 100 dims (dim block 3 zero-padded)."""
    wl = workload("gauss128", n=6000, nq=300, n_calib=200, n_val=0, D=100)
    ix = O.fit(wl["base"], wl["calib"], nlist=200, storage="f32", kmeans_iters=6, calib_k=10,
               calib_nprobe=16, seed=7)
    ix["centroids"] = ix["centroids"].astype(np.float32).astype(np.float64)
    g = _index(ix)
    Q = wl["queries"]
    rng = np.random.default_rng(3)
    ks = rng.choice([1, 10, 50], size=Q.shape[0]).astype(np.int32)
    nps = rng.integers(1, 60, size=Q.shape[0]).astype(np.int32)
    ids, d, off, st = _all_forms(g, lambda: g.search_var(Q, ks, nps, 0.1))
    assert 0 < st["two_phase_sums"] <= st["candidates"]
    for qi in range(Q.shape[0]):
        ora = O.search(ix, Q[qi:qi + 1], int(ks[qi]), int(nps[qi]), 0.1)
        r = check_search(ids[off[qi]:off[qi + 1]][None], d[off[qi]:off[qi + 1]][None], ora, ix)
        assert not r["bad"], (qi, r["bad"])


@pytest.mark.parametrize("shift", [3.0, 300.0])
def test_stage1_matrix_cancellation_near_the_threshold(shift):
    """The rotated space translated by `shift` along each of the 32 axes of dim block 0 (stored
    values, centroids and the mean moved together, so every distance is unchanged): the
    block-0 norms reach 40 (shift 3) and 4 10^5 (shift 300) times the stage-1 distances, the
    expanded form loses that many digits, and the bound must send the undecided candidates (some,
    then all) to the direct recheck; results and counters stay bit-identical."""
    wl = workload("gauss128", n=8000, nq=400, n_calib=300, n_val=0)
    ix = O.fit(wl["base"], wl["calib"], nlist=32, storage="f32", kmeans_iters=6, calib_k=10,
               calib_nprobe=8, seed=5)
    s = np.zeros(ix["Y"].shape[1])
    s[:32] = shift
    ix = dict(ix, Y=(ix["Y"] + s).astype(np.float32).astype(np.float64),
              centroids=(ix["centroids"] + s).astype(np.float32).astype(np.float64),
              mu=ix["mu"] - s @ ix["R"])
    g = _index(ix)
    ids, d, st = _all_forms(g, lambda: g.search(wl["queries"], 10, 8, 0.1))
    assert 0 < st["two_phase_sums"] <= st["candidates"]
    assert np.all(np.diff(d, axis=1) >= 0) and np.all(ids >= 0)


@pytest.mark.parametrize("storage", ["f32", "bf16"])
@pytest.mark.parametrize("mode,alpha,k,nprobe", [("learned", 0.1, 10, 8), ("learned", 0.3, 100, 20)])
def test_stage1_expanded_sums_match_oracle(storage, mode, alpha, k, nprobe):
    """stage1_matrix = 2: the scan takes the expanded-form sums as they are.  Bit-identical
    across its two-phase launch shapes, within FP32 rounding of the bit-identical form (same ids
    except near decisions, distances 1e-4), and matching the oracle."""
    ix = oracle_index(storage=storage, n_calib=300)
    w = workload("gauss128")
    g = _index(ix)
    Q = np.concatenate([w["queries"], w["val"][:200]])
    ref = g.search(Q, k, nprobe, alpha, mode=mode)
    out = None
    for wv, la, p in SHAPES:
        g.set_launch(waves_per_query=wv, lookahead=la, persistent=p, two_phase=1, stage1_matrix=2)
        r = g.search(Q, k, nprobe, alpha, mode=mode)
        if out is None:
            out = r
        else:
            _same(out, r)
    g.set_launch(waves_per_query=0, lookahead=-1, persistent=-1, two_phase=-1, stage1_matrix=0)
    ids, d, st = out
    assert 0 < st["two_phase_sums"] <= st["candidates"]
    same = (ids == ref[0]).all(1)
    assert same.mean() >= 0.95
    np.testing.assert_allclose(d[same], ref[1][same], rtol=1e-4)
    ora = O.search(ix, Q, k, nprobe, alpha, mode=mode)
    r = check_search(ids, d, ora, ix)
    print(f"expanded {storage} k={k}: {r['same']}/{r['nq']} identical, {r['excused']} excused")
    assert not r["bad"], r["bad"][:5]


@pytest.mark.parametrize("storage", ["f32", "f16"])
@pytest.mark.parametrize("k,nprobe,alpha", [(10, 8, 0.1), (100, 20, 0.3)])
def test_stage1_expanded_fp8_prestage_sums_match_oracle(storage, k, nprobe, alpha):
    """stage1_matrix = 2 on an index with the FP8 pre-stage: the pre-stage's sums over the
    leading 64 dims from the matrix cores (codes decoded with the tile scale as the scan decodes
    them), taken as they are.  The survivors restart at dim 0, so every returned distance is the
    one the default scan returns for that id; ids equal except near pre-stage decisions; the
    oracle's bar holds; the mode-1 setting keeps the pre-stage in the scan's arithmetic (bit
    for bit the default)."""
    ix = oracle_index(storage=storage, n_calib=300, fp8_lead=64)
    w = workload("gauss128")
    g = _index(ix)
    Q = np.concatenate([w["queries"], w["val"][:200]])
    run = lambda: g.search(Q, k, nprobe, alpha)
    g.set_launch(waves_per_query=1, lookahead=1, persistent=0, two_phase=0, stage1_matrix=0)
    ref = run()
    g.set_launch(two_phase=1, stage1_matrix=1)
    _same(ref, run())
    out = None
    for wv, la, p in SHAPES:
        g.set_launch(waves_per_query=wv, lookahead=la, persistent=p, two_phase=1, stage1_matrix=2)
        r = run()
        if out is None:
            out = r
        else:
            _same(out, r)
    g.set_launch(waves_per_query=0, lookahead=-1, persistent=-1, two_phase=-1, stage1_matrix=0)
    ids, d, st = out
    assert st["two_phase_sums"] == st["prestage_reads"] > 0
    same = (ids == ref[0]).all(1)
    assert same.mean() >= 0.95
    np.testing.assert_array_equal(d[same], ref[1][same])
    ora = O.search(ix, Q, k, nprobe, alpha)
    r = check_search(ids, d, ora, ix)
    print(f"expanded FP8 pre-stage {storage} k={k}: {r['same']}/{r['nq']} identical, {r['excused']} excused")
    assert not r["bad"], r["bad"][:5]


@pytest.mark.parametrize("L", [1, 3])
def test_stage1_matrix_lagged_and_lag_parallel(L):
    """A lagged index (blocks of 64, lag 1 and 3): the bounded matrix first phase with one wave
    per query and in the lag-parallel shapes (two waves from L = 1, four from L = 3) equals the
    direct first phase and the one-phase scan bit for bit, counters included."""
    ix = oracle_index(B=64, L=L, n_calib=300)
    w = workload("gauss128")
    g = _index(ix)
    Q = w["queries"]
    run = lambda: g.search(Q, 10, 8, 0.1)
    g.set_launch(waves_per_query=1, lookahead=1, persistent=0, two_phase=0, stage1_matrix=0)
    ref = run()
    for wv in (1, 2, 4):
        for p in (0, 1):
            for m in (0, 1):
                g.set_launch(waves_per_query=wv, lookahead=1, persistent=p, two_phase=1, stage1_matrix=m)
                _same(ref, run())
    g.set_launch(waves_per_query=0, lookahead=-1, persistent=-1, two_phase=-1, stage1_matrix=0)
    assert 0 < ref[2]["candidates"]


def test_stage1_matrix_knob_validation_and_default():
    ix = oracle_index(storage="f32", n_calib=300)
    g = _index(ix)
    assert g.launch()["stage1_matrix"] == 0
    with pytest.raises(Exception):
        g.set_launch(stage1_matrix=3)
    assert g.launch()["stage1_matrix"] == 0
