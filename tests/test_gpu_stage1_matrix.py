"""The two-phase scan with the stage-1 sums on the matrix cores (launch knob stage1_matrix): for
every stored tile and every query probing its list, the partial distance over dim block 0 is
formed as ||q'_1||^2 + ||y_1||^2 - 2 <q'_1, y_1> (FP32 products), clamped at 0, and the scan
tests and extends it as usual.  Its results match the oracle's search (stage tests in FP64 on
the direct form) to the parity bar, equal the default scan's up to FP32 rounding, and are
bit-identical across the launch shapes that share the matrix first phase."""
import numpy as np
import pytest

import oracle as O
from parity_util import artifacts, check_search, oracle_index, workload

pytestmark = pytest.mark.gpu

SHAPES = [(w, la, p) for p in (0, 1) for w in (1, 4) for la in (0, 1)]


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"


def _index(ix):
    from paper_2404_16322_amd import Index
    return Index.from_artifacts(artifacts(ix))


def _matrix_shapes(g, run):
    out = []
    for w, la, p in SHAPES:
        g.set_launch(waves_per_query=w, lookahead=la, persistent=p, two_phase=1, stage1_matrix=1)
        out.append(run())
    g.set_launch(waves_per_query=0, lookahead=-1, persistent=-1, two_phase=-1, stage1_matrix=0)
    for r in out[1:]:
        for a, b in zip(out[0], r):
            if isinstance(a, np.ndarray):
                np.testing.assert_array_equal(a, b)
            elif isinstance(a, dict):
                for key in ("candidates", "refined", "stage_slices", "two_phase_sums"):
                    assert a[key] == b[key], key
    return out[0]


@pytest.mark.parametrize("storage", ["f32", "bf16", "f16"])
@pytest.mark.parametrize("mode,alpha,k,nprobe", [("learned", 0.1, 10, 8), ("learned", 0.3, 100, 20),
                                                 ("lossless", 0.0, 10, 8)])
def test_stage1_matrix_matches_oracle(storage, mode, alpha, k, nprobe):
    ix = oracle_index(storage=storage, n_calib=300)
    w = workload("gauss128")
    g = _index(ix)
    # more queries than a 64-pair chunk per list: 1,200 queries x nprobe over 64 lists
    Q = np.concatenate([w["queries"], w["val"][:200]])
    ids, d, st = _matrix_shapes(g, lambda: g.search(Q, k, nprobe, alpha, mode=mode))
    assert 0 < st["two_phase_sums"] <= st["candidates"]   # a query's first block runs untested
    ora = O.search(ix, Q, k, nprobe, alpha, mode=mode)
    r = check_search(ids, d, ora, ix)
    print(f"{storage} {mode} k={k} nprobe={nprobe}: {r['same']}/{r['nq']} identical, "
          f"{r['excused']} excused")
    assert not r["bad"], r["bad"][:5]
    # the default scan (direct-form stage 1): same ids except near decisions, distances 1e-4
    di, dd, _ = g.search(Q, k, nprobe, alpha, mode=mode)
    same = (di == ids).all(1)
    assert same.mean() >= 0.95
    np.testing.assert_allclose(d[same], dd[same], rtol=1e-4)


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
    ids, d, off, st = _matrix_shapes(g, lambda: g.search_var(Q, ks, nps, 0.1))
    assert 0 < st["two_phase_sums"] <= st["candidates"]   # a query's first block runs untested
    for qi in range(Q.shape[0]):
        ora = O.search(ix, Q[qi:qi + 1], int(ks[qi]), int(nps[qi]), 0.1)
        r = check_search(ids[off[qi]:off[qi + 1]][None], d[off[qi]:off[qi + 1]][None], ora, ix)
        assert not r["bad"], (qi, r["bad"])


def test_stage1_matrix_knob_validation_and_default():
    ix = oracle_index(storage="f32", n_calib=300)
    g = _index(ix)
    assert g.launch()["stage1_matrix"] == 0
    with pytest.raises(Exception):
        g.set_launch(stage1_matrix=2)
    assert g.launch()["stage1_matrix"] == 0
