"""GPU parity on the paths the 960-d and 768-d workloads take:

* BF16 query rotation (both operands rounded to bfloat16, FP32 accumulation on the matrix
  cores) against the oracle's BF16 rotation reading, then the whole search (probe selection,
  staged scan, merge) against the oracle searching from that same reading;
* 960-d BF16 storage and 768-d FP16 storage with the FP8 pre-stage over the leading 64 dims,
  with per-query K in {10, 50, 100} (tables at K_c = 10, 50, 100) and per-query nprobe up to
  256, in every launch shape; at 768 dims with 16-bit storage the deep look-ahead is entered
  from the pre-stage's alive list;
* more probed lists than the scan keeps in LDS (nprobe_max > 256), so list ids, lengths and
  first tiles come from memory, in both wave shapes, one pass and persistent, one phase and
  two-phase, also lagged.
"""
import numpy as np
import pytest

import oracle as O
from parity_util import artifacts, check_search, workload

pytestmark = pytest.mark.gpu

VARIANTS = [(w, la, p, t) for t in (0, 1) for p in (0, 1) for w in (1, 4) for la in (0, 1)]


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"


def _index(ix, rotation="f32"):
    from paper_2404_16322_amd import Index
    art = artifacts(ix)
    art["rotation"] = rotation
    return Index.from_artifacts(art)


def _fit(name, n, nq, n_calib, nlist, storage, fp8=0, seed=7):
    w = workload(name, n=n, nq=nq, n_calib=n_calib, n_val=0)
    ix = O.fit(w["base"], w["calib"], nlist=nlist, storage=storage, kmeans_iters=8, calib_k=10,
               calib_nprobe=16, B=256, seed=seed, fp8_lead=fp8, calib_k_extra=(50, 100))
    ix["centroids"] = ix["centroids"].astype(np.float32).astype(np.float64)
    ix["rotation"] = "bf16"
    return w, ix


@pytest.fixture(scope="module")
def gist_bf16():
    return _fit("gist1m", 16000, 96, 200, 256, "bf16")


@pytest.fixture(scope="module")
def embed_fp8():
    return _fit("embed768", 16000, 96, 200, 256, "f16", fp8=64)


def _per_query(nq, seed, np_hi=256):
    rng = np.random.default_rng(seed)
    ks = rng.choice([10, 50, 100], size=nq).astype(np.int32)
    nps = rng.integers(8, np_hi + 1, size=nq).astype(np.int32)
    return ks, nps


def _check_var(g, ix, Q, ks, nps, alpha, label):
    res = []
    for w, la, p, t in VARIANTS:
        g.set_launch(waves_per_query=w, lookahead=la, persistent=p, two_phase=t)
        res.append(g.search_var(Q, ks, nps, alpha))
    g.set_launch(waves_per_query=0, lookahead=-1, persistent=-1, two_phase=-1)
    ids, d, off, st = res[0]
    for r in res[1:]:     # every launch shape: bit-identical results and work counters
        np.testing.assert_array_equal(r[0], ids)
        np.testing.assert_array_equal(r[1], d)
        for key in ("candidates", "refined", "stage_slices"):
            assert r[3][key] == st[key], key
    same = excused = replayed = 0
    for qi in range(Q.shape[0]):
        ora = O.search(ix, Q[qi:qi + 1], int(ks[qi]), int(nps[qi]), alpha)
        r = check_search(ids[off[qi]:off[qi + 1]][None], d[off[qi]:off[qi + 1]][None], ora, ix)
        assert not r["bad"], (label, qi, r["bad"])
        same += r["same"]
        excused += r["excused"]
        replayed += r["replayed"]
    print(f"{label}: {same}/{Q.shape[0]} identical, {excused} excused ({replayed} by replay)")
    assert excused <= 0.05 * Q.shape[0] + 1
    return st


def test_bf16_rotation_matches_the_bf16_reading(gist_bf16):
    w, ix = gist_bf16
    g = _index(ix, "bf16")
    Q = w["queries"]
    qr, probes = g.debug_intermediates(Q, 64)
    ref = O.rotate_bf16(Q, ix["mu"], ix["R"])
    # the operands are the reading's exactly; only the FP32 accumulation order is open:
    # |error| <= n u sum |products| with n = 960 terms, u = 2^-24
    x32 = Q.astype(np.float32) - ix["mu"].astype(np.float32)[None, :]
    c = np.abs(O.round_storage(x32, "bf16"))
    rb = np.abs(O.round_storage(ix["R"].astype(np.float32), "bf16"))
    bound = Q.shape[1] * 2.0 ** -24 * (c @ rb.T)
    err = np.abs(qr - ref)
    assert np.all(err <= bound + 1e-30), float((err / (bound + 1e-30)).max())
    print(f"bf16 rotation: max |err| / bound = {float((err / (bound + 1e-30)).max()):.3g}")
    # probes from the GPU rotation equal the oracle's from the reading, up to near ties
    for qi in range(Q.shape[0]):
        top, _, margin = O.probe_order(ref[qi], ix["centroids"], 64)
        if probes[qi].tolist() != top.tolist():
            assert margin < 1e-4, qi


@pytest.mark.parametrize("alpha", [0.1, 0.3])
def test_gist_bf16_rotation_search_per_query_k_nprobe(gist_bf16, alpha):
    w, ix = gist_bf16
    g = _index(ix, "bf16")
    ks, nps = _per_query(w["queries"].shape[0], 21)
    st = _check_var(g, ix, w["queries"], ks, nps, alpha, f"gist bf16 alpha={alpha}")
    assert st["refined"] < st["candidates"]


@pytest.mark.parametrize("alpha", [0.1, 0.3])
def test_embed768_fp16_fp8_bf16_rotation_per_query_k_nprobe(embed_fp8, alpha):
    w, ix = embed_fp8
    g = _index(ix, "bf16")
    ks, nps = _per_query(w["queries"].shape[0], 22)
    st = _check_var(g, ix, w["queries"], ks, nps, alpha, f"embed768 fp8 alpha={alpha}")
    assert st["prestage_reads"] > 0
    assert st["prestage_pruned"] > 0


@pytest.fixture(scope="module")
def many_lists():
    w = workload("gauss128")
    out = {}
    for lag in (0, 2):
        ix = O.fit(w["base"], w["calib"][:300], nlist=512, kmeans_iters=8, calib_k=10, calib_nprobe=64,
                   B=64, L=lag, seed=7)
        ix["centroids"] = ix["centroids"].astype(np.float32).astype(np.float64)
        out[lag] = ix
    return w, out


@pytest.mark.parametrize("lag", [0, 2])
def test_probe_table_beyond_lds(many_lists, lag):
    """nprobe_max > 256: the scan reads every probed list's id, length and first tile from
    memory; fixed nprobe 300 and per-query nprobe in 200..400 with K up to 100."""
    w, ixs = many_lists
    ix = ixs[lag]
    g = _index(ix)
    Q = w["queries"][:40]
    shapes = [(wv, p, t) for t in (0, 1) for wv in (1, 4) for p in (0, 1)]   # (waves, persistent, two-phase)
    fixed = []
    for wv, p, t in shapes:
        g.set_launch(waves_per_query=wv, lookahead=0, persistent=p, two_phase=t)
        fixed.append(g.search(Q, 10, 300, 0.1)[:2])
    for r in fixed[1:]:
        np.testing.assert_array_equal(r[0], fixed[0][0])
        np.testing.assert_array_equal(r[1], fixed[0][1])
    r = check_search(fixed[0][0], fixed[0][1], O.search(ix, Q, 10, 300, 0.1), ix)
    assert not r["bad"], r["bad"][:3]
    rng = np.random.default_rng(4)
    ks = rng.choice([1, 10, 50, 100], size=Q.shape[0]).astype(np.int32)
    nps = rng.integers(200, 401, size=Q.shape[0]).astype(np.int32)
    var = []
    for wv, p, t in shapes:
        g.set_launch(waves_per_query=wv, lookahead=0, persistent=p, two_phase=t)
        var.append(g.search_var(Q, ks, nps, 0.1))
    g.set_launch(waves_per_query=0, lookahead=-1, persistent=-1)
    for r in var[1:]:
        np.testing.assert_array_equal(r[0], var[0][0])
        np.testing.assert_array_equal(r[1], var[0][1])
    ids, d, off, _ = var[0]
    for qi in range(Q.shape[0]):
        ora = O.search(ix, Q[qi:qi + 1], int(ks[qi]), int(nps[qi]), 0.1)
        r = check_search(ids[off[qi]:off[qi + 1]][None], d[off[qi]:off[qi + 1]][None], ora, ix)
        assert not r["bad"], (qi, r["bad"])
