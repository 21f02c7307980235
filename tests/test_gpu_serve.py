"""Continuous-batching server on the GPU: results identical alone and in the mix, the HBM
budget is respected, oversized requests are refused."""
import threading
import time

import numpy as np
import pytest

from parity_util import artifacts, oracle_index, workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def index():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_2404_16322_amd import Index
    return Index.from_artifacts(artifacts(oracle_index()))


def _requests(seed, count, D=128):
    rng = np.random.default_rng(seed)
    w = workload("gauss128")
    pool = np.vstack([w["queries"], w["val"]])
    reqs = []
    for _ in range(count):
        nq = int(rng.integers(1, 33))
        rows = rng.integers(0, pool.shape[0], size=nq)
        reqs.append((pool[rows], rng.integers(1, 101, size=nq).astype(np.int32),
                     rng.integers(1, 33, size=nq).astype(np.int32)))
    return reqs


def _collect(srv, tickets, timeout=60.0):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for t in tickets:
            if t not in out:
                r = srv.poll(t)
                if r is not None:
                    out[t] = r
        assert time.time() - t0 < timeout, "server did not finish"
        time.sleep(0.001)
    return [out[t] for t in tickets]


def test_results_identical_alone_and_in_the_mix(index):
    from paper_2404_16322_amd import Server
    reqs = _requests(1, 60)
    srv = Server(index, n_streams=4, max_batch=128, hbm_budget_bytes=1 << 30, alpha=0.1)
    tickets = [srv.submit(q, k, npb) for q, k, npb in reqs]
    res = _collect(srv, tickets)
    st = srv.stats()
    srv.close()
    assert st["requests_done"] == 60 and st["max_concurrent"] >= 1
    for (q, k, npb), (ids, d, off, _) in zip(reqs, res):
        a_ids, a_d, a_off, _ = index.search_var(q, k, npb, 0.1)
        np.testing.assert_array_equal(off, a_off)
        np.testing.assert_array_equal(ids, a_ids)      # bitwise: per-query computation
        np.testing.assert_array_equal(d, a_d)


def test_budget_bounds_in_flight_memory_and_refuses_oversized(index):
    from paper_2404_16322_amd import DdcError, Server
    reqs = _requests(2, 30)
    # room for a few small batches at a time; a 64-query x 256-result request never fits
    budget = 256 << 10
    srv = Server(index, n_streams=4, max_batch=64, hbm_budget_bytes=budget, alpha=0.1)
    tickets = []
    for q, k, npb in reqs:
        try:
            tickets.append(srv.submit(q, k, npb))
        except DdcError as e:
            assert e.status == -5
    res = _collect(srv, tickets)
    st = srv.stats()
    assert st["budget_peak_bytes"] <= budget
    big = np.zeros((64, 128), np.float32)
    with pytest.raises(DdcError) as ei:
        srv.submit(big, np.full(64, 256, np.int32), np.full(64, 64, np.int32))
    assert ei.value.status == -5
    srv.close()
    assert len(res) == len(tickets) > 0


def test_poisson_arrivals_report_latency(index):
    from paper_2404_16322_amd import Server
    reqs = _requests(3, 80)
    srv = Server(index, n_streams=4, max_batch=256, hbm_budget_bytes=1 << 30, alpha=0.1)
    rng = np.random.default_rng(4)
    gaps = rng.exponential(0.002, size=len(reqs))
    tickets = []

    def producer():
        t = time.monotonic()
        for (q, k, npb), g in zip(reqs, gaps):
            t += g
            while time.monotonic() < t:
                pass
            tickets.append(srv.submit(q, k, npb))

    th = threading.Thread(target=producer)
    th.start()
    th.join()
    _collect(srv, tickets)
    st = srv.stats()
    srv.close()
    assert st["requests_done"] == len(reqs)
    assert 0 < st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]


def test_quantization_test_served_like_searched_alone():
    """BSA-O's quantization test (Sec. V-B) through the server: every request's results equal
    searching its queries alone with the same test and significance."""
    from paper_2404_16322_amd import Index, Server
    ix = Index.from_artifacts(artifacts(oracle_index(pq_m=32, n_calib=400)))
    reqs = _requests(3, 24)
    srv = Server(ix, n_streams=3, max_batch=96, hbm_budget_bytes=1 << 30, alpha=0.1, mode="bsao")
    tickets = [srv.submit(q, k, npb) for q, k, npb in reqs]
    res = _collect(srv, tickets)
    srv.close()
    for (q, k, npb), (ids, d, off, _) in zip(reqs, res):
        a_ids, a_d, a_off, _ = ix.search_var(q, k, npb, 0.1, mode="bsao")
        np.testing.assert_array_equal(off, a_off)
        np.testing.assert_array_equal(ids, a_ids)
        np.testing.assert_array_equal(d, a_d)
