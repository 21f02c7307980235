"""Allocation failures injected from the host (ddc_set_fault "alloc:<n>": the n-th device or
pinned-host allocation fails before the runtime is asked).  For every n up to the call's own
allocation count, fit, import, the host and device searches and server creation return
DDC_ENOMEM, hold no allocation afterwards (the library's live-allocation count is back where it
was), and a failed search leaves the index answering as before.  No kernel is made to fail."""
import numpy as np
import pytest

from parity_util import artifacts, oracle_index, workload

pytestmark = pytest.mark.gpu

ENOMEM = -2


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_2404_16322_amd import binding as B
    yield
    B.set_fault("alloc:0")


def _sweep(call, limit=400):
    """call() under alloc:1, alloc:2, ... until it succeeds; returns the failures seen."""
    from paper_2404_16322_amd import binding as B
    from paper_2404_16322_amd import DdcError
    fails = 0
    for n in range(1, limit + 1):
        before = B.live_allocations()
        B.set_fault(f"alloc:{n}")
        try:
            out = call()
        except DdcError as e:
            B.set_fault("alloc:0")
            assert e.status == ENOMEM, (n, e)
            assert "injected" in str(e), (n, str(e))
            assert B.live_allocations() == before, (n, before, B.live_allocations())
            fails += 1
            continue
        B.set_fault("alloc:0")
        return fails, out
    raise AssertionError(f"still failing after {limit} injected faults")


def test_fit_fails_cleanly_at_every_allocation():
    from paper_2404_16322_amd import Index
    w = workload("gauss128")
    fails, ix = _sweep(lambda: Index.fit(w["base"][:3000], w["calib"][:200], nlist=16, kmeans_iters=3,
                                         calib_k=10, calib_nprobe=4, seed=3))
    print(f"fit: {fails} injected failures before it succeeded")
    assert fails >= 5
    ids, d, _ = ix.search(w["queries"], 10, 4, 0.1)
    assert (ids >= 0).all()
    ix.close()


def test_import_fails_cleanly_and_searches_leave_the_index_unchanged():
    import torch
    from paper_2404_16322_amd import Index
    ix_o = oracle_index(storage="f32", n_calib=300)
    w = workload("gauss128")
    fails, g = _sweep(lambda: Index.from_artifacts(artifacts(ix_o)))
    assert fails >= 3
    Q = w["queries"]
    ref = g.search(Q, 10, 8, 0.1)[:2]            # also fills the index's cached tables
    fails, res = _sweep(lambda: g.search(Q, 10, 8, 0.1)[:2])
    assert fails >= 2
    np.testing.assert_array_equal(res[0], ref[0])
    np.testing.assert_array_equal(res[1], ref[1])
    # device entry point on a new stream: its workspace is among the allocations that fail
    q = torch.from_numpy(np.ascontiguousarray(Q, dtype=np.float32)).cuda()
    ids = torch.empty((Q.shape[0], 10), dtype=torch.int64, device="cuda")
    d = torch.empty((Q.shape[0], 10), dtype=torch.float32, device="cuda")
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()

    def dev():
        g.search_device(q.data_ptr(), Q.shape[0], 10, 8, 0.1, "learned", ids.data_ptr(), d.data_ptr(),
                        stream=stream.cuda_stream)
        torch.cuda.synchronize()
        return ids.cpu().numpy(), d.cpu().numpy()
    fails, res = _sweep(dev)
    assert fails >= 1
    np.testing.assert_array_equal(res[0], ref[0])
    np.testing.assert_array_equal(res[1], ref[1])
    g.close()


def test_server_create_fails_cleanly():
    from paper_2404_16322_amd import Index, Server
    ix_o = oracle_index(storage="f32", n_calib=300)
    g = Index.from_artifacts(artifacts(ix_o))
    w = workload("gauss128")
    # the index caches its correction rows per significance (the server's warm-up search builds
    # them); build them first, so only the server's own allocations are counted
    g.search(w["queries"][:4], 10, 8, 0.1)
    fails, srv = _sweep(lambda: Server(g, n_streams=2, max_batch=64, hbm_budget_bytes=1 << 28, alpha=0.1))
    assert fails >= 10                          # two streams' device and pinned buffers
    t = srv.submit(w["queries"][:5], np.full(5, 10, np.int32), np.full(5, 8, np.int32))
    import time
    for _ in range(2000):
        r = srv.poll(t)
        if r is not None:
            break
        time.sleep(0.001)
    assert r is not None and (r[0] >= 0).all()
    srv.close()
    g.close()
