"""The allocation-free device entry point (ddc_search_device_noalloc): on the same device
buffers it returns what ddc_search_device returns, bit for bit, for two calls in a row on one
stream (the second with a smaller batch, so the fixed scratch keeps the first call's contents),
with one K and N_probe for all queries and with per-query K and N_probe; a batch whose scratch
exceeds the fixed array is refused before any device work; and after a first call, further
calls change the device's free memory by nothing."""
import numpy as np
import pytest

from parity_util import artifacts, oracle_index, workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_2404_16322_amd import Index
    ix = oracle_index(storage="f32", n_calib=300)
    w = workload("gauss128")
    return ix, Index.from_artifacts(artifacts(ix)), np.concatenate([w["queries"], w["val"]])


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _both(g, Q, k, nprobe, alpha, mode, stream):
    """(ids, dists, counters) from ddc_search_device, then from ddc_search_device_noalloc."""
    import torch
    q = _dev(Q.astype(np.float32))
    out = []
    for fn in (g.search_device, g.search_device_noalloc):
        ids = torch.full((Q.shape[0], k), -7, dtype=torch.int64, device="cuda")
        d = torch.full((Q.shape[0], k), -7.0, dtype=torch.float32, device="cuda")
        ctr = torch.zeros(71, dtype=torch.int64, device="cuda")
        torch.cuda.synchronize()
        fn(q.data_ptr(), Q.shape[0], k, nprobe, alpha, mode, ids.data_ptr(), d.data_ptr(),
           d_counters=ctr.data_ptr(), stream=stream.cuda_stream)
        torch.cuda.synchronize()
        out.append((ids.cpu().numpy(), d.cpu().numpy(), ctr.cpu().numpy()))
    return out


@pytest.mark.parametrize("mode,alpha", [("learned", 0.1), ("lossless", 0.0), ("none", 0.0)])
def test_noalloc_equals_device_entry_on_two_calls(setup, mode, alpha):
    import torch
    _, g, Q = setup
    stream = torch.cuda.Stream()
    for n, k, nprobe in ((700, 10, 16), (37, 5, 8)):
        (ri, rd, rc), (ni, nd, nc) = _both(g, Q[:n], k, nprobe, alpha, mode, stream)
        print(f"{mode} n={n}: {int(rc[0])} candidates, {int(rc[1])} refined")
        np.testing.assert_array_equal(ni, ri)
        np.testing.assert_array_equal(nd, rd)
        # every counter but the two-phase sums read (the allocation-free call runs one phase)
        np.testing.assert_array_equal(np.delete(nc, 3), np.delete(rc, 3))
        assert (ni >= 0).all()


def test_noalloc_per_query_k_and_nprobe_on_two_calls(setup):
    import torch
    _, g, Q = setup
    stream = torch.cuda.Stream()
    rng = np.random.default_rng(11)
    for n in (500, 60):
        ks = rng.integers(1, 60, size=n).astype(np.int32)
        nps = rng.integers(1, 40, size=n).astype(np.int32)
        off = np.concatenate([[0], np.cumsum(ks)]).astype(np.int64)
        q, kd, npd, od = _dev(Q[:n].astype(np.float32)), _dev(ks), _dev(nps), _dev(off)
        res = []
        for fn in (g.search_device, g.search_device_noalloc):
            ids = torch.full((int(off[-1]),), -7, dtype=torch.int64, device="cuda")
            d = torch.full((int(off[-1]),), -7.0, dtype=torch.float32, device="cuda")
            torch.cuda.synchronize()
            fn(q.data_ptr(), n, 0, 0, 0.1, "learned", ids.data_ptr(), d.data_ptr(),
               stream=stream.cuda_stream, d_k=kd.data_ptr(), k_max=int(ks.max()),
               d_nprobe=npd.data_ptr(), nprobe_max=int(nps.max()), d_offsets=od.data_ptr())
            torch.cuda.synchronize()
            res.append((ids.cpu().numpy(), d.cpu().numpy()))
        np.testing.assert_array_equal(res[1][0], res[0][0])
        np.testing.assert_array_equal(res[1][1], res[0][1])


def test_noalloc_refuses_a_batch_beyond_its_scratch_and_runs_one_within():
    """4,096 lists: a query needs about 17 KB of scratch, so 5,000 queries do not fit the
    64 MiB array (refused before any device work, outputs untouched) and 3,000 do (equal to
    ddc_search_device)."""
    import torch
    from paper_2404_16322_amd import Index, DdcError
    from paper_2404_16322_amd import binding as B
    assert B.load_library().ddc_search_device_noalloc_bytes() == 64 << 20
    rng = np.random.default_rng(3)
    D, nlist, n = 128, 4096, 20000
    y = rng.standard_normal((n, D)).astype(np.float32)
    cent = y[rng.choice(n, nlist, replace=False)]
    assign = rng.integers(0, nlist, size=n).astype(np.int32)
    g = Index.from_artifacts(dict(mu=np.zeros(D), R=np.eye(D), centroids=cent, assign=assign, y=y))
    Q = rng.standard_normal((5000, D)).astype(np.float32)
    q = _dev(Q)
    ids = torch.full((5000, 10), -7, dtype=torch.int64, device="cuda")
    d = torch.full((5000, 10), -7.0, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    with pytest.raises(DdcError) as e:
        g.search_device_noalloc(q.data_ptr(), 5000, 10, 48, 0.0, "lossless", ids.data_ptr(), d.data_ptr())
    assert "at most about" in str(e.value)
    torch.cuda.synchronize()
    assert (ids.cpu().numpy() == -7).all()
    stream = torch.cuda.Stream()
    (ri, rd, rc), (ni, nd, nc) = _both(g, Q[:3000], 10, 48, 0.0, "lossless", stream)
    np.testing.assert_array_equal(ni, ri)
    np.testing.assert_array_equal(nd, rd)
    np.testing.assert_array_equal(np.delete(nc, 3), np.delete(rc, 3))


def test_noalloc_calls_leave_free_device_memory_unchanged(setup):
    import torch
    _, g, Q = setup
    stream = torch.cuda.Stream()
    q = _dev(Q[:400].astype(np.float32))
    ids = torch.empty((400, 10), dtype=torch.int64, device="cuda")
    d = torch.empty((400, 10), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    g.search_device_noalloc(q.data_ptr(), 400, 10, 16, 0.2, "learned", ids.data_ptr(), d.data_ptr(),
                            stream=stream.cuda_stream)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for n, alpha in ((400, 0.05), (100, 0.3)):   # new significances: their tables go to the array too
        g.search_device_noalloc(q.data_ptr(), n, 10, 16, alpha, "learned", ids.data_ptr(), d.data_ptr(),
                                stream=stream.cuda_stream)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
