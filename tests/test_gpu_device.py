"""The device-buffer entry point (ddc_search_device): results on device buffers equal the host
entry point's bit for bit, for consecutive calls on one stream whose batch sizes grow and shrink
(the stream's scratch workspace is made, grown and reused), on the default stream, and with
per-query K and nprobe; and they match the oracle."""
import numpy as np
import pytest

import oracle as O
from parity_util import artifacts, check_search, oracle_index, workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_2404_16322_amd import Index
    ix = oracle_index(storage="f32", n_calib=300)
    w = workload("gauss128")
    # the workload's queries, then its held-out validation vectors as more queries
    return ix, Index.from_artifacts(artifacts(ix)), np.concatenate([w["queries"], w["val"]])


def _device_search(g, Q, k, nprobe, alpha, stream):
    import torch
    q = torch.from_numpy(np.ascontiguousarray(Q, dtype=np.float32)).cuda()
    ids = torch.empty((Q.shape[0], k), dtype=torch.int64, device="cuda")
    d = torch.empty((Q.shape[0], k), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    g.search_device(q.data_ptr(), Q.shape[0], k, nprobe, alpha, "learned", ids.data_ptr(), d.data_ptr(),
                    stream=stream.cuda_stream if stream is not None else 0)
    torch.cuda.synchronize()
    return ids.cpu().numpy(), d.cpu().numpy()


@pytest.mark.parametrize("sizes", [(37, 700, 5, 300), (1, 2)])
def test_device_calls_on_one_stream_equal_host(setup, sizes):
    import torch
    ix, g, Q = setup
    stream = torch.cuda.Stream()
    for n in sizes:
        Qn = Q[:n]
        di, dd = _device_search(g, Qn, 10, 8, 0.1, stream)
        hi, hd, _ = g.search(Qn, 10, 8, 0.1)
        np.testing.assert_array_equal(di, hi)
        np.testing.assert_array_equal(dd, hd)
    ora = O.search(ix, Q[:300], 10, 8, 0.1, mode="learned")
    di, dd = _device_search(g, Q[:300], 10, 8, 0.1, stream)
    r = check_search(di, dd, ora, ix)
    assert not r["bad"], r["bad"][:5]


def test_device_default_stream_and_two_streams(setup):
    import torch
    ix, g, Q = setup
    hi, hd, _ = g.search(Q[:64], 10, 16, 0.1)
    for stream in (None, torch.cuda.Stream(), torch.cuda.Stream()):
        di, dd = _device_search(g, Q[:64], 10, 16, 0.1, stream)
        np.testing.assert_array_equal(di, hi)
        np.testing.assert_array_equal(dd, hd)


def test_device_per_query_k_and_nprobe(setup):
    import torch
    ix, g, Q = setup
    rng = np.random.default_rng(5)
    n = 120
    ks = rng.integers(1, 40, size=n).astype(np.int32)
    nps = rng.integers(1, 24, size=n).astype(np.int32)
    off = np.concatenate([[0], np.cumsum(ks)]).astype(np.int64)
    hi, hd, _off, _ = g.search_var(Q[:n], ks, nps, 0.1)
    q = torch.from_numpy(np.ascontiguousarray(Q[:n], dtype=np.float32)).cuda()
    k_dev = torch.from_numpy(ks).cuda()
    np_dev = torch.from_numpy(nps).cuda()
    off_dev = torch.from_numpy(off).cuda()
    ids = torch.empty(int(off[-1]), dtype=torch.int64, device="cuda")
    d = torch.empty(int(off[-1]), dtype=torch.float32, device="cuda")
    stream = torch.cuda.Stream()
    for _ in range(2):
        torch.cuda.synchronize()
        g.search_device(q.data_ptr(), n, 0, 0, 0.1, "learned", ids.data_ptr(), d.data_ptr(),
                        stream=stream.cuda_stream, d_k=k_dev.data_ptr(), k_max=int(ks.max()),
                        d_nprobe=np_dev.data_ptr(), nprobe_max=int(nps.max()), d_offsets=off_dev.data_ptr())
        torch.cuda.synchronize()
        np.testing.assert_array_equal(ids.cpu().numpy(), hi)
        np.testing.assert_array_equal(d.cpu().numpy(), hd)


def test_device_calls_from_two_threads_on_their_own_streams(setup):
    """Two host threads, each with its own stream (and so its own workspace), search at the
    same time; every result equals the host entry point's."""
    import threading
    import torch
    ix, g, Q = setup
    sizes = (64, 300, 17)
    ref = {n: g.search(Q[:n], 10, 8, 0.1)[:2] for n in sizes}
    errors = []

    def worker(seed):
        try:
            stream = torch.cuda.Stream()
            q = torch.from_numpy(np.ascontiguousarray(Q[:max(sizes)], dtype=np.float32)).cuda()
            ids = torch.empty((max(sizes), 10), dtype=torch.int64, device="cuda")
            d = torch.empty((max(sizes), 10), dtype=torch.float32, device="cuda")
            torch.cuda.synchronize()   # the upload above ran on the default stream
            rng = np.random.default_rng(seed)
            for _ in range(12):
                n = int(rng.choice(sizes))
                stream.synchronize()
                g.search_device(q.data_ptr(), n, 10, 8, 0.1, "learned", ids.data_ptr(), d.data_ptr(),
                                stream=stream.cuda_stream)
                stream.synchronize()
                hi, hd = ref[n]
                if not (np.array_equal(ids[:n].cpu().numpy(), hi) and np.array_equal(d[:n].cpu().numpy(), hd)):
                    errors.append((seed, n))
        except Exception as e:   # reported below
            errors.append((seed, repr(e)))

    ths = [threading.Thread(target=worker, args=(s,)) for s in (1, 2)]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    assert not errors, errors[:4]
