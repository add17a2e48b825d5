"""The allocation-free query entry point (messi_query_noalloc), called
through the C ABI: its answers equal those of messi_query, the entry point
it is a variant of, bit for bit, on two calls in a row (the second with
fewer queries, so stale contents of the shared scratch array must not
matter), under ED and DTW; a request larger than the scratch array is
refused with MESSI_EINVAL; and both agree with the oracle (ids exactly,
distances within 1e-4 relative)."""
import ctypes

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pm():
    import paper_2110_07519_amd as pm

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    pm.lib()
    return pm


def _call_noalloc(pm, idx, qt, k, distance, window):
    """Straight through the C ABI (the binding only marshals arguments)."""
    nq = qt.shape[0]
    ids = torch.full((nq, k), -7, dtype=torch.int64, device="cuda")
    d = torch.full((nq, k), -7.0, dtype=torch.float32, device="cuda")
    rc = pm.lib().messi_query_noalloc(idx.handle, ctypes.c_void_p(qt.data_ptr()), nq, k, distance,
                                      window, ctypes.c_void_p(ids.data_ptr()), ctypes.c_void_p(d.data_ptr()))
    return rc, ids.cpu().numpy(), d.cpu().numpy()


@pytest.mark.parametrize("distance,window,k", [(0, 0, 3), (1, 12, 2)])
def test_noalloc_equals_messi_query_twice(pm, distance, window, k):
    n, length = 20_000, 128
    raw = synth.randomwalk(n, length)
    t = torch.from_numpy(raw).cuda()
    idx = pm.messi_build(t, 16, 256, 500)
    qs = np.concatenate([synth.random_queries(10, length), synth.noisy_queries(10, n, length)[0]])
    for nq in (20, 7):  # the second call is smaller
        qt = torch.from_numpy(np.ascontiguousarray(qs[:nq])).cuda()
        rc, ids, d = _call_noalloc(pm, idx, qt, k, distance, window)
        assert rc == pm.MESSI_OK, pm.lib().messi_last_error()
        rids, rd = pm.messi_query(idx, qt, k, distance, window)
        assert np.array_equal(ids, rids.cpu().numpy())
        assert np.array_equal(d.view(np.uint32), rd.cpu().numpy().view(np.uint32))
        oids, od2 = oracle.knn(raw, qs[:nq], k, distance=distance, r=window)
        assert np.array_equal(ids, oids)
        od = np.sqrt(od2)
        assert np.all(np.abs(d - od) <= 1e-4 * np.maximum(od, 1e-3))
    idx.free()


def test_noalloc_refuses_requests_beyond_its_scratch(pm):
    n, length = 300_000, 64
    raw = synth.randomwalk(n, length)
    t = torch.from_numpy(raw).cuda()
    idx = pm.messi_build(t, 16, 256, 100)  # small leaves: many chunks per query
    qs = synth.random_queries(1024, length)
    qt = torch.from_numpy(qs).cuda()
    rc, ids, _ = _call_noalloc(pm, idx, qt, 1, 0, 0)
    assert rc == pm.MESSI_EINVAL
    assert b"scratch" in pm.lib().messi_last_error()
    assert np.all(ids == -7)  # nothing launched
    rc, _, _ = _call_noalloc(pm, idx, torch.cat([qt, qt[:1]]), 1, 0, 0)
    assert rc == pm.MESSI_EINVAL  # more than 1024 queries
    # a request that fits still works after the refusals
    rc, ids, d = _call_noalloc(pm, idx, qt[:4], 1, 0, 0)
    assert rc == pm.MESSI_OK
    oids, _ = oracle.knn(raw, qs[:4], 1)
    assert np.array_equal(ids, oids)
    idx.free()
