"""GPU parity of the LB_Improved filter (MESSI_LB_IMPROVED): DTW answers with
the flag equal, id for id and bit for bit, those without it, and the
oracle's (ids exact, distances within 1e-4 relative), on the band kernels
(exact and masked radii) and on the wave kernel (radius past the band);
the second pass runs and removes DTW evaluations."""
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


def _check(ids, d, oids, od2):
    assert np.array_equal(ids, oids), (np.nonzero((ids != oids).any(axis=1))[0], ids[:3], oids[:3])
    od = np.sqrt(od2)
    fin = np.isfinite(od)
    assert np.array_equal(np.isfinite(d), fin)
    assert np.all(np.abs(d[fin] - od[fin]) <= 1e-4 * np.maximum(od[fin], 1e-3))


@pytest.mark.parametrize("length,r", [(128, 12), (128, 5), (256, 25), (256, 100), (64, 3)])
def test_lb_improved_same_answers(pm, length, r):
    n = 20_000
    raw = synth.randomwalk(n, length, seed=61)
    raw = np.concatenate([raw, raw[:30]])  # exact duplicates: ties
    qn, _, _ = synth.noisy_queries(20, n, length, data_seed=61)
    qs = np.concatenate([qn, synth.random_queries(4, length), raw[[9]]])
    nq = len(qs)
    t = torch.from_numpy(raw).cuda()
    idx = pm.messi_build(t, 16, 256, 200)
    qt = torch.from_numpy(qs).cuda()
    ks = [1 if i % 2 else 5 for i in range(nq)]
    dist, win = [1] * nq, [r] * nq
    base = pm.messi_query_batch(idx, qt, ks, dist, win, kmax=5, stats=True)
    lbi = pm.messi_query_batch(idx, qt, ks, dist, win, kmax=5, flags=pm.MESSI_LB_IMPROVED, stats=True)
    b_ids, b_d = base[0].cpu().numpy(), base[1].cpu().numpy()
    l_ids, l_d = lbi[0].cpu().numpy(), lbi[1].cpu().numpy()
    assert np.array_equal(b_ids, l_ids) and np.array_equal(b_d, l_d)
    oids, od2 = oracle.knn(raw, qs, 5, distance=oracle.DTW, r=r)
    for i in range(nq):
        _check(l_ids[i:i + 1, :ks[i]], l_d[i:i + 1, :ks[i]], oids[i:i + 1, :ks[i]], od2[i:i + 1, :ks[i]])
    assert base[2]["lb_improved"] == 0
    assert lbi[2]["lb_improved"] > 0
    assert lbi[2]["refined"] < base[2]["refined"], (lbi[2], base[2])
    idx.free()


def test_lb_improved_in_the_server_and_errors(pm):
    n, length = 10_000, 128
    raw = synth.randomwalk(n, length, seed=62)
    t = torch.from_numpy(raw).cuda()
    idx = pm.messi_build(t, 16, 256, 200)
    qs, _, _ = synth.noisy_queries(12, n, length, data_seed=62)
    srv = pm.Server(idx, workers=2, max_batch=8, flags=pm.MESSI_LB_IMPROVED, kmax=3)
    ids_of = {srv.submit(qs[i], 3, 1, 12): i for i in range(12)}
    got = {}
    for _ in range(2000):
        for rid, status, ids, d, _ in srv.poll(64, timeout_ms=50):
            got[rid] = (status, ids, d)
        if len(got) == 12:
            break
    srv.stop()
    assert len(got) == 12
    oids, od2 = oracle.knn(raw, qs, 3, distance=oracle.DTW, r=12)
    for rid, (status, ids, d) in got.items():
        i = ids_of[rid]
        assert status == 0
        _check(ids[None, :3], d[None, :3], oids[i:i + 1], od2[i:i + 1])
    qt = torch.from_numpy(qs).cuda()
    with pytest.raises(pm.MessiError):
        pm.messi_query_batch(idx, qt, [1] * 12, [1] * 12, [3] * 12, flags=8)
    # ED queries ignore the flag
    e_ids, e_d = pm.messi_query_batch(idx, qt, [2] * 12, [0] * 12, [0] * 12, flags=pm.MESSI_LB_IMPROVED)
    oids, od2 = oracle.knn(raw, qs, 2)
    _check(e_ids.cpu().numpy(), e_d.cpu().numpy(), oids, od2)
    idx.free()
