"""GPU parity for long series, up to the largest length the build accepts
(4096 points): exact k-NN under ED at 1024-4096 and DTW (band and wide
windows) at 1024-4096 against the oracle, ids exact and distances within
1e-4 relative.  At 4096, DTW with r <= 31 (FP64 recheck in registers)
fits; wider windows need LDS rows a block cannot have and are refused with
MESSI_EINVAL."""
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
    assert np.all(np.abs(d - od) <= 1e-4 * np.maximum(od, 1e-3))


def _case(pm, n, length, seed):
    raw = synth.randomwalk(n, length, seed=seed)
    qn, _, _ = synth.noisy_queries(4, n, length, data_seed=seed)
    qs = np.concatenate([qn, synth.random_queries(1, length, seed=seed + 1), raw[[7]]])
    idx = pm.messi_build(torch.from_numpy(raw).cuda(), 16, 256, 100)
    return raw, qs, idx


def _query(pm, idx, qs, k, distance=0, window=0):
    ids, d = pm.messi_query(idx, torch.from_numpy(qs).cuda(), k, distance, window)
    return ids.cpu().numpy(), d.cpu().numpy()


@pytest.mark.parametrize("length", [1024, 2048, 4096])
def test_long_series_ed(pm, length):
    raw, qs, idx = _case(pm, 2500, length, seed=70 + length // 1024)
    oids, od2 = oracle.knn(raw, qs, 3)
    _check(*_query(pm, idx, qs, 3), oids, od2)
    idx.free()


@pytest.mark.parametrize("length,r", [(1024, 10), (1024, 100), (2048, 20), (3072, 8), (4096, 31)])
def test_long_series_dtw(pm, length, r):
    raw, qs, idx = _case(pm, 600, length, seed=80 + length // 1024)
    oids, od2 = oracle.knn(raw, qs[:4], 2, distance=oracle.DTW, r=r)
    _check(*_query(pm, idx, qs[:4], 2, 1, r), oids, od2)
    idx.free()


def test_dtw_too_long_for_lds_is_refused(pm):
    raw, qs, idx = _case(pm, 300, 4096, seed=90)
    for r in (40, 400):  # the FP64 recheck's, then the wave kernel's rows exceed a block's LDS
        with pytest.raises(pm.MessiError) as e:
            _query(pm, idx, qs[:1], 1, 1, r)
        assert e.value.code == pm.MESSI_EINVAL
    ids, d = _query(pm, idx, qs[:1], 1)  # ED at this length still works
    assert ids[0, 0] >= 0
    idx.free()
