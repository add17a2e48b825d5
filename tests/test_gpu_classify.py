"""GPU parity of the k-NN classifier (messi_classify, Section 5.4): the
majority class of each query's k nearest neighbours against the oracle's
vote over the oracle's k-NN lists, for ED (with and without the BF16
screen) and DTW, with trend classes of the generated series."""
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


def test_device_trend_labels_match_host():
    raw = synth.randomwalk(5000, 96, seed=3)
    t = torch.from_numpy(raw).cuda()
    out = torch.empty(5000, dtype=torch.int32, device="cuda")
    synth.trend_labels_device(t, out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), synth.trend_labels(raw))


@pytest.mark.parametrize("k,distance,window,flags", [
    (1, 0, 0, 0), (7, 0, 0, 0), (50, 0, 0, 0), (7, 0, 0, 1), (50, 0, 0, 1), (7, 1, 12, 0),
])
def test_classify_matches_oracle(pm, k, distance, window, flags):
    n, length = 20_000, 128
    raw = synth.randomwalk(n, length, seed=17)
    labels = synth.trend_labels(raw)
    labels[::97] = -1  # not a class: not counted
    idx = pm.messi_build(torch.from_numpy(raw).cuda(), 16, 256, 300)
    qs = np.concatenate([synth.noisy_queries(40, n, length, data_seed=17)[0],
                         synth.random_queries(8, length)])
    cls, ids, d = pm.messi_classify(idx, torch.from_numpy(labels).cuda(), 4,
                                    torch.from_numpy(qs).cuda(), k, distance, window, flags)
    oids, od2 = oracle.knn(raw, qs, k, distance=distance, r=window)
    assert np.array_equal(ids.cpu().numpy(), oids)
    od = np.sqrt(od2)
    assert np.all(np.abs(d.cpu().numpy() - od) <= 1e-4 * np.maximum(od, 1e-3))
    assert np.array_equal(cls.cpu().numpy(), oracle.knn_vote(oids, labels, 4))
    idx.free()


def test_classify_argument_errors(pm):
    raw = synth.randomwalk(100, 64)
    idx = pm.messi_build(torch.from_numpy(raw).cuda(), 16, 256, 10)
    lab = torch.zeros(100, dtype=torch.int32, device="cuda")
    q = torch.from_numpy(synth.random_queries(2, 64)).cuda()
    with pytest.raises(pm.MessiError):
        pm.messi_classify(idx, lab, 0, q, 3)
    with pytest.raises(pm.MessiError):
        pm.messi_classify(idx, lab, 5000, q, 3)
    with pytest.raises(pm.MessiError):
        pm.messi_classify(idx, lab, 2, q, 3, flags=8)
    idx.free()
