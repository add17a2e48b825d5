"""GPU parity of the in-place build (messi_build_ex with inplace): the
caller's buffer becomes the z-normalised store (bitwise the oracle's
z-normalisation), the summaries and leaves equal those of the copying
build, and every kind of query answers exactly as the oracle and the
copying index do."""
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


@pytest.mark.parametrize("length,leaf", [(256, 500), (100, 40)])
def test_inplace_build_and_queries(pm, length, leaf):
    n = 20_000
    raw = synth.randomwalk(n, length, seed=23)
    raw[11] = 2.5  # a flat series
    w = 16 if length % 16 == 0 else 4
    copy_idx = pm.messi_build(torch.from_numpy(raw).cuda(), w, 256, leaf)
    buf = torch.from_numpy(raw.copy()).cuda()
    ip_idx = pm.messi_build_ex(buf, w, 256, leaf, inplace=True, bf16_screen=True)
    got, want = buf.cpu().numpy(), oracle.znorm(raw)
    bad = np.argwhere(got.view(np.uint32) != want.view(np.uint32))
    assert len(bad) == 0, (len(bad), bad[:5], got[tuple(bad[0])] if len(bad) else None,
                           want[tuple(bad[0])] if len(bad) else None,
                           np.unique(bad[:, 0])[:10] if len(bad) else None)
    assert np.array_equal(pm.messi_get_words(ip_idx), pm.messi_get_words(copy_idx))
    assert np.array_equal(pm.messi_get_perm(ip_idx), pm.messi_get_perm(copy_idx))
    a, b = pm.messi_get_leaves(ip_idx), pm.messi_get_leaves(copy_idx)
    assert np.array_equal(a["begin"], b["begin"]) and np.array_equal(a["sym"], b["sym"])
    qs = np.concatenate([synth.noisy_queries(36, n, length, data_seed=23)[0],
                         synth.random_queries(4, length)])
    qt = torch.from_numpy(qs).cuda()
    for dist, r, k in [(0, 0, 5), (1, length // 10, 3)]:
        i1, d1 = pm.messi_query(ip_idx, qt, k, dist, r)
        i2, d2 = pm.messi_query(copy_idx, qt, k, dist, r)
        assert torch.equal(i1, i2) and torch.equal(d1, d2)
        oids, od2 = oracle.knn(raw, qs, k, distance=dist, r=r)
        assert np.array_equal(i1.cpu().numpy(), oids)
    ks = [1, 4] * 20
    flags = pm.MESSI_SCREEN_BF16
    b1 = pm.messi_query_batch(ip_idx, qt, ks, 0, 0, kmax=4, flags=flags)
    b2 = pm.messi_query_batch(copy_idx, qt, ks, 0, 0, kmax=4, flags=flags)
    assert torch.equal(b1[0], b2[0]) and torch.equal(b1[1], b2[1])
    ip_idx.free()
    copy_idx.free()


@pytest.mark.parametrize("length", [256, 100])
def test_store_and_words_at_extreme_scales(pm, length):
    """Rows whose (mu, sd) fall outside the range where the build divides
    by a hoisted reciprocal (sd below 2^-40 or above 2^40, mu exactly zero)
    take the plain division; both kinds mixed within each wave give the
    oracle's store and words bit for bit."""
    n = 4096
    raw = synth.randomwalk(n, length, seed=29)
    rows = np.arange(n)
    raw[rows % 7 == 1] *= np.float32(1e-14)             # sd about 1e-14
    raw[rows % 7 == 2] *= np.float32(1e14)              # sd about 1e14
    sym = rows[rows % 7 == 3]                           # mean exactly zero: +a, -a pairs
    half = raw[sym, : length // 2]
    raw[sym, 0::2] = half
    raw[sym, 1::2] = -half
    raw[rows % 7 == 4] += np.float32(1e6)               # large offset, ordinary sd
    raw[5] = -3.0                                       # flat
    w = 16 if length % 16 == 0 else 4
    buf = torch.from_numpy(raw.copy()).cuda()
    idx = pm.messi_build_ex(buf, w, 256, 64, inplace=True)
    got, want = buf.cpu().numpy(), oracle.znorm(raw)
    bad = np.argwhere(got.view(np.uint32) != want.view(np.uint32))
    assert len(bad) == 0, (len(bad), bad[:5], np.unique(bad[:, 0] % 7))
    Wo = oracle.words(raw, w, 8)
    assert np.array_equal(pm.messi_get_words(idx), Wo)
    perm, _ = oracle.leaf_partition(Wo, 64, 8)
    assert np.array_equal(pm.messi_get_perm(idx), perm)
    bt = pm.messi_build_times(idx)
    assert 0.0 <= bt["alloc_ms"] <= bt["build_ms"]
    idx.free()
