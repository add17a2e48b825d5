"""The seeded input generator: reproducible, chunk-addressable, and drawing
the distributions the paper's workloads name (Section 5.1: N(0,1) steps of a
random walk; Section 5.3: Gaussian noise on collection series)."""
import math

import numpy as np
import scipy.stats as st

import synth


def test_log_and_sqrt_accuracy():
    rng = np.random.default_rng(0)
    for x in np.concatenate([rng.random(2000), rng.random(200) * 1e-30, [0.5, 1.0, 2.0, 1e-300]]):
        if x <= 0:
            continue
        assert abs(synth.host().synth_host_log(float(x)) - math.log(x)) <= 4e-16 * max(1.0, abs(math.log(x)))
        assert abs(synth.host().synth_host_sqrt(float(x)) - math.sqrt(x)) <= 4e-16 * math.sqrt(x)


def test_normals_are_standard_normal():
    z = synth.normals(1 << 18, seed=11, stream=3)
    assert st.kstest(z, "norm").pvalue > 1e-3
    assert abs(z.mean()) < 0.01 and abs(z.var() - 1) < 0.01


def test_uniforms_open_interval():
    u = synth.uniforms(1 << 16, seed=5)
    assert np.all(u > 0) and np.all(u < 1)
    assert st.kstest(u, "uniform").pvalue > 1e-3


def test_randomwalk_deterministic_and_chunkable():
    a = synth.randomwalk(1000, 128, seed=1)
    b = synth.randomwalk(1000, 128, seed=1)
    assert np.array_equal(a, b)
    c = np.concatenate([synth.randomwalk(300, 128, seed=1, id0=0),
                        synth.randomwalk(700, 128, seed=1, id0=300)])
    assert np.array_equal(a, c)
    assert not np.array_equal(a, synth.randomwalk(1000, 128, seed=2))


def test_randomwalk_increments_are_normal():
    x = synth.randomwalk(400, 256, seed=1).astype(np.float64)
    steps = np.diff(x, axis=1).ravel()
    assert abs(steps.std() - 1.0) < 0.01
    assert abs(x[:, 0].std() - 1.0) < 0.15  # x_0 ~ N(0, 1)


def test_noisy_queries_recipe():
    n = 5000
    q, src, sig = synth.noisy_queries(30, n, 256)
    assert list(sig[:6]) == [0.01, 0.1, 1.0, 0.01, 0.1, 1.0]
    assert np.all((src >= 0) & (src < n))
    base = synth.randomwalk(n, 256)
    for j in range(30):
        x = base[src[j]].astype(np.float64)
        noise = q[j].astype(np.float64) - x
        assert abs(noise.std() / x.std() - sig[j]) < 0.35 * sig[j]


def test_ar1_series_follows_its_recursion():
    x = synth.ar1_series(5000, phi=0.99)
    e = synth.normals(5000, seed=synth.SEED_DATA, stream=11)
    y = np.empty(5000)
    y[0] = e[0]
    for t in range(1, 5000):
        y[t] = 0.99 * y[t - 1] + np.sqrt(1.0 - 0.99 * 0.99) * e[t]
    assert np.allclose(x, y.astype(np.float32), rtol=1e-5, atol=1e-5)
    assert np.array_equal(x, synth.ar1_series(5000, phi=0.99))  # seeded
