"""The seeded input generators: deterministic by seed, right shapes and
recipe properties.  They hold no clustering arithmetic."""
import numpy as np

import datagen


def test_deterministic_by_seed_and_thread_count():
    s = datagen.spec("C2", N=50_000, chunks=4)
    a, ma = datagen.generate(s, threads=1)
    b, mb = datagen.generate(s, threads=4)
    assert a.dtype == np.float32 and a.shape == (3, 50_000)
    assert np.array_equal(a, b)
    assert np.array_equal(ma["centres"], mb["centres"])
    c, _ = datagen.generate(datagen.spec("C2", N=50_000, chunks=4, seed=s.seed + 1))
    assert not np.array_equal(a, c)


def test_padding_and_noise_fraction():
    s = datagen.spec("C2", N=10_001)
    X, meta = datagen.generate(s, ld=datagen.round_up(s.N, 4))
    assert X.shape == (3, 10_004)
    assert np.all(X[:, 10_001:] == 0)
    assert meta["n_noise"] == 100


def test_recipe_ranges():
    s = datagen.spec("C1", N=40_000)
    X, meta = datagen.generate(s)
    assert meta["centres"].shape == (4, 2)
    assert np.all(np.abs(meta["centres"]) <= 10)
    assert np.allclose(meta["weights"], 0.25)
    s3 = datagen.spec("C3", N=200_000)
    X3, m3 = datagen.generate(s3)
    assert X3.shape == (3, 200_000)
    assert np.all(m3["stds"][:, 0] == m3["stds"][:, 1])        # isotropic
    assert np.all((m3["stds"] >= 0.5) & (m3["stds"] <= 3.0))


def test_init_sample_distinct_points():
    s = datagen.spec("C1", N=1000)
    X, _ = datagen.generate(s)
    mu = datagen.init_sample(X, s.N, 50, 3)
    assert mu.dtype == np.float64 and mu.shape == (50, 2)
    cols = {tuple(r) for r in mu}
    assert len(cols) == 50
    pts = {tuple(c) for c in X.T.astype(np.float64)}
    assert cols <= pts
    assert np.array_equal(mu, datagen.init_sample(X, s.N, 50, 3))


def test_batched_specs():
    sp = datagen.batched_specs(64)
    assert len(sp) == 64
    for s in sp:
        assert 1000 <= s.N <= 1_000_000 and s.d in (2, 3) and 2 <= s.K <= 32
        assert len(s.extra["restart_seeds"]) == 8
