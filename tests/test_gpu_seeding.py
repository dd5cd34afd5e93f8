"""GPU parity of k-means++ seeding (kmeans_pp_init through the C ABI) against
the numpy oracle: the chosen indices must be identical (integer work, exact
weights), on sizes that span one and many blocks, ragged tails, padded rows,
both dimensions, K up to 64 and the degenerate cases."""
import numpy as np
import pytest

import datagen
from oracle import seeding

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def km():
    from paper_2405_12052_amd import KMeans
    k = KMeans(0)
    yield k
    k.close()


def log(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("d,K,N", [(2, 1, 1), (2, 2, 2), (3, 5, 5), (2, 4, 1003),
                                   (3, 16, 50_003), (3, 64, 200_001), (2, 33, 1_048_577),
                                   (3, 16, 1_000_000)])
def test_pp_matches_oracle(km, d, K, N):
    log(f"pp d={d} K={K} N={N}")
    s = datagen.spec("C2", N=N, d=d, K=max(K, 2), seed=6000 + K + N)
    X, _ = datagen.generate(s)
    Xd = torch.from_numpy(X).cuda()
    for rep in range(3):
        u = np.random.default_rng(100 * rep + K).random(K)
        cen, idx = km.pp_init(Xd, K, u=u, return_index=True)
        ref = seeding.kmeanspp(X, N, K, u)
        np.testing.assert_array_equal(idx, ref)
        np.testing.assert_array_equal(cen, seeding.centres(X, ref))


def test_pp_padded_rows(km):
    N, ld, K = 70_001, 70_016, 12
    s = datagen.spec("C2", N=N, d=3, K=K, seed=6100)
    X, _ = datagen.generate(s)
    Xp = np.zeros((3, ld), np.float32)
    Xp[:, :N] = X
    Xp[:, N:] = 1e6        # padding must never be read as points
    u = np.random.default_rng(3).random(K)
    idx = km.pp_init(torch.from_numpy(Xp).cuda(), K, u=u, N=N, return_index=True)[1]
    np.testing.assert_array_equal(idx, seeding.kmeanspp(X, N, K, u))


def test_pp_duplicates_and_ties(km):
    # Integer grid with many duplicates: equal D^2 everywhere, exact zeros.
    rng = np.random.default_rng(4)
    N = 100_003
    X = rng.integers(-3, 4, size=(3, N)).astype(np.float32)
    for K in (8, 64):
        u = rng.random(K)
        idx = km.pp_init(torch.from_numpy(X).cuda(), K, u=u, return_index=True)[1]
        np.testing.assert_array_equal(idx, seeding.kmeanspp(X, N, K, u))


def test_pp_all_points_equal(km):
    X = np.full((2, 5000), -1.25, np.float32)
    u = np.array([0.3, 0.6, 0.9])
    idx = km.pp_init(torch.from_numpy(X).cuda(), 3, u=u, return_index=True)[1]
    np.testing.assert_array_equal(idx, [1500, 3000, 4500])


def test_pp_repeatable(km):
    s = datagen.spec("C5", N=300_000, seed=6200)
    X, _ = datagen.generate(s)
    Xd = torch.from_numpy(X).cuda()
    a = km.pp_init(Xd, 16, seed=5, return_index=True)[1]
    b = km.pp_init(Xd, 16, seed=5, return_index=True)[1]
    np.testing.assert_array_equal(a, b)


def test_pp_errors(km):
    from paper_2405_12052_amd import KMeansError
    X = np.random.default_rng(5).normal(size=(3, 1000)).astype(np.float32)
    Xd = torch.from_numpy(X).cuda()
    with pytest.raises(KMeansError):
        km.pp_init(Xd, 3, u=[0.1, 1.0, 0.2])
    with pytest.raises(KMeansError):
        km.pp_init(Xd, 3, u=[0.1, -0.5, 0.2])
    with pytest.raises(KMeansError):
        km.pp_init(Xd, 65, seed=1)
    X[2, 17] = np.nan
    with pytest.raises(KMeansError):
        km.pp_init(torch.from_numpy(X).cuda(), 4, seed=1)
    # the context stays usable
    X[2, 17] = 0.0
    idx = km.pp_init(torch.from_numpy(X).cuda(), 4, u=[0.2, 0.4, 0.6, 0.8], return_index=True)[1]
    np.testing.assert_array_equal(idx, seeding.kmeanspp(X, 1000, 4, [0.2, 0.4, 0.6, 0.8]))
