"""The two reassignment scans (keys on the vector ALUs, KM_OPT_KEYS = 1, and
on the matrix cores, KM_OPT_KEYS = 2) must give identical labels, centres, E
and T, in the 2-D/3-D kernels and in the general-shape kernels (widths 8 to
16): both certify only winners that are the first-index float64 direct-form
argmin and re-scan the rest in that form.  Only the objective's float64
summation order differs.  (Parity of the default scans with the oracle is
covered by the other GPU test files.)"""
import numpy as np
import pytest

import datagen
import oracle
from parity import label_check

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def km():
    from paper_2405_12052_amd import KMeans
    k = KMeans(0)
    yield k
    k.set_option(5, 0)
    k.close()


def log(*a):
    print(*a, flush=True)


def both(km, fn):
    from paper_2405_12052_amd import KM_OPT_KEYS
    out = []
    for keys in (1, 2):
        km.set_option(KM_OPT_KEYS, keys)
        out.append(fn())
    km.set_option(KM_OPT_KEYS, 0)
    return out


@pytest.mark.parametrize("name,d,K,N", [
    ("C3", 3, 64, 1_000_003), ("C2", 3, 17, 300_001), ("C2", 2, 33, 200_001),
    ("C2", 3, 32, 100_000), ("C2", 2, 64, 5_003), ("C2", 3, 4, 70_001), ("C2", 3, 16, 1)])
def test_fit_identical_across_scans(km, name, d, K, N):
    log(f"keys fit {name} d={d} K={K} N={N}")
    kw = {"N": N, "K": K} if name == "C2" else {"N": N}
    if name == "C2":
        kw["d"] = d
    s = datagen.spec(name, seed=7100 + K + N, **kw)
    X, _ = datagen.generate(s)
    Xd = torch.from_numpy(X).cuda()
    Kf = min(K, N)
    mu0 = datagen.init_sample(X, N, Kf, 3)
    a, b = both(km, lambda: km.fit(Xd, mu0, tol=1e-6, max_iter=30))
    assert a.iters == b.iters
    assert np.array_equal(a.centroids, b.centroids)
    assert a.E == b.E
    assert np.array_equal(a.labels.cpu().numpy(), b.labels.cpu().numpy())
    assert b.objective == pytest.approx(a.objective, rel=1e-9)
    # and the matrix-core scan against the oracle on the final centres
    mism, near, _, _ = label_check(b.labels.cpu().numpy(), X, b.centroids, N)
    log(f"  T={b.iters} mismatches vs oracle {mism} (near-ties {near})")


@pytest.mark.parametrize("d", [2, 3])
def test_assign_ties_identical_across_scans(km, d):
    """Tie-heavy integer grid: many points fail both certificates and take
    the direct-form re-scan with its lowest-index rule."""
    rng = np.random.default_rng(70 + d)
    N, K = 200_003, 48
    X = rng.integers(-5, 6, size=(d, N)).astype(np.float32)
    mu = (rng.integers(-5, 5, size=(K, d)) + 0.5).astype(np.float64)
    mu[:, 0] = np.round(mu[:, 0])
    Xd = torch.from_numpy(X).cuda()
    (la, Ja), (lb, Jb) = both(km, lambda: km.assign(Xd, mu))
    ref, dmin, dsec = oracle.assign(X, mu)
    assert (dsec == dmin).mean() > 0.1
    assert np.array_equal(la.cpu().numpy(), ref)
    assert np.array_equal(lb.cpu().numpy(), ref)
    assert Jb == pytest.approx(Ja, rel=1e-12)


def test_far_points_and_large_offsets(km):
    """Points far from every centre and data offset from the origin: keys
    are dominated by |m|^2 and 2 m.x, the regime where the rounding bound
    matters most.  This case caught a runner-up bound that allowed for the
    index bits of another triple's packed minimum only when it undercut the
    winning triple's second key: 45 points were mislabelled once the key
    bound was made tight."""
    rng = np.random.default_rng(80)
    N, K = 150_001, 40
    X = (rng.normal(size=(3, N)) * 3 + 1000.0).astype(np.float32)
    X[:, ::97] += 5000.0                   # a sprinkle of far outliers
    mu = (rng.normal(size=(K, 3)) * 3 + 1000.0)
    Xd = torch.from_numpy(X).cuda()
    (la, _), (lb, _) = both(km, lambda: km.assign(Xd, mu))
    assert np.array_equal(la.cpu().numpy(), lb.cpu().numpy())
    mism, near, _, _ = label_check(lb.cpu().numpy(), X, mu, N)
    log(f"  far/offset: mismatches vs oracle {mism} (near-ties {near})")


def test_unaligned_rows_identical_across_scans(km):
    N, ld, K = 90_001, 90_003, 37
    s = datagen.spec("C2", N=N, K=K, seed=7200)
    X, _ = datagen.generate(s)
    buf = torch.zeros(3 * ld + 1, dtype=torch.float32, device="cuda")
    Xu = buf[1:1 + 3 * ld].view(3, ld)      # rows 4 bytes off 16-byte alignment
    Xu[:, :N] = torch.from_numpy(X).cuda()
    mu0 = datagen.init_sample(X, N, K, 5)
    a, b = both(km, lambda: km.fit(Xu, mu0, tol=1e-6, max_iter=20, N=N))
    assert a.iters == b.iters
    assert np.array_equal(a.centroids, b.centroids)
    assert np.array_equal(a.labels.cpu().numpy(), b.labels.cpu().numpy())


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("xs,ms", [(1e-15, 1e-15), (1e-3, 1e-3), (1e4, 1e4), (1e15, 1e15),
                                   (1.0, 1e6), (1e6, 1.0), (1.0, 0.0)])
def test_scales_identical_across_scans(km, d, xs, ms):
    """Data and centres at extreme magnitudes, and centres far larger or
    smaller than the data: the matrix-core scan scales both operands by
    powers of two before splitting them, and must still certify only exact
    winners (ms = 0: every centre at the origin, all keys tie)."""
    rng = np.random.default_rng(90 + d)
    N, K = 60_001, 64
    X = (rng.normal(size=(d, N)) * xs).astype(np.float32)
    mu = rng.normal(size=(K, d)) * ms
    log(f"  scales d={d} data {xs:g} centres {ms:g}")
    Xd = torch.from_numpy(X).cuda()
    (la, Ja), (lb, Jb) = both(km, lambda: km.assign(Xd, mu))
    a, b = la.cpu().numpy(), lb.cpu().numpy()
    assert np.array_equal(a, b)
    mism, near, _, _ = label_check(b, X, mu, N)
    log(f"    mismatches vs oracle {mism} (near-ties {near})")
    assert Jb == pytest.approx(Ja, rel=1e-12)


# ------------------------------------------------------------ general shapes
# The general-shape kernels take the matrix-core keys for widths 8 to 16
# (KM_OPT_KEYS = 0: K >= 64; 2: any K whose operands fit in LDS).

@pytest.mark.parametrize("d,K,N", [
    (16, 256, 100_003), (8, 100, 60_001), (12, 300, 40_001), (9, 64, 50_000),
    (13, 128, 30_011), (16, 40, 20_000), (16, 5, 7), (11, 1, 100), (16, 33, 64)])
def test_general_fit_identical_across_scans(km, d, K, N):
    log(f"general keys fit d={d} K={K} N={N}")
    s = datagen.spec("C2", N=N, d=d, K=K, seed=7300 + d + K)
    X, _ = datagen.generate(s)
    Xd = torch.from_numpy(X).cuda()
    mu0 = datagen.init_sample(X, N, K, 3)
    a, b = both(km, lambda: km.fit(Xd, mu0, tol=1e-6, max_iter=30))
    assert a.iters == b.iters
    assert np.array_equal(a.centroids, b.centroids)
    assert a.E == b.E
    assert np.array_equal(a.labels.cpu().numpy(), b.labels.cpu().numpy())
    assert b.objective == pytest.approx(a.objective, rel=1e-9)
    mism, near, _, _ = label_check(b.labels.cpu().numpy(), X, b.centroids, N)
    log(f"  T={b.iters} mismatches vs oracle {mism} (near-ties {near})")


@pytest.mark.parametrize("d", [8, 16])
def test_general_ties_identical_across_scans(km, d):
    """Integer points and half-integer centres: exact ties everywhere, which
    the matrix-core certificate must reject (the float64 re-scan then takes
    the lowest index)."""
    rng = np.random.default_rng(170 + d)
    N, K = 100_003, 96
    X = rng.integers(-3, 4, size=(d, N)).astype(np.float32)
    mu = (rng.integers(-3, 3, size=(K, d)) + 0.5).astype(np.float64)
    mu[:, : d // 2] = np.round(mu[:, : d // 2])
    Xd = torch.from_numpy(X).cuda()
    (la, Ja), (lb, Jb) = both(km, lambda: km.assign(Xd, mu))
    ref, dmin, dsec = oracle.assign(X, mu)
    assert (dsec == dmin).mean() > 0.05
    assert np.array_equal(la.cpu().numpy(), ref)
    assert np.array_equal(lb.cpu().numpy(), ref)
    assert Jb == pytest.approx(Ja, rel=1e-12)


def test_general_far_points_and_large_offsets(km):
    rng = np.random.default_rng(180)
    d, N, K = 16, 120_001, 200
    X = (rng.normal(size=(d, N)) * 3 + 1000.0).astype(np.float32)
    X[:, ::97] += 5000.0
    mu = rng.normal(size=(K, d)) * 3 + 1000.0
    Xd = torch.from_numpy(X).cuda()
    (la, _), (lb, _) = both(km, lambda: km.assign(Xd, mu))
    assert np.array_equal(la.cpu().numpy(), lb.cpu().numpy())
    mism, near, _, _ = label_check(lb.cpu().numpy(), X, mu, N)
    log(f"  general far/offset: mismatches vs oracle {mism} (near-ties {near})")


@pytest.mark.parametrize("xs,ms", [(1e-15, 1e-15), (1e-3, 1e-3), (1e4, 1e4), (1e15, 1e15),
                                   (1.0, 1e6), (1e6, 1.0), (1.0, 0.0)])
def test_general_scales_identical_across_scans(km, xs, ms):
    """Extreme magnitudes in 12-D (beyond the matrix-core scale's range every
    point goes to the float64 re-scan; ms = 0: all keys tie)."""
    rng = np.random.default_rng(190)
    d, N, K = 12, 30_001, 70
    X = (rng.normal(size=(d, N)) * xs).astype(np.float32)
    mu = rng.normal(size=(K, d)) * ms
    log(f"  general scales data {xs:g} centres {ms:g}")
    Xd = torch.from_numpy(X).cuda()
    (la, Ja), (lb, Jb) = both(km, lambda: km.assign(Xd, mu))
    a, b = la.cpu().numpy(), lb.cpu().numpy()
    assert np.array_equal(a, b)
    mism, near, _, _ = label_check(b, X, mu, N)
    log(f"    mismatches vs oracle {mism} (near-ties {near})")
    assert Jb == pytest.approx(Ja, rel=1e-12)


def test_general_unaligned_rows_identical_across_scans(km):
    d, N, ld, K = 12, 50_001, 50_003, 80
    s = datagen.spec("C2", N=N, d=d, K=K, seed=7400)
    X, _ = datagen.generate(s)
    buf = torch.zeros(d * ld + 1, dtype=torch.float32, device="cuda")
    Xu = buf[1:1 + d * ld].view(d, ld)
    Xu[:, :N] = torch.from_numpy(X).cuda()
    mu0 = datagen.init_sample(X, N, K, 5)
    a, b = both(km, lambda: km.fit(Xu, mu0, tol=1e-6, max_iter=20, N=N))
    assert a.iters == b.iters
    assert np.array_equal(a.centroids, b.centroids)
    assert np.array_equal(a.labels.cpu().numpy(), b.labels.cpu().numpy())
