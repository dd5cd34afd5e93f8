"""GPU parity of the general-shape path (d outside {2, 3}, K > 64, or
KM_OPT_WIDE) through the C ABI against the FP64 oracle: reassignment, step
by step updates, whole fits, the cross-check with the 2-D/3-D kernels on the
shapes both take, determinism, edge cases, errors, and sampled checks at the
benchmark's full size."""
import numpy as np
import pytest

import datagen
import oracle
from parity import centre_check, e_check, e_tol, gap_for_dim, label_check

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


def mixture(N, d, K, seed):
    s = datagen.spec("C2", N=N, d=d, K=K, seed=seed)
    X, _ = datagen.generate(s)
    return s, X, torch.from_numpy(X).cuda()


# --------------------------------------------------------------- reassignment
@pytest.mark.parametrize("d,K,N", [
    (1, 70, 10_001), (2, 100, 50_003), (3, 1024, 30_001), (4, 65, 20_000), (5, 200, 40_007),
    (8, 585, 20_003), (12, 300, 10_001), (16, 309, 25_001), (24, 210, 9_999), (32, 159, 12_345),
    (16, 3, 5), (7, 1, 1), (9, 128, 130),
    # beyond one block's LDS: the tiled kernels (several tiles, ragged last tile)
    (16, 310, 9_001), (16, 2048, 30_001), (32, 512, 10_001), (3, 4096, 20_011), (8, 1700, 7_777)])
def test_assign_matches_oracle(km, d, K, N):
    log(f"wide assign d={d} K={K} N={N}")
    s, X, Xd = mixture(N, d, max(K, 2), 5000 + d * 1000 + K)
    mu = X[:, np.random.default_rng(d + K).integers(0, N, K)].T.astype(np.float64)
    mu += np.random.default_rng(1).normal(size=mu.shape) * 0.37   # centres off the data
    lab, J = km.assign(Xd, mu)
    mism, near, _, dmin = label_check(lab.cpu().numpy(), X, mu)
    ref = dmin.sum()
    assert abs(J - ref) <= gap_for_dim(d) * ref + 1e-12
    log(f"  mismatches {mism} (near-ties {near})")


def test_exact_ties_go_to_the_lowest_index(km):
    """Integer points and centres on a half-integer grid in 6-D: many points
    are exactly equidistant from several centres (all distances are exact in
    float32 here), so the first index must win, as in the oracle."""
    rng = np.random.default_rng(61)
    d, N, K = 6, 100_003, 90
    X = rng.integers(-3, 4, size=(d, N)).astype(np.float32)
    mu = (rng.integers(-3, 3, size=(K, d)) + 0.5).astype(np.float64)
    mu[:, :3] = np.round(mu[:, :3])
    lab, J = km.assign(torch.from_numpy(X).cuda(), mu)
    ref, dmin, dsec = oracle.assign(X, mu)
    assert (dsec == dmin).mean() > 0.1
    assert np.array_equal(lab.cpu().numpy(), ref)
    assert J == pytest.approx(dmin.sum(), rel=1e-12)


def test_far_points_and_large_offsets(km):
    """Data far from the origin and a sprinkle of far outliers in 8-D: the
    keys are dominated by |m|^2 / 2 and m.x, and the direct form by |x|^2,
    the regime where the certificate's bounds matter most."""
    rng = np.random.default_rng(81)
    d, N, K = 8, 150_001, 150
    X = (rng.normal(size=(d, N)) * 3 + 1000.0).astype(np.float32)
    X[:, ::97] += 5000.0
    mu = rng.normal(size=(K, d)) * 3 + 1000.0
    lab, J = km.assign(torch.from_numpy(X).cuda(), mu)
    mism, near, _, dmin = label_check(lab.cpu().numpy(), X, mu)
    assert abs(J - dmin.sum()) <= gap_for_dim(d) * dmin.sum()
    log(f"  far/offset 8-D: mismatches vs oracle {mism} (near-ties {near})")


# -------------------------------------------------------------- step parity
@pytest.mark.parametrize("d,K,N,steps", [(5, 70, 60_001, 8), (16, 256, 40_000, 6),
                                         (3, 500, 80_001, 6), (32, 100, 20_001, 5),
                                         (1, 129, 10_000, 8),
                                         (16, 2048, 30_000, 3), (32, 512, 20_001, 3),
                                         (2, 4096, 60_001, 3)])
def test_stepwise_parity(km, d, K, N, steps):
    """Each update from the GPU's float64 centres mu^t: labels against the
    oracle's reassignment, mu^{t+1}, E and the empty-cluster count against the
    oracle's mean step on those labels."""
    s, X, Xd = mixture(N, d, K, 7000 + d + K)
    mu = datagen.init_sample(X, N, K, 3)
    worst_c = worst_e = 0.0
    total = 0
    for t in range(steps):
        lab, _ = km.assign(Xd, mu)
        gl = lab.cpu().numpy()
        mism, _, _, _ = label_check(gl, X, mu)
        total += mism
        r = km.fit(Xd, mu, tol=0.0, max_iter=1, labels=False)
        ref = oracle.update(X, gl, mu)
        worst_c = max(worst_c, centre_check(r.centroids, ref["mu"]))
        worst_e = max(worst_e, e_check(r.E, ref["E"]))
        assert r.iters == 1 and r.empty_events == ref["empty"]
        mu = r.centroids
    log(f"d={d} K={K}: {steps} steps, max centre err {worst_c:.2e}, max |dE| {worst_e:.2e}, "
        f"label mismatches {total}")


# ---------------------------------------------------------------- end to end
@pytest.mark.parametrize("d,K,N", [(5, 70, 20_000), (16, 100, 20_000), (2, 200, 30_000),
                                   (32, 40, 8_000), (4, 16, 50_001),
                                   (16, 700, 15_000), (32, 300, 6_000)])
def test_fit_end_to_end(km, d, K, N):
    s, X, Xd = mixture(N, d, K, 9000 + d + K)
    mu0 = datagen.init_sample(X, N, K, 4)
    r = km.fit(Xd, mu0, tol=1e-6, max_iter=80)
    ref = oracle.fit(X, mu0, tol=1e-6, max_iter=80)
    log(f"d={d} K={K}: T gpu {r.iters} oracle {ref['T']}, E {r.E:.3e}/{ref['E']:.3e}, "
        f"J {r.objective:.9e}/{ref['J']:.9e}")
    assert r.iters == ref["T"] and r.converged == ref["converged"]
    centre_check(r.centroids, ref["mu"])
    e_check(r.E, ref["E"])
    assert abs(r.objective - ref["J"]) <= gap_for_dim(d) * ref["J"]
    assert r.empty_events == ref["empty_events"]
    label_check(r.labels.cpu().numpy(), X, r.centroids)
    Eh, Jh = km.history()
    assert len(Eh) == r.iters
    assert all(abs(a - b) <= e_tol(b) for a, b in zip(Eh, ref["E_hist"]))
    assert np.all(np.abs(Jh - ref["J_hist"]) <= gap_for_dim(d) * ref["J_hist"])


# --------------------------------- the two implementations on shared shapes
@pytest.mark.parametrize("d,K,N", [(2, 1, 1), (3, 16, 100_003), (2, 64, 50_000), (3, 64, 200_001),
                                   (3, 5, 7)])
def test_general_kernels_equal_the_2d_3d_kernels(km, d, K, N):
    """KM_OPT_WIDE runs the general-shape kernels on a shape the 2-D/3-D
    kernels also take: both give the first-index minimum of the float64
    direct form and the same exact integer sums, so labels, centres and T are
    identical."""
    from paper_2405_12052_amd import KM_OPT_WIDE
    s, X, Xd = mixture(N, d, max(K, 2), 11_000 + d + K + N)
    mu0 = datagen.init_sample(X, N, K, 6)
    a = km.fit(Xd, mu0, tol=1e-6, max_iter=40)
    km.set_option(KM_OPT_WIDE, 1)
    try:
        b = km.fit(Xd, mu0, tol=1e-6, max_iter=40)
        la, Ja = km.assign(Xd, a.centroids)
    finally:
        km.set_option(KM_OPT_WIDE, 0)
    lb, Jb = km.assign(Xd, a.centroids)
    assert a.iters == b.iters and a.empty_events == b.empty_events
    assert np.array_equal(a.centroids, b.centroids)
    assert np.array_equal(a.labels.cpu().numpy(), b.labels.cpu().numpy())
    assert np.array_equal(la.cpu().numpy(), lb.cpu().numpy())
    assert b.E == pytest.approx(a.E, rel=1e-12, abs=1e-300)
    assert Jb == pytest.approx(Ja, rel=1e-12)


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("xs,ms", [(1e6, 1.0), (1.0, 1e6), (1e-15, 1e-15), (1e15, 1e15)])
def test_general_and_2d_3d_labels_equal_at_extreme_scales(km, d, xs, ms):
    """Data far from small centres (the float32 direct form errs by more than
    many key gaps), centres far from the data, and extreme magnitudes: the
    two implementations certify different sets of points, yet both give the
    first-index float64 minimum, so their labels are identical and equal the
    oracle's."""
    from paper_2405_12052_amd import KM_OPT_WIDE
    rng = np.random.default_rng(120 + d)
    N, K = 50_001, 64
    X = (rng.normal(size=(d, N)) * xs).astype(np.float32)
    mu = rng.normal(size=(K, d)) * ms
    log(f"  scales d={d} data {xs:g} centres {ms:g}")
    Xd = torch.from_numpy(X).cuda()
    la, Ja = km.assign(Xd, mu)
    km.set_option(KM_OPT_WIDE, 1)
    try:
        lb, Jb = km.assign(Xd, mu)
    finally:
        km.set_option(KM_OPT_WIDE, 0)
    a, b = la.cpu().numpy(), lb.cpu().numpy()
    assert np.array_equal(a, b)
    _, near, _, _ = label_check(a, X, mu)
    log(f"    identical, equal to the oracle's ({near} near-ties)")
    assert Jb == pytest.approx(Ja, rel=1e-12)


# -------------------------------------------------------------- determinism
def test_bitwise_repeat_and_grid_independence(km):
    from paper_2405_12052_amd import KM_OPT_BLOCKS, KM_OPT_GRAPH
    s, X, Xd = mixture(300_001, 12, 150, 12_345)
    mu0 = datagen.init_sample(X, s.N, 150, 9)
    outs = []
    for blocks, graph in ((0, 1), (0, 1), (1, 1), (37, 0), (1024, 1)):
        km.set_option(KM_OPT_BLOCKS, blocks)
        km.set_option(KM_OPT_GRAPH, graph)
        outs.append(km.fit(Xd, mu0, tol=0.0, max_iter=7))
    km.set_option(KM_OPT_BLOCKS, 0)
    km.set_option(KM_OPT_GRAPH, 1)
    a = outs[0]
    for b in outs[1:]:
        assert np.array_equal(a.centroids, b.centroids) and a.E == b.E and b.iters == 7
        assert np.array_equal(a.labels.cpu().numpy(), b.labels.cpu().numpy())


def test_tiled_bitwise_repeat_and_grid_independence(km):
    """The tiled kernels (centres staged through LDS tile by tile, sums added
    into each block's row in device memory): the same results for every grid
    and with or without graphs."""
    from paper_2405_12052_amd import KM_OPT_BLOCKS, KM_OPT_GRAPH
    s, X, Xd = mixture(50_001, 16, 1000, 2468)
    mu0 = datagen.init_sample(X, s.N, 1000, 3)
    outs = []
    for blocks, graph in ((0, 1), (0, 1), (1, 1), (37, 0), (512, 1)):
        km.set_option(KM_OPT_BLOCKS, blocks)
        km.set_option(KM_OPT_GRAPH, graph)
        outs.append(km.fit(Xd, mu0, tol=0.0, max_iter=4))
    km.set_option(KM_OPT_BLOCKS, 0)
    km.set_option(KM_OPT_GRAPH, 1)
    a = outs[0]
    for b in outs[1:]:
        assert np.array_equal(a.centroids, b.centroids) and a.E == b.E and b.iters == 4
        assert np.array_equal(a.labels.cpu().numpy(), b.labels.cpu().numpy())
    label_check(a.labels.cpu().numpy(), X, a.centroids)


def test_tiled_empty_clusters_and_tiny(km):
    """K beyond the LDS limit with far-away centres that stay empty, and a
    tiled shape with fewer points than a block takes."""
    d, N, K = 16, 20_000, 400
    s, X, Xd = mixture(N, d, K, 97)
    mu0 = datagen.init_sample(X, N, K - 3, 5)
    mu0 = np.vstack([mu0, np.full((3, d), 1e5) + np.arange(3)[:, None]])
    r = km.fit(Xd, mu0, tol=1e-6, max_iter=40)
    ref = oracle.fit(X, mu0, tol=1e-6, max_iter=40)
    assert r.iters == ref["T"] and r.empty_events == ref["empty_events"] > 0
    centre_check(r.centroids, ref["mu"])
    e_check(r.E, ref["E"])
    assert np.array_equal(r.centroids[K - 3:], mu0[K - 3:])
    Xs = np.ascontiguousarray(X[:, :700])
    mu1 = Xs[:, :400].T.astype(np.float64)
    r1 = km.fit(torch.from_numpy(Xs).cuda(), mu1, tol=1e-6, max_iter=10)
    ref1 = oracle.fit(Xs, mu1, tol=1e-6, max_iter=10)
    assert r1.iters == ref1["T"]
    centre_check(r1.centroids, ref1["mu"])
    assert np.array_equal(r1.labels.cpu().numpy(), ref1["labels"])


def test_resume_equals_one_long_run(km):
    s, X, Xd = mixture(100_000, 6, 80, 777)
    mu0 = datagen.init_sample(X, s.N, 80, 2)
    a = km.fit(Xd, mu0, tol=0.0, max_iter=5, labels=False)
    b = km.fit(Xd, a.centroids, tol=0.0, max_iter=7)
    c = km.fit(Xd, mu0, tol=0.0, max_iter=12)
    assert np.array_equal(b.centroids, c.centroids) and b.E == c.E
    assert np.array_equal(b.labels.cpu().numpy(), c.labels.cpu().numpy())


# --------------------------------------------------------------- edge cases
@pytest.mark.parametrize("d,N", [(5, 1), (7, 2), (6, 3), (16, 5), (1, 7), (24, 4097), (4, 4098)])
def test_tiny_and_ragged(km, d, N):
    rng = np.random.default_rng(N + d)
    X = rng.normal(size=(d, N)).astype(np.float32) * 10
    K = min(N, 3)
    mu0 = X[:, :K].T.astype(np.float64)
    r = km.fit(torch.from_numpy(X).cuda(), mu0, tol=1e-6, max_iter=50)
    ref = oracle.fit(X, mu0, tol=1e-6, max_iter=50)
    assert r.iters == ref["T"]
    centre_check(r.centroids, ref["mu"])
    assert np.array_equal(r.labels.cpu().numpy(), ref["labels"])


def test_unaligned_rows_use_the_scalar_path(km):
    d, N, K = 6, 50_001, 90
    s, X, _ = mixture(N, d, K, 4242)
    big = np.zeros((d, N + 2), np.float32)
    big[:, 1:N + 1] = X
    Xd = torch.from_numpy(big).cuda()[:, 1:]            # row start off 16 bytes, odd ld
    assert Xd.data_ptr() % 16 != 0 and Xd.stride(0) % 4 != 0
    mu0 = datagen.init_sample(X, N, K, 1)
    r = km.fit(Xd, mu0, tol=1e-6, max_iter=30, N=N)
    a = km.fit(torch.from_numpy(X).cuda(), mu0, tol=1e-6, max_iter=30)
    assert np.array_equal(r.centroids, a.centroids) and r.iters == a.iters
    assert np.array_equal(r.labels.cpu().numpy(), a.labels.cpu().numpy())


def test_empty_clusters_and_duplicates(km):
    d, N, K = 4, 40_000, 70
    s, X, Xd = mixture(N, d, K, 31)
    mu0 = datagen.init_sample(X, N, K - 2, 8)
    mu0 = np.vstack([mu0, mu0[1:2], np.full((1, d), 1e6)])   # a duplicate and a far centre
    r = km.fit(Xd, mu0, tol=1e-6, max_iter=100)
    ref = oracle.fit(X, mu0, tol=1e-6, max_iter=100)
    assert r.iters == ref["T"] and r.empty_events == ref["empty_events"] > 0
    centre_check(r.centroids, ref["mu"])
    assert np.array_equal(r.centroids[K - 1], mu0[K - 1])


def test_k_equals_n_and_k1(km):
    X = np.random.default_rng(0).normal(size=(5, 100)).astype(np.float32)
    Xd = torch.from_numpy(X).cuda()
    r = km.fit(Xd, X.T.astype(np.float64), tol=1e-6, max_iter=5)
    assert r.iters == 1 and r.E < 1e-12 and np.array_equal(r.labels.cpu().numpy(), np.arange(100))
    r1 = km.fit(Xd, np.zeros((1, 5)), tol=1e-6, max_iter=5)
    ref = oracle.fit(X, np.zeros((1, 5)), tol=1e-6, max_iter=5)
    assert r1.iters == ref["T"] == 2
    centre_check(r1.centroids, ref["mu"])


def test_indicator_stability_stop_matches_oracle(km):
    s, X, Xd = mixture(30_000, 8, 90, 555)
    mu0 = datagen.init_sample(X, s.N, 90, 5)
    tiny = 5e-324
    r = km.fit(Xd, mu0, tol=tiny, max_iter=300)
    ref = oracle.fit(X, mu0, tol=tiny, max_iter=300)
    assert r.converged and r.E == 0.0 and r.iters == ref["T"]
    centre_check(r.centroids, ref["mu"])


def test_error_paths(km):
    from paper_2405_12052_amd import KM_EINVAL, KM_EUNSUPPORTED, KMeansError
    X = np.random.default_rng(0).normal(size=(16, 2000)).astype(np.float32)
    Xd = torch.from_numpy(X).cuda()
    with pytest.raises(KMeansError) as e:
        km.fit(Xd, np.zeros((4097, 16)))                 # K beyond the largest supported
    assert e.value.code == KM_EUNSUPPORTED
    X33 = torch.zeros((33, 100), dtype=torch.float32, device="cuda")
    with pytest.raises(KMeansError) as e:
        km.fit(X33, np.zeros((2, 33)))
    assert e.value.code == KM_EUNSUPPORTED
    Xn = X.copy()
    Xn[9, 1234] = np.nan
    mu = X[:, :70].T.astype(np.float64)
    with pytest.raises(KMeansError, match="NaN") as e:
        km.fit(torch.from_numpy(Xn).cuda(), mu)
    assert e.value.code == KM_EINVAL
    with pytest.raises(KMeansError) as e:
        km.assign(torch.from_numpy(Xn).cuda(), mu)
    assert e.value.code == KM_EINVAL
    r = km.fit(Xd, mu, tol=1e-6, max_iter=10)        # the context still works
    ref = oracle.fit(X, mu, tol=1e-6, max_iter=10)
    centre_check(r.centroids, ref["mu"])



@pytest.mark.parametrize("col, val, off", [(2001, np.nan, 0), (17, np.inf, 0), (1500, -np.inf, 1),
                                           (2002, np.nan, 1)])
def test_scan_stops_on_non_finite_coordinates(km, col, val, off):
    """The data scan reads rows 16 bytes at a time where they are aligned and
    one float at a time for the N % 4 tail and for unaligned rows; a NaN or
    infinity in either part stops the fit and the assignment with an error."""
    from paper_2405_12052_amd import KM_EINVAL, KMeansError
    N = 2003
    X = np.random.default_rng(2).normal(size=(16, N)).astype(np.float32)
    X[11, col] = val
    big = np.zeros((16, 2008), np.float32)            # ld % 4 == 0
    big[:, off:off + N] = X
    Xd = torch.from_numpy(big).cuda()[:, off:off + N]
    assert (Xd.data_ptr() % 16 != 0) == bool(off) and Xd.stride(0) == 2008
    mu = X[:, :40].T.astype(np.float64)
    mu[~np.isfinite(mu)] = 0.0
    with pytest.raises(KMeansError) as e:
        km.fit(Xd, mu, N=N)
    assert e.value.code == KM_EINVAL
    with pytest.raises(KMeansError) as e:
        km.assign(Xd, mu, N=N)
    assert e.value.code == KM_EINVAL


# ------------------------------------------- the benchmark's shape, sampled
@pytest.fixture(scope="module")
def w1():
    s = datagen.spec("W1")
    X, _ = datagen.generate(s)
    return s, X, torch.from_numpy(X).cuda()


def test_full_size_sampled(km, w1):
    """W1 at full size (N = 1e7, d = 16, K = 256), the launch configuration the
    benchmark times: labels of a sample of points against the oracle, and the
    next update against the oracle's mean step on the GPU's (checked) labels
    over all N points."""
    s, X, Xd = w1
    mu0 = datagen.init_sample(X, s.N, s.K, s.init_seed)
    a = km.fit(Xd, mu0, tol=0.0, max_iter=3)
    gl = a.labels.cpu().numpy()
    idx = np.sort(np.random.default_rng(3).choice(s.N, 20_000, replace=False))
    mism, near, _, _ = label_check(gl[idx], np.ascontiguousarray(X[:, idx]), a.centroids)
    b = km.fit(Xd, mu0, tol=0.0, max_iter=4, labels=False)
    ref = oracle.update(X, gl, a.centroids)
    err = centre_check(b.centroids, ref["mu"])
    e_check(b.E, ref["E"])
    assert b.empty_events - a.empty_events == ref["empty"]
    log(f"W1 full size: sampled label mismatches {mism} (near-ties {near}), centre err {err:.2e}")
