"""The per-cluster sums (the numerators of the mean step in the paper's "The
Lloyd's Algorithm") on inputs that stress their fixed-point form, in all three
implementations: the 2-D/3-D kernels, the general-shape kernels (KM_OPT_WIDE)
and the batched persistent fit.

* A tight cluster near the origin beside one far point: the far point sets
  the magnitude of the data, and with it the grid every coordinate is
  rounded to; the cluster's mean must still be within the centre tolerance
  and E within its bound of the oracle's.
* Data with max|x| >= 2^28, beyond the range in which the sums guarantee the
  centre tolerance: fits refuse it (KM_EUNSUPPORTED); reassignment alone,
  which takes no sums, still works.
* More points than one block may add into its int64 slots (2^19): a grid
  forced to one block is raised, a batched instance on single blocks is taken
  in chunks; the results must equal the default schedule's bit for bit.
"""
import numpy as np
import pytest

import oracle
from parity import centre_check, e_check, label_check

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


def tight_and_far(far, d=3):
    """5000 copies of (0.3, ..., 0.3), 3000 of a second point near the origin,
    and one point at (far, ..., far)."""
    X = np.empty((d, 8001), np.float32)
    X[:, :5000] = 0.3
    X[:, 5000:8000] = np.array([-0.7, 0.1, 0.55][:d], np.float32)[:, None]
    X[:, 8000] = far
    return X


def inits(X, far):
    d = X.shape[0]
    at_means = X[:, [0, 5000, 8000]].T.astype(np.float64)
    off = np.array([[0.0] * d, [-1.0] * d, [far * 0.5] * d], np.float64)
    return [at_means, off]


def run_path(km, path, Xd, mu0, tol, max_iter):
    """A fit through one of the three implementations, as (centroids, E, T)."""
    from paper_2405_12052_amd import KM_OPT_WIDE
    if path == "batched":
        out = km.fit_batched([(Xd, Xd.shape[1], mu0[None])], tol=tol, max_iter=max_iter,
                             labels=False)[0]
        return out["centroids"], out["E"], out["iters"]
    km.set_option(KM_OPT_WIDE, 1 if path == "wide" else 0)
    try:
        r = km.fit(Xd, mu0, tol=tol, max_iter=max_iter, labels=False)
    finally:
        km.set_option(KM_OPT_WIDE, 0)
    return r.centroids, r.E, r.iters


PATHS = ["single", "wide", "batched"]


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("far", [2e4, 1e5, 1e6])
def test_tight_cluster_beside_a_far_point(km, path, far):
    X = tight_and_far(far)
    Xd = torch.from_numpy(X).cuda()
    for q, mu0 in enumerate(inits(X, far)):
        log(f"{path}: far point {far:g}, init {q}")
        # one update against the oracle's update from the same centres
        c, E, T = run_path(km, path, Xd, mu0, 0.0, 1)
        ref = oracle.step(X, mu0)
        err = centre_check(c, ref["mu"])
        de = e_check(E, ref["E"], ref["mu"])
        assert T == 1
        # and a whole fit against the oracle's fit
        c2, E2, T2 = run_path(km, path, Xd, mu0, 1e-6, 50)
        ref2 = oracle.fit(X, mu0, tol=1e-6, max_iter=50, labels=False)
        assert T2 == ref2["T"]
        err2 = centre_check(c2, ref2["mu"])
        e_check(E2, ref2["E"], ref2["mu"])
        log(f"  step: centre err {err:.2e}, |dE| {de:.2e}; fit: T={T2}, centre err {err2:.2e}")


@pytest.mark.parametrize("d", [2, 3])
def test_tight_cluster_error_far_below_tolerance(km, d):
    """The bound behind the design: each mean coordinate within
    2^(ilogb(max|x|) - 44) of the exact mean.  With max|x| = 1e6 that is
    2^-25 < 3e-8, so the cluster at 0.3 must come out within 1e-7."""
    X = tight_and_far(1e6, d)
    Xd = torch.from_numpy(X).cuda()
    mu0 = inits(X, 1e6)[0]
    ref = oracle.step(X, mu0)
    for path in PATHS:
        c, _, _ = run_path(km, path, Xd, mu0, 0.0, 1)
        assert np.abs(c - ref["mu"]).max() <= 2.0 ** -25, (path, np.abs(c - ref["mu"]).max())


@pytest.mark.parametrize("path", PATHS)
def test_data_beyond_the_range_are_refused(km, path):
    from paper_2405_12052_amd import KMeansError
    X = tight_and_far(3.0e8)          # max|x| >= 2^28
    Xd = torch.from_numpy(X).cuda()
    mu0 = inits(X, 3.0e8)[0]
    with pytest.raises(KMeansError) as e:
        run_path(km, path, Xd, mu0, 1e-6, 10)
    assert e.value.code == -5, e.value           # KM_EUNSUPPORTED
    assert "2^28" in str(e.value)
    # the context stays usable, and reassignment alone still works
    lab, _ = km.assign(Xd, mu0)
    label_check(lab.cpu().numpy(), X, mu0)
    Xs = tight_and_far(1e6)
    m = inits(Xs, 1e6)[0]
    c, _, _ = run_path(km, path, torch.from_numpy(Xs).cuda(), m, 0.0, 1)
    centre_check(c, oracle.step(Xs, m)["mu"])


def blob_data(N, d, K, seed):
    rng = np.random.default_rng(seed)
    c = rng.uniform(-50, 50, size=(K, d))
    lab = rng.integers(0, K, size=N)
    X = (c[lab] + rng.normal(size=(N, d))).T.astype(np.float32)
    return np.ascontiguousarray(X), X[:, rng.choice(N, K, replace=False)].T.astype(np.float64)


@pytest.mark.parametrize("path", ["single", "wide"])
def test_one_block_grid_is_raised(km, path):
    """KM_OPT_BLOCKS = 1 with N = 1.3e6: one block would add all the points
    into its int64 slots; the grid is raised to N / 2^19 blocks and the result
    equals the default grid's bit for bit."""
    from paper_2405_12052_amd import KM_OPT_BLOCKS
    X, mu0 = blob_data(1_300_001, 3, 12, 5)
    Xd = torch.from_numpy(X).cuda()
    a = run_path(km, path, Xd, mu0, 0.0, 4)
    km.set_option(KM_OPT_BLOCKS, 1)
    try:
        b = run_path(km, path, Xd, mu0, 0.0, 4)
    finally:
        km.set_option(KM_OPT_BLOCKS, 0)
    assert np.array_equal(a[0], b[0]) and a[1] == b[1] and a[2] == b[2]
    ref = oracle.fit(X, mu0, tol=0.0, max_iter=4, labels=False)
    centre_check(a[0], ref["mu"])
    e_check(a[1], ref["E"], ref["mu"])


def test_batched_instance_in_chunks(km):
    """A batched instance of 1.2e6 points on single blocks (no teams) is taken
    in three chunks of at most 2^19 points whose sums are added in 128 bits;
    on teams of 4 it is one chunk per block.  Both equal the single fit."""
    X, mu0 = blob_data(1_200_003, 2, 9, 6)
    Xd = torch.from_numpy(X).cuda()
    inits2 = np.stack([mu0, mu0[::-1].copy()])
    single = [km.fit(Xd, m, tol=1e-6, max_iter=60, labels=False) for m in inits2]
    for team, big in ((1, 0.0), (4, 1.0)):
        km.set_batched_schedule(team_size=team, blocks_per_cu=2, big_work=big)
        try:
            out = km.fit_batched([(Xd, Xd.shape[1], inits2)], tol=1e-6, max_iter=60)[0]
        finally:
            km.set_batched_schedule(0, 0, 0.0)
        b = out["best_restart"]
        assert np.array_equal(out["centroids"], single[b].centroids), team
        assert out["iters"] == single[b].iters and out["E"] == single[b].E
        assert list(out["restart_iters"]) == [s.iters for s in single]
    ref = oracle.fit(X, inits2[b], tol=1e-6, max_iter=60, labels=False)
    assert ref["T"] == single[b].iters
    centre_check(single[b].centroids, ref["mu"])
