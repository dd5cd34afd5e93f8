"""Indicator tracking (KM_OPT_TRACK) on the GPU against the oracle's
fit_track: the per-update counts of changed labels, the stop after the first
update that changes none (the criterion of the paper's section "The Lloyd's
Algorithm"), and the centres and labels it ends with, in the 2-D/3-D kernels
(both scans) and the general-shape kernels."""
import numpy as np
import pytest

import datagen
import oracle
from parity import centre_check, label_check

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


def run(km, Xd, mu0, tol, max_iter, keys=0, wide=0, graph=1):
    from paper_2405_12052_amd import KM_OPT_GRAPH, KM_OPT_KEYS, KM_OPT_TRACK, KM_OPT_WIDE
    km.set_option(KM_OPT_TRACK, 1)
    km.set_option(KM_OPT_KEYS, keys)
    km.set_option(KM_OPT_WIDE, wide)
    km.set_option(KM_OPT_GRAPH, graph)
    try:
        r = km.fit(Xd, mu0, tol=tol, max_iter=max_iter)
        return r, km.changes()
    finally:
        km.set_option(KM_OPT_TRACK, 0)
        km.set_option(KM_OPT_KEYS, 0)
        km.set_option(KM_OPT_WIDE, 0)
        km.set_option(KM_OPT_GRAPH, 1)


def check(km, X, Xd, N, mu0, tol=0.0, max_iter=500, **kw):
    r, chg = run(km, Xd, mu0, tol, max_iter, **kw)
    o = oracle.fit_track(X, mu0, tol=tol, max_iter=max_iter, N=N)
    log(f"  T {r.iters} (oracle {o['T']}), changed {chg[:4].tolist()}... {chg[-3:].tolist()}")
    assert r.iters == o["T"] and bool(r.converged) == o["converged"]
    assert chg.tolist() == o["changed"].tolist()
    centre_check(r.centroids, o["mu"])
    lab = r.labels.cpu().numpy()
    if o["converged"] and o["changed"][-1] == 0:
        # stopped by the indicators: the final labels are the tracked ones
        assert np.array_equal(lab, o["labels"])
    label_check(lab, X, r.centroids, N)
    return r, chg


@pytest.mark.parametrize("name,kw,keys", [
    ("C5", dict(N=50_000, seed=91), 0),          # d = 3, K = 16: VALU keys
    ("C3", dict(N=100_003, seed=92), 0),         # d = 3, K = 64: matrix-core keys (2 tiles)
    ("C3", dict(N=100_003, seed=92), 1),         # the same on the VALU keys
    ("C2", dict(N=60_001, d=2, K=30, seed=93), 0),  # d = 2, K = 30: one matrix-core tile
])
def test_tracked_counts_match_oracle(km, name, kw, keys):
    log(f"track {name} {kw} keys={keys}")
    s = datagen.spec(name, **kw)
    X, _ = datagen.generate(s)
    Xd = torch.from_numpy(X).cuda()
    mu0 = datagen.init_sample(X, s.N, s.K, 5)
    r, chg = check(km, X, Xd, s.N, mu0, keys=keys)
    assert chg[0] == s.N


def test_tracked_stop_by_tolerance_first(km):
    """tol large enough to stop before the labels settle: the counts still
    follow the oracle's and the fit ends by E < tol."""
    s = datagen.spec("C5", N=40_000, seed=94)
    X, _ = datagen.generate(s)
    Xd = torch.from_numpy(X).cuda()
    mu0 = datagen.init_sample(X, s.N, s.K, 6)
    r, chg = check(km, X, Xd, s.N, mu0, tol=1e-2)
    assert r.converged and chg[-1] > 0


def test_tracked_without_graphs_and_at_max_iter(km):
    s = datagen.spec("C5", N=30_011, seed=95)
    X, _ = datagen.generate(s)
    Xd = torch.from_numpy(X).cuda()
    mu0 = datagen.init_sample(X, s.N, s.K, 7)
    r, chg = check(km, X, Xd, s.N, mu0, graph=0)
    r2, chg2 = check(km, X, Xd, s.N, mu0, max_iter=3)
    assert r2.iters == 3 and not r2.converged and chg2.tolist() == chg[:3].tolist()


@pytest.mark.parametrize("d,K,N,wide", [(5, 40, 30_000, 0), (16, 100, 20_001, 0), (3, 16, 25_000, 1),
                                        (16, 500, 12_001, 0)])
def test_tracked_general_shapes(km, d, K, N, wide):
    log(f"track general d={d} K={K} N={N} wide={wide}")
    s = datagen.spec("C2", N=N, d=d, K=K, seed=96 + d)
    X, _ = datagen.generate(s)
    Xd = torch.from_numpy(X).cuda()
    mu0 = datagen.init_sample(X, N, K, 8)
    check(km, X, Xd, N, mu0, wide=wide)


def test_tracking_errors(km):
    from paper_2405_12052_amd import KM_EINVAL, KM_OPT_TRACK, KMeansError
    X = np.random.default_rng(0).normal(size=(3, 1000)).astype(np.float32)
    Xd = torch.from_numpy(X).cuda()
    mu0 = X[:, :4].T.astype(np.float64)
    km.fit(Xd, mu0, tol=1e-6, max_iter=5)
    with pytest.raises(KMeansError) as e:
        km.changes()
    assert e.value.code == KM_EINVAL
    km.set_option(KM_OPT_TRACK, 1)
    try:
        with pytest.raises(KMeansError) as e:
            km.fit(Xd, mu0, tol=1e-6, max_iter=5, labels=False)
        assert e.value.code == KM_EINVAL
    finally:
        km.set_option(KM_OPT_TRACK, 0)
    with pytest.raises(KMeansError):
        km.set_option(KM_OPT_TRACK, 2)
