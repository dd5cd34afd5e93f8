"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Nothing here calls the GPU library.  Each test is chosen so that a plausible
slip in the oracle (a dropped coordinate, a sign, a transposed operand, E taken
as a norm instead of a squared norm, an off-by-one in the iteration count, a
wrong tie or empty-cluster rule, labels against the wrong centres) fails at
least one of them.  The definitions are those of the paper's section "The
Lloyd's Algorithm" (reassignment, mean calculation) and the error term and
tolerance test of "Serial Lloyd's Algorithm".
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle
import datagen

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def soa(points):
    return np.ascontiguousarray(np.asarray(points, dtype=np.float32).T)


# --------------------------------------------------------------- worked example
def test_worked_example_stepwise():
    g = json.load(open(os.path.join(GOLD, "worked_example_k2.json")))
    X = soa(g["points_xy"])
    mu = np.array(g["init"], np.float64)
    for s in g["steps"]:
        r = oracle.step(X, mu)
        assert r["labels"].tolist() == s["labels"], s["t"]
        assert np.array_equal(r["mu"], np.array(s["mu_next"], np.float64)), s["t"]
        assert r["E"] == s["E"], s["t"]
        assert r["J"] == s["J"], s["t"]
        mu = r["mu"]


def test_worked_example_fit():
    g = json.load(open(os.path.join(GOLD, "worked_example_k2.json")))
    X = soa(g["points_xy"])
    r = oracle.fit(X, np.array(g["init"], np.float64), tol=g["tol"], max_iter=100)
    assert r["T"] == g["T"]
    assert r["J"] == g["J_final"]
    assert r["converged"]
    assert r["E_hist"].tolist() == [s["E"] for s in g["steps"]]
    assert r["E_hist"].tolist() != g["sqrtE_reading_would_give"]
    assert r["J_hist"].tolist() == [s["J"] for s in g["steps"]]
    assert r["labels"].tolist() == g["steps"][-1]["labels"]


def test_tolerance_test_is_strict():
    # E reaches exactly 0 at the third update; with tol = 0 the strict test
    # E < tol never holds, so the loop runs to max_iter
    g = json.load(open(os.path.join(GOLD, "worked_example_k2.json")))
    X = soa(g["points_xy"])
    r = oracle.fit(X, np.array(g["init"], np.float64), tol=0.0, max_iter=7)
    assert r["T"] == 7 and not r["converged"] and r["E"] == 0.0
    r = oracle.fit(X, np.array(g["init"], np.float64), tol=10.0, max_iter=7)
    assert r["T"] == 3                      # E_1 = 10 is not < 10; E_2 = 0 is


def test_worked_example_max_iter_labels_against_final_centres():
    g = json.load(open(os.path.join(GOLD, "worked_example_k2.json")))
    X = soa(g["points_xy"])
    m = g["max_iter_1"]
    r = oracle.fit(X, np.array(g["init"], np.float64), tol=g["tol"], max_iter=1)
    assert r["T"] == 1 and not r["converged"]
    assert np.array_equal(r["mu"], np.array(m["mu"], np.float64))
    # labels are recomputed against mu^1, not the labels the update used
    assert r["labels"].tolist() == m["final_labels"]
    assert r["J"] == m["J_final"] and r["E"] == m["E"]


# ------------------------------------------------------------------- assignment
def test_exact_ties_go_to_lowest_index():
    # every point is equidistant from centres 1 and 2 (and farther from 0)
    X = soa([[1, 0], [1, 5], [1, -3]])
    mu = np.array([[-50, 0], [0, 0], [2, 0]], np.float64)
    lab, dmin, dsec = oracle.assign(X, mu)
    assert lab.tolist() == [1, 1, 1]
    assert np.array_equal(dmin, dsec)
    # reorder so that the tied pair is (0, 2): lowest index again
    lab, _, _ = oracle.assign(X, mu[[1, 0, 2]])
    assert lab.tolist() == [0, 0, 0]


@pytest.mark.parametrize("d,K", [(2, 7), (3, 7), (1, 9), (5, 70), (16, 12), (32, 3)])
def test_assign_brute_force_and_second_distance(d, K):
    rng = np.random.default_rng(5 + d * 100 + K)
    X = rng.normal(size=(d, 50)).astype(np.float32)
    mu = rng.normal(size=(K, d))
    lab, dmin, dsec = oracle.assign(X, mu, assign_f32=False)
    for i in range(50):
        D = [math.fsum((float(X[j, i]) - mu[k, j]) ** 2 for j in range(d)) for k in range(K)]
        order = sorted(range(K), key=lambda k: (D[k], k))
        assert lab[i] == order[0]
        assert math.isclose(dmin[i], D[order[0]], rel_tol=1e-14)
        assert math.isclose(dsec[i], D[order[1]], rel_tol=1e-14)


@pytest.mark.parametrize("d,K,grid", [(1, 5, False), (2, 7, False), (3, 64, False), (7, 9, False),
                                       (16, 12, False), (2, 6, True), (3, 10, True)])
def test_assign_f32_is_the_float64_direct_form_on_rounded_centres(d, K, grid):
    """The reassignment rule the library's labels must match bit for bit:
    centres rounded to float32, each point's squared distance summed left to
    right in float64 (every difference, square and partial sum rounded, no
    fused operations), first index of the minimum.  Written out here with
    Python floats (IEEE float64, one rounding per operation); the oracle's C
    code must give the same labels and the same minimum distances exactly,
    also on an integer grid full of exact ties."""
    rng = np.random.default_rng(40 + d * 10 + K)
    N = 60
    if grid:
        X = rng.integers(-3, 4, size=(d, N)).astype(np.float32)
        mu = rng.integers(-3, 3, size=(K, d)).astype(np.float64) + 0.5
        mu[: K // 2] = np.round(mu[: K // 2] - 0.5)
        mu[K - 1] = mu[0]                            # a duplicate: exact ties, first index wins
    else:
        X = (rng.normal(size=(d, N)) * 3).astype(np.float32)
        mu = rng.normal(size=(K, d)) * 3 + 1e-9
    lab, dmin, _ = oracle.assign(X, mu)              # assign_f32 defaults to True
    m32 = [[float(np.float32(mu[k, j])) for j in range(d)] for k in range(K)]
    ties = 0
    for i in range(N):
        best, arg = math.inf, 0
        dists = []
        for k in range(K):
            D = 0.0
            for j in range(d):
                t = float(X[j, i]) - m32[k][j]
                D = D + t * t
            dists.append(D)
            if D < best:
                best, arg = D, k
        ties += dists.count(best) > 1
        assert lab[i] == arg and (not grid or arg != K - 1)
        assert dmin[i] == best
    if grid:
        assert ties > 0


def test_assign_f32_rounds_only_the_centres():
    X = soa([[0.0, 0.0]])
    mu = np.array([[1.0 / 3.0, 0.0]])
    _, d64, _ = oracle.assign(X, mu, assign_f32=False)
    _, d32, _ = oracle.assign(X, mu, assign_f32=True)
    assert d64[0] == (1.0 / 3.0) ** 2
    assert d32[0] == float(np.float32(1.0 / 3.0)) ** 2


def test_sorted_1d_data_gives_contiguous_runs():
    rng = np.random.default_rng(1)
    x = np.sort(rng.uniform(-10, 10, 200)).astype(np.float32)
    X = np.stack([x, np.zeros_like(x)])
    mu = np.stack([np.sort(rng.uniform(-10, 10, 6)), np.zeros(6)], axis=1)
    lab, _, _ = oracle.assign(X, mu)
    assert np.all(np.diff(lab) >= 0)  # centres sorted -> labels non-decreasing


# ----------------------------------------------------------------------- update
def test_centroid_is_mean_of_assigned_points():
    rng = np.random.default_rng(2)
    for d, K in ((2, 4), (3, 9)):
        X = (rng.normal(size=(d, 3000)) * 30 + 7).astype(np.float32)
        mu = X[:, rng.choice(3000, K, replace=False)].T.astype(np.float64)
        r = oracle.step(X, mu)
        assert r["counts"].sum() == 3000
        for k in range(K):
            m = r["labels"] == k
            assert r["counts"][k] == m.sum()
            for j in range(d):
                ref = math.fsum(X[j, m].astype(np.float64)) / m.sum()
                assert math.isclose(r["mu"][k, j], ref, rel_tol=1e-12, abs_tol=1e-12)


def test_k1_global_mean_then_zero_error():
    X = soa([[0, 0], [1, 0], [0, 1]])            # mean (1/3, 1/3): not a float32
    r = oracle.fit(X, np.array([[5.0, 5.0]]), tol=1e-6, max_iter=10)
    assert r["T"] == 2 and r["converged"]
    assert np.array_equal(r["mu"], np.array([[1 / 3, 1 / 3]]))
    assert r["E_hist"][1] == 0.0                 # E uses the float64 centres
    assert r["labels"].tolist() == [0, 0, 0]


def test_empty_cluster_keeps_its_centre():
    rng = np.random.default_rng(3)
    X = rng.normal(size=(2, 100)).astype(np.float32)
    mu = np.array([[0.0, 0.0], [1e6, 1e6], [0.5, 0.0]])
    r = oracle.step(X, mu)
    assert r["counts"][1] == 0 and r["empty"] == 1
    assert np.array_equal(r["mu"][1], mu[1])
    f = oracle.fit(X, mu, tol=1e-9, max_iter=50)
    assert np.array_equal(f["mu"][1], mu[1])
    assert f["empty_events"] == f["T"]


# ------------------------------------------------------------------- invariants
def test_objective_never_increases():
    for seed in range(6):
        s = datagen.spec("C1", N=20_000, seed=100 + seed)
        X, _ = datagen.generate(s)
        for K in (3, 4, 9):
            mu0 = datagen.init_sample(X, s.N, K, seed)
            r = oracle.fit(X, mu0, tol=0.0, max_iter=40)
            J = np.append(r["J_hist"], r["J"])
            assert np.all(J[1:] <= J[:-1] * (1 + 1e-12)), (seed, K)


def test_translation_equivariance_exact():
    rng = np.random.default_rng(4)
    X = (np.round(rng.normal(size=(3, 400)) * 16) / 4).astype(np.float32)  # grid of 1/4
    mu0 = X[:, :5].T.astype(np.float64)
    a = oracle.fit(X, mu0, tol=1e-6, max_iter=100)
    c = np.array([64.0, -128.0, 32.0])
    b = oracle.fit((X + c[:, None].astype(np.float32)).astype(np.float32), mu0 + c,
                   tol=1e-6, max_iter=100)
    assert a["T"] == b["T"]
    assert np.array_equal(a["labels"], b["labels"])
    assert np.allclose(b["mu"] - c, a["mu"], rtol=0, atol=1e-12)


def test_point_permutation_invariance():
    rng = np.random.default_rng(6)
    X = rng.normal(size=(2, 1000)).astype(np.float32) * 5
    mu0 = X[:, :6].T.astype(np.float64)
    p = rng.permutation(1000)
    a = oracle.fit(X, mu0, tol=1e-6, max_iter=100)
    b = oracle.fit(np.ascontiguousarray(X[:, p]), mu0, tol=1e-6, max_iter=100)
    assert a["T"] == b["T"]
    assert np.array_equal(a["labels"][p], b["labels"])
    assert np.allclose(a["mu"], b["mu"], rtol=1e-13, atol=1e-13)


def test_layout_row_stride():
    rng = np.random.default_rng(7)
    X = rng.normal(size=(3, 101)).astype(np.float32)
    Xp = np.zeros((3, 128), np.float32)
    Xp[:, :101] = X
    Xp[:, 101:] = 1e9      # padding must never be read
    mu = X[:, :4].T.astype(np.float64)
    a = oracle.step(X, mu)
    b = oracle.step(Xp, mu, N=101)
    assert np.array_equal(a["mu"], b["mu"]) and a["E"] == b["E"]


# ------------------------------------------------------------------ brute force
def _fixed_points(P, K):
    """All labellings with every cluster non-empty that the reassignment step
    reproduces from their own means (lowest-index ties)."""
    N = len(P)
    out = []
    for lab in itertools.product(range(K), repeat=N):
        if len(set(lab)) != K:
            continue
        mu = [tuple(math.fsum(P[i][j] for i in range(N) if lab[i] == k) /
                    sum(1 for i in range(N) if lab[i] == k) for j in range(len(P[0])))
              for k in range(K)]
        ok = True
        for i in range(N):
            D = [math.fsum((P[i][j] - mu[k][j]) ** 2 for j in range(len(P[0]))) for k in range(K)]
            if min(range(K), key=lambda k: (D[k], k)) != lab[i]:
                ok = False
                break
        if ok:
            out.append((lab, mu))
    return out


def _cost(P, mu):
    return math.fsum(min(math.fsum((p[j] - m[j]) ** 2 for j in range(len(p))) for m in mu) for p in P)


@pytest.mark.parametrize("seed", range(8))
def test_brute_force_fixed_points(seed):
    rng = np.random.default_rng(1000 + seed)
    N = int(rng.integers(5, 9))
    K = int(rng.integers(2, 4))
    P = [tuple(float(v) for v in np.float32(rng.normal(size=2) * 3)) for _ in range(N)]
    X = soa(P)
    fps = _fixed_points(P, K)
    assert fps
    # the globally optimal partition is among the fixed points
    def partition_cost(lab):
        tot = []
        for k in range(K):
            idx = [i for i in range(N) if lab[i] == k]
            m = [math.fsum(P[i][j] for i in idx) / len(idx) for j in range(2)]
            tot += [(P[i][j] - m[j]) ** 2 for i in idx for j in range(2)]
        return math.fsum(tot)
    best = min((lab for lab in itertools.product(range(K), repeat=N) if len(set(lab)) == K),
               key=partition_cost)
    assert best in [f[0] for f in fps]
    # every (tie-free) fixed point is a strict local minimum of
    # f(mu) = sum_i min_k ||x_i - mu_k||^2 in centre space
    for lab, mu in fps:
        f0 = _cost(P, mu)
        for r in range(20):
            delta = rng.normal(size=(K, 2)) * 1e-4
            mu2 = [tuple(mu[k][j] + delta[k][j] for j in range(2)) for k in range(K)]
            assert _cost(P, mu2) >= f0 - 1e-12
        # and the oracle leaves it unchanged (E = 0, same labels)
        r1 = oracle.step(X, np.array(mu), assign_f32=False)
        assert tuple(r1["labels"].tolist()) == lab
        assert r1["E"] < 1e-24
    # Lloyd from any K distinct data points lands on an enumerated fixed point
    labs = {f[0] for f in fps}
    for init in itertools.combinations(range(N), K):
        mu0 = np.array([P[i] for i in init], np.float64)
        r = oracle.fit(X, mu0, tol=1e-12, max_iter=100, assign_f32=False)
        assert r["converged"]
        if len(set(r["labels"].tolist())) == K:
            assert tuple(r["labels"].tolist()) in labs


# --------------------------------------------------------------- blob recovery
def test_well_separated_blobs_recover_sample_means():
    rng = np.random.default_rng(8)
    d, C, n = 3, 6, 4000
    centres = np.array([[i * 40.0, (i % 2) * 40.0, -(i % 3) * 40.0] for i in range(C)])
    comp = rng.integers(0, C, n)
    X = (centres[comp] + rng.normal(size=(n, d))).astype(np.float32).T.copy()
    first = [int(np.flatnonzero(comp == c)[0]) for c in range(C)]
    mu0 = X[:, first].T.astype(np.float64)
    r = oracle.fit(X, mu0, tol=1e-6, max_iter=100)
    assert np.array_equal(r["labels"], comp)
    for c in range(C):
        for j in range(d):
            ref = math.fsum(X[j, comp == c].astype(np.float64)) / (comp == c).sum()
            assert math.isclose(r["mu"][c, j], ref, rel_tol=1e-12, abs_tol=1e-12)


# ----------------------------------------------------------- library cross-check
def test_scipy_kmeans2_same_iterates():
    from scipy.cluster.vq import kmeans2
    for seed, d, K in ((0, 2, 4), (1, 3, 7), (2, 3, 16), (3, 8, 80), (4, 1, 5), (5, 16, 20)):
        s = datagen.spec("C2", N=30_000, d=d, K=K, seed=300 + seed)
        X, _ = datagen.generate(s)
        mu0 = datagen.init_sample(X, s.N, K, seed)
        for T in (1, 3, 8):
            r = oracle.fit(X, mu0, tol=0.0, max_iter=T, assign_f32=False)
            if r["empty_events"]:
                continue
            ref, _ = kmeans2(X.T.astype(np.float64), mu0.copy(), iter=T, minit="matrix",
                             missing="raise")
            assert np.allclose(r["mu"], ref, rtol=1e-11, atol=1e-11), (seed, T)


# ---------------------------------------- the paper's other stopping rule
def test_smallest_positive_tol_is_the_indicator_stability_rule():
    # The Lloyd's Algorithm section calls the method converged when no
    # indicator changes any more.  With sums taken in a fixed order, unchanged
    # indicators give bit-identical means, so E == 0 exactly; and E == 0 (same
    # centres) gives unchanged indicators.  E < 5e-324 is the test E == 0.
    s = datagen.spec("C1", N=20_000, seed=77)
    X, _ = datagen.generate(s)
    mu0 = datagen.init_sample(X, s.N, s.K, 3)
    f = oracle.fit(X, mu0, tol=5e-324, max_iter=1000)
    T = f["T"]
    assert f["converged"] and f["E"] == 0.0 and T >= 2
    assert f["E_hist"][T - 2] > 0.0                # it did not stop before
    prev = oracle.fit(X, mu0, tol=0.0, max_iter=T - 1)
    # the centres the last update started from already had stable indicators
    assert np.array_equal(prev["labels"], f["labels"])
    nxt = oracle.step(X, f["mu"])
    assert nxt["E"] == 0.0 and np.array_equal(nxt["labels"], f["labels"])


def test_fit_track_worked_example():
    # hand-counted indicator changes of the worked example: all 4 points at
    # the first update (no labels before it), then the point (2, 0), then none
    g = json.load(open(os.path.join(GOLD, "worked_example_k2.json")))
    X = soa(g["points_xy"])
    f = oracle.fit_track(X, np.array(g["init"], np.float64), tol=0.0, max_iter=50)
    assert f["changed"].tolist() == [s["changed"] for s in g["steps"]]
    assert f["T"] == g["T"] and f["converged"]
    assert np.array_equal(f["mu"], np.array(g["steps"][-1]["mu_next"], np.float64))
    assert f["labels"].tolist() == g["steps"][-1]["labels"]
    # max_iter reached first: not converged
    f1 = oracle.fit_track(X, np.array(g["init"], np.float64), tol=0.0, max_iter=2)
    assert f1["T"] == 2 and not f1["converged"] and f1["changed"].tolist() == [4, 1]


def _brute_labels(P, mu):
    # first-index argmin of the float64 squared distance (distinct points,
    # generic centres: no ties)
    return [min(range(len(mu)), key=lambda k: sum((p[j] - mu[k][j]) ** 2 for j in range(len(p))))
            for p in P]


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_fit_track_counts_against_brute_force(seed):
    # the changed counts of each update equal those of a brute-force Lloyd
    # loop (Python floats, math.fsum means) over the same tiny data
    rng = np.random.default_rng(seed)
    N, d, K = 40, 2, 4
    P = rng.normal(size=(N, d)).astype(np.float32).astype(np.float64)
    mu = [list(P[i]) for i in rng.choice(N, K, replace=False)]
    f = oracle.fit_track(P.T.astype(np.float32), np.array(mu), tol=0.0, max_iter=100,
                         assign_f32=False)
    prev, counts = None, []
    for _ in range(100):
        lab = _brute_labels(P.tolist(), mu)
        counts.append(N if prev is None else sum(a != b for a, b in zip(lab, prev)))
        for k in range(K):
            mem = [P[i] for i in range(N) if lab[i] == k]
            if mem:
                mu[k] = [math.fsum(p[j] for p in mem) / len(mem) for j in range(d)]
        prev = lab
        if counts[-1] == 0:
            break
    assert f["changed"].tolist() == counts
    assert f["labels"].tolist() == prev
    assert np.allclose(f["mu"], np.array(mu), rtol=0, atol=1e-12)


def test_fit_track_stops_with_the_e_zero_rule():
    # on data without repeated points the first update that changes no label
    # is the first with E == 0: the same T, centres and labels as tol = 5e-324
    s = datagen.spec("C1", N=20_000, seed=78)
    X, _ = datagen.generate(s)
    mu0 = datagen.init_sample(X, s.N, s.K, 4)
    f = oracle.fit_track(X, mu0, tol=0.0, max_iter=1000)
    g = oracle.fit(X, mu0, tol=5e-324, max_iter=1000)
    assert f["converged"] and f["T"] == g["T"]
    assert f["changed"][0] == s.N and f["changed"][-1] == 0 and np.all(f["changed"][:-1] > 0)
    assert np.array_equal(f["E_hist"], g["E_hist"])
    assert np.array_equal(f["mu"], g["mu"]) and np.array_equal(f["labels"], g["labels"])
