"""Pins of the k-means++ oracle against the definition of D^2 seeding
(Arthur and Vassilvitskii, 2007): centre 0 uniform over the points, each next
centre drawn with probability proportional to the squared distance to the
nearest chosen centre."""
import math

import numpy as np
import pytest

from oracle import seeding


def _points(N, d, seed):
    return np.random.default_rng(seed).normal(size=(d, N)).astype(np.float32) * 10


def _d2_64(X, chosen):
    """Textbook D^2 in float64: squared distance to the nearest chosen point."""
    X = X.astype(np.float64)
    return np.min([((X - X[:, [c]]) ** 2).sum(axis=0) for c in chosen], axis=0)


def test_first_centre_is_uniform_index():
    X = _points(1000, 2, 0)
    for u0 in (0.0, 0.25, 0.5, 0.999999, 0.1234):
        assert seeding.kmeanspp(X, 1000, 1, [u0])[0] == min(999, math.floor(u0 * 1000))


@pytest.mark.parametrize("d", [2, 3])
def test_second_centre_probability_is_d2_share(d):
    # Sweep u_1 over a fine uniform grid: the share of the grid that selects
    # point i must be D_i^2 / sum D^2 (to the grid spacing).
    N = 7
    X = _points(N, d, 1 + d)
    u0 = 3.5 / N                        # centre 0 = point 3
    p = _d2_64(X, [3])
    p /= p.sum()
    n = 20000
    counts = np.zeros(N)
    for k in range(n):
        counts[seeding.kmeanspp(X, N, 2, [u0, (k + 0.5) / n])[1]] += 1
    assert counts[3] == 0
    np.testing.assert_allclose(counts / n, p, atol=2.0 / n)


def test_third_centre_uses_nearest_chosen_centre():
    N = 6
    X = np.array([[0, 1, 2, 10, 11, 30], [0, 0, 0, 0, 0, 0]], np.float32)
    u0 = 0.5 / N                        # centre 0 = point 0
    # u_1 just below 1 picks the farthest point (index 5, D^2 = 900)
    first2 = seeding.kmeanspp(X, N, 2, [u0, 0.999])
    assert list(first2) == [0, 5]
    p = _d2_64(X, [0, 5])               # min over both chosen centres
    p /= p.sum()
    n = 20000
    counts = np.zeros(N)
    for k in range(n):
        counts[seeding.kmeanspp(X, N, 3, [u0, 0.999, (k + 0.5) / n])[2]] += 1
    np.testing.assert_allclose(counts / n, p, atol=2.0 / n)
    assert counts[0] == counts[5] == 0


def test_agrees_with_float64_inverse_cdf_draw():
    # The textbook draw (float64 cumulative probabilities, inverse CDF at u)
    # picks the same points except within rounding of a CDF step.
    X = _points(5000, 3, 7)
    rng = np.random.default_rng(8)
    agree = total = 0
    for _ in range(20):
        u = rng.random(8)
        idx = seeding.kmeanspp(X, 5000, 8, u)
        for j in range(1, 8):
            p = _d2_64(X, idx[:j])
            cdf = np.cumsum(p) / p.sum()
            ref = int(np.searchsorted(cdf, u[j], side="right"))
            agree += int(ref == idx[j])
            total += 1
    assert agree >= total - 1


def test_never_picks_a_chosen_point_while_others_remain():
    X = _points(50, 2, 9)
    rng = np.random.default_rng(10)
    for _ in range(50):
        idx = seeding.kmeanspp(X, 50, 20, rng.random(20))
        assert len(set(idx.tolist())) == 20


def test_all_points_equal_falls_back_to_uniform_index():
    X = np.full((3, 40), 2.5, np.float32)
    u = [0.1, 0.5, 0.77, 0.999]
    idx = seeding.kmeanspp(X, 40, 4, u)
    assert list(idx) == [math.floor(v * 40) for v in u]


def test_scaling_by_power_of_two_keeps_the_draw():
    # Doubling every coordinate scales each D^2 by 4 exactly; the integer
    # weights (scaled relative to the maximum) and so the draw are unchanged.
    X = _points(3000, 3, 11)
    u = np.random.default_rng(12).random(16)
    np.testing.assert_array_equal(seeding.kmeanspp(X, 3000, 16, u),
                                  seeding.kmeanspp(X * 2, 3000, 16, u))


def test_weights_fit_int64():
    N = 1 << 20
    assert seeding.weight_bits(N) == 42
    assert seeding.weight_bits(N + 1) == 41
    assert seeding.weight_bits(1) == 62
    assert N * 2 ** seeding.weight_bits(N) <= 2 ** 62


def test_rejects_non_finite_and_bad_u():
    X = _points(10, 2, 13)
    with pytest.raises(ValueError):
        seeding.kmeanspp(X, 10, 2, [0.5, 1.0])
    X[1, 4] = np.nan
    with pytest.raises(ValueError):
        seeding.kmeanspp(X, 10, 2, [0.0, 0.5])
