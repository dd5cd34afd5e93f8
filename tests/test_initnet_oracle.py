"""Pins of the FP64 oracle of the learned initialiser (no GPU): its gradient
against central finite differences of its own loss (plain float64 mode), the
matching against brute force over permutations, bfloat16 rounding against
torch's conversion, permutation invariance of the pooled network, and a zero
loss with zero gradient at a perfect prediction."""
import itertools

import numpy as np
import pytest

from oracle import initnet as net


def data(B=3, P=48, K=4, seed=0):
    rng = np.random.default_rng(seed)
    pts = rng.normal(size=(B, P, 3))
    tgt = rng.normal(size=(B, K, 3))
    return pts, tgt


def test_param_count_matches_the_architecture():
    # 3*64+64 + 64*64+64 + 128*256+256 + 256*48+48 for K = 16
    assert net.param_count(16) == 49776


def test_gradient_against_finite_differences():
    K = 4
    pts, tgt = data(K=K)
    theta = net.init_params(K, seed=1)
    L, g, pi = net.loss_and_grad(theta, pts, tgt, K, bf16_mode=False)
    rng = np.random.default_rng(2)
    # every bias and weight block is sampled
    idx = rng.choice(theta.size, 300, replace=False)
    eps = 1e-6
    bad = 0
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += eps
        tm[i] -= eps
        Lp, _, _ = net.loss_and_grad(tp, pts, tgt, K, bf16_mode=False, pi=pi)
        Lm, _, _ = net.loss_and_grad(tm, pts, tgt, K, bf16_mode=False, pi=pi)
        fd = (Lp - Lm) / (2 * eps)
        if abs(fd - g[i]) > 1e-6 * max(abs(fd), abs(g[i])) + 1e-9:
            bad += 1
    assert bad == 0


def test_matching_is_the_optimal_assignment():
    rng = np.random.default_rng(3)
    for _ in range(20):
        K = 6
        pred, tgt = rng.normal(size=(K, 3)), rng.normal(size=(K, 3))
        pi = net.match(pred, tgt)
        cost = ((pred[pi] - tgt) ** 2).sum()
        brute = min(((pred[list(p)] - tgt) ** 2).sum() for p in itertools.permutations(range(K)))
        assert np.isclose(cost, brute, rtol=1e-12)
        assert sorted(pi.tolist()) == list(range(K))


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(4)
    x = np.concatenate([rng.normal(size=1000) * 10.0 ** rng.integers(-8, 8, 1000),
                        [1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -1 - 2 ** -8, 0.0, 65504.0]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(net.bf16(x), ref)


def test_permutation_invariance():
    K = 4
    pts, _ = data(B=2, P=40, K=K, seed=5)
    theta = net.init_params(K, seed=6)
    y1, _ = net.forward(theta, pts, K)
    perm = np.random.default_rng(7).permutation(40)
    y2, _ = net.forward(theta, pts[:, perm], K)
    assert np.allclose(y1, y2, rtol=0, atol=1e-12)


def test_zero_loss_at_a_perfect_prediction():
    K = 4
    pts, _ = data(K=K, seed=8)
    theta = net.init_params(K, seed=9)
    y, _ = net.forward(theta, pts, K, bf16_mode=False)
    tgt = y[:, ::-1].copy()                 # the same centres in another order
    L, g, pi = net.loss_and_grad(theta, pts, tgt, K, bf16_mode=False)
    assert L < 1e-24 and np.abs(g).max() < 1e-12
    assert pi[0].tolist() == list(range(K))[::-1]
