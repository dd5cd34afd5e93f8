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


def _golden_tiny():
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                    "initnet_forward_tiny.json")))
    K = g["K"]
    blocks = {name: np.zeros(s) for name, s in net.shapes(K)}
    for name, idx, v in g["weights"]:
        blocks[name][tuple(idx)] = v
    return g, K, net.pack(blocks, K), np.asarray(g["points"], np.float64)[None]


@pytest.mark.parametrize("bf16_mode", [False, True])
def test_forward_against_hand_computed_golden(bf16_mode):
    """The forward pass on sparse, hand-chosen weights against values computed
    by hand (tests/golden/initnet_forward_tiny.json): the ReLU zeros, the
    biases, mean (not sum) pooling in features 0..63 and max pooling in
    64..127, the first point on a tied maximum, and the head."""
    g, K, theta, pts = _golden_tiny()
    y, c = net.forward(theta, pts, K, bf16_mode=bf16_mode)
    assert np.array_equal(y.reshape(-1), np.asarray(g["y"], np.float64))
    h1 = np.maximum(c["a1"][0], 0.0)
    h2 = np.maximum(c["a2"][0], 0.0)
    for j in range(net.H):
        assert np.array_equal(h1[:, j], np.asarray(g["h1"].get(str(j), [0] * 4), np.float64)), j
        assert np.array_equal(h2[:, j], np.asarray(g["h2"].get(str(j), [0] * 4), np.float64)), j
        assert c["amax"][0, j] == g["argmax_point"].get(str(j), 0), j
    pool = c["poolr"][0]
    for j in range(net.H):
        assert pool[j] == g["pool_mean"].get(str(j), 0.0), j
        assert pool[net.H + j] == g["pool_max"].get(str(j), 0.0), j
    z = np.maximum(c["a3"][0], 0.0)
    for j in range(net.Z):
        assert z[j] == g["z"].get(str(j), 0.0), j
