"""GPU parity of the learned initialiser's kernels (through the C ABI) with
the FP64 oracle of the network: pooled features and predictions, gradients of
every parameter block, the device Hungarian matching against scipy, bitwise
repeatability, a decreasing loss under Adam, and the inference pipeline
(gather + normalise + forward + de-normalise)."""
import numpy as np
import pytest

from oracle import initnet as onet

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

K = 16


@pytest.fixture(scope="module")
def km():
    from paper_2405_12052_amd import KMeans
    k = KMeans(0)
    yield k
    k.close()


def setup(B=4, P=256, seed=0):
    rng = np.random.default_rng(seed)
    pts = rng.normal(size=(B, P, 3)).astype(np.float32)
    tgt = rng.normal(size=(B, K, 3)).astype(np.float32)
    theta = onet.init_params(K, seed=seed + 1).astype(np.float32)
    return pts, tgt, theta


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def blocks(vec):
    out, o = {}, 0
    for name, s in onet.shapes(K):
        n = int(np.prod(s))
        out[name] = np.asarray(vec[o:o + n], np.float64)
        o += n
    return out


def cos(a, b):
    return float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-300))


def test_param_count(km):
    from paper_2405_12052_amd import initnet_param_count
    assert initnet_param_count(K) == onet.param_count(K) == 49776
    assert initnet_param_count(17) == -1


def test_forward_matches_oracle(km):
    pts, _, theta = setup()
    pred, pool = km.initnet_forward(dev(pts), K, dev(theta))
    y, c = onet.forward(theta.astype(np.float64), pts, K)
    ref_pool = np.concatenate([np.maximum(c["a2"], 0).mean(axis=1),
                               np.maximum(c["a2"], 0).max(axis=1)], axis=1)
    gp = pool.cpu().numpy()
    assert np.abs(gp - ref_pool).max() <= 1e-2 * np.abs(ref_pool).max()
    gy = pred.cpu().numpy()
    assert np.abs(gy - y).max() <= 2e-2 * np.abs(y).max()
    assert cos(gy.ravel(), y.ravel()) > 0.9999


def test_gradients_match_oracle(km):
    pts, tgt, theta = setup(B=6, P=512, seed=3)
    g, L, match = km.initnet_grad(dev(pts), dev(tgt), K, dev(theta))
    pi = match.cpu().numpy().astype(np.int64)
    Lr, gr, pir = onet.loss_and_grad(theta.astype(np.float64), pts, tgt, K)
    assert np.array_equal(pi, pir), "device matching differs from scipy"
    assert abs(L - Lr) <= 1e-3 * Lr
    gb, rb = blocks(g.cpu().numpy()), blocks(gr)
    for name in gb:
        c = cos(gb[name], rb[name])
        rel = np.linalg.norm(gb[name] - rb[name]) / (np.linalg.norm(rb[name]) + 1e-300)
        print(f"{name}: cos {c:.6f} rel {rel:.2e}", flush=True)
        assert c >= 0.999 and rel <= 1e-2, name


def _scipy_pi(y, t):
    from scipy.optimize import linear_sum_assignment
    C = ((y[:, None, :] - t[None, :, :]) ** 2).sum(axis=2)
    rows, cols = linear_sum_assignment(C)
    pi = np.empty(len(t), np.int64)
    pi[cols] = rows
    return pi, C


def test_device_hungarian_equals_scipy(km):
    # W3 = W4 = 0 makes every prediction equal the output bias b4: well
    # separated random centres, so the optimal assignment is unique
    pts, tgt, theta = setup(B=64, P=64, seed=5)
    w = blocks(theta)
    o = 0
    for name, sh in onet.shapes(K):
        n = int(np.prod(sh))
        if name in ("W3", "W4"):
            theta[o:o + n] = 0.0
        if name == "b4":
            theta[o:o + n] = np.random.default_rng(6).normal(size=n) * 2
        o += n
    _, _, match = km.initnet_grad(dev(pts), dev(tgt), K, dev(theta))
    pred, _ = km.initnet_forward(dev(pts), K, dev(theta))
    y = pred.cpu().numpy().astype(np.float64)
    m = match.cpu().numpy()
    for b in range(64):
        pi, _ = _scipy_pi(y[b], tgt[b].astype(np.float64))
        assert np.array_equal(m[b], pi), b


def test_device_hungarian_cost_is_optimal(km):
    # generic network outputs may tie: the assignment's cost must be optimal
    pts, tgt, theta = setup(B=64, P=64, seed=15)
    _, _, match = km.initnet_grad(dev(pts), dev(tgt), K, dev(theta))
    pred, _ = km.initnet_forward(dev(pts), K, dev(theta))
    y = pred.cpu().numpy().astype(np.float64)
    m = match.cpu().numpy()
    for b in range(64):
        pi, C = _scipy_pi(y[b], tgt[b].astype(np.float64))
        assert sorted(m[b].tolist()) == list(range(K))
        assert C[m[b], np.arange(K)].sum() <= C[pi, np.arange(K)].sum() * (1 + 1e-12) + 1e-15


def test_gradient_is_bitwise_repeatable(km):
    pts, tgt, theta = setup(B=8, P=256, seed=7)
    g1, L1, _ = km.initnet_grad(dev(pts), dev(tgt), K, dev(theta))
    g2, L2, _ = km.initnet_grad(dev(pts), dev(tgt), K, dev(theta))
    assert torch.equal(g1, g2) and L1 == L2


def test_adam_steps_reduce_the_loss(km):
    pts, tgt, theta = setup(B=16, P=256, seed=9)
    p = dev(theta)
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    P, T = dev(pts), dev(tgt)
    losses = [km.initnet_train_step(P, T, K, p, m, v, 1e-3, s) for s in range(1, 41)]
    print(f"loss {losses[0]:.4f} -> {losses[-1]:.4f}", flush=True)
    assert losses[-1] < 0.7 * losses[0]


def test_inference_pipeline(km):
    rng = np.random.default_rng(11)
    N = 50_000
    X = (rng.normal(size=(3, N)) * 7 + np.array([[3.0], [-20.0], [40.0]])).astype(np.float32)
    theta = onet.init_params(K, seed=12).astype(np.float32)
    idx = np.random.Generator(np.random.PCG64(13)).choice(N, 4096, replace=False).astype(np.int32)
    out = km.init_learned(dev(X), K, dev(theta), idx=dev(idx))
    S = X[:, idx].astype(np.float64)
    mean = S.mean(axis=1)
    sd = np.sqrt(((S - mean[:, None]) ** 2).mean())
    pts = ((S - mean[:, None]) / sd).T[None].astype(np.float32)
    y, _ = onet.forward(theta.astype(np.float64), pts, K)
    ref = y[0] * sd + mean
    assert np.abs(out - ref).max() <= 2e-2 * sd * np.abs(y).max()
