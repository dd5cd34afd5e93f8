"""FP64 oracle of the learned initialiser -- TEST INFRASTRUCTURE ONLY.

Only the tests (and the training script's target file) use it; the library
never imports it.  Plain numpy, float64, written from the network's
definition:

  per point    h1 = relu(x W1 + b1)          3 -> 64
               h2 = relu(h1 W2 + b2)         64 -> 64
  pooling      p  = [mean_points h2, max_points h2]   (128; max: first point on ties)
  head         z  = relu(p W3 + b3)          128 -> 256
               y  = z W4 + b4                256 -> 3K, read as K centres of 3
  loss         L  = (1/B) sum_b sum_k || y_b[pi_b(k)] - t_b[k] ||^2
               with pi_b the assignment of predicted to target centres of least
               total squared distance (Hungarian matching, scipy's
               linear_sum_assignment), held fixed when differentiating.

With bf16=True the matrices and the activations entering the matrix products
are rounded to bfloat16 (round to nearest even) at the points where the GPU
kernels round them (W1..W4, h1, p, z, and the back-propagated signals entering
the products: dh2, dz, dy); everything else stays float64.  Gradients treat
the roundings as the identity (the parameters' float32 masters receive the
gradient of their bf16 copies).  With bf16=False the function is plain float64
and the tests pin its gradient with central finite differences.

Parameter layout (one flat float vector, row-major blocks in this order):
W1 [3, 64], b1 [64], W2 [64, 64], b2 [64], W3 [128, 256], b3 [256],
W4 [256, 3K], b4 [3K].
"""
from __future__ import annotations

import numpy as np

H = 64      # per-point width
Z = 256     # head width
D = 3       # point dimension


def shapes(K: int):
    return [("W1", (D, H)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)),
            ("W3", (2 * H, Z)), ("b3", (Z,)), ("W4", (Z, D * K)), ("b4", (D * K,))]


def param_count(K: int) -> int:
    return sum(int(np.prod(s)) for _, s in shapes(K))


def unpack(flat, K):
    out, o = {}, 0
    for name, s in shapes(K):
        n = int(np.prod(s))
        out[name] = np.asarray(flat[o:o + n], dtype=np.float64).reshape(s)
        o += n
    return out


def pack(d, K):
    return np.concatenate([np.asarray(d[name], np.float64).reshape(-1) for name, _ in shapes(K)])


def bf16(x):
    """Round to bfloat16 (nearest even), via float32, returned as float64."""
    a = np.asarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def match(pred, tgt):
    """pi[k] = index of the predicted centre assigned to target k."""
    from scipy.optimize import linear_sum_assignment
    C = ((pred[:, None, :] - tgt[None, :, :]) ** 2).sum(axis=2)   # [pred, target]
    rows, cols = linear_sum_assignment(C)
    pi = np.empty(len(tgt), np.int64)
    pi[cols] = rows
    return pi


def forward(params, pts, K, bf16_mode=True):
    """pts: [B, P, 3].  Returns the predicted centres [B, K, 3] and a cache."""
    r = bf16 if bf16_mode else (lambda v: np.asarray(v, np.float64))
    w = unpack(params, K)
    W1, W2, W3, W4 = r(w["W1"]), r(w["W2"]), r(w["W3"]), r(w["W4"])
    x = np.asarray(pts, np.float64)
    B, P, _ = x.shape
    a1 = x @ W1 + w["b1"]                 # [B, P, 64]
    h1 = np.maximum(a1, 0.0)
    h1r = r(h1)
    a2 = h1r @ W2 + w["b2"]
    h2 = np.maximum(a2, 0.0)
    pmean = h2.mean(axis=1)               # [B, 64]
    amax = h2.argmax(axis=1)              # first index of the maximum
    pmax = np.take_along_axis(h2, amax[:, None, :], axis=1)[:, 0, :]
    pool = np.concatenate([pmean, pmax], axis=1)   # [B, 128]
    poolr = r(pool)
    a3 = poolr @ W3 + w["b3"]
    z = np.maximum(a3, 0.0)
    zr = r(z)
    y = zr @ W4 + w["b4"]                 # [B, 3K]
    cache = dict(x=x, W1=W1, W2=W2, W3=W3, W4=W4, a1=a1, h1r=h1r, a2=a2, amax=amax,
                 poolr=poolr, a3=a3, zr=zr, r=r, P=P)
    return y.reshape(B, K, D), cache


def loss_and_grad(params, pts, tgt, K, bf16_mode=True, pi=None):
    """Matched loss, its gradient (flat, parameter layout) and the matching."""
    y, c = forward(params, pts, K, bf16_mode)
    r = c["r"]
    B, P = y.shape[0], c["P"]
    tgt = np.asarray(tgt, np.float64)
    if pi is None:
        pi = np.stack([match(y[b], tgt[b]) for b in range(B)])
    dy = np.zeros_like(y)
    L = 0.0
    for b in range(B):
        diff = y[b, pi[b]] - tgt[b]
        L += (diff ** 2).sum()
        dy[b, pi[b]] = 2.0 * diff / B
    L /= B
    dy = dy.reshape(B, -1)
    g = {}
    dyr = r(dy)
    g["W4"] = c["zr"].T @ dyr
    g["b4"] = dy.sum(axis=0)
    dz = (dyr @ c["W4"].T) * (c["a3"] > 0)
    dzr = r(dz)
    g["W3"] = c["poolr"].T @ dzr
    g["b3"] = dz.sum(axis=0)
    dpool = dzr @ c["W3"].T                              # [B, 128]
    dmean, dmax = dpool[:, :H], dpool[:, H:]
    dh2 = np.repeat((dmean / P)[:, None, :], P, axis=1)
    bi = np.arange(B)[:, None]
    fi = np.arange(H)[None, :]
    dh2[bi, c["amax"], fi] += dmax
    dz2 = dh2 * (c["a2"] > 0)
    dz2r = r(dz2)
    g["W2"] = np.einsum("bpi,bpj->ij", c["h1r"], dz2r)
    g["b2"] = dz2.sum(axis=(0, 1))
    dh1 = dz2r @ c["W2"].T
    dz1 = dh1 * (c["a1"] > 0)
    g["W1"] = np.einsum("bpi,bpj->ij", c["x"], dz1)
    g["b1"] = dz1.sum(axis=(0, 1))
    return L, pack(g, K), pi


def init_params(K, seed=0, scale=1.0):
    """He-style random parameters for the tests."""
    rng = np.random.default_rng(seed)
    d = {}
    for name, s in shapes(K):
        if name.startswith("W"):
            d[name] = rng.normal(size=s) * scale * np.sqrt(2.0 / s[0])
        else:
            d[name] = rng.normal(size=s) * 0.01 * scale
    return pack(d, K)
