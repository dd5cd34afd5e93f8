"""k-means++ seeding, plain numpy -- TEST INFRASTRUCTURE ONLY.

Only the tests and the benchmark's CPU leg use this module; the library never
imports it.  It states the exact, reproducible k-means++ draw (D^2 weighting,
Arthur and Vassilvitskii 2007) that the library's seeding entry point
implements, step by step and with no blocking:

  centre 0  = point min(N-1, floor(u_0 N));
  round j   : D_i^2 = float32 squared distance of point i to its nearest
              chosen centre, ((x0-c0)^2 + (x1-c1)^2) + (x2-c2)^2, every
              operation rounded to float32 on its own;
              w_i = rint(D_i^2 2^G) (integers), G = B - ilogb(max D^2) - 1,
              B = 62 - ceil(log2 N), so w_i <= 2^B and sum_i w_i < 2^63;
              S = sum w_i;  S == 0: point min(N-1, floor(u_j N));
              otherwise R = min(S-1, floor(u_j S)) and the first i with
              w_0 + ... + w_i > R.

The integer weights make the draw independent of summation order; up to the
2^-B granularity of the weights the probability of choosing point i is
D_i^2 / sum D^2, which is what the tests pin.
"""
from __future__ import annotations

import math

import numpy as np


def weight_bits(N: int) -> int:
    """B = 62 - ceil(log2 N)."""
    return 62 - (int(N) - 1).bit_length()


def kmeanspp(X, N, K, u):
    """Indices [K] (int64) of the k-means++ centres of the first N columns
    of X ([d, >= N] float32) for the uniforms u[0..K)."""
    X = np.asarray(X, dtype=np.float32)[:, :N]
    d = X.shape[0]
    u = np.asarray(u, dtype=np.float64)
    if np.any(u < 0.0) or np.any(u >= 1.0):
        raise ValueError("u must lie in [0, 1)")
    B = weight_bits(N)
    idx = [min(N - 1, int(math.floor(u[0] * N)))]
    D2 = None
    for j in range(1, K):
        c = X[:, idx[-1]]
        t = [X[q] - c[q] for q in range(d)]          # float32
        dist = t[0] * t[0] + t[1] * t[1]
        if d == 3:
            dist = dist + t[2] * t[2]
        D2 = dist if D2 is None else np.minimum(D2, dist)
        M = float(D2.max())
        if not math.isfinite(M):
            raise ValueError("X holds a NaN or an infinity")
        G = B - (math.frexp(M)[1] - 1) - 1 if M > 0.0 else 0
        w = np.rint(np.ldexp(D2.astype(np.float64), G)).astype(np.int64)
        S = int(w.sum())
        if S == 0:
            i = min(N - 1, int(math.floor(u[j] * N)))
        else:
            R = min(S - 1, int(math.floor(u[j] * float(S))))
            i = int(np.searchsorted(np.cumsum(w), R, side="right"))
        idx.append(i)
    return np.array(idx, np.int64)


def centres(X, idx):
    """The chosen points as float64 centres [K, d]."""
    X = np.asarray(X, dtype=np.float32)
    return X[:, idx].T.astype(np.float64)
