"""Tolerances of the GPU-vs-oracle comparisons and helpers to apply them.

Labels: identical except at points whose best and second-best squared
distances (float64, same float32-rounded centres) differ by less than a
relative gap; such points may take either centre but must take one of the
near-tied ones.  The gap is 1e-6, or for d-dimensional points whatever is
larger of 1e-6 and 2.01 * gamma_{d+2} (gap_for_dim): the float32 direct form
rounds d differences, d squares and d-1 additions, each term of the sum
picking up at most d+2 roundings of relative size 2^-24, and all terms are
positive, so the computed distance is within gamma_{d+2} = (d+2)u/(1-(d+2)u)
of the exact one; two centres can swap only when their exact distances are
within 2 gamma_{d+2} of the larger one.  Centres: |mu_gpu - mu_ref| <= 1e-5 *
max(|mu_ref_k|_inf, 1) per centre.  E: |E_gpu - E_ref| <= 1e-6 absolute,
plus, where the caller passes the shape and max|x| (e_tol), the effect of the
GPU's fixed-point sums: every point is rounded to a grid of step 2^-G <=
max|x| * 2^-29, so each mean coordinate is within half a step of the exact
mean, the K*d shifts move by at most that much, and E = sum of squared
shifts moves by at most 2 sqrt(E) sqrt(K d) (step / 2) to first order.
"""
import numpy as np

import oracle

REL_GAP = 1e-6
CENTRE_RTOL = 1e-5
E_ATOL = 1e-6


def gap_for_dim(d):
    """Relative near-tie window for d-dimensional float32 direct-form distances."""
    u = 2.0 ** -24
    n = d + 2
    return max(REL_GAP, 2.01 * n * u / (1.0 - n * u))


def label_check(gpu_labels, X, mu, N=None, rel=None):
    """Compare labels with the oracle's reassignment at centres mu.

    rel: the near-tie window (default gap_for_dim of X's dimension).
    Returns (n_mismatch, n_near_ties, ref_labels, ref_dmin); raises AssertionError when a
    mismatch is not excused or an excused label is not a near-tied centre."""
    ref, dmin, dsec = oracle.assign(X, mu, N=N)
    gpu = np.asarray(gpu_labels)
    rel = gap_for_dim(np.asarray(X).shape[0]) if rel is None else rel
    near = (dsec - dmin) <= rel * dsec
    mism = gpu != ref
    bad = mism & ~near
    assert not bad.any(), (f"{int(bad.sum())} labels differ outside near-ties, first at "
                           f"{np.flatnonzero(bad)[:5].tolist()}")
    idx = np.flatnonzero(mism)
    if idx.size:
        m32 = mu.astype(np.float32).astype(np.float64)
        pts = X[:, idx].astype(np.float64)
        Dg = ((pts - m32[gpu[idx]].T) ** 2).sum(axis=0)
        assert np.all(Dg - dmin[idx] <= rel * Dg), "an excused label is not near-tied"
    return int(mism.sum()), int(near.sum()), ref, dmin


def centre_check(mu_gpu, mu_ref):
    scale = np.maximum(np.abs(mu_ref).max(axis=1, keepdims=True), 1.0)
    err = np.abs(mu_gpu - mu_ref) / scale
    assert np.all(err <= CENTRE_RTOL), f"centre error {err.max():.3e}"
    return float(err.max())


def e_tol(E_ref, K=0, d=0, absmax=0.0):
    """Tolerance on E (see the module docstring)."""
    step = float(absmax) * 2.0 ** -29
    return E_ATOL + 2.0 * np.sqrt(max(E_ref, 0.0) * K * d) * step / 2.0 + K * d * step * step


def e_check(E_gpu, E_ref, K=0, d=0, absmax=0.0):
    assert abs(E_gpu - E_ref) <= e_tol(E_ref, K, d, absmax), (E_gpu, E_ref)
    return abs(E_gpu - E_ref)
