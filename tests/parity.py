"""Tolerances of the GPU-vs-oracle comparisons and helpers to apply them.

Labels: bit-identical.  The library's reassignment rule is the first index of
the minimum of the squared distance to the float32-rounded centres evaluated
in float64 (each difference, square and partial sum rounded to float64, left
to right), which is what the oracle's assign computes with its default
assign_f32 (its C source is built without FMA contraction).  The GPU reaches
it either through a certified winner, whose margin exceeds every rounding
involved, or through a float64 re-scan of the near-ties, so no label may
differ.  gap_for_dim still gives the relative window within which the float32
direct form (used for the objective) can swap two centres: d differences, d
squares and d-1 additions, each term picking up at most d+2 roundings of
relative size 2^-24, all terms positive, so a computed distance is within
gamma_{d+2} = (d+2)u/(1-(d+2)u) of the exact one.  Centres: |mu_gpu - mu_ref| <= 1e-5 *
max(|mu_ref_k|_inf, 1) per centre.  E: |E_gpu - E_ref| <= 1e-6 absolute,
plus (where the caller passes the reference centres mu) what float64 itself
allows when E is large: both sides form E = sum (m' - m)^2 in float64 from
means each rounded once to float64 (relative error u = 2^-53 per operation),
so each side's E is within 4u sqrt(E) |m'|_F (the rounding of the means) +
K d u E (the sum of K d squares) of the exact E, and the two within twice
that.  It is the float64 precision that the method's update is specified in,
not the GPU's own quantisation: the fixed-point sums (|x| 2^F < 2^44) must
and do fit inside the 1e-6 for the data the tests use.
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
    """Compare labels with the oracle's reassignment at centres mu (the
    centres the GPU labelled against): they must be identical.

    rel: the near-tie window used to count near-ties for the log (default
    gap_for_dim of X's dimension).  Returns (n_mismatch, n_near_ties,
    ref_labels, ref_dmin); raises AssertionError on any mismatch."""
    ref, dmin, dsec = oracle.assign(X, mu, N=N)
    gpu = np.asarray(gpu_labels)
    rel = gap_for_dim(np.asarray(X).shape[0]) if rel is None else rel
    near = (dsec - dmin) <= rel * dsec
    mism = gpu != ref
    assert not mism.any(), (f"{int(mism.sum())} labels differ from the oracle's (of them "
                            f"{int((mism & near).sum())} near-ties), first at "
                            f"{np.flatnonzero(mism)[:5].tolist()}")
    return 0, int(near.sum()), ref, dmin


def centre_check(mu_gpu, mu_ref):
    scale = np.maximum(np.abs(mu_ref).max(axis=1, keepdims=True), 1.0)
    err = np.abs(mu_gpu - mu_ref) / scale
    assert np.all(err <= CENTRE_RTOL), f"centre error {err.max():.3e}"
    return float(err.max())


def e_tol(E_ref, mu=None):
    """Tolerance on E (see the module docstring); mu: the reference centres
    after the update (K x d), or None for the plain 1e-6."""
    if mu is None:
        return E_ATOL
    u = 2.0 ** -53
    mu = np.asarray(mu, dtype=np.float64)
    E = max(float(E_ref), 0.0)
    return E_ATOL + 2.0 * (4.0 * u * np.sqrt(E) * np.linalg.norm(mu) + mu.size * u * E)


def e_check(E_gpu, E_ref, mu=None):
    assert abs(E_gpu - E_ref) <= e_tol(E_ref, mu), (E_gpu, E_ref, e_tol(E_ref, mu))
    return abs(E_gpu - E_ref)
