"""FP64 CPU oracle for Lloyd's K-means -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  The library (the HIP kernels and their Python binding)
never imports, links or runs anything here, and this package never imports the
library: the two share no code.

`kmeans_oracle.c` holds the arithmetic (plain loops in float64, see its header
for the definitions and readings it follows); this module loads it with ctypes
and wraps it for numpy arrays.  `build()` compiles it with gcc.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kmeans_oracle.c")
_LIB = os.path.join(_HERE, "libkmeans_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle (gcc, -O2, OpenMP, no FMA contraction, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = C.CDLL(_LIB)
        f32p = C.POINTER(C.c_float)
        f64p = C.POINTER(C.c_double)
        i32p = C.POINTER(C.c_int32)
        i64p = C.POINTER(C.c_int64)
        ip = C.POINTER(C.c_int)
        lib.oracle_threads.argtypes = [C.c_int]
        lib.oracle_threads.restype = C.c_int
        lib.oracle_assign.argtypes = [f32p, C.c_int64, C.c_int64, C.c_int, C.c_int,
                                      f64p, C.c_int, i32p, f64p, f64p]
        lib.oracle_step.argtypes = [f32p, C.c_int64, C.c_int64, C.c_int, C.c_int,
                                    f64p, C.c_int, i32p, i64p, f64p, f64p, f64p,
                                    f64p, i64p]
        lib.oracle_update.argtypes = [f32p, C.c_int64, C.c_int64, C.c_int, C.c_int, i32p,
                                      f64p, i64p, f64p, f64p, f64p, i64p]
        lib.oracle_fit.argtypes = [f32p, C.c_int64, C.c_int64, C.c_int, C.c_int,
                                   f64p, C.c_double, C.c_int, C.c_int, f64p, i32p,
                                   ip, f64p, f64p, ip, f64p, f64p, i64p]
        for f in (lib.oracle_assign, lib.oracle_step, lib.oracle_update, lib.oracle_fit):
            f.restype = C.c_int
        _lib = lib
    return _lib


def _ptr(a, ct):
    return None if a is None else a.ctypes.data_as(C.POINTER(ct))


def _prep(X, N):
    X = np.asarray(X)
    if X.dtype != np.float32 or X.ndim != 2:
        raise TypeError("X must be a float32 array of shape (d, ld)")
    if not X.flags.c_contiguous:
        X = np.ascontiguousarray(X)
    d, ld = X.shape
    N = ld if N is None else int(N)
    if N > ld:
        raise ValueError("N exceeds the row length of X")
    return X, N, d, ld


def threads(n: int = 0) -> int:
    """Set (n > 0) and return the OpenMP thread count the oracle uses."""
    return _load().oracle_threads(int(n))


def assign(X, mu, N=None, assign_f32=True):
    """Labels, minimum distance and second-smallest distance for every point."""
    lib = _load()
    X, N, d, ld = _prep(X, N)
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    K = mu.shape[0]
    assert mu.shape == (K, d)
    labels = np.empty(N, np.int32)
    dmin = np.empty(N, np.float64)
    dsec = np.empty(N, np.float64)
    rc = lib.oracle_assign(_ptr(X, C.c_float), N, ld, d, K, _ptr(mu, C.c_double),
                           int(bool(assign_f32)), _ptr(labels, C.c_int32),
                           _ptr(dmin, C.c_double), _ptr(dsec, C.c_double))
    if rc:
        raise ValueError(f"oracle_assign failed ({rc})")
    return labels, dmin, dsec


def step(X, mu, N=None, assign_f32=True):
    """One Lloyd update from centres mu; returns a dict."""
    lib = _load()
    X, N, d, ld = _prep(X, N)
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    K = mu.shape[0]
    labels = np.empty(N, np.int32)
    counts = np.empty(K, np.int64)
    sums = np.empty((K, d), np.float64)
    nxt = np.empty((K, d), np.float64)
    E = C.c_double()
    J = C.c_double()
    emp = C.c_int64()
    rc = lib.oracle_step(_ptr(X, C.c_float), N, ld, d, K, _ptr(mu, C.c_double),
                         int(bool(assign_f32)), _ptr(labels, C.c_int32),
                         _ptr(counts, C.c_int64), _ptr(sums, C.c_double),
                         _ptr(nxt, C.c_double), C.byref(E), C.byref(J), C.byref(emp))
    if rc:
        raise ValueError(f"oracle_step failed ({rc})")
    return {"labels": labels, "counts": counts, "sums": sums, "mu": nxt,
            "E": E.value, "J": J.value, "empty": emp.value}


def update(X, labels, mu, N=None):
    """Mean step for given labels (0..K-1) from centres mu; returns a dict."""
    lib = _load()
    X, N, d, ld = _prep(X, N)
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    K = mu.shape[0]
    labels = np.ascontiguousarray(labels, dtype=np.int32)
    assert labels.shape == (N,)
    counts = np.empty(K, np.int64)
    sums = np.empty((K, d), np.float64)
    nxt = np.empty((K, d), np.float64)
    E = C.c_double()
    emp = C.c_int64()
    rc = lib.oracle_update(_ptr(X, C.c_float), N, ld, d, K, _ptr(labels, C.c_int32),
                           _ptr(mu, C.c_double), _ptr(counts, C.c_int64),
                           _ptr(sums, C.c_double), _ptr(nxt, C.c_double), C.byref(E),
                           C.byref(emp))
    if rc:
        raise ValueError(f"oracle_update failed ({rc})")
    return {"counts": counts, "sums": sums, "mu": nxt, "E": E.value, "empty": emp.value}


def fit(X, mu0, tol=1e-6, max_iter=100, N=None, assign_f32=True, labels=True):
    """Lloyd's algorithm until E < tol or max_iter updates; returns a dict."""
    lib = _load()
    X, N, d, ld = _prep(X, N)
    mu0 = np.ascontiguousarray(mu0, dtype=np.float64)
    K = mu0.shape[0]
    out = np.empty((K, d), np.float64)
    lab = np.empty(N, np.int32) if labels else None
    T = C.c_int()
    E = C.c_double()
    J = C.c_double()
    conv = C.c_int()
    Eh = np.zeros(max_iter, np.float64)
    Jh = np.zeros(max_iter, np.float64)
    ev = C.c_int64()
    rc = lib.oracle_fit(_ptr(X, C.c_float), N, ld, d, K, _ptr(mu0, C.c_double),
                        float(tol), int(max_iter), int(bool(assign_f32)),
                        _ptr(out, C.c_double), _ptr(lab, C.c_int32), C.byref(T),
                        C.byref(E), C.byref(J), C.byref(conv), _ptr(Eh, C.c_double),
                        _ptr(Jh, C.c_double), C.byref(ev))
    if rc:
        raise ValueError(f"oracle_fit failed ({rc})")
    return {"mu": out, "labels": lab, "T": T.value, "E": E.value,
            "J": J.value, "converged": bool(conv.value),
            "E_hist": Eh[:T.value].copy(), "J_hist": Jh[:T.value].copy(),
            "empty_events": ev.value}


def fit_track(X, mu0, tol=0.0, max_iter=100, N=None, assign_f32=True):
    """Lloyd's algorithm with the indicators tracked from update to update
    (section "The Lloyd's Algorithm": the iteration has converged once no
    cluster indicator changes).  Update t assigns every point to its nearest
    centre of mu^t (the step above), counts the points whose label differs
    from update t-1's (every point at t = 0, when there is none) and forms
    mu^{t+1}; the loop stops after the first update that changes no label,
    or whose E is below tol, or after max_iter updates.  Returns a dict with
    the final centres, T, E, the per-update changed counts and E history,
    whether it converged, and the labels of the last update."""
    mu = np.ascontiguousarray(mu0, dtype=np.float64)
    prev = None
    changed, E_hist = [], []
    conv = False
    r = None
    for t in range(max_iter):
        r = step(X, mu, N=N, assign_f32=assign_f32)
        lab = r["labels"]
        c = int(lab.shape[0]) if prev is None else int(np.count_nonzero(lab != prev))
        changed.append(c)
        E_hist.append(r["E"])
        mu = r["mu"]
        prev = lab
        if c == 0 or r["E"] < tol:
            conv = True
            break
    return {"mu": mu, "T": len(changed), "E": r["E"], "changed": np.array(changed, np.int64),
            "E_hist": np.array(E_hist), "converged": conv, "labels": prev}
