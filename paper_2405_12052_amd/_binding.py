"""ctypes binding of libkmeans_mi355x.so (include/kmeans.h).

Argument marshalling only: every step of the clustering runs in the library's
HIP kernels.  PyTorch supplies device memory (the points and label tensors)
and the HIP stream.  There is no fallback: if the shared library is missing
the import of this module's functions raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkmeans_mi355x.so")

KM_OK, KM_EINVAL, KM_ENODEV, KM_EHIP, KM_ENOMEM, KM_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
KM_OPT_GRAPH, KM_OPT_UNROLL, KM_OPT_BLOCKS, KM_OPT_TIMING = 1, 2, 3, 4


class KMeansError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


_STATUS = {0: "KM_OK", -1: "KM_EINVAL", -2: "KM_ENODEV", -3: "KM_EHIP", -4: "KM_ENOMEM",
           -5: "KM_EUNSUPPORTED"}


class km_result(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("E", C.c_double),
                ("shift_l2", C.c_double), ("objective", C.c_double),
                ("empty_events", C.c_int64)]


_lib = None


def load_library():
    """Load the in-tree shared library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it first "
                           "(python -c 'import __graft_entry__ as g; g.build()')")
    lib = C.CDLL(LIB_PATH)
    vp, f32p, f64p, i32p = C.c_void_p, C.c_void_p, C.POINTER(C.c_double), C.c_void_p
    sig = {
        "kmeans_abi_version": (C.c_int, []),
        "kmeans_status_string": (C.c_char_p, [C.c_int]),
        "kmeans_last_error": (C.c_char_p, [vp]),
        "kmeans_validate": (C.c_int, [C.c_int64, C.c_int64, C.c_int32, C.c_int32, C.c_double,
                                      C.c_int32]),
        "kmeans_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int, vp, C.c_uint32]),
        "kmeans_destroy": (None, [vp]),
        "kmeans_set_option": (C.c_int, [vp, C.c_int32, C.c_int64]),
        "kmeans_assign": (C.c_int, [vp, f32p, C.c_int64, C.c_int64, C.c_int32, C.c_int32, f64p,
                                    i32p, f64p]),
        "kmeans_fit": (C.c_int, [vp, f32p, C.c_int64, C.c_int64, C.c_int32, C.c_int32, f64p,
                                 C.c_double, C.c_int32, f64p, i32p, C.POINTER(km_result)]),
        "kmeans_get_history": (C.c_int, [vp, f64p, f64p, C.c_int32]),
        "kmeans_get_timing": (C.c_int, [vp, f64p, C.POINTER(C.c_int64)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def validate(N, ld, d, K, tol=1e-6, max_iter=100) -> int:
    """Host-only argument check (no GPU needed); returns the status code."""
    return load_library().kmeans_validate(N, ld, d, K, tol, max_iter)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


@dataclass
class FitResult:
    centroids: np.ndarray      # (K, d) float64
    labels: object             # torch int32 tensor (N,) on the device, or None
    iters: int
    converged: bool
    E: float
    shift_l2: float
    objective: float
    empty_events: int


class KMeans:
    """A library context bound to one device and one HIP stream.

    X is a float32 CUDA tensor of shape (d, >= N) with unit stride along the
    points (structure of arrays); row stride = X.stride(0).
    """

    def __init__(self, device: int | None = None, stream=None):
        import torch
        self._torch = torch
        lib = load_library()
        dev = torch.cuda.current_device() if device is None else int(device)
        s = torch.cuda.current_stream(dev) if stream is None else stream
        self.device = dev
        self.stream = s
        ctx = C.c_void_p()
        rc = lib.kmeans_create(C.byref(ctx), dev, C.c_void_p(s.cuda_stream), 0)
        if rc != KM_OK:
            raise KMeansError(rc, lib.kmeans_last_error(None).decode())
        self._ctx = ctx
        self._lib = lib

    # -------------------------------------------------------------- helpers
    def _check(self, rc):
        if rc != KM_OK:
            raise KMeansError(rc, self._lib.kmeans_last_error(self._ctx).decode())

    def _points(self, X, N):
        t = self._torch
        if not isinstance(X, t.Tensor) or X.dtype != t.float32 or not X.is_cuda or X.dim() != 2:
            raise TypeError("X must be a float32 CUDA tensor of shape (d, N)")
        if X.stride(1) != 1:
            raise ValueError("X must have unit stride along the points")
        n = X.shape[1] if N is None else int(N)
        return X.data_ptr(), n, X.stride(0), X.shape[0]

    def set_option(self, option: int, value: int):
        self._check(self._lib.kmeans_set_option(self._ctx, option, int(value)))

    # ------------------------------------------------------------ API calls
    def assign(self, X, centroids, N=None, labels=True):
        """Labels (int32 device tensor or None) and objective for `centroids`."""
        ptr, n, ld, d = self._points(X, N)
        mu = _f64(centroids)
        K = mu.shape[0]
        lab = self._torch.empty(n, dtype=self._torch.int32, device=X.device) if labels else None
        obj = C.c_double()
        self._check(self._lib.kmeans_assign(self._ctx, ptr, n, ld, d, K, _dptr(mu),
                                            lab.data_ptr() if labels else None, C.byref(obj)))
        return lab, obj.value

    def fit(self, X, init, tol=1e-6, max_iter=100, N=None, labels=True) -> FitResult:
        """Lloyd's algorithm from `init` (K x d) until E < tol or max_iter."""
        ptr, n, ld, d = self._points(X, N)
        mu0 = _f64(init)
        K = mu0.shape[0]
        out = np.empty((K, d), np.float64)
        lab = self._torch.empty(n, dtype=self._torch.int32, device=X.device) if labels else None
        res = km_result()
        self._check(self._lib.kmeans_fit(self._ctx, ptr, n, ld, d, K, _dptr(mu0), float(tol),
                                         int(max_iter), _dptr(out),
                                         lab.data_ptr() if labels else None, C.byref(res)))
        return FitResult(out, lab, res.iters, bool(res.converged), res.E, res.shift_l2,
                         res.objective, res.empty_events)

    def history(self, cap: int = 1 << 20):
        E = np.empty(cap, np.float64)
        J = np.empty(cap, np.float64)
        n = self._lib.kmeans_get_history(self._ctx, _dptr(E), _dptr(J), cap)
        if n < 0:
            self._check(n)
        return E[:n].copy(), J[:n].copy()

    def timing(self):
        ms = C.c_double()
        k = C.c_int64()
        self._check(self._lib.kmeans_get_timing(self._ctx, C.byref(ms), C.byref(k)))
        return ms.value, k.value

    def close(self):
        if getattr(self, "_ctx", None):
            self._lib.kmeans_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
