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
KM_OPT_GRAPH, KM_OPT_UNROLL, KM_OPT_BLOCKS, KM_OPT_TIMING, KM_OPT_KEYS, KM_OPT_PERSIST = 1, 2, 3, 4, 5, 6
KM_OPT_WIDE = 7
KM_OPT_TRACK = 8


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


class km_instance(C.Structure):
    _fields_ = [("X", C.c_void_p), ("N", C.c_int64), ("ld", C.c_int64), ("d", C.c_int32),
                ("K", C.c_int32), ("n_restarts", C.c_int32), ("init", C.POINTER(C.c_double)),
                ("centroids_out", C.POINTER(C.c_double)), ("labels_out", C.c_void_p),
                ("restart_objective", C.POINTER(C.c_double)),
                ("restart_iters", C.POINTER(C.c_int32)), ("best_restart", C.c_int32),
                ("res", km_result)]


def _instance_dtype():
    """numpy view of km_instance (same field offsets and size), so that a whole
    batch's descriptors are filled and read column by column."""
    f, r = km_instance, km_result
    ro = f.res.offset
    fields = [("X", np.uint64, f.X.offset), ("N", np.int64, f.N.offset), ("ld", np.int64, f.ld.offset),
              ("d", np.int32, f.d.offset), ("K", np.int32, f.K.offset),
              ("n_restarts", np.int32, f.n_restarts.offset), ("init", np.uint64, f.init.offset),
              ("centroids_out", np.uint64, f.centroids_out.offset),
              ("labels_out", np.uint64, f.labels_out.offset),
              ("restart_objective", np.uint64, f.restart_objective.offset),
              ("restart_iters", np.uint64, f.restart_iters.offset),
              ("best_restart", np.int32, f.best_restart.offset),
              ("iters", np.int32, ro + r.iters.offset), ("converged", np.int32, ro + r.converged.offset),
              ("E", np.float64, ro + r.E.offset), ("objective", np.float64, ro + r.objective.offset),
              ("empty_events", np.int64, ro + r.empty_events.offset)]
    return np.dtype({"names": [n for n, _, _ in fields], "formats": [t for _, t, _ in fields],
                     "offsets": [o for _, _, o in fields], "itemsize": C.sizeof(km_instance)})


_KM_INSTANCE_DT = _instance_dtype()


class km_schedule(C.Structure):
    _fields_ = [("team_size", C.c_int32), ("blocks_per_cu", C.c_int32), ("big_work", C.c_double),
                ("restart_group", C.c_int32), ("mfma_min_k", C.c_int32)]


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
        "kmeans_get_changes": (C.c_int, [vp, vp, C.c_int32]),
        "kmeans_get_timing": (C.c_int, [vp, f64p, C.POINTER(C.c_int64)]),
        "kmeans_fit_batched": (C.c_int, [vp, C.c_int32, C.POINTER(km_instance), C.c_double,
                                         C.c_int32]),
        "kmeans_set_batched_schedule": (C.c_int, [vp, C.POINTER(km_schedule)]),
        "kmeans_get_batched_schedule": (C.c_int, [vp, C.POINTER(km_schedule)]),
        "kmeans_tune_batched": (C.c_int, [vp, C.c_int32, C.POINTER(km_instance), C.c_double,
                                          C.c_int32, C.c_char_p, C.POINTER(km_schedule)]),
        "kmeans_initnet_param_count": (C.c_int32, [C.c_int32]),
        "kmeans_initnet_forward": (C.c_int, [vp, vp, C.c_int32, C.c_int32, C.c_int32, vp, vp, vp]),
        "kmeans_initnet_grad": (C.c_int, [vp, vp, vp, C.c_int32, C.c_int32, C.c_int32, vp, vp,
                                          C.POINTER(C.c_double), vp]),
        "kmeans_initnet_train_step": (C.c_int, [vp, vp, vp, C.c_int32, C.c_int32, C.c_int32, vp,
                                                vp, vp, C.c_float, C.c_int32,
                                                C.POINTER(C.c_double)]),
        "kmeans_init_learned": (C.c_int, [vp, vp, C.c_int64, C.c_int64, C.c_int32, vp, C.c_int32,
                                          vp, f64p]),
        "kmeans_pp_init": (C.c_int, [vp, f32p, C.c_int64, C.c_int64, C.c_int32, C.c_int32, f64p,
                                     f64p, C.POINTER(C.c_int64)]),
        "kmeans_measure_peaks": (C.c_int, [vp, f64p]),
        "kmeans_fit_noalloc": (C.c_int, [C.c_int, vp, f32p, C.c_int64, C.c_int64, C.c_int32,
                                         C.c_int32, f64p, C.c_double, C.c_int32, f64p, i32p,
                                         C.POINTER(km_result)]),
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


def initnet_param_count(K: int) -> int:
    """Floats in the learned initialiser's parameter array for K centres."""
    return load_library().kmeans_initnet_param_count(int(K))


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


def fit_noalloc(X, init, tol=1e-6, max_iter=100, N=None, labels=None, stream=None) -> FitResult:
    """kmeans_fit_noalloc: the fit of KMeans.fit without a context and without
    any allocation inside the library (its scratch is a static device array).
    X: float32 CUDA tensor (d, >= N), unit stride along the points; labels:
    an int32 CUDA tensor of at least N entries to receive the labels, or None;
    stream: a torch stream of X's device (default: its current stream)."""
    import torch
    lib = load_library()
    if not isinstance(X, torch.Tensor) or X.dtype != torch.float32 or not X.is_cuda or X.dim() != 2:
        raise TypeError("X must be a float32 CUDA tensor of shape (d, N)")
    if X.stride(1) != 1:
        raise ValueError("X must have unit stride along the points")
    n = X.shape[1] if N is None else int(N)
    dev = X.device.index if X.device.index is not None else torch.cuda.current_device()
    s = torch.cuda.current_stream(dev) if stream is None else stream
    if labels is not None and (labels.dtype != torch.int32 or not labels.is_cuda
                               or labels.numel() < n or not labels.is_contiguous()):
        raise ValueError("labels must be a contiguous int32 CUDA tensor of at least N entries")
    mu0 = _f64(init)
    K, d = mu0.shape[0], X.shape[0]
    out = np.empty((K, d), np.float64)
    res = km_result()
    rc = lib.kmeans_fit_noalloc(dev, C.c_void_p(s.cuda_stream), X.data_ptr(), n, X.stride(0), d, K,
                                _dptr(mu0), float(tol), int(max_iter), _dptr(out),
                                labels.data_ptr() if labels is not None else None, C.byref(res))
    if rc != KM_OK:
        raise KMeansError(rc, lib.kmeans_last_error(None).decode())
    return FitResult(out, labels, res.iters, bool(res.converged), res.E, res.shift_l2,
                     res.objective, res.empty_events)


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

    # ------------------------------------------------------- batched fits
    def _instances(self, instances, labels):
        """instances: sequence of (X, N, init) with X a float32 CUDA tensor of
        shape (d, >= N) (unit stride along the points) and init an array of
        shape (R, K, d).  Returns the descriptor array (numpy, km_instance
        layout) and the buffers it points into: every instance's initial
        centres, outputs and labels are slices of one buffer each."""
        t = self._torch
        n = len(instances)
        shp = np.empty((n, 6), np.int64)  # X, N, ld, d, K, R
        inits = []
        for i, (X, N, init) in enumerate(instances):
            ptr, n_pts, ld, d = self._points(X, N)
            mu0 = _f64(init)
            if mu0.ndim != 3 or mu0.shape[2] != d:
                raise ValueError("init must have shape (restarts, K, d)")
            shp[i] = (ptr, n_pts, ld, d, mu0.shape[1], mu0.shape[0])
            inits.append(mu0.ravel())
        Ns, ds, Ks, Rs = shp[:, 1], shp[:, 3], shp[:, 4], shp[:, 5]

        def offsets(sizes):
            o = np.zeros(n + 1, np.int64)
            np.cumsum(sizes, out=o[1:])
            return o

        io, co, ro = offsets(Rs * Ks * ds), offsets(Ks * ds), offsets(Rs)
        ibuf = np.concatenate(inits) if n else np.empty(0)
        cbuf = np.empty(int(co[-1]), np.float64)
        robj = np.empty(int(ro[-1]), np.float64)
        rit = np.empty(int(ro[-1]), np.int32)
        a = np.zeros(n, _KM_INSTANCE_DT)
        a["X"], a["N"], a["ld"] = shp[:, 0], Ns, shp[:, 2]
        a["d"], a["K"], a["n_restarts"] = ds, Ks, Rs
        a["init"] = ibuf.ctypes.data + 8 * io[:-1]
        a["centroids_out"] = cbuf.ctypes.data + 8 * co[:-1]
        a["restart_objective"] = robj.ctypes.data + 8 * ro[:-1]
        a["restart_iters"] = rit.ctypes.data + 4 * ro[:-1]
        lab = None
        if labels and n:
            lo = offsets(Ns)
            lab = t.empty(int(lo[-1]), dtype=t.int32, device=instances[0][0].device)
            a["labels_out"] = lab.data_ptr() + 4 * lo[:-1]
        keep = {"shape": shp, "offsets": (co, ro), "bufs": (ibuf, cbuf, robj, rit), "labels": lab}
        return a, keep

    @staticmethod
    def _instance_ptr(a):
        return a.ctypes.data_as(C.POINTER(km_instance))

    def fit_batched(self, instances, tol=1e-6, max_iter=300, labels=True):
        """Independent fits of many instances with restarts in one persistent
        launch; returns one dict per instance (kept restart)."""
        a, keep = self._instances(instances, labels)
        self._check(self._lib.kmeans_fit_batched(self._ctx, len(instances), self._instance_ptr(a),
                                                 float(tol), int(max_iter)))
        shp, (co, ro), (_, cbuf, robj, rit), lab = (keep["shape"], keep["offsets"], keep["bufs"],
                                                    keep["labels"])
        Ns, ds, Ks = shp[:, 1].tolist(), shp[:, 3].tolist(), shp[:, 4].tolist()
        labs = lab.split(Ns) if lab is not None else [None] * len(Ns)
        co, ro = co.tolist(), ro.tolist()
        best, iters, conv = a["best_restart"].tolist(), a["iters"].tolist(), a["converged"].tolist()
        E, obj, emp = a["E"].tolist(), a["objective"].tolist(), a["empty_events"].tolist()
        res = []
        for i in range(len(Ns)):
            res.append({"centroids": cbuf[co[i]:co[i + 1]].reshape(Ks[i], ds[i]), "labels": labs[i],
                        "best_restart": best[i], "restart_objective": robj[ro[i]:ro[i + 1]],
                        "restart_iters": rit[ro[i]:ro[i + 1]], "iters": iters[i],
                        "converged": bool(conv[i]), "E": E[i], "objective": obj[i],
                        "empty_events": emp[i]})
        return res

    def set_batched_schedule(self, team_size=0, blocks_per_cu=0, big_work=0.0, restart_group=0,
                             mfma_min_k=0):
        s = km_schedule(int(team_size), int(blocks_per_cu), float(big_work), int(restart_group),
                        int(mfma_min_k))
        self._check(self._lib.kmeans_set_batched_schedule(self._ctx, C.byref(s)))

    def batched_schedule(self):
        s = km_schedule()
        self._check(self._lib.kmeans_get_batched_schedule(self._ctx, C.byref(s)))
        return {"team_size": s.team_size, "blocks_per_cu": s.blocks_per_cu, "big_work": s.big_work,
                "restart_group": s.restart_group, "mfma_min_k": s.mfma_min_k}

    def tune_batched(self, instances, tol=1e-6, max_iter=300, cache_path=None):
        """Search the batched schedule on `instances`; keeps the fastest."""
        a, keep = self._instances(instances, False)
        s = km_schedule()
        cp = cache_path.encode() if cache_path else None
        self._check(self._lib.kmeans_tune_batched(self._ctx, len(instances), self._instance_ptr(a),
                                                  float(tol),
                                                  int(max_iter), cp, C.byref(s)))
        return {"team_size": s.team_size, "blocks_per_cu": s.blocks_per_cu, "big_work": s.big_work,
                "restart_group": s.restart_group, "mfma_min_k": s.mfma_min_k}

    # ------------------------------------------------ learned initialiser
    def _net_args(self, pts, K, params):
        t = self._torch
        if pts.dtype != t.float32 or not pts.is_cuda or pts.dim() != 3 or pts.shape[2] != 3:
            raise TypeError("pts must be a float32 CUDA tensor [B, P, 3]")
        if not pts.is_contiguous():
            raise ValueError("pts must be contiguous")
        if params.dtype != t.float32 or not params.is_cuda or params.numel() != initnet_param_count(K):
            raise TypeError("params must be a float32 CUDA tensor of initnet_param_count(K) values")
        return pts.shape[0], pts.shape[1]

    def initnet_forward(self, pts, K, params):
        """Predicted normalised centres [B, K, 3] and pooled features [B, 128]."""
        B, P = self._net_args(pts, K, params)
        pred = self._torch.empty((B, K, 3), dtype=self._torch.float32, device=pts.device)
        pool = self._torch.empty((B, 128), dtype=self._torch.float32, device=pts.device)
        self._check(self._lib.kmeans_initnet_forward(self._ctx, pts.data_ptr(), B, P, K,
                                                     params.data_ptr(), pred.data_ptr(),
                                                     pool.data_ptr()))
        return pred, pool

    def initnet_grad(self, pts, targets, K, params):
        """Gradient (parameter layout), loss and matching [B, K] at params."""
        B, P = self._net_args(pts, K, params)
        grad = self._torch.empty_like(params)
        match = self._torch.empty((B, K), dtype=self._torch.int32, device=pts.device)
        loss = C.c_double()
        self._check(self._lib.kmeans_initnet_grad(self._ctx, pts.data_ptr(),
                                                  targets.contiguous().data_ptr(), B, P, K,
                                                  params.data_ptr(), grad.data_ptr(),
                                                  C.byref(loss), match.data_ptr()))
        return grad, loss.value, match

    def initnet_train_step(self, pts, targets, K, params, m, v, lr, step, want_loss=True):
        """One Adam step in place on params/m/v; the loss before it (or None)."""
        B, P = self._net_args(pts, K, params)
        loss = C.c_double()
        self._check(self._lib.kmeans_initnet_train_step(
            self._ctx, pts.data_ptr(), targets.data_ptr(), B, P, K, params.data_ptr(),
            m.data_ptr(), v.data_ptr(), float(lr), int(step),
            C.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def init_learned(self, X, K, params, N=None, P=4096, seed=0, idx=None):
        """K x 3 initial centres proposed by the network from a seeded sample
        of P points of X (drawn with replacement; float64, host).  Raises
        KMeansError if the network yields a non-finite centre."""
        ptr, n, ld, d = self._points(X, N)
        if d != 3:
            raise ValueError("the learned initialiser takes 3-D points")
        if idx is None:
            rng = np.random.Generator(np.random.PCG64(seed))
            idx = self._torch.from_numpy(rng.integers(0, n, size=P).astype(np.int32)).to(X.device)
        out = np.empty((K, 3), np.float64)
        self._check(self._lib.kmeans_init_learned(self._ctx, ptr, n, ld, K, idx.data_ptr(),
                                                  idx.numel(), params.data_ptr(), _dptr(out)))
        return out

    def pp_init(self, X, K, u=None, seed=0, N=None, return_index=False):
        """k-means++ initial centres (K x d float64, host) from the uniforms u
        (K values in [0, 1); drawn from a PCG64 generator seeded with `seed`
        when not given)."""
        ptr, n, ld, d = self._points(X, N)
        if u is None:
            u = np.random.Generator(np.random.PCG64(seed)).random(K)
        u = _f64(u)
        if u.size != K:
            raise ValueError(f"u holds {u.size} values, K = {K}")
        out = np.empty((K, d), np.float64)
        idx = np.empty(K, np.int64)
        self._check(self._lib.kmeans_pp_init(self._ctx, ptr, n, ld, d, K, _dptr(u), _dptr(out),
                                             idx.ctypes.data_as(C.POINTER(C.c_int64))))
        return (out, idx) if return_index else out

    def measure_peaks(self):
        """Measured rates on this device: non-packed FP32 FMA, v_min3 and
        v_med3 in lane-operations/s, and the HBM read rate in bytes/s."""
        r = np.zeros(4, np.float64)
        self._check(self._lib.kmeans_measure_peaks(self._ctx, _dptr(r)))
        return {"fma_lane_ops_per_s": r[0], "min3_lane_ops_per_s": r[1],
                "med3_lane_ops_per_s": r[2], "hbm_read_bytes_per_s": r[3]}

    def history(self, cap: int = 1 << 20):
        E = np.empty(cap, np.float64)
        J = np.empty(cap, np.float64)
        n = self._lib.kmeans_get_history(self._ctx, _dptr(E), _dptr(J), cap)
        if n < 0:
            self._check(n)
        return E[:n].copy(), J[:n].copy()

    def changes(self, cap: int = 1 << 20):
        """Per-update changed-label counts of the last fit (KM_OPT_TRACK)."""
        out = np.empty(cap, np.int64)
        n = self._lib.kmeans_get_changes(self._ctx, out.ctypes.data_as(C.c_void_p), cap)
        if n < 0:
            self._check(n)
        return out[:n].copy()

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
