"""The C-ABI library without a GPU: it loads, exports every entry point that
include/kmeans.h declares, validates arguments on the host, and reports the
absence of a device."""
import ctypes
import os
import re
import subprocess

import pytest

import paper_2405_12052_amd as km

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(kmeans_\w+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    lib = km.load_library()
    names = declared_functions()
    assert {"kmeans_create", "kmeans_fit", "kmeans_assign"} <= names
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", km.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (kmeans_\w+)", out))
    assert names <= exported
    assert exported <= names, f"undeclared exports: {exported - names}"


def test_abi_version():
    assert km.load_library().kmeans_abi_version() == 2


@pytest.mark.parametrize("args,code", [
    ((100, 100, 3, 4, 1e-6, 10), km.KM_OK),
    ((100, 128, 2, 64, 0.0, 1), km.KM_OK),
    ((100, 100, 4, 4, 1e-6, 10), km.KM_OK),
    ((100, 100, 1, 4, 1e-6, 10), km.KM_OK),
    ((100, 100, 3, 65, 1e-6, 10), km.KM_OK),
    ((2000, 2000, 3, 1024, 1e-6, 10), km.KM_OK),
    ((2000, 2000, 16, 309, 1e-6, 10), km.KM_OK),
    ((2000, 2000, 16, 310, 1e-6, 10), km.KM_OK),       # the tiled general-shape kernels
    ((2000, 2000, 32, 160, 1e-6, 10), km.KM_OK),
    ((5000, 5000, 16, 4096, 1e-6, 10), km.KM_OK),
    ((5000, 5000, 32, 4096, 1e-6, 10), km.KM_OK),
    ((5000, 5000, 16, 4097, 1e-6, 10), km.KM_EUNSUPPORTED),
    ((2000, 2000, 33, 2, 1e-6, 10), km.KM_EUNSUPPORTED),
    ((5000, 5000, 2, 4097, 1e-6, 10), km.KM_EUNSUPPORTED),
    ((100, 100, 0, 4, 1e-6, 10), km.KM_EINVAL),
    ((10, 10, 2, 11, 1e-6, 10), km.KM_EINVAL),
    ((0, 0, 2, 1, 1e-6, 10), km.KM_EINVAL),
    ((100, 99, 2, 4, 1e-6, 10), km.KM_EINVAL),
    ((100, 100, 2, 0, 1e-6, 10), km.KM_EINVAL),
    ((100, 100, 2, 4, -1.0, 10), km.KM_EINVAL),
    ((100, 100, 2, 4, float("nan"), 10), km.KM_EINVAL),
    ((100, 100, 2, 4, float("inf"), 10), km.KM_EINVAL),
    ((100, 100, 2, 4, 1e-6, 0), km.KM_EINVAL),
    ((2 ** 31, 2 ** 31, 2, 4, 1e-6, 10), km.KM_EINVAL),
])
def test_host_validation(args, code):
    assert km.validate(*args) == code


def test_status_strings():
    lib = km.load_library()
    assert lib.kmeans_status_string(km.KM_EUNSUPPORTED) == b"KM_EUNSUPPORTED"
    assert lib.kmeans_status_string(7) == b"KM_UNKNOWN"


def test_create_without_gpu_reports_enodev():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    lib = km.load_library()
    ctx = ctypes.c_void_p()
    assert lib.kmeans_create(ctypes.byref(ctx), 0, None, 0) == km.KM_ENODEV
    assert ctx.value is None
    assert b"no HIP device" in lib.kmeans_last_error(None)
    assert lib.kmeans_create(ctypes.byref(ctx), 0, None, 1) == km.KM_EINVAL
    lib.kmeans_destroy(None)                      # accepted


def test_null_context_is_rejected():
    lib = km.load_library()
    assert lib.kmeans_fit(None, None, 10, 10, 2, 2, None, 1e-6, 10, None, None, None) == km.KM_EINVAL
    assert lib.kmeans_set_option(None, 1, 1) == km.KM_EINVAL


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2405_12052_amd import _binding
    monkeypatch.setattr(_binding, "_lib", None)
    monkeypatch.setattr(_binding, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="missing"):
        _binding.load_library()


def test_batched_descriptor_view_matches_the_struct():
    """The binding fills a batch's km_instance descriptors as one numpy record
    array; every field written through it reads back through the ctypes
    structure (and the result fields the library writes read back through it)."""
    import numpy as np

    from paper_2405_12052_amd import _binding as b

    dt = b._KM_INSTANCE_DT
    assert dt.itemsize == ctypes.sizeof(b.km_instance)
    a = np.zeros(3, dt)
    a["X"] = [0x1000, 0x2000, 0x3000]
    a["N"], a["ld"], a["d"], a["K"], a["n_restarts"] = [5, 6, 7], [8, 8, 12], [2, 3, 2], [4, 5, 6], [1, 8, 3]
    a["init"], a["centroids_out"], a["labels_out"] = [16, 32, 48], [64, 80, 96], [0, 112, 128]
    a["restart_objective"], a["restart_iters"] = [144, 160, 176], [192, 208, 224]
    s = (b.km_instance * 3).from_buffer(a)
    for i in range(3):
        assert s[i].X == int(a["X"][i]) and s[i].N == a["N"][i] and s[i].ld == a["ld"][i]
        assert (s[i].d, s[i].K, s[i].n_restarts) == (a["d"][i], a["K"][i], a["n_restarts"][i])
        assert ctypes.cast(s[i].init, ctypes.c_void_p).value == int(a["init"][i])
        assert ctypes.cast(s[i].centroids_out, ctypes.c_void_p).value == int(a["centroids_out"][i])
        assert (s[i].labels_out or 0) == int(a["labels_out"][i])
        assert ctypes.cast(s[i].restart_objective, ctypes.c_void_p).value == int(a["restart_objective"][i])
        assert ctypes.cast(s[i].restart_iters, ctypes.c_void_p).value == int(a["restart_iters"][i])
        s[i].best_restart, s[i].res.iters, s[i].res.converged = i + 1, 10 * i, i % 2
        s[i].res.E, s[i].res.objective, s[i].res.empty_events = 0.5 * i, 2.0 * i, 3 * i
    assert a["best_restart"].tolist() == [1, 2, 3] and a["iters"].tolist() == [0, 10, 20]
    assert a["converged"].tolist() == [0, 1, 0] and a["E"].tolist() == [0.0, 0.5, 1.0]
    assert a["objective"].tolist() == [0.0, 2.0, 4.0] and a["empty_events"].tolist() == [0, 3, 6]
