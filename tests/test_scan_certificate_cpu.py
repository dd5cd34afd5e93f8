"""The reassignment scan's certificate, checked on the CPU: the library's own
device header (lloyd_device.h: nearest4 and its centre tables) is compiled
for the host with g++ (tests/host_scan: a stand-in for the HIP runtime
header; the one inline-assembly bitfield insert is replaced by the same bit
operation in C, and the clang vector type of the loads by a plain struct),
and run on adversarial inputs.  Every point the scan
certifies must carry the exact label -- the first index of the minimum of
the float64 direct-form distance to the float32 centres, as the oracle
computes it -- whatever the data: offsets far from the origin, outliers,
near-duplicate centres, exact ties, extreme scales, K not a multiple of 3.
Points it does not certify go to the float64 re-scan (covered by the GPU
tests); here they only have to be a minority where the data allow it."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2405_12052_amd", "csrc")
BFI_ASM = 'asm("v_bfi_b32 %0, 31, %1, %2" : "=v"(r) : "s"(g), "v"(v));'
BFI_C = "r = __uint_as_float((__float_as_uint(v) & ~31u) | ((uint32_t)g & 31u));"
# the clang vector type of the global loads, as a plain struct for g++ (which
# ignores the address-space attribute of the pointer typedefs)
VEC4 = "typedef float f32x4 __attribute__((ext_vector_type(4)));"
VEC4_C = "struct f32x4 { float x, y, z, w; };"


@pytest.fixture(scope="module")
def scan(tmp_path_factory):
    d = tmp_path_factory.mktemp("host_scan")
    src = open(os.path.join(CSRC, "lloyd_device.h")).read()
    assert src.count(BFI_ASM) == 1, "the bitfield insert of with_index moved"
    assert src.count(VEC4) == 1, "the vector type of load_group moved"
    open(d / "lloyd_device_host.h", "w").write(src.replace(BFI_ASM, BFI_C).replace(VEC4, VEC4_C))
    lib = d / "scan_host.so"
    cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-Wno-unknown-pragmas", "-Wno-attributes", "-I", str(d), "-I", os.path.join(HERE, "host_scan"),
           "-I", CSRC, "-o", str(lib), os.path.join(HERE, "host_scan", "scan_host.cpp")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    so = C.CDLL(str(lib))
    so.scan_points_host.argtypes = [C.c_void_p, C.c_int64, C.c_int64, C.c_int, C.c_void_p,
                                    C.c_int, C.c_uint32, C.c_void_p, C.c_void_p]
    so.scan_points_host.restype = C.c_int

    def run(X, mu):
        X = np.ascontiguousarray(X, np.float32)
        d_, N = X.shape
        mu32 = np.zeros((mu.shape[0], 4), np.float32)
        mu32[:, :d_] = mu.astype(np.float32)
        xmax = np.float32(np.abs(X).max()).view(np.uint32)
        arg = np.empty(N, np.int32)
        ok = np.empty(N, np.int32)
        rc = so.scan_points_host(X.ctypes.data, N, N, d_, mu32.ctypes.data, mu.shape[0],
                                 int(xmax), arg.ctypes.data, ok.ctypes.data)
        assert rc == 0
        return arg, ok.astype(bool)
    return run


def check(scan, X, mu, min_certified=0.0):
    X = np.ascontiguousarray(X, np.float32)
    arg, ok = scan(X, mu)
    ref, dmin, dsec = oracle.assign(X, mu)
    wrong = ok & (arg != ref)
    assert not wrong.any(), (f"{int(wrong.sum())} certified labels differ from the exact argmin "
                             f"(first at {int(np.flatnonzero(wrong)[0])})")
    assert ok.mean() >= min_certified, ok.mean()
    return ok.mean()


def test_mixture_at_scale_and_offset(scan):
    rng = np.random.default_rng(1)
    for d in (2, 3):
        for K in (1, 2, 3, 4, 5, 7, 16, 31, 61, 63, 64):
            c = rng.uniform(-100, 100, size=(K, d))
            X = (c[rng.integers(0, K, 20_000)] + rng.normal(size=(20_000, d)) * 3).T
            mu = c + rng.normal(size=c.shape)
            check(scan, X, mu, min_certified=0.95)


def test_far_offsets_and_outliers(scan):
    """Data and centres at 1000 +- 3, outliers at +5000: the expanded keys
    cancel (|m|^2 ~ 3e6 against gaps of order 1), so the bound certifies few
    points (about 1 %) and the float64 re-scan takes the rest; the certified
    ones must still be exact."""
    rng = np.random.default_rng(2)
    N, K = 60_001, 40
    X = (rng.normal(size=(3, N)) * 3 + 1000.0)
    X[:, ::97] += 5000.0
    mu = rng.normal(size=(K, 3)) * 3 + 1000.0
    assert check(scan, X, mu) > 0.0


def test_near_duplicate_centres(scan):
    """Pairs of centres one float32 unit apart: points near either are near
    ties, and a certified point must still get the lower-distance (or, on an
    exact tie, the lower) index."""
    rng = np.random.default_rng(3)
    for d in (2, 3):
        base = rng.uniform(-50, 50, size=(20, d)).astype(np.float32)
        twin = np.nextafter(base, np.float32(np.inf))
        mu = np.concatenate([base, twin]).astype(np.float64)[rng.permutation(40)]
        X = (mu[rng.integers(0, 40, 40_000)] + rng.normal(size=(40_000, d)) * 0.5).T
        check(scan, X, mu)


def test_exact_ties_on_a_grid(scan):
    rng = np.random.default_rng(4)
    for d in (2, 3):
        X = rng.integers(-5, 6, size=(d, 50_003)).astype(np.float64)
        mu = rng.integers(-5, 5, size=(48, d)) + 0.5
        mu[:, 0] = np.round(mu[:, 0])
        check(scan, X, mu)


@pytest.mark.parametrize("xs,ms", [(1e-15, 1e-15), (1e-3, 1e-3), (1e4, 1e4), (1e6, 1e6),
                                   (1.0, 1e6), (1e6, 1.0), (1.0, 0.0), (1e3, 1e-3)])
def test_extreme_scales(scan, xs, ms):
    rng = np.random.default_rng(5)
    for d in (2, 3):
        X = rng.normal(size=(d, 30_001)) * xs
        mu = rng.normal(size=(64, d)) * ms
        check(scan, X, mu)


def test_points_on_bisectors(scan):
    """Points placed exactly, then one unit in the last place off, the
    bisector of two centres: the keys' rounding decides, and only a bound
    that covers it keeps certified labels exact."""
    rng = np.random.default_rng(6)
    for d in (2, 3):
        K = 17
        mu = rng.uniform(-30, 30, size=(K, d)).astype(np.float32).astype(np.float64)
        a, b = rng.integers(0, K, 30_000), rng.integers(0, K, 30_000)
        t = rng.uniform(0.3, 0.7, size=(30_000, 1))
        mid = (mu[a] + mu[b]) / 2 + (rng.normal(size=(30_000, d)) * 1e-3) * (t - 0.5)
        X = mid.astype(np.float32)
        X = np.concatenate([X, np.nextafter(X, np.float32(np.inf)),
                            np.nextafter(X, np.float32(-np.inf))]).T.astype(np.float64)
        check(scan, X, mu)


def test_random_adversarial_batches(scan):
    """Mixed magnitudes within one data set: most points near the origin, a
    few far away (the bound grows with max|x|), centres drawn from the data
    and nudged."""
    rng = np.random.default_rng(7)
    for trial in range(12):
        d = int(rng.integers(2, 4))
        K = int(rng.integers(1, 65))
        N = 20_000
        X = rng.normal(size=(d, N)) * 10 ** rng.uniform(-2, 3)
        far = rng.random(N) < 0.001
        X[:, far] *= 10 ** rng.uniform(1, 4)
        idx = rng.choice(N, K, replace=False)
        mu = X[:, idx].T * (1 + rng.normal(size=(K, d)) * 1e-4)
        check(scan, X, mu)
