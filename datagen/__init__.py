"""Seeded synthetic workloads for Lloyd's K-means (inputs only).

This module is shared by the tests, the benchmark and the CPU oracle's callers.
It draws data points and initial centroids and nothing else: it holds none of
the clustering arithmetic (no distances, no argmin, no means), so that the
oracle and the GPU path stay independent of each other.

The paper clusters its own 2-D and 3-D Gaussian-mixture datasets of 1e5..1e6
points (Serial Lloyd's Algorithm section); those files are not published, so the
recipes below stand in for them at the shapes of the benchmark workloads:

  C1  N=1e5,  d=2, 4 isotropic components (std 1), centres U[-10,10]^2, equal weights
  C2  N=1e7,  d=3, 16 axis-aligned components, per-axis std U[0.5,2], centres
      U[-50,50]^3, weights Dirichlet(1), plus 1% points uniform in the mixture's
      axis-aligned bounding box
  C3  N=2e8,  d=3, 64 isotropic components, std U[0.5,3], centres U[-100,100]^3,
      equal weights, drawn in 20 chunks of 1e7 from spawned seed streams
  C4  4096 instances, N=round(10^U[3,6]), d in {2,3}, K in U{2..32}, C2 recipe
  C5  N=1e6,  d=3, K=16, C2 recipe

Points are float32 in structure-of-arrays layout: an array of shape (d, N),
row j holding coordinate j of every point (the paper's X in R^{d x N}).
Initial centroids are K distinct data points chosen by a seeded generator
(the paper's initialisation step), widened exactly to float64.
"""
from __future__ import annotations

import concurrent.futures as _cf
import os
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "MixtureSpec", "CONFIGS", "spec", "generate", "init_sample", "batched_specs",
    "batched_generate", "round_up",
]


def round_up(n: int, m: int) -> int:
    return (n + m - 1) // m * m


@dataclass(frozen=True)
class MixtureSpec:
    """Parameters of one synthetic instance."""
    name: str
    N: int
    d: int
    K: int                    # clusters requested from Lloyd
    seed: int
    components: int = 0       # mixture components (defaults to K)
    box: float = 10.0         # centres ~ U[-box, box]^d
    std: tuple = (1.0, 1.0)   # std ~ U[std[0], std[1]]
    axis_aligned: bool = False  # per-axis std (True) or one std per component
    dirichlet: bool = False   # weights ~ Dirichlet(1) (True) or equal
    noise_frac: float = 0.0   # fraction of points uniform in the bounding box
    chunks: int = 1           # independent seed streams for the points
    init_seed: int = 0        # seed of the initial-centroid sample
    max_iter: int = 100
    tol: float = 1e-6
    extra: dict = field(default_factory=dict, compare=False)

    @property
    def n_components(self) -> int:
        return self.components or self.K


CONFIGS = {
    "C1": MixtureSpec("C1", N=100_000, d=2, K=4, seed=20240501, box=10.0,
                      std=(1.0, 1.0), init_seed=11, max_iter=100),
    "C2": MixtureSpec("C2", N=10_000_000, d=3, K=16, seed=20240502, box=50.0,
                      std=(0.5, 2.0), axis_aligned=True, dirichlet=True,
                      noise_frac=0.01, init_seed=12, max_iter=300),
    "C3": MixtureSpec("C3", N=200_000_000, d=3, K=64, seed=20240503, box=100.0,
                      std=(0.5, 3.0), chunks=20, init_seed=13, max_iter=50,
                      tol=0.0),
    "C5": MixtureSpec("C5", N=1_000_000, d=3, K=16, seed=20240505, box=50.0,
                      std=(0.5, 2.0), axis_aligned=True, dirichlet=True,
                      noise_frac=0.01, init_seed=15, max_iter=300),
    # beyond the paper's 2-D/3-D problem: 16-D points, K = 256
    "W1": MixtureSpec("W1", N=10_000_000, d=16, K=256, seed=20240506, box=50.0,
                      std=(0.5, 2.0), axis_aligned=True, dirichlet=True,
                      noise_frac=0.01, chunks=16, init_seed=16, max_iter=20,
                      tol=0.0),
}


def spec(name: str, **overrides) -> MixtureSpec:
    """The named workload, optionally with fields replaced (e.g. a smaller N)."""
    base = CONFIGS[name]
    if not overrides:
        return base
    d = {f: getattr(base, f) for f in base.__dataclass_fields__}
    d.update(overrides)
    return MixtureSpec(**d)


def _params(rng: np.random.Generator, s: MixtureSpec):
    C, d = s.n_components, s.d
    centres = rng.uniform(-s.box, s.box, size=(C, d))
    if s.axis_aligned:
        stds = rng.uniform(s.std[0], s.std[1], size=(C, d))
    else:
        stds = np.repeat(rng.uniform(s.std[0], s.std[1], size=(C, 1)), d, axis=1)
    if s.dirichlet:
        w = rng.dirichlet(np.ones(C))
    else:
        w = np.full(C, 1.0 / C)
    return centres, stds, w


def _chunk(seed_seq, n, centres, stds, w, equal_w, out):
    rng = np.random.Generator(np.random.PCG64(seed_seq))
    C, d = centres.shape
    if equal_w:
        comp = rng.integers(0, C, size=n)
    else:
        comp = rng.choice(C, size=n, p=w)
    eps = rng.standard_normal(size=(n, d))
    pts = centres[comp] + stds[comp] * eps          # float64
    out[:, :] = pts.T.astype(np.float32)


def generate(s: MixtureSpec, ld: int | None = None, threads: int | None = None):
    """Draw the points of instance `s`.

    Returns (X, meta): X is float32 with shape (d, ld) (ld >= N, default N); the
    first N columns are the points, padding columns are zero. meta holds the
    mixture parameters and the generating component of each mixture point
    (-1 for uniform noise points), for recovery tests.
    """
    ld = s.N if ld is None else ld
    assert ld >= s.N
    root = np.random.SeedSequence(s.seed)
    kids = root.spawn(2 + s.chunks)
    prng = np.random.Generator(np.random.PCG64(kids[0]))
    centres, stds, w = _params(prng, s)
    X = np.zeros((s.d, ld), dtype=np.float32)
    n_noise = int(round(s.noise_frac * s.N))
    n_mix = s.N - n_noise
    # mixture points fill positions [0, n_mix); noise (if any) is scattered below
    bounds = np.linspace(0, n_mix, s.chunks + 1).astype(np.int64)
    equal_w = not s.dirichlet
    jobs = []
    threads = threads or min(16, os.cpu_count() or 1)
    with _cf.ThreadPoolExecutor(max_workers=min(threads, s.chunks)) as ex:
        for c in range(s.chunks):
            a, b = int(bounds[c]), int(bounds[c + 1])
            jobs.append(ex.submit(_chunk, kids[2 + c], b - a, centres, stds, w,
                                  equal_w, X[:, a:b]))
        for j in jobs:
            j.result()
    comp_of = None
    if n_noise:
        nrng = np.random.Generator(np.random.PCG64(kids[1]))
        lo = X[:, :n_mix].min(axis=1).astype(np.float64)
        hi = X[:, :n_mix].max(axis=1).astype(np.float64)
        noise = nrng.uniform(lo, hi, size=(n_noise, s.d)).astype(np.float32).T
        # scatter: a seeded permutation of all N positions
        perm = nrng.permutation(s.N)
        allpts = np.concatenate([X[:, :n_mix], noise], axis=1)
        X[:, :s.N] = allpts[:, perm]
    meta = {"centres": centres, "stds": stds, "weights": w, "n_noise": n_noise}
    return X, meta


def init_sample(X: np.ndarray, N: int, K: int, seed: int) -> np.ndarray:
    """K distinct data points chosen without replacement, as float64 (K, d)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    idx = rng.choice(N, size=K, replace=False)
    return np.ascontiguousarray(X[:, idx].T.astype(np.float64))


def batched_specs(n_inst: int = 4096, seed: int = 20240504, restarts: int = 8,
                  n_range=(3.0, 6.0), k_range=(2, 32)):
    """Per-instance specs of the batched workload (C4): N log-uniform, d in
    {2,3}, K uniform, C2-style mixtures with K components, and `restarts`
    seeded initial samples per instance."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Ns = np.rint(10.0 ** rng.uniform(n_range[0], n_range[1], size=n_inst)).astype(np.int64)
    ds = rng.integers(2, 4, size=n_inst)
    Ks = rng.integers(k_range[0], k_range[1] + 1, size=n_inst)
    specs = []
    for i in range(n_inst):
        N, d, K = int(Ns[i]), int(ds[i]), int(Ks[i])
        K = min(K, N)
        specs.append(MixtureSpec(
            f"C4[{i}]", N=N, d=d, K=K, seed=seed * 7919 + i, box=50.0,
            std=(0.5, 2.0), axis_aligned=True, dirichlet=True, noise_frac=0.01,
            init_seed=seed * 104729 + i, max_iter=300,
            extra={"restart_seeds": [seed * 104729 + i * 131 + r for r in range(restarts)]}))
    return specs


def batched_generate(specs, restarts=None, threads=None):
    """Points and restart initialisations of a batch.

    Returns (flat, offsets, inits): flat is one float32 array holding every
    instance's (d, round_up(N, 4)) rows back to back (each instance starts at a
    multiple of 4 floats, so its rows are 16-byte aligned when the buffer is);
    offsets[i] is instance i's first element; inits[i] has shape (R, K, d), the
    R seeded samples of K distinct points (R = len(restart_seeds) unless
    `restarts` overrides it)."""
    offsets, total = [], 0
    for s in specs:
        offsets.append(total)
        total += s.d * round_up(s.N, 4)
    flat = np.zeros(total, dtype=np.float32)

    def one(i):
        s, off = specs[i], offsets[i]
        ld = round_up(s.N, 4)
        X, _ = generate(s, ld=ld, threads=1)
        flat[off:off + s.d * ld] = X.reshape(-1)
        seeds = s.extra.get("restart_seeds", [s.init_seed])
        if restarts is not None:
            seeds = [seeds[q % len(seeds)] + 7 * (q // len(seeds)) for q in range(restarts)]
        return np.stack([init_sample(X, s.N, s.K, sd) for sd in seeds])

    threads = threads or min(16, os.cpu_count() or 1)
    with _cf.ThreadPoolExecutor(max_workers=threads) as ex:
        inits = list(ex.map(one, range(len(specs))))
    return flat, offsets, inits
