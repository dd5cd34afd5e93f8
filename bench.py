"""Benchmark of the Lloyd K-means hot path on one MI355X.

One step = one complete kmeans_fit of the HBM-scale workload (N=2e8 points,
d=3, K=64 isotropic Gaussian mixture, float32 structure-of-arrays, 2.4 GB),
from a seeded sample of K data points, exactly 50 updates (tol = 0), then the
final labels against the last centres.  The points are resident in HBM
before the timed region.  Prints one JSON line with point-iterations/s, the
roofline position of the dominant kernel (the per-iteration kernel) and the
CPU oracle's rate on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Published MI355X peaks used for the roofline.
PEAK_FP32_TFLOPS = 157.3   # FP32 vector (packed FMA = 2 flop per lane)
PEAK_FP16_MFMA_TFLOPS = 2500.0  # dense fp16 matrix cores
PEAK_HBM_GBS = 8000.0


def alg_flops_per_point(d: int, K: int) -> int:
    """FP32 work of one point in one update: per centre d subtractions, d
    multiplies, d-1 adds and one compare; plus d+1 accumulation adds."""
    return 3 * d * K + (d + 1)


def alg_bytes_per_point(d: int) -> int:
    """One float32 read per coordinate; labels are written only after the
    last update and the centres and partials are < 0.1 %."""
    return 4 * d


def scan_tiles(K: int, keys: int) -> int:
    """Template argument of the iteration kernel the library runs for K
    centres under KM_OPT_KEYS = keys (0 = the VALU scan, 1 / 2 = matrix-core
    tiles of 32 centres): the library's automatic choice for keys = 0."""
    tiles = 2 if K > 32 else 1
    if keys == 1:
        return 0
    if keys == 2:
        return tiles
    return tiles if (24 < K <= 32 or K > 44) else 0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


KERNEL_SOURCES = ["lloyd_kernels.hip", "lloyd_device.h", "lloyd_mfma.h", "km_internal.h"]


def kernel_source_hash() -> str:
    """Hash of the sources the iteration kernel is compiled from."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2405_12052_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profile(name: str):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current kernel source; None otherwise."""
    p = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(p):
        return None
    try:
        rec = json.load(open(p))
    except ValueError:
        return None
    if rec.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline(X, mu0, n_sample: int, target_s: float = 12.0, threads: int = 0):
    """The FP64 oracle on the host cores over the first n_sample points of the
    same data and initial centres; as many updates as fit in ~target_s.
    threads: OpenMP threads (0 = all host cores)."""
    import oracle
    all_threads = oracle.threads()
    cores = oracle.threads(threads) if threads else all_threads
    try:
        Xs = X[:, :n_sample].copy()
        t = time.perf_counter()
        oracle.fit(Xs, mu0, tol=0.0, max_iter=1, labels=False)
        one = time.perf_counter() - t               # one update + one final pass
        iters = max(1, min(20, int(target_s / max(one / 1.5, 1e-3))))
        t = time.perf_counter()
        r = oracle.fit(Xs, mu0, tol=0.0, max_iter=iters, labels=False)
        el = time.perf_counter() - t
    finally:
        oracle.threads(all_threads)
    assert r["T"] == iters
    return {"value": n_sample * iters / el, "unit": "point-iters/s", "cores": cores,
            "kind": "oracle",
            "sample": f"first {n_sample} of the {X.shape[1]} points, same K={mu0.shape[0]} "
                      f"initial centres, {iters} float64 updates + final labels, {el:.1f} s"}


def bench_batched(args):
    """The batched workload: 4096 instances (N log-uniform in [1e3, 1e6], d in
    {2, 3}, K in [2, 32], C2-style mixtures), 8 seeded restarts each, to
    E < 1e-6 or 300 updates, best restart kept, labels written; one
    kmeans_fit_batched call per step with the schedule from the autotuner
    (searched on the whole batch, outside the timed region)."""
    import numpy as np
    import torch

    import datagen
    from paper_2405_12052_amd import KMeans

    t0 = time.time()
    specs = datagen.batched_specs(args.instances)
    flat, offs, inits = datagen.batched_generate(specs)
    log(f"generated {len(specs)} instances ({flat.nbytes / 1e9:.2f} GB) in {time.time() - t0:.1f}s")
    dev = torch.from_numpy(flat).cuda()
    inst = []
    for s, off, ini in zip(specs, offs, inits):
        ld = datagen.round_up(s.N, 4)
        inst.append((dev[off:off + s.d * ld].view(s.d, ld), s.N, ini))
    km = KMeans(0)
    t0 = time.time()
    if args.schedule:
        # a fixed schedule (A/B timing of kernel changes): team size, blocks per
        # compute unit, work threshold of the teams
        f = args.schedule.split(",")
        km.set_batched_schedule(int(f[0]), int(f[1]), float(f[2]), int(f[3]) if len(f) > 3 else 0,
                                int(f[4]) if len(f) > 4 else 0)
        sched = km.batched_schedule()
        log(f"fixed schedule: {sched}")
    else:
        sched = km.tune_batched(inst, tol=1e-6, max_iter=300,
                                cache_path=os.environ.get("KMEANS_TUNE_CACHE"))
        log(f"tuned on the {len(inst)} instances in {time.time() - t0:.1f}s: {sched}")
    for i in range(args.warmup):
        km.fit_batched(inst, tol=1e-6, max_iter=300)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for i in range(args.steps):
        out = km.fit_batched(inst, tol=1e-6, max_iter=300)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t) / args.steps
    pt_iters = sum(s.N * int(o["restart_iters"].sum()) for s, o in zip(specs, out))
    flops = sum(s.N * int(o["restart_iters"].sum()) * alg_flops_per_point(s.d, s.K)
                for s, o in zip(specs, out))
    achieved = flops / el / 1e12
    n_restarts = sum(len(i) for i in inits)
    res = {
        "metric": "Lloyd point-iters/s (batched restarts)", "value": pt_iters / el,
        "unit": "point-iters/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": el * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"batched: {len(specs)} instances x 8 restarts, N log-uniform "
                               f"[1e3,1e6], d in {{2,3}}, K in [2,32], E<1e-6 or 300 updates, "
                               f"best restart kept + its labels, one persistent launch",
                   "instances": len(specs), "restarts": n_restarts,
                   "points": int(sum(s.N for s in specs)), "schedule": sched,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS, "traffic": None,
                     "kernel": "batched_fit (whole call, updates only counted)"},
        "cpu_baseline": None,
    }
    print(json.dumps(res), flush=True)
    km.close()


def bench_wide(args):
    """The general-shape workload W1 (beyond the paper's 2-D/3-D problem):
    N = 1e7 points in 16 dimensions, K = 256, a Gaussian mixture with
    per-axis spreads and Dirichlet weights, float32 SoA (640 MB); one step =
    one kmeans_fit from a seeded sample of K points, exactly 20 updates
    (tol = 0), then the final labels.  Each update is two kernels
    (wide_update: reassignment and per-block sums; wide_reduce: totals and the
    float64 mean step); their time per update comes from HIP events around
    the graph replays on the library's stream."""
    import torch

    import datagen
    from paper_2405_12052_amd import KM_OPT_KEYS, KM_OPT_TIMING, KMeans

    over = {k: v for k, v in (("N", args.N), ("K", args.K), ("d", args.d)) if v is not None}
    s = datagen.spec("W1", **over)
    iters = s.max_iter
    t0 = time.time()
    X, _ = datagen.generate(s)
    mu0 = datagen.init_sample(X, s.N, s.K, s.init_seed)
    log(f"generated N={s.N} d={s.d} K={s.K} in {time.time() - t0:.1f}s")
    Xd = torch.from_numpy(X).cuda()
    torch.cuda.synchronize()
    km = KMeans(0)
    km.set_option(KM_OPT_TIMING, 1)
    km.set_option(KM_OPT_KEYS, args.keys)
    for i in range(args.warmup):
        r = km.fit(Xd, mu0, tol=0.0, max_iter=iters)
        log(f"warmup {i}: T={r.iters} J={r.objective:.6e}")
    torch.cuda.synchronize()
    kern_ms, kern_n = 0.0, 0
    t = time.perf_counter()
    for i in range(args.steps):
        r = km.fit(Xd, mu0, tol=0.0, max_iter=iters)
        ms, n = km.timing()
        kern_ms += ms
        kern_n += n
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    assert r.iters == iters
    per_update_s = kern_ms / kern_n / 1e3
    log(f"timed {args.steps} fits in {el:.3f}s; {per_update_s * 1e6:.1f} us per update "
        f"(wide_update + wide_reduce)")
    flops = alg_flops_per_point(s.d, s.K) * s.N
    achieved = flops / per_update_s / 1e12
    peaks = km.measure_peaks()
    fma_peak = 2.0 * peaks["fma_lane_ops_per_s"] / 1e12
    variant = wide_variant(s.d, s.K, args.keys)
    # the contraction on the matrix cores is priced at their fp16 peak (the
    # algorithmic flops count each of the d K multiply-adds once, the kernel
    # performs three fp16 products for each); otherwise the FP32 vector peak
    peak = PEAK_FP16_MFMA_TFLOPS if variant == "_mfma" else PEAK_FP32_TFLOPS
    roof = {"bound": "mfma" if variant == "_mfma" else "alu", "achieved": achieved, "peak": peak,
            "unit": "TFLOP/s", "frac": achieved / peak, "traffic": None,
            "frac_of_fp32_vector_peak": achieved / PEAK_FP32_TFLOPS,
            "kernel": f"wide_update{variant}<{s.d}> + wide_reduce (one update)",
            "avg_update_us": per_update_s * 1e6, "alg_flops_per_update": flops,
            "alg_bytes_per_update": alg_bytes_per_point(s.d) * s.N,
            "frac_of_measured_nonpacked_fma_peak": achieved / fma_peak}
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline ...")
        cpu = cpu_baseline(X, mu0, min(200_000, s.N))
        log(f"cpu baseline {cpu['value']:.3e} pt-it/s on {cpu['cores']} threads")
    out = {
        "metric": "Lloyd point-iters/s (general shape)", "value": s.N * iters * args.steps / el,
        "unit": "point-iters/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"general shape W1: N={s.N}, d={s.d}, K={s.K} Gaussian mixture "
                               f"(per-axis spreads, Dirichlet weights), float32 SoA, "
                               f"seeded-sample init, {iters} updates (tol=0) + final labels",
                   "N": s.N, "d": s.d, "K": s.K, "iterations": iters,
                   "parallelism": "single GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "measured_peaks": {"fp32_fma_nonpacked_tflops": fma_peak},
    }
    print(json.dumps(out), flush=True)
    km.close()


def wide_variant(d, K, keys):
    """The general-shape update kernel's suffix for (d, K) and KM_OPT_KEYS
    (the selection rules stated in include/kmeans.h)."""
    w = d if d <= 4 else next(v for v in (6, 8, 12, 16, 24, 32) if d <= v)
    if w in (8, 12, 16) and keys != 1 and (keys == 2 or K >= 64):
        kt = (K + 31) // 32
        steps = (3 * (w // 2) + 7) // 8
        lds = ((8 * K * (d + 1) + 63) & ~63) + kt * steps * 1024 + kt * 128 + 4272
        if lds <= 65536:
            return "_mfma"
    return "_tiled" if wide_tiled(d, K) else ""


def wide_tiled(d, K):
    """Whether (d, K) exceeds one block's LDS and takes the tiled general-shape
    kernels (the shape rule stated in include/kmeans.h)."""
    w = d if d <= 4 else next(v for v in (6, 8, 12, 16, 24, 32) if d <= v)
    s = (w + 3) & ~3
    kp = 3 * ((K + 2) // 3)
    r16 = lambda n: (n + 15) & ~15
    return r16(8 * K * (d + 1)) + 4 * kp * s + r16(4 * kp) + 2224 > 65536


def _c5_instance(seed):
    import datagen
    s = datagen.spec("C5", seed=int(seed), init_seed=int(seed))
    X, _ = datagen.generate(s, threads=1)
    return int(seed), X


def c5_instances(seeds, workers: int = 8):
    """The held-out C5 instances, in seed order, drawn by host threads (numpy
    releases the interpreter lock while it draws): no child processes, so a
    profiled run holds one process on the GPU."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=workers) as ex:
        yield from ex.map(_c5_instance, seeds)


def converge_run(km, Xd, mu0, N, tol=1e-6, max_iter=1000, repeats=3):
    """kmeans_fit from mu0 to E < tol (cap max_iter) on resident points: the
    wall-clock span of the call, median of `repeats` (identical results)."""
    import numpy as np
    import torch
    times = []
    for _ in range(repeats):
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = km.fit(Xd, mu0, tol=tol, max_iter=max_iter, labels=False)
        times.append(time.perf_counter() - t)
    s = float(np.median(times))
    return {"tol": tol, "max_iter": max_iter, "T": r.iters, "converged": bool(r.converged),
            "E": r.E, "objective": r.objective, "ms": s * 1e3,
            "point_iters_per_s": N * r.iters / s}


def time_to_converge(km, X, Xd, N, K, seed, method, weights=None, repeats=3):
    """One initialisation method followed by kmeans_fit (E < 1e-6 or 300
    updates) on resident points; the wall-clock span covers the
    initialisation (sampling, seeding or network inference included), the
    fit and its final synchronisation.  Median over `repeats` runs (all runs
    give identical results).  Returns (seconds, updates, objective, fell_back)."""
    import numpy as np
    import torch

    import datagen
    from paper_2405_12052_amd import KMeansError
    times = []
    for _ in range(repeats):
        torch.cuda.synchronize()
        t = time.perf_counter()
        fell_back = False
        if method == "sample":
            mu0 = datagen.init_sample(X, N, K, seed)
        elif method == "kmeans++":
            mu0 = km.pp_init(Xd, K, seed=seed)
        elif method == "learned":
            rng = np.random.Generator(np.random.PCG64(seed))
            idx = torch.from_numpy(rng.integers(0, N, size=4096).astype(np.int32)).to(
                Xd.device, non_blocking=True)
            try:
                mu0 = km.init_learned(Xd, K, weights, idx=idx)
            except KMeansError:
                mu0 = datagen.init_sample(X, N, K, seed)
                fell_back = True
        else:
            raise ValueError(method)
        r = km.fit(Xd, mu0, tol=1e-6, max_iter=300, labels=False)
        times.append(time.perf_counter() - t)
    return float(np.median(times)), r.iters, r.objective, fell_back


def learned_vs_plain(km, seeds, weights, repeats=3, progress=False):
    """Time-to-converge from a seeded sample of data points, from k-means++ and
    from the learned initialiser on the held-out C5 instances `seeds` (N=1e6,
    d=3, K=16: 16 axis-aligned Gaussian components in [-50, 50]^3, Dirichlet
    weights, 1% uniform noise).  Per method: the median time-to-converge, the
    mean updates, the geometric-mean ratios of time and objective to the seeded
    sample, and the share of instances whose objective is within 0.1% of the
    seeded sample's (or lower), alone and together with a shorter wall-clock
    time."""
    import numpy as np
    import torch

    methods = ["sample", "kmeans++", "learned"]
    rec = {m: [] for m in methods}
    K, N = 16, 1_000_000
    t0 = time.time()
    warm = False
    for n_done, (seed, X) in enumerate(c5_instances(seeds)):
        Xd = torch.from_numpy(X).cuda()
        if not warm:        # first-call set-up (graphs, workspaces) out of the records
            for m in methods:
                time_to_converge(km, X, Xd, N, K, seed, m, weights, repeats=1)
            warm = True
        for m in methods:
            rec[m].append(time_to_converge(km, X, Xd, N, K, seed, m, weights, repeats))
        if progress and (n_done + 1) % 10 == 0:
            log(f"{n_done + 1}/{len(seeds)} instances, {time.time() - t0:.0f}s")
        del Xd
    a = {m: np.array([r[:3] for r in rec[m]], np.float64) for m in methods}
    base = a["sample"]
    summary = {}
    for m in methods:
        summary[m] = {
            "median_ms": float(np.median(a[m][:, 0]) * 1e3),
            "mean_updates": float(a[m][:, 1].mean()),
            "geomean_time_ratio": float(np.exp(np.mean(np.log(a[m][:, 0] / base[:, 0])))),
            "geomean_J_ratio": float(np.exp(np.mean(np.log(a[m][:, 2] / base[:, 2])))),
            "share_J_within_0.1pct": float(np.mean(a[m][:, 2] <= 1.001 * base[:, 2])),
            "share_J_within_0.1pct_and_faster": float(
                np.mean((a[m][:, 2] <= 1.001 * base[:, 2]) & (a[m][:, 0] < base[:, 0]))),
        }
    summary["learned"]["fallbacks"] = int(sum(r[3] for r in rec["learned"]))
    summary["per_instance"] = [
        {"seed": int(sd), **{m: {"ms": float(a[m][i, 0] * 1e3), "T": int(a[m][i, 1]),
                                "J": float(a[m][i, 2])} for m in methods}}
        for i, sd in enumerate(seeds)]
    return summary


def bench_learned(args):
    """Learned initialiser against a seeded sample of data points and against
    k-means++ on held-out instances of the N=1e6, d=3, K=16 mixture, seeds
    9_000_000 + i, disjoint from the training seeds (learned_vs_plain)."""
    import torch

    from paper_2405_12052_amd import KMeans, initnet
    # instances are drawn by threads of this process (c5_instances); the GPU is
    # initialised here, before any of them
    weights = torch.from_numpy(initnet.load_weights(args.weights or initnet.DEFAULT_WEIGHTS)).cuda()
    km = KMeans(0)
    seeds = [9_000_000 + i for i in range(args.instances)]
    summary = learned_vs_plain(km, seeds, weights, args.repeats, progress=True)
    km.close()
    L = summary["learned"]
    res = {
        "metric": "time-to-converge, learned init vs seeded sample (geomean ratio)",
        "value": L["geomean_time_ratio"], "unit": "ratio", "n_gpus": 1,
        "steps": len(seeds), "warmup": 1, "ms_per_step": L["median_ms"],
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{len(seeds)} held-out instances, N=1e6, d=3, K=16, E<1e-6 or "
                               "300 updates; time spans init + fit + sync on resident points",
                   "parallelism": "single GPU", "repeats": args.repeats},
        "methods": summary,
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(res), flush=True)


def bench_configs(args):
    """Time-to-converge on the small and medium workloads (N=1e5 2-D K=4;
    N=1e7 3-D K=16; N=1e6 3-D K=16) and on the shapes of the paper's timing
    tables (2-D N=5e5 and 3-D N=1e6 with K = 4, 8, 11), and two fixed-K series
    over N (2-D K=8, 3-D K=4: its Tables 2-3 and time-vs-N figures), on
    synthetic stand-ins of its unpublished Gaussian-mixture datasets: GPU
    (kmeans_fit, points resident) beside the float64 CPU oracle with 1 .. all
    host threads up to 2e6 points, with the speedup T_1/T_p and efficiency
    speedup/p of the oracle's threads.  E < 1e-6, as the paper's tolerance, or
    the workload's cap."""
    import numpy as np
    import torch

    import datagen
    import oracle
    from paper_2405_12052_amd import KMeans

    km = KMeans(0)
    all_threads = oracle.threads()
    thread_counts = sorted({t for t in (1, 2, 4, 8, 16, all_threads) if t <= all_threads})

    def gpu_time(Xd, mu0, max_iter):
        times = []
        for _ in range(4):
            torch.cuda.synchronize()
            t = time.perf_counter()
            r = km.fit(Xd, mu0, tol=1e-6, max_iter=max_iter, labels=False)
            times.append(time.perf_counter() - t)
        return float(np.median(times[1:])), r.iters, r.objective

    def oracle_time(X, mu0, max_iter, p, updates_cap=None):
        oracle.threads(p)
        mi = max_iter if updates_cap is None else min(max_iter, updates_cap)
        t = time.perf_counter()
        f = oracle.fit(X, mu0, tol=1e-6, max_iter=mi, labels=False)
        return time.perf_counter() - t, f["T"], f["J"]

    rows = []
    cases = [("N=1e5, d=2, K=4 (isotropic, equal weights)", datagen.spec("C1"), 100, True),
             ("N=1e6, d=3, K=16 (axis-aligned, Dirichlet, 1% noise)", datagen.spec("C5"), 300, True),
             ("N=1e7, d=3, K=16 (axis-aligned, Dirichlet, 1% noise)", datagen.spec("C2"), 300, True)]
    for K in (4, 8, 11):
        cases.append((f"paper Table 1 shape: N=5e5, d=2, K={K}",
                      datagen.spec("C1", N=500_000, K=K, seed=31000 + K), 1000, True))
        cases.append((f"paper Table 1 shape: N=1e6, d=3, K={K}",
                      datagen.spec("C2", N=1_000_000, K=K, seed=32000 + K), 1000, True))
    # the paper's Tables 2 (2-D, K = 8) and 3 (3-D, K = 4) and its time-vs-N
    # figures: fixed-K series over N, beside the oracle up to 2e6 points and
    # on the GPU alone beyond
    for N in (100_000, 200_000, 500_000, 1_000_000, 2_000_000, 10_000_000, 100_000_000):
        cases.append((f"series 2-D K=8 (paper Table 2 shape): N={N}",
                      datagen.spec("C1", N=N, K=8, seed=33000 + N // 1000), 1000, N <= 2_000_000))
    for N in (100_000, 200_000, 400_000, 800_000, 1_000_000, 2_000_000, 10_000_000, 100_000_000):
        cases.append((f"series 3-D K=4 (paper Table 3 shape): N={N}",
                      datagen.spec("C2", N=N, K=4, seed=34000 + N // 1000), 1000, N <= 2_000_000))
    for name, s, max_iter, with_oracle in cases:
        X, _ = datagen.generate(s)
        Xd = torch.from_numpy(X).cuda()
        mu0 = datagen.init_sample(X, s.N, s.K, s.init_seed)
        g_s, g_T, g_J = gpu_time(Xd, mu0, max_iter)
        row = {"workload": name, "N": s.N, "d": s.d, "K": s.K, "T": g_T,
               "gpu_ms": g_s * 1e3, "gpu_point_updates_per_s": s.N * g_T / g_s, "oracle": {}}
        if with_oracle:
            big = s.N * s.K > 5e7
            for p in thread_counts:
                # a bounded number of updates on one thread for the largest case
                cap = 5 if (big and p == 1) else None
                o_s, o_T, o_J = oracle_time(X, mu0, max_iter, p, cap)
                row["oracle"][str(p)] = {"s": o_s, "T": o_T, "point_updates_per_s": s.N * o_T / o_s}
                if cap is None:
                    # the same run: same number of updates, same objective
                    row["oracle"][str(p)]["same_T"] = o_T == g_T
                    row["oracle"][str(p)]["J_rel_diff"] = abs(o_J - g_J) / max(abs(o_J), 1e-300)
            # speedup psi_p = T_1 / T_p and efficiency eps_p = psi_p / p of the
            # oracle's threads (the paper's scaling measures), and the GPU's
            # speedup over one and over all host threads; a capped one-thread
            # run is scaled to the full T from its rate
            o1 = row["oracle"]["1"]
            t1 = o1["s"] if o1["T"] == g_T else o1["s"] * g_T / o1["T"]
            row["t1_estimated_from_rate"] = o1["T"] != g_T
            tp = {p: (t1 if p == "1" else row["oracle"][p]["s"]) for p in row["oracle"]}
            row["speedup"] = {p: t1 / tp[p] for p in row["oracle"]}
            row["efficiency"] = {p: row["speedup"][p] / int(p) for p in row["oracle"]}
            row["gpu_speedup_vs_1_thread"] = t1 / g_s
            row["gpu_speedup_vs_all_threads"] = row["oracle"][str(all_threads)]["s"] / g_s
        rows.append(row)
        msg = f"{name}: T={g_T} GPU {g_s * 1e3:.2f} ms"
        if with_oracle:
            msg += f", oracle {all_threads} threads {row['oracle'][str(all_threads)]['s'] * 1e3:.1f} ms"
        log(msg)
        del Xd
    oracle.threads(all_threads)
    km.close()
    res = {"metric": "time-to-converge (E < 1e-6), GPU vs CPU oracle", "value": rows[0]["gpu_ms"],
           "unit": "ms", "n_gpus": 1, "steps": len(rows), "warmup": 1,
           "ms_per_step": rows[0]["gpu_ms"], "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "configs and the shapes of the paper's timing tables",
                      "oracle_threads": thread_counts, "parallelism": "single GPU"},
           "rows": rows, "roofline": None, "cpu_baseline": None}
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--iters", type=int, default=50)
    ap.add_argument("--N", type=int, default=None, help="override N (testing only)")
    ap.add_argument("--K", type=int, default=None,
                    help="default workload only: K centres seeded from the same K=64 mixture "
                         "(testing only)")
    ap.add_argument("--d", type=int, default=None,
                    help="--workload wide only: dimension of the points (testing only)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-converge", action="store_true",
                    help="default workload: skip the run to E < 1e-6 and the learned-vs-plain "
                         "comparison")
    ap.add_argument("--learned-instances", type=int, default=16,
                    help="default workload: held-out N=1e6 instances of the learned-vs-plain "
                         "comparison (0: none)")
    ap.add_argument("--cpu-sample", type=int, default=20_000_000)
    ap.add_argument("--workload", choices=["hbm", "batched", "learned", "configs", "wide"],
                    default="hbm",
                    help="hbm: the N=2e8, K=64 fit (default); batched: 4096 instances; "
                         "wide: N=1e7, d=16, K=256 (general-shape kernels); "
                         "learned: learned init vs seeded sample and k-means++ on N=1e6, K=16; "
                         "configs: time-to-converge on smaller workloads and the paper's table "
                         "shapes, GPU beside the CPU oracle")
    ap.add_argument("--instances", type=int, default=None,
                    help="instances (batched: 4096, learned: 100)")
    ap.add_argument("--repeats", type=int, default=3)
    ap.add_argument("--schedule", default=None, metavar="TEAM,BLOCKS_PER_CU,BIG_WORK[,RESTART_GROUP[,MFMA_MIN_K]]",
                    help="--workload batched: use this schedule instead of the autotuner's")
    ap.add_argument("--weights", default=None, help="learned initialiser weights (.npy)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="before the workload, copy a device buffer of BYTES twice (a plain "
                         "copy kernel of known size, to calibrate traffic counters)")
    ap.add_argument("--print-source-hash", action="store_true")
    ap.add_argument("--track", action="store_true",
                    help="time the fits with indicator tracking on (KM_OPT_TRACK: labels read "
                         "and rewritten every update, changed-label counts)")
    ap.add_argument("--keys", type=int, default=0, choices=[0, 1, 2],
                    help="reassignment scan (KM_OPT_KEYS): 0 automatic (matrix cores at K = 64), "
                         "1 VALU, 2 matrix cores")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU data-parallel design is described, not built)", file=sys.stderr)
        sys.exit(2)

    if args.print_source_hash:
        print(kernel_source_hash())
        return
    if args.copy_probe:
        import torch
        n = args.copy_probe // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(2):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        log(f"copy probe: 2 x {args.copy_probe} bytes")
    if args.workload == "batched":
        args.instances = args.instances or 4096
        bench_batched(args)
        return
    if args.workload == "learned":
        args.instances = args.instances or 100
        bench_learned(args)
        return
    if args.workload == "configs":
        bench_configs(args)
        return
    if args.workload == "wide":
        bench_wide(args)
        return

    import numpy as np
    import torch

    import datagen
    from paper_2405_12052_amd import KM_OPT_KEYS, KM_OPT_TIMING, KM_OPT_TRACK, KMeans

    s = datagen.spec("C3") if args.N is None else datagen.spec("C3", N=args.N)
    K = s.K if args.K is None else args.K
    t0 = time.time()
    X, _ = datagen.generate(s)
    mu0 = datagen.init_sample(X, s.N, K, s.init_seed)
    log(f"generated N={s.N} d={s.d} K={K} in {time.time() - t0:.1f}s")
    Xd = torch.from_numpy(X).cuda()
    torch.cuda.synchronize()

    km = KMeans(0)
    km.set_option(KM_OPT_TIMING, 1)
    km.set_option(KM_OPT_KEYS, args.keys)
    km.set_option(KM_OPT_TRACK, 1 if args.track else 0)
    for i in range(args.warmup):
        r = km.fit(Xd, mu0, tol=0.0, max_iter=args.iters)
        log(f"warmup {i}: T={r.iters} J={r.objective:.6e}")
    torch.cuda.synchronize()
    kern_ms, kern_n = 0.0, 0
    t = time.perf_counter()
    for i in range(args.steps):
        r = km.fit(Xd, mu0, tol=0.0, max_iter=args.iters)
        ms, n = km.timing()
        kern_ms += ms
        kern_n += n
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    assert r.iters == args.iters
    if args.track:
        log(f"changed labels per update: {km.changes()[:5].tolist()} ... {km.changes()[-3:].tolist()}")
        km.set_option(KM_OPT_TRACK, 0)
    log(f"timed {args.steps} fits in {el:.3f}s; iteration kernel {kern_ms / kern_n * 1e3:.1f} us")

    pt_iters = s.N * args.iters * args.steps
    value = pt_iters / el
    avg_kernel_s = kern_ms / kern_n / 1e3
    flops = alg_flops_per_point(s.d, K) * s.N
    achieved = flops / avg_kernel_s / 1e12
    roof = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_TFLOPS,
            "traffic": (traffic_from_profile("lloyd_iter_C3_traffic.json")
                        if args.keys == 0 and args.N is None and args.K is None
                        and not args.track else None),
            "kernel": f"lloyd_iter{'_track' if args.track else ''}<{s.d},true,"
                      f"{scan_tiles(K, args.keys)}>",
            "avg_launch_us": avg_kernel_s * 1e6,
            "alg_flops_per_launch": flops,
            "alg_bytes_per_launch": alg_bytes_per_point(s.d) * s.N,
            "hbm_gbs_alg": alg_bytes_per_point(s.d) * s.N / avg_kernel_s / 1e9}
    # measured issue rates of the scan's instructions and the HBM read rate
    peaks = km.measure_peaks()
    roof["frac_of_measured_nonpacked_fma_peak"] = achieved / (2.0 * peaks["fma_lane_ops_per_s"] / 1e12)
    measured = {"fp32_fma_nonpacked_tflops": 2.0 * peaks["fma_lane_ops_per_s"] / 1e12,
                "v_min3_tops": peaks["min3_lane_ops_per_s"] / 1e12,
                "v_med3_tops": peaks["med3_lane_ops_per_s"] / 1e12,
                "hbm_read_gbs": peaks["hbm_read_bytes_per_s"] / 1e9}
    log(f"measured peaks: {measured}")
    # the metric's second half, outside the timed region: time to converge
    # (E < 1e-6) on this workload, and learned vs plain initialisation
    ttc = None
    if not args.no_converge and args.N is None and args.K is None:
        ttc = {"C3_run_to_tol": converge_run(km, Xd, mu0, s.N)}
        log(f"converge run: {ttc['C3_run_to_tol']}")
        if args.learned_instances > 0:
            from paper_2405_12052_amd import initnet
            weights = torch.from_numpy(initnet.load_weights(initnet.DEFAULT_WEIGHTS)).cuda()
            seeds = [9_000_000 + i for i in range(args.learned_instances)]
            summ = learned_vs_plain(km, seeds, weights, repeats=3)
            summ.pop("per_instance")
            ttc["learned_vs_plain"] = {
                "workload": f"{len(seeds)} held-out instances (seeds 9000000+i), N=1e6, d=3, "
                            "K=16 axis-aligned mixture with 1% noise; E<1e-6 or 300 updates; "
                            "time spans init + fit + sync, points resident; median of 3",
                "methods": summ}
            log(f"learned vs plain: {summ}")
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline ...")
        cpu = cpu_baseline(X, mu0, min(args.cpu_sample, s.N))
        log(f"cpu baseline {cpu['value']:.3e} pt-it/s on {cpu['cores']} threads")
        one = cpu_baseline(X, mu0, min(args.cpu_sample // 10, s.N), target_s=8.0, threads=1)
        cpu["single_thread"] = {k: one[k] for k in ("value", "unit", "cores", "sample")}
        log(f"cpu baseline {one['value']:.3e} pt-it/s on 1 thread")
    out = {
        "metric": "Lloyd point-iters/s", "value": value, "unit": "point-iters/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"plain Lloyd, HBM scale: N={s.N}, d={s.d}, K={K} isotropic "
                               f"Gaussian mixture, float32 SoA, seeded-sample init, "
                               f"{args.iters} updates (tol=0) + final labels",
                   "N": s.N, "d": s.d, "K": K, "iterations": args.iters,
                   "parallelism": "single GPU",
                   **({"indicator_tracking": True} if args.track else {})},
        "roofline": roof,
        "cpu_baseline": cpu,
        "measured_peaks": measured,
        "time_to_converge": ttc,
    }
    print(json.dumps(out), flush=True)
    km.close()


if __name__ == "__main__":
    main()
