"""Training targets of the learned initialiser, computed by the FP64 oracle.

TEST/TRAINING INFRASTRUCTURE: this script calls only the oracle and the input
generators.  For each training instance (the C5 recipe -- 16 axis-aligned
Gaussian components in [-50, 50]^3, Dirichlet weights, 1% uniform noise --
drawn with N = 4096 points from seed base + i) it runs Lloyd's algorithm in
the oracle from 4 seeded samples of K = 16 points (E < 1e-6 or 300 updates)
and, with --means-start, also from the generator's 16 component means (an
informed start that usually reaches the best basin), keeps the run with the
smallest final objective, and stores its centres
normalised by the instance's point mean and scalar standard deviation
(x - mean) / s with s^2 = mean over points and coordinates of (x - mean)^2,
the same normalisation the network's input uses.

Output: an .npz with seeds [n] int64, targets [n, 16, 3] float32, J [n]
float64 (objective of the kept restart) and T [n, 4] int32 (updates per
restart; with --means-start a fifth column for the informed start).  Usage:
    python oracle/make_initnet_targets.py OUT.npz --n 200000 --base 1000000 --procs 8 [--means-start]
"""
from __future__ import annotations

import argparse
import os
import sys
import time
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

P_POINTS = 4096
K = 16
RESTARTS = 4


def instance_spec(seed: int):
    import datagen
    return datagen.spec("C5", N=P_POINTS, seed=seed, init_seed=seed)


def normalise(X):
    """Mean per coordinate and one scalar std over all coordinates."""
    m = X.astype(np.float64).mean(axis=1)
    s = float(np.sqrt(((X.astype(np.float64) - m[:, None]) ** 2).mean()))
    return m, s


MEANS_START = False


def one(seed: int):
    import datagen
    import oracle
    oracle.threads(1)
    s = instance_spec(seed)
    X, meta = datagen.generate(s, threads=1)
    starts = [datagen.init_sample(X, s.N, K, seed * 16 + r) for r in range(RESTARTS)]
    if MEANS_START:
        starts.append(np.asarray(meta["centres"], np.float64))
    best = None
    Ts = []
    for mu0 in starts:
        f = oracle.fit(X, mu0, tol=1e-6, max_iter=300, labels=False)
        Ts.append(f["T"])
        if best is None or f["J"] < best["J"]:
            best = f
    m, sd = normalise(X)
    tgt = ((best["mu"] - m[None, :]) / sd).astype(np.float32)
    return seed, tgt, best["J"], Ts


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("out")
    ap.add_argument("--n", type=int, default=200_000)
    ap.add_argument("--base", type=int, default=1_000_000)
    ap.add_argument("--procs", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--means-start", action="store_true")
    args = ap.parse_args()
    global MEANS_START
    MEANS_START = args.means_start
    seeds = list(range(args.base, args.base + args.n))
    t0 = time.time()
    res = []
    with Pool(args.procs) as pool:
        for i, r in enumerate(pool.imap(one, seeds, chunksize=64)):
            res.append(r)
            if (i + 1) % 5000 == 0:
                print(f"{i + 1}/{args.n} instances, {time.time() - t0:.0f}s", flush=True)
    seeds_a = np.array([r[0] for r in res], np.int64)
    tg = np.stack([r[1] for r in res]).astype(np.float32)
    J = np.array([r[2] for r in res], np.float64)
    T = np.array([r[3] for r in res], np.int32)
    tmp = args.out + ".tmp.npz"
    np.savez(tmp, seeds=seeds_a, targets=tg, J=J, T=T)
    os.replace(tmp, args.out)
    print(f"wrote {args.out}: {len(res)} instances in {time.time() - t0:.0f}s", flush=True)


if __name__ == "__main__":
    main()
