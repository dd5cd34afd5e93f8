"""Training and use of the learned initialiser (include/kmeans.h, "learned
initialiser").

The network is trained on the GPU by the library's own kernels
(kmeans_initnet_train_step: forward, Hungarian matching, backward, Adam).
Each training instance is a 4096-point sample of the C5 recipe (16 Gaussian
components in [-50, 50]^3, axis-aligned std U[0.5, 2], Dirichlet weights, 1%
uniform noise), regenerated here from its seed; its target is the set of
converged Lloyd centres stored in a target file (an .npz with `seeds` and
normalised `targets` [n, 16, 3], written by a separate script that runs the
float64 reference implementation).  Points and targets are normalised by the
instance's mean and scalar standard deviation.

    python -m paper_2405_12052_amd.initnet train TARGETS.npz OUT.npy [--epochs E]

The shipped weights (weights/initnet_c5_k16.npy) come from that command with
its defaults (40 epochs of Adam, batch 256, learning rate 5e-3 decaying
exponentially to 1e-4, 2048 instances held out) on 200,000 instances with
seeds 1,000,000 + i, targets from
    python oracle/make_initnet_targets.py T.npz --n 200000 --base 1000000
Held-out matched loss: 233.6 at initialisation, 11.56 after training (sum
over the 16 centres of squared errors in normalised units).
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

P_POINTS = 4096
K = 16
HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "weights", "initnet_c5_k16.npy")


def shapes(k):
    return [(3, 64), (64,), (64, 64), (64,), (128, 256), (256,), (256, 3 * k), (3 * k,)]


def init_params(k, seed=0):
    """He-normal weights, zero biases."""
    rng = np.random.default_rng(seed)
    out = []
    for s in shapes(k):
        if len(s) == 2:
            out.append(rng.normal(size=s) * np.sqrt(2.0 / s[0]))
        else:
            out.append(np.zeros(s))
    return np.concatenate([a.reshape(-1) for a in out]).astype(np.float32)


def instance_points(seed):
    """The normalised 4096-point training instance of `seed` [P, 3]."""
    sys.path.insert(0, os.path.dirname(HERE))
    import datagen
    s = datagen.spec("C5", N=P_POINTS, seed=int(seed), init_seed=int(seed))
    X, _ = datagen.generate(s, threads=1)
    X = X.astype(np.float64)
    m = X.mean(axis=1)
    sd = np.sqrt(((X - m[:, None]) ** 2).mean())
    return ((X - m[:, None]) / sd).T.astype(np.float32)


def _chunk_points(seeds):
    return np.stack([instance_points(s) for s in seeds])


def load_points(seeds, procs=16, chunk=1000):
    """Regenerate many instances with a pool of worker processes (numpy only;
    the workers never touch the GPU)."""
    import multiprocessing as mp
    out = np.empty((len(seeds), P_POINTS, 3), np.float32)
    parts = [list(seeds[a:a + chunk]) for a in range(0, len(seeds), chunk)]
    if len(parts) <= 1 or procs <= 1:
        for i, p in enumerate(parts):
            out[i * chunk:i * chunk + len(p)] = _chunk_points(p)
        return out
    with mp.get_context("spawn").Pool(procs) as pool:
        for i, arr in enumerate(pool.imap(_chunk_points, parts)):
            out[i * chunk:i * chunk + len(arr)] = arr
    return out


def load_training_set(targets_path, log=print):
    """(points [n, P, 3], targets [n, K, 3]) of a target file, as float32 CUDA
    tensors."""
    import torch
    d = np.load(targets_path)
    seeds, tg = d["seeds"], d["targets"].astype(np.float32)
    t0 = time.time()
    pts = load_points(seeds)
    log(f"regenerated {len(seeds)} training instances in {time.time() - t0:.1f}s")
    return torch.from_numpy(pts).cuda(), torch.from_numpy(tg).cuda()


def train(targets_path, out_path, epochs=40, batch=256, lr=5e-3, lr_end=1e-4, holdout=2048,
          seed=0, log=print, data=None):
    """Adam on the matched loss; the last `holdout` instances are held out.
    `data` = load_training_set(...) output, to reuse loaded points."""
    import torch
    from . import KMeans
    P, T = data if data is not None else load_training_set(targets_path, log)
    n = P.shape[0]
    dev = P.device
    n_train = n - holdout
    params = torch.from_numpy(init_params(K, seed)).to(dev)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    km = KMeans(0)
    rng = np.random.default_rng(seed)
    steps_per_epoch = n_train // batch
    total = epochs * steps_per_epoch
    step = 0
    hist = []

    def heldout_loss():
        losses = []
        for a in range(n_train, n, batch):
            b = min(n, a + batch)
            g, L, _ = km.initnet_grad(P[a:b].contiguous(), T[a:b].contiguous(), K, params)
            losses.append(L * (b - a))
        return float(np.sum(losses) / (n - n_train))

    log(f"held-out loss before training {heldout_loss():.4f}")
    t0 = time.time()
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(n_train)).to(dev)
        run = []
        for s in range(steps_per_epoch):
            step += 1
            frac = (step - 1) / max(1, total - 1)
            lr_t = lr * (lr_end / lr) ** frac
            idx = perm[s * batch:(s + 1) * batch]
            want = (s % 50) == 0
            L = km.initnet_train_step(P[idx].contiguous(), T[idx].contiguous(), K, params, m, v,
                                      lr_t, step, want_loss=want)
            if want:
                run.append(L)
        hl = heldout_loss()
        hist.append(hl)
        log(f"epoch {ep + 1}/{epochs}: train loss ~{np.mean(run):.4f}, held-out {hl:.4f}, "
            f"{time.time() - t0:.1f}s")
    w = params.cpu().numpy()
    os.makedirs(os.path.dirname(os.path.abspath(out_path)), exist_ok=True)
    np.save(out_path, w)
    km.close()
    return w, hist


def load_weights(path=DEFAULT_WEIGHTS):
    return np.load(path, allow_pickle=False).astype(np.float32)


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("targets")
    t.add_argument("out")
    t.add_argument("--epochs", type=int, default=40)
    t.add_argument("--batch", type=int, default=256)
    t.add_argument("--lr", type=float, default=5e-3)
    a = ap.parse_args()
    if a.cmd == "train":
        train(a.targets, a.out, epochs=a.epochs, batch=a.batch, lr=a.lr,
              log=lambda *x: print(*x, flush=True))


if __name__ == "__main__":
    main()
