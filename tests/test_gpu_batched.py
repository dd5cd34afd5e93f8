"""GPU tests of the batched persistent fit (many instances x restarts in one
launch): every restart equals a single kmeans_fit from the same initial
centres, the kept restart has the smallest objective, results do not depend
on the schedule, the kept restart matches the FP64 oracle, and the error
paths and the autotuner cache work."""
import json

import numpy as np
import pytest

import datagen
import oracle
from parity import centre_check, e_check, label_check

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def km():
    from paper_2405_12052_amd import KMeans
    k = KMeans(0)
    yield k
    k.close()


def log(*a):
    print(*a, flush=True)


def make_batch(n, seed, n_range=(3.0, 5.0), restarts=None):
    specs = datagen.batched_specs(n, seed=seed, n_range=n_range)
    flat, offs, inits = datagen.batched_generate(specs)
    if restarts is not None:
        rng = np.random.default_rng(seed)
        inits = [ini[:int(rng.integers(1, restarts + 1))] for ini in inits]
    dev = torch.from_numpy(flat).cuda()
    inst, host = [], []
    for s, off, ini in zip(specs, offs, inits):
        ld = datagen.round_up(s.N, 4)
        X = dev[off:off + s.d * ld].view(s.d, ld)
        inst.append((X, s.N, ini))
        host.append(flat[off:off + s.d * ld].reshape(s.d, ld))
    return specs, inst, host, dev


@pytest.fixture(scope="module")
def batch():
    return make_batch(40, 777, restarts=8)



def test_instances_in_separate_allocations(km, batch):
    """The same instances with their points in separate device allocations (and
    an unaligned copy) as in one flat tensor: identical results, labels
    included (the descriptors carry every pointer as given)."""
    specs, inst, host, _ = batch
    sub = inst[:6]
    base = km.fit_batched(sub, tol=1e-6, max_iter=300)
    sep = []
    for q, (X, N, ini) in enumerate(sub):
        if q == 2:      # rows off 16-byte alignment, odd ld
            big = torch.zeros((X.shape[0], N + 2), dtype=torch.float32, device="cuda")
            big[:, 1:N + 1] = X[:, :N]
            sep.append((big[:, 1:], N, ini))
        else:
            sep.append((X.clone(), N, ini))
    out = km.fit_batched(sep, tol=1e-6, max_iter=300)
    for a, b in zip(base, out):
        assert np.array_equal(a["centroids"], b["centroids"]) and a["iters"] == b["iters"]
        assert np.array_equal(a["restart_objective"], b["restart_objective"])
        assert a["best_restart"] == b["best_restart"] and a["E"] == b["E"]
        assert np.array_equal(a["labels"].cpu().numpy(), b["labels"].cpu().numpy())

def test_every_restart_equals_a_single_fit(km, batch):
    specs, inst, host, _ = batch
    out = km.fit_batched(inst, tol=1e-6, max_iter=300)
    n_restarts = 0
    for s, (X, N, ini), r in zip(specs, inst, out):
        singles = [km.fit(X, ini[q], tol=1e-6, max_iter=300, N=N) for q in range(len(ini))]
        n_restarts += len(ini)
        J = np.array([f.objective for f in singles])
        assert np.allclose(r["restart_objective"], J, rtol=1e-12, atol=0), s.name
        assert r["restart_iters"].tolist() == [f.iters for f in singles]
        b = r["best_restart"]
        assert b == int(np.argmin(r["restart_objective"]))
        f = singles[b]
        assert np.array_equal(r["centroids"], f.centroids), s.name
        assert r["iters"] == f.iters and r["E"] == f.E and r["converged"] == f.converged
        assert r["empty_events"] == f.empty_events
        assert np.array_equal(r["labels"].cpu().numpy(), f.labels.cpu().numpy())
    log(f"{len(specs)} instances, {n_restarts} restarts: identical to single fits")


def test_kept_restart_matches_the_oracle(km, batch):
    specs, inst, host, _ = batch
    out = km.fit_batched(inst, tol=1e-6, max_iter=300)
    for i in (0, 5, 11, 23, 39):
        s, (X, N, ini), r = specs[i], inst[i], out[i]
        ref = oracle.fit(host[i], ini[r["best_restart"]], tol=1e-6, max_iter=300, N=N)
        assert r["iters"] == ref["T"], s.name
        centre_check(r["centroids"], ref["mu"])
        e_check(r["E"], ref["E"])
        assert abs(r["objective"] - ref["J"]) <= 1e-6 * ref["J"]
        label_check(r["labels"].cpu().numpy(), host[i], r["centroids"], N=N)


def test_schedule_independence(km, batch):
    specs, inst, host, _ = batch
    runs = []
    for sch in [(1, 1, 0.0), (4, 2, 1.0), (16, 1, 1e6), (8, 2, 0.0)]:
        km.set_batched_schedule(*sch)
        runs.append((sch, km.fit_batched(inst, tol=1e-6, max_iter=300)))
    km.set_batched_schedule(0, 0, 0.0)
    base = runs[0][1]
    for sch, out in runs[1:]:
        for a, b in zip(base, out):
            assert np.array_equal(a["centroids"], b["centroids"]), sch
            assert a["iters"] == b["iters"] and a["E"] == b["E"], sch
            assert a["best_restart"] == b["best_restart"], sch
            assert np.allclose(a["restart_objective"], b["restart_objective"], rtol=1e-12, atol=0)
            assert np.array_equal(a["labels"].cpu().numpy(), b["labels"].cpu().numpy())


@pytest.mark.parametrize("group", [4, 3, 2, 1])
def test_restart_groups_give_the_same_results(km, batch, group):
    """Restart fusion (km_schedule.restart_group): an instance's restarts run
    as work items of at most `group` restarts, the kept restart chosen across
    them and its labels copied from a later item when it ran there.  Every
    output equals the one-item run's, on a batch of 1 to 8 restarts per
    instance, with and without teams."""
    specs, inst, host, _ = batch
    for team in (8, 1):
        # The objective's float64 summation order follows the team layout, so
        # each grouping is compared with the one-item run on the same teams.
        km.set_batched_schedule(team, 2, 0.0, 0)
        base = km.fit_batched(inst, tol=1e-6, max_iter=300)
        sch = (team, 2, 0.0, group)
        km.set_batched_schedule(*sch)
        out = km.fit_batched(inst, tol=1e-6, max_iter=300)
        for s, a, b in zip(specs, base, out):
            assert a["best_restart"] == b["best_restart"], (sch, s.name)
            assert np.array_equal(a["centroids"], b["centroids"]), sch
            assert a["iters"] == b["iters"] and a["E"] == b["E"], sch
            assert a["objective"] == b["objective"], sch
            assert np.array_equal(a["restart_objective"], b["restart_objective"]), sch
            assert np.array_equal(a["restart_iters"], b["restart_iters"]), sch
            assert np.array_equal(a["labels"].cpu().numpy(), b["labels"].cpu().numpy()), sch
    km.set_batched_schedule(0, 0, 0.0, 0)


@pytest.mark.parametrize("team", [8, 1])
def test_matrix_core_pass_gives_the_same_results(km, batch, team):
    """km_schedule.mfma_min_k: the update pass with matrix-core keys for the
    3-D instances (all restarts' centres as rows of 32-row tiles, 8 / 16 / 32
    rows per restart by K) against the VALU pass, on the same team layout:
    every output is identical, the objectives included."""
    specs, inst, host, _ = batch
    km.set_batched_schedule(team, 2, 0.0, 0, 33)  # VALU keys only
    base = km.fit_batched(inst, tol=1e-6, max_iter=300)
    km.set_batched_schedule(team, 2, 0.0, 0, 1)   # matrix-core keys for every K
    out = km.fit_batched(inst, tol=1e-6, max_iter=300)
    km.set_batched_schedule(0, 0, 0.0, 0, 0)
    ks = sorted({s.K for s in specs if s.d == 3})
    assert ks[0] <= 8 and ks[-1] > 16, ks          # all three row widths are exercised
    for s, a, b in zip(specs, base, out):
        assert a["best_restart"] == b["best_restart"], s.name
        assert np.array_equal(a["centroids"], b["centroids"]), s.name
        assert a["iters"] == b["iters"] and a["E"] == b["E"], s.name
        assert np.array_equal(a["restart_objective"], b["restart_objective"]), s.name
        assert np.array_equal(a["restart_iters"], b["restart_iters"]), s.name
        assert np.array_equal(a["labels"].cpu().numpy(), b["labels"].cpu().numpy()), s.name


def test_matrix_core_pass_unaligned_rows(km):
    """The matrix-core pass on rows that are not 16-byte aligned (offset by
    one float, odd row stride) and N not a multiple of 64: the guarded
    32-bit loads of every unit.  Identical to the VALU pass; the kept
    restart of one instance matches the oracle."""
    import dataclasses
    specs = [s for s in datagen.batched_specs(40, seed=4242, n_range=(3.0, 4.3)) if s.d == 3][:6]
    specs = [dataclasses.replace(s, K=min(k, s.N)) for s, k in zip(specs, (5, 12, 20, 32, 9, 27))]
    flat, offs, inits = datagen.batched_generate(specs)
    inst, host = [], []
    for s, off, ini in zip(specs, offs, inits):
        ld = s.N + 1                                  # odd stride
        buf = torch.zeros(1 + s.d * ld, dtype=torch.float32, device="cuda")
        Xh = flat[off:off + s.d * datagen.round_up(s.N, 4)].reshape(s.d, -1)[:, :s.N]
        view = buf[1:].view(s.d, ld)                  # offset by one float
        view[:, :s.N] = torch.from_numpy(np.ascontiguousarray(Xh)).cuda()
        inst.append((view, s.N, ini))
        host.append(np.ascontiguousarray(Xh))
    assert any(s.N % 64 for s in specs)
    km.set_batched_schedule(1, 2, 0.0, 0, 33)
    base = km.fit_batched(inst, tol=1e-6, max_iter=300)
    km.set_batched_schedule(1, 2, 0.0, 0, 1)
    out = km.fit_batched(inst, tol=1e-6, max_iter=300)
    km.set_batched_schedule(0, 0, 0.0, 0, 0)
    for s, a, b in zip(specs, base, out):
        assert a["best_restart"] == b["best_restart"], s.name
        assert np.array_equal(a["centroids"], b["centroids"]), s.name
        assert a["iters"] == b["iters"] and a["E"] == b["E"], s.name
        assert np.array_equal(a["restart_objective"], b["restart_objective"]), s.name
        assert np.array_equal(a["labels"].cpu().numpy(), b["labels"].cpu().numpy()), s.name
    s, (X, N, ini), r = specs[3], inst[3], out[3]
    ref = oracle.fit(host[3], ini[r["best_restart"]], tol=1e-6, max_iter=300)
    assert r["iters"] == ref["T"], s.name
    centre_check(r["centroids"], ref["mu"])
    label_check(r["labels"].cpu().numpy(), host[3], r["centroids"])


def test_batched_errors(km, batch):
    from paper_2405_12052_amd import KM_EINVAL, KM_EUNSUPPORTED, KMeansError
    specs, inst, host, dev = batch
    X, N, ini = inst[0]
    bad_k = np.zeros((1, 33, X.shape[0]))
    with pytest.raises(KMeansError) as e:
        km.fit_batched([(X, N, bad_k)])
    assert e.value.code == KM_EUNSUPPORTED
    with pytest.raises(KMeansError) as e:
        km.fit_batched([(X, N, np.concatenate([ini] * 2)[:9] if len(ini) >= 5 else np.zeros((9, 2, X.shape[0])))])
    assert e.value.code in (KM_EUNSUPPORTED, KM_EINVAL)
    Xn = X.clone()
    Xn[0, 3] = float("nan")
    with pytest.raises(KMeansError, match="NaN") as e:
        km.fit_batched([inst[1], (Xn, N, ini)])
    assert e.value.code == KM_EINVAL
    for bad in ({"mfma_min_k": 34}, {"mfma_min_k": -1}, {"restart_group": 9}):
        with pytest.raises(KMeansError) as e:
            km.set_batched_schedule(8, 2, 0.0, **bad)
        assert e.value.code == KM_EINVAL
    out = km.fit_batched(inst[:3])          # the context still works
    assert len(out) == 3


def test_tuner_and_cache(km, tmp_path):
    specs, inst, host, _ = make_batch(24, 999, n_range=(3.0, 5.5), restarts=4)
    cache = str(tmp_path / "tune.json")
    best = km.tune_batched(inst, tol=1e-6, max_iter=300, cache_path=cache)
    log(f"tuned schedule {best}")
    lines = open(cache).read().strip().splitlines()
    assert len(lines) == 1 and json.loads(lines[0])["team_size"] == best["team_size"]
    assert json.loads(lines[0])["restart_group"] == best["restart_group"]
    assert json.loads(lines[0])["mfma_min_k"] == best["mfma_min_k"]
    again = km.tune_batched(inst, tol=1e-6, max_iter=300, cache_path=cache)
    assert again == best and len(open(cache).read().strip().splitlines()) == 1
    assert km.batched_schedule() == best
    km.set_batched_schedule(0, 0, 0.0)


def test_bench_size_slice_on_teams(km):
    """The largest instances of the 4096-instance batch the benchmark times
    (N close to 1e6, 8 restarts each), run as teams of 8 blocks as the tuned
    schedule runs them: every restart's T and objective equal a single fit
    from the same start, and the kept restart equals the float64 oracle (T,
    centres, E, objective, labels at its final centres)."""
    specs = datagen.batched_specs(4096)
    big = sorted(range(len(specs)), key=lambda i: -specs[i].N)[:6]
    sub = [specs[i] for i in big]
    log("bench-size slice: " + ", ".join(f"{s.name} N={s.N} d={s.d} K={s.K}" for s in sub))
    flat, offs, inits = datagen.batched_generate(sub)
    dev = torch.from_numpy(flat).cuda()
    inst, host = [], []
    for s, off, ini in zip(sub, offs, inits):
        ld = datagen.round_up(s.N, 4)
        inst.append((dev[off:off + s.d * ld].view(s.d, ld), s.N, ini))
        host.append(flat[off:off + s.d * ld].reshape(s.d, ld))
    km.set_batched_schedule(8, 2, 0.0)
    try:
        out = km.fit_batched(inst, tol=1e-6, max_iter=300)
    finally:
        km.set_batched_schedule(0, 0, 0.0)
    for s, (X, N, ini), r, h in zip(sub, inst, out, host):
        singles = [km.fit(X, ini[q], tol=1e-6, max_iter=300, N=N, labels=False)
                   for q in range(len(ini))]
        assert r["restart_iters"].tolist() == [f.iters for f in singles], s.name
        assert np.allclose(r["restart_objective"], [f.objective for f in singles],
                           rtol=1e-12, atol=0), s.name
        b = r["best_restart"]
        ref = oracle.fit(h, ini[b], tol=1e-6, max_iter=300, N=N)
        assert r["iters"] == ref["T"], s.name
        centre_check(r["centroids"], ref["mu"])
        e_check(r["E"], ref["E"])
        assert abs(r["objective"] - ref["J"]) <= 1e-6 * ref["J"], s.name
        label_check(r["labels"].cpu().numpy(), h, r["centroids"], N=N)
        log(f"  {s.name}: kept restart {b}, T={ref['T']}, oracle parity")
