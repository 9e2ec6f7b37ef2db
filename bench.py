"""Throughput benchmark of the q-LSKUM pseudo-time iteration on one MI355X.

Workload: O-type cloud of 1250 x 2000 = 2.5M points around NACA 0012
(cubic-Hermite O-grid, 5 x 5 lattice-box stencils, interior points jittered
by U(-0.1, 0.1) local spacings, splitmix64 seed 2108), Hilbert-reordered;
M 0.85, alpha 1 deg, Venkatakrishnan limiter K = 5, CFL 0.2, 3 inner
iterations, FP64.  A step is one pseudo-time iteration (local time step,
four Runge-Kutta stages of q-derivatives + flux residual + update, residual
norm).  The state is resident in HBM before the timed region starts.

Prints one JSON line (see the repository's measurement notes for the
roofline and CPU-baseline definitions).
"""
import argparse
import functools
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Workloads: the 2.5M-point cloud the headline number is quoted on, and the
# 40M-point cloud of the same generator (5000 x 8000; interior points
# jittered like the 2.5M cloud, whose unjittered trailing-edge stencils
# cannot be repaired at these resolutions).
WORKLOADS = {
    "naca2.5m": dict(ns=1250, nr=2000,
                     metric="Mpoint-iter/s at 2.5M pts, FP64 vs mixed; time to 1e-6 residual, "
                            "warm vs cold"),
    "naca40m": dict(ns=5000, nr=8000, metric="Mpoint-iter/s at 40M pts, FP64 vs mixed"),
}
FLOW = dict(mach=0.85, alpha_deg=1.0, limiter=1, venkat_k=5.0, cfl=0.2, n_inner=3)
FP64_VALU_PEAK_TFLOPS = 78.6  # MI355X FP64 vector peak
PREC_NAME = {0: "fp64", 1: "mixed"}

# Algorithmic FP64 operations of one flux-residual launch (one RK stage),
# the roofline's unit: 940 per neighbour entry and point with the limiter,
# 690 without (software transcendentals at 20-30 operations each), times
# the cloud's mean neighbour count and its points.
FLOPS_PER_ENTRY_UNIT = {1: 940, 0: 690}
# An itemised count of the same launch, reported beside it: per neighbour
# entry that enters at least one split stencil, and per split stencil it
# enters; transcendentals and divides at fixed costs (exp 20, log 20,
# erfc 30, sqrt 10, divide 10).
FLOPS_ENTRY_COMMON = 202       # geometry, reconstruction, two q~ -> primitive states
FLOPS_ENTRY_LIMITER = 125      # Venkatakrishnan factors of 8 increments, eps^2
FLOPS_PER_STENCIL = 191        # two split fluxes, their difference, weighted sum


# HBM bytes of the flux kernel from committed rocprofv3 counters: the record
# line of this file holds FETCH_SIZE / WRITE_SIZE (KiB per launch), the
# calibration factors and the hash of the kernel sources it was taken with.
TRAFFIC_RECORD = {"naca2.5m": os.path.join(ROOT, "profiles", "pmc_hbm_bytes_c2_fp64.md"),
                  "naca40m": os.path.join(ROOT, "profiles", "pmc_hbm_bytes_c5_fp64.md")}
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2108_07031_amd", "csrc", f) for f in
                  ("qlskum_kernels.hip", "qlskum_internal.h", "qlskum_erfc.h",
                   "qlskum_erfc_coeffs.h")]


def kernel_sources_sha256():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def committed_traffic(workload):
    """Bytes per flux launch, or None when the record is missing or was
    taken with other kernel sources."""
    try:
        with open(TRAFFIC_RECORD[workload]) as fh:
            for line in fh:
                if line.startswith("record: "):
                    rec = json.loads(line[len("record: "):])
                    if rec.get("sources_sha256") != kernel_sources_sha256():
                        return None
                    return (rec["fetch_kib"] * 1024.0 * rec["fetch_scale"] +
                            rec["write_kib"] * 1024.0 * rec["write_scale"])
    except (OSError, ValueError, KeyError):
        return None
    return None


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def flux_flops_unit(n, nnz, limiter):
    """Algorithmic FP64 operations of one flux-residual launch in the
    roofline's unit: per point, FLOPS_PER_ENTRY_UNIT x the mean number of
    neighbour entries."""
    return int(round(FLOPS_PER_ENTRY_UNIT[1 if limiter else 0] * (nnz / n) * n))  # k_mean x n


def flux_flops_per_launch(flags, kind, ptr, limiter):
    """Itemised FP64 operations of one flux-residual launch, from the
    library's split-membership flags (walls drop their n+ stencil; outer
    points carry no residual)."""
    npt = kind.shape[0]
    owner = np.repeat(np.arange(npt), np.diff(ptr))
    f = flags.astype(np.int64)
    f = np.where(kind[owner] == 1, f & ~4, f)
    f = np.where(kind[owner] == 2, 0, f)
    used = f != 0
    stencils = ((f & 3) != 0).astype(np.int64) + ((f & 12) != 0).astype(np.int64)
    common = FLOPS_ENTRY_COMMON + (FLOPS_ENTRY_LIMITER if limiter else 0)
    return int(used.sum()) * common + int(stencils.sum()) * FLOPS_PER_STENCIL


def cpu_baseline(cloud, budget_s=30.0, max_iter=10):
    """The oracle as it stands on a bounded sample of the same workload.
    Main figure: the OpenMP build of the oracle (results bit for bit the
    serial build's) on every host thread it is given (OMP_NUM_THREADS),
    whole iterations of the full cloud from the freestream start -- one
    timed iteration, then as many more (up to max_iter in all) as fit the
    time budget.  Beside it, the serial build on one core: one stage
    evaluation of the full cloud (an iteration is four stages)."""
    import oracle
    omp = oracle.load(oracle.OMP_LIB)
    o = oracle.Oracle(cloud, oracle.params(**FLOW), lib=omp)
    U = o.freestream()
    t0 = time.perf_counter()
    U, _ = o.run(U, 1)
    t1 = time.perf_counter() - t0
    more = int(min(max_iter - 1, max(0.0, budget_s - t1) // t1))
    t = t1
    if more > 0:
        t0 = time.perf_counter()
        o.run(U, more)
        t += time.perf_counter() - t0
    iters = 1 + more
    threads = int(omp.ora_num_threads())
    s = oracle.Oracle(cloud, oracle.params(**FLOW))
    t0 = time.perf_counter()
    s.evaluate(s.freestream())
    ts = time.perf_counter() - t0
    return {"value": cloud.n * iters / t / 1e6, "unit": "Mpoint-iter/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{iters} iteration(s) of the full {cloud.n}-point cloud from the freestream "
                      f"({t:.1f} s) with the OpenMP build of the oracle on {threads} threads",
            "single_thread": {"value": cloud.n / (4.0 * ts) / 1e6, "unit": "Mpoint-iter/s",
                              "cores": 1,
                              "sample": f"one stage evaluation of the full cloud ({ts:.1f} s); "
                                        f"iteration = 4 stages"}}


# Learned warm start (time to a 1e-6 residual drop, warm vs cold) on small
# clouds: training conditions converged in one batched run, a network
# 6 -> 4 x 128 (tanh) -> 4 trained on their converged primitive fields, then
# held-out conditions solved cold and warm, one at a time.
WARM = dict(ns=64, nr=24, n_train=48, n_test=8, seed_train=1, seed_test=2, drop=1e-6,
            max_iter=40000, widths=[6, 128, 128, 128, 128, 4], steps=8000, batch=8192,
            lr=2e-3, floor=0.05)


# Batched form: 64 independent clouds of log-uniform sizes in [40k, 640k]
# points, each with its own flow condition, advanced by the same launches
# (one captured iteration replayed) in mixed precision with the limiter,
# against the same clouds run one after the other.
BATCH = dict(n_case=64, n_lo=40000, n_hi=640000, seed=7031, iters=200, precision=1)


def batch_study():
    import torch
    from paper_2108_07031_amd import qlskum as ql
    B = BATCH
    conds, clouds = _batch_clouds(1)
    total = sum(cl.n for cl in clouds)
    prm = dict(limiter=1, precision=B["precision"])
    log(f"  {B['n_case']} clouds, {total} points")
    s = ql.Solver(**prm)
    s.upload_batch(clouds, [c["mach"] for c in conds], [c["alpha"] for c in conds])
    s.init_freestream()
    s.batch_run(1e-300, 5, check_every=5)  # warm-up and graph capture
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.batch_run(1e-300, B["iters"], check_every=B["iters"])
    t_batch = time.perf_counter() - t0
    s.close()
    t_solo = 0.0
    for cl, c in zip(clouds, conds):
        so = ql.Solver(cl, mach=c["mach"], alpha_deg=c["alpha"], **prm)
        so.init_freestream()
        so.step(5, want_history=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        so.step(B["iters"], want_history=False)
        torch.cuda.synchronize()
        t_solo += time.perf_counter() - t0
        so.close()
    return {"cases": B["n_case"], "points_total": total, "precision": PREC_NAME[B["precision"]],
            "points_min_max": [min(cl.n for cl in clouds), max(cl.n for cl in clouds)],
            "iterations": B["iters"],
            "batched_mpt_it_s": total * B["iters"] / t_batch / 1e6,
            "sequential_mpt_it_s": total * B["iters"] / t_solo / 1e6,
            "speedup": t_solo / t_batch}


def _batch_clouds(scale):
    """The batched study's 64 conditions and clouds, sizes divided by scale."""
    from cloudgen import naca_ocloud, sample_conditions, uniform01
    B = BATCH
    u = uniform01(B["seed"], B["n_case"])
    lo, hi = B["n_lo"] / scale, B["n_hi"] / scale
    sizes = np.exp(np.log(lo) + u * (np.log(hi) - np.log(lo)))
    conds = sample_conditions(B["seed"] + 1, B["n_case"], mach=(0.3, 0.85))
    clouds = []
    for k, (nn, c) in enumerate(zip(sizes, conds)):
        ns = 2 * int(round(np.sqrt(5.0 * nn / 8.0) / 2))  # Ns:Nr = 5:8, Ns even
        clouds.append(naca_ocloud(ns, int(round(nn / ns)), tau=c["tau"], jitter=0.1,
                                  seed=B["seed"] + 10 + k))
    return conds, clouds


def _progress_logger(tag, every=10000):
    """A progress callback for batched runs (called by the library after each
    check window): logs when the number of active cases changes, and every
    `every` iterations, with the seconds since start() was called."""
    state = {"active": None, "t0": time.perf_counter()}

    def fn(it, active):
        if active != state["active"] or it % every == 0:
            log(f"    {tag}: iteration {it}, {active} cases active "
                f"({time.perf_counter() - state['t0']:.1f} s)")
            state["active"] = active

    def start():
        state["t0"] = time.perf_counter()
    fn.start = start
    return fn


def batch_drop_study(scale, max_iter, check_every=500, switch=3e-5, sequential=True):
    """The batched form run to each case's 1e-6 drop of its first residual:
    mixed precision with the precision switch, one batch (captured iteration
    replayed, per-case retirement on the device) against the same cases run
    one after the other the same way; clouds scale x smaller than the
    throughput study's."""
    import torch
    from paper_2108_07031_amd import qlskum as ql
    conds, clouds = _batch_clouds(scale)
    total = sum(cl.n for cl in clouds)
    prm = dict(limiter=1, precision=1, mixed_switch=switch)
    log(f"  to the drop: {len(clouds)} clouds, {total} points")
    s = ql.Solver(**prm)
    s.upload_batch(clouds, [c["mach"] for c in conds], [c["alpha"] for c in conds])
    s.init_freestream()
    progress = _progress_logger("batch")
    s.set_progress(progress)
    torch.cuda.synchronize()
    progress.start()
    t0 = time.perf_counter()
    iters, _ = s.batch_run(1e-6, max_iter, check_every=check_every)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    sw = s.batch_switched()
    status = s.batch_status()
    s.close()
    log(f"  batched: {t_batch:.1f} s, iterations {int(iters.min())}..{int(iters.max())}")
    t_solo, iters_solo = 0.0, []
    for k, (cl, c) in enumerate(zip(clouds, conds) if sequential else ()):
        so = ql.Solver(cl, mach=c["mach"], alpha_deg=c["alpha"], **prm)
        so.init_freestream()
        so.set_progress(_progress_logger(f"case {k}", every=20000))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        it, _ = so.batch_run(1e-6, max_iter, check_every=check_every)
        torch.cuda.synchronize()
        t_solo += time.perf_counter() - t0
        iters_solo.append(int(it[0]))
        so.close()
        if k % 8 == 7:
            log(f"  one after the other: {k + 1} cases, {t_solo:.1f} s")
    work = float(sum(cl.n * int(i) for cl, i in zip(clouds, iters)))
    return {"cases": len(clouds), "points_total": total, "scale": scale,
            "points_min_max": [min(cl.n for cl in clouds), max(cl.n for cl in clouds)],
            "precision": f"mixed, switch to FP64 fluxes at {switch:g} of the first residual",
            "drop": 1e-6, "max_iter": max_iter,
            "reached": int(sum(1 for st, i in zip(status, iters)
                               if st == ql.QL_OK and i < max_iter)),
            "iterations": [int(i) for i in iters], "iterations_solo": iters_solo,
            "switched_after": [int(i) for i in sw],
            "wall_batched_s": t_batch, "wall_sequential_s": t_solo if sequential else None,
            "batched_mpt_it_s": work / t_batch / 1e6,
            "sequential_mpt_it_s": work / t_solo / 1e6 if sequential else None,
            "speedup": t_solo / t_batch if sequential else None}


def _prims(U, gamma=1.4):
    rho = U[0]
    u, v = U[1] / rho, U[2] / rho
    return np.stack([rho, u, v, (gamma - 1.0) * (U[3] - 0.5 * rho * (u * u + v * v))], axis=1)


def warm_study():
    import torch
    from cloudgen import (glorot_weights, naca_ocloud, sample_conditions, uniform01,
                          warm_features)
    from paper_2108_07031_amd import qlskum as ql
    W = WARM
    t_all = time.perf_counter()
    train = sample_conditions(W["seed_train"], W["n_train"])
    test = sample_conditions(W["seed_test"], W["n_test"])
    cloud_of = lambda c: naca_ocloud(W["ns"], W["nr"], tau=c["tau"])
    clouds = [cloud_of(c) for c in train]
    # 1. converge the training conditions together
    s = ql.Solver(limiter=1)
    offs = s.upload_batch(clouds, [c["mach"] for c in train], [c["alpha"] for c in train])
    s.init_freestream()
    t0 = time.perf_counter()
    it_train, _ = s.batch_run(W["drop"], W["max_iter"], check_every=500)
    t_conv = time.perf_counter() - t0
    # train on the cases that reached the drop (a failed case is retired
    # with its status and keeps an unusable state)
    ok_case = (s.batch_status() == ql.QL_OK) & (np.asarray(it_train) < W["max_iter"])
    U = s.fetch_state()
    d = s.wall_distance()
    s.close()
    F = np.concatenate([warm_features(cl, d[offs[i]:offs[i + 1]], c["mach"], c["alpha"],
                                      c["tau"]) for i, (cl, c) in enumerate(zip(clouds, train))])
    keep = (np.concatenate([cl.kind for cl in clouds]) != 2) & np.repeat(
        ok_case, [cl.n for cl in clouds])
    F, P = F[keep], _prims(U)[keep]
    fm, fs = F.mean(axis=0), F.std(axis=0) + 1e-12
    pm, ps = P.mean(axis=0), P.std(axis=0) + 1e-12
    X = torch.tensor((F - fm) / fs, dtype=torch.float32, device="cuda")
    Y = torch.tensor((P - pm) / ps, dtype=torch.float32, device="cuda")
    # 2. train (minibatches from a seeded shuffle of the samples)
    m = ql.Mlp(W["widths"], max_batch=W["batch"])
    m.set_weights(glorot_weights(W["widths"], 2108))
    nb = X.shape[0] // W["batch"]
    order = torch.tensor(np.argsort(uniform01(31, X.shape[0] * 64).reshape(64, -1), axis=1),
                         device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loss = None
    for step in range(W["steps"]):
        ep, b = divmod(step, max(nb, 1))
        idx = order[ep % 64, b * W["batch"]:(b + 1) * W["batch"]]
        lr = W["lr"] * (0.1 if step >= 0.75 * W["steps"] else 1.0)
        loss = m.train_step(X[idx].contiguous(), Y[idx].contiguous(), lr,
                            want_loss=(step == W["steps"] - 1))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    # 3. held-out conditions, cold and warm
    rows = []
    for c in test:
        cl = cloud_of(c)
        prm = dict(limiter=1, mach=c["mach"], alpha_deg=c["alpha"])
        sc = ql.Solver(cl, **prm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sc.init_freestream()
        ic, rc_last = sc.batch_run(W["drop"], W["max_iter"], check_every=100)
        if sc.batch_status()[0] != ql.QL_OK:
            raise RuntimeError(f"cold run failed at M {c['mach']:.3f}, alpha {c['alpha']:.2f}")
        t_cold = time.perf_counter() - t0
        dw = sc.wall_distance()
        sc.close()
        sw = ql.Solver(cl, **prm)
        Xc = torch.tensor((warm_features(cl, dw, c["mach"], c["alpha"], c["tau"]) - fm) / fs,
                          dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rcold, rwarm, used = sw.warm_start(m, Xc, np.concatenate([pm, ps]), W["floor"])
        iw, _ = sw.batch_run(W["drop"], W["max_iter"], check_every=100, ref=rcold[:, 0])
        if sw.batch_status()[0] != ql.QL_OK:
            raise RuntimeError(f"warm run failed at M {c['mach']:.3f}, alpha {c['alpha']:.2f}")
        t_warm = time.perf_counter() - t0
        sw.close()
        rows.append(dict(iters_cold=int(ic[0]), iters_warm=int(iw[0]), t_cold=t_cold,
                         t_warm=t_warm, used=bool(used[0]),
                         r1_ratio=float(rwarm[0, 0] / rcold[0, 0])))
        log(f"warm study: M {c['mach']:.3f} alpha {c['alpha']:.2f} tau {c['tau']:.3f}: "
            f"cold {ic[0]} its {t_cold:.2f} s, warm {iw[0]} its {t_warm:.2f} s, "
            f"R1 warm/cold {rows[-1]['r1_ratio']:.3f}, used {bool(used[0])}")
    m.close()
    ratio = [r["t_warm"] / r["t_cold"] for r in rows]
    return {
        "cases_train": W["n_train"], "cases_test": W["n_test"],
        "points_per_case": W["ns"] * W["nr"],
        "drop": W["drop"], "max_iter": W["max_iter"],
        "train_converged": int(np.sum(ok_case)),
        "train_solve_s": t_conv, "train_net_s": t_train, "train_loss": loss,
        "network": "6-128x4-4 tanh, bf16 MFMA, FP32 accumulate, Adam",
        "iters_cold": [r["iters_cold"] for r in rows],
        "iters_warm": [r["iters_warm"] for r in rows],
        "time_ratio_median": float(np.median(ratio)),
        "iters_ratio_median": float(np.median([r["iters_warm"] / r["iters_cold"]
                                                for r in rows])),
        "fallbacks": int(sum(not r["used"] for r in rows)),
        "r1_warm_over_cold": [r["r1_ratio"] for r in rows],
        "study_s": time.perf_counter() - t_all,
    }


# A larger warm-start study: the C3 sampler's Mach range, 128 training
# conditions on 10k-point clouds and 16 held-out ones on 40k-point clouds,
# every solve a batch in mixed precision with the precision switch.
WARM_LARGE = dict(ns=80, nr=128, ns_test=160, nr_test=256, n_train=128, n_test=16, seed_train=1,
                  seed_test=2, mach=(0.3, 0.85), drop=1e-6, max_iter=150000,
                  widths=[6, 128, 128, 128, 128, 4], steps=8000, batch=8192, lr=2e-3, floor=0.05,
                  switch=3e-5)


def _features(clouds, conds, d, offs):
    from cloudgen import warm_features
    return np.concatenate([warm_features(cl, d[offs[i]:offs[i + 1]], c["mach"], c["alpha"],
                                         c["tau"]) for i, (cl, c) in enumerate(zip(clouds, conds))])


def warm_study_large():
    """Training data from one batched solve; the held-out cases solved cold
    as one batch and warm (inference, per-case fallback, then the run) as
    another, with the same reference (the freestream's first residual); a
    held-out case counts when its cold run reaches the drop."""
    import torch
    from cloudgen import glorot_weights, naca_ocloud, sample_conditions, uniform01
    from paper_2108_07031_amd import qlskum as ql
    W = WARM_LARGE
    t_all = time.perf_counter()
    prm = dict(limiter=1, precision=1, mixed_switch=W["switch"])
    train = sample_conditions(W["seed_train"], W["n_train"], mach=W["mach"])
    test = sample_conditions(W["seed_test"], W["n_test"], mach=W["mach"])
    # jittered like the throughput clouds (the unjittered generator cannot
    # repair every trailing-edge stencil at these resolutions)
    clouds = [naca_ocloud(W["ns"], W["nr"], tau=c["tau"], jitter=0.1, seed=100 + k)
              for k, c in enumerate(train)]
    tclouds = [naca_ocloud(W["ns_test"], W["nr_test"], tau=c["tau"], jitter=0.1, seed=1000 + k)
               for k, c in enumerate(test)]

    progress = functools.partial(_progress_logger, every=20000)
    s = ql.Solver(**prm)
    offs = s.upload_batch(clouds, [c["mach"] for c in train], [c["alpha"] for c in train])
    s.set_progress(progress("training solve"))
    s.init_freestream()
    t0 = time.perf_counter()
    it_train, _ = s.batch_run(W["drop"], W["max_iter"], check_every=500)
    t_conv = time.perf_counter() - t0
    ok_case = (s.batch_status() == ql.QL_OK) & (np.asarray(it_train) < W["max_iter"])
    U = s.fetch_state()
    d = s.wall_distance()
    s.close()
    F = _features(clouds, train, d, offs)
    keep = (np.concatenate([cl.kind for cl in clouds]) != 2) & np.repeat(
        ok_case, [cl.n for cl in clouds])
    F, P = F[keep], _prims(U)[keep]
    fm, fs = F.mean(axis=0), F.std(axis=0) + 1e-12
    pm, ps = P.mean(axis=0), P.std(axis=0) + 1e-12
    X = torch.tensor((F - fm) / fs, dtype=torch.float32, device="cuda")
    Y = torch.tensor((P - pm) / ps, dtype=torch.float32, device="cuda")
    log(f"  training net on {X.shape[0]} samples from {int(ok_case.sum())} converged cases")
    m = ql.Mlp(W["widths"], max_batch=W["batch"])
    m.set_weights(glorot_weights(W["widths"], 2108))
    nb = X.shape[0] // W["batch"]
    order = torch.tensor(np.argsort(uniform01(31, X.shape[0] * 8).reshape(8, -1), axis=1),
                         device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loss = None
    for step in range(W["steps"]):
        ep, b = divmod(step, max(nb, 1))
        idx = order[ep % 8, b * W["batch"]:(b + 1) * W["batch"]]
        lr = W["lr"] * (0.1 if step >= 0.75 * W["steps"] else 1.0)
        loss = m.train_step(X[idx].contiguous(), Y[idx].contiguous(), lr,
                            want_loss=(step == W["steps"] - 1))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    del X, Y
    mach, alpha = [c["mach"] for c in test], [c["alpha"] for c in test]
    sc = ql.Solver(**prm)
    toffs = sc.upload_batch(tclouds, mach, alpha)
    sc.set_progress(progress("held-out cold"))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sc.init_freestream()
    ic, _ = sc.batch_run(W["drop"], W["max_iter"], check_every=500)
    t_cold = time.perf_counter() - t0
    st_cold = sc.batch_status()
    dw = sc.wall_distance()
    sc.close()
    sw = ql.Solver(**prm)
    sw.upload_batch(tclouds, mach, alpha)
    sw.set_progress(progress("held-out warm"))
    Xc = torch.tensor((_features(tclouds, test, dw, toffs) - fm) / fs, dtype=torch.float32,
                      device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rcold, rwarm, used = sw.warm_start(m, Xc, np.concatenate([pm, ps]), W["floor"])
    iw, _ = sw.batch_run(W["drop"], W["max_iter"], check_every=500, ref=rcold[:, 0])
    t_warm = time.perf_counter() - t0
    st_warm = sw.batch_status()
    sw.close()
    m.close()
    ok = [(st_cold[k] == ql.QL_OK and ic[k] < W["max_iter"]) for k in range(W["n_test"])]
    ratios = [iw[k] / ic[k] for k in range(W["n_test"]) if ok[k]]
    return {
        "cases_train": W["n_train"], "points_per_train_case": clouds[0].n,
        "cases_test": W["n_test"], "points_per_test_case": tclouds[0].n,
        "mach_range": list(W["mach"]), "drop": W["drop"], "max_iter": W["max_iter"],
        "precision": f"mixed, switch to FP64 fluxes at {W['switch']:g} of the first residual",
        "train_converged": int(np.sum(ok_case)), "train_samples": int(keep.sum()),
        "train_solve_s": t_conv, "train_net_s": t_train, "train_loss": loss,
        "network": "6-128x4-4 tanh, bf16 MFMA, FP32 accumulate, Adam",
        "test_cold_reached": int(sum(ok)),
        "iters_cold": [int(i) for i in ic], "iters_warm": [int(i) for i in iw],
        "status_cold": [int(x) for x in st_cold], "status_warm": [int(x) for x in st_warm],
        "used": [bool(u) for u in used],
        "iters_ratio_median": float(np.median(ratios)) if ratios else None,
        "wall_cold_batch_s": t_cold, "wall_warm_batch_s": t_warm,
        "wall_ratio_batch": t_warm / t_cold,
        "r1_warm_over_cold": [float(a / b) for a, b in zip(rwarm[:, 0], rcold[:, 0])],
        "study_s": time.perf_counter() - t_all,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--flux-split", type=int, default=0, choices=(0, 1, 2),
                    help="FP64 flux sweep as one launch (0), s and n launches (1) or one "
                         "launch per split stencil (2): the kernel-splitting ablation")
    ap.add_argument("--accuracy-iters", type=int, default=1000, metavar="N",
                    help="continue both timed runs (untimed) to N iterations and compare "
                         "mixed with FP64 lift, drag and density (0: skip)")
    ap.add_argument("--no-warm-study", action="store_true")
    ap.add_argument("--warm-study-large", action="store_true",
                    help="also run the larger warm-start study (minutes of GPU time)")
    ap.add_argument("--batch-drop-study", type=float, default=0, metavar="SCALE",
                    help="also run the batched cases to each one's 1e-6 drop, on clouds SCALE "
                         "times smaller (0: off)")
    ap.add_argument("--batch-drop-max-iter", type=int, default=200000)
    ap.add_argument("--batch-drop-no-sequential", action="store_true",
                    help="skip the one-after-the-other comparison of that study")
    ap.add_argument("--no-fp64-data-mixed", action="store_true",
                    help="skip the mixed run whose q-derivative sweeps read FP64 data")
    ap.add_argument("--no-batch-study", action="store_true")
    ap.add_argument("--precision", choices=("both", "fp64", "mixed"), default="both")
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="naca2.5m",
                    help="naca40m runs the throughput runs only (no studies, no CPU baseline)")
    ap.add_argument("--reorder", choices=("hilbert", "rcm", "none"), default="hilbert",
                    help="point order the library works in (results are the same bit for bit)")
    ap.add_argument("--cloud-cache", default="", metavar="NPZ",
                    help="keep the generated cloud in this file and reuse it when present")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run one plain device copy of MIB MiB (reference kernel for "
                         "hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU sharding is a design note, not a built path.", file=sys.stderr)
        sys.exit(2)

    import torch
    from cloudgen import naca_ocloud_cached
    from paper_2108_07031_amd import qlskum as ql

    wl = WORKLOADS[args.workload]
    reorder = {"none": 0, "hilbert": 1, "rcm": 2}[args.reorder]
    order_name = {"none": "caller order", "hilbert": "Hilbert order", "rcm": "RCM order"}[args.reorder]
    headline = args.workload == "naca2.5m"
    if not headline:
        args.accuracy_iters = 0  # the 40M runs report throughput only
    t0 = time.perf_counter()
    cloud = naca_ocloud_cached(args.cloud_cache, wl["ns"], wl["nr"], jitter=0.1, seed=2108,
                               progress=lambda m: log(f"  [{time.perf_counter() - t0:6.1f} s] {m}"))
    log(f"cloud {cloud.n} points, {cloud.nnz} entries ({time.perf_counter() - t0:.1f} s)")

    torch.cuda.init()
    stream = torch.cuda.Stream()  # default priority
    torch.cuda.set_stream(stream)

    def timed_run(precision, mixed_grad=0):
        t_up = time.perf_counter()
        split = dict(flux_split=args.flux_split) if precision == 0 else dict(mixed_grad=mixed_grad)
        s = ql.Solver(cloud, stream=stream, precision=precision, reorder=reorder, **split, **FLOW)
        label = PREC_NAME[precision] + (", FP64-data q-derivatives" if mixed_grad else "")
        log(f"[{label}] upload {time.perf_counter() - t_up:.1f} s")
        flags = s.flags()
        s.init_freestream()
        log(f"[{label}] warmup {args.warmup}")
        s.step(args.warmup, want_history=False)
        ql.ql_set_timing(s.h, 1)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        log(f"[{label}] timed: {args.steps} iterations")
        wall0 = time.perf_counter()
        ev0.record(stream)
        hist = s.step(args.steps)
        ev1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - wall0
        gpu_ms = ev0.elapsed_time(ev1)
        ktime = {k: ql.ql_kernel_time(s.h, k) for k in range(4)}
        ql.ql_set_timing(s.h, 0)
        log(f"[{label}] wall {wall:.3f} s, events {gpu_ms / 1e3:.3f} s, "
            f"residual {hist[0, 0]:.3e} -> {hist[-1, 0]:.3e}")
        for k, name in enumerate(("grad0", "gradk", "flux", "resnorm")):
            ms, cnt = ktime[k]
            log(f"  {name}: {cnt} launches, avg {ms / max(cnt, 1) * 1e3:.1f} us, "
                f"share {ms / gpu_ms * 100:.1f}%")
        cl, cd = s.forces()
        acc = None
        more = args.accuracy_iters - args.warmup - args.steps
        if args.accuracy_iters > 0 and args.precision == "both":
            # the same run continued (untimed) to a fixed iteration count, for
            # the FP64 vs mixed comparison of lift, drag and density
            if more > 0:
                log(f"[{label}] continued to {args.accuracy_iters} iterations")
                s.step(more, want_history=False)
            acc = dict(iterations=max(args.accuracy_iters, args.warmup + args.steps),
                       cl_cd=s.forces(), rho=s.fetch_state()[0].copy())
        s.close()
        elapsed = max(wall, gpu_ms / 1e3)
        return dict(flags=flags, elapsed=elapsed, ktime=ktime, hist=hist, cl=cl, cd=cd, acc=acc,
                    value=cloud.n * args.steps / elapsed / 1e6)

    if args.copy_calibration > 0:
        nel = args.copy_calibration * (1 << 20) // 8
        src = torch.ones(nel, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {args.copy_calibration} MiB read + written")
        del src, dst

    runs = {p: timed_run(p) for p in ((0, 1) if args.precision == "both" else
                                      (0,) if args.precision == "fp64" else (1,))}
    if args.precision == "both" and not args.no_fp64_data_mixed:
        # the mixed path with FP64-data q-derivative sweeps, for comparison
        runs["mixed_grad1"] = timed_run(1, mixed_grad=1)
    head = runs[0] if 0 in runs else runs[1]
    flops = flux_flops_unit(cloud.n, cloud.nnz, FLOW["limiter"])
    flops_item = flux_flops_per_launch(head["flags"], cloud.kind, cloud.nbr_ptr, FLOW["limiter"])
    flux_ms, flux_cnt = head["ktime"][2]
    flux_avg_s = flux_ms / max(flux_cnt, 1) / 1e3
    achieved = flops / flux_avg_s / 1e12
    out = {
        "metric": wl["metric"],
        "value": head["value"],
        "unit": "Mpoint-iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["elapsed"] * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if 0 in runs else "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": f"q-LSKUM, NACA 0012 O-cloud {wl['ns']}x{wl['nr']} "
                        f"({cloud.n / 1e6:g}M pts), jitter 0.1 seed 2108, {order_name}, M 0.85, "
                        "alpha 1, Venkatakrishnan K 5, CFL 0.2, 3 inner iterations",
            "n_points": cloud.n,
            "nnz": cloud.nnz,
            "precision": "fp64" if 0 in runs else "mixed",
        },
        "roofline": {
            "kernel": "k_flux (flux residual + RK stage)",
            "bound": "alu",
            "achieved": achieved,
            "peak": FP64_VALU_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP64_VALU_PEAK_TFLOPS,
            "traffic": committed_traffic(args.workload),
            "flops_per_launch": flops,
            "flops_unit": f"{FLOPS_PER_ENTRY_UNIT[FLOW['limiter']]} x k_mean per point",
            "avg_launch_us": flux_avg_s * 1e6,
            "itemised": {"flops_per_launch": flops_item,
                         "achieved": flops_item / flux_avg_s / 1e12,
                         "frac": flops_item / flux_avg_s / 1e12 / FP64_VALU_PEAK_TFLOPS},
        },
        "residual_first_last": [float(head["hist"][0, 0]), float(head["hist"][-1, 0])],
        "cl_cd": [head["cl"], head["cd"]],
    }
    if 0 in runs and 1 in runs:
        out["mixed"] = {"value": runs[1]["value"], "unit": "Mpoint-iter/s",
                        "ms_per_step": runs[1]["elapsed"] * 1e3 / args.steps,
                        "over_fp64": runs[1]["value"] / runs[0]["value"],
                        "dtype": "f32 flux body and q-derivative data; f64 q-derivative "
                                 "arithmetic, sums and update"}

        def vs_fp64(a0, a1):
            # mixed vs FP64 from the same freestream start after the same
            # number of iterations (the configuration's 1000)
            return {"iterations": a0["iterations"],
                    "cl_cd_fp64": list(a0["cl_cd"]), "cl_cd_mixed": list(a1["cl_cd"]),
                    "abs_dcl": abs(a1["cl_cd"][0] - a0["cl_cd"][0]),
                    "abs_dcd": abs(a1["cl_cd"][1] - a0["cl_cd"][1]),
                    "density_max_rel": float(np.abs(a1["rho"] - a0["rho"]).max()
                                             / np.abs(a0["rho"]).max())}
        if runs[0]["acc"] and runs[1]["acc"]:
            out["mixed"]["vs_fp64"] = vs_fp64(runs[0]["acc"], runs[1]["acc"])
        if "mixed_grad1" in runs:
            r = runs["mixed_grad1"]
            out["mixed"]["fp64_data_q_derivatives"] = {
                "value": r["value"], "ms_per_step": r["elapsed"] * 1e3 / args.steps,
                "over_fp64": r["value"] / runs[0]["value"]}
            if runs[0]["acc"] and r["acc"]:
                out["mixed"]["fp64_data_q_derivatives"]["vs_fp64"] = vs_fp64(runs[0]["acc"],
                                                                              r["acc"])
    if not headline:
        args.no_batch_study = args.no_warm_study = args.no_cpu_baseline = True
    if not args.no_batch_study:
        log("batched-cases study")
        try:
            out["batched"] = batch_study()
        except Exception as e:  # reported, never hides the throughput line
            out["batched"] = {"error": f"{type(e).__name__}: {e}"}
    if args.batch_drop_study > 0:
        log("batched cases to the drop")
        try:
            out["batched_to_drop"] = batch_drop_study(
                args.batch_drop_study, args.batch_drop_max_iter,
                sequential=not args.batch_drop_no_sequential)
        except Exception as e:  # reported, never hides the throughput line
            out["batched_to_drop"] = {"error": f"{type(e).__name__}: {e}"}
    if args.warm_study_large:
        log("larger warm-start study")
        try:
            out["warm_start_large"] = warm_study_large()
        except Exception as e:  # reported, never hides the throughput line
            out["warm_start_large"] = {"error": f"{type(e).__name__}: {e}"}
    if not args.no_warm_study:
        log("warm-start study")
        try:
            out["warm_start"] = warm_study()
        except Exception as e:  # reported, never hides the throughput line
            out["warm_start"] = {"error": f"{type(e).__name__}: {e}"}
    if not args.no_cpu_baseline:
        log("cpu baseline (OpenMP oracle, whole iterations; serial oracle, one stage)")
        out["cpu_baseline"] = cpu_baseline(cloud)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
