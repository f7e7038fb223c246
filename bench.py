#!/usr/bin/env python3
"""Benchmark of the block-step Hermite hot path on one MI355X.

Workload: King W0=7 cluster, N = 2^20 equal-mass stars (Henon units,
eps = 1e-4), 6th-order Hermite.  One step is one full pass of the hot path --
block-step scheduler, predictor over all N, pairwise force on the active
set, corrector + interpolation + time step -- with every particle on one
level (k_min = k_max = 10), so each step has N_act = N and does N_act * N =
2^40 pair interactions (self pair counted).  Metric: pair interactions per
second of the whole step, MIXED force precision, with the FP64 force timed
beside it and the error of both against the CPU oracle on a sample of rows.

A second workload, --workload batched, advances 256 independent Plummer
clusters (N_c = round(2^U(10, 16)), 6th order, MIXED, eta = 0.1) by the same
number of block steps per cluster twice: through the batched entry points
(one captured HIP graph per batched step, replayed) and with one context per
cluster (one nbody_step per cluster and block step).  Metric: aggregate pair
interactions per second of each.

A third workload, --workload microbench, times the force call alone
(nbody_predict once, then nbody_force_block) on a King W0=6 model of
N = 262144 for active sets N_act in {1, 16, 256, 4096, 65536, N} (random
subsets), FP64 vs MIXED vs DS, and reports pair interactions/s, % of the
VALU peak and the error against the oracle on sampled active rows.

Two integration workloads: --workload c2 (Plummer N = 131072, 6th order,
FP64 vs MIXED to t_end, with the active-block histogram, whole-run
interactions/s and energy drift) and --workload c3 (King W0=7 with 2^20 stars
plus a black-hole binary, 8th order, MIXED, a short run).

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1312_1789_amd.abi import TICK_BITS, TICKS_PER_UNIT as TICKS  # noqa: E402  (no torch import)

METRIC = "pair interactions/s & % VALU peak, 6th-order N=1M, mixed vs FP64 at stated error"
# Algorithmic flops per pair interaction: the minimal operation list of the
# pairwise force with its potential (add/sub/mul = 1, FMA = 2, rsqrt = 1) is
# 43 / 80 / 127 at orders 4 / 6 / 8, 2 of them the potential's.  The force
# kernels of a block step, and every kernel timed here, do not sum the
# potential, so their work is 41 / 78 / 125 flops per interaction.
FLOPS_WITH_POT = {4: 43, 6: 80, 8: 127}
FLOPS_PER_INTERACTION = {4: 41, 6: 78, 8: 125}
# The count commonly quoted for Hermite N-body codes (weights rsqrt heavier):
FLOPS_LITERATURE = {4: 60, 6: 97, 8: 144}
# VALU peaks of MI355X: 256 CUs x 4 SIMDs x 64 lanes x 2 flops (FMA) x 2.4 GHz
# at one wave instruction per SIMD every 4 cycles = 78.6 TFLOP/s, the FP64
# peak; FP32 instructions of two waves can issue together (measured on gfx950
# for VGPR-operand FP32 ops, unpacked), doubling that to 157.3 TFLOP/s, the
# FP32 peak the MIXED kernel is measured against.
PEAK_FP32_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "force_mixed_p6_n1M_traffic.md")
FORCE_SOURCES = [os.path.join(ROOT, "paper_1312_1789_amd", "csrc", f) for f in ("force.hip", "pairwise.h", "records.h")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_digest() -> str:
    """Digest of the force-kernel sources with comments and blank lines
    removed (a comment edit does not change the profiled kernel)."""
    import re
    h = hashlib.sha256()
    for f in FORCE_SOURCES:
        text = open(f).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        lines = [ln.rstrip() for ln in text.split("\n") if ln.strip()]
        h.update("\n".join(lines).encode())
    return h.hexdigest()[:16]


def read_traffic(n_act: int, n: int, shape):
    """HBM bytes per force launch from the committed counter summary, or None
    when it is missing or was taken on a different force-kernel source or
    launch shape."""
    if not os.path.exists(PROFILE_TRAFFIC):
        return None
    vals = {}
    for line in open(PROFILE_TRAFFIC):
        if ":" in line and line.strip().startswith("- "):
            k, v = line.strip()[2:].split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("force_source_sha") != source_digest():
        return None
    if int(vals.get("n", -1)) != n or int(vals.get("n_act", -1)) != n_act:
        return None
    if shape is None or vals.get("launch") != "%d,%d,%d,%d" % tuple(shape):
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def kernel_name(used, order):
    """The force kernel a MIXED launch ran, from the shape the library
    reports for it (ni, block, n_split, jpath)."""
    ni, block, n_split, jpath = used
    k = {1: "k_force", 2: "k_force_lds", 3: "k_force_ws"}.get(jpath, "k_force")
    return "%s<PolMx<%d, no potential>, ni=%d> block %d, %d j-splits (MIXED pairwise force)" % (
        k, order, ni, block, n_split)


def cpu_model() -> str:
    """The host CPU's model name (as lscpu reports it)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def run_precision(model, precision, order, steps, warmup, level, tune_max, force_shape=None):
    import torch
    from paper_1312_1789_amd import Simulation
    sim = Simulation(model.m, model.x, model.v, order=order, precision=precision, eps2=1e-8, eta=0.1,
                     eta_start=0.01, k_min=level, k_max=level)
    t0 = time.perf_counter()
    sim.init()
    torch.cuda.synchronize()
    log("[%s] init (two FP64 force passes) %.2f s" % (precision, time.perf_counter() - t0))
    shape = None
    if force_shape:
        ni, block, n_split, jpath = force_shape
        sim.set_launch(ni, block, n_split, jpath)
        shape = {"ni": ni, "block": block, "n_split": n_split, "jpath": jpath, "set_by": "--force-shape"}
        log("[%s] force launch shape set: %s" % (precision, shape))
    elif tune_max > 0:
        t0 = time.perf_counter()
        sim.predict(0)
        sim.autotune(tune_max, 2)
        table = sim.tuning()
        r = table[-1]
        shape = {"ni": r[1], "block": r[2], "n_split": r[3], "jpath": r[4], "tuned_up_to_n_act": r[0]}
        log("[%s] autotune up to n_act %d: %.1f s; shape for the full active set %s"
            % (precision, r[0], time.perf_counter() - t0, shape))
    for w in range(warmup):
        t, na = sim.step()
        log("[%s] warmup step %d: tick %d n_act %d" % (precision, w, t, na))
    sim.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n_act_sum = 0
    for k in range(steps):
        t, na = sim.step()
        n_act_sum += na
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    phases, nt = sim.timers()
    ms_step = wall / steps * 1e3
    inter = float(n_act_sum) * model.n
    used = sim.last_launch()
    log("[%s] %d steps: %.1f ms/step, %.4e interactions/s; phases (ms/step) %s; force launched as ni %d, "
        "block %d, %d splits, jpath %d" % (precision, steps, ms_step, inter / wall,
                                          {k: round(v / nt, 3) for k, v in phases.items()}, *used))
    if shape is not None:
        shape["used"] = {"ni": used[0], "block": used[1], "n_split": used[2], "jpath": used[3]}
    return sim, {"ms_per_step": ms_step, "interactions_per_s": inter / wall, "n_act_per_step": n_act_sum / steps,
                 "phase_ms_per_step": {k: v / nt for k, v in phases.items()}, "launch": shape, "used": used}


def cpu_baseline_and_error(model, sims, order, target_s):
    """The oracle on the host cores: force on a bounded sample of active rows
    of the same step (the state of the MIXED run, predicted to its next
    time), timed; and the error of each GPU precision on those rows."""
    import torch
    import oracle
    import nbody_ics
    from oracle import OracleConfig
    n = model.n
    sim = sims["mixed"]
    h = sim.to_numpy()
    T = int((h["t_tick"] + (1 << (TICK_BITS - h["level"].astype(np.int64)))).min())
    cfg = OracleConfig(order=order, eps2=1e-8)
    st = oracle.State(h["m"], h["x"], h["v"], order, h["d"], h["t_tick"], h["level"])
    xp, vp, ap, jp = oracle.predict(cfg, st, T)
    # calibrate the sample size on 128 rows
    cal = nbody_ics.active_subset(n, 128, 1500)
    t0 = time.perf_counter()
    oracle.force(cfg, h["m"], xp, vp, ap, None, act=cal)
    rate = 128 * n / (time.perf_counter() - t0)
    rows = int(min(max(256, target_s * rate / n), 65536)) // 64 * 64
    sample = nbody_ics.active_subset(n, rows, 1500 + 12)
    t0 = time.perf_counter()
    ref = oracle.force(cfg, h["m"], xp, vp, ap, None, act=sample)
    dt = time.perf_counter() - t0
    cores = oracle.num_threads()
    log("[cpu] oracle: %d rows x %d j in %.1f s on %d threads = %.3e interactions/s" % (rows, n, dt, cores,
                                                                                      rows * n / dt))
    errors = {}
    act = torch.as_tensor(sample, device="cuda:0")
    for prec, s in sims.items():
        s.load_state(h["x"], h["v"], h["d"], h["t_tick"], h["level"])
        s.predict(T)
        out = s.force_block(act)
        torch.cuda.synchronize()
        e = {}
        for key in ("acc", "jrk", "snp"):
            g = out[key].cpu().numpy()
            r = np.linalg.norm(g - ref[key], axis=0) / np.linalg.norm(ref[key], axis=0)
            e[key] = {"rms": float(np.sqrt(np.mean(r * r))), "max": float(r.max())}
        errors[prec] = e
        log("[cpu] %s error vs oracle: %s" % (prec, {k: "%.2e/%.2e" % (v["rms"], v["max"]) for k, v in e.items()}))
    base = {"value": rows * n / dt, "unit": "interactions/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "sample": "%d random active rows x all %d j-particles of the same 6th-order step (FP64 C oracle, "
                      "OpenMP over rows), %.1f s" % (rows, n, dt)}
    return base, errors, rows


BATCH_METRIC = "aggregate pair interactions/s, 256 batched Plummer clusters, 6th order, mixed"


def batched_clusters(n_clusters: int, seed: int = 1400):
    """Cluster sizes round(2^U(10, 16)) from one seeded draw; cluster c is a
    Plummer model with seed seed + c."""
    import nbody_ics
    return nbody_ics.batched_plummer(n_clusters, seed)


def run_batched(args):
    import torch
    from paper_1312_1789_amd import Batch, Simulation
    t0 = time.perf_counter()
    models = batched_clusters(args.clusters)
    sizes = [m.n for m in models]
    log("workload: %d Plummer clusters, n total %d (min %d, max %d), %.1f s to generate"
        % (len(models), sum(sizes), min(sizes), max(sizes), time.perf_counter() - t0))
    kw = dict(order=6, eps2=1e-8, eta=0.1, eta_start=0.01, k_min=3, k_max=20)
    clusters = [(m.m, m.x, m.v) for m in models]
    B = Batch(clusters, precision="mixed", **kw)
    if args.batch_per_wg or args.batch_grid or args.batch_itile:
        B.set_launch(args.batch_grid, args.batch_per_wg, args.batch_itile)
    t0 = time.perf_counter()
    B.init()
    B.synchronize()
    log("[batched] init %.2f s" % (time.perf_counter() - t0))
    # start-up transient: every cluster to t_warm (all particles synchronised there)
    t_warm = int(args.warm_time * TICKS)
    B.set_end(t_warm)
    B.capture()
    t0 = time.perf_counter()
    replays = 0
    while True:
        B.replay(64)
        replays += 64
        live, tcur = B.poll()
        if live == 0:
            break
        if replays % 1024 == 0:
            log("[batched] warm-up replay %d: %d clusters live, min time %.5f" % (replays, live, min(tcur) / TICKS))
    log("[batched] warm-up to t = %.4f: %d replays, %.1f s" % (t_warm / TICKS, replays, time.perf_counter() - t0))
    B.set_end(1 << 62)
    tuned = None
    if args.autotune_steps > 0:
        t0 = time.perf_counter()
        st0 = B.stats().steps
        B.autotune(args.autotune_steps)
        tuned = B.get_launch()
        log("[batched] autotune (every shape timed on the same %d steps, %d batched steps taken): force_grid %d, "
            "items per workgroup %d, i_tile %d, %.1f s"
            % (args.autotune_steps, B.stats().steps - st0, tuned[0], tuned[1], tuned[2], time.perf_counter() - t0))
    shape = B.get_launch()
    h = B.to_numpy()   # the common starting state of the three timed runs
    B.capture()
    B.replay(args.warmup)
    B.synchronize()
    s0 = B.stats()
    t0 = time.perf_counter()
    B.replay(args.steps)
    B.synchronize()
    wall = time.perf_counter() - t0
    s1 = B.stats()
    inter = s1.interactions - s0.interactions
    nact = (s1.sum_n_act - s0.sum_n_act) / args.steps
    live, tcur = B.poll()
    log("[batched] %d graph replays: %.3f ms/replay, %.4e interactions/s, mean active %.0f per replay, "
        "cluster times %.4f..%.4f" % (args.steps, wall / args.steps * 1e3, inter / wall, nact,
                                      min(tcur) / TICKS, max(tcur) / TICKS))
    batched = {"interactions_per_s": inter / wall, "ms_per_batched_step": wall / args.steps * 1e3,
               "interactions": inter, "mean_active_per_batched_step": nact,
               "launch": {"force_grid": shape[0], "items_per_wg": shape[1], "i_tile": shape[2]},
               "cluster_time_range": [min(tcur) / TICKS, max(tcur) / TICKS]}
    h_graph = B.to_numpy()
    # the shape of the work: over a few more batched steps, the pair
    # evaluations done against those the i-tiles pad to (64 or 256 rows), and
    # the share of the work in tiles of at most 16 rows
    occ = {"steps": 0, "interactions": 0.0, "padded_64": 0.0, "padded_256": 0.0, "padded_64_pow2_tail": 0.0,
           "work_in_small_tiles": 0.0}
    nsz = np.array(sizes, dtype=np.float64)
    for _ in range(args.occupancy_steps):
        B.step(1)
        aoff = np.array(B.last_step()[0], dtype=np.int64)
        a = np.diff(aoff).astype(np.float64)
        occ["steps"] += 1
        occ["interactions"] += float(np.sum(a * nsz))
        occ["padded_64"] += float(np.sum(np.ceil(a / 64) * 64 * nsz))
        occ["padded_256"] += float(np.sum(np.ceil(a / 256) * 256 * nsz))
        # 64-row tiles with each cluster's last tile cut to the next power of two of its rows
        rem = a % 64
        tail = np.where(rem > 0, 2.0 ** np.ceil(np.log2(np.maximum(rem, 1))), 0.0)
        occ["padded_64_pow2_tail"] += float(np.sum((np.floor(a / 64) * 64 + tail) * nsz))
        occ["work_in_small_tiles"] += float(np.sum(np.where(a % 64 <= 16, (a % 64) * nsz, 0.0)))
    if occ["steps"]:
        log("[batched] work over %d more steps: %.3e interactions; tiles of 64 rows padded to %.3e (%.1f%% used), "
            "of 256 rows to %.3e (%.1f%% used), of 64 rows with power-of-two last tiles to %.3e (%.1f%% used); "
            "%.1f%% of the work in tiles of at most 16 rows"
            % (occ["steps"], occ["interactions"], occ["padded_64"], 100 * occ["interactions"] / occ["padded_64"],
               occ["padded_256"], 100 * occ["interactions"] / occ["padded_256"], occ["padded_64_pow2_tail"],
               100 * occ["interactions"] / occ["padded_64_pow2_tail"],
               100 * occ["work_in_small_tiles"] / occ["interactions"]))
    batched["work_shape"] = occ
    del B
    # the same steps launched eagerly (no graph)
    E = Batch(clusters, precision="mixed", **kw)
    E.set_launch(0, shape[1], shape[2])
    E.load_state(h)
    E.step(args.warmup)
    E.synchronize()
    e0 = E.stats()
    t0 = time.perf_counter()
    E.step(args.steps)
    E.synchronize()
    ewall = time.perf_counter() - t0
    e1 = E.stats()
    log("[batched eager] %.3f ms/step, %.4e interactions/s" % (ewall / args.steps * 1e3,
                                                              (e1.interactions - e0.interactions) / ewall))
    h_eager = E.to_numpy()
    same = all(np.array_equal(h_graph[k], h_eager[k]) for k in ("x", "v", "t_tick", "level")) and \
        all(np.array_equal(a, b) for a, b in zip(h_graph["d"], h_eager["d"]))
    log("[batched eager] final state %s the graph replays' bit for bit" % ("equals" if same else "DIFFERS FROM"))
    eager = {"interactions_per_s": (e1.interactions - e0.interactions) / ewall,
             "ms_per_batched_step": ewall / args.steps * 1e3, "final_state_equals_graph": bool(same)}
    del E
    # one context per cluster, the same number of block steps each, same start
    tot_inter, tot_wall, tot_steps = 0.0, 1e-30, 0
    # clusters whose final state is compared with the batched run's (the
    # single-system force kernels sum in another order: not bit for bit)
    check = set(np.argsort(sizes)[[0, len(sizes) // 2, len(sizes) - 1]].tolist())
    state_diff = {}
    for c, m in enumerate([] if args.skip_per_cluster else models):
        sim = Simulation(m.m, m.x, m.v, precision="mixed", **kw)
        a, b = sum(sizes[:c]), sum(sizes[:c + 1])
        sim.load_state(h["x"][:, a:b], h["v"][:, a:b], [d[:, a:b] for d in h["d"]], h["t_tick"][a:b],
                       h["level"][a:b])
        for _ in range(args.warmup):
            sim.step()
        torch.cuda.synchronize()
        a0 = sim.stats().interactions
        t0 = time.perf_counter()
        for _ in range(args.steps):
            sim.step()
        torch.cuda.synchronize()
        tot_wall += time.perf_counter() - t0
        tot_inter += sim.stats().interactions - a0
        tot_steps += args.steps
        if c in check:
            hc = sim.to_numpy()
            same_t = bool(np.array_equal(hc["t_tick"], h_graph["t_tick"][a:b]))
            dx = float(np.max(np.abs(hc["x"] - h_graph["x"][:, a:b])))
            state_diff[int(c)] = {"n": int(m.n), "times_equal": same_t, "max_abs_dx": dx}
            log("[per-cluster] cluster %d (n %d) vs batched: times %s, max |dx| %.2e"
                % (c, m.n, "equal" if same_t else "DIFFER", dx))
        if c % 32 == 31:
            log("[per-cluster] %d clusters done, %.1f s timed" % (c + 1, tot_wall))
        sim.close()
        del sim
    log("[per-cluster] %d steps over %d contexts: %.1f s, %.4e interactions/s"
        % (tot_steps, len(models), tot_wall, tot_inter / tot_wall))
    per_cluster = {"interactions_per_s": tot_inter / tot_wall, "seconds": tot_wall, "interactions": tot_inter,
                   "skipped": bool(args.skip_per_cluster), "final_state_vs_batched": state_diff}
    line = {
        "metric": BATCH_METRIC,
        "value": batched["interactions_per_s"],
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": batched["ms_per_batched_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "%d Plummer clusters, N_c = round(2^U(10,16)) (seed 1400 + c), n = %d, 6th-order "
                               "Hermite block steps, MIXED force, eta = 0.1, eps = 1e-4, from t = %.4f; one batched "
                               "step = one block step of every cluster" % (len(models), sum(sizes),
                                                                            t_warm / TICKS),
                   "n": sum(sizes), "clusters": len(models), "order": 6, "precision": "mixed"},
        "autotuned": tuned is not None,
        "batched_graph": batched,
        "batched_eager": eager,
        "one_context_per_cluster": per_cluster,
        "graph_over_per_cluster": (batched["interactions_per_s"] / per_cluster["interactions_per_s"]
                                   if per_cluster["interactions_per_s"] > 0 else None),
    }
    print(json.dumps(line), flush=True)


MICRO_METRIC = "force call: pair interactions/s and % VALU peak per N_act, King W0=6 N=262144"


def _time_launches(fn, min_ms=30.0, max_reps=50):
    """Median duration (ms) of fn() from HIP events on the current stream."""
    import torch
    fn()
    fn()
    s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s0.record()
    fn()
    s1.record()
    torch.cuda.synchronize()
    one = max(s0.elapsed_time(s1), 1e-3)
    reps = int(min(max(3, min_ms / one), max_reps))
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    return float(np.median(times)), reps


def run_microbench(args):
    import torch
    import nbody_ics
    import oracle
    from oracle import OracleConfig
    from paper_1312_1789_amd import Simulation
    n = args.micro_n
    t0 = time.perf_counter()
    model = nbody_ics.king(n, 6.0, 15)
    d_all = nbody_ics.random_derivs(n, 1515, 8)
    log("workload: King W0=6 n=%d (%.1f s to generate)" % (n, time.perf_counter() - t0))
    sizes = [k for k in (1, 16, 256, 4096, 65536) if k < n] + [n]
    orders = [int(o) for o in args.micro_orders.split(",")]
    tick0 = 5 * (TICKS >> 3)
    table = []
    for order in orders:
        d = d_all[: order - 2]
        cfg = OracleConfig(order=order, eps2=1e-8)
        acts = {k: nbody_ics.active_subset(n, k, 1500 + int(np.log2(k))) for k in sizes}
        refs = {}
        t0 = time.perf_counter()
        for k in sizes:
            rows = acts[k][: min(k, args.micro_rows)]
            refs[k] = (rows, oracle.force(cfg, model.m, model.x, model.v, d[0] if order >= 6 else None,
                                          d[1] if order >= 8 else None, act=rows, with_pot=False))
        log("[micro] order %d: oracle rows %.1f s" % (order, time.perf_counter() - t0))
        for prec in ("fp64", "mixed", "ds"):
            sim = Simulation(model.m, model.x, model.v, order=order, precision=prec, eps2=1e-8, eta=0.1)
            sim.load_state(model.x, model.v, d, np.full(n, tick0, np.int64), np.full(n, 3, np.int32))
            sim.predict(tick0)
            tuning = None
            if args.micro_tune_max > 0:
                t0 = time.perf_counter()
                sim.autotune(args.micro_tune_max, 2)
                tuning = sim.tuning()
                log("[micro] p%d %s autotune %.1f s: %s" % (order, prec, time.perf_counter() - t0,
                                                             [(r[0], r[1], r[2], r[3], r[4]) for r in tuning]))
            peak = PEAK_FP64_TFLOPS if prec == "fp64" else PEAK_FP32_TFLOPS
            for k in sizes:
                act = torch.as_tensor(acts[k], device="cuda:0")
                out = sim.alloc_forces(k)
                ms, reps = _time_launches(lambda: sim.force_block(act, out, with_pot=False))
                inter = float(k) * n
                rate = inter / (ms * 1e-3)
                tf = FLOPS_PER_INTERACTION[order] * rate / 1e12
                rows, ref = refs[k]
                pos = np.searchsorted(acts[k], rows)
                err = {}
                for key in ("acc", "jrk", "snp", "crk")[: order // 2]:
                    g = out[key][:, pos].cpu().numpy()
                    e = np.linalg.norm(g - ref[key], axis=0) / np.linalg.norm(ref[key], axis=0)
                    err[key] = {"rms": float(np.sqrt(np.mean(e * e))), "max": float(e.max())}
                shape = None
                if tuning:
                    r = next((r for r in tuning if r[0] >= k), tuning[-1])
                    shape = {"ni": r[1], "block": r[2], "n_split": r[3], "jpath": r[4]}
                row = {"order": order, "precision": prec, "n_act": k, "ms": ms, "reps": reps, "tuned_shape": shape,
                       "interactions_per_s": rate, "tflops": tf, "frac_of_peak": tf / peak, "peak_tflops": peak,
                       "error": err, "error_rows": int(len(rows))}
                table.append(row)
                log("[micro] p%d %-5s n_act %7d: %9.4f ms  %.3e int/s  %6.2f TF  %5.1f%% peak  acc rms %.1e jrk rms %.1e"
                    % (order, prec, k, ms, rate, tf, 100 * tf / peak, err["acc"]["rms"], err["jrk"]["rms"]))
            sim.close()
            del sim
    head = [r for r in table if r["precision"] == "mixed" and r["n_act"] == n and r["order"] == orders[0]][0]
    line = {
        "metric": MICRO_METRIC,
        "value": head["interactions_per_s"],
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": None,
        "warmup": 2,
        "ms_per_step": head["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "King W0=6 n=%d, stored derivatives seeded (|a| ~ 1), force call on random active "
                               "subsets; flops per interaction %s" % (n, FLOPS_PER_INTERACTION),
                   "n": n, "orders": orders},
        "table": table,
    }
    print(json.dumps(line), flush=True)


def _state_bytes(order):
    """Bytes of stored state the predictor reads per particle: m, t_tick and
    x, v, a^(0..p-3) (3 doubles each).  The separate predictor also writes a
    record that the force kernel reads back."""
    return 8 + 8 + 3 * 8 * order


def run_smallstep(args):
    """Prediction of all n particles plus the force on a small active set,
    the work of a block step with few active particles: the predictor kernel
    followed by the wave j-split force kernel, against the one kernel that
    predicts the j-particles in its loads."""
    import torch
    import nbody_ics
    from paper_1312_1789_amd import Simulation
    table = []
    sizes = [1, 2, 4, 8, 16, 32]
    for n in [int(v) for v in args.small_n.split(",")]:
        t0 = time.perf_counter()
        model = nbody_ics.king(n, 7.0, 23)
        rng = np.random.default_rng(24)
        level = rng.integers(3, 21, n).astype(np.int32)
        T = 3 * (TICKS >> 3) + (TICKS >> 5)
        dt = 1 << (TICK_BITS - level.astype(np.int64))
        t_tick = (T // dt) * dt
        T = int((t_tick + dt).min())
        log("[small] King W0=7 n=%d, random block state (%.1f s to generate)" % (n, time.perf_counter() - t0))
        for order in [int(o) for o in args.micro_orders.split(",")]:
            d = nbody_ics.random_derivs(n, 25, order)
            for prec in ("fp64", "mixed"):
                sim = Simulation(model.m, model.x, model.v, order=order, precision=prec, eps2=1e-8, eta=0.1)
                sim.load_state(model.x, model.v, d, t_tick, level)
                rec_b = {4: 64, 6: 80, 8: 112}[order] if prec == "fp64" else {4: 64, 6: 64, 8: 80}[order]
                for k in sizes:
                    act = torch.as_tensor(nbody_ics.active_subset(n, k, 2400 + k), device="cuda:0")
                    out = {}
                    ms = {}
                    for fuse in (False, True):
                        sim.set_fusion(fuse)
                        o = sim.alloc_forces(k)
                        ms[fuse], _ = _time_launches(lambda: sim.predict_force(T, act, o, with_pot=False))
                        out[fuse] = o
                    same = all(torch.equal(out[False][key], out[True][key]) for key in ("acc", "jrk", "snp", "crk")[: order // 2])
                    fused_bytes = float(n) * _state_bytes(order)
                    plain_bytes = fused_bytes + 2.0 * n * rec_b
                    row = {"n": n, "order": order, "precision": prec, "n_act": k, "ms_plain": ms[False],
                           "ms_fused": ms[True], "speedup": ms[False] / ms[True], "bitwise_equal": bool(same),
                           "fused_GBps": fused_bytes / (ms[True] * 1e-3) / 1e9,
                           "plain_GBps": plain_bytes / (ms[False] * 1e-3) / 1e9}
                    table.append(row)
                    log("[small] n %8d p%d %-5s n_act %3d: predict+force %.4f ms, fused %.4f ms (%.2fx), %s; "
                        "algorithmic HBM rate fused %.0f GB/s, plain %.0f GB/s"
                        % (n, order, prec, k, ms[False], ms[True], ms[False] / ms[True],
                           "bitwise equal" if same else "DIFFERENT", row["fused_GBps"], row["plain_GBps"]))
                sim.close()
                del sim
                torch.cuda.empty_cache()
    line = {"metric": "predict + force time for small active sets (fused vs separate kernels)",
            "value": float(np.mean([r["speedup"] for r in table])), "unit": "x (mean speedup)", "n_gpus": 1,
            "higher_is_better": True, "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
            "config": {"workload": "King W0=7, random block state (levels 3..20), seeded derivatives; "
                                   "n in %s, n_act 1..32" % args.small_n},
            "table": table}
    print(json.dumps(line), flush=True)


def run_neighbour(args):
    """The force split by neighbour spheres with the neighbour lists (the
    regular-force call of an Ahmad-Cohen scheme), next to the plain force call
    on the same active rows: King W0=7, 4th order, each active row's radius
    enclosing its nearest --nb-k particles."""
    import torch
    import nbody_ics
    from paper_1312_1789_amd import Simulation
    n = args.nb_n
    model = nbody_ics.king(n, 7.0, 29)
    x = torch.as_tensor(model.x, device="cuda:0")
    table = []
    for n_act in [int(v) for v in args.nb_act.split(",")]:
        act_np = nbody_ics.active_subset(n, n_act, 2900 + n_act % 97)
        act = torch.as_tensor(act_np, device="cuda:0")
        # radius^2 half way between the k-th and (k+1)-th nearest squared distance
        h2 = torch.empty(n_act, dtype=torch.float64, device="cuda:0")
        for c0 in range(0, n_act, 256):
            xi = x[:, act[c0:c0 + 256].long()]
            d2 = ((x[:, None, :] - xi[:, :, None]) ** 2).sum(0)
            d2[torch.arange(xi.shape[1]), act[c0:c0 + 256].long()] = float("inf")
            v, _ = torch.topk(d2, args.nb_k + 1, dim=1, largest=False)
            h2[c0:c0 + 256] = (v[:, -2] * v[:, -1]).sqrt()
            del d2
        for prec in ("fp64", "mixed"):
            sim = Simulation(model.m, model.x, model.v, order=4, precision=prec, eps2=1e-8, eta=0.01)
            sim.predict(0)
            out_nb = sim.force_block_nb(act, h2, args.nb_max)
            out = sim.alloc_forces(n_act)
            ms_nb, _ = _time_launches(lambda: sim.force_block_nb(act, h2, args.nb_max, out_nb))
            ms_f, _ = _time_launches(lambda: sim.force_block(act, out, with_pot=False))
            cnt = out_nb["nb_count"].cpu().numpy()
            tot = (out_nb["acc_irr"] + out_nb["acc_reg"] - out["acc"]).norm(dim=0) / out["acc"].norm(dim=0)
            rate = float(n_act) * n / (ms_nb * 1e-3)
            peak = PEAK_FP64_TFLOPS if prec == "fp64" else PEAK_FP32_TFLOPS
            row = {"n": n, "n_act": n_act, "precision": prec, "ms_nb": ms_nb, "ms_force": ms_f,
                   "interactions_per_s": rate, "frac_of_peak": FLOPS_PER_INTERACTION[4] * rate / 1e12 / peak,
                   "nb_mean": float(cnt.mean()), "nb_max": int(cnt.max()),
                   "irr_plus_reg_vs_full_max": float(tot.max())}
            table.append(row)
            log("[nb] n %d n_act %6d %-5s: split force + lists %.4f ms (%.3e int/s, %.1f%% of peak at 41 flops), "
                "plain force %.4f ms (%.2fx); neighbours mean %.1f max %d; |irr + reg - full| / |full| max %.1e"
                % (n, n_act, prec, ms_nb, rate, 100 * row["frac_of_peak"], ms_f, ms_nb / ms_f,
                   cnt.mean(), cnt.max(), row["irr_plus_reg_vs_full_max"]))
            sim.close()
            del sim
            torch.cuda.empty_cache()
    line = {"metric": "neighbour-split force with neighbour lists (Ahmad-Cohen regular force), interactions/s",
            "value": max(r["interactions_per_s"] for r in table if r["precision"] == "mixed"),
            "unit": "interactions/s", "n_gpus": 1, "higher_is_better": True, "vs_baseline": None,
            "dtype": "f32+f64", "data": "synthetic",
            "config": {"workload": "King W0=7 n=%d, 4th order, radii enclosing the %d nearest particles, list cap %d"
                                   % (n, args.nb_k, args.nb_max)},
            "table": table}
    print(json.dumps(line), flush=True)


def binary_gw(h, c, i=0, j=1):
    from paper_1312_1789_amd.diagnostics import binary_gw as _gw
    return _gw(h, c, i, j)


def run_pn(args):
    """Block steps of a cluster with a black-hole binary with and without the
    post-Newtonian terms of the binary (4th order, MIXED): whole-step rate,
    the binary's semi-major axis, and the cost of the terms; then a two-body
    inspiral against Peters' rate."""
    import torch
    import nbody_ics
    from paper_1312_1789_amd import Simulation
    n_stars = args.pn_stars
    model = nbody_ics.with_bh_binary(nbody_ics.king(n_stars, 7.0, 31), 0.01, 0.2)
    t_end = int(args.pn_t_end * TICKS)

    def binary_a(h):
        M = h["m"][0] + h["m"][1]
        r = np.linalg.norm(h["x"][:, 0] - h["x"][:, 1])
        w = h["v"][:, 0] - h["v"][:, 1]
        return -M / (2.0 * (0.5 * np.dot(w, w) - M / r))

    runs = {}
    for label, c, terms in (("newtonian", 0.0, 0), ("pn_1_2_2.5", args.pn_c, 7)):
        sim = Simulation(model.m, model.x, model.v, order=4, precision="mixed", eps2=1e-8, n_hard=2, eta=0.01,
                         eta_start=0.01, c_light=c, pn_terms=terms)
        sim.init()
        a0 = binary_a(sim.to_numpy())
        sim.predict(0)
        sim.autotune(min(65536, model.n), 2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        steps, _ = sim.run(t_end)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        st = sim.stats()
        h_end = sim.to_numpy()
        a1 = binary_a(h_end)
        runs[label] = {"steps": steps, "wall_s": wall, "interactions_per_s": st.interactions / wall,
                       "ms_per_step": wall / max(steps, 1) * 1e3, "binary_a": [a0, a1],
                       "binary_end": binary_gw(h_end, args.pn_c)}
        log("[pn] %-9s binary at the end: %s" % (label, runs[label]["binary_end"]))
        log("[pn] %-9s %d steps to t = %.5f in %.2f s (%.3f ms/step, %.3e int/s); binary a %.6f -> %.6f"
            % (label, steps, t_end / TICKS, wall, runs[label]["ms_per_step"], runs[label]["interactions_per_s"],
               a0, a1))
        sim.close()
        del sim
        torch.cuda.empty_cache()
    # two bodies with the 2.5PN terms alone: Peters' rate
    m = np.array([0.6, 0.4])
    x = np.array([[0.4, -0.6], [0.0, 0.0], [0.0, 0.0]])
    v = np.array([[0.0, 0.0], [0.4, -0.6], [0.0, 0.0]])
    sim = Simulation(m, x, v, order=4, precision="fp64", eps2=0.0, n_hard=2, eta=0.01, eta_start=0.01,
                     c_light=8.0, pn_terms=4)
    sim.init()
    T = 16.0
    sim.integrate(int(T * TICKS))
    h = sim.to_numpy()
    rate = (binary_a(h) - 1.0) / T
    peters = -64.0 / 5.0 * 0.24 / 8.0 ** 5
    log("[pn] two-body inspiral (c = 8, 2.5PN): da/dt %.5e, Peters %.5e (ratio %.4f)" % (rate, peters, rate / peters))
    sim.close()
    line = {"metric": "whole-step interactions/s with post-Newtonian black-hole terms (4th order, MIXED)",
            "value": runs["pn_1_2_2.5"]["interactions_per_s"], "unit": "interactions/s", "n_gpus": 1,
            "higher_is_better": True, "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
            "config": {"workload": "King W0=7 %d stars + BH binary (0.01 + 0.01 at separation 0.2), c = %g, "
                                   "t = 0 -> %.5f" % (n_stars, args.pn_c, t_end / TICKS)},
            "runs": runs, "pn_over_newtonian_time_per_step":
                runs["pn_1_2_2.5"]["ms_per_step"] / runs["newtonian"]["ms_per_step"],
            "two_body_inspiral": {"da_dt": rate, "peters": peters}}
    print(json.dumps(line), flush=True)


def integrate_run(model, label, t_end_tick, hist_pass=True, fuse=True, **kw):
    """Integrate a Simulation to t_end_tick with nbody_step; returns the run
    record (steps, interactions/s, N_act histogram, energies, phase times).
    fuse: predictor inside the small-block force kernel (nbody_set_fusion)."""
    import torch
    from paper_1312_1789_amd import Simulation
    sim = Simulation(model.m, model.x, model.v, **kw)
    sim.set_fusion(fuse)
    sim.init()
    E0 = sum(sim.energy())
    sim.predict(0)
    sim.autotune(min(65536, model.n), 2)
    torch.cuda.synchronize()
    hist = np.zeros(32)
    whist = np.zeros(32)
    # nbody_run in slices of 1/64 time unit (progress lines), then one pass with
    # nbody_step per step for the active-block histogram, which needs each n_act
    steps = 0
    t0 = time.perf_counter()
    t_cur = 0
    while t_cur < t_end_tick:
        t_slice = min(t_end_tick, t_cur + (TICKS >> 6))
        k, _ = sim.run(t_slice)
        steps += k
        t_cur = t_slice
        log("[%s] t = %.5f, %d steps" % (label, t_cur / TICKS, steps))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    n_act_sum = sim.stats().sum_n_act
    if hist_pass:
        h_sim = Simulation(model.m, model.x, model.v, **kw)
        h_sim.init()
        while True:
            before = h_sim.stats().sum_n_act
            k, _ = h_sim.run(t_end_tick, 1)
            if k == 0:
                break
            na = h_sim.stats().sum_n_act - before
            b = int(np.log2(na))
            hist[b] += 1
            whist[b] += float(na) * model.n
        h_sim.close()
    E1 = sum(sim.energy())
    st = sim.stats()
    rec = {"steps": steps, "wall_s": wall, "interactions": st.interactions,
           "interactions_per_s": st.interactions / wall, "mean_n_act": n_act_sum / max(steps, 1),
           "dE_over_E": (E1 - E0) / E0, "dt_rule": sim.dt_rule, "dt_underflow": st.dt_underflow,
           "n_act_hist_log2": {"bins": [int(2 ** b) for b in range(32) if hist[b] > 0],
                               "steps": [int(hist[b]) for b in range(32) if hist[b] > 0],
                               "interaction_share": [float(whist[b] / whist.sum()) for b in range(32) if hist[b] > 0]}}
    if not hist_pass:
        rec.pop("n_act_hist_log2")
    log("[%s] %d steps to t = %.4f in %.1f s: %.4e interactions/s (whole steps), mean n_act %.0f, |dE/E| %.3e, "
        "rule %d" % (label, steps, t_end_tick / TICKS, wall, rec["interactions_per_s"], rec["mean_n_act"],
                     abs(rec["dE_over_E"]), sim.dt_rule))
    return sim, rec


def integrate_batched_one(model, t_end_tick, kw):
    """The same integration through the batched entry points with a single
    cluster: block steps replayed from a captured graph, no host round trip
    per step (the host polls every 256 replays)."""
    import torch
    from paper_1312_1789_amd import Batch
    B = Batch([(model.m, model.x, model.v)], precision="mixed", **kw)
    B.init()
    E0 = sum(t + w for t, w in zip(*B.energy()))
    h0 = B.to_numpy()
    B.set_end(t_end_tick)
    B.autotune(2)
    # the autotuner's steps are real: restart from the initial state for the timed run
    B.load_state(h0)
    B.capture()
    B.synchronize()
    s0 = B.stats()
    t0 = time.perf_counter()
    while True:
        B.replay(256)
        live, tcur = B.poll()
        if live == 0:
            break
    wall = time.perf_counter() - t0
    s1 = B.stats()
    E1 = sum(t + w for t, w in zip(*B.energy()))
    steps = s1.steps - s0.steps
    rec = {"steps_incl_idle_replays": steps, "wall_s": wall, "interactions": s1.interactions - s0.interactions,
           "interactions_per_s": (s1.interactions - s0.interactions) / wall, "dE_over_E": (E1 - E0) / E0,
           "dt_underflow": s1.dt_underflow, "launch": B.get_launch(), "t_end_reached": tcur[0] / TICKS}
    log("[mixed, one-cluster batch, graph] %d replays in %.1f s: %.4e interactions/s, |dE/E| %.3e, shape %s"
        % (steps, wall, rec["interactions_per_s"], abs(rec["dE_over_E"]), rec["launch"]))
    B.close()
    return rec


def run_c2(args):
    import nbody_ics
    n = args.c2_n
    model = nbody_ics.plummer(n, 12)
    t_end = int(args.c2_t_end * TICKS)
    log("workload: Plummer n=%d, 6th order, eta 0.1, to t = %.4f" % (n, t_end / TICKS))
    kw = dict(order=6, eps2=1e-8, eta=0.1, eta_start=0.01, k_min=3, k_max=20)
    runs = {}
    for label, prec, rule, fuse in (("mixed", "mixed", 0, True), ("mixed_no_fusion", "mixed", 0, False),
                                    ("fp64_rule_order4", "fp64", 2, True), ("fp64", "fp64", 0, True)):
        sim, runs[label] = integrate_run(model, label, t_end, hist_pass=(label == "mixed"), fuse=fuse,
                                         precision=prec, dt_rule=rule, **kw)
        sim.close()
        del sim
    runs["mixed_one_cluster_graph"] = integrate_batched_one(model, t_end, kw)
    mixed = runs["mixed"]
    line = {
        "metric": "C2: whole-run pair interactions/s, Plummer N=131072, 6th order, MIXED vs FP64",
        "value": mixed["interactions_per_s"], "unit": "interactions/s", "n_gpus": 1, "steps": mixed["steps"],
        "warmup": 0, "ms_per_step": mixed["wall_s"] / max(mixed["steps"], 1) * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "Plummer n=%d (seed 12), eps = 1e-4, 6th-order Hermite block steps, eta = 0.1, "
                               "t = 0 -> %.4f" % (n, t_end / TICKS), "n": n, "order": 6},
        "runs": runs,
        "mixed_over_fp64_same_rule": mixed["interactions_per_s"] / runs["fp64_rule_order4"]["interactions_per_s"],
    }
    print(json.dumps(line), flush=True)


def run_c3(args):
    import torch
    import nbody_ics
    n_stars = args.c3_stars
    model = nbody_ics.with_bh_binary(nbody_ics.king(n_stars, 7.0, 13), 0.01, 0.2)
    t_end = int(args.c3_t_end * TICKS)
    k_min = max(args.c3_k_min, int(np.ceil(-np.log2(args.c3_t_end))))
    log("workload: King W0=7 %d stars + BH binary, 8th order MIXED, to t = %.5f (k_min %d, k_max %d)"
        % (n_stars, t_end / TICKS, k_min, args.c3_k_max))
    x0 = model.x[:, :2].copy()
    kw = dict(order=8, precision=args.c3_precision, eps2=1e-8, n_hard=2, eta=args.c3_eta, eta_start=0.01,
              k_min=k_min, k_max=args.c3_k_max)
    plain = None
    if args.c3_compare:
        sim, plain = integrate_run(model, "c3, no fusion", t_end, hist_pass=False, fuse=False, **kw)
        sim.close()
        del sim
        torch.cuda.empty_cache()
    if args.c3_c > 0:
        sim, relat = integrate_run(model, "c3, post-Newtonian", t_end, hist_pass=False, c_light=args.c3_c,
                                   pn_terms=7, **kw)
        sim.close()
        del sim
        torch.cuda.empty_cache()
    sim, rec = integrate_run(model, "c3", t_end, hist_pass=False, **kw)
    if plain is not None:
        rec["without_fusion"] = {k: plain[k] for k in ("steps", "wall_s", "interactions_per_s", "dE_over_E")}
    if args.c3_c > 0:
        rec["post_newtonian"] = {k: relat[k] for k in ("steps", "wall_s", "interactions_per_s", "dE_over_E")}
        rec["post_newtonian"]["c_light"] = args.c3_c
    h = sim.to_numpy()
    sep0 = float(np.linalg.norm(x0[:, 0] - x0[:, 1]))
    sep1 = float(np.linalg.norm(h["x"][:, 0] - h["x"][:, 1]))
    rec["bh_separation"] = [sep0, sep1]
    rec["bh_binary_end"] = binary_gw(h, args.c3_c)
    log("[c3] BH separation %.6f -> %.6f; binary at the end %s" % (sep0, sep1, rec["bh_binary_end"]))
    line = {
        "metric": "C3: whole-run pair interactions/s, King W0=7 2^20 stars + BH binary, 8th order, MIXED",
        "value": rec["interactions_per_s"], "unit": "interactions/s", "n_gpus": 1, "steps": rec["steps"],
        "warmup": 0, "ms_per_step": rec["wall_s"] / max(rec["steps"], 1) * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "King W0=7 %d stars (seed 13) + two 0.01-mass BHs on a circular orbit of separation "
                               "0.2 (mutually unsoftened), eps = 1e-4, 8th-order Hermite, eta = 0.1, t = 0 -> %.5f, "
                               "steps 2^-%d .. 2^-%d" % (n_stars, t_end / TICKS, k_min, args.c3_k_max),
                   "n": model.n, "order": 8, "k_max": args.c3_k_max},
        "run": rec,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--workload", choices=["king1m", "batched", "microbench", "smallstep", "neighbour", "pn", "c2", "c3"], default="king1m")
    ap.add_argument("--c2-n", type=int, default=131072)
    ap.add_argument("--c2-t-end", type=float, default=1.0)
    ap.add_argument("--c3-stars", type=int, default=1 << 20)
    ap.add_argument("--c3-t-end", type=float, default=0.25)
    ap.add_argument("--c3-k-max", type=int, default=30, help="c3: smallest step 2^-k_max")
    ap.add_argument("--c3-k-min", type=int, default=9,
                    help="c3: largest step 2^-k_min (steps of 2^-8 or longer miss star-star passages at the "
                         "softening length at this n; see the design notes)")
    ap.add_argument("--c3-precision", default="mixed", choices=["mixed", "fp64", "ds"])
    ap.add_argument("--c3-eta", type=float, default=0.1)
    ap.add_argument("--c3-compare", action="store_true", help="c3: also run without the fused small-block kernel")
    ap.add_argument("--c3-c", type=float, default=0.0, help="c3: also run with 1PN + 2PN + 2.5PN terms at this c")
    ap.add_argument("--micro-n", type=int, default=262144)
    ap.add_argument("--micro-orders", default="6")
    ap.add_argument("--small-n", default="131072,1048576", help="smallstep: particle counts")
    ap.add_argument("--nb-n", type=int, default=1 << 20, help="neighbour: particle count")
    ap.add_argument("--nb-act", default="256,1024,4096,16384", help="neighbour: active-set sizes")
    ap.add_argument("--nb-k", type=int, default=64, help="neighbour: particles inside each sphere")
    ap.add_argument("--nb-max", type=int, default=256, help="neighbour: list capacity per row")
    ap.add_argument("--pn-stars", type=int, default=1 << 18, help="pn: cluster stars")
    ap.add_argument("--pn-c", type=float, default=1.0, help="pn: speed of light in model units")
    ap.add_argument("--pn-t-end", type=float, default=1.0 / 64, help="pn: end time")
    ap.add_argument("--micro-rows", type=int, default=512, help="microbench: active rows checked against the oracle")
    ap.add_argument("--micro-tune-max", type=int, default=65536,
                    help="microbench: autotune the force launch up to this n_act first (0 = untuned defaults)")
    ap.add_argument("--clusters", type=int, default=256)
    ap.add_argument("--batch-per-wg", type=int, default=0, help="work items aimed for per workgroup (0 = default)")
    ap.add_argument("--batch-grid", type=int, default=0, help="persistent force workgroups (0 = resident)")
    ap.add_argument("--batch-itile", type=int, default=0, help="active rows per work item, 64 or 256 (0 = default)")
    ap.add_argument("--warm-time", type=float, default=1.0 / 64, help="batched: integrate to this time first")
    ap.add_argument("--autotune-steps", type=int, default=4,
                    help="batched: steps on which the autotuner times every shape (0 = off)")
    ap.add_argument("--skip-per-cluster", action="store_true", help="batched: skip the one-context-per-cluster run")
    ap.add_argument("--occupancy-steps", type=int, default=20, help="batched: steps whose active counts are tallied")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--order", type=int, default=6)
    ap.add_argument("--level", type=int, default=10, help="shared block level (dt = 2^-level)")
    ap.add_argument("--fp64-steps", type=int, default=None, help="timed FP64 steps (default: --steps)")
    # default shapes: what nbody_autotune selects for this workload on MI355X
    # (fixed here so that the timed kernel is the profiled one); "" = autotune
    ap.add_argument("--force-shape-mixed", default="2,256,16,2",
                    help="ni,block,n_split,jpath of the MIXED force ('' = autotune up to --tune-max)")
    ap.add_argument("--force-shape-fp64", default="2,128,16,1",
                    help="ni,block,n_split,jpath of the FP64 force ('' = autotune up to --tune-max)")
    ap.add_argument("--tune-max", type=int, default=65536,
                    help="autotune the force launch up to this n_act before timing (0 = untuned defaults)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="first copy a buffer of this many MiB on the device (a kernel of known traffic that "
                         "scales the HBM byte counters of a profiling run)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import nbody_ics
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    from paper_1312_1789_amd import abi
    abi.lib()
    if args.calibrate_copy_mib > 0:
        src = torch.ones(args.calibrate_copy_mib << 18, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: %d MiB read + %d MiB written" % (args.calibrate_copy_mib, args.calibrate_copy_mib))
        del src, dst
    if args.workload == "batched":
        run_batched(args)
        return
    if args.workload == "microbench":
        run_microbench(args)
        return
    if args.workload == "smallstep":
        run_smallstep(args)
        return
    if args.workload == "neighbour":
        run_neighbour(args)
        return
    if args.workload == "pn":
        run_pn(args)
        return
    if args.workload == "c2":
        run_c2(args)
        return
    if args.workload == "c3":
        run_c3(args)
        return

    t0 = time.perf_counter()
    model = nbody_ics.king(args.n, 7.0, 13)
    log("workload: King W0=7 n=%d (%.1f s to generate)" % (args.n, time.perf_counter() - t0))

    sims, res = {}, {}
    for prec, k in (("mixed", args.steps), ("fp64", args.fp64_steps or args.steps)):
        fs = args.force_shape_mixed if prec == "mixed" else args.force_shape_fp64
        fs = tuple(int(v) for v in fs.split(",")) if fs else None
        sims[prec], res[prec] = run_precision(model, prec, args.order, k, args.warmup, args.level, args.tune_max, fs)

    n = args.n
    mixed = res["mixed"]
    force_ms = mixed["phase_ms_per_step"]["force"]
    n_act = int(round(mixed["n_act_per_step"]))
    flops_launch = FLOPS_PER_INTERACTION[args.order] * float(n_act) * n
    achieved = flops_launch / (force_ms * 1e-3) / 1e12
    traffic = read_traffic(n_act, n, mixed["used"])
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": traffic,
                "kernel": kernel_name(mixed["used"], args.order),
                "launch": mixed["launch"],
                "flops_per_interaction": FLOPS_PER_INTERACTION[args.order],
                "flops_convention": "minimal operation list without the potential (add/sub/mul 1, FMA 2, rsqrt 1); "
                                    "%d with the potential" % FLOPS_WITH_POT[args.order],
                "force_ms_per_launch": round(force_ms, 3),
                "frac_literature_%d_flops" % FLOPS_LITERATURE[args.order]:
                    round(achieved * FLOPS_LITERATURE[args.order] / FLOPS_PER_INTERACTION[args.order]
                          / PEAK_FP32_TFLOPS, 4)}

    cpu, errors, rows = None, None, 0
    if not args.no_cpu_baseline:
        cpu, errors, rows = cpu_baseline_and_error(model, sims, args.order, args.cpu_seconds)

    fp64 = res["fp64"]
    fp64_force_ms = fp64["phase_ms_per_step"]["force"]
    line = {
        "metric": METRIC,
        "value": mixed["interactions_per_s"],
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mixed["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "King W0=7 cluster, n=%d, 6th-order Hermite block step with all n particles "
                               "active (one shared level k=%d), MIXED pairwise force" % (n, args.level),
                   "n": n, "order": args.order, "precision": "mixed",
                   "accumulation": "double-single position and velocity differences, FP32 pair arithmetic, FP32 "
                                   "partial sums over chunks of 128 j added into FP64 accumulators (the chunked "
                                   "mixed mode)",
                   "n_act": n_act, "eps": 1e-4,
                   "interactions_per_step": float(n_act) * n, "interaction_count": "n_act * n (self pair counted)"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "force_only": {"mixed_interactions_per_s": float(n_act) * n / (force_ms * 1e-3),
                       "fp64_interactions_per_s": float(n_act) * n / (fp64_force_ms * 1e-3),
                       "mixed_over_fp64": fp64_force_ms / force_ms,
                       "mixed_gflops": achieved * 1e3,
                       "mixed_gflops_literature": FLOPS_LITERATURE[args.order] * float(n_act) * n
                       / (force_ms * 1e-3) / 1e9},
        "fp64": {"value": fp64["interactions_per_s"], "ms_per_step": fp64["ms_per_step"],
                 "phase_ms_per_step": fp64["phase_ms_per_step"],
                 "force_launch_used": {"ni": fp64["used"][0], "block": fp64["used"][1], "n_split": fp64["used"][2],
                                       "jpath": fp64["used"][3]},
                 "force_tflops": FLOPS_PER_INTERACTION[args.order] * float(n_act) * n / (fp64_force_ms * 1e-3) / 1e12,
                 "frac_of_fp64_peak": FLOPS_PER_INTERACTION[args.order] * float(n_act) * n
                 / (fp64_force_ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS},
        "phase_ms_per_step": mixed["phase_ms_per_step"],
        "error_vs_oracle": errors,
        "error_rows": rows,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
