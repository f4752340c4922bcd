"""Benchmark: ECMC events/s on one MI355X for hard disks, N = 2^20, eta = 0.708.

One step = one leg (breakpoint interval) of the whole hot path: home-cell build,
1024 chains running the event kernel to the breakpoint (restarts included),
breakpoint reduction and write-back.  Directions alternate +x/+y.  Inputs are
seeded synthetic lattices resident in HBM before the timed region starts.

The headline value is measured after an untimed, labelled burn-in of at least
50 liftings per disk.  The lattice start is a transient: its first legs run
faster, and the rate settles after about 40 liftings per disk.  The figure
from the lattice (warm-up legs only) is reported beside it.

Prints ONE JSON line.  Besides the headline it carries both forms, the other
workloads (256, 4096 and 65536 disks), the violation probability per
breakpoint against the generalized birthday estimate (Sec. 3.4) over a sweep
of leg lengths, the roofline of the event kernel with the measured gather and
latency bounds, the replica batch, and the oracle timed on the host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, published
# Algorithmic bytes per lifting: what the method has to move, per lifting, with
# about 7.5 cells of 0.9 disks scanned: per scanned cell 4 B of cell header
# plus 20 B per disk record (binary64 a, p, id) or 8 B (binary32 cell-relative
# offsets); 3 local-time reads of the horizon set 24 B, claim 8 B, target
# re-read 16 B, commit writes 32 B, tag release 4 B, log 4 B; FP32-mixed adds
# the winner's id 4 B and its binary64 refinement 16 B.
ALG_BYTES_PER_EVENT = {"fp64": 250.0, "fp32": 190.0}
# The same at 64-byte line granularity (rows of cells padded to lines, about 8
# further scattered lines per lifting).
LINE_BYTES_PER_EVENT = {"fp64": 1500.0, "fp32": 1050.0}
# Bytes this implementation moves (reported separately): per scanned slot the
# fixed record (p, id; 16 B) and the mutable record (a, t; 16 B); per lifting
# next-event time 8, reservation 8, activation-record invalidation 8, claim 4,
# target re-read 16, lane-minima re-read 48, reservation read 8, undo record
# 60, commit 24, activation record 36, reservation release 8, tag release 4,
# log 4: 236 B.
IMPL_BYTES_PER_SLOT = 32
IMPL_BYTES_PER_EVENT = 236
# the scanned working set of the 2^20-disk workload: fixed and mutable slot
# records and tags of 1078^2 cells x 4 slots
WORKING_SET_BYTES = 1078 * 1078 * 4 * (16 + 16 + 4)
PAPER_CONTEXT = {
    "x86": "Alg. 6 (C++/OpenMP, constraint graph G256, k=80, N=65536, eta=0.708, runs continue through "
           "horizon violations): ~1.7e12 events/hour (~4.7e8 events/s) at 40 threads on one Intel Xeon "
           "Gold 6230 (20 cores, 2.1-3.9 GHz); x12 over 1 thread at 20 threads, x16 at 40",
    "arm": "NVIDIA Jetson (ARM Cortex-A57, 4 cores, 1.43 GHz): x4.0 at 4 threads, about 7x below x86 "
           "at a comparable thread count",
    "cell_serial": "cell-based serial production code: ~3e10 events/hour (~8.3e6 events/s)",
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _src_hash():
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_2004_11040_amd", "csrc", "ecmc_kernels.hip"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def pmc_summary_path(form):
    return os.path.join(ROOT, "profiles", f"event_kernel_N1048576_{form}_pmc.json")


def _pmc(form):
    try:
        with open(pmc_summary_path(form)) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("source_sha256_16") != _src_hash():
        return None
    return d


def _traffic(form, events_per_launch):
    """HBM bytes per event-kernel launch: the bytes per lifting measured by the
    committed rocprofv3 counter summary (FETCH_SIZE + WRITE_SIZE, calibrated on
    a copy of known size) times this run's liftings per launch.  None if the
    summary is missing or was taken on another kernel source."""
    d = _pmc(form)
    if not d or not d.get("hbm_bytes_per_event"):
        return None
    return d["hbm_bytes_per_event"] * events_per_launch


# ---------------------------------------------------------------------------
# the oracle on the host (runs before anything touches the GPU)
# ---------------------------------------------------------------------------
def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(seconds: float):
    """The oracle, as it stands, on a bounded sample of the headline workload,
    pinned to one host core."""
    import oracle
    import workloads as W
    avail = sorted(os.sched_getaffinity(0))
    os.sched_setaffinity(0, {avail[0]})
    try:
        s = W.config(4)
        x, y, act = s.x, s.y, s.active
        events, t_used, legs = 0, 0.0, 0
        while t_used < seconds and legs < 8:
            t0 = time.perf_counter()
            r = oracle.run(x, y, s.sigma, s.L, act, [legs % 2], s.T, log=False)
            t_used += time.perf_counter() - t0
            log(f"cpu baseline: leg {legs} done, {t_used:.1f} s")
            events += r.n_events
            x, y, act = r.x, r.y, r.active
            legs += 1
    finally:
        os.sched_setaffinity(0, set(avail))
    return {"value": events / t_used, "unit": "events/s", "cores": 1, "kind": "oracle",
            "sample": f"first {legs} legs ({events} liftings) of the N=1048576 eta=0.708 k=1024 "
                      f"workload from the lattice, serial C global-time event queue, pinned to one core",
            "cpu_model": _cpu_model(), "host_cores": os.cpu_count(), "cores_available": len(avail)}


def _oracle_replica(args):
    import oracle
    x, y, L, act, T, target = args
    t0 = time.perf_counter()
    ev, leg = 0, 0
    while ev < target:
        r = oracle.run(x, y, 1.0, L, act, [leg % 2], T, log=False)
        ev += r.n_events
        x, y, act = r.x, r.y, r.active
        leg += 1
    return ev, time.perf_counter() - t0


def cpu_baseline_batch(n_rep, per_replica, max_procs=16):
    """The oracle on the replica workload on all usable host cores (one
    process per core, replicas handed out one at a time)."""
    import multiprocessing as mp

    import workloads as W
    reps = W.replica_batch(n_rep)
    tasks = [(s.x, s.y, s.L, s.active, s.T, per_replica) for s in reps]
    procs = max(1, min(max_procs, len(os.sched_getaffinity(0))))
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(procs) as pool:
        res = pool.map(_oracle_replica, tasks, chunksize=1)
    wall = time.perf_counter() - t0
    ev = sum(r[0] for r in res)
    log(f"cpu baseline batch: {ev} liftings on {procs} processes in {wall:.1f} s")
    return {"value": ev / wall, "unit": "events/s", "cores": procs, "kind": "oracle",
            "sample": f"{n_rep} replicas, whole legs until >= {per_replica} liftings each, "
                      f"one process per core", "cpu_model": _cpu_model()}


# ---------------------------------------------------------------------------
# GPU measurements
# ---------------------------------------------------------------------------
def _stats_delta(st0, st1):
    d = {k: st1[k] - st0[k] for k in st1 if isinstance(st1[k], (int, float))}
    d["violations_by_kind"] = [b - a for a, b in zip(st0["violations_by_kind"], st1["violations_by_kind"])]
    return d


NEIGHBOURS = {"cells": 0, "graph": 1}
_neighbours = "graph"
_cooperative = False
_clock_period_ns = 0   # pacing of the clock workgroup for the headline context (set from the command line)


def _make(s, form, lanes, window_micro, log_cap=1 << 12, max_splits=0, neighbours=None, clock_period_ns=0):
    import numpy as np

    import paper_2004_11040_amd as pkg
    flags = pkg.FP32_MIXED if form == "fp32" else pkg.FP64
    e = pkg.Ecmc(np.stack([s.x, s.y], 1), s.sigma, s.L, flags=flags, max_chains=s.k, log_cap=log_cap)
    e.set_option(pkg.OPT_LANES, lanes)
    e.set_option(pkg.OPT_KERNEL_TIMING, 1)
    e.set_option(pkg.OPT_WINDOW_MICRO, window_micro)
    e.set_option(pkg.OPT_NEIGHBOURS, NEIGHBOURS[neighbours or _neighbours])
    e.set_option(pkg.OPT_COOPERATIVE, 1 if _cooperative else 0)
    e.set_option(pkg.OPT_CLOCK_PERIOD_NS, clock_period_ns)
    if max_splits:
        e.set_option(pkg.OPT_MAX_SPLITS, max_splits)
    e.set_active(s.active)
    return e


def timed_legs(e, s, n_legs=None, target_events=None, label="", chunk=10):
    """Run whole legs (alternating when the workload alternates) in one timed
    region: n_legs of them, or until target_events more liftings."""
    import torch

    import paper_2004_11040_amd as pkg
    direction = pkg.DIR_ALTERNATE if s.alternate else pkg.DIR_X
    st0 = e.stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    legs, ev0 = 0, st0["events"]
    while True:
        if n_legs is not None and legs >= n_legs:
            break
        n = chunk if n_legs is None else min(chunk, n_legs - legs)
        e.run(n * s.T, s.T, direction)
        legs += n
        if target_events is not None:
            if e.stats()["events"] - ev0 >= target_events:
                break
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st1 = e.stats()
    d = _stats_delta(st0, st1)
    log(f"{label}: {legs} legs, {d['events']} liftings, {d['events'] / wall / 1e6:.2f} M/s")
    return d, wall


def _summary(d, wall, form):
    launches = max(d["event_launches"], 1)
    kdur = d["event_kernel_ms"] / launches / 1e3
    epl = d["timed_events"] / launches
    alg = ALG_BYTES_PER_EVENT[form] * epl
    impl = (d["timed_slots"] * IMPL_BYTES_PER_SLOT + d["timed_events"] * IMPL_BYTES_PER_EVENT) / launches
    return {
        "events": d["events"], "wall_s": wall, "events_per_s": d["events"] / wall,
        "legs": d["legs"], "legs_violated": d["legs_violated"], "reruns": d["reruns"],
        "global_legs": d["global_legs"], "lockstep_runs": d["lockstep_runs"],
        "violations_screened": d["violations_screened"], "claim_yields": d["claim_yields"],
        "spin_aborts": d["spin_aborts"], "violations_by_kind": d["violations_by_kind"],
        "nonresident_launches": d["nonresident_launches"],
        "attempts": d["attempts"], "slots_per_event": d["slots_scanned"] / max(d["events"], 1),
        "events_per_launch": epl, "kernel_ms_avg": kdur * 1e3,
        "alg_bytes_per_launch": alg, "implementation_bytes_per_launch": impl,
        "achieved_gbs": alg / kdur / 1e9 if kdur > 0 else 0.0,
        "kernel_time_frac": d["event_kernel_ms"] / 1e3 / wall if wall > 0 else 0.0,
        "pressure_raw": 1.0 + d["sum_b"] / d["chain_time"] if d["chain_time"] else None,
        "violation_probability_per_breakpoint": d["legs_violated"] / max(d["legs"], 1),
    }


BURN_IN_PER_DISK = 50.0


def burn_in(e, s, per_disk=BURN_IN_PER_DISK):
    """Untimed legs until at least per_disk liftings per disk since set-up."""
    import paper_2004_11040_amd as pkg
    direction = pkg.DIR_ALTERNATE if s.alternate else pkg.DIR_X
    legs = 0
    while e.stats()["events"] < per_disk * s.n:
        e.run(10 * s.T, s.T, direction)
        legs += 10
    return legs


def production_loop(e, s, n_legs, seed=11):
    """Legs whose direction is drawn per leg, uniformly over +x, +y, -x, -y
    (seeded), with the constraint graph rebuilt for every leg: the production
    loop of the closing paragraph of Sec. 3.4."""
    import numpy as np
    import torch
    dirs = np.random.Generator(np.random.PCG64(seed)).integers(0, 4, n_legs).astype(np.int32)
    st0 = e.stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(0, n_legs, 10):
        e.run_directions(s.T, dirs[i:i + 10])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    d = _stats_delta(st0, e.stats())
    log(f"production loop: {n_legs} legs, {d['events']} liftings, {d['events'] / wall / 1e6:.2f} M/s")
    return {"legs": n_legs, "directions": "drawn per leg, uniform over +x +y -x -y (PCG64 seed 11)",
            "events": d["events"], "wall_s": wall, "events_per_s": d["events"] / wall,
            "reruns": d["reruns"], "legs_violated": d["legs_violated"]}


def violation_sweep(e, s, Ts, n_legs, window_micro):
    """Violation probability per breakpoint (legs whose first attempt saw a
    horizon violation / legs) for each leg length T, with the same bounded lag
    at every size so that the sizes compare (and the clock unpaced at every
    size)."""
    import paper_2004_11040_amd as pkg
    e.set_option(pkg.OPT_WINDOW_MICRO, window_micro)
    e.set_option(pkg.OPT_CLOCK_PERIOD_NS, 0)
    out = {}
    direction = pkg.DIR_ALTERNATE if s.alternate else pkg.DIR_X
    for T in Ts:
        st0 = e.stats()
        e.run(n_legs * T, T, direction)
        st1 = e.stats()
        out[f"{T:g}"] = (st1["legs_violated"] - st0["legs_violated"]) / max(st1["legs"] - st0["legs"], 1)
    return out


LATTICE_LEGS = 20      # timed legs from the lattice (the transient, reported beside the headline)
PRODUCTION_LEGS = 20   # legs of the production loop (directions drawn per leg)


def run_form(form, steps, warmup, lanes, window_micro, max_splits=0, sweep_Ts=(), sweep_legs=40, neighbours=None,
             clock_period_ns=0):
    """The headline workload in one form: `warmup` untimed legs and
    LATTICE_LEGS timed legs from the lattice, then a burn-in to >= 50
    liftings per disk and `steps` timed legs (the headline), then the
    production loop and the violation sweep."""
    import workloads as W
    s = W.config(4)
    e = _make(s, form, lanes, window_micro, max_splits=max_splits, neighbours=neighbours,
              clock_period_ns=clock_period_ns)
    if warmup:
        e.run(warmup * s.T, s.T, 4)
    d0, w0 = timed_legs(e, s, n_legs=LATTICE_LEGS, label=f"{form} from the lattice")
    bl = burn_in(e, s)
    d1, w1 = timed_legs(e, s, n_legs=steps, label=f"{form} after burn-in")
    res = _summary(d1, w1, form)
    res["timed_legs"] = steps
    res["burn_in_legs"] = bl + warmup + LATTICE_LEGS
    res["liftings_per_disk_before_timing"] = (e.stats()["events"] - d1["events"]) / s.n
    res["from_lattice"] = _summary(d0, w0, form)
    res["neighbours"] = neighbours or _neighbours
    res["window_sigma"] = window_micro * 1e-6
    res["clock_period_ns"] = clock_period_ns
    if form == "fp64" and (neighbours or _neighbours) == "graph":
        res["production_loop"] = production_loop(e, s, PRODUCTION_LEGS)
    res["overlaps"] = e.overlaps()
    if sweep_Ts:
        res["violation_sweep"] = violation_sweep(e, s, sweep_Ts, sweep_legs, window_micro)
    e.close()
    return res


def run_small_configs(lanes, sweep_Ts, sweep_legs, window_micro):
    """The 256-disk (FP64, +x, 1e5 liftings) and 4096-disk (FP64, alternating,
    1e7 liftings, violation rate per breakpoint) workloads."""
    import workloads as W
    out = {}
    s = W.config(0)
    e = _make(s, "fp64", lanes, 0)
    d, w = timed_legs(e, s, target_events=s.target_events, label="N=256", chunk=50)
    out["N256"] = {"workload": "N=256 eta=0.60 square lattice, k=4, +x, T=0.5 L, FP64",
                   **_summary(d, w, "fp64"), "overlaps": e.overlaps()}
    e.close()
    s = W.config(1)
    # k = sqrt(N) chains need the bounded lag (free-running: ~9x the rollbacks);
    # the 256-disk workload's 4 chains rarely meet and run free
    e = _make(s, "fp64", lanes, window_micro)
    d, w = timed_legs(e, s, target_events=s.target_events, label="N=4096", chunk=50)
    r = {"workload": "N=4096 eta=0.70 centred-rectangular lattice, k=64, alternating +x/+y, T=0.25 L, FP64, "
                     f"bounded lag {window_micro * 1e-6:g} sigma",
         **_summary(d, w, "fp64"), "overlaps": e.overlaps()}
    if sweep_Ts:
        r["violation_sweep"] = violation_sweep(e, s, sweep_Ts, sweep_legs, window_micro)
    out["N4096"] = r
    e.close()
    return out


def run_precision_config(lanes, window_micro, target, prefix_events, sweep_Ts, sweep_legs):
    """The 65536-disk workload in both forms: the error of each form against
    the binary64 oracle over the legs that cover the first prefix_events
    liftings, then timed legs up to `target` liftings, and the pressure.
    FP32-mixed runs on the corridor scan, where its binary32 filter acts (the
    graph path has no binary32 stage), beside FP64 on the same scan (a tenth
    of the liftings) and FP64 on graph candidates (the default)."""
    import numpy as np

    import oracle
    import workloads as W
    s = W.config(2)
    out = {"workload": "N=65536 eta=0.708 centred-rectangular lattice, k=256, alternating +x/+y, T=33.896"}
    # the oracle over the prefix
    t0 = time.perf_counter()
    legs, ref_ev = 0, 0
    while ref_ev < prefix_events:
        legs += 1
        ref = oracle.run(s.x, s.y, s.sigma, s.L, s.active, s.leg_dirs(legs), s.T, log_cap=1 << 23)
        ref_ev = ref.n_events
    log(f"N=65536 oracle prefix: {legs} legs, {ref_ev} liftings, {time.perf_counter() - t0:.1f} s")
    for key, form, nb, tgt in (("fp64", "fp64", "graph", target), ("fp32", "fp32", "cells", target),
                               ("fp64_cells", "fp64", "cells", max(target // 10, prefix_events))):
        e = _make(s, form, lanes, window_micro, log_cap=1 << 14, neighbours=nb)
        e.run(legs * s.T, s.T, 4)
        pos = e.positions()
        dx = np.abs((pos[:, 0] - ref.x + s.L / 2) % s.L - s.L / 2).max()
        dy = np.abs((pos[:, 1] - ref.y + s.L / 2) % s.L - s.L / 2).max()
        bad_chains = sum(not np.array_equal(e.log(c).targets, ref.targets(c)) for c in range(s.k))
        sb, _ = e.chain_sums()
        err = {"legs": legs, "liftings": int(e.stats()["events"]), "oracle_liftings": int(ref_ev),
               "chains_with_other_targets": int(bad_chains),
               "max_abs_position_error": float(max(dx, dy)),
               "max_abs_local_time_error": float(np.abs(e.stamps() - ref.stamps).max()),
               "max_abs_sum_b_error": float(np.abs(sb - ref.sum_b).max()),
               "active_set_equal": bool(np.array_equal(e.active(), ref.active))}
        d, w = timed_legs(e, s, target_events=tgt, label=f"N=65536 {key}", chunk=20)
        r = {"error_vs_fp64_oracle": err, **_summary(d, w, form), "neighbours": nb, "overlaps": e.overlaps()}
        if key == "fp64" and sweep_Ts:
            r["violation_sweep"] = violation_sweep(e, s, sweep_Ts, sweep_legs, window_micro)
        out[key] = r
        e.close()
    out["fp32_over_fp64"] = out["fp32"]["events_per_s"] / out["fp64_cells"]["events_per_s"]
    out["fp32_over_fp64_default"] = out["fp32"]["events_per_s"] / out["fp64"]["events_per_s"]
    return out


def birthday(sweeps):
    """Generalized birthday estimate (Sec. 3.4): p = 1 - exp(-k^2 / (2 N')),
    with N' = N / alpha cells of constant area; alpha fitted per leg length on
    the 4096-disk workload, then predicted for the larger ones."""
    fit_n, fit_k = 4096, 64
    out = {"model": "p = 1 - exp(-alpha k^2 / (2 N)), alpha fitted at N=4096, k=64; every size with "
                    "the headline's bounded lag, after >= 1000 liftings per disk (N=4096, 65536) or "
                    "the burn-in (N=2^20)", "by_T": {}}
    for T, p1 in sweeps["N4096"].items():
        n_legs = sweeps["legs"]
        pc = min(max(p1, 0.5 / n_legs), 1.0 - 0.5 / n_legs)
        alpha = -2.0 * fit_n * math.log(1.0 - pc) / (fit_k * fit_k)
        row = {"alpha": alpha, "alpha_is_bound": p1 in (0.0, 1.0), "N4096_measured": p1}
        for name, n, k in (("N65536", 65536, 256), ("N1048576", 1 << 20, 1024)):
            if T in sweeps.get(name, {}):
                row[f"{name}_measured"] = sweeps[name][T]
                row[f"{name}_predicted"] = 1.0 - math.exp(-alpha * k * k / (2.0 * n))
        out["by_T"][T] = row
    return out


def run_probes(k):
    """Dependent-load latency and random-line gather bandwidth over a buffer of
    the headline working-set size (and of 2 GiB, beyond the Infinity Cache)."""
    import numpy as np
    import torch

    import paper_2004_11040_amd as pkg
    out = {}
    for name, nbytes in (("working_set", WORKING_SET_BYTES), ("2GiB", 2 << 30)):
        n_lines = nbytes // 64
        rng = np.random.Generator(np.random.PCG64(7))
        perm = rng.permutation(n_lines).astype(np.uint32)
        nxt = np.empty(n_lines, np.uint32)
        nxt[perm] = np.roll(perm, -1)          # one cycle through every line
        host = np.zeros((n_lines, 16), np.uint32)
        host[:, 0] = nxt
        buf = torch.from_numpy(host.reshape(-1)).to("cuda")
        del host
        r = {"bytes": int(n_lines * 64)}
        for scope, tag in ((1, "agent_scope"), (0, "plain")):
            r[f"chase_ns_{tag}"] = pkg.probe_chase(buf, 200_000, scope)
            r[f"gather_gbs_{tag}"] = pkg.probe_gather(buf, 2048, 256, scope)
        out[name] = r
        del buf
        torch.cuda.empty_cache()
    lat = out["working_set"]["chase_ns_agent_scope"] * 1e-9
    out["littles_law_events_per_s"] = k / (3.0 * lat)
    log(f"probes: latency {lat * 1e9:.0f} ns, gather {out['working_set']['gather_gbs_agent_scope']:.0f} GB/s")
    return out


def run_batch(n_rep, target, t_frac, graph=1, window_micro=0, max_splits=0, form="fp64", neighbours="graph",
              clock_period_ns=0):
    """The replica workload: n_rep seeded replicas of N in {1024..16384}, eta in
    [0.60, 0.72], k = round(sqrt N), run in one persistent launch (captured in
    a hipGraph) until every replica has `target` liftings; the autotuner's legs
    come first and are not timed.  With graph candidates every time of flight
    is binary64 (form fp64); FP32-mixed acts on the corridor scan."""
    import numpy as np
    import torch

    import paper_2004_11040_amd as pkg
    import workloads as W
    reps = W.replica_batch(n_rep)
    systems = []
    for s in reps:
        e = pkg.Ecmc(np.stack([s.x, s.y], 1), s.sigma, s.L, flags=pkg.FP32_MIXED if form == "fp32" else pkg.FP64,
                     max_chains=s.k, log_cap=1 << 8)
        e.set_active(s.active)
        systems.append(e)
    b = pkg.Batch(systems)
    b.set_option(pkg.OPT_GRAPH, graph)
    b.set_option(pkg.OPT_NEIGHBOURS, NEIGHBOURS[neighbours])
    b.set_option(pkg.OPT_WINDOW_MICRO, window_micro)
    b.set_option(pkg.OPT_CLOCK_PERIOD_NS, clock_period_ns)
    if max_splits:
        b.set_option(pkg.OPT_MAX_SPLITS, max_splits)
    T = [t_frac * s.L for s in reps]
    big = np.full(n_rep, 1 << 60, np.int64)
    # two untimed legs at fixed settings first, so that no tuning candidate
    # runs the fast first legs of the lattice
    b.set_option(pkg.OPT_LANES, 4)
    b.set_option(pkg.OPT_CELL_PCT, 100)
    b.run(big, T, pkg.DIR_ALTERNATE, max_legs=2)
    b.set_option(pkg.OPT_LANES, 0)
    b.set_option(pkg.OPT_CELL_PCT, 0)
    b.run(big, T, pkg.DIR_ALTERNATE, max_legs=1)  # autotune (one leg per candidate)
    tune = b.info()
    ev0 = sum(e.stats()["events"] for e in systems)
    ov0 = sum(e.stats()["overflow_legs"] for e in systems)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.run(np.full(n_rep, target, np.int64), T, pkg.DIR_ALTERNATE, max_legs=0)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    info = b.info()
    ev1 = sum(e.stats()["events"] for e in systems)
    ov1 = sum(e.stats()["overflow_legs"] for e in systems)
    log(f"batch: {ev1 - ev0} liftings in {wall:.2f} s, {ov1 - ov0} legs replayed after an undo overflow")
    overlaps = sum(e.overlaps() for e in systems)
    out = {"workload": f"{n_rep} replicas, N in 64*[16,256], eta in [0.60,0.72], k=round(sqrt N), "
                       f"legs of {t_frac} L alternating +x/+y, {form} with {neighbours} candidates, "
                       f"{target} liftings per replica, "
                       f"bounded lag {window_micro * 1e-6:g} sigma, H recomputed at most every "
                       f"{clock_period_ns} ns",
           "events": ev1 - ev0, "wall_s": wall, "events_per_s": (ev1 - ev0) / wall,
           "device_ms": info["device_ms"], "lanes": info["lanes"], "graph": info["graph"],
           "workgroups": info["workgroups"], "legs": info["legs"], "rollbacks": info["rollbacks"],
           "global_runs": info["global_runs"],
           # legs replayed whole in global-time order: a chain outran its
           # undo records (4096) after the last settled time, then a race
           "overflow_replays": ov1 - ov0,
           "rollbacks_per_replica_leg": info["rollbacks"] / max(info["legs"], 1),
           "global_runs_per_replica_leg": info["global_runs"] / max(info["legs"], 1),
           # per-leg counts grow with the leg length; per lifting they do not
           "rollbacks_per_1000_liftings": 1000.0 * info["rollbacks"] / max(ev1 - ev0, 1),
           "global_runs_per_1000_liftings": 1000.0 * info["global_runs"] / max(ev1 - ev0, 1),
           "autotune_events_per_ms_by_lane_cap": dict(zip(("4", "8", "16", "32"), tune["tune_events_per_ms"])),
           "autotune_events_per_ms_by_cell_pct": dict(zip(("100", "115", "130", "141"),
                                                          tune["tune_cell_events_per_ms"])),
           "cell_pct": info["cell_pct"],
           "replica_ms_max": info["replica_ms_max"],
           "load_balance": info["replica_ms_sum"] / max(info["workgroups"] * info["device_ms"], 1e-9),
           "overlaps": overlaps, "total_disks": int(sum(s.n for s in reps)),
           "total_chains": int(sum(s.k for s in reps))}
    b.close()
    for e in systems:
        e.close()
    return out


def save_state(path, lanes, window_micro):
    """Burn the headline workload in (>= 50 liftings per disk) and save the
    configuration, so that a profiled process can start from it and count
    only the legs it measures."""
    import numpy as np

    import workloads as W
    s = W.config(4)
    e = _make(s, "fp64", lanes, window_micro, clock_period_ns=_clock_period_ns)
    legs = burn_in(e, s)
    np.savez(path, x=e.positions()[:, 0], y=e.positions()[:, 1], active=e.active(), legs=legs,
             liftings=e.stats()["events"])
    log(f"saved the state after {legs} burn-in legs to {path}")


def profile_run(legs, lanes, window_micro, form, state=None):
    """Short run for hardware counters and kernel traces: `legs` legs of the
    headline workload (from a state saved by --save-state, else from the
    lattice), then a device copy of 256 MiB (read 256 MiB, write 256 MiB)
    whose counter readings calibrate the bytes the counters report."""
    import numpy as np
    import torch

    import workloads as W
    s = W.config(4)
    if state:  # saved after an even number of legs: the next one is +x
        z = np.load(state)
        s.x, s.y, s.active = z["x"], z["y"], z["active"].astype(np.int32)
        assert int(z["legs"]) % 2 == 0
    e = _make(s, form, lanes, window_micro, clock_period_ns=_clock_period_ns if _neighbours == "graph" else 0)
    st0 = e.stats()
    e.run(legs * s.T, s.T, 4)
    d = _stats_delta(st0, e.stats())
    print(json.dumps({"profile_run": True, "form": form, "lanes": lanes, "legs": legs,
                      "neighbours": _neighbours, "from_state": bool(state),
                      "events": d["events"], "attempts": d["attempts"],
                      "event_launches": d["event_launches"], "timed_events": d["timed_events"],
                      "slots_scanned": d["slots_scanned"]}), flush=True)
    a = torch.ones(256 << 20, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()


def _pmc_values(path, counter):
    """Per-dispatch values of one counter from a rocprofv3 counter_collection
    CSV: list of (dispatch id, kernel name, value)."""
    import csv
    out = []
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            if row.get("Counter_Name") == counter:
                out.append((int(row.get("Dispatch_Id", 0) or 0), row.get("Kernel_Name", ""),
                            float(row["Counter_Value"])))
    return out


DERIVED_PCT = ("VALUBusy", "VALUUtilization", "OccupancyPercent")


def trace_summary(trace_csv, bench_json, out_txt, command):
    """Kernel statistics of a rocprofv3 kernel trace of a bench run, as text,
    beside the bench's own device-timed mean duration of the event kernel per
    form.  Event launches enqueued past the end of a leg return at once; the
    launches that ran an attempt are told apart by their duration (over
    RAN_US, a few times the empty launch's)."""
    import csv
    ran_us = 10.0
    stats = {}
    with open(trace_csv, newline="") as f:
        for row in csv.DictReader(f):
            name = row["Kernel_Name"]
            dur = (int(row["End_Timestamp"]) - int(row["Start_Timestamp"])) * 1e-3  # us
            st = stats.setdefault(name, [0, 0.0, 0, 0.0])
            st[0] += 1
            st[1] += dur
            if dur > ran_us:
                st[2] += 1
                st[3] += dur
    with open(bench_json) as f:
        line = json.loads(next(ln for ln in f if ln.startswith("{")))
    total = sum(v[1] for v in stats.values())

    def short(n):
        n = n.replace("(anonymous namespace)::", "")
        return n.split("(")[0] if not n.startswith("void ") else n[5:].split("(")[0]

    out = ["# rocprofv3 kernel statistics of a bench run (one MI355X)", "#",
           "# command (from /tmp with TMPDIR=/tmp; <repo> = the repository root):"]
    out += [f"#   {c}" for c in command]
    out += [f"# source: paper_2004_11040_amd/csrc/ecmc_kernels.hip sha256[:16] = {_src_hash()}",
            f"# bench line: value {line['value'] / 1e6:.2f} M liftings/s ({line['config']['form']}, "
            f"{line['config']['neighbours']}), lag {line['config']['window_sigma']:g} sigma, clock period "
            f"{line['config'].get('clock_period_ns', 0)} ns", "",
            f"{'kernel':58s} {'calls':>7s} {'total_ms':>10s} {'avg_us':>9s} {'pct':>6s}  {'ran':>6s} {'avg_us_ran':>10s}"]
    for name, (n, tot, nr, tr) in sorted(stats.items(), key=lambda kv: -kv[1][1])[:24]:
        out.append(f"{short(name)[:58]:58s} {n:7d} {tot / 1e3:10.3f} {tot / n:9.2f} {100 * tot / total:6.2f}"
                   f"  {nr:6d} {(tr / nr if nr else 0.0):10.2f}")
    out += ["", "# event kernel: mean duration of the launches that ran an attempt",
            "#   rocprofv3 (duration > 10 us) against the bench's device timing (s_memrealtime, first",
            "#   workgroup start to last workgroup end)"]
    tags = {"k_event<64, false, true>": "graph", "k_event<64, true, false>": "cells fp32",
            "k_event<64, false, false>": "cells fp64"}
    for kname, tag in tags.items():
        hits = [v for n, v in stats.items() if short(n).replace(" ", "") == kname.replace(" ", "")]
        if not hits:
            continue
        n, tot, nr, tr = hits[0]
        out.append(f"  {kname:28s} rocprofv3 {tr / max(nr, 1):8.1f} us over {nr} launches")
    for key, r in line.get("forms", {}).items():
        out.append(f"  bench form {key:12s} ({r.get('neighbours')}): {r['kernel_ms_avg'] * 1e3:8.1f} us per launch, "
                   f"{r['events_per_launch']:.0f} liftings per launch, {r['events_per_s'] / 1e6:.2f} M liftings/s")
    with open(out_txt, "w") as f:
        f.write("\n".join(out) + "\n")
    print("\n".join(out))


def pmc_summary(fetch_csv, write_csv, profile_log, extra_csvs=()):
    """Turn the counter runs of --profile-run (FETCH_SIZE, then WRITE_SIZE, and
    optionally L2 hit/miss and VALU counters) into the committed summary.
    Only the event-kernel dispatches after the burn-in count: the last
    `event_launches` dispatches that did work, plus the rounds that returned
    at once, are taken as the dispatches after the burn-in's."""
    copy_bytes = 256 << 20
    with open(profile_log) as f:
        run = next(json.loads(line) for line in f if line.startswith("{") and "profile_run" in line)

    def event_vals(csv_path, counter):
        vals = [(i, v) for i, n, v in _pmc_values(csv_path, counter) if "k_event" in n]
        vals.sort()
        return vals

    def copy_val(csv_path, counter):
        return max(v for _, n, v in _pmc_values(csv_path, counter)
                   if "copy" in n.lower() or "elementwise" in n.lower())

    fe, wr = event_vals(fetch_csv, "FETCH_SIZE"), event_vals(write_csv, "WRITE_SIZE")
    cp_f, cp_w = copy_val(fetch_csv, "FETCH_SIZE"), copy_val(write_csv, "WRITE_SIZE")
    f_cal = copy_bytes / (cp_f * 1024.0)  # counters are in KiB
    w_cal = copy_bytes / (cp_w * 1024.0)
    launches = max(run["event_launches"], 1)
    events_per_launch = run["timed_events"] / launches
    # every event-kernel dispatch of the process belongs to the profiled legs
    # (rounds enqueued past the end of a leg return at once and add little)
    tail_f, tail_w = fe, wr
    total = sum(v for _, v in tail_f) * 1024.0 * f_cal + sum(v for _, v in tail_w) * 1024.0 * w_cal
    per_launch = total / launches
    form = run.get("form", "fp64")
    d = {"source_sha256_16": _src_hash(), "form": form, "neighbours": run.get("neighbours"),
         "from_state": run.get("from_state"),
         "kernel": f"k_event<{run.get('lanes', 64)}, {form}, {run.get('neighbours')}>",
         "dispatches_counted": len(tail_f), "copy_fetch_kib": cp_f, "copy_write_kib": cp_w,
         "fetch_calibration": f_cal, "write_calibration": w_cal,
         "launches_that_ran": run["event_launches"], "liftings": run["timed_events"],
         "hbm_bytes_per_launch": per_launch, "events_per_launch": events_per_launch,
         "hbm_bytes_per_event": per_launch / events_per_launch if events_per_launch else None,
         "write_bytes_per_event": (sum(v for _, v in tail_w) * 1024.0 * w_cal / max(run["timed_events"], 1))}
    for path in extra_csvs:
        import csv
        with open(path, newline="") as f:
            names = sorted({row["Counter_Name"] for row in csv.DictReader(f)})
        weight = dict(event_vals(path, "GRBM_GUI_ACTIVE")) if "GRBM_GUI_ACTIVE" in names else None
        for c in names:
            vals = event_vals(path, c)
            if c in DERIVED_PCT and weight:
                # a percentage per dispatch: weighted by the dispatch's active cycles
                wsum = sum(weight.get(i, 0.0) for i, _ in vals)
                d[c] = sum(v * weight.get(i, 0.0) for i, v in vals) / wsum if wsum else None
            else:
                # other runs enqueue other numbers of rounds: sums, not per-launch values
                d[f"{c}_sum"] = sum(v for _, v in vals)
        if "TCC_HIT_sum" in names and "TCC_MISS_sum" in names:
            hit = sum(v for _, v in event_vals(path, "TCC_HIT_sum"))
            miss = sum(v for _, v in event_vals(path, "TCC_MISS_sum"))
            d["L2_hit_rate"] = hit / (hit + miss) if hit + miss else None
    with open(pmc_summary_path(form), "w") as f:
        json.dump(d, f, indent=1)
    print(json.dumps(d))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--profile-run", type=int, default=0, metavar="LEGS",
                    help="only run LEGS legs and a 256 MiB copy (for rocprofv3 counters and traces)")
    ap.add_argument("--save-state", metavar="NPZ", help="burn the headline workload in and save it")
    ap.add_argument("--load-state", metavar="NPZ", help="--profile-run starts from a saved state")
    ap.add_argument("--trace-summary", nargs="+", metavar="ARG",
                    help="TRACE_CSV BENCH_JSON OUT_TXT COMMAND...: text summary of a kernel trace")
    ap.add_argument("--pmc-summary", nargs="+", metavar="CSV",
                    help="FETCH_CSV WRITE_CSV PROFILE_LOG [EXTRA_CSV ...]: write the counter summary")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4800,
                    help="timed legs of the headline form after the burn-in (4800: just over 1e9 liftings "
                         "at N=2^20, the workload's budget per form)")
    ap.add_argument("--warmup", type=int, default=5, help="untimed legs before the lattice timing")
    ap.add_argument("--form", choices=["fp64", "fp32", "both"], default="both")
    ap.add_argument("--lanes", type=int, default=64)
    ap.add_argument("--max-splits", type=int, default=0,
                    help="rollbacks without progress before a lockstep stretch (0: library default)")
    ap.add_argument("--window-micro", type=int, default=200_000,
                    help="bounded lag between chains, in 1e-6 sigma (0: free running), for the headline "
                         "form and the smaller workloads")
    ap.add_argument("--clock-period-ns", type=int, default=4000,
                    help="least time between two passes of the clock workgroup of the headline form")
    ap.add_argument("--cells-window-micro", type=int, default=160_000,
                    help="bounded lag of the two forms on the corridor scan at N=2^20 (clock unpaced)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--cpu-batch-events", type=int, default=20_000,
                    help="liftings per replica for the all-cores oracle run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch-replicas", type=int, default=512)
    ap.add_argument("--batch-events", type=int, default=1_000_000)
    ap.add_argument("--batch-leg-frac", type=float, default=0.25)
    ap.add_argument("--batch-window-micro", type=int, default=200_000,
                    help="bounded lag between a replica's chains, in 1e-6 sigma (0: free running)")
    ap.add_argument("--batch-clock-period-ns", type=int, default=8000,
                    help="least time between two recomputations of a replica's H by its waiting chains")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-max-splits", type=int, default=0,
                    help="batches: rollbacks without progress before a global-order stretch "
                         "(0: library default)")
    ap.add_argument("--batch-only", action="store_true",
                    help="run only the replica batch (FP64, graph candidates) and print its result")
    ap.add_argument("--no-configs", action="store_true", help="skip the 256/4096/65536-disk workloads")
    ap.add_argument("--precision-events", type=int, default=100_000_000)
    ap.add_argument("--sweep-legs", type=int, default=40)
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-probes", action="store_true")
    ap.add_argument("--neighbours", choices=sorted(NEIGHBOURS), default=_neighbours,
                    help="candidates from the corridor scan over home cells, or from the constraint graph G(3)")
    ap.add_argument("--cooperative-launch", action="store_true",
                    help="launch the event kernel cooperatively (the runtime guarantees co-residency) "
                         "instead of the plain launch that checks it itself")
    args = ap.parse_args()
    globals()["_neighbours"] = args.neighbours
    globals()["_cooperative"] = args.cooperative_launch
    globals()["_clock_period_ns"] = args.clock_period_ns
    if args.trace_summary:
        a = args.trace_summary
        trace_summary(a[0], a[1], a[2], a[3:])
        return
    if args.pmc_summary:
        a = args.pmc_summary
        pmc_summary(a[0], a[1], a[2], a[3:])
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.batch_only:
        import torch
        assert torch.cuda.is_available(), "bench.py needs a GPU"
        torch.cuda.set_device(0)
        r = run_batch(args.batch_replicas, args.batch_events, args.batch_leg_frac,
                      window_micro=args.batch_window_micro, max_splits=args.batch_max_splits,
                      clock_period_ns=args.batch_clock_period_ns)
        print(json.dumps({"batch": r}), flush=True)
        return
    if args.save_state or args.profile_run:
        import torch
        assert torch.cuda.is_available(), "bench.py needs a GPU"
        if args.save_state:
            save_state(args.save_state, args.lanes, args.window_micro)
        else:
            profile_run(args.profile_run, args.lanes, args.window_micro,
                        "fp64" if args.form == "fp64" else "fp32", args.load_state)
        return

    # the oracle first: its process pool forks from a process that has not used the GPU
    cpu = cpu_batch = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.cpu_seconds)
        if not args.no_batch:
            cpu_batch = cpu_baseline_batch(args.batch_replicas, args.cpu_batch_events)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    sweep_Ts = () if args.no_sweep else (2.0, 4.0, 8.0, 16.0, 33.896)

    # the headline: FP64 with the default candidates (the constraint graph);
    # FP32-mixed on the corridor scan, where its binary32 filter acts, beside
    # FP64 on the same scan (the graph build has no binary32 stage)
    # (the clock pacing pays on graph candidates only; the scan forms were
    # measured best unpaced, at a smaller lag)
    head = (args.window_micro, args.clock_period_ns)
    cells = (args.cells_window_micro, 0)
    if args.form == "both":
        plan = [("fp64", "fp64", args.neighbours, head), ("fp32", "fp32", "cells", cells),
                ("fp64_cells", "fp64", "cells", cells)]
    else:
        plan = [(args.form, args.form, args.neighbours, head if args.neighbours == "graph" else cells)]
    # FP64 on the corridor scan is a like-for-like reference for the FP32-mixed
    # form: a tenth of the legs
    results = {key: run_form(form, args.steps if key != "fp64_cells" else max(args.steps // 10, 20),
                             args.warmup, args.lanes, sched[0], args.max_splits,
                             sweep_Ts=sweep_Ts if key == "fp64" else (), sweep_legs=args.sweep_legs,
                             neighbours=nb, clock_period_ns=sched[1])
               for key, form, nb, sched in plan}
    main_key = plan[0][0]
    main_form = plan[0][1]
    r = results[main_key]
    import workloads as W
    s4 = W.config(4)
    roof = {"bound": "hbm", "achieved": r["achieved_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": r["achieved_gbs"] / HBM_PEAK_GBS,
            "traffic": _traffic(main_form, r["events_per_launch"]),
            "kernel": f"k_event<{args.lanes}, {main_form}, {plan[0][2]}>",
            "alg_bytes_per_event": ALG_BYTES_PER_EVENT[main_form],
            "events_per_launch": r["events_per_launch"],
            "bytes_per_launch": r["alg_bytes_per_launch"], "avg_launch_ms": r["kernel_ms_avg"],
            "implementation_bytes_per_launch": r["implementation_bytes_per_launch"]}
    pm = _pmc(main_form)
    if pm:
        roof["counters"] = {k: v for k, v in pm.items()
                            if k.endswith("_per_launch") or k.endswith("_per_event") or k == "L2_hit_rate"
                            or k in DERIVED_PCT}
    line = {
        "metric": "ECMC events/sec on 1 GPU, N=2^20 disks η=0.708: FP32-mixed vs FP64 form",
        "value": r["events_per_s"], "unit": "events/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": r["wall_s"] / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if main_form == "fp32" else "f64", "data": "synthetic",
        "config": {"workload": "hard disks N=1048576 eta=0.708, jittered 1024x1024 centred-rectangular "
                               "lattice, k=1024 chains, legs of T=33.896 alternating +x/+y, timed after an "
                               "untimed burn-in of >= 50 liftings per disk",
                   "form": main_form, "lanes_per_chain": args.lanes, "neighbours": plan[0][2],
                   "cooperative_launch": args.cooperative_launch,
                   "window_sigma": plan[0][3][0] * 1e-6, "clock_period_ns": plan[0][3][1],
                   "parallelism": "1 GPU"},
        "roofline": roof,
        "forms": results,
    }
    if "fp32" in results and "fp64_cells" in results:
        # like for like: both forms on the corridor scan
        line["fp32_over_fp64"] = results["fp32"]["events_per_s"] / results["fp64_cells"]["events_per_s"]
        line["fp32_over_fp64_default"] = results["fp32"]["events_per_s"] / results["fp64"]["events_per_s"]
    if not args.no_probes:
        pr = run_probes(s4.k)
        ws = pr["working_set"]
        pr["gather_roofline_events_per_s"] = ws["gather_gbs_agent_scope"] * 1e9 / LINE_BYTES_PER_EVENT[main_form]
        pr["value_over_gather_roofline"] = r["events_per_s"] / pr["gather_roofline_events_per_s"]
        pr["value_over_littles_law"] = r["events_per_s"] / pr["littles_law_events_per_s"]
        pr["value_over_spec_line_roofline"] = r["events_per_s"] / (HBM_PEAK_GBS * 1e9 / LINE_BYTES_PER_EVENT[main_form])
        line["roofline_context"] = pr
    if not args.no_configs:
        cfg = run_small_configs(args.lanes, sweep_Ts, args.sweep_legs, args.window_micro)
        cfg["N65536"] = run_precision_config(args.lanes, args.window_micro, args.precision_events,
                                             1_000_000, sweep_Ts, args.sweep_legs)
        line["configs"] = cfg
        if sweep_Ts and "fp64" in results:
            line["birthday"] = birthday({
                "legs": args.sweep_legs, "N4096": cfg["N4096"]["violation_sweep"],
                "N65536": cfg["N65536"]["fp64"]["violation_sweep"],
                "N1048576": results["fp64"]["violation_sweep"]})
    if not args.no_batch:
        line["batch"] = run_batch(args.batch_replicas, args.batch_events, args.batch_leg_frac,
                                  window_micro=args.batch_window_micro, max_splits=args.batch_max_splits,
                                  clock_period_ns=args.batch_clock_period_ns)
        # the FP32-mixed batch: on the corridor scan, where the binary32 filter acts
        line["batch_fp32_cells"] = run_batch(args.batch_replicas, args.batch_events, args.batch_leg_frac,
                                             window_micro=args.batch_window_micro,
                                             clock_period_ns=args.batch_clock_period_ns, form="fp32",
                                             neighbours="cells")
        if cpu_batch:
            line["batch"]["cpu_oracle_all_cores"] = cpu_batch
        # the batched form against the plain FP64 form (different workloads:
        # 512 replicas of 1024-16384 disks against one box of 2^20)
        line["batch_over_fp64"] = line["batch"]["events_per_s"] / r["events_per_s"]
    if cpu:
        line["cpu_baseline"] = cpu
    line["paper_context"] = PAPER_CONTEXT
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
