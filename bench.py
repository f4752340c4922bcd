"""Benchmark: ECMC events/s on one MI355X for hard disks, N = 2^20, eta = 0.708.

One step = one leg (breakpoint interval) of the whole hot path: home-cell build,
1024 chains running the event kernel to the breakpoint (reruns included),
breakpoint reduction and write-back.  Directions alternate +x/+y.  Inputs are
seeded synthetic lattices resident in HBM before the timed region starts.

Prints ONE JSON line (see the repository's design notes for the fields).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, published
# Algorithmic bytes of the event kernel.  Per scanned cell slot: the fixed
# record (p, id; 16 B) and the mutable record (a, t; 16 B).  Per lifting:
# next-event time 8, reservation 8, activation-record invalidation 8, claim 4,
# target re-read 16, lane-minima re-read 48, reservation read 8, undo record
# 60, commit (t_j, t_i, a_i) 24, activation record 36, reservation release 8,
# tag release 4, log 4: 236 B.
BYTES_PER_SLOT = 32
BYTES_PER_EVENT = 236


def _src_hash():
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_2004_11040_amd", "csrc", "ecmc_kernels.hip"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def pmc_summary_path(form):
    return os.path.join(ROOT, "profiles", f"event_kernel_N1048576_{form}_pmc.json")


def _traffic(form, events_per_launch):
    """HBM bytes per event-kernel launch: the bytes per lifting measured by the
    committed rocprofv3 counter summary (FETCH_SIZE + WRITE_SIZE, calibrated on
    a copy of known size) times this run's liftings per launch.  None if the
    summary is missing or was taken on another kernel source."""
    try:
        with open(pmc_summary_path(form)) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("source_sha256_16") != _src_hash() or not d.get("hbm_bytes_per_event"):
        return None
    return d["hbm_bytes_per_event"] * events_per_launch


def cpu_baseline(seconds: float):
    """The oracle, as it stands, on a bounded sample of the same workload."""
    import oracle
    import workloads as W
    s = W.config(4)
    x, y, act = s.x, s.y, s.active
    events, t_used, legs = 0, 0.0, 0
    while t_used < seconds and legs < 8:
        t0 = time.perf_counter()
        r = oracle.run(x, y, s.sigma, s.L, act, [legs % 2], s.T, log=False)
        t_used += time.perf_counter() - t0
        print(f"[bench] cpu baseline: leg {legs} done, {t_used:.1f} s", file=sys.stderr, flush=True)
        events += r.n_events
        x, y, act = r.x, r.y, r.active
        legs += 1
    return {"value": events / t_used, "unit": "events/s", "cores": 1, "kind": "oracle",
            "sample": f"first {legs} legs ({events} liftings) of the N=1048576 eta=0.708 k=1024 "
                      f"workload, serial C global-time event queue, 1 host thread"}


def _stats_delta(st0, st1):
    d = {k: st1[k] - st0[k] for k in st1 if isinstance(st1[k], (int, float))}
    d["violations_by_kind"] = [b - a for a, b in zip(st0["violations_by_kind"], st1["violations_by_kind"])]
    return d


def run_form(form, steps, warmup, lanes, window_micro, max_splits=0):
    import numpy as np
    import torch

    import paper_2004_11040_amd as pkg
    import workloads as W

    s = W.config(4)
    flags = pkg.FP32_MIXED if form == "fp32" else pkg.FP64
    e = pkg.Ecmc(np.stack([s.x, s.y], 1), s.sigma, s.L, flags=flags, max_chains=s.k, log_cap=1 << 12)
    e.set_option(pkg.OPT_LANES, lanes)
    e.set_option(pkg.OPT_KERNEL_TIMING, 1)
    e.set_option(pkg.OPT_WINDOW_MICRO, window_micro)
    if max_splits:
        e.set_option(pkg.OPT_MAX_SPLITS, max_splits)
    e.set_active(s.active)
    if warmup:
        e.run(warmup * s.T, s.T, pkg.DIR_ALTERNATE)
    st0 = e.stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < steps:  # chunks only to report progress; one timed region
        n = min(10, steps - done)
        e.run(n * s.T, s.T, pkg.DIR_ALTERNATE)
        done += n
        print(f"[bench] {form}: {done}/{steps} legs", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st1 = e.stats()
    d = _stats_delta(st0, st1)
    wall = t1 - t0
    launches = max(d["event_launches"], 1)
    kbytes = (d["timed_slots"] * BYTES_PER_SLOT + d["timed_events"] * BYTES_PER_EVENT) / launches
    kdur = d["event_kernel_ms"] / launches / 1e3
    achieved = kbytes / kdur / 1e9 if kdur > 0 else 0.0
    overlaps = e.overlaps()
    res = {
        "events": d["events"], "wall_s": wall, "events_per_s": d["events"] / wall,
        "legs": d["legs"], "legs_violated": d["legs_violated"], "reruns": d["reruns"],
        "global_legs": d["global_legs"], "lockstep_runs": d["lockstep_runs"],
        "violations_screened": d["violations_screened"], "claim_yields": d["claim_yields"],
        "spin_aborts": d["spin_aborts"],
        "violations_by_kind": d["violations_by_kind"], "attempts": d["attempts"],
        "slots_per_event": d["slots_scanned"] / max(d["events"], 1),
        "events_per_launch": d["timed_events"] / launches,
        "kernel_ms_avg": kdur * 1e3, "kernel_bytes_per_launch": kbytes, "achieved_gbs": achieved,
        "kernel_time_frac": d["event_kernel_ms"] / 1e3 / wall, "overlaps": overlaps,
        "pressure_raw": 1.0 + d["sum_b"] / d["chain_time"] if d["chain_time"] else None,
        "violation_probability_per_breakpoint": d["legs_violated"] / max(d["legs"], 1),
    }
    e.close()
    return res


def birthday_estimate(k, L, T, sigma=1.0):
    """Generalized birthday estimate of the violation probability per
    breakpoint (Sec. 3.4): k chains, each confined during a leg to a region of
    area about T x 4 sigma (its path along v and the corridor around it), in a
    box of area L^2 cut into L^2 / (4 sigma T) such regions; p = 1 - exp(-k^2 / 2 n)."""
    import math
    n_regions = L * L / (4.0 * sigma * T)
    return 1.0 - math.exp(-k * k / (2.0 * n_regions))


def run_batch(n_rep, target, t_frac, graph=1, window_micro=0, max_splits=0):
    """The replica workload: n_rep seeded replicas of N in {1024..16384}, eta in
    [0.60, 0.72], k = round(sqrt N), FP32-mixed, run in one persistent launch
    (captured in a hipGraph) until every replica has `target` liftings; the
    autotuner's legs come first and are not timed."""
    import numpy as np
    import torch

    import paper_2004_11040_amd as pkg
    import workloads as W
    reps = W.replica_batch(n_rep)
    systems = []
    for s in reps:
        e = pkg.Ecmc(np.stack([s.x, s.y], 1), s.sigma, s.L, flags=pkg.FP32_MIXED, max_chains=s.k,
                     log_cap=1 << 8)
        e.set_active(s.active)
        systems.append(e)
    b = pkg.Batch(systems)
    b.set_option(pkg.OPT_GRAPH, graph)
    b.set_option(pkg.OPT_WINDOW_MICRO, window_micro)
    if max_splits:
        b.set_option(pkg.OPT_MAX_SPLITS, max_splits)
    T = [t_frac * s.L for s in reps]
    big = np.full(n_rep, 1 << 60, np.int64)
    b.run(big, T, pkg.DIR_ALTERNATE, max_legs=1)  # autotune (one leg per lane count)
    tune = b.info()
    ev0 = sum(e.stats()["events"] for e in systems)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.run(np.full(n_rep, target, np.int64), T, pkg.DIR_ALTERNATE, max_legs=0)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    info = b.info()
    ev1 = sum(e.stats()["events"] for e in systems)
    print(f"[bench] batch: {ev1 - ev0} liftings in {wall:.2f} s", file=sys.stderr, flush=True)
    overlaps = sum(e.overlaps() for e in systems)
    out = {"workload": f"{n_rep} replicas, N in 64*[16,256], eta in [0.60,0.72], k=round(sqrt N), "
                       f"legs of {t_frac} L alternating +x/+y, FP32-mixed, {target} liftings per replica, "
                       f"bounded lag {window_micro * 1e-6:g} sigma",
           "events": ev1 - ev0, "wall_s": wall, "events_per_s": (ev1 - ev0) / wall,
           "device_ms": info["device_ms"], "lanes": info["lanes"], "graph": info["graph"],
           "workgroups": info["workgroups"], "legs": info["legs"], "rollbacks": info["rollbacks"],
           "global_runs": info["global_runs"], "autotune_events_per_ms": tune["tune_events_per_ms"],
           "replica_ms_max": info["replica_ms_max"],
           "load_balance": info["replica_ms_sum"] / max(info["workgroups"] * info["device_ms"], 1e-9),
           "overlaps": overlaps, "total_disks": int(sum(s.n for s in reps)),
           "total_chains": int(sum(s.k for s in reps))}
    b.close()
    for e in systems:
        e.close()
    return out


def profile_run(legs, lanes, window_micro, form):
    """Short run for hardware-counter collection: a few legs of the workload,
    then a device copy of 256 MiB (read 256 MiB, write 256 MiB) whose counter
    readings calibrate the bytes the counters report."""
    import numpy as np
    import torch

    import paper_2004_11040_amd as pkg
    import workloads as W
    s = W.config(4)
    flags = pkg.FP32_MIXED if form == "fp32" else pkg.FP64
    e = pkg.Ecmc(np.stack([s.x, s.y], 1), s.sigma, s.L, max_chains=s.k, log_cap=1 << 12, flags=flags)
    e.set_option(pkg.OPT_LANES, lanes)
    e.set_option(pkg.OPT_WINDOW_MICRO, window_micro)
    e.set_option(pkg.OPT_KERNEL_TIMING, 1)
    e.set_active(s.active)
    e.run(legs * s.T, s.T, pkg.DIR_ALTERNATE)
    st = e.stats()
    print(json.dumps({"profile_run": True, "form": form, "lanes": lanes,
                      "events": st["events"], "attempts": st["attempts"],
                      "event_launches": st["event_launches"], "timed_events": st["timed_events"],
                      "slots_scanned": st["slots_scanned"]}), flush=True)
    a = torch.ones(256 << 20, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()


def _pmc_values(path, counter):
    """Per-dispatch values of one counter from a rocprofv3 counter_collection
    CSV: list of (kernel name, value)."""
    import csv
    out = []
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            if row.get("Counter_Name") == counter:
                out.append((row.get("Kernel_Name", ""), float(row["Counter_Value"])))
    return out


def pmc_summary(fetch_csv, write_csv, profile_log):
    """Turn two counter runs of --profile-run (FETCH_SIZE, then WRITE_SIZE) into
    the committed summary: bytes per event-kernel dispatch and per lifting,
    each counter calibrated by its reading on the 256 MiB device copy."""
    copy_bytes = 256 << 20
    fe, wr = _pmc_values(fetch_csv, "FETCH_SIZE"), _pmc_values(write_csv, "WRITE_SIZE")
    ev_f = [v for n, v in fe if "k_event" in n]
    ev_w = [v for n, v in wr if "k_event" in n]
    cp_f = max(v for n, v in fe if "copy" in n.lower() or "elementwise" in n.lower())
    cp_w = max(v for n, v in wr if "copy" in n.lower() or "elementwise" in n.lower())
    f_cal = copy_bytes / (cp_f * 1024.0)  # counters are in KiB
    w_cal = copy_bytes / (cp_w * 1024.0)
    with open(profile_log) as f:
        run = next(json.loads(line) for line in f if line.startswith("{") and "profile_run" in line)
    # rounds enqueued past the end of a leg are dispatched but return at once:
    # totals over every dispatch, per launch that ran an attempt
    total = sum(ev_f) * 1024.0 * f_cal + sum(ev_w) * 1024.0 * w_cal
    per_launch = total / max(run["event_launches"], 1)
    events_per_launch = run["timed_events"] / max(run["event_launches"], 1)
    form = run.get("form", "fp64")
    d = {"source_sha256_16": _src_hash(), "form": form,
         "kernel": f"k_event<{run.get('lanes', 64)}, {'true' if form == 'fp32' else 'false'}>",
         "dispatches": len(ev_f),
         "fetch_kib_mean": sum(ev_f) / max(len(ev_f), 1), "write_kib_mean": sum(ev_w) / max(len(ev_w), 1),
         "copy_fetch_kib": cp_f, "copy_write_kib": cp_w, "fetch_calibration": f_cal, "write_calibration": w_cal,
         "launches_that_ran": run["event_launches"], "liftings": run["timed_events"],
         "hbm_bytes_per_launch": per_launch, "events_per_launch": events_per_launch,
         "hbm_bytes_per_event": per_launch / events_per_launch if events_per_launch else None}
    with open(pmc_summary_path(form), "w") as f:
        json.dump(d, f, indent=1)
    print(json.dumps(d))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--profile-run", type=int, default=0, metavar="LEGS",
                    help="only run LEGS legs and a 256 MiB copy (for rocprofv3 counters)")
    ap.add_argument("--pmc-summary", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "PROFILE_LOG"),
                    help="write the counter summary from two --profile-run counter runs")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200, help="timed legs")
    ap.add_argument("--warmup", type=int, default=4, help="untimed legs")
    ap.add_argument("--form", choices=["fp64", "fp32", "both"], default="both")
    ap.add_argument("--lanes", type=int, default=64)
    ap.add_argument("--max-splits", type=int, default=0,
                    help="rollbacks without progress before a lockstep stretch (0: library default)")
    ap.add_argument("--window-micro", type=int, default=160_000,
                    help="bounded lag between chains, in 1e-6 sigma (0: free running)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch-replicas", type=int, default=512)
    ap.add_argument("--batch-events", type=int, default=1_000_000)
    ap.add_argument("--batch-leg-frac", type=float, default=0.25)
    ap.add_argument("--batch-window-micro", type=int, default=350_000,
                    help="bounded lag between a replica's chains, in 1e-6 sigma (0: free running)")
    ap.add_argument("--no-batch", action="store_true")
    args = ap.parse_args()
    if args.pmc_summary:
        pmc_summary(*args.pmc_summary)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.profile_run:
        profile_run(args.profile_run, args.lanes, args.window_micro,
                    "fp64" if args.form == "fp64" else "fp32")
        return

    forms = ["fp64", "fp32"] if args.form == "both" else [args.form]
    results = {f: run_form(f, args.steps, args.warmup, args.lanes, args.window_micro, args.max_splits)
               for f in forms}
    main_form = "fp32" if "fp32" in results else "fp64"
    r = results[main_form]
    kb = r["kernel_bytes_per_launch"]
    roof = {"bound": "hbm", "achieved": r["achieved_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": r["achieved_gbs"] / HBM_PEAK_GBS,
            "traffic": _traffic(main_form, r["events_per_launch"]),
            "kernel": f"k_event<{args.lanes}, {main_form}>", "bytes_per_launch": kb,
            "avg_launch_ms": r["kernel_ms_avg"]}
    import workloads as W
    s4 = W.config(4)
    for f in results.values():
        f["birthday_estimate_per_breakpoint"] = birthday_estimate(s4.k, s4.L, s4.T)
    line = {
        "metric": "ECMC events/sec on 1 GPU, N=2^20 disks η=0.708: FP32-mixed vs FP64 form",
        "value": r["events_per_s"], "unit": "events/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": r["wall_s"] / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if main_form == "fp32" else "f64", "data": "synthetic",
        "config": {"workload": "hard disks N=1048576 eta=0.708, jittered 1024x1024 centred-rectangular "
                               "lattice, k=1024 chains, legs of T=33.896 alternating +x/+y",
                   "form": main_form, "lanes_per_chain": args.lanes,
                   "window_sigma": args.window_micro * 1e-6, "parallelism": "1 GPU"},
        "roofline": roof,
        "forms": results,
    }
    if "fp32" in results and "fp64" in results:
        line["fp32_over_fp64"] = results["fp32"]["events_per_s"] / results["fp64"]["events_per_s"]
    if not args.no_batch:
        line["batch"] = run_batch(args.batch_replicas, args.batch_events, args.batch_leg_frac,
                                  window_micro=args.batch_window_micro)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
