"""Batched replicas in one persistent launch versus the oracle, per replica.

Every replica is an independent system; the batch runs its legs, rollbacks
and global-order fallback on the device.  Results must equal the oracle's
(Alg. 2) bit for bit, whatever the lane count, with or without the hipGraph.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2004_11040_amd as pkg  # noqa: E402


def _small_replicas(n_rep, seed):
    """Replicas of uneven size and density (N = 64 m, eta in [0.60, 0.72])."""
    out = []
    for ss in np.random.SeedSequence(seed).spawn(n_rep):
        rng = np.random.Generator(np.random.PCG64(ss))
        n = 64 * int(rng.integers(4, 17))
        eta = float(rng.uniform(0.60, 0.72))
        nx, ny, a, L = W.choose_grid(n, eta)
        amp = min(0.05, 0.45 * (a - 2.0))
        x, y, L = W.centred_rect_jittered(nx, ny, eta, amp, rng, n_sites=n)
        k = int(round(math.sqrt(n)))
        act = W.active_set(rng, n, k)
        out.append((x, y, L, act, 0.25 * L))
    return out


def _make(reps, flags=pkg.FP64):
    systems = []
    for x, y, L, act, T in reps:
        e = pkg.Ecmc(np.stack([x, y], 1), 1.0, L, flags=flags, max_chains=len(act), log_cap=1 << 14)
        e.set_active(act)
        systems.append(e)
    return systems


def _check(e, ref, k, tag):
    st = e.stats()
    assert st["events"] == ref.n_events, (tag, st["events"], ref.n_events)
    for c in range(k):
        assert np.array_equal(e.log(c).targets, ref.targets(c)), (tag, c)
    assert np.array_equal(e.active(), ref.active), tag
    pos = e.positions()
    assert np.array_equal(pos[:, 0], ref.x) and np.array_equal(pos[:, 1], ref.y), tag
    assert np.array_equal(e.stamps(), ref.stamps), tag
    sb, _ = e.chain_sums()
    assert np.array_equal(sb, ref.sum_b), tag
    return st


@pytest.mark.parametrize("lanes,graph,cell_pct,neighbours", [
    (4, 0, 100, pkg.NEIGHBOURS_CELLS), (8, 1, 115, pkg.NEIGHBOURS_GRAPH), (16, 0, 130, pkg.NEIGHBOURS_CELLS),
    (16, 1, 141, pkg.NEIGHBOURS_GRAPH), (32, 1, 100, pkg.NEIGHBOURS_CELLS)])
def test_batch_parity(lanes, graph, cell_pct, neighbours):
    """Lane caps (each replica takes the largest lane count up to the cap that
    fits its chains in the workgroup) and home-cell widths change the layout
    and the schedule only."""
    reps = _small_replicas(6, 7)
    systems = _make(reps)
    b = pkg.Batch(systems)
    b.set_option(pkg.OPT_LANES, lanes)
    b.set_option(pkg.OPT_CELL_PCT, cell_pct)
    b.set_option(pkg.OPT_GRAPH, graph)
    b.set_option(pkg.OPT_NEIGHBOURS, neighbours)
    legs = 3
    big = np.full(len(reps), 1 << 60, np.int64)
    b.run(big, [r[4] for r in reps], pkg.DIR_ALTERNATE, max_legs=legs)
    info = b.info()
    assert info["lanes"] == lanes and info["cell_pct"] == cell_pct, info
    assert info["legs"] == legs * len(reps), info
    for i, ((x, y, L, act, T), e) in enumerate(zip(reps, systems)):
        ref = oracle.run(x, y, 1.0, L, act, [0, 1, 0], T)
        _check(e, ref, len(act), f"rep{i} lanes={lanes}")
    # a second call continues the alternation (+y next)
    b.run(big, [r[4] for r in reps], pkg.DIR_ALTERNATE, max_legs=1)
    for i, ((x, y, L, act, T), e) in enumerate(zip(reps, systems)):
        ref = oracle.run(x, y, 1.0, L, act, [0, 1, 0, 1], T)
        _check(e, ref, len(act), f"rep{i} continued")


@pytest.mark.parametrize("window_micro,lanes,flags,clock_ns", [
    (50_000, 4, pkg.FP64, 0), (200_000, 8, pkg.FP32_MIXED, 0), (1_000_000, 16, pkg.FP64, 0),
    (200_000, 4, pkg.FP64, 8000), (200_000, 16, pkg.FP64, 50_000), (200_000, 8, pkg.FP32_MIXED, 8000)])
def test_batch_bounded_lag_parity(window_micro, lanes, flags, clock_ns):
    """A replica's chains wait at a bounded lag, each taking H from the
    others' next-event times itself, at most once per clock period in a
    replica when it is paced: scheduling only, same liftings and bits."""
    reps = _small_replicas(6, 17)
    systems = _make(reps, flags=flags)
    b = pkg.Batch(systems)
    b.set_option(pkg.OPT_LANES, lanes)
    b.set_option(pkg.OPT_CELL_PCT, 100)
    b.set_option(pkg.OPT_GRAPH, 1)
    b.set_option(pkg.OPT_WINDOW_MICRO, window_micro)
    b.set_option(pkg.OPT_CLOCK_PERIOD_NS, clock_ns)
    # the FP32-mixed form on the corridor scan, where its binary32 filter acts
    b.set_option(pkg.OPT_NEIGHBOURS, pkg.NEIGHBOURS_CELLS if flags == pkg.FP32_MIXED else pkg.NEIGHBOURS_GRAPH)
    big = np.full(len(reps), 1 << 60, np.int64)
    b.run(big, [r[4] for r in reps], pkg.DIR_ALTERNATE, max_legs=3)
    for i, ((x, y, L, act, T), e) in enumerate(zip(reps, systems)):
        ref = oracle.run(x, y, 1.0, L, act, [0, 1, 0], T)
        _check(e, ref, len(act), f"lag rep{i} w={window_micro} lanes={lanes} clock={clock_ns}")


def test_batch_fp32_mixed_and_autotune():
    reps = _small_replicas(5, 11)
    systems = _make(reps, flags=pkg.FP32_MIXED)
    b = pkg.Batch(systems)
    big = np.full(len(reps), 1 << 60, np.int64)
    b.run(big, [r[4] for r in reps], pkg.DIR_ALTERNATE, max_legs=2)
    info = b.info()
    tried = [v for v in info["tune_events_per_ms"] if v > 0]
    tried_cells = [v for v in info["tune_cell_events_per_ms"] if v > 0]
    assert len(tried) >= 2 and len(tried_cells) >= 2, info
    assert info["lanes"] in (4, 8, 16, 32) and 100 <= info["cell_pct"] <= 141
    assert not info["tune_from_cache"]
    # the tuning legs count: one per tried lane cap and cell width, then two more
    n_legs = len(tried) + len(tried_cells) + 2
    for i, ((x, y, L, act, T), e) in enumerate(zip(reps, systems)):
        dirs = [l % 2 for l in range(n_legs)]
        ref = oracle.run(x, y, 1.0, L, act, dirs, T)
        st = _check(e, ref, len(act), f"fp32 rep{i}")
        assert st["legs"] == n_legs


def test_batch_event_targets():
    """Replicas stop at the end of the leg in which they reach their target."""
    reps = _small_replicas(4, 13)
    systems = _make(reps)
    b = pkg.Batch(systems)
    b.set_option(pkg.OPT_LANES, 8)
    b.set_option(pkg.OPT_CELL_PCT, 100)
    targets = np.array([1, 2000, 5000, 0], np.int64)
    b.run(targets, [r[4] for r in reps], pkg.DIR_X)
    for i, ((x, y, L, act, T), e) in enumerate(zip(reps, systems)):
        st = e.stats()
        if targets[i] == 0:
            assert st["legs"] == 0 and st["events"] == 0
            continue
        ref = oracle.run(x, y, 1.0, L, act, [0] * st["legs"], T)
        _check(e, ref, len(act), f"target rep{i}")
        assert st["events"] >= targets[i]
        if st["legs"] > 1:
            prev = oracle.run(x, y, 1.0, L, act, [0] * (st["legs"] - 1), T, log=False)
            assert prev.n_events < targets[i]


def test_batch_replica_workload_sample():
    """The first replicas of the 512-replica workload (N up to 16384, k up to
    128), one leg each, against the oracle."""
    reps = W.replica_batch(3)
    systems = []
    for s in reps:
        e = pkg.Ecmc(np.stack([s.x, s.y], 1), 1.0, s.L, flags=pkg.FP32_MIXED, max_chains=s.k,
                     log_cap=1 << 12)
        e.set_active(s.active)
        systems.append(e)
    b = pkg.Batch(systems)
    b.set_option(pkg.OPT_LANES, 4)
    b.set_option(pkg.OPT_CELL_PCT, 100)
    b.set_option(pkg.OPT_WINDOW_MICRO, 300_000)
    big = np.full(len(reps), 1 << 60, np.int64)
    b.run(big, [s.T for s in reps], pkg.DIR_ALTERNATE, max_legs=1)
    for s, e in zip(reps, systems):
        ref = oracle.run(s.x, s.y, 1.0, s.L, s.active, [0], s.T, log_cap=1 << 20)
        _check(e, ref, s.k, s.name)


def test_batch_one_replica_one_chain():
    """The smallest batch: one replica with one chain (the rest of the
    workgroup idle), three alternating legs."""
    x, y, L, act, T = _small_replicas(1, 23)[0]
    act = act[:1]
    e = pkg.Ecmc(np.stack([x, y], 1), 1.0, L, max_chains=1, log_cap=1 << 14)
    e.set_active(act)
    b = pkg.Batch([e])
    b.set_option(pkg.OPT_LANES, 4)
    b.set_option(pkg.OPT_CELL_PCT, 100)
    b.run(np.array([1 << 60], np.int64), [T], pkg.DIR_ALTERNATE, max_legs=3)
    ref = oracle.run(x, y, 1.0, L, act, [0, 1, 0], T)
    _check(e, ref, 1, "one replica, one chain")


def test_batch_replica_at_the_chain_limit():
    """A replica with 128 chains at 4 lanes fills its workgroup's 512 threads
    (the largest k of the 512-replica workload, N = 16384), one leg."""
    s = W.replica_batch(512)[230]
    assert s.k == 128
    e = pkg.Ecmc(np.stack([s.x, s.y], 1), 1.0, s.L, flags=pkg.FP32_MIXED, max_chains=s.k, log_cap=1 << 12)
    e.set_active(s.active)
    b = pkg.Batch([e])
    b.set_option(pkg.OPT_LANES, 32)      # capped at 4 lanes for 128 chains
    b.set_option(pkg.OPT_CELL_PCT, 130)
    b.set_option(pkg.OPT_WINDOW_MICRO, 350_000)
    b.run(np.array([1 << 60], np.int64), [s.T], pkg.DIR_ALTERNATE, max_legs=1)
    ref = oracle.run(s.x, s.y, 1.0, s.L, s.active, [0], s.T, log_cap=1 << 20)
    _check(e, ref, s.k, s.name)


def _workload_systems(n_rep, flags=pkg.FP32_MIXED):
    reps = W.replica_batch(n_rep)
    systems = []
    for s in reps:
        e = pkg.Ecmc(np.stack([s.x, s.y], 1), 1.0, s.L, flags=flags, max_chains=s.k, log_cap=1 << 14)
        e.set_active(s.active)
        systems.append(e)
    return reps, systems


def _oracle_final_state(task):
    """The oracle's final state of one replica (a worker of a forked pool:
    the oracle is C code on the host and touches no GPU)."""
    x, y, L, act, dirs, T = task
    r = oracle.run(x, y, 1.0, L, act, dirs, T, log=False)
    return r.x, r.y, r.stamps, r.active, r.sum_b, r.n_events


def test_batch_all_replicas_match_the_oracle():
    """All 512 replicas of the workload, the first four legs from the lattice
    (about 6.6e7 liftings; chains make some 10^4 liftings each in the first
    leg, so undo-overflow replays can occur), in the benchmark's FP64
    settings with lanes and cells fixed: every replica's positions, stamps,
    active disks, lifting count and per-chain sums of b equal the oracle's
    bit for bit.  Replicas are handed out two legs at a time, and the 256
    that have not started displace the first 256 after their first turn, so
    most replicas run their second turn on another workgroup, often on
    another XCD.  The oracle runs in a forked pool of host processes, one
    per core up to 16."""
    import multiprocessing as mp
    import os

    reps, systems = _workload_systems(512, flags=pkg.FP64)
    b = pkg.Batch(systems)
    b.set_option(pkg.OPT_GRAPH, 1)
    b.set_option(pkg.OPT_NEIGHBOURS, pkg.NEIGHBOURS_GRAPH)
    b.set_option(pkg.OPT_WINDOW_MICRO, 200_000)
    b.set_option(pkg.OPT_CLOCK_PERIOD_NS, 8000)
    b.set_option(pkg.OPT_LANES, 4)
    b.set_option(pkg.OPT_CELL_PCT, 141)
    b.run(np.full(len(reps), 1 << 60, np.int64), [s.T for s in reps], pkg.DIR_ALTERNATE, max_legs=4)
    tasks = [(s.x, s.y, s.L, s.active, s.leg_dirs(4), s.T) for s in reps]
    procs = max(1, min(16, len(os.sched_getaffinity(0))))
    with mp.get_context("fork").Pool(procs) as pool:
        refs = pool.map(_oracle_final_state, tasks, chunksize=1)
    bad = []
    for s, e, (x, y, stamps, act, sb, nev) in zip(reps, systems, refs):
        pos = e.positions()
        ok = (e.stats()["events"] == nev and np.array_equal(pos[:, 0], x) and np.array_equal(pos[:, 1], y)
              and np.array_equal(e.stamps(), stamps) and np.array_equal(e.active(), act)
              and np.array_equal(e.chain_sums()[0], sb))
        if not ok:
            bad.append(s.name)
    replays = sum(e.stats()["overflow_legs"] for e in systems)
    print(f"512 replicas, four legs: {sum(e.stats()['events'] for e in systems)} liftings, "
          f"{replays} overflow replays, {len(bad)} differ from the oracle", flush=True)
    assert not bad, bad[:8]


def test_batch_workload_sixteen_replicas_two_legs():
    """16 replicas of the 512-replica workload (N from 1024 to 16384, k =
    round(sqrt N)) over two legs in the benchmark's settings (graph, bounded
    lag 0.2 sigma, H recomputed at most every 8 us, autotuned lanes and cells)
    against the oracle."""
    reps, systems = _workload_systems(16)
    b = pkg.Batch(systems)
    b.set_option(pkg.OPT_GRAPH, 1)
    b.set_option(pkg.OPT_WINDOW_MICRO, 200_000)
    b.set_option(pkg.OPT_CLOCK_PERIOD_NS, 8000)
    big = np.full(len(reps), 1 << 60, np.int64)
    b.run(big, [s.T for s in reps], pkg.DIR_ALTERNATE, max_legs=2)
    for s, e in zip(reps, systems):
        n_legs = e.stats()["legs"]
        assert n_legs >= 2
        ref = oracle.run(s.x, s.y, 1.0, s.L, s.active, s.leg_dirs(n_legs), s.T, log_cap=1 << 22)
        _check(e, ref, s.k, s.name)
        assert e.overlaps() == 0


def test_batch_options_take_effect_between_graph_replays():
    """Every option travels in the replica descriptors: switching the
    reservations off between two replays of one captured graph must stop
    the chains from giving claims back."""
    reps, systems = _workload_systems(12)
    b = pkg.Batch(systems)
    b.set_option(pkg.OPT_GRAPH, 1)
    b.set_option(pkg.OPT_LANES, 4)
    b.set_option(pkg.OPT_CELL_PCT, 100)
    big = np.full(len(reps), 1 << 60, np.int64)
    T = [s.T for s in reps]
    b.run(big, T, pkg.DIR_ALTERNATE, max_legs=1)
    y0 = sum(e.stats()["claim_yields"] for e in systems)
    assert y0 > 0
    b.set_option(pkg.OPT_FEATURES, pkg.FEAT_ALL & ~pkg.FEAT_RESERVE)
    b.set_option(pkg.OPT_LANES, 8)
    b.run(big, T, pkg.DIR_ALTERNATE, max_legs=1)
    assert sum(e.stats()["claim_yields"] for e in systems) == y0
    assert b.info()["lanes"] == 8 and b.info()["graph"] == 1
    for s, e in zip(reps, systems):
        ref = oracle.run(s.x, s.y, 1.0, s.L, s.active, [0, 1], s.T, log_cap=1 << 22)
        _check(e, ref, s.k, s.name)


def test_batch_tune_cache_round_trip(tmp_path):
    """The autotuner stores its choice under the batch's signature; an
    identical batch takes it from the file without tuning legs."""
    path = str(tmp_path / "tune.json")
    reps = _small_replicas(5, 31)
    first = _make(reps, flags=pkg.FP32_MIXED)
    b = pkg.Batch(first)
    b.set_option(pkg.OPT_GRAPH, 1)
    b.tune_cache(path)
    big = np.full(len(reps), 1 << 60, np.int64)
    T = [r[4] for r in reps]
    b.run(big, T, pkg.DIR_ALTERNATE, max_legs=1)
    i1 = b.info()
    assert not i1["tune_from_cache"]
    text = open(path).read()
    assert text.startswith("{") and "lanes_cap" in text and "cell_pct" in text
    second = _make(reps, flags=pkg.FP32_MIXED)
    b2 = pkg.Batch(second)
    b2.set_option(pkg.OPT_GRAPH, 1)
    b2.tune_cache(path)
    b2.run(big, T, pkg.DIR_ALTERNATE, max_legs=1)
    i2 = b2.info()
    assert i2["tune_from_cache"] and i2["lanes"] == i1["lanes"] and i2["cell_pct"] == i1["cell_pct"]
    assert all(v == 0 for v in i2["tune_events_per_ms"] + i2["tune_cell_events_per_ms"])
    for (x, y, L, act, TT), e in zip(reps, second):
        assert e.stats()["legs"] == 1
        ref = oracle.run(x, y, 1.0, L, act, [0], TT)
        _check(e, ref, len(act), "from cache")


def test_batch_workload_all_replicas_invariants():
    """All 512 replicas of the workload, six legs each in the benchmark's
    settings (FP64, graph candidates, lag 0.2 sigma, H recomputed at most
    every 8 us; lanes and cells fixed, no autotuning): properties that hold
    at any size, on every replica (the oracle covers 16 of them): k distinct
    active disks stamped with the breakpoint, static disks stamped before
    it, no overlaps, non-negative sums of lifting distances."""
    reps, systems = _workload_systems(512, flags=pkg.FP64)
    b = pkg.Batch(systems)
    b.set_option(pkg.OPT_GRAPH, 1)
    b.set_option(pkg.OPT_NEIGHBOURS, pkg.NEIGHBOURS_GRAPH)
    b.set_option(pkg.OPT_WINDOW_MICRO, 200_000)
    b.set_option(pkg.OPT_CLOCK_PERIOD_NS, 8000)
    b.set_option(pkg.OPT_LANES, 4)
    b.set_option(pkg.OPT_CELL_PCT, 141)
    big = np.full(len(reps), 1 << 60, np.int64)
    b.run(big, [s.T for s in reps], pkg.DIR_ALTERNATE, max_legs=6)
    bad = []
    for s, e in zip(reps, systems):
        st = e.stats()
        act = e.active()
        stamps = e.stamps()
        is_act = np.zeros(s.n, bool)
        is_act[act] = True
        sb, ev = e.chain_sums()
        ok = (st["legs"] == 6 and len(np.unique(act)) == s.k and np.all(stamps[is_act] == s.T)
              and np.all((stamps[~is_act] >= 0.0) & (stamps[~is_act] < s.T)) and e.overlaps() == 0
              and np.all(sb >= 0.0) and int(ev.sum()) == st["events"])
        if not ok:
            bad.append(s.name)
    info = b.info()
    print(f"512 replicas: {sum(e.stats()['events'] for e in systems)} liftings, "
          f"{info['rollbacks']} rollbacks, {info['global_runs']} global stretches", flush=True)
    assert not bad, bad[:8]


def test_batch_forms_agree_on_all_replicas():
    """The 512-replica workload, six legs, in the benchmark's two batch forms
    (FP64 on graph candidates; FP32-mixed on the corridor scan, whose
    binary32 filter decides nothing without a binary64 recomputation), lanes
    and cells fixed: every replica ends in bit-identical states (positions,
    stamps, active disks, per-chain lifting counts and sums).  Replicas whose
    chains make some 10^4 liftings in a leg from the jittered lattice take
    the undo-overflow replay in one run and not in another."""
    out = []
    for flags, nb in ((pkg.FP64, pkg.NEIGHBOURS_GRAPH), (pkg.FP32_MIXED, pkg.NEIGHBOURS_CELLS)):
        reps, systems = _workload_systems(512, flags=flags)
        b = pkg.Batch(systems)
        b.set_option(pkg.OPT_GRAPH, 1)
        b.set_option(pkg.OPT_NEIGHBOURS, nb)
        b.set_option(pkg.OPT_WINDOW_MICRO, 200_000)
        b.set_option(pkg.OPT_CLOCK_PERIOD_NS, 8000)
        b.set_option(pkg.OPT_LANES, 4)
        b.set_option(pkg.OPT_CELL_PCT, 141)
        b.run(np.full(len(reps), 1 << 60, np.int64), [s.T for s in reps], pkg.DIR_ALTERNATE, max_legs=6)
        out.append([(e.positions(), e.stamps(), e.active(), *e.chain_sums()) for e in systems])
        b.close()
        for e in systems:
            e.close()
    bad = [reps[r].name for r, (x, y) in enumerate(zip(*out))
           if not all(np.array_equal(u, v) for u, v in zip(x, y))]
    print(f"512 replicas, two forms: {len(bad)} differ", flush=True)
    assert not bad, bad[:8]


@pytest.mark.parametrize("mode", ["context", "batch"])
def test_undo_overflow_replays_the_leg_in_global_order(mode):
    """A chain that commits more liftings after the settled time than its
    undo records hold (4096) cannot be rolled back: the leg is replayed from
    its breakpoint in global-time order (Alg. 2).  The chains' disks must be
    tagged as moving before that replay, or a chain lifts to a disk where it
    stood at the breakpoint while another chain still moves it.  Forced here
    with the test hook: chain 7 of a 4544-disk replica of the workload
    (about 10^4 liftings per chain in its first leg) reports a violation at
    its 4200th lifting of an attempt.  The result must equal the oracle's
    bit for bit."""
    s = W.replica_batch(512)[146]
    e = pkg.Ecmc(np.stack([s.x, s.y], 1), 1.0, s.L, flags=pkg.FP64, max_chains=s.k, log_cap=1 << 15)
    e.set_active(s.active)
    e.set_option(pkg.OPT_INJECT_EVENT, 4200)
    e.set_option(pkg.OPT_INJECT_CHAIN, 7)
    if mode == "batch":
        b = pkg.Batch([e])
        b.set_option(pkg.OPT_GRAPH, 1)
        b.set_option(pkg.OPT_NEIGHBOURS, pkg.NEIGHBOURS_GRAPH)
        b.set_option(pkg.OPT_WINDOW_MICRO, 200_000)
        b.set_option(pkg.OPT_LANES, 4)
        b.set_option(pkg.OPT_CELL_PCT, 141)
        b.run(np.array([1 << 60], np.int64), [s.T], pkg.DIR_ALTERNATE, max_legs=1)
    else:
        e.set_option(pkg.OPT_NEIGHBOURS, pkg.NEIGHBOURS_GRAPH)
        e.run(s.T, s.T, 0)
    ref = oracle.run(s.x, s.y, 1.0, s.L, s.active, [0], s.T)
    st = _check(e, ref, s.k, mode)
    print(f"{mode}: {st['events']} liftings, {st['overflow_legs']} overflow replays, "
          f"{st['reruns']} rollbacks", flush=True)
    assert st["legs"] == 1 and st["overflow_legs"] >= 1
