"""The constraint graph G(3) on the GPU (Sec. 3.1) and both candidate
sources of the event kernel, against the oracle.

* ecmc_graph: the arrows built on the device equal the oracle's brute-force
  G(3) (every disk, or a sample at 65536 disks), in all four directions.
* ECMC_NEIGHBOURS_GRAPH (the default) and ECMC_NEIGHBOURS_CELLS (the corridor
  scan, where FP32-mixed filters in binary32): the same liftings, bit for
  bit, as the oracle (Lemma 2), the batch included.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle import constraint_graph as CG

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2004_11040_amd as pkg  # noqa: E402
from test_gpu_parity import _square, check_parity, gpu_run  # noqa: E402

GRAPH = ((pkg.OPT_NEIGHBOURS, pkg.NEIGHBOURS_GRAPH),)
CELLS = ((pkg.OPT_NEIGHBOURS, pkg.NEIGHBOURS_CELLS),)
MODES = pytest.mark.parametrize("mode", [GRAPH, CELLS], ids=["graph", "cells"])


FORMS = pytest.mark.parametrize("flags", [pkg.FP64, pkg.FP32_MIXED], ids=["fp64", "fp32"])


@pytest.mark.parametrize("cfg,direction", [(0, 0), (0, 3), (1, 0), (1, 1), (1, 2), (1, 3), (2, 1), (4, 0)])
@FORMS
def test_device_graph_equals_the_oracle(cfg, direction, flags):
    """The tiled build (FP64, and FP32-mixed with its binary32 filter) against
    brute force; at 2^20 disks on a sample of 150."""
    s = W.config(cfg)
    e = pkg.Ecmc(np.stack([s.x, s.y], 1), s.sigma, s.L, flags=flags, max_chains=s.k, log_cap=16)
    e.set_active(s.active)
    got = e.graph(direction, s.T)
    rows = None
    if s.n > 5000:
        rows = np.random.Generator(np.random.PCG64(3)).choice(s.n, 1500 if s.n < 100_000 else 150, replace=False)
    want, _, _ = CG.g3(s.x, s.y, s.sigma, s.L, direction, horizon=s.T, rows=rows)
    if rows is not None:
        got, want = got[rows], want[rows]
    assert np.array_equal(got, want), (cfg, direction, np.argwhere(got != want)[:5])
    print(f"[graph] cfg={cfg} dir={direction}: out-degree {np.mean((got >= 0).sum(1)):.3f}")


@pytest.mark.parametrize("direction", [0, 1, 2, 3])
@FORMS
def test_device_graph_dilute_walks_past_the_halo(direction, flags):
    """A dilute square lattice (eta = 0.03, spacing ~10 sigma) with a long
    horizon: the off-centre lanes are mostly empty, so walks run far past the
    staged tile and continue on global memory."""
    x, y, L, act = _square(7, 64, 0.03, 64)
    T = 0.4 * L
    e = pkg.Ecmc(np.stack([x, y], 1), 1.0, L, flags=flags, max_chains=64, log_cap=16)
    e.set_active(act)
    got = e.graph(direction, T)
    rows = np.random.Generator(np.random.PCG64(5)).choice(x.shape[0], 800, replace=False)
    want, _, _ = CG.g3(x, y, 1.0, L, direction, horizon=T, rows=rows)
    assert np.array_equal(got[rows], want[rows]), np.argwhere(got[rows] != want[rows])[:5]
    print(f"[graph] dilute dir={direction}: out-degree {np.mean((got >= 0).sum(1)):.3f}")


@pytest.mark.parametrize("lanes", [64, 32, 16])
@MODES
def test_graph_small_parity(lanes, mode):
    s = W.config(0)
    dirs = [0] * 10
    e = gpu_run(s.x, s.y, s.L, s.active, dirs, s.T, lanes=lanes, opts=mode)
    ref = oracle.run(s.x, s.y, 1.0, s.L, s.active, dirs, s.T)
    check_parity(e, ref, s.L, s.k, f"graph lanes={lanes}")


@pytest.mark.parametrize("seed,n_side,eta,k,tfrac", [
    (101, 8, 0.50, 1, 0.25), (103, 12, 0.70, 12, 0.20), (105, 9, 0.40, 5, 0.20)])
@MODES
def test_graph_alternating_parity(seed, n_side, eta, k, tfrac, mode):
    x, y, L, act = _square(seed, n_side, eta, k)
    T = tfrac * L
    dirs = [0, 1] * 4
    e = gpu_run(x, y, L, act, dirs, T, opts=mode)
    ref = oracle.run(x, y, 1.0, L, act, dirs, T)
    check_parity(e, ref, L, k, f"graph seed={seed}")


@pytest.mark.parametrize("window_micro,lanes", [(0, 64), (200_000, 64), (200_000, 16)])
@MODES
def test_graph_many_chains_with_violations(window_micro, lanes, mode):
    """k = 4 sqrt(N): violations, rollbacks and the ladder with graph candidates."""
    x, y, L, act = _square(111, 32, 0.70, 128)
    T = 0.2 * L
    dirs = [0, 1, 0, 1]
    e = gpu_run(x, y, L, act, dirs, T, lanes=lanes,
                opts=mode + ((pkg.OPT_WINDOW_MICRO, window_micro),))
    ref = oracle.run(x, y, 1.0, L, act, dirs, T)
    st = check_parity(e, ref, L, 128, f"graph k=128 w={window_micro} lanes={lanes}")
    print("graph violated legs", st["legs_violated"], "reruns", st["reruns"])


@pytest.mark.parametrize("flags", [pkg.FP64, pkg.FP32_MIXED])
@MODES
def test_graph_mid_size_parity(flags, mode):
    s = W.config(1)
    dirs = s.leg_dirs(4)
    e = gpu_run(s.x, s.y, s.L, s.active, dirs, s.T, flags=flags, log_cap=1 << 14,
                opts=mode + ((pkg.OPT_WINDOW_MICRO, 160_000),))
    ref = oracle.run(s.x, s.y, 1.0, s.L, s.active, dirs, s.T)
    check_parity(e, ref, s.L, s.k, "graph mid-size")


@MODES
def test_graph_forced_global_and_injected_violation(mode):
    s = W.config(1)
    dirs = s.leg_dirs(2)
    e = gpu_run(s.x, s.y, s.L, s.active, dirs, s.T, log_cap=1 << 14,
                opts=mode + ((pkg.OPT_INJECT_CHAIN, 3), (pkg.OPT_INJECT_EVENT, 40)))
    ref = oracle.run(s.x, s.y, 1.0, s.L, s.active, dirs, s.T)
    st = check_parity(e, ref, s.L, s.k, "graph injected")
    assert st["reruns"] >= 1


@MODES
def test_graph_headline_first_legs(mode):
    """The N = 2^20, k = 1024 workload in the benchmark's launch
    configuration (64 lanes, bounded lag 0.16 sigma) with graph candidates:
    two legs, +x then +y, against the oracle."""
    s = W.config(4)
    dirs = s.leg_dirs(2)
    e = gpu_run(s.x, s.y, s.L, s.active, dirs, s.T, log_cap=1 << 12,
                opts=mode + ((pkg.OPT_WINDOW_MICRO, 160_000),))
    ref = oracle.run(s.x, s.y, 1.0, s.L, s.active, dirs, s.T, log_cap=1 << 23)
    check_parity(e, ref, s.L, s.k, "graph headline")


def test_graph_time_reversal():
    s = W.config(1)
    e = pkg.Ecmc(np.stack([s.x, s.y], 1), s.sigma, s.L, max_chains=s.k, log_cap=1 << 16)
    e.set_option(pkg.OPT_NEIGHBOURS, pkg.NEIGHBOURS_GRAPH)
    e.set_active(s.active)
    e.run(s.T, s.T, pkg.DIR_Y)
    e.run(s.T, s.T, pkg.DIR_MY)
    pos = e.positions()
    tol = 1e-12 * s.L
    assert np.abs((pos[:, 0] - s.x + s.L / 2) % s.L - s.L / 2).max() <= tol
    assert np.abs((pos[:, 1] - s.y + s.L / 2) % s.L - s.L / 2).max() <= tol
    assert np.array_equal(e.active(), s.active)


def test_graph_batch_parity():
    """Replicas with graph candidates, each against the oracle."""
    reps = W.replica_batch(12)
    systems = []
    for r in reps:
        e = pkg.Ecmc(np.stack([r.x, r.y], 1), 1.0, r.L, flags=pkg.FP32_MIXED, max_chains=r.k,
                     log_cap=1 << 14)
        e.set_active(r.active)
        systems.append(e)
    b = pkg.Batch(systems)
    b.set_option(pkg.OPT_NEIGHBOURS, pkg.NEIGHBOURS_GRAPH)
    b.set_option(pkg.OPT_GRAPH, 1)
    b.set_option(pkg.OPT_LANES, 8)
    b.set_option(pkg.OPT_CELL_PCT, 115)
    b.set_option(pkg.OPT_WINDOW_MICRO, 350_000)
    big = np.full(len(reps), 1 << 60, np.int64)
    b.run(big, [r.T for r in reps], pkg.DIR_ALTERNATE, max_legs=2)
    for r, e in zip(reps, systems):
        ref = oracle.run(r.x, r.y, 1.0, r.L, r.active, r.leg_dirs(2), r.T, log_cap=1 << 22)
        st = e.stats()
        assert st["events"] == ref.n_events, r.name
        for c in range(r.k):
            assert np.array_equal(e.log(c).targets, ref.targets(c)), (r.name, c)
        pos = e.positions()
        assert np.array_equal(pos[:, 0], ref.x) and np.array_equal(pos[:, 1], ref.y), r.name
