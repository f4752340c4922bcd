"""A production loop (Sec. 3.4, closing paragraph on production codes): v
changes between breakpoints by a direction the caller draws for every leg,
and the constraint graph is rebuilt for each new v (Sec. 3.1).  Against the
oracle run with the same sequence of directions (Lemma 2), through
ecmc_run_directions.

Legs along -x and -y run on the reflected coordinate, which rounds once per
disk and leg (as in the time-reversal test).  Over many legs the collisions
amplify those roundings: a perpendicular offset perturbed by e changes b by
about e dp / b, large near grazing contacts, and every later lifting of the
disk carries it on (measured: up to 8e-12 L after 12 legs at 4096 disks,
1.6e-12 L after 16 legs at 256, 3e-13 L after 8 legs at 65536).  So the
contract is: event counts, every chain's lifting sequence and the active set
bit-exact (every decision taken the same way); positions and local times
within 1e-9 L and per-chain sums of b within 1e-9 relative, two orders of
magnitude above what was measured.
"""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2004_11040_amd as pkg  # noqa: E402


def check(e, ref, s, tag):
    st = e.stats()
    assert st["events"] == ref.n_events, (tag, st["events"], ref.n_events)
    for c in range(s.k):
        assert np.array_equal(e.log(c).targets, ref.targets(c)), (tag, c)
    assert np.array_equal(e.active(), ref.active), tag
    sb, _ = e.chain_sums()
    assert np.all(np.abs(sb - ref.sum_b) <= 1e-9 * np.abs(ref.sum_b)), (tag, sb - ref.sum_b)
    pos = e.positions()
    wrap = lambda a, b: np.abs((a - b + s.L / 2) % s.L - s.L / 2)  # noqa: E731
    tol = 1e-9 * s.L
    dx, dy = float(wrap(pos[:, 0], ref.x).max()), float(wrap(pos[:, 1], ref.y).max())
    dt = float(np.abs(e.stamps() - ref.stamps).max())
    db = float(np.max(np.abs(sb - ref.sum_b) / np.abs(ref.sum_b)))
    print(f"[directions] {tag}: max |dx| {dx:.3g} |dy| {dy:.3g} |dt| {dt:.3g} (L {s.L:.4g}), sum b rel {db:.3g}",
          flush=True)
    assert dx <= tol and dy <= tol and dt <= tol, (tag, dx, dy, dt)
    return st


def _dirs(seed, n):
    return np.random.Generator(np.random.PCG64(seed)).integers(0, 4, n).astype(np.int32)


def _ctx(s, flags, neighbours, window_micro, log_cap):
    e = pkg.Ecmc(np.stack([s.x, s.y], 1), s.sigma, s.L, flags=flags, max_chains=s.k, log_cap=log_cap)
    e.set_option(pkg.OPT_NEIGHBOURS, neighbours)
    e.set_option(pkg.OPT_WINDOW_MICRO, window_micro)
    e.set_active(s.active)
    return e


@pytest.mark.parametrize("neighbours", [pkg.NEIGHBOURS_GRAPH, pkg.NEIGHBOURS_CELLS], ids=["graph", "cells"])
@pytest.mark.parametrize("cfg,n_legs,seed", [(0, 16, 1), (1, 12, 2)])
def test_resampled_directions_match_the_oracle(cfg, n_legs, seed, neighbours):
    s = W.config(cfg)
    dirs = _dirs(seed, n_legs)
    assert len(set(dirs.tolist())) == 4
    e = _ctx(s, pkg.FP64, neighbours, 160_000, 1 << 14)
    e.run_directions(s.T, dirs)
    ref = oracle.run(s.x, s.y, s.sigma, s.L, s.active, dirs.tolist(), s.T)
    st = check(e, ref, s, f"cfg={cfg} directions")
    assert st["legs"] == n_legs and e.overlaps() == 0


def test_resampled_directions_at_65536_disks_both_forms():
    s = W.config(2)
    dirs = _dirs(3, 8)
    ref = oracle.run(s.x, s.y, s.sigma, s.L, s.active, dirs.tolist(), s.T, log_cap=1 << 23)
    for flags, neighbours in ((pkg.FP64, pkg.NEIGHBOURS_GRAPH), (pkg.FP32_MIXED, pkg.NEIGHBOURS_CELLS)):
        e = _ctx(s, flags, neighbours, 160_000, 1 << 13)
        e.run_directions(s.T, dirs)
        check(e, ref, s, f"N=65536 directions flags={flags}")


def test_direction_arguments_are_checked():
    s = W.config(0)
    e = _ctx(s, pkg.FP64, pkg.NEIGHBOURS_GRAPH, 0, 16)
    for bad in ([0, 4], [-1], [1, 2, 5]):
        with pytest.raises(pkg.EcmcError) as ei:
            e.run_directions(s.T, bad)
        assert ei.value.code == pkg.EINVAL
    with pytest.raises(pkg.EcmcError):
        e.run_directions(0.0, [0])
    e.run_directions(s.T, [])          # no legs: nothing happens
    assert e.stats()["legs"] == 0
