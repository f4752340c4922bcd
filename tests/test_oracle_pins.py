"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test names the passage of the paper (Li, Todo, Maggs, Krauth) or the
textbook result it relies on:

* literal Alg. 2 (eager positions, explicit periodic images)  -> same liftings
* brute-force scan over all disks                              -> bit-identical
* one row of disks = 1-D hard rods on a ring                   -> closed form
* k disks move at unit speed at every instant                   -> sum of moves
* all disks active (k = N)                                      -> no lifting
* time-reversal invariance (Remark 3)                          -> inverse run
* positivity of local-time updates (Remark 2), meaning of local
  times (Remark 1), no overlaps                                -> invariants
* global balance (Lemma 1) via the low-density virial series   -> statistics
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import literal_alg2


def _small_system(seed, n_side=6, eta=0.5, amp=0.1, k=3):
    rng = np.random.Generator(np.random.PCG64(seed))
    a = W.box_side(n_side * n_side, eta) / n_side
    amp = min(amp, 0.45 * (a - 2.0))          # jitter that cannot create overlaps
    x, y, L = W.square_jittered(n_side, eta, amp, rng)
    assert W.min_distance(x, y, L) > 2.0
    act = W.active_set(rng, n_side * n_side, k)
    return x, y, L, act


def _wrapdiff(a, b, L):
    return np.abs((a - b + L / 2) % L - L / 2)


# ---------------------------------------------------------------------------
# Alg. 2 written literally (eager positions, geometric contact times)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed,n_side,eta,k,legs,tfrac", [
    (11, 5, 0.40, 1, [0, 1, 2, 3], 0.45),
    (12, 6, 0.50, 3, [0, 1, 2, 3, 0, 1], 0.30),
    (13, 6, 0.65, 4, [1, 0, 3, 2], 0.25),
    (14, 7, 0.30, 5, [0, 0, 1, 1], 0.40),
    (15, 8, 0.70, 2, [0, 1, 0, 1, 0, 1, 0, 1], 0.20),
    (16, 4, 0.55, 16, [0, 1], 0.30),   # every disk active
])
def test_matches_literal_alg2(seed, n_side, eta, k, legs, tfrac):
    x, y, L, act = _small_system(seed, n_side, eta, 0.08, k)
    T = tfrac * L
    ro = oracle.run(x, y, 1.0, L, act, legs, T)
    rl = literal_alg2.run(x, y, 1.0, L, act, legs, T)
    assert ro.n_events == len(rl["to"])
    assert np.array_equal(ro.log_chain, rl["chain"])
    assert np.array_equal(ro.log_from, rl["frm"])
    assert np.array_equal(ro.log_to, rl["to"])
    if ro.n_events:
        np.testing.assert_allclose(ro.log_time, rl["time"], rtol=0, atol=1e-9)
        np.testing.assert_allclose(ro.log_b, rl["b"], rtol=0, atol=1e-7)
    assert _wrapdiff(ro.x, rl["x"], L).max() < 1e-9
    assert _wrapdiff(ro.y, rl["y"], L).max() < 1e-9
    assert np.array_equal(ro.active, rl["active"])
    np.testing.assert_allclose(ro.stamps, rl["stamps"], atol=1e-9)


def test_literal_liftings_are_contacts():
    """Geometric check of the literal run itself: at every lifting the pair is
    exactly one contact distance apart (Eq. 1: in-state at contact) and no
    active disk is closer than contact to any static disk."""
    x, y, L, act = _small_system(21, 7, 0.6, 0.08, 4)
    rl = literal_alg2.run(x, y, 1.0, L, act, [0, 1, 2, 3], 0.3 * L)
    assert len(rl["to"]) > 20
    np.testing.assert_allclose(rl["contact"], 2.0, atol=1e-9)
    assert np.min(rl["clearance"]) > 2.0 - 1e-9


# ---------------------------------------------------------------------------
# Cell search versus visiting every disk: identical arithmetic, identical bits
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("case", ["cfg0", "small_all_dirs", "dilute", "cfg1_prefix"])
def test_cells_equal_bruteforce(case):
    if case == "cfg0":
        s = W.config(0)
        x, y, L, act, legs, T = s.x, s.y, s.L, s.active, [0] * 8, s.T
    elif case == "small_all_dirs":
        x, y, L, act = _small_system(31, 10, 0.6, 0.1, 6)
        legs, T = [0, 1, 2, 3] * 3, 0.3 * L
    elif case == "dilute":
        rng = np.random.Generator(np.random.PCG64(32))
        x, y, L = W.random_dilute(120, 0.08, rng)
        act = W.active_set(rng, 120, 5)
        legs, T = [0, 1, 2, 3, 1, 0], 0.4 * L
    else:
        s = W.config(1)
        x, y, L, act, legs, T = s.x, s.y, s.L, s.active, [0, 1], s.T
    a = oracle.run(x, y, 1.0, L, act, legs, T, mode=0)
    b = oracle.run(x, y, 1.0, L, act, legs, T, mode=1)
    assert a.n_events == b.n_events > 0
    for f in ("log_chain", "log_from", "log_to", "log_time", "log_b", "x", "y",
              "active", "sum_b", "stamps"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f


# ---------------------------------------------------------------------------
# One row of disks: 1-D hard rods on a ring.  Every pair on the row has
# dp = 0, so b = 2 sigma exactly and each flight consumes the gap in front of
# the moving disk.  Closed form: let a_0 be the first active disk and g_l the
# initial gap in front of a_l (l-th disk after a_0 in ring order), free =
# L - N 2 sigma.  Each full turn of the lifting label (N liftings) costs
# free plus the gap the turn starts with, and the gaps rotate by one disk per
# turn, so the (m N)-th lifting happens at m * free + g_0 + ... + g_{m-1}.
# ---------------------------------------------------------------------------
def _ring_reference(xs, L, a0, T, d=2.0):
    """1-D hard-rod ring, one moving rod at a time (exact gap bookkeeping)."""
    x = [float(v) for v in xs]
    n = len(x)
    order = sorted(range(n), key=lambda i: x[i])
    nxt = {order[m]: order[(m + 1) % n] for m in range(n)}
    t, a, times, targets = 0.0, a0, [], []
    while True:
        j = nxt[a]
        gap = (x[j] - x[a]) % L - d
        if not (t + gap < T):
            break
        x[a] = (x[a] + gap) % L
        t += gap
        times.append(t)
        targets.append(j)
        a = j
    return np.array(targets), np.array(times)


@pytest.mark.parametrize("n_row,L,turns", [(10, 40.0, 3), (7, 31.5, 5), (25, 80.0, 2)])
def test_one_row_hard_rods(n_row, L, turns):
    rng = np.random.Generator(np.random.PCG64(40 + n_row))
    x, y = W.tonks_row(n_row, L, rng)
    free = L - n_row * 2.0
    a0 = 3
    order = sorted(range(n_row), key=lambda i: x[i])
    pos = order.index(a0)
    ring = [order[(pos + l) % n_row] for l in range(n_row)]
    gaps = [((x[ring[(l + 1) % n_row]] - x[ring[l]]) % L) - 2.0 for l in range(n_row)]
    t_turn = [m * free + sum(gaps[:m]) for m in range(1, turns + 1)]
    T = t_turn[-1] + 1e-6
    r = oracle.run(x, y, 1.0, L, np.array([a0], np.int32), [0], T)
    assert r.n_events == turns * n_row
    for m in range(1, turns + 1):
        assert abs(r.log_time[m * n_row - 1] - t_turn[m - 1]) < 1e-9
    assert np.all(r.log_b == 2.0)
    ref_t, ref_time = _ring_reference(x, L, a0, T)
    assert np.array_equal(r.log_to, ref_t)
    np.testing.assert_allclose(r.log_time, ref_time, atol=1e-9)
    # exactly one disk moves at unit speed at any time: displacements add to T
    # (forward displacement of each disk; none of them travels a full lap here)
    fwd = (r.x - x) % L
    assert fwd.max() < L - 4.0
    assert abs(fwd.sum() - T) < 1e-9
    assert np.all(y == r.y)


def test_total_displacement_is_k_times_T():
    """With k chains, k disks move at unit speed at every instant (Alg. 1), so
    the displacements along v add up to k (h' - h) in every leg."""
    s = W.config(1)
    r = oracle.run(s.x, s.y, 1.0, s.L, s.active, [0], s.T)
    dx = (r.x - s.x) % s.L          # +x leg: every displacement is forward
    assert abs(dx.sum() - s.k * s.T) < 1e-8 * s.k * s.T
    assert np.array_equal(r.y, s.y)


# ---------------------------------------------------------------------------
# k = N: no static disk is left, nothing can be lifted to (j not in A in
# Alg. 2); every disk moves by exactly T.
# ---------------------------------------------------------------------------
def test_all_disks_active():
    x, y, L, _ = _small_system(51, 5, 0.5, 0.1, 1)
    act = np.arange(25, dtype=np.int32)
    r = oracle.run(x, y, 1.0, L, act, [0, 1], 0.2 * L)
    assert r.n_events == 0
    assert _wrapdiff(r.x, np.mod(x + 0.2 * L, L), L).max() < 1e-12
    assert _wrapdiff(r.y, np.mod(y + 0.2 * L, L), L).max() < 1e-12


def test_single_chain_zero_length_leg():
    x, y, L, act = _small_system(52, 5, 0.5, 0.1, 2)
    r = oracle.run(x, y, 1.0, L, act, [0], 0.0)
    assert r.n_events == 0 and np.array_equal(r.x, x) and np.array_equal(r.y, y)


# ---------------------------------------------------------------------------
# Time-reversal invariance (Remark 3): running -v from the final lifted
# configuration retraces the run; the lifting set is the same with arrows
# reversed and times mirrored (t -> T - t).
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed,direction", [(61, 0), (62, 1), (63, 0)])
def test_time_reversal(seed, direction):
    rng = np.random.Generator(np.random.PCG64(seed))
    x, y, L = W.centred_rect_jittered(12, 12, 0.62, 0.08, rng)
    act = W.active_set(rng, 144, 4)
    T = 0.35 * L
    fwd = oracle.run(x, y, 1.0, L, act, [direction], T)
    back = oracle.run(fwd.x, fwd.y, 1.0, L, fwd.active, [direction + 2], T)
    assert fwd.n_events == back.n_events > 10
    assert np.array_equal(np.sort(act), np.sort(back.active))
    assert _wrapdiff(back.x, x, L).max() < 1e-9
    assert _wrapdiff(back.y, y, L).max() < 1e-9
    f = sorted((int(i), int(j), round(t, 7)) for i, j, t in zip(fwd.log_from, fwd.log_to, fwd.log_time))
    b = sorted((int(j), int(i), round(T - t, 7)) for i, j, t in zip(back.log_from, back.log_to, back.log_time))
    assert f == b


# ---------------------------------------------------------------------------
# Invariants: positivity of local-time updates (Remark 2), local times of
# active disks equal h' and of static disks are below it (Remark 1), exactly k
# distinct active disks, no overlaps beyond rounding of contact positions.
# ---------------------------------------------------------------------------
def test_invariants_over_many_legs():
    s = W.config(1)
    legs = s.leg_dirs(6)
    r = oracle.run(s.x, s.y, 1.0, s.L, s.active, legs, s.T)
    assert len(set(r.active.tolist())) == s.k
    ulp = math.ulp(s.L)
    assert oracle.overlaps(r.x, r.y, 1.0, s.L, 4 * ulp) == 0
    # positivity: within a leg, a target's local time strictly increases at
    # the lifting (it last changed when the disk last stopped or started).
    # Global time is non-decreasing along the log inside one leg.
    leg_starts = [0] + [m for m in range(1, r.n_events) if r.log_time[m] < r.log_time[m - 1]]
    assert len(leg_starts) == 6
    bounds = leg_starts + [r.n_events]
    for a, b in zip(bounds[:-1], bounds[1:]):
        last = {}
        for i, j, t in zip(r.log_from[a:b], r.log_to[a:b], r.log_time[a:b]):
            assert t > last.get(int(j), 0.0)
            last[int(i)] = t
            last[int(j)] = t
    T = s.T
    is_act = np.zeros(s.n, bool)
    is_act[r.active] = True
    assert np.all(r.stamps[is_act] == T)
    assert np.all(r.stamps[~is_act] < T)


def test_overlap_counter_counts_planted_overlap():
    x, y, L, _ = _small_system(71, 6, 0.5, 0.05, 1)
    assert oracle.overlaps(x, y, 1.0, L) == 0
    x2 = x.copy()
    x2[7] = (x[6] + 1.5) % L      # row neighbours at distance 1.5 < 2
    y2 = y.copy()
    y2[7] = y[6]
    assert oracle.overlaps(x2, y2, 1.0, L) >= 1


# ---------------------------------------------------------------------------
# Global balance (Lemma 1) checked statistically: the ECMC pressure estimator
# beta P / rho = 1 + sum(b) / (k * total chain time) must reproduce the
# low-density virial series of hard disks,
#   1 + 2 eta + 3.12802 eta^2 + 4.25785 eta^3 + O(eta^4)
# (B3/B2^2 = 4/3 - sqrt(3)/pi and B4/B2^3 = 2 - 9 sqrt(3)/(2 pi) + 10/pi^2 are
# exact textbook values; the eta^4 term is below 4e-5 at eta = 0.05).
# ---------------------------------------------------------------------------
def _virial(eta):
    b3 = 4.0 * (4.0 / 3.0 - math.sqrt(3.0) / math.pi)
    b4 = 8.0 * (2.0 - 9.0 * math.sqrt(3.0) / (2.0 * math.pi) + 10.0 / math.pi ** 2)
    return 1.0 + 2.0 * eta + b3 * eta ** 2 + b4 * eta ** 3


# One chain (k = 1): the classic single-chain estimator.  With k > 1 an
# active disk never collides with the other k - 1 active disks, so the raw
# estimator's excess is lower by a factor close to (N - k)/(N - 1); that is a
# property of the estimator, checked separately below, not of the dynamics.
@pytest.mark.parametrize("eta,n,seed", [(0.05, 512, 81), (0.10, 512, 82)])
def test_pressure_matches_virial_series(eta, n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    x, y, L = W.random_dilute(n, eta, rng)
    act = W.active_set(rng, n, 1)
    T = 0.45 * L
    n_batches, legs_per_batch = 60, 100
    est = []
    xs, ys, a = x, y, act
    for bi in range(n_batches):
        r = oracle.run(xs, ys, 1.0, L, a, [0, 1] * (legs_per_batch // 2), T, log=False)
        est.append(1.0 + r.sum_b.sum() / (legs_per_batch * T))
        xs, ys, a = r.x, r.y, r.active
    est = np.array(est[3:])                      # drop the first batches
    mean = est.mean()
    err = est.std(ddof=1) / math.sqrt(est.size)
    ref = _virial(eta)
    # truncation (next terms ~ 5.34 eta^4) and finite-N (excess / N) allowance
    slack = 6.0 * eta ** 4 + (ref - 1.0) / n
    assert err < 0.003
    assert abs(mean - ref) < 3.5 * err + slack, (mean, err, ref)
    # far from the ideal gas and from the first-order value
    assert mean - 1.0 > 1.5 * eta


def test_multichain_estimator_scaling():
    """k chains at fixed (N, eta): after scaling the excess by (N-1)/(N-k) the
    estimates for k = 1 and k = 16 agree (statistical, 4 sigma)."""
    eta, n = 0.08, 256
    vals = {}
    for k in (1, 16):
        rng = np.random.Generator(np.random.PCG64(99))
        x, y, L = W.random_dilute(n, eta, rng)
        act = W.active_set(rng, n, k)
        T = 0.45 * L
        est, xs, ys, a = [], x, y, act
        for bi in range(60 if k == 16 else 150):
            r = oracle.run(xs, ys, 1.0, L, a, [0, 1] * 50, T, log=False)
            est.append(r.sum_b.sum() / (k * 100 * T) * (n - 1) / (n - k))
            xs, ys, a = r.x, r.y, r.active
        e = np.array(est[3:])
        vals[k] = (e.mean(), e.std(ddof=1) / math.sqrt(e.size))
    (m1, e1), (m16, e16) = vals[1], vals[16]
    assert abs(m1 - m16) < 4.0 * math.hypot(e1, e16), vals
