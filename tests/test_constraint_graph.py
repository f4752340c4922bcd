"""The constraint-graph oracle (Sec. 3.1-3.2) against definitions it does not
share code with: a literal per-pair loop for G(3), and the liftings of the
serial oracle, which must all be arrows of any valid graph built at the leg's
breakpoint (graph validation, Sec. 3.3)."""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import constraint_graph as CG


def _literal_g3(x, y, sigma, L, direction, horizon):
    """G(3) written out pair by pair in plain Python."""
    n = len(x)
    d = 2.0 * sigma
    out = [[-1, -1, -1] for _ in range(n)]
    best = [[(math.inf, n), (math.inf, n), (math.inf, n)] for _ in range(n)]
    for i in range(n):
        for j in range(n):
            if i == j:
                continue
            if direction % 2 == 0:
                ai, aj, pi, pj = x[i], x[j], y[i], y[j]
            else:
                ai, aj, pi, pj = y[i], y[j], x[i], x[j]
            dp = pj - pi
            if dp > L / 2:
                dp -= L
            elif dp < -L / 2:
                dp += L
            if not dp * dp < d * d:
                continue
            da = (aj - ai) if direction < 2 else (ai - aj)
            if da < 0:
                da += L
            tau = max(da - math.sqrt(d * d - dp * dp), 0.0)
            if horizon is not None and not tau < horizon:
                continue
            q = 0 if abs(dp) < sigma else (1 if dp > 0 else 2)
            if (tau, j) < best[i][q]:
                best[i][q] = (tau, j)
                out[i][q] = j
    return np.array(out)


@pytest.mark.parametrize("direction", [0, 1, 2, 3])
def test_g3_matches_the_literal_definition(direction):
    rng = np.random.Generator(np.random.PCG64(41 + direction))
    x, y, L = W.random_dilute(48, 0.45, rng)
    for horizon in (None, 4.0):
        A, _, _ = CG.g3(x, y, 1.0, L, direction, horizon)
        assert np.array_equal(A, _literal_g3(x, y, 1.0, L, direction, horizon))


def _graphs(x, y, s, d):
    A, b, _ = CG.g3(x, y, s.sigma, s.L, d, horizon=s.T)
    Am, bm, _ = CG.g3(x, y, s.sigma, s.L, (d + 2) % 4, horizon=s.T)
    P = CG.prune_first_order(x, y, s.sigma, s.L, A, b, d)
    Pm = CG.prune_first_order(x, y, s.sigma, s.L, Am, bm, (d + 2) % 4)
    return A, P, CG.symmetrize(P, Pm)


@pytest.mark.parametrize("cfg,legs", [(0, 3), (1, 4)])
def test_every_lifting_is_an_arrow(cfg, legs):
    """Every lifting of each leg is an arrow of G(3), of the first-order
    pruned graph and of the symmetrized graph built at its breakpoint; the
    pruned graphs are strictly smaller once the lattice has disordered."""
    s = W.config(cfg)
    x, y, act = s.x, s.y, s.active
    degs = []
    for d in s.leg_dirs(legs):
        A, P, S = _graphs(x, y, s, d)
        r = oracle.run(x, y, s.sigma, s.L, act, [d], s.T)
        for G in (A, P, S):
            cov, tot = CG.liftings_covered(G, r.log_from, r.log_to)
            assert cov == tot and tot > 0
        assert CG.out_degree(S) <= CG.out_degree(P) <= CG.out_degree(A) <= 3.0
        degs.append((CG.out_degree(A), CG.out_degree(S)))
        x, y, act = r.x, r.y, r.active
    if cfg == 1:
        assert degs[-1][1] < degs[-1][0]


def test_reversed_leg_uses_the_reversed_arrows():
    """A leg along -v from the end of a +v leg lifts j -> i for each i -> j of
    the +v leg (Remark on time-reversal invariance); those are arrows of the
    graph for -v built at that breakpoint."""
    s = W.config(1)
    fwd = oracle.run(s.x, s.y, s.sigma, s.L, s.active, [0], s.T)
    back = oracle.run(fwd.x, fwd.y, s.sigma, s.L, fwd.active, [2], s.T)
    assert {(int(i), int(j)) for i, j in zip(back.log_from, back.log_to)} == \
        {(int(j), int(i)) for i, j in zip(fwd.log_from, fwd.log_to)}
    A, P, S = _graphs(fwd.x, fwd.y, s, 2)
    for G in (A, P, S):
        cov, tot = CG.liftings_covered(G, back.log_from, back.log_to)
        assert cov == tot


def test_dilute_random_configurations():
    """Random dilute configurations (every lane geometry occurs), several
    chains and legs in all four directions."""
    for seed in range(3):
        rng = np.random.Generator(np.random.PCG64(500 + seed))
        x, y, L = W.random_dilute(200, 0.35, rng)
        act = W.active_set(rng, 200, 6)
        T = 0.2 * L
        for d in (0, 1, 2, 3):
            A, b, _ = CG.g3(x, y, 1.0, L, d, horizon=T)
            Am, bm, _ = CG.g3(x, y, 1.0, L, (d + 2) % 4, horizon=T)
            P = CG.prune_first_order(x, y, 1.0, L, A, b, d)
            S = CG.symmetrize(P, CG.prune_first_order(x, y, 1.0, L, Am, bm, (d + 2) % 4))
            r = oracle.run(x, y, 1.0, L, act, [d], T)
            for G in (A, P, S):
                cov, tot = CG.liftings_covered(G, r.log_from, r.log_to)
                assert cov == tot
            x, y, act = r.x, r.y, r.active
