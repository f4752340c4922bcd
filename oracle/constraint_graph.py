"""Constraint graphs of hard-disk ECMC between two breakpoints (Sec. 3.1-3.2).

TEST INFRASTRUCTURE, like the rest of ``oracle/``: only ``tests/`` use it.  It
shares no code with the GPU library.

Definitions followed (for a configuration C_h and velocity v; a is the
coordinate along v, p the one across it):

* ``g3``: the graph G(3).  Disk i has up to three out-arrows: to the disk j0
  with the smallest time of flight among disks in the corridor |dp| < sigma,
  to j+ among sigma <= dp < 2 sigma and to j- among -2 sigma < dp <= -sigma
  (Sec. 3.1).  Time of flight tau_ij = (forward distance along v) - b_ij,
  b_ij = sqrt(4 sigma^2 - dp^2), clamped at 0 (contact), ties to the smaller
  disk id.  Disks closer than 2 sigma in p cannot pass each other, so the
  arrows hold for the whole leg.  With ``horizon`` only arrows with
  tau < horizon are kept (a leg of that length cannot reach further).
* ``prune_first_order``: an arrow i -> k goes if i has another out-arrow
  i -> j with j behind k in k's corridor (so a_j <= a_k - b_jk for the whole
  leg) and b_ij + b_jk > b_ik: then a_i <= a_k - b_ik can never be tight, and
  i never lifts to k (Sec. 3.2, first-order pruning; the arrow j -> k itself
  is not needed).
* ``symmetrize``: keep i -> j of G(+v) only if j -> i is in G(-v), because
  the minimal graph satisfies G_min(v) = G_min(-v) with arrows reversed
  (Sec. 3.1, Remark on constraint graphs and irreducibility).
* ``liftings_covered``: every lifting i -> j of a leg must be an arrow of any
  valid constraint graph built at the leg's breakpoint (the paper's graph
  validation runs cell-based ECMC and checks exactly this).

Arrays: arrows (n, 3) int64 of target ids (-1: none), lanes in the order
(0, +, -); b (n, 3) float64.  Pure numpy brute force, O(n^2) per graph: for the
small and mid-size workloads only.
"""
from __future__ import annotations

import numpy as np

LANES = ("0", "+", "-")


def _axes(x, y, direction):
    """(a, p, sign): a along the velocity axis, p across it; sign of v."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    if direction not in (0, 1, 2, 3):
        raise ValueError("direction must be 0 (+x), 1 (+y), 2 (-x) or 3 (-y)")
    a, p = (x, y) if direction % 2 == 0 else (y, x)
    return a, p, (1.0 if direction < 2 else -1.0)


def _pair(a, p, sign, L, d, i, js):
    """dp (minimum image), forward distance and b from disk i to disks js."""
    dp = p[js] - p[i]
    dp = np.where(dp > 0.5 * L, dp - L, np.where(dp < -0.5 * L, dp + L, dp))
    da = (a[js] - a[i]) if sign > 0 else (a[i] - a[js])
    da = np.where(da < 0.0, da + L, da)
    with np.errstate(invalid="ignore"):
        b = np.sqrt(d * d - dp * dp)
    return dp, da, b


def g3(x, y, sigma, L, direction=0, horizon=None, rows=None):
    """G(3): (arrows, b, tau), each (n, 3), lanes (0, +, -).  With `rows`,
    only those disks' arrows are computed (the others stay -1)."""
    a, p, sign = _axes(x, y, direction)
    n = a.shape[0]
    d = 2.0 * sigma
    arrows = np.full((n, 3), -1, np.int64)
    bb = np.zeros((n, 3))
    tt = np.full((n, 3), np.inf)
    ids = np.arange(n)
    for i in (range(n) if rows is None else rows):
        js = ids[ids != i]
        dp, da, b = _pair(a, p, sign, L, d, i, js)
        inside = dp * dp < d * d
        tau = np.where(inside, np.maximum(da - b, 0.0), np.inf)
        lane = np.where(np.abs(dp) < sigma, 0, np.where(dp > 0.0, 1, 2))
        for q in range(3):
            m = inside & (lane == q)
            if horizon is not None:
                m &= tau < horizon
            if not m.any():
                continue
            cand = np.flatnonzero(m)
            best = cand[np.lexsort((js[cand], tau[cand]))[0]]   # smallest (tau, id)
            arrows[i, q] = js[best]
            bb[i, q] = b[best]
            tt[i, q] = tau[best]
    return arrows, bb, tt


def prune_first_order(x, y, sigma, L, arrows, b, direction=0):
    """Arrows of G(3) left after first-order pruning (same layout, pruned
    entries set to -1)."""
    a, p, sign = _axes(x, y, direction)
    d = 2.0 * sigma
    out = arrows.copy()
    n = arrows.shape[0]
    for i in range(n):
        for qk in range(3):
            k = arrows[i, qk]
            if k < 0:
                continue
            _, da_ik, _ = _pair(a, p, sign, L, d, i, np.array([k]))
            for qj in range(3):
                j = arrows[i, qj]
                if j < 0 or qj == qk or j == k:
                    continue
                _, da_ij, _ = _pair(a, p, sign, L, d, i, np.array([j]))
                dp_jk, da_jk, b_jk = _pair(a, p, sign, L, d, j, np.array([k]))
                # j behind k in k's corridor: a_j <= a_k - b_jk for the whole leg
                if not (dp_jk[0] ** 2 < d * d and da_ij[0] < da_ik[0] and da_jk[0] >= b_jk[0]):
                    continue
                if b[i, qj] + b_jk[0] > b[i, qk]:
                    out[i, qk] = -1
                    break
    return out


def arrow_set(arrows):
    return {(int(i), int(j)) for i, row in enumerate(arrows) for j in row if j >= 0}


def symmetrize(arrows_plus, arrows_minus):
    """Arrows i -> j of G(+v) whose reverse j -> i is an arrow of G(-v)."""
    back = arrow_set(arrows_minus)
    out = arrows_plus.copy()
    for i in range(out.shape[0]):
        for q in range(3):
            j = out[i, q]
            if j >= 0 and (int(j), i) not in back:
                out[i, q] = -1
    return out


def out_degree(arrows):
    return float((arrows >= 0).sum()) / max(arrows.shape[0], 1)


def liftings_covered(arrows, log_from, log_to):
    """(covered, total): liftings i -> j of one leg that are arrows."""
    s = arrow_set(arrows)
    pairs = list(zip(np.asarray(log_from).tolist(), np.asarray(log_to).tolist()))
    return sum((i, j) in s for i, j in pairs), len(pairs)
