"""Literal global-time ECMC (Alg. 2, Sec. 2.1) for tiny systems -- TEST ONLY.

Independent second implementation used to pin ``oracle.run``:

* positions are advanced eagerly: at every iteration *all* active disks move to
  the new global time, exactly as Alg. 2 states it;
* the time of flight is found geometrically, as the smallest non-negative root
  s of |x_i + s v - (x_j + image)|^2 = (2 sigma)^2 over explicit periodic
  images of j, with the discriminant written as (v.D)^2 - (|D|^2 - d^2);
* the minimum is taken over every (active i, static j) pair at every step
  (no caching, no cells).

It shares no arithmetic with ``ecmc_oracle.c``: the two agree on which disk is
lifted to at every event (exactly) and on times and positions up to rounding.
Cost is O(k N) per event: for N up to a few hundred.
"""
from __future__ import annotations

import numpy as np

_VEL = {0: (1.0, 0.0), 1: (0.0, 1.0), 2: (-1.0, 0.0), 3: (0.0, -1.0)}


def _contact_times(px, py, qx, qy, vx, vy, d, L):
    """Earliest s >= 0 at which a disk at (px,py) moving with (vx,vy) touches a
    static disk at (qx,qy), over periodic images; +inf if never (for s < L).

    px,py: shape (m,1); qx,qy: shape (1,n). Returns (s, b) of shape (m,n)."""
    best = np.full(np.broadcast(px, qx).shape, np.inf)
    bb = np.zeros_like(best)
    for n_img in (-1, 0, 1, 2):
        for m_img in (-1, 0, 1, 2):
            Dx = qx + n_img * L - px
            Dy = qy + m_img * L - py
            along = vx * Dx + vy * Dy
            disc = along * along - (Dx * Dx + Dy * Dy - d * d)
            ok = (along > 0.0) & (disc > 0.0)
            root = np.sqrt(np.where(ok, disc, 0.0))
            s = along - root
            # touching within rounding counts as an immediate contact
            s = np.where(ok & (s < 0.0) & (s > -1e-9 * L), 0.0, s)
            ok &= s >= 0.0
            better = ok & (s < best)
            best = np.where(better, s, best)
            bb = np.where(better, root, bb)
    return best, bb


def run(x, y, sigma, L, active, legs, T):
    """Return dict(x, y, active, chain, frm, to, time, b, contact, clearance,
    stamps); contact is the centre distance of the lifting pair at the lifting,
    clearance the smallest active-static distance at that moment."""
    x = np.array(x, dtype=np.float64)
    y = np.array(y, dtype=np.float64)
    act = [int(a) for a in active]
    n = x.shape[0]
    d = 2.0 * sigma
    log = {"chain": [], "frm": [], "to": [], "time": [], "b": [], "contact": [],
           "clearance": []}
    stamps = np.zeros(n)
    for code in legs:
        vx, vy = _VEL[int(code)]
        stamps[:] = 0.0
        t = 0.0
        while True:
            is_act = np.zeros(n, bool)
            is_act[act] = True
            stat = np.nonzero(~is_act)[0]
            if stat.size == 0 or len(act) == 0:
                s_min = np.inf
            else:
                ai = np.array(act)
                s, bmat = _contact_times(x[ai][:, None], y[ai][:, None],
                                         x[stat][None, :], y[stat][None, :], vx, vy, d, L)
                s_min = s.min()
            if not (t + s_min < T):
                step = T - t
                for i in act:
                    x[i] = (x[i] + step * vx) % L
                    y[i] = (y[i] + step * vy) % L
                for i in act:
                    stamps[i] = T
                break
            # ties: smallest chain index, then smallest disk id
            cands = np.argwhere(s == s_min)
            c, jj = min((int(r[0]), int(stat[r[1]])) for r in cands)
            b = float(bmat[c, np.searchsorted(stat, jj)])
            for i in act:
                x[i] = (x[i] + s_min * vx) % L
                y[i] = (y[i] + s_min * vy) % L
            t = t + s_min
            i = act[c]
            stamps[i] = t
            stamps[jj] = t
            # geometry at the lifting: i touches jj, and no active disk is
            # closer than contact to any static one
            dxm = (x[jj] - x[i] + L / 2) % L - L / 2
            dym = (y[jj] - y[i] + L / 2) % L - L / 2
            ai = np.array(act)
            ex = (x[stat][None, :] - x[ai][:, None] + L / 2) % L - L / 2
            ey = (y[stat][None, :] - y[ai][:, None] + L / 2) % L - L / 2
            log["contact"].append(float(np.hypot(dxm, dym)))
            log["clearance"].append(float(np.sqrt((ex * ex + ey * ey).min())))
            log["chain"].append(c); log["frm"].append(i); log["to"].append(jj)
            log["time"].append(t); log["b"].append(b)
            act[c] = jj
    out = {k: np.array(v) for k, v in log.items()}
    out.update(x=x, y=y, active=np.array(act, dtype=np.int32), stamps=stamps)
    return out
