"""Exact enumeration of every interleaving of multithreaded ECMC on tiny suites.

TEST INFRASTRUCTURE.  Like the rest of ``oracle/``, only ``tests/`` may use
this module; it shares no code with the GPU library and never calls it.

What it computes (Sec. 2.3, Alg. 5 and Lemma 3).  The multithreading stage of
the multithreaded algorithm is a finite Markov chain when the initial
configuration is fixed: a state is every disk's tag, position and local time
plus every thread's program counter and local variables; a step lets a
randomly chosen thread execute its next statement.  The chain has two kinds
of absorbing states: *abort* (a thread found a horizon violation, Eq. 2) and
*terminate* (every thread reached its wait).  This module builds every state
reachable from the initial one, with exact rational arithmetic, and checks:

* every state can reach an absorbing state (the chain is absorbing), so
  P(terminate) + P(abort) = 1, computed exactly;
* every terminate state carries the output of global-time ECMC (Alg. 2):
  the same positions, local times, active set and, per chain, the same
  sequence of (target, lifting time).  The reference output is supplied by
  the caller (the tests pass the serial C oracle's result), so the oracle is
  pinned by an independent model of the multithreaded algorithm.

Two programs are modelled.

``alg5``    the paper's sequential-consistency model as stated in Sec. 2.3:
            one statement per step, in the paper's statement order (scan all
            other disks, reading each disk's position and then checking its
            local time; claim with a compare-and-swap; re-check the target's
            position; write the target's local time, the moving disk's local
            time, its position, release its tag; or stall at h').

``kernel``  the protocol of the gfx950 event kernel in this repository, one
            shared-memory access per step.  Accesses that the kernel issues
            without a completion wait between them may take effect in any
            order (same-address accesses keep program order), which models
            relaxed atomics ordered only by waits:
              scan    loads of (a, t) of every other disk, except the one
                      that stopped at the chain's last lifting (it sits at
                      contact behind, out of reach within a leg);
              Eq. 2   on the nearest disk of each lane of the corridor;
              stall   t_i <- h'; wait; a_i <- a_i + rest; wait; tag <- stalled;
              claim   {t_i <- t_i + tau, CAS(tag_j, static -> c)}; wait;
              won     {re-read a_j, t_j, the lane minima, and the next scan};
                      a lane minimum whose record changed is checked again
                      (Eq. 2 on the new record: a violation; ahead of the
                      target: scan again); a_j or t_j changed: restore t_i,
                      wait, release tag_j, scan again;
              commit  {t_j <- t_i + tau, a_i <- a_i + tau}; wait; tag_i <- static;
              lost    restore t_i; a stalled target is a violation; after W
                      failed claims, re-read the lane minima and, if they
                      still pass Eq. 2, publish a move up to contact:
                      t_i <- t + tau; wait; a_i <- a + tau (Remark on
                      active-sphere necklaces).

Mutations (``mutation=``) reorder or drop single statements (Remark on the
CAS statement, Remark on lock-free programming, Remark on memory-order
directives, Remark on active-sphere necklaces); the tests show that each one
breaks one of the checks above on at least one suite.

Geometry is exact: suites use a contact distance d and perpendicular offsets
whose b = sqrt(d^2 - dp^2) is rational (d = 5 with dp in {0, +-3, +-4}), and
positions that are multiples of a power of two, so binary64 arithmetic in the
C oracle is exact as well and agreement is checked with ``==``.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field
from fractions import Fraction as Fr

INF = math.inf
STATIC, STALLED = -1, -2  # tags; a tag >= 0 names the thread that owns the disk
ABORT = "abort"


class Invariant(str):
    """A transition that breaks a property every correct run keeps: a lifting
    to a disk the thread does not own (Remark on the CAS statement), or a
    negative update of the target's local time (Remark on positivity)."""


def invariant(msg: str) -> Invariant:
    return Invariant(msg)


# ---------------------------------------------------------------------------
# suites and exact geometry
# ---------------------------------------------------------------------------
@dataclass(frozen=True)
class Suite:
    """Disks in a periodic square box of side L, velocity +x (a = x, p = y)."""
    name: str
    L: Fr
    sigma: Fr                 # radius; contact distance d = 2 sigma
    a: tuple                  # coordinates along v
    p: tuple                  # perpendicular coordinates
    active: tuple             # disk of each thread
    T: Fr                     # leg length h' - h (h = 0)

    @property
    def n(self) -> int:
        return len(self.a)

    @property
    def d(self) -> Fr:
        return 2 * self.sigma


def _exact_sqrt(q: Fr) -> Fr:
    n, m = q.numerator, q.denominator
    rn, rm = math.isqrt(n), math.isqrt(m)
    if rn * rn != n or rm * rm != m:
        raise ValueError(f"sqrt({q}) is irrational: choose offsets with rational b")
    return Fr(rn, rm)


class Geometry:
    """Time of flight (Sec. 2.2): tau_ij = forward distance - b_ij, b_ij =
    sqrt(d^2 - dp^2), dp the minimum image, the forward distance in [0, L),
    a negative tau (contact) clamped to 0; outside the corridor tau = inf.

    Every length and time is held as an integer multiple of 1/S, S the least
    common denominator of the suite's rationals (and of the b_ij), so that
    the arithmetic stays exact and cheap."""

    def __init__(self, s: Suite):
        L, d, sigma = Fr(s.L), Fr(s.d), Fr(s.sigma)
        p = tuple(Fr(v) for v in s.p)
        n = s.n
        bs = []
        for i in range(n):
            for j in range(n):
                if i != j:
                    dp = p[j] - p[i]
                    if dp > L / 2:
                        dp -= L
                    elif dp < -L / 2:
                        dp += L
                    if dp * dp < d * d:
                        bs.append(_exact_sqrt(d * d - dp * dp))
        S = 1
        for v in (L, d, sigma, Fr(s.T), *map(Fr, s.a), *p, *bs):
            S = S * v.denominator // math.gcd(S, v.denominator)
        self.S = S
        self.L, self.d, self.sigma, self.T = int(L * S), int(d * S), int(sigma * S), int(Fr(s.T) * S)
        self.p = tuple(int(v * S) for v in p)
        self.a0 = tuple(int(Fr(v) * S) for v in s.a)
        self.dp = [[None] * n for _ in range(n)]
        self.b = [[None] * n for _ in range(n)]
        for i in range(n):
            for j in range(n):
                if i == j:
                    continue
                dp = self.p[j] - self.p[i]
                if 2 * dp > self.L:
                    dp -= self.L
                elif 2 * dp < -self.L:
                    dp += self.L
                self.dp[i][j] = dp
                if dp * dp < self.d * self.d:
                    self.b[i][j] = int(_exact_sqrt(Fr(self.d * self.d - dp * dp)))

    def tof(self, i: int, ai, j: int, aj):
        b = self.b[i][j]
        if b is None:
            return INF
        da = aj - ai
        if da < 0:
            da += self.L
        tau = da - b
        return tau if tau > 0 else 0

    def lane(self, i: int, j: int) -> int:
        """Lane of the corridor: 0 |dp| < sigma, 1 sigma <= dp, 2 dp <= -sigma."""
        dp = self.dp[i][j]
        if abs(dp) < self.sigma:
            return 0
        return 1 if dp > 0 else 2

    def fwd(self, a, dist):
        r = a + dist
        if r >= self.L:
            r -= self.L
        return r


# ---------------------------------------------------------------------------
# shared memory: per disk (tag, a, t) at indices 3q, 3q+1, 3q+2
# ---------------------------------------------------------------------------
def _tag(q):
    return 3 * q


def _pos(q):
    return 3 * q + 1


def _time(q):
    return 3 * q + 2


# ---------------------------------------------------------------------------
# program: the paper's sequential-consistency model (Sec. 2.3)
# thread state: (pc, i, tau, j, x, dist, idx, x_nbr, tau_nbr, log)
# ---------------------------------------------------------------------------
class Alg5:
    MUTATIONS = ("swap_15_16", "split_cas", "no_x_check")

    def __init__(self, s: Suite, mutation: str | None = None):
        if mutation is not None and mutation not in self.MUTATIONS:
            raise ValueError(mutation)
        self.s, self.g, self.mut = s, Geometry(s), mutation

    def init_thread(self, c: int):
        return (1, self.s.active[c], None, None, None, self.g.T, 0, None, None, ())

    def is_wait(self, th) -> bool:
        return th[0] == 26

    def project(self, th):
        return (26, th[1], None, None, None, None, None, None, None, th[9])

    def step(self, c: int, th, mem: list):
        """Execute the statement at th's program counter; returns the new
        thread state, or ABORT.  mem is modified in place."""
        g, s = self.g, self.s
        pc, i, tau, j, x, dist, idx, xn, taun, log = th
        others = [q for q in range(s.n) if q != i]
        if pc == 1:
            return (2, i, dist, i, INF, dist, 0, None, None, log)
        if pc == 2:  # for nbr in {1..n} \ i
            if idx < len(others):
                return (3, i, tau, j, x, dist, idx, None, None, log)
            return (10, i, tau, j, x, dist, idx, None, None, log)
        nbr = others[idx] if idx < len(others) else None
        if pc == 3:  # x_nbr <- nbr.x
            return (4, i, tau, j, x, dist, idx, mem[_pos(nbr)], None, log)
        if pc == 4:  # tau_inbr <- x_nbr - i.x - b_inbr
            return (5, i, tau, j, x, dist, idx, xn, g.tof(i, mem[_pos(i)], nbr, xn), log)
        if pc == 5:  # horizon condition, Eq. 2
            if taun != INF and mem[_time(i)] + taun < mem[_time(nbr)]:
                return ABORT
            return (6, i, tau, j, x, dist, idx, xn, taun, log)
        if pc == 6:
            if taun < tau:
                return (7, i, tau, j, x, dist, idx, xn, taun, log)
            return (2, i, tau, j, x, dist, idx + 1, None, None, log)
        if pc == 7:
            return (8, i, tau, nbr, x, dist, idx, xn, taun, log)
        if pc == 8:
            return (9, i, tau, j, xn, dist, idx, xn, taun, log)
        if pc == 9:
            return (2, i, taun, j, x, dist, idx + 1, None, None, log)
        if pc == 10:  # CAS(static -> c) on j's tag
            if self.mut == "split_cas":
                return (101 if mem[_tag(j)] == STATIC else 11, i, tau, j, x, dist, idx, None, None, log)
            if mem[_tag(j)] == STATIC:
                mem[_tag(j)] = c
            return (11, i, tau, j, x, dist, idx, None, None, log)
        if pc == 101:  # second half of a split CAS
            mem[_tag(j)] = c
            return (11, i, tau, j, x, dist, idx, None, None, log)
        if pc == 11:
            if mem[_tag(j)] == c:
                return (12, i, tau, j, x, dist, idx, None, None, log)
            return (1, i, None, None, None, dist, 0, None, None, log)
        if pc == 12:
            return ((13 if tau < dist else 21), i, tau, j, x, dist, idx, None, None, log)
        if pc == 13:
            if self.mut == "no_x_check" or x == mem[_pos(j)]:
                return (14, i, tau, j, x, dist, idx, None, None, log)
            return (20, i, tau, j, x, dist, idx, None, None, log)
        if pc == 14:
            if mem[_tag(j)] != c:
                return invariant("lifting to a disk this thread does not own")
            if mem[_time(i)] + tau < mem[_time(j)]:
                return invariant("negative local-time update of the target")
            mem[_time(j)] = mem[_time(i)] + tau
            return ((16 if self.mut == "swap_15_16" else 15), i, tau, j, x, dist, idx, None, None, log)
        if pc == 15:
            mem[_time(i)] = mem[_time(i)] + tau
            nxt = 17 if self.mut == "swap_15_16" else 16
            return (nxt, i, tau, j, x, dist, idx, None, None, log)
        if pc == 16:
            mem[_pos(i)] = g.fwd(mem[_pos(i)], tau)
            nxt = 15 if self.mut == "swap_15_16" else 17
            return (nxt, i, tau, j, x, dist, idx, None, None, log)
        if pc == 17:
            mem[_tag(i)] = STATIC
            return (18, i, tau, j, x, dist, idx, None, None, log)
        if pc == 18:
            return (19, i, tau, j, x, dist - tau, idx, None, None, log)
        if pc == 19:  # i <- j; the lifting (target, time) joins the chain's log
            return (25, j, None, None, None, dist, 0, None, None, log + ((j, mem[_time(j)]),))
        if pc == 20:
            mem[_tag(j)] = STATIC
            return (1, i, None, None, None, dist, 0, None, None, log)
        if pc == 21:
            mem[_time(i)] = mem[_time(i)] + tau
            return (22, i, tau, j, x, dist, idx, None, None, log)
        if pc == 22:
            mem[_pos(i)] = g.fwd(mem[_pos(i)], tau)
            return (23, i, tau, j, x, dist, idx, None, None, log)
        if pc == 23:
            return (24, i, tau, j, x, 0, idx, None, None, log)
        if pc == 24:
            mem[_tag(i)] = STALLED
            return (25, i, None, None, None, dist, 0, None, None, log)
        if pc == 25:
            if dist > 0:
                return (1, i, None, None, None, dist, 0, None, None, log)
            return (26, i, None, None, None, None, None, None, None, log)
        raise AssertionError(pc)

    def arm(self, th, mem):
        return th

    def moves(self, c: int, threads: tuple, mem: tuple):
        """Successors when thread c moves: list of (weight, threads or ABORT /
        Invariant, mem)."""
        m = list(mem)
        r = self.step(c, threads[c], m)
        if isinstance(r, str):
            return [(1, r, None)]
        return [(1, threads[:c] + (r,) + threads[c + 1:], tuple(m))]


# ---------------------------------------------------------------------------
# program: the gfx950 event kernel's protocol, one shared access per step
# thread state: (phase, i, aref, tref, tpub, retries, xs, pend, seen, ctx, log)
#   pend: pending stores and compare-and-swaps of the current group,
#         ('st', addr, value) | ('cas', addr, expected, new); a new group also
#         lists its loads as ('ld', addr) until arm() turns them into `seen`
#   seen: for every load of the group, the values its address has held since
#         the group began (the load may take effect at any moment before the
#         group ends); for a performed CAS (key -1 - addr) the value it found
#   ctx:  phase-specific locals
# A group ends with a step of its own once its stores and CAS have been
# performed: each load then takes one of the values it could have seen.  This
# gives exactly the outcomes of loads performed one by one in any order,
# without a state for every subset of performed loads.
# ---------------------------------------------------------------------------
class Kernel:
    MUTATIONS = ("pos_before_time", "split_cas", "no_aj_check", "no_tj_check", "no_recheck",
                 "no_contact_move", "no_lane_recheck")

    def __init__(self, s: Suite, mutation: str | None = None, wait_retries: int = 2):
        if mutation is not None and mutation not in self.MUTATIONS:
            raise ValueError(mutation)
        self.s, self.g, self.mut = s, Geometry(s), mutation
        self.W = wait_retries

    # -- helpers -------------------------------------------------------------
    def _scan_loads(self, i, xs):
        ops = []
        for q in range(self.s.n):
            if q != i and q != xs:
                ops.append(("ld", _pos(q)))
                ops.append(("ld", _time(q)))
        return ops

    def init_thread(self, c: int):
        i = self.s.active[c]
        return ("scan", i, self.g.a0[i], 0, 0, 0, -1,
                tuple(self._scan_loads(i, -1)), (), (), ())

    def arm(self, th, mem):
        """Move the loads of a new group into `seen`, each with the value its
        address holds now."""
        if isinstance(th, str) or not any(op[0] == "ld" for op in th[7]):
            return th
        seen = dict(th[8])
        rest = []
        for op in th[7]:
            if op[0] == "ld":
                seen[op[1]] = (mem[op[1]],)
            else:
                rest.append(op)
        return th[:7] + (tuple(rest), tuple(sorted(seen.items()))) + th[9:]

    def is_wait(self, th) -> bool:
        return th[0] == "wait" and not th[7] and not th[8]

    def project(self, th):
        return ("wait", th[1], None, None, None, None, None, (), (), (), th[10])

    def _scan_result(self, c, th, vals, carry):
        """Local computation after a scan: lane minima, Eq. 2, target; returns
        the next thread state (with its first access group) or ABORT."""
        g, s = self.g, self.s
        _, i, aref, tref, tpub, retries, xs, _, _, _, log = th
        T = g.T
        trem = T - tref
        best = [(INF, 1 << 30, None, None)] * 3  # (tau, id, a, t) per lane
        for q in range(s.n):
            if q == i or q == xs:
                continue
            aq, tq = vals[_pos(q)], vals[_time(q)]
            tau = g.tof(i, aref, q, aq)
            if tau == INF:
                continue
            if tref + tau < tq and tq <= 0:  # came to rest behind before the attempt began (h = 0)
                continue
            ln = g.lane(i, q)
            if (tau, q) < best[ln][:2]:
                best[ln] = (tau, q, aq, tq)
        # horizon condition (Eq. 2) on the lane minima whose lifting falls before h'
        for tau, q, aq, tq in best:
            if tau != INF and tau < trem and tref + tau < tq:
                return ABORT
        tau, j, aj, tj = min(best, key=lambda e: (e[0], e[1]))
        lanes = tuple((b[1], b[2], b[3]) for b in best if b[0] != INF and b[0] < trem)
        if not (tau < trem):  # stall at h' (Remark on stalled spheres)
            pend = tuple(carry) + (("st", _time(i), T),)
            return ("stall1", i, aref, tref, tpub, retries, xs, pend, (), (g.fwd(aref, trem),), log)
        ctx = (tau, j, aj, tj, lanes)
        if self.mut == "split_cas":
            pend = tuple(carry) + (("st", _time(i), tref + tau), ("ld", _tag(j)))
            return ("cas_test", i, aref, tref, tpub, retries, xs, pend, (), ctx, log)
        if self.mut == "pos_before_time":
            pend = tuple(carry) + (("cas", _tag(j), STATIC, c),)
        else:
            pend = tuple(carry) + (("st", _time(i), tref + tau), ("cas", _tag(j), STATIC, c))
        return ("claim", i, aref, tref, tpub, retries, xs, pend, (), ctx, log)

    def _rescan(self, th, carry=(), **upd):
        phase, i, aref, tref, tpub, retries, xs, pend, got, ctx, log = th
        retries = upd.get("retries", retries)
        tpub = upd.get("tpub", tpub)
        pend = tuple(carry) + tuple(self._scan_loads(i, xs))
        return ("scan", i, aref, tref, tpub, retries, xs, pend, (), (), log)

    def _group_done(self, c, th, mem, vals):
        """The current group completed with load results `vals`: run the local
        code that follows."""
        g, s = self.g, self.s
        phase, i, aref, tref, tpub, retries, xs, pend, got, ctx, log = th
        if phase == "scan":
            return self._scan_result(c, th, vals, ())
        if phase == "stall1":  # wait; a_i <- a_i + (h' - t_i)
            return ("stall2", i, aref, tref, tpub, retries, xs, (("st", _pos(i), ctx[0]),), (), (), log)
        if phase == "stall2":  # wait; tag <- stalled
            return ("wait", i, aref, tref, tpub, retries, xs, (("st", _tag(i), STALLED),), (), (), log)
        if phase == "wait":
            return ("wait", i, aref, tref, tpub, retries, xs, (), (), (), log)
        if phase == "cas_test":  # split CAS: test ...
            tau, j = ctx[0], ctx[1]
            if vals[_tag(j)] == STATIC:
                return ("cas_set", i, aref, tref, tpub, retries, xs, (("st", _tag(j), c),), (), ctx, log)
            return self._claim_result(c, th, won=False, old=vals[_tag(j)])
        if phase == "cas_set":  # ... and set
            return self._claim_result(c, th, won=True, old=STATIC)
        if phase == "claim":
            j = ctx[1]
            old = vals[-1 - _tag(j)]
            return self._claim_result(c, th, won=(old == STATIC), old=old)
        if phase == "post":
            return self._post_claim(c, th, vals, mem)
        if phase == "commit":  # wait; release the tag of the disk that stopped
            nxt_vals = dict(ctx[1])
            oi = ctx[0]
            carry = (("st", _tag(oi), STATIC),)
            return self._scan_result(c, th, nxt_vals, carry)
        if phase == "commit_t":  # pos_before_time: wait; t_i <- e; wait; release
            oi = ctx[0]
            return ("commit_rel", i, aref, tref, tpub, retries, xs, (("st", _time(oi), ctx[2]),), (),
                    ctx, log)
        if phase == "commit_rel":
            oi = ctx[0]
            return self._scan_result(c, th, dict(ctx[1]), (("st", _tag(oi), STATIC),))
        if phase == "giveback":  # restore of t_i completed; release the target, scan again
            j = ctx[0]
            return self._rescan(th, carry=(("st", _tag(j), STATIC),))
        if phase == "move_check":  # restore completed; re-read the lane minima
            tau, j, aj, tj, lanes = ctx
            ops = []
            for q, _, _ in lanes:
                ops += [("ld", _pos(q)), ("ld", _time(q))]
            return ("move_read", i, aref, tref, tpub, 0, xs, tuple(ops), (), ctx, log)
        if phase == "move_read":
            tau, j, aj, tj, lanes = ctx
            for q, _, _ in lanes:
                if tref + g.tof(i, aref, q, vals[_pos(q)]) < vals[_time(q)]:
                    return self._rescan(th, retries=0)  # left to the next scan
            tn = tref + tau
            return ("move_t", i, aref, tref, tpub, 0, xs, (("st", _time(i), tn),), (), ctx, log)
        if phase == "move_t":  # wait; a_i <- a + tau; then scan again (no wait)
            tau = ctx[0]
            carry = (("st", _pos(i), g.fwd(aref, tau)),)
            return self._rescan(th, carry=carry, retries=0, tpub=tref + tau)
        raise AssertionError(phase)

    def _claim_result(self, c, th, won, old):
        g = self.g
        phase, i, aref, tref, tpub, retries, xs, pend, got, ctx, log = th
        tau, j, aj, tj, lanes = ctx
        if not won:
            restore = () if self.mut == "pos_before_time" else (("st", _time(i), tpub),)
            if old == STALLED:  # it waits at h' with t = h', reached earlier: Eq. 2 fails
                return ABORT
            if self.mut != "no_contact_move":  # (without the move there is nothing to count)
                retries += 1
            if self.mut != "no_contact_move" and retries >= self.W:
                if tref + tau > tpub:
                    return ("move_check", i, aref, tref, tpub, 0, xs, restore, (), ctx, log)
                retries = 0
            return self._rescan(th, carry=restore, retries=retries)
        ops = [("ld", _pos(j)), ("ld", _time(j))]
        if self.mut != "no_lane_recheck":
            for q, _, _ in lanes:
                if q != j:
                    ops += [("ld", _pos(q)), ("ld", _time(q))]
        # the next scan's loads are issued with the post-claim reads (prefetch):
        # every disk but the new moving disk j and the disk i that will stop
        for q in range(self.s.n):
            if q != i and q != j:
                for a in (("ld", _pos(q)), ("ld", _time(q))):
                    if a not in ops:
                        ops.append(a)
        return ("post", i, aref, tref, tpub, retries, xs, tuple(ops), (), ctx, log)

    def _post_claim(self, c, th, vals, mem):
        g = self.g
        phase, i, aref, tref, tpub, retries, xs, pend, got, ctx, log = th
        tau, j, aj, tj, lanes = ctx
        aj2, tj2 = vals[_pos(j)], vals[_time(j)]
        stale = 0
        if self.mut != "no_lane_recheck":
            for q, aq, tq in lanes:
                if q == j:
                    continue
                aq2, tq2 = vals[_pos(q)], vals[_time(q)]
                if aq2 != aq or tq2 != tq:
                    tq_new = g.tof(i, aref, q, aq2)
                    if tref + tq_new < tq2:
                        stale = 2
                    elif (tq_new, q) < (tau, j) and stale == 0:
                        stale = 1
        if stale == 2:
            return ABORT
        changed = (aj2 != aj and self.mut not in ("no_aj_check", "no_recheck")) or \
                  (tj2 != tj and self.mut not in ("no_tj_check", "no_recheck"))
        if changed or stale:
            restore = () if self.mut == "pos_before_time" else (("st", _time(i), tpub),)
            if not restore:
                return self._rescan(th, carry=(("st", _tag(j), STATIC),))
            return ("giveback", i, aref, tref, tpub, retries, xs, restore, (), (j,), log)
        # commit the lifting (Eq. 1): t_j <- e, a_i <- a_i + tau; the chain continues with j
        e = tref + tau
        if mem[_tag(j)] != c:
            return invariant("lifting to a disk this thread does not own")
        if e < mem[_time(j)]:
            return invariant("negative local-time update of the target")
        nxt = tuple(sorted((k, v) for k, v in vals.items() if k >= 0))
        nlog = log + ((j, e),)
        if self.mut == "pos_before_time":
            pend = (("st", _time(j), e), ("st", _pos(i), g.fwd(aref, tau)))
            return ("commit_t", j, aj2, e, e, 0, i, pend, (), (i, nxt, e), nlog)
        pend = (("st", _time(j), e), ("st", _pos(i), g.fwd(aref, tau)))
        return ("commit", j, aj2, e, e, 0, i, pend, (), (i, nxt), nlog)

    def _finish(self, c, th, mem, vals):
        """Run the code after a completed group, then the groups that have no
        accesses, and arm the next group's loads."""
        nth = self._group_done(c, th, mem, vals)
        while not isinstance(nth, str) and not nth[7] and not nth[8] and nth[0] != "wait":
            nth = self._group_done(c, nth, mem, {})
        return self.arm(nth, mem)

    def moves(self, c: int, threads: tuple, mem: tuple):
        th = threads[c]
        pend, seen = th[7], th[8]
        if not pend and not seen:
            if th[0] == "wait":
                return []
            raise AssertionError(th)
        out = []
        if pend:
            done = set()
            for k, op in enumerate(pend):
                addr = op[1]
                if addr in done:
                    continue  # an earlier access to the same address goes first
                done.add(addr)
                m = list(mem)
                nseen = dict(seen)
                written = None
                if op[0] == "st":
                    m[addr] = op[2]
                    written = op[2]
                else:  # compare-and-swap
                    old = m[addr]
                    if old == op[2]:
                        m[addr] = op[3]
                        written = op[3]
                    nseen[-1 - addr] = (old,)
                rest = pend[:k] + pend[k + 1:]
                nth = th[:7] + (rest, tuple(sorted(nseen.items()))) + th[9:]
                m = tuple(m)
                if not rest and all(key < 0 for key in nseen):  # nothing left to load
                    nth = self._finish(c, nth, m, {key: v[0] for key, v in nseen.items()})
                if isinstance(nth, str):
                    out.append((nth, None))
                    continue
                nthreads = list(threads)
                nthreads[c] = nth
                if written is not None:  # loads of other threads in flight may see the new value
                    for d in range(len(threads)):
                        if d != c:
                            nthreads[d] = _observe(nthreads[d], addr, written)
                out.append((tuple(nthreads), m))
        else:
            keys = [key for key, _ in seen]
            for combo in itertools.product(*[v for _, v in seen]):
                nth = self._finish(c, th[:7] + ((), ()) + th[9:], mem, dict(zip(keys, combo)))
                if isinstance(nth, str):
                    out.append((nth, None))
                else:
                    out.append((threads[:c] + (nth,) + threads[c + 1:], mem))
        w = Fr(1, len(out))
        return [(w, r, m) for r, m in out]


def _observe(th, addr, value):
    """A store to addr became visible: a pending load of addr may return it."""
    seen = th[8]
    if not seen or not isinstance(seen[0], tuple):
        return th
    for q, (key, vals) in enumerate(seen):
        if key == addr:
            if value in vals:
                return th
            nv = tuple(sorted(vals + (value,)))
            return th[:8] + (seen[:q] + ((key, nv),) + seen[q + 1:],) + th[9:]
    return th


# ---------------------------------------------------------------------------
# the Markov chain
# ---------------------------------------------------------------------------
@dataclass
class Outcome:
    states: int
    terminate: dict                     # projected terminate state -> probability
    p_abort: Fr
    p_terminate: Fr
    p_error: Fr                         # probability of a transition that breaks an invariant
    trapped: int                        # states that cannot reach an absorbing state
    mismatched: list = field(default_factory=list)   # terminate outputs that differ from the reference
    invariant_errors: list = field(default_factory=list)

    @property
    def absorbing(self) -> bool:
        return self.trapped == 0

    @property
    def ok(self) -> bool:
        return (self.absorbing and not self.mismatched and not self.invariant_errors
                and self.p_error == 0 and self.p_abort + self.p_terminate == 1)


def initial_memory(s: Suite, g: Geometry) -> tuple:
    mem = []
    for q in range(s.n):
        mem += [s.active.index(q) if q in s.active else STATIC, g.a0[q], 0]
    return tuple(mem)


def output_of(s: Suite, mem: tuple, threads: tuple, S: int) -> dict:
    """The output of a terminate state (Alg. 1 output): positions, local
    times, active set (disk owned by each chain at the end) and the logs,
    as exact rationals."""
    a = tuple(Fr(mem[_pos(q)], S) for q in range(s.n))
    t = tuple(Fr(mem[_time(q)], S) for q in range(s.n))
    logs = tuple(tuple((j, Fr(e, S)) for j, e in th[-1]) for th in threads)
    active = tuple(th[1] for th in threads)
    return {"a": a, "t": t, "tags": tuple(mem[_tag(q)] for q in range(s.n)),
            "active": active, "logs": logs}


def enumerate_chain(s: Suite, program: str = "kernel", mutation: str | None = None,
                    reference: dict | None = None, max_states: int = 2_000_000,
                    wait_retries: int = 2) -> Outcome:
    """Build every state reachable from the initial lifted configuration and
    solve the absorbing chain exactly.  ``reference`` is the expected output
    (keys a, t, active, logs as produced by ``output_of``); every terminate
    state is compared with it."""
    prog = Alg5(s, mutation) if program == "alg5" else Kernel(s, mutation, wait_retries)
    k = len(s.active)
    mem0 = initial_memory(s, prog.g)
    init = (mem0, tuple(prog.arm(prog.init_thread(c), mem0) for c in range(k)))
    index = {init: 0}
    states = [init]
    succ: list = []   # per state: list of (prob, target id) ; target -1 = abort
    term_of: dict = {}   # state id -> projected output key
    errors: list = []    # (message, state) of transitions that break an invariant
    frontier = [0]
    while frontier:
        sid = frontier.pop()
        mem, threads = states[sid]
        while len(succ) <= sid:
            succ.append(None)
        live = [c for c in range(k) if not prog.is_wait(threads[c])]
        if not live:
            term_of[sid] = None
            succ[sid] = []
            continue
        edges = {}
        for c in live:
            for w, r, nmem in prog.moves(c, threads, mem):
                pr = Fr(w) / len(live)  # the switch picks a thread that can move
                if isinstance(r, Invariant):
                    errors.append((str(r), states[sid]))
                    edges[-2] = edges.get(-2, 0) + pr
                    continue
                if r == ABORT:
                    edges[-1] = edges.get(-1, 0) + pr
                    continue
                r = tuple(prog.project(t) if prog.is_wait(t) else t for t in r)
                nst = (nmem, r)
                nid = index.get(nst)
                if nid is None:
                    nid = len(states)
                    if nid >= max_states:
                        raise RuntimeError(f"more than {max_states} states")
                    index[nst] = nid
                    states.append(nst)
                    frontier.append(nid)
                edges[nid] = edges.get(nid, 0) + pr
        succ[sid] = sorted(edges.items())
    while len(succ) < len(states):
        succ.append([])
    n = len(states)

    # terminate states and their outputs
    outcome_key = {}
    mismatched, inv = [], []
    for sid in term_of:
        mem, threads = states[sid]
        out = output_of(s, mem, threads, prog.g.S)
        key = (out["a"], out["t"], out["tags"], out["active"], out["logs"])
        outcome_key[sid] = key
        # invariants: k distinct active disks, all stalled at h', every tag consistent
        if len(set(out["active"])) != k:
            inv.append(("active set not k distinct disks", out["active"]))
        for q in range(s.n):
            tag = out["tags"][q]
            if (q in out["active"]) != (tag == STALLED):
                inv.append(("tag of disk %d" % q, tag))
        if reference is not None:
            ref = (tuple(reference["a"]), tuple(reference["t"]), tuple(reference["active"]),
                   tuple(tuple(x) for x in reference["logs"]))
            if (out["a"], out["t"], out["active"], out["logs"]) != ref:
                mismatched.append(out)

    # states that can reach an absorbing state (reverse reachability)
    pred = [[] for _ in range(n)]
    reach_abort = []
    for v in range(n):
        for t_, pr in succ[v]:
            if t_ < 0:
                reach_abort.append(v)
            else:
                pred[t_].append(v)
    good = [False] * n
    stack = list(term_of) + reach_abort
    for v in stack:
        good[v] = True
    while stack:
        v = stack.pop()
        for u in pred[v]:
            if not good[u]:
                good[u] = True
                stack.append(u)
    trapped = n - sum(good)

    # exact absorption probabilities, strongly connected components in reverse
    # topological order (Tarjan, iterative)
    p_abort = [None] * n
    p_term = [None] * n
    p_err = [None] * n
    p_each = [None] * n   # per terminate key
    keys = sorted(set(outcome_key.values()), key=repr)
    kidx = {kk: q for q, kk in enumerate(keys)}
    nk = len(keys)

    def solve_scc(comp):
        if len(comp) == 1:
            v = comp[0]
            if v in outcome_key:
                p_abort[v], p_term[v], p_err[v] = Fr(0), Fr(1), Fr(0)
                p_each[v] = [Fr(int(q == kidx[outcome_key[v]])) for q in range(nk)]
                return
            if all(t_ != v for t_, _ in succ[v]):
                pa = pt = pe = Fr(0)
                pk = [Fr(0)] * nk
                for t_, pr in succ[v]:
                    if t_ == -1:
                        pa += pr
                    elif t_ == -2:
                        pe += pr
                    else:
                        pa += pr * p_abort[t_]
                        pt += pr * p_term[t_]
                        pe += pr * p_err[t_]
                        for q in range(nk):
                            if p_each[t_][q]:
                                pk[q] += pr * p_each[t_][q]
                p_abort[v], p_term[v], p_err[v], p_each[v] = pa, pt, pe, pk
                return
        cset = set(comp)
        loc = {v: q for q, v in enumerate(comp)}
        m = len(comp)
        # x_v = sum_{u in comp} P_vu x_u + r_v   =>   (I - Q) x = r
        A = [[Fr(0)] * m for _ in range(m)]
        R = [[Fr(0)] * (3 + nk) for _ in range(m)]
        for v in comp:
            r = loc[v]
            A[r][r] += 1
            if v in outcome_key:
                R[r][1] = Fr(1)
                R[r][2 + kidx[outcome_key[v]]] = Fr(1)
                continue
            for t_, pr in succ[v]:
                if t_ == -2:
                    R[r][2 + nk] += pr
                elif t_ == -1:
                    R[r][0] += pr
                elif t_ in cset:
                    A[r][loc[t_]] -= pr
                else:
                    R[r][0] += pr * p_abort[t_]
                    R[r][1] += pr * p_term[t_]
                    R[r][2 + nk] += pr * p_err[t_]
                    for q in range(nk):
                        if p_each[t_][q]:
                            R[r][2 + q] += pr * p_each[t_][q]
        # Gaussian elimination (I - Q is nonsingular when the component can leave;
        # a closed non-absorbing component is singular: its states are trapped)
        singular = False
        for col in range(m):
            piv = next((r for r in range(col, m) if A[r][col] != 0), None)
            if piv is None:
                singular = True
                break
            A[col], A[piv] = A[piv], A[col]
            R[col], R[piv] = R[piv], R[col]
            inv_p = 1 / A[col][col]
            rowc = A[col]
            rc = R[col]
            for r in range(m):
                if r != col and A[r][col] != 0:
                    f = A[r][col] * inv_p
                    rowr = A[r]
                    for cc in range(col, m):
                        if rowc[cc]:
                            rowr[cc] -= f * rowc[cc]
                    rr = R[r]
                    for cc in range(3 + nk):
                        if rc[cc]:
                            rr[cc] -= f * rc[cc]
        for v in comp:
            r = loc[v]
            if singular or not good[v]:
                p_abort[v], p_term[v], p_err[v], p_each[v] = Fr(0), Fr(0), Fr(0), [Fr(0)] * nk
            else:
                d = A[r][r]
                p_abort[v] = R[r][0] / d
                p_term[v] = R[r][1] / d
                p_err[v] = R[r][2 + nk] / d
                p_each[v] = [R[r][2 + q] / d for q in range(nk)]

    # Tarjan
    idx = [-1] * n
    low = [0] * n
    onst = [False] * n
    st = []
    counter = 0
    for root in range(n):
        if idx[root] != -1:
            continue
        work = [(root, 0)]
        while work:
            v, pi = work[-1]
            if pi == 0:
                idx[v] = low[v] = counter
                counter += 1
                st.append(v)
                onst[v] = True
            edges_v = [t_ for t_, _ in succ[v] if t_ >= 0]
            advanced = False
            while pi < len(edges_v):
                w = edges_v[pi]
                pi += 1
                if idx[w] == -1:
                    work[-1] = (v, pi)
                    work.append((w, 0))
                    advanced = True
                    break
                if onst[w]:
                    low[v] = min(low[v], idx[w])
            if advanced:
                continue
            work.pop()
            if work:
                u = work[-1][0]
                low[u] = min(low[u], low[v])
            if low[v] == idx[v]:
                comp = []
                while True:
                    w = st.pop()
                    onst[w] = False
                    comp.append(w)
                    if w == v:
                        break
                solve_scc(comp)

    term_probs = {keys[q]: p_each[0][q] for q in range(nk)}
    inv += [m for m, _ in errors]
    return Outcome(states=n, terminate=term_probs, p_abort=p_abort[0], p_terminate=p_term[0],
                   p_error=p_err[0], trapped=trapped, mismatched=mismatched, invariant_errors=inv)


def reference_from_oracle(s: Suite, res) -> dict:
    """Turn an ``oracle.run`` result for the suite (one leg along +x) into the
    form of ``output_of``: exact rationals of the binary64 values."""
    k = len(s.active)
    logs = []
    for c in range(k):
        tg = res.targets(c)
        tm = res.times(c)
        logs.append(tuple((int(j), Fr(float(e))) for j, e in zip(tg, tm)))
    return {"a": [Fr(float(v)) for v in res.x], "t": [Fr(float(v)) for v in res.stamps],
            "active": [int(v) for v in res.active], "logs": logs}
