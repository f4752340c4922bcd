"""Exact enumeration of every interleaving of the multithreaded algorithm on
tiny suites (Sec. 2.3, Alg. 5, Lemma 3), CPU only.

Each suite is a handful of disks with two threads (chains), built so that
every time of flight is an exact rational (contact distance 5, perpendicular
offsets 0, 3 or 4, positions in halves) and the binary64 oracle is exact too.
For the paper's sequential-consistency program and for the gfx950 kernel's
protocol (shared accesses between completion waits in any order) the tests
check that every state reaches an absorbing state, that P(terminate) +
P(abort) = 1 exactly, and that every terminate state carries the output of
the serial oracle (global-time Alg. 2): positions, local times, active set and
each chain's (target, time) sequence.  Then each single-statement mutation
(Remark on the CAS statement, Remark on lock-free programming, Remark on
memory-order directives, Remark on active-sphere necklaces) must break one of
these on at least one suite.
"""
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle
from oracle.enumerate_alg5 import Suite, enumerate_chain, reference_from_oracle

H = Fr(1, 2)
SUITES = {
    # two active disks in one lane of a ring: each one's target is the other
    # (Remark on active-sphere necklaces); no lifting, both move by T
    "necklace2": Suite("necklace2", Fr(24), 5 * H, (Fr(0), Fr(12)), (Fr(0), Fr(0)), (0, 1), Fr(10)),
    # three disks in one lane: chain 1 lifts to disk 2, then chain 0 lifts to
    # disk 1 once it has stopped (a re-check of the target's record matters)
    "row3": Suite("row3", Fr(24), 5 * H, (Fr(0), Fr(8), Fr(16)), (Fr(0), Fr(0), Fr(0)), (0, 1), Fr(10)),
    # two chains in different lanes aim at one static disk (CAS statement)
    "shared_target": Suite("shared_target", Fr(24), 5 * H, (Fr(0), Fr(1), Fr(8)), (Fr(0), Fr(6), Fr(3)),
                           (0, 1), Fr(10)),
    # disks 2 and 3 touch (a lifting 2 -> 3 has tau = 0); chains 0 and 1 aim
    # at disk 2 from two lanes, chain 1 first in global time.  A zero-tau
    # lifting leaves x_2 unchanged while t_2 moves: re-checking x alone is an
    # ABA hazard
    "zero_tau": Suite("zero_tau", Fr(24), 5 * H, (Fr(2), Fr(3), Fr(10), Fr(15)), (Fr(9), Fr(15), Fr(12), Fr(12)),
                      (0, 1), Fr(10)),
    # four disks, two chains (found by a seeded search over small suites):
    # writing a position before its local time lets a horizon check pass on a
    # half-written record
    "swap4": Suite("swap4", Fr(24), 5 * H, (17 * H, Fr(23), Fr(19), Fr(16)), (Fr(7), Fr(7), Fr(11), Fr(4)),
                   (2, 3), Fr(10)),
    # four disks, two chains (seeded search): a lane minimum that is not the
    # target changes between the scan and the claim; without re-reading it
    # after the claim the chain commits on a stale horizon set
    "lane4": Suite("lane4", Fr(24), 5 * H, (Fr(16), Fr(7), Fr(4), 21 * H), (Fr(11), Fr(8), Fr(0), Fr(4)),
                   (1, 2), Fr(10)),
    # two chains whose corridors never meet: no violation is possible
    "apart": Suite("apart", Fr(24), 5 * H, (Fr(0), Fr(8), Fr(3), Fr(13)), (Fr(0), Fr(0), Fr(12), Fr(12)),
                   (0, 2), Fr(10)),
}


def reference(s):
    r = oracle.run(np.array([float(v) for v in s.a]), np.array([float(v) for v in s.p]), float(s.sigma),
                   float(s.L), np.array(s.active), [oracle.DIR_PX], float(s.T))
    return reference_from_oracle(s, r)


_cache = {}


def outcome(name, program, mutation=None):
    key = (name, program, mutation)
    if key not in _cache:
        s = SUITES[name]
        _cache[key] = enumerate_chain(s, program, mutation, reference(s))
    return _cache[key]


def test_suites_are_exact_in_binary64():
    """The oracle's binary64 run on every suite is exact: its event times and
    positions are the suite's rationals (multiples of 1/2)."""
    for s in SUITES.values():
        ref = reference(s)
        for v in list(ref["a"]) + list(ref["t"]) + [e for lg in ref["logs"] for _, e in lg]:
            assert (v * 2).denominator == 1, (s.name, v)


# ---- the kernel's protocol ------------------------------------------------------
@pytest.mark.parametrize("name", ["necklace2", "row3", "shared_target", "zero_tau", "swap4", "lane4", "apart"])
def test_kernel_protocol_is_absorbing_and_matches_the_oracle(name):
    o = outcome(name, "kernel")
    assert o.absorbing, o.trapped
    assert o.p_abort + o.p_terminate == 1
    assert o.p_error == 0 and not o.invariant_errors
    assert not o.mismatched
    assert len(o.terminate) == 1 and o.p_terminate > 0      # one terminate state, reachable


def test_independent_chains_never_abort():
    o = outcome("apart", "kernel")
    assert o.p_abort == 0 and o.p_terminate == 1
    p = outcome("apart", "alg5")
    assert p.p_abort == 0 and p.p_terminate == 1


# ---- the paper's sequential-consistency program ------------------------------------
@pytest.mark.parametrize("name", ["row3", "shared_target", "swap4", "apart"])
def test_alg5_is_absorbing_and_matches_the_oracle(name):
    """Lemma 3 on our own suites: Alg. 5 terminates only in the output of Alg. 2."""
    o = outcome(name, "alg5")
    assert o.ok
    assert len(o.terminate) == 1 and o.p_terminate > 0


def test_alg5_deadlocks_on_a_necklace():
    """Remark on active-sphere necklaces: Alg. 5 restarts a thread whose target
    is active; on a ring of two active disks no state can reach an absorbing
    one.  The kernel moves up to contact after W failed claims and absorbs."""
    o = outcome("necklace2", "alg5")
    assert o.trapped == o.states and o.p_terminate == 0 and o.p_abort == 0
    assert outcome("necklace2", "kernel").absorbing


def test_alg5_x_recheck_misses_a_zero_tau_lifting():
    """Statement 13 re-checks the target's position only.  After a lifting
    with tau = 0 the target sits where it was with a later local time, and
    Alg. 5 can lift to it at an earlier time (a negative local-time update,
    against the Remark on positivity).  The kernel re-checks the local time
    too and stays exact on the same suite."""
    o = outcome("zero_tau", "alg5")
    assert "negative local-time update of the target" in o.invariant_errors
    assert o.p_error > 0
    assert outcome("zero_tau", "kernel").ok


# ---- mutations: each one is caught on some suite ------------------------------------
@pytest.mark.parametrize("program,mutation,name", [
    ("alg5", "split_cas", "shared_target"),      # Remark on the CAS statement
    ("alg5", "no_x_check", "row3"),              # Remark on lock-free programming
    ("alg5", "swap_15_16", "swap4"),             # Remark on memory-order directives
    ("kernel", "split_cas", "shared_target"),
    ("kernel", "no_aj_check", "row3"),
    ("kernel", "no_tj_check", "zero_tau"),
    ("kernel", "no_recheck", "row3"),
    ("kernel", "no_contact_move", "necklace2"),  # Remark on active-sphere necklaces
    ("kernel", "no_lane_recheck", "lane4"),
])
def test_mutation_is_caught(program, mutation, name):
    base = outcome(name, program)
    assert base.absorbing and not base.mismatched
    o = outcome(name, program, mutation)
    assert not o.ok, (program, mutation, name)
    assert o.trapped or o.mismatched or o.invariant_errors


def test_split_cas_activates_one_disk_on_two_chains():
    o = outcome("shared_target", "kernel", "split_cas")
    assert any(len(set(m["active"])) < 2 for m in o.mismatched) or \
        "lifting to a disk this thread does not own" in o.invariant_errors


def test_probabilities_are_exact_rationals():
    o = outcome("row3", "kernel")
    assert isinstance(o.p_terminate, Fr) and isinstance(o.p_abort, Fr)
    assert 0 < o.p_terminate < 1 and o.p_abort + o.p_terminate == 1


def test_exact_tie_between_chains_is_resolved_by_the_claim():
    """Two chains reach one static disk at exactly the same time (t = 11/2).
    The oracle breaks such ties by chain id (Alg. 2's heap order); the kernel
    lets whichever claim lands first lift, and equal times pass Eq. 2.  Both
    outcomes are liftings of Alg. 2 at the same time with a different tie
    order; exact ties have probability zero for generic positions (the paper
    assumes distinct event times), which is why the suites above have none."""
    s = Suite("tie", Fr(24), 5 * H, (33 * H, 31 * H, Fr(1)), (Fr(7), Fr(0), Fr(3)), (0, 1), Fr(6))
    ref = reference(s)
    assert ref["logs"] == [((2, 11 * H),), ()]
    o = enumerate_chain(s, "kernel", None, ref)
    assert o.absorbing and not o.invariant_errors and len(o.terminate) == 2
    assert len(o.mismatched) == 1 and o.mismatched[0]["logs"] == ((), ((2, 11 * H),))
