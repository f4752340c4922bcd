"""CPU model of the event kernel's wavefront reductions (64 lanes), lane by lane.

The lane minima of a scan pass are reduced with VALU cross-lane moves: DPP
quad permutations [1,0,3,2] and [2,3,0,1], DPP row rotations by 4 and by 8
inside rows of 16 lanes, then the gfx950 row swaps (permlane16_swap: the odd
rows of the first operand trade places with the even rows of the second;
permlane32_swap: the upper half of the first with the lower half of the
second).  With the FP32-mixed filter a lane of the corridor mostly keeps one
candidate; the kernel then reads that lane with readlane instead of reducing.

These tests restate the moves as index maps (the lane layouts were checked on
the GPU with an in-bounds probe) and check, for random and adversarial
inputs, that (a) every lane ends with the wavefront minimum, (b) the 64-bit
minimum taken on 32-bit halves moved together equals the lexicographic one,
(c) the smallest id among the lanes holding the minimum time wins, and
(d) the single-candidate readlane path gives what the full reduction gives.
They also show two layout mistakes that a variant could make, each failing
(a): reading a row's minimum from its first lane after shifts instead of
rotations, and combining the two 32-bit halves of a key independently.
"""
import numpy as np
import pytest

LANES = 64


def quad_perm(x, perm):
    idx = np.arange(LANES)
    return x[(idx & ~3) + np.array(perm)[idx & 3]]


def row_ror(x, n):
    """Rotate right by n inside each row of 16: lane i reads lane i - n."""
    idx = np.arange(LANES)
    return x[(idx & ~15) + ((idx - n) & 15)]


def row_shr(x, n, old):
    """Shift right by n inside each row (bound_ctrl off): lanes 0..n-1 of a
    row have no source and keep `old`."""
    idx = np.arange(LANES)
    src = idx - n
    valid = (idx & 15) >= n
    return np.where(valid, x[np.clip(src, 0, LANES - 1)], old)


def permlane16_swap(a, b):
    """Returns (a', b'): odd rows of a swapped with even rows of b."""
    a2, b2 = a.copy(), b.copy()
    for r in (0, 2):
        a2[(r + 1) * 16:(r + 2) * 16] = b[r * 16:(r + 1) * 16]
        b2[r * 16:(r + 1) * 16] = a[(r + 1) * 16:(r + 2) * 16]
    return a2, b2


def permlane32_swap(a, b):
    a2, b2 = a.copy(), b.copy()
    a2[32:] = b[:32]
    b2[:32] = a[32:]
    return a2, b2


def wave_umin(x):
    """The kernel's wave_umin32/wave_umin64 on one array of keys."""
    x = np.minimum(x, quad_perm(x, [1, 0, 3, 2]))
    x = np.minimum(x, quad_perm(x, [2, 3, 0, 1]))
    x = np.minimum(x, row_ror(x, 4))
    x = np.minimum(x, row_ror(x, 8))
    a, b = permlane16_swap(x, x)
    x = np.minimum(a, b)
    a, b = permlane32_swap(x, x)
    return np.minimum(a, b)


def wave_umin64_halves(k):
    """wave_umin64: each move carries the two 32-bit halves of a key together."""
    lo, hi = (k & 0xFFFFFFFF).astype(np.uint64), (k >> np.uint64(32)).astype(np.uint64)

    def join(h, l):
        return (h << np.uint64(32)) | l

    def step(k, mv):
        l2, h2 = mv((k & 0xFFFFFFFF).astype(np.uint64)), mv((k >> np.uint64(32)).astype(np.uint64))
        return np.minimum(k, join(h2, l2))

    k = join(hi, lo)
    k = step(k, lambda v: quad_perm(v, [1, 0, 3, 2]))
    k = step(k, lambda v: quad_perm(v, [2, 3, 0, 1]))
    k = step(k, lambda v: row_ror(v, 4))
    k = step(k, lambda v: row_ror(v, 8))
    for swap in (permlane16_swap, permlane32_swap):
        la, lb = swap(k & np.uint64(0xFFFFFFFF), k & np.uint64(0xFFFFFFFF))
        ha, hb = swap(k >> np.uint64(32), k >> np.uint64(32))
        k = np.minimum(join(ha, la), join(hb, lb))
    return k


def _times(rng):
    t = rng.exponential(1.0, LANES)
    t[rng.random(LANES) < 0.3] = np.inf
    if rng.random() < 0.3:  # ties on the minimum
        t[rng.choice(LANES, 3, replace=False)] = t[np.isfinite(t)].min() if np.isfinite(t).any() else 1.0
    return t


def _bits(t):
    return np.ascontiguousarray(t + 0.0).view(np.uint64)


@pytest.mark.parametrize("seed", range(20))
def test_wave_minimum_reaches_every_lane(seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.integers(0, 2**32, LANES, dtype=np.uint64)
    assert np.all(wave_umin(x) == x.min())
    t = _times(rng)
    k = _bits(t)
    assert np.all(wave_umin64_halves(k) == k.min())
    # non-negative binary64 values order like their bit patterns
    assert np.all(wave_umin64_halves(k).view(np.float64) == t.min())


@pytest.mark.parametrize("seed", range(20))
def test_group_minimum_breaks_ties_by_id(seed):
    """grp_min<64>: the minimum time, then the smallest id among its holders."""
    rng = np.random.Generator(np.random.PCG64(100 + seed))
    t = _times(rng)
    ids = rng.permutation(5000)[:LANES].astype(np.uint64)
    k = _bits(t)
    m = wave_umin64_halves(k)
    idm = wave_umin(np.where(k == m, ids, np.uint64(0x7FFFFFFF)))
    holders = np.flatnonzero(t == t.min())
    want = ids[holders].min() if np.isfinite(t.min()) else min(ids.min(), 0x7FFFFFFF)
    if np.isfinite(t.min()):
        assert np.all(idm == want)


@pytest.mark.parametrize("seed", range(20))
def test_single_candidate_readlane_equals_the_reduction(seed):
    """With at most one lane flagged as a candidate of a corridor lane (the
    ballot has one bit), readlane of that lane combined with the earlier
    passes' minimum equals the full reduction: every other lane's key is
    above the binary32 upper bound, which the candidate or the earlier
    minimum undercuts."""
    rng = np.random.Generator(np.random.PCG64(200 + seed))
    earlier_t, earlier_id = rng.exponential(1.0), int(rng.integers(0, 100))
    t = np.full(LANES, np.inf)
    ids = np.full(LANES, 0x7FFFFFFF, np.int64)
    lane = int(rng.integers(0, LANES))
    if rng.random() < 0.8:
        t[lane] = rng.exponential(1.0)
        ids[lane] = int(rng.integers(0, 100))
    mask = np.isfinite(t)
    # readlane path
    if mask.any():
        l = int(np.flatnonzero(mask)[0])
        rt, ri = t[l], ids[l]
        got = (rt, ri) if (rt, ri) < (earlier_t, earlier_id) else (earlier_t, earlier_id)
    else:
        got = (earlier_t, earlier_id)
    # full reduction with the earlier minimum held in every lane
    allt = np.minimum(t, earlier_t)
    k = _bits(np.where(t < earlier_t, t, earlier_t))
    kid = np.where(t < earlier_t, ids, np.where(t == earlier_t, np.minimum(ids, earlier_id), earlier_id))
    m = wave_umin64_halves(k)
    idm = wave_umin(np.where(k == m, kid.astype(np.uint64), np.uint64(0x7FFFFFFF)))
    assert (m[0].view(np.float64), int(idm[0])) == got
    assert np.all(allt.min() == got[0])


def test_two_layout_mistakes_fail_the_model():
    """A row minimum built with shifts is complete only in the row's last
    lane, so reading the first lane of each row misses values; combining the
    halves of a 64-bit key separately mixes keys.  Both give a minimum that is
    not the wavefront's."""
    rng = np.random.Generator(np.random.PCG64(7))
    wrong_shift = wrong_halves = 0
    for _ in range(200):
        x = rng.integers(0, 2**32, LANES, dtype=np.uint64)
        r = x.copy()
        for n in (1, 2, 4, 8):
            r = np.minimum(r, row_shr(r, n, r))
        assert np.all(r[15::16] == x.reshape(4, 16).min(1))   # the last lane is complete
        wrong_shift += int(min(r[0], r[16], r[32], r[48]) != x.min())
        t = rng.exponential(1.0, LANES)
        k = _bits(t)
        lo = wave_umin(k & np.uint64(0xFFFFFFFF))
        hi = wave_umin(k >> np.uint64(32))
        wrong_halves += int(((hi[0] << np.uint64(32)) | lo[0]) != k.min())
    assert wrong_shift > 100 and wrong_halves > 100
