"""Error bounds of the FP32-mixed filter (time of flight of Sec. 2.2), on the CPU.

The event kernel's binary32 filter gives each scanned slot an interval
[lo, hi] for the time of flight and the corridor lanes the slot may lie in; a
slot is recomputed in binary64 unless its lo cannot undercut a lane's bound.
The binary64 result is therefore exact only if (a) every disk inside the
corridor gets a finite lo, (b) lo <= tau <= hi for the binary64 tau, and
(c) a lane the filter calls certain is the binary64 lane.

This test restates the filter's binary32 arithmetic with numpy float32 (IEEE
round to nearest, no fused operations: the kernel is built with
-ffp-contract=off) and models v_sqrt_f32 as the correctly rounded root moved
by one ulp either way.  It checks (a)-(c) against the binary64 definition of
tau (forward distance along v minus sqrt(d^2 - dp^2), dp the minimum image)
on random slots and on slots placed at the boundaries that matter: grazing
contact, the lane borders at |dp| = sigma, and forward distances near 0 and L.
"""
import numpy as np
import pytest

F = np.float32
U = F(5.9604645e-8)  # 2^-24


def _filter(mc, dr, rai, rpi, raj, rpj, c32, L32, d2_32, s32, sqrt_nudge):
    """The filter's arithmetic, operation by operation, in binary32."""
    def sq(v):
        r = np.sqrt(v)
        return np.nextafter(r, F(np.inf) if sqrt_nudge > 0 else F(0)) if sqrt_nudge else r

    off = mc.astype(F) * c32
    da0 = (off + raj) - rai
    eda0 = F(4) * U * (np.abs(off) + np.abs(raj) + np.abs(rai) + c32 * mc.astype(F))
    neg, over = da0 < F(0), da0 >= L32
    da = np.where(neg, da0 + L32, np.where(over, da0 - L32, da0))
    eda = np.where(neg | over, eda0 + F(4) * U * L32, eda0)
    unsure = (neg & (da0 > -eda0)) | (da < eda) | (da > L32 - eda)
    dp = (dr.astype(F) * c32 + rpj) - rpi
    edp = F(4) * U * (c32 + np.abs(rpj) + np.abs(rpi))
    adp = np.abs(dp)
    x = d2_32 - dp * dp
    ex = (F(2) * adp + F(2) * edp) * edp + F(4) * U * (d2_32 + dp * dp)
    inside = x + ex > F(0)
    blo = sq(np.maximum(x - ex, F(0))) * (F(1) - F(8) * U)
    bhi = sq(np.maximum(x + ex, F(0))) * (F(1) + F(8) * U)
    err = eda + F(8) * U * (da + bhi) + F(1e-30)
    lo = np.where(~inside, F(np.inf), np.where(unsure, F(0), np.maximum((da - bhi) - err, F(0))))
    hi = np.where(inside & (x - ex > F(0)) & ~unsure, np.maximum((da - blo) + err, F(0)) + F(1e-30), F(np.inf))
    es = edp + F(4) * U * s32
    c0, c1, c2 = adp + es < s32, dp - es >= s32, dp + es <= -s32
    cls = np.where(~inside, -1, np.where(c0, 0, np.where(c1, 1, np.where(c2, 2, -1))))
    mask = np.where(~inside, 0, np.where(c0, 1, np.where(c1, 2, np.where(c2, 4, np.where(dp > F(0), 3, 5)))))
    return lo, hi, cls, mask


def _cases(rng, n, mode):
    """Slots around a moving disk, in binary64 absolute coordinates."""
    sigma, d = 1.0, 2.0
    c = rng.uniform(d * (1 + 1e-9), np.sqrt(2) * d, n)
    nc = rng.integers(5, 1100, n)
    L = nc * c
    col0, row0 = rng.integers(0, nc), rng.integers(0, nc)
    mc = rng.integers(0, 10, n) % np.maximum(nc - 2, 1)
    dr = rng.integers(-1, 2, n)
    ui, vi = rng.uniform(0, 1, n) * c, rng.uniform(0, 1, n) * c
    uj, vj = rng.uniform(0, 1, n) * c, rng.uniform(0, 1, n) * c
    ai, pi = col0 * c + ui, row0 * c + vi
    colj, rowj = (col0 + mc) % nc, (row0 + dr) % nc
    # boundaries: place j so that dp (or the forward distance) sits on an edge
    eps = rng.uniform(-1e-6, 1e-6, n) * rng.choice([1.0, 1e-3, 1e-6], n)
    sgn = rng.choice([-1.0, 1.0], n)
    pj = rowj * c + vj
    aj = colj * c + uj
    if mode == "grazing":
        pj = pi + sgn * (d + eps)
    elif mode == "lane":
        pj = pi + sgn * (sigma + eps)
    elif mode == "wrap":
        aj = ai + eps  # forward distance near 0 (or, below 0, near L)
        mc = np.zeros(n, np.int64)
        colj = col0 * np.ones(n, np.int64)
    pj = np.mod(pj, L)
    aj = np.mod(aj, L)
    rowj = np.floor(pj / c).astype(np.int64) % nc
    colj = np.floor(aj / c).astype(np.int64) % nc
    dr = (rowj - row0 + 1) % nc - 1
    mc = (colj - col0) % nc
    keep = (np.abs(dr) <= 1) & (mc <= 9) & (mc <= nc - 3)
    return dict(c=c, L=L, col0=col0, row0=row0, colj=colj, rowj=rowj, mc=mc, dr=dr,
                ai=ai, pi=pi, aj=aj, pj=pj, keep=keep)


def _tau64(k):
    """Binary64 definition: minimum-image dp, forward distance in [0, L)."""
    d2 = 4.0
    dp = k["pj"] - k["pi"]
    dp = dp - k["L"] * np.round(dp / k["L"])
    da = k["aj"] - k["ai"]
    da = np.where(da < 0, da + k["L"], da)
    inside = dp * dp < d2
    b = np.sqrt(np.maximum(d2 - dp * dp, 0.0))
    tau = np.where(inside, np.maximum(da - b, 0.0), np.inf)
    lane = np.where(np.abs(dp) < 1.0, 0, np.where(dp > 0, 1, 2))
    return tau, lane, inside


@pytest.mark.parametrize("mode", ["random", "grazing", "lane", "wrap"])
@pytest.mark.parametrize("nudge", [-1, 0, 1])
def test_fp32_filter_interval_contains_binary64(mode, nudge):
    rng = np.random.Generator(np.random.PCG64(9000 + 10 * ["random", "grazing", "lane", "wrap"].index(mode) + nudge))
    k = _cases(rng, 200_000, mode)
    m = k["keep"]
    k = {key: v[m] for key, v in k.items() if key != "keep"}
    # the kernel's inputs: binary32 offsets of both disks inside their home cells
    col0, row0 = k["col0"], k["row0"]
    u = k["ai"] - col0 * k["c"]
    u = np.where(u < 0, u + k["L"], u)
    rai = u.astype(F)
    rpi = (k["pi"] - row0 * k["c"]).astype(F)
    raj = (k["aj"] - k["colj"] * k["c"]).astype(F)
    rpj = (k["pj"] - k["rowj"] * k["c"]).astype(F)
    lo, hi, cls, mask = _filter(k["mc"], k["dr"], rai, rpi, raj, rpj, k["c"].astype(F), k["L"].astype(F),
                                F(4.0), F(1.0), nudge)
    tau, lane, inside = _tau64(k)
    assert inside.sum() > 1000
    # (a) a disk in the corridor is never filtered out as outside
    assert np.all(lo[inside] < np.inf)
    # (b) the interval holds the binary64 time of flight
    ti, li, hi_i = tau[inside], lo[inside].astype(np.float64), hi[inside].astype(np.float64)
    bad_lo = li > ti
    bad_hi = hi_i < ti
    assert not bad_lo.any(), (ti[bad_lo][:5], li[bad_lo][:5])
    assert not bad_hi.any(), (ti[bad_hi][:5], hi_i[bad_hi][:5])
    # (c) certain lanes are the binary64 lanes, and the mask always holds the lane
    sure = inside & (cls >= 0)
    assert np.array_equal(cls[sure], lane[sure])
    assert np.all((mask[inside] >> lane[inside]) & 1)


@pytest.mark.parametrize("nudge", [-1, 0, 1])
def test_fp32_filter_with_disks_moved_past_their_home_cells(nudge):
    """During a leg the records keep their home slots while the disks move on:
    the kernel passes raj = a_j - (home column of j) c with a_j the current
    position (up to T past the home column, wrapping past L, so raj ranges
    over (-L, c + T)), and u = a_i - (home column of i) c for the moving
    disk's reference, up to c + T.  The interval must still hold the binary64
    time of flight computed from the absolute positions."""
    rng = np.random.Generator(np.random.PCG64(9500 + nudge))
    k = _cases(rng, 300_000, "random")
    m = k["keep"]
    k = {key: v[m] for key, v in k.items() if key != "keep"}
    c, L = k["c"], k["L"]
    T = np.minimum(L - 4.0 * c - 2.0, 40.0) * rng.uniform(0.0, 1.0, c.shape[0])
    ok = T > 0
    k = {key: v[ok] for key, v in k.items()}
    c, L, T = k["c"], k["L"], T[ok]
    n = c.shape[0]
    # both disks advance along v; the records stay in their home slots
    k["ai"] = np.mod(k["ai"] + rng.uniform(0.0, 1.0, n) * T, L)
    k["aj"] = np.mod(k["aj"] + rng.uniform(0.0, 1.0, n) * T, L)
    col0, row0 = k["col0"], k["row0"]
    u = k["ai"] - col0 * c
    u = np.where(u < 0, u + L, u)
    rai = u.astype(F)
    rpi = (k["pi"] - row0 * c).astype(F)
    raj = (k["aj"] - k["colj"] * c).astype(F)
    rpj = (k["pj"] - k["rowj"] * c).astype(F)
    assert (raj < 0).any() and (u > 2 * c).any()   # the ranges this test is about do occur
    lo, hi, cls, mask = _filter(k["mc"], k["dr"], rai, rpi, raj, rpj, c.astype(F), L.astype(F),
                                F(4.0), F(1.0), nudge)
    tau, lane, inside = _tau64(k)
    assert inside.sum() > 1000
    assert np.all(lo[inside] < np.inf)
    ti, li, hi_i = tau[inside], lo[inside].astype(np.float64), hi[inside].astype(np.float64)
    assert not (li > ti).any(), (ti[li > ti][:5], li[li > ti][:5])
    assert not (hi_i < ti).any(), (ti[hi_i < ti][:5], hi_i[hi_i < ti][:5])
    sure = inside & (cls >= 0)
    assert np.array_equal(cls[sure], lane[sure])
    assert np.all((mask[inside] >> lane[inside]) & 1)
