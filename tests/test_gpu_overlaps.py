"""The FP64 overlap count (zero tolerance beyond the rounding of contact
positions; the hard-disk model, Sec. 1) against the oracle at its threshold,
2 sigma - 4 ulp(box), on configurations with a known number of planted
near-contacts on both sides of it.

Each planted pair puts a disk at 2 sigma - m ulp(box) from its neighbour
along x (m = 0 ... 8).  Pairs with m <= 3 are contacts within rounding and
do not count; pairs with m >= 5 count; m = 4 falls either way, and the GPU
must fall the oracle's way (both compare dx^2 + dy^2 with the squared limit
in binary64, without contraction).
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2004_11040_amd as pkg  # noqa: E402


def _ulp(L):
    return math.nextafter(L, math.inf) - L


def _plant(s, ms, seed):
    """Move the right-hand row neighbour r of disk a to 2 sigma - m ulp(box)
    along x, for one disjoint pair per m.  Returns (x, y)."""
    x, y = s.x.copy(), s.y.copy()
    u = _ulp(s.L)
    rng = np.random.Generator(np.random.PCG64(seed))
    used = set()
    for m in ms:
        while True:
            a = int(rng.integers(s.n))
            dx = (x - x[a]) % s.L
            dy = (y - y[a] + 0.5 * s.L) % s.L - 0.5 * s.L
            ok = (dx > 0.5 * s.sigma) & (dx < 4.0 * s.sigma) & (np.abs(dy) < 0.5 * s.sigma)
            if not ok.any():
                continue
            r = int(np.flatnonzero(ok)[np.argmin(dx[ok])])
            # keep the pairs apart: no disk of an earlier pair within 6 sigma
            if any(min(abs((x[q] - x[a] + 0.5 * s.L) % s.L - 0.5 * s.L),
                       abs((y[q] - y[a] + 0.5 * s.L) % s.L - 0.5 * s.L)) < 6.0 * s.sigma for q in used):
                continue
            break
        x[r] = (x[a] + (2.0 * s.sigma - m * u)) % s.L
        y[r] = y[a]
        used.update((a, r))
    return x, y


@pytest.mark.parametrize("cfg", [1, 2])
def test_count_at_the_threshold_matches_the_oracle(cfg):
    s = W.config(cfg)
    u = _ulp(s.L)
    x, y = _plant(s, ms=list(range(9)), seed=40 + cfg)
    ref = oracle.overlaps(x, y, s.sigma, s.L, tol=4.0 * u)
    wide = oracle.overlaps(x, y, s.sigma, s.L, tol=-0.05 * s.sigma)   # every pair within 2.05 sigma
    print(f"[overlaps] N={s.n}: oracle {ref} at 2 sigma - 4 ulp, {wide} within 2.05 sigma", flush=True)
    assert 4 <= ref <= 5 and wide >= 9          # m = 5..8 count, m = 4 either way
    dev = torch.from_numpy(np.stack([x, y], 1)).to("cuda").contiguous()
    assert pkg.overlaps_noalloc(dev, s.sigma, s.L) == ref
    with pytest.raises(pkg.EcmcError) as ei:    # the context refuses the overlapping input
        pkg.Ecmc(np.stack([x, y], 1), s.sigma, s.L, max_chains=s.k)
    assert ei.value.code == pkg.EOVERLAP


@pytest.mark.parametrize("cfg", [1, 2])
def test_contacts_within_rounding_are_accepted_and_kept(cfg):
    """Only m <= 3: the count is zero on both sides, the context accepts the
    input, and after legs that lift through these contacts the count is the
    oracle's on the final configuration (zero)."""
    s = W.config(cfg)
    u = _ulp(s.L)
    x, y = _plant(s, ms=[0, 1, 2, 3, 0, 1, 2, 3], seed=50 + cfg)
    assert oracle.overlaps(x, y, s.sigma, s.L, tol=4.0 * u) == 0
    assert oracle.overlaps(x, y, s.sigma, s.L, tol=-0.05 * s.sigma) >= 8
    e = pkg.Ecmc(np.stack([x, y], 1), s.sigma, s.L, max_chains=s.k, log_cap=1 << 10)
    assert e.overlaps() == 0
    e.set_active(s.active)
    e.run(4 * s.T, s.T, pkg.DIR_ALTERNATE)
    pos = e.positions()
    ref = oracle.overlaps(pos[:, 0], pos[:, 1], s.sigma, s.L, tol=4.0 * u)
    assert e.overlaps() == ref == 0
    e.close()
