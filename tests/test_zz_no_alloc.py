"""The allocation-free overlap count (ecmc_overlaps_noalloc) against the
context's count (ecmc_overlaps) and the oracle's, through the C ABI: two
calls in a row, the second on a smaller system, then planted overlaps and
the argument checks."""
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


def _ulp4(L):
    return 4.0 * (math.nextafter(L, math.inf) - L)


def _after_legs(cfg, legs):
    s = W.config(cfg)
    e = pkg.Ecmc(np.stack([s.x, s.y], 1), s.sigma, s.L, max_chains=s.k, log_cap=1 << 10)
    e.set_active(s.active)
    e.run(legs * s.T, s.T, pkg.DIR_ALTERNATE)
    return s, e


def test_noalloc_count_matches_the_context_count_twice():
    """Two calls in a row, the second with a smaller input: each equals the
    context's ecmc_overlaps on the same configuration and the oracle's."""
    for cfg, legs in ((2, 2), (1, 3)):
        s, e = _after_legs(cfg, legs)
        pos = e.positions()
        want = e.overlaps()
        got = pkg.overlaps_noalloc(torch.from_numpy(pos).to("cuda").contiguous(), s.sigma, s.L)
        ref = oracle.overlaps(pos[:, 0], pos[:, 1], s.sigma, s.L, tol=_ulp4(s.L))
        print(f"[noalloc] N={s.n}: context {want}, noalloc {got}, oracle {ref}", flush=True)
        assert got == want == ref == 0
        e.close()


def test_noalloc_counts_planted_overlaps_like_the_oracle():
    """Planted pairs at 1.5 sigma (and one at 2 sigma - 10 ulp): the count is
    the oracle's, exactly; then a smaller system again."""
    for cfg, n_plant in ((2, 40), (1, 7)):
        s = W.config(cfg)
        x, y = s.x.copy(), s.y.copy()
        rng = np.random.Generator(np.random.PCG64(17 + cfg))
        idx = rng.choice(s.n, 2 * n_plant, replace=False)
        for a, b in zip(idx[::2], idx[1::2]):
            x[b] = (x[a] + 1.5 * s.sigma) % s.L
            y[b] = y[a]
        a0, b0 = idx[0], idx[1]
        x[b0] = (x[a0] + (2.0 * s.sigma - 10 * (math.nextafter(s.L, math.inf) - s.L))) % s.L
        ref = oracle.overlaps(x, y, s.sigma, s.L, tol=_ulp4(s.L))
        dev = torch.from_numpy(np.stack([x, y], 1)).to("cuda").contiguous()
        try:
            got = pkg.overlaps_noalloc(dev, s.sigma, s.L)
        except pkg.EcmcError as err:  # five centres in one cell: disks overlap
            assert err.code == pkg.EOVERLAP and ref > 0
            continue
        print(f"[noalloc] planted N={s.n}: noalloc {got}, oracle {ref}", flush=True)
        assert got == ref and ref >= n_plant


def test_noalloc_rejects_bad_arguments():
    s = W.config(1)
    dev = torch.from_numpy(np.stack([s.x, s.y], 1)).to("cuda").contiguous()
    for sigma, box in ((0.0, s.L), (s.sigma, 0.0), (s.sigma, 2.0 * s.sigma), (0.5, 1201.0 * 2.0)):
        with pytest.raises(pkg.EcmcError) as ei:
            pkg.overlaps_noalloc(dev, sigma, box)
        assert ei.value.code == pkg.EINVAL
    bad = dev.clone()
    bad[5, 0] = s.L  # outside [0, box)
    with pytest.raises(pkg.EcmcError) as ei:
        pkg.overlaps_noalloc(bad, s.sigma, s.L)
    assert ei.value.code == pkg.EINVAL
    assert pkg.overlaps_noalloc(dev, s.sigma, s.L) == 0  # and it still works afterwards
