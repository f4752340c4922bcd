"""Legs along -x and -y on the GPU, and time reversal (Remark on
time-reversal invariance: Alg. 1 run with -v from the lifted configuration
it produced with +v returns the initial configuration, with the same set of
liftings, each i -> j now run as j -> i).

The library runs -x / -y legs on the reflected coordinate L - x (L - y); the
oracle runs them with the sign of v.  Both evaluate the same events, but the
reflection rounds once per disk and leg, so a leg along -v is compared with
the oracle on lifting sequences (exact) and on positions and local times
within 1e-12 L, the bound the time-reversal pin of the oracle uses as well.
"""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2004_11040_amd as pkg  # noqa: E402


def _wrapdiff(a, b, L):
    return np.abs((a - b + L / 2) % L - L / 2)


def _targets_since(e, c, start):
    lg = e.log(c)
    return lg.targets[start:]


@pytest.mark.parametrize("cfg,fwd,lanes,flags", [
    (0, pkg.DIR_X, 64, pkg.FP64),
    (0, pkg.DIR_Y, 32, pkg.FP64),
    (1, pkg.DIR_X, 64, pkg.FP32_MIXED),
    (1, pkg.DIR_Y, 64, pkg.FP64),
    (2, pkg.DIR_Y, 64, pkg.FP32_MIXED),
])
def test_time_reversal(cfg, fwd, lanes, flags):
    s = W.config(cfg)
    back = fwd + 2
    print(f"[reverse] cfg={cfg} N={s.n} k={s.k} fwd={fwd} back={back} lanes={lanes} flags={flags}",
          flush=True)
    e = pkg.Ecmc(np.stack([s.x, s.y], 1), s.sigma, s.L, flags=flags, max_chains=s.k,
                 log_cap=1 << 16)
    e.set_option(pkg.OPT_LANES, lanes)
    e.set_active(s.active)
    start = np.stack([s.x, s.y], 1).copy()

    # leg 1 along +v: bit-exact against the oracle
    e.run(s.T, s.T, fwd)
    ref1 = oracle.run(s.x, s.y, s.sigma, s.L, s.active, [fwd], s.T)
    n1 = [e.log(c).count for c in range(s.k)]
    assert e.stats()["events"] == ref1.n_events
    for c in range(s.k):
        assert np.array_equal(e.log(c).targets, ref1.targets(c)), c
    mid_active = e.active()
    assert np.array_equal(mid_active, ref1.active)

    # leg 2 along -v: against the oracle's two legs
    e.run(s.T, s.T, back)
    ref2 = oracle.run(s.x, s.y, s.sigma, s.L, s.active, [fwd, back], s.T)
    st = e.stats()
    assert st["events"] == ref2.n_events, (st["events"], ref2.n_events)
    for c in range(s.k):
        got = _targets_since(e, c, n1[c])
        want = ref2.targets(c)[n1[c]:]
        assert np.array_equal(got, want), (c, got[:8], want[:8])
    pos = e.positions()
    tol = 1e-12 * s.L
    assert _wrapdiff(pos[:, 0], ref2.x, s.L).max() <= tol
    assert _wrapdiff(pos[:, 1], ref2.y, s.L).max() <= tol
    assert np.abs(e.stamps() - ref2.stamps).max() <= tol
    assert np.array_equal(e.active(), ref2.active)

    # time reversal: back to the start, same active set, each chain's arrows reversed
    assert _wrapdiff(pos[:, 0], start[:, 0], s.L).max() <= tol
    assert _wrapdiff(pos[:, 1], start[:, 1], s.L).max() <= tol
    assert np.array_equal(e.active(), np.asarray(s.active))
    for c in range(s.k):
        fwd_t = e.log(c).targets[:n1[c]]
        moved = np.concatenate([[s.active[c]], fwd_t])   # disks chain c moved, in order
        assert np.array_equal(_targets_since(e, c, n1[c]), moved[:-1][::-1]), c
    assert e.overlaps() == 0
    print(f"[reverse] ok: {ref1.n_events} liftings each way, reruns {st['reruns']}", flush=True)
