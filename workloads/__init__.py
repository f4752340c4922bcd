"""Seeded synthetic hard-disk workloads shared by the tests, the oracle checks
and the benchmark.

This module only generates inputs (lattices, jitter, active sets, replica sets)
and checks that they do not overlap.  It holds none of the event-chain
arithmetic, and it imports neither the GPU library nor the oracle.

Units: disk radius sigma = 1 (contact distance 2), periodic square box of side
L = sqrt(N pi sigma^2 / eta) for packing fraction eta (definition of eta in the
paper's Sec. 3.2).  The paper's equilibrated 65536-disk sample is not available;
jittered lattices with the same N and eta stand in for it.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SIGMA = 1.0


def box_side(n: int, eta: float, sigma: float = SIGMA) -> float:
    return math.sqrt(n * math.pi * sigma * sigma / eta)


def min_distance(x, y, L):
    """Smallest centre distance (minimum image), O(N) with a cell grid."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    n = x.shape[0]
    nc = max(1, int(L // 2.5))
    if nc < 3 or n < 64:
        dx = x[:, None] - x[None, :]
        dy = y[:, None] - y[None, :]
        dx -= L * np.round(dx / L)
        dy -= L * np.round(dy / L)
        r2 = dx * dx + dy * dy
        np.fill_diagonal(r2, np.inf)
        return float(np.sqrt(r2.min()))
    cw = L / nc
    cx = np.minimum((x / cw).astype(np.int64), nc - 1)
    cy = np.minimum((y / cw).astype(np.int64), nc - 1)
    cell = cy * nc + cx
    order = np.argsort(cell, kind="stable")
    starts = np.searchsorted(cell[order], np.arange(nc * nc + 1))
    best = np.inf
    for oy in (-1, 0, 1):
        for ox in (-1, 0, 1):
            nb = ((cy + oy) % nc) * nc + (cx + ox) % nc
            # pair every disk with every member of its neighbour cell
            cnt = starts[nb + 1] - starts[nb]
            maxc = int(cnt.max()) if cnt.size else 0
            for q in range(maxc):
                has = cnt > q
                i = np.nonzero(has)[0]
                j = order[starts[nb[i]] + q]
                keep = j != i
                i, j = i[keep], j[keep]
                dx = x[j] - x[i]
                dy = y[j] - y[i]
                dx -= L * np.round(dx / L)
                dy -= L * np.round(dy / L)
                if i.size:
                    best = min(best, float(np.sqrt((dx * dx + dy * dy).min())))
    return best


def _lattice(nx: int, ny: int, L: float, offset_rows: bool):
    ax, ay = L / nx, L / ny
    ix, iy = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    x = (ix + 0.5) * ax + (0.5 * ax * (iy % 2) if offset_rows else 0.0)
    y = (iy + 0.5) * ay
    return np.mod(x.ravel(), L), np.mod(y.ravel(), L)


def lattice_min_distance(nx: int, ny: int, L: float, offset_rows: bool) -> float:
    ax, ay = L / nx, L / ny
    if not offset_rows:
        return min(ax, ay)
    return min(ax, math.hypot(0.5 * ax, ay), 2.0 * ay)


def _jitter(rng, x, y, amp, L):
    x = np.mod(x + rng.uniform(-amp, amp, x.shape), L)
    y = np.mod(y + rng.uniform(-amp, amp, y.shape), L)
    # a coordinate exactly equal to L after rounding is folded to 0
    x[x >= L] = 0.0
    y[y >= L] = 0.0
    return x, y


@dataclass
class System:
    """One seeded input: positions, box, active set and run parameters."""
    name: str
    x: np.ndarray
    y: np.ndarray
    L: float
    eta: float
    active: np.ndarray
    T: float                      # leg length h' - h
    alternate: bool               # legs alternate +x/+y, else all +x
    target_events: int
    sigma: float = SIGMA
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def k(self) -> int:
        return int(self.active.shape[0])

    def leg_dirs(self, n_legs: int, first_leg: int = 0):
        if self.alternate:
            return [(first_leg + i) % 2 for i in range(n_legs)]
        return [0] * n_legs


def square_jittered(n_side: int, eta: float, amp: float, rng):
    n = n_side * n_side
    L = box_side(n, eta)
    x, y = _lattice(n_side, n_side, L, offset_rows=False)
    return _jitter(rng, x, y, amp, L) + (L,)


def centred_rect_jittered(nx: int, ny: int, eta: float, amp: float, rng, n_sites=None):
    """Centred-rectangular lattice (rows offset by half a spacing, ny even),
    optionally keeping only n_sites seeded sites (vacancies elsewhere)."""
    assert ny % 2 == 0
    n = nx * ny if n_sites is None else n_sites
    L = box_side(n, eta)
    x, y = _lattice(nx, ny, L, offset_rows=True)
    if n_sites is not None and n_sites < nx * ny:
        keep = np.sort(rng.choice(nx * ny, n_sites, replace=False))
        x, y = x[keep], y[keep]
    return _jitter(rng, x, y, amp, L) + (L,)


def choose_grid(n: int, eta: float):
    """Smallest centred-rectangular grid (ny even) with >= n sites whose nearest
    neighbour distance exceeds the contact distance; prefer nx/ny near 1."""
    L = box_side(n, eta)
    best = None
    side = int(math.isqrt(n))
    for ny in range(max(2, side - 8) // 2 * 2, side + 12, 2):
        for nx in range(max(1, side - 8), side + 12):
            if nx * ny < n:
                continue
            a = lattice_min_distance(nx, ny, L, True)
            if a <= 2.0 * SIGMA:
                continue
            key = (nx * ny, abs(math.log(nx / ny)), -a)
            if best is None or key < best[0]:
                best = (key, nx, ny, a)
    if best is None:
        raise ValueError(f"no lattice for n={n} eta={eta}")
    return best[1], best[2], best[3], L


def active_set(rng, n: int, k: int) -> np.ndarray:
    """k distinct disks; their order defines the chain ids."""
    return rng.choice(n, k, replace=False).astype(np.int32)


# ----------------------------------------------------------------------------
# The five workloads (small parity case, mid-size, precision form, replica
# batch, headline scale run).
# ----------------------------------------------------------------------------

def config(idx: int) -> System:
    if idx == 0:
        rng = np.random.Generator(np.random.PCG64(1))
        x, y, L = square_jittered(16, 0.60, 0.05, rng)
        act = active_set(rng, 256, 4)
        return System("N256_eta0.60_k4", x, y, L, 0.60, act, 0.5 * L, False, 100_000)
    if idx == 1:
        rng = np.random.Generator(np.random.PCG64(2))
        x, y, L = centred_rect_jittered(64, 64, 0.70, 0.05, rng)
        act = active_set(rng, 4096, 64)
        return System("N4096_eta0.70_k64", x, y, L, 0.70, act, 0.25 * L, True, 10_000_000)
    if idx == 2:
        rng = np.random.Generator(np.random.PCG64(3))
        x, y, L = centred_rect_jittered(256, 256, 0.708, 0.05, rng)
        act = active_set(rng, 65536, 256)
        T = 0.25 * box_side(4096, 0.70)
        return System("N65536_eta0.708_k256", x, y, L, 0.708, act, T, True, 100_000_000)
    if idx == 4:
        rng = np.random.Generator(np.random.PCG64(5))
        x, y, L = centred_rect_jittered(1024, 1024, 0.708, 0.05, rng)
        act = active_set(rng, 1 << 20, 1024)
        T = 0.25 * box_side(4096, 0.70)
        return System("N1048576_eta0.708_k1024", x, y, L, 0.708, act, T, True, 1_000_000_000)
    raise ValueError("config index must be 0, 1, 2 or 4 (3 is the replica batch)")


def replica_batch(n_rep: int = 512, seed: int = 4):
    """Independent replicas of uneven size and density, all seeded."""
    children = np.random.SeedSequence(seed).spawn(n_rep)
    out = []
    for r, ss in enumerate(children):
        rng = np.random.Generator(np.random.PCG64(ss))
        n = 64 * int(rng.integers(16, 257))
        eta = float(rng.uniform(0.60, 0.72))
        nx, ny, a, L = choose_grid(n, eta)
        amp = min(0.05, 0.45 * (a - 2.0 * SIGMA))
        x, y, L = centred_rect_jittered(nx, ny, eta, amp, rng, n_sites=n)
        k = int(round(math.sqrt(n)))
        act = active_set(rng, n, k)
        out.append(System(f"rep{r}_N{n}_eta{eta:.3f}", x, y, L, eta, act, 0.25 * L, True,
                          1_000_000, meta={"grid": (nx, ny), "jitter": amp}))
    return out


def tonks_row(n_row: int, L: float, rng, y0: float = None):
    """One row of disks on a line along x (every pair has dp = 0): a 1-D hard-rod
    gas embedded in the periodic box."""
    gaps = rng.uniform(0.0, 1.0, n_row)
    free = L - n_row * 2.0 * SIGMA
    gaps = gaps / gaps.sum() * free
    # x_0 = offset, x_{m+1} = x_m + 2 sigma + g_m; the last gap closes the ring
    xs = np.concatenate([[0.0], np.cumsum(2.0 * SIGMA + gaps)[:-1]]) + rng.uniform(0, L)
    xs = np.mod(xs, L)
    xs[xs >= L] = 0.0
    y = np.full(n_row, L / 2.0 if y0 is None else y0)
    return xs, y


def random_dilute(n: int, eta: float, rng):
    """Random sequential placement without overlap (dilute systems)."""
    L = box_side(n, eta)
    xs, ys = [], []
    while len(xs) < n:
        px, py = rng.uniform(0, L), rng.uniform(0, L)
        ok = True
        for qx, qy in zip(xs, ys):
            dx = (px - qx + L / 2) % L - L / 2
            dy = (py - qy + L / 2) % L - L / 2
            if dx * dx + dy * dy < (2.0 * SIGMA * 1.000001) ** 2:
                ok = False
                break
        if ok:
            xs.append(px)
            ys.append(py)
    return np.array(xs), np.array(ys), L
