"""Test-only CPU oracle for hard-disk event-chain Monte Carlo between breakpoints.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import this package.  It shares no code with
the GPU library in ``paper_2004_11040_amd`` and never calls it.

Contents
--------
``run``            global-time ECMC (Alg. 2 of Li, Todo, Maggs, Krauth, Sec. 2.1),
                   serial C in ``ecmc_oracle.c``: the reference every GPU result
                   is compared with.
``overlaps``       number of disk pairs closer than the contact distance.
``literal_alg2``   (module) Alg. 2 written literally with eager positions and
                   explicit periodic images, pure numpy: pins ``run`` on tiny
                   systems.
``enumerate_alg5`` (module) exact enumeration of every interleaving of the
                   multithreaded algorithm on tiny suites as an absorbing Markov
                   chain (Sec. 2.3, Alg. 5, Lemma 3), for the paper's
                   sequential-consistency program and for the gfx950 kernel's
                   protocol: every terminate state is compared with ``run``, and
                   single-statement mutations must break a check.
``constraint_graph`` (module) the constraint graph G(3), its first-order
                   pruning and symmetrization (Sec. 3.1-3.2), and the check
                   that every lifting of a leg is an arrow.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ecmc_oracle.c")
_LIB = os.path.join(_HERE, "libecmc_oracle.so")

DIR_PX, DIR_PY, DIR_MX, DIR_MY = 0, 1, 2, 3


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (IEEE binary64, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
             "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.oracle_run.restype = ctypes.c_int
        lib.oracle_run.argtypes = [
            ctypes.c_int64, ctypes.c_double, ctypes.c_double, P, P,
            ctypes.c_int32, P, ctypes.c_int32, P, ctypes.c_double, ctypes.c_int32,
            ctypes.c_int64, P, P, P, P, P, P, P, P]
        lib.oracle_overlaps.restype = ctypes.c_int64
        lib.oracle_overlaps.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                        P, P, ctypes.c_double]
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


@dataclass
class Result:
    x: np.ndarray            # final positions
    y: np.ndarray
    active: np.ndarray       # disk of each chain at the end
    n_events: int
    sum_b: np.ndarray        # per-chain sum of b_ij over liftings (event order)
    stamps: np.ndarray       # local times at the end of the last leg
    log_chain: np.ndarray | None = None
    log_from: np.ndarray | None = None
    log_to: np.ndarray | None = None
    log_time: np.ndarray | None = None
    log_b: np.ndarray | None = None

    def targets(self, chain: int) -> np.ndarray:
        """Sequence of target disks lifted to by `chain`, in order."""
        return self.log_to[self.log_chain == chain]

    def times(self, chain: int) -> np.ndarray:
        return self.log_time[self.log_chain == chain]


def run(x, y, sigma, L, active, legs, T, mode=0, log=True, log_cap=None,
        sum_b=None) -> Result:
    """Global-time ECMC over ``len(legs)`` legs of length ``T``.

    legs: sequence of direction codes (0:+x 1:+y 2:-x 3:-y), one per leg.
    mode: 0 cell search, 1 brute-force scan of all disks (must agree bit for bit).
    Times in the log are relative to the start of each leg (h = 0).
    """
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64).copy()
    y = np.ascontiguousarray(y, dtype=np.float64).copy()
    act = np.ascontiguousarray(active, dtype=np.int32).copy()
    dirs = np.ascontiguousarray(legs, dtype=np.int32)
    n, k = x.shape[0], act.shape[0]
    sb = np.zeros(max(k, 1), np.float64) if sum_b is None else np.ascontiguousarray(sum_b, np.float64).copy()
    stamps = np.zeros(n, np.float64)
    nev = ctypes.c_int64(0)
    if log:
        cap = int(log_cap) if log_cap is not None else 1 << 22
        lc = np.zeros(cap, np.int32); lf = np.zeros(cap, np.int32); lt = np.zeros(cap, np.int32)
        ltm = np.zeros(cap, np.float64); lb = np.zeros(cap, np.float64)
    else:
        cap = 0
        lc = lf = lt = ltm = lb = None
    rc = lib.oracle_run(n, float(sigma), float(L), _ptr(x), _ptr(y), k, _ptr(act),
                        dirs.shape[0], _ptr(dirs), float(T), int(mode), cap,
                        _ptr(lc), _ptr(lf), _ptr(lt), _ptr(ltm), _ptr(lb),
                        ctypes.byref(nev), _ptr(sb), _ptr(stamps))
    if rc == -3:
        raise RuntimeError("oracle log capacity exceeded; pass a larger log_cap")
    if rc != 0:
        raise ValueError(f"oracle_run failed with code {rc}")
    ne = int(nev.value)
    res = Result(x, y, act, ne, sb[:k], stamps)
    if log:
        res.log_chain, res.log_from, res.log_to = lc[:ne], lf[:ne], lt[:ne]
        res.log_time, res.log_b = ltm[:ne], lb[:ne]
    return res


def overlaps(x, y, sigma, L, tol=0.0) -> int:
    """Pairs (minimum image) with centre distance below 2*sigma - tol."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    r = lib.oracle_overlaps(x.shape[0], float(sigma), float(L), _ptr(x), _ptr(y), float(tol))
    if r < 0:
        raise MemoryError("oracle_overlaps")
    return int(r)
