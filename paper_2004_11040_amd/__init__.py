"""Python binding of the MI355X hard-disk event-chain Monte Carlo library.

Thin ctypes marshalling over the C ABI declared in ``include/ecmc.h``; every
step of the method runs in the HIP kernels of ``libecmc.so``.  PyTorch only
provides the device workspace and the stream.  There is no CPU fallback: if the
built library cannot be loaded, importing the binding's functions raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libecmc.so")
PROBE_LIB_PATH = os.path.join(_HERE, "libecmc_probe.so")

OK = 0
EINVAL, EOVERLAP, EDEVICE, ECELL, EHANG, ESTATE = -1, -2, -3, -4, -5, -6
FP64, FP32_MIXED = 0, 1
OPT_LANES, OPT_WAIT_RETRIES, OPT_MAX_SPLITS, OPT_FORCE_GLOBAL = 1, 2, 3, 4
OPT_INJECT_CHAIN, OPT_INJECT_EVENT, OPT_KERNEL_TIMING, OPT_STRICT_ORDER = 5, 6, 7, 8
OPT_WINDOW_MICRO = 9
OPT_FEATURES = 10
OPT_GRAPH = 11
OPT_CELL_PCT = 12
OPT_NEIGHBOURS = 13
OPT_COOPERATIVE = 14
OPT_TEST_NONRESIDENT = 15
OPT_CLOCK_PERIOD_NS = 16
NEIGHBOURS_CELLS, NEIGHBOURS_GRAPH = 0, 1
FEAT_SCREEN, FEAT_RESERVE, FEAT_REREAD, FEAT_FRESH, FEAT_UNRESERVE, FEAT_ALL = 1, 2, 4, 8, 16, 31
FEAT_DEFAULT = 30
DIR_X, DIR_Y, DIR_MX, DIR_MY, DIR_ALTERNATE = 0, 1, 2, 3, 4

# every symbol include/ecmc_probe.h declares (libecmc_probe.so)
PROBE_EXPORTS = ("ecmc_probe_chase", "ecmc_probe_gather", "ecmc_probe_litmus_mp", "ecmc_probe_litmus_cas")

# every symbol include/ecmc.h declares
EXPORTS = (
    "ecmc_workspace_bytes", "ecmc_init", "ecmc_set_active", "ecmc_run", "ecmc_run_directions", "ecmc_stats",
    "ecmc_get_positions", "ecmc_get_stamps", "ecmc_get_active", "ecmc_get_chain_sums",
    "ecmc_get_log", "ecmc_overlaps", "ecmc_overlaps_noalloc", "ecmc_graph", "ecmc_set_option",
    "ecmc_last_error",
    "ecmc_free",
    "ecmc_batch_scratch_bytes", "ecmc_batch_create", "ecmc_batch_set_option", "ecmc_batch_run",
    "ecmc_batch_info", "ecmc_batch_last_error", "ecmc_batch_free", "ecmc_batch_tune_cache",
)


class EcmcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ecmc error {code}: {msg}")
        self.code = code


class Stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in (
        "events", "legs", "legs_violated", "attempts", "reruns", "global_legs", "cas_fail",
        "active_waits", "contact_moves", "fp32_refines", "slots_scanned", "overlaps")] + [
        (n, ctypes.c_double) for n in ("sum_b", "chain_time", "pressure", "device_ms",
                                       "event_kernel_ms")] + [
        (n, ctypes.c_int64) for n in ("event_launches", "timed_events", "timed_slots")] + [
        ("violations_by_kind", ctypes.c_int64 * 4)] + [
        (n, ctypes.c_int32) for n in ("last_violation_kind", "last_violation_chain",
                                      "last_violation_disk", "pad_")] + [
        (n, ctypes.c_double) for n in ("last_violation_t", "last_violation_tj",
                                       "last_violation_tau", "last_violation_h")] + [
        (n, ctypes.c_int64) for n in ("lockstep_runs", "violations_screened", "claim_yields",
                                      "spin_aborts", "nonresident_launches", "cooperative", "clock_iters",
                                      "overflow_legs")]

    def as_dict(self):
        d = {n: getattr(self, n) for n, _ in self._fields_ if n != "pad_"}
        d["violations_by_kind"] = list(self.violations_by_kind)
        return d


class BatchInfo(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("lanes", "graph", "workgroups", "cell_pct")] + [
        ("device_ms", ctypes.c_double)] + [
        (n, ctypes.c_int64) for n in ("events", "legs", "rollbacks", "global_runs")] + [
        ("tune_events_per_ms", ctypes.c_double * 4), ("tune_cell_events_per_ms", ctypes.c_double * 4)] + [
        (n, ctypes.c_int32) for n in ("tune_from_cache", "pad2_")] + [
        (n, ctypes.c_double) for n in ("replica_ms_max", "replica_ms_sum")]

    def as_dict(self):
        d = {n: getattr(self, n) for n, _ in self._fields_ if not n.startswith("pad")}
        d["tune_events_per_ms"] = list(self.tune_events_per_ms)
        d["tune_cell_events_per_ms"] = list(self.tune_cell_events_per_ms)
        return d


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libecmc.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run __graft_entry__.build() first")
    lib = ctypes.CDLL(path)
    P, I32, I64, D, U32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_uint32
    lib.ecmc_workspace_bytes.restype = I64
    lib.ecmc_workspace_bytes.argtypes = [I64, D, D, I32, I32, I64, U32]
    lib.ecmc_init.restype = ctypes.c_int
    lib.ecmc_init.argtypes = [ctypes.POINTER(P), P, I64, D, D, I32, U32, P, I64, I32, I64, P]
    lib.ecmc_set_active.restype = ctypes.c_int
    lib.ecmc_set_active.argtypes = [P, P, I32]
    lib.ecmc_run.restype = ctypes.c_int
    lib.ecmc_run.argtypes = [P, I32, D, D, I32]
    lib.ecmc_run_directions.restype = ctypes.c_int
    lib.ecmc_run_directions.argtypes = [P, I32, D, I64, P]
    lib.ecmc_stats.restype = ctypes.c_int
    lib.ecmc_stats.argtypes = [P, ctypes.POINTER(Stats)]
    for name in ("ecmc_get_positions", "ecmc_get_stamps", "ecmc_get_active"):
        getattr(lib, name).restype = ctypes.c_int
        getattr(lib, name).argtypes = [P, P]
    lib.ecmc_get_chain_sums.restype = ctypes.c_int
    lib.ecmc_get_chain_sums.argtypes = [P, P, P]
    lib.ecmc_get_log.restype = ctypes.c_int
    lib.ecmc_get_log.argtypes = [P, I32, P, I64, ctypes.POINTER(I64)]
    lib.ecmc_overlaps.restype = ctypes.c_int
    lib.ecmc_overlaps.argtypes = [P, ctypes.POINTER(I64)]
    lib.ecmc_graph.restype = ctypes.c_int
    lib.ecmc_graph.argtypes = [P, I32, D, P]
    lib.ecmc_overlaps_noalloc.restype = ctypes.c_int
    lib.ecmc_overlaps_noalloc.argtypes = [P, I64, D, D, ctypes.POINTER(I64), P]
    lib.ecmc_set_option.restype = ctypes.c_int
    lib.ecmc_set_option.argtypes = [P, I32, I64]
    lib.ecmc_last_error.restype = ctypes.c_char_p
    lib.ecmc_last_error.argtypes = [P]
    lib.ecmc_free.restype = None
    lib.ecmc_free.argtypes = [P]
    lib.ecmc_batch_scratch_bytes.restype = I64
    lib.ecmc_batch_scratch_bytes.argtypes = [I32]
    lib.ecmc_batch_create.restype = ctypes.c_int
    lib.ecmc_batch_create.argtypes = [ctypes.POINTER(P), P, I32, P, I64]
    lib.ecmc_batch_set_option.restype = ctypes.c_int
    lib.ecmc_batch_set_option.argtypes = [P, I32, I64]
    lib.ecmc_batch_run.restype = ctypes.c_int
    lib.ecmc_batch_run.argtypes = [P, P, P, I32, I32]
    lib.ecmc_batch_info.restype = ctypes.c_int
    lib.ecmc_batch_info.argtypes = [P, ctypes.POINTER(BatchInfo)]
    lib.ecmc_batch_last_error.restype = ctypes.c_char_p
    lib.ecmc_batch_last_error.argtypes = [P]
    lib.ecmc_batch_free.restype = None
    lib.ecmc_batch_free.argtypes = [P]
    lib.ecmc_batch_tune_cache.restype = ctypes.c_int
    lib.ecmc_batch_tune_cache.argtypes = [P, ctypes.c_char_p]
    _lib = lib
    return lib


def overlaps_noalloc(positions, sigma, box) -> int:
    """ecmc_overlaps_noalloc on a device tensor of n x 2 doubles."""
    import torch
    lib = load_library()
    if positions.dtype != torch.float64 or positions.dim() != 2 or positions.shape[1] != 2 \
            or not positions.is_cuda or not positions.is_contiguous():
        raise ValueError("positions must be a contiguous n x 2 float64 CUDA tensor")
    out = ctypes.c_int64(0)
    rc = lib.ecmc_overlaps_noalloc(ctypes.c_void_p(positions.data_ptr()), int(positions.shape[0]),
                                   float(sigma), float(box), ctypes.byref(out),
                                   ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    if rc != OK:
        raise EcmcError(rc, "ecmc_overlaps_noalloc failed")
    return int(out.value)


_probe_lib = None


def load_probe_library(path: str = PROBE_LIB_PATH):
    """Load libecmc_probe.so, the memory microbenchmarks (raises if missing)."""
    global _probe_lib
    if _probe_lib is not None:
        return _probe_lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run __graft_entry__.build() first")
    lib = ctypes.CDLL(path)
    P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.ecmc_probe_chase.restype = ctypes.c_int
    lib.ecmc_probe_chase.argtypes = [P, I64, I64, I32, P, ctypes.POINTER(ctypes.c_double)]
    lib.ecmc_probe_gather.restype = ctypes.c_int
    lib.ecmc_probe_gather.argtypes = [P, I64, I32, I32, I32, P, ctypes.POINTER(ctypes.c_double)]
    lib.ecmc_probe_litmus_mp.restype = ctypes.c_int
    lib.ecmc_probe_litmus_mp.argtypes = [P, P, I32, I32, I32, I32, P, ctypes.POINTER(I64), ctypes.POINTER(I64)]
    lib.ecmc_probe_litmus_cas.restype = ctypes.c_int
    lib.ecmc_probe_litmus_cas.argtypes = [P, P, I32, I32, I32, I32, P, ctypes.POINTER(I64)]
    _probe_lib = lib
    return lib


def probe_chase(lines, hops, scope=1) -> float:
    """Mean dependent-load latency in ns over a device uint8/uint32 tensor of
    64-byte lines whose first word holds the next line's index."""
    import torch
    lib = load_probe_library()
    out = ctypes.c_double(0.0)
    n_lines = lines.numel() * lines.element_size() // 64
    rc = lib.ecmc_probe_chase(ctypes.c_void_p(lines.data_ptr()), n_lines, int(hops), int(scope),
                              ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), ctypes.byref(out))
    if rc:
        raise EcmcError(rc, "ecmc_probe_chase failed")
    return out.value


def probe_gather(lines, blocks, loads_per_thread, scope=1) -> float:
    """Random-line gather bandwidth (64 B per load) in GB/s over a device tensor."""
    import torch
    lib = load_probe_library()
    out = ctypes.c_double(0.0)
    n_lines = lines.numel() * lines.element_size() // 64
    rc = lib.ecmc_probe_gather(ctypes.c_void_p(lines.data_ptr()), n_lines, int(blocks), int(loads_per_thread),
                               int(scope), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                               ctypes.byref(out))
    if rc:
        raise EcmcError(rc, "ecmc_probe_gather failed")
    return out.value


def litmus_mp(pairs, iters, spin, waits=True):
    """Message-passing litmus test; returns (seen, stale)."""
    import torch
    lib = load_probe_library()
    data = torch.zeros(pairs * 64 * iters, dtype=torch.int32, device="cuda")
    flag = torch.zeros_like(data)
    seen, stale = ctypes.c_int64(0), ctypes.c_int64(0)
    rc = lib.ecmc_probe_litmus_mp(ctypes.c_void_p(data.data_ptr()), ctypes.c_void_p(flag.data_ptr()), int(pairs),
                                  int(iters), int(spin), int(bool(waits)),
                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                                  ctypes.byref(seen), ctypes.byref(stale))
    if rc:
        raise EcmcError(rc, "ecmc_probe_litmus_mp failed")
    return seen.value, stale.value


def litmus_cas(locs, blocks, rounds, tries):
    """Compare-and-swap exclusivity litmus test; returns (acquired, counter sum)."""
    import torch
    lib = load_probe_library()
    tag = torch.zeros(locs, dtype=torch.int32, device="cuda")
    counter = torch.zeros_like(tag)
    acquired = ctypes.c_int64(0)
    rc = lib.ecmc_probe_litmus_cas(ctypes.c_void_p(tag.data_ptr()), ctypes.c_void_p(counter.data_ptr()), int(locs),
                                   int(blocks), int(rounds), int(tries),
                                   ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), ctypes.byref(acquired))
    if rc:
        raise EcmcError(rc, "ecmc_probe_litmus_cas failed")
    return acquired.value, int(counter.to(torch.int64).sum().item()), int(tag.abs().sum().item())


def workspace_bytes(n, sigma, box, cells=0, max_chains=1, log_cap=1, flags=FP64) -> int:
    return int(load_library().ecmc_workspace_bytes(int(n), float(sigma), float(box), int(cells),
                                                   int(max_chains), int(log_cap), int(flags)))


def _np_ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class ChainLog:
    count: int
    targets: np.ndarray


class Ecmc:
    """One periodic box of hard disks on the current GPU.

    positions: (n, 2) float64 array (host or torch tensor); copied to the GPU.
    """

    def __init__(self, positions, sigma, box, cells=0, flags=FP64, max_chains=1, log_cap=1 << 16,
                 stream=None, device="cuda"):
        import torch
        self._torch = torch
        self.lib = load_library()
        self.n = int(positions.shape[0])
        self.sigma, self.box, self.flags = float(sigma), float(box), int(flags)
        self.max_chains, self.log_cap = int(max_chains), int(log_cap)
        nbytes = self.lib.ecmc_workspace_bytes(self.n, self.sigma, self.box, int(cells),
                                               self.max_chains, self.log_cap, self.flags)
        if nbytes < 0:
            raise EcmcError(int(nbytes), "invalid sizes for ecmc_workspace_bytes")
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        # torch owns the device memory; 256-byte alignment is guaranteed by its allocator
        self.workspace = torch.empty(int(nbytes), dtype=torch.uint8, device=device)
        pos = torch.as_tensor(np.ascontiguousarray(positions, dtype=np.float64)
                              if not isinstance(positions, torch.Tensor) else positions,
                              dtype=torch.float64).to(device).contiguous()
        self._ctx = ctypes.c_void_p()
        rc = self.lib.ecmc_init(ctypes.byref(self._ctx), ctypes.c_void_p(pos.data_ptr()), self.n,
                                self.sigma, self.box, int(cells), self.flags,
                                ctypes.c_void_p(self.workspace.data_ptr()), int(nbytes),
                                self.max_chains, self.log_cap,
                                ctypes.c_void_p(self.stream.cuda_stream))
        if rc != OK:
            raise EcmcError(rc, {EOVERLAP: "input disks overlap", EINVAL: "invalid argument"}.get(
                rc, "ecmc_init failed"))
        self.k = 0

    # -- helpers -------------------------------------------------------------
    def _check(self, rc):
        if rc != OK:
            msg = self.lib.ecmc_last_error(self._ctx)
            raise EcmcError(rc, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "_ctx", None) and self._ctx.value:
            self.lib.ecmc_free(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- API -----------------------------------------------------------------
    def set_active(self, idx):
        a = np.ascontiguousarray(idx, dtype=np.int32)
        self._check(self.lib.ecmc_set_active(self._ctx, _np_ptr(a), a.shape[0]))
        self.k = int(a.shape[0])

    def run(self, chain_time, breakpoint_interval, direction=DIR_ALTERNATE, n_chains=None):
        self._check(self.lib.ecmc_run(self._ctx, self.k if n_chains is None else int(n_chains),
                                      float(chain_time), float(breakpoint_interval), int(direction)))

    def run_legs(self, n_legs, T, direction=DIR_ALTERNATE):
        self.run(n_legs * T, T, direction)

    def run_directions(self, T, directions, n_chains=None):
        """One leg of length T per entry of `directions` (0 +x, 1 +y, 2 -x, 3 -y)."""
        d = np.ascontiguousarray(directions, dtype=np.int32)
        self._check(self.lib.ecmc_run_directions(self._ctx, self.k if n_chains is None else int(n_chains),
                                                 float(T), int(d.shape[0]), _np_ptr(d)))

    def set_option(self, key, value):
        self._check(self.lib.ecmc_set_option(self._ctx, int(key), int(value)))

    def stats(self) -> dict:
        s = Stats()
        self._check(self.lib.ecmc_stats(self._ctx, ctypes.byref(s)))
        return s.as_dict()

    def positions(self) -> np.ndarray:
        out = np.empty((self.n, 2), np.float64)
        self._check(self.lib.ecmc_get_positions(self._ctx, _np_ptr(out)))
        return out

    def stamps(self) -> np.ndarray:
        out = np.empty(self.n, np.float64)
        self._check(self.lib.ecmc_get_stamps(self._ctx, _np_ptr(out)))
        return out

    def active(self) -> np.ndarray:
        out = np.empty(self.k, np.int32)
        self._check(self.lib.ecmc_get_active(self._ctx, _np_ptr(out)))
        return out

    def chain_sums(self):
        sb = np.empty(self.k, np.float64)
        ev = np.empty(self.k, np.int64)
        self._check(self.lib.ecmc_get_chain_sums(self._ctx, _np_ptr(sb), _np_ptr(ev)))
        return sb, ev

    def log(self, chain) -> ChainLog:
        """Target disk ids of the chain's liftings (the most recent log_cap)."""
        n = ctypes.c_int64(0)
        rc = self.lib.ecmc_get_log(self._ctx, int(chain), None, 0, ctypes.byref(n))
        count = int(n.value)
        keep = min(count, self.log_cap)
        if keep == 0:
            self._check(rc)
            return ChainLog(count, np.empty(0, np.int32))
        buf = np.empty(keep, np.int32)
        self._check(self.lib.ecmc_get_log(self._ctx, int(chain), _np_ptr(buf), keep,
                                          ctypes.byref(n)))
        return ChainLog(count, buf)

    def graph(self, direction, horizon) -> np.ndarray:
        """Arrows of the constraint graph G(3), (n, 3) target ids (-1: none),
        lanes (0, +, -), for the current configuration."""
        out = np.empty(3 * self.n, np.int32)
        self._check(self.lib.ecmc_graph(self._ctx, int(direction), float(horizon), _np_ptr(out)))
        return out.reshape(self.n, 3)

    def overlaps(self) -> int:
        c = ctypes.c_int64(0)
        self._check(self.lib.ecmc_overlaps(self._ctx, ctypes.byref(c)))
        return int(c.value)


class Batch:
    """Independent replicas (each an Ecmc with its active set) run together
    in one persistent launch; results are read from the Ecmc objects."""

    def __init__(self, systems, device="cuda"):
        import torch
        self.lib = load_library()
        self.systems = list(systems)
        n = len(self.systems)
        nbytes = int(self.lib.ecmc_batch_scratch_bytes(n))
        if nbytes < 0:
            raise EcmcError(nbytes, "invalid batch size")
        self.scratch = torch.empty(nbytes, dtype=torch.uint8, device=device)
        handles = (ctypes.c_void_p * n)(*[e._ctx.value for e in self.systems])
        self._b = ctypes.c_void_p()
        rc = self.lib.ecmc_batch_create(ctypes.byref(self._b), handles, n,
                                        ctypes.c_void_p(self.scratch.data_ptr()), nbytes)
        if rc != OK:
            raise EcmcError(rc, "ecmc_batch_create failed")

    def _check(self, rc):
        if rc != OK:
            msg = self.lib.ecmc_batch_last_error(self._b)
            raise EcmcError(rc, msg.decode() if msg else "")

    def set_option(self, key, value):
        self._check(self.lib.ecmc_batch_set_option(self._b, int(key), int(value)))

    def tune_cache(self, path):
        """Keep the autotuner's choice in a JSON file (None: no cache)."""
        self._check(self.lib.ecmc_batch_tune_cache(self._b, None if path is None else os.fsencode(path)))

    def run(self, target_events, leg_T, direction=DIR_ALTERNATE, max_legs=0):
        tg = np.ascontiguousarray(target_events, dtype=np.int64)
        lt = np.ascontiguousarray(leg_T, dtype=np.float64)
        if tg.shape[0] != len(self.systems) or lt.shape[0] != len(self.systems):
            raise ValueError("one target and one leg length per replica")
        self._check(self.lib.ecmc_batch_run(self._b, _np_ptr(tg), _np_ptr(lt), int(direction),
                                            int(max_legs)))

    def info(self) -> dict:
        s = BatchInfo()
        self._check(self.lib.ecmc_batch_info(self._b, ctypes.byref(s)))
        return s.as_dict()

    def close(self):
        if getattr(self, "_b", None) and self._b.value:
            self.lib.ecmc_batch_free(self._b)
            self._b = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
