"""TEST INFRASTRUCTURE ONLY: the CPU oracle for the ASEP / KPZ lattice gas.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library and its
Python binding) never does.

``asep_oracle.c`` is the plain C reference (one byte per site, scalar loops,
the paper's steps in order); this module is its ctypes wrapper plus the exact
small-system tools in :mod:`oracle.master_equation`.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "asep_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")

RING = 0
TWO_LANE = 1
INIT_FLAT = 0
INIT_BERNOULLI = 1
SCHED_SHIFTED = 0
SCHED_SUBLATTICE = 1


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (plain -O2, no SIMD of our own)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-Wall", "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("model", ctypes.c_uint32),
        ("init", ctypes.c_uint32),
        ("L", ctypes.c_uint64),
        ("density", ctypes.c_double),
        ("p", ctypes.c_double),
        ("q", ctypes.c_double),
        ("slow_frac", ctypes.c_double),
        ("slow_factor", ctypes.c_double),
        ("samples_per_disorder", ctypes.c_uint32),
        ("lane_rate", ctypes.c_double),
        ("turn_frac", ctypes.c_double),
        ("seed", ctypes.c_uint32),
        ("stream", ctypes.c_uint32),
        ("cell_log2", ctypes.c_uint32),
        ("subsweeps", ctypes.c_uint32),
        ("rbits", ctypes.c_int32),
        ("schedule", ctypes.c_uint32),
    ]


class _Sched(ctypes.Structure):
    _fields_ = [
        (n, ctypes.c_uint32)
        for n in ("ell", "lam", "ebits", "B", "b", "w", "A", "per_block", "a", "S")
    ] + [
        ("TB", ctypes.c_uint64 * 4),
        ("T", ctypes.c_uint64 * 4),
        ("T_init", ctypes.c_uint64),
        ("T_slow", ctypes.c_uint64),
        ("T_turn", ctypes.c_uint64),
        ("bc", ctypes.c_uint32),
        ("jlow", ctypes.c_uint32),
    ]


class _Record(ctypes.Structure):
    _fields_ = [
        ("S1", ctypes.c_int64),
        ("S2_lo", ctypes.c_uint64),
        ("S2_hi", ctypes.c_int64),
        ("J", ctypes.c_int64),
        ("N", ctypes.c_int64),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = build()
        L = ctypes.CDLL(path)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        i64p = ctypes.POINTER(ctypes.c_int64)
        L.orc_philox.argtypes = [u32p, u32p, u32p]
        L.orc_threshold.argtypes = [ctypes.c_double, ctypes.c_int]
        L.orc_threshold.restype = ctypes.c_uint64
        L.orc_lower.argtypes = [ctypes.POINTER(_Params), ctypes.POINTER(_Sched)]
        L.orc_init_state.argtypes = [ctypes.POINTER(_Params), ctypes.POINTER(_Sched),
                                     ctypes.c_uint32, u8p]
        L.orc_init_masks.argtypes = [ctypes.POINTER(_Params), ctypes.POINTER(_Sched),
                                     ctypes.c_uint32, u8p, u8p, u8p]
        L.orc_sums.argtypes = [u8p, ctypes.c_uint64, i64p, u64p, i64p, i64p]
        L.orc_w2.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_uint64, ctypes.c_int64]
        L.orc_w2.restype = ctypes.c_double
        L.orc_run.argtypes = [ctypes.POINTER(_Params), ctypes.c_uint32, u64p, ctypes.c_uint32,
                              ctypes.POINTER(_Record), u8p]
        L.orc_advance.argtypes = [ctypes.POINTER(_Params), ctypes.c_uint32, u8p,
                                  ctypes.c_uint64, ctypes.c_uint64, i64p]
        L.orc_rsu.argtypes = [ctypes.POINTER(_Params), ctypes.c_uint32, u8p,
                              ctypes.c_uint64, ctypes.c_uint64, i64p]
        L.orc_sample_times.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                                       u64p, ctypes.c_uint32]
        L.orc_sample_times.restype = ctypes.c_uint32
        _lib = L
    return _lib


@dataclass
class Params:
    """Run parameters (same meaning as the library's, written separately)."""

    L: int
    model: int = RING
    init: int = INIT_FLAT
    density: float = 0.5
    p: float = 1.0
    q: float = 0.0
    slow_frac: float = 0.0
    slow_factor: float = 1.0
    samples_per_disorder: int = 1
    lane_rate: float = 0.0
    turn_frac: float = 0.0
    seed: int = 1
    stream: int = 0
    cell_log2: int = 6
    subsweeps: int = 4
    rbits: int = -1
    schedule: int = SCHED_SHIFTED

    def c(self) -> _Params:
        return _Params(self.model, self.init, self.L, self.density, self.p, self.q,
                       self.slow_frac, self.slow_factor, self.samples_per_disorder,
                       self.lane_rate, self.turn_frac, self.seed & 0xFFFFFFFF,
                       self.stream & 0xFFFFFFFF, self.cell_log2, self.subsweeps, self.rbits,
                       self.schedule)

    @property
    def planes(self) -> int:
        return 2 if self.model == TWO_LANE else 1


def _u8(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def philox(ctr, key) -> np.ndarray:
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib().orc_philox(c, k, o)
    return np.array(list(o), dtype=np.uint32)


def threshold(x: float, bits: int) -> int:
    return int(lib().orc_threshold(float(x), int(bits)))


def lower(P: Params) -> dict:
    s = _Sched()
    rc = lib().orc_lower(ctypes.byref(P.c()), ctypes.byref(s))
    if rc != 0:
        raise ValueError("invalid parameters for the oracle")
    d = {n: getattr(s, n) for n, _ in _Sched._fields_ if n not in ("TB", "T")}
    d["TB"] = list(s.TB)
    d["T"] = list(s.T)
    return d


def init_state(P: Params, sample: int) -> np.ndarray:
    s = _Sched()
    pc = P.c()
    if lib().orc_lower(ctypes.byref(pc), ctypes.byref(s)) != 0:
        raise ValueError("invalid parameters")
    st = np.zeros(P.L * P.planes, dtype=np.uint8)
    lib().orc_init_state(ctypes.byref(pc), ctypes.byref(s), sample, _u8(st))
    return st


def init_masks(P: Params, realization: int):
    """Returns (slow_p, slow_q, turn) byte planes (None where the model has none)."""
    s = _Sched()
    pc = P.c()
    if lib().orc_lower(ctypes.byref(pc), ctypes.byref(s)) != 0:
        raise ValueError("invalid parameters")
    sp = np.zeros(P.L, np.uint8)
    sq = np.zeros(P.L, np.uint8)
    tu = np.zeros(P.L, np.uint8)
    lib().orc_init_masks(ctypes.byref(pc), ctypes.byref(s), realization, _u8(sp), _u8(sq), _u8(tu))
    if P.model == TWO_LANE and P.schedule != SCHED_SUBLATTICE:
        return None, None, tu
    if P.slow_frac > 0:
        return sp, (sq if (P.q > 0 or P.model == TWO_LANE) else None), None
    return None, None, None


def sums(state: np.ndarray, L: int):
    """(S1, S2, N) of the first L sites: S2 as a Python int."""
    st = np.ascontiguousarray(state[:L], dtype=np.uint8)
    s1 = ctypes.c_int64()
    lo = ctypes.c_uint64()
    hi = ctypes.c_int64()
    n = ctypes.c_int64()
    lib().orc_sums(_u8(st), L, ctypes.byref(s1), ctypes.byref(lo), ctypes.byref(hi), ctypes.byref(n))
    return s1.value, (hi.value << 64) + lo.value, n.value


def w2(L: int, S1: int, S2: int) -> float:
    lo = S2 & ((1 << 64) - 1)
    hi = S2 >> 64
    return float(lib().orc_w2(L, S1, lo, hi))


@dataclass
class RunResult:
    S1: np.ndarray  # [n_times]
    S2: list        # [n_times] python ints
    J: np.ndarray
    N: np.ndarray
    state: np.ndarray  # final bytes [planes * L]
    times: list = field(default_factory=list)

    def w2(self, L: int) -> np.ndarray:
        return np.array([w2(L, int(a), int(b)) for a, b in zip(self.S1, self.S2)])


def run(P: Params, sample: int, times) -> RunResult:
    times = [int(t) for t in times]
    n = len(times)
    tarr = (ctypes.c_uint64 * max(n, 1))(*times)
    recs = (_Record * max(n, 1))()
    st = np.zeros(P.L * P.planes, dtype=np.uint8)
    rc = lib().orc_run(ctypes.byref(P.c()), sample, tarr, n, recs, _u8(st))
    if rc != 0:
        raise ValueError("oracle run failed (%d)" % rc)
    S1 = np.array([recs[i].S1 for i in range(n)], dtype=np.int64)
    S2 = [(recs[i].S2_hi << 64) + recs[i].S2_lo for i in range(n)]
    J = np.array([recs[i].J for i in range(n)], dtype=np.int64)
    N = np.array([recs[i].N for i in range(n)], dtype=np.int64)
    return RunResult(S1, S2, J, N, st, times)


def advance(P: Params, sample: int, state: np.ndarray, t0: int, n_mcs: int, J: int = 0):
    """Advance a byte state in place by n_mcs MCS starting at MCS t0; returns J."""
    assert state.dtype == np.uint8 and state.flags.c_contiguous
    j = ctypes.c_int64(J)
    rc = lib().orc_advance(ctypes.byref(P.c()), sample, _u8(state), t0, n_mcs, ctypes.byref(j))
    if rc != 0:
        raise ValueError("invalid parameters")
    return j.value


def rsu(P: Params, sample: int, state: np.ndarray, t0: int, n_mcs: int, J: int = 0):
    """Random-sequential update of a byte state in place; returns J."""
    j = ctypes.c_int64(J)
    lib().orc_rsu(ctypes.byref(P.c()), sample, _u8(state), t0, n_mcs, ctypes.byref(j))
    return j.value


def sample_times(t0: float, factor: float, t_max: int, cap: int = 100000) -> list:
    out = (ctypes.c_uint64 * cap)()
    n = lib().orc_sample_times(float(t0), float(factor), int(t_max), out, cap)
    return [int(out[i]) for i in range(n)]


def pack_words(state: np.ndarray) -> np.ndarray:
    """Bytes (one per site) -> uint64 words, site 64w+b at bit b (layout only)."""
    bits = np.asarray(state, dtype=np.uint8).reshape(-1, 64)
    weights = (np.uint64(1) << np.arange(64, dtype=np.uint64))
    return (bits.astype(np.uint64) * weights).sum(axis=1, dtype=np.uint64)


def unpack_words(words: np.ndarray) -> np.ndarray:
    w = np.asarray(words, dtype=np.uint64)
    bits = (w[:, None] >> np.arange(64, dtype=np.uint64)) & np.uint64(1)
    return bits.astype(np.uint8).reshape(-1)
