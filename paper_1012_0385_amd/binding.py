"""ctypes binding of ``libasep.so`` (argument marshalling only).

Every function of ``include/asep.h`` is exposed under the same name with the
same arguments.  All simulation work runs in the HIP library; PyTorch is used
only to hand device memory and streams to ``asep_create_ext``.  Loading fails
loudly when the library has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libasep.so")

ASEP_ABI_VERSION = 3
ASEP_OK = 0
ASEP_E_INVAL = -1
ASEP_E_UNSUPPORTED = -2
ASEP_E_NOMEM = -3
ASEP_E_DEVICE = -4
ASEP_E_BUSY = -5
ASEP_E_PENDING = -6
ASEP_E_CANCELLED = -7
ASEP_E_TIMEOUT = -8
ASEP_E_NOTFOUND = -9
ASEP_E_TOO_LARGE = -10
NOALLOC_SCRATCH_BYTES = 32 << 20
ASEP_MODEL_RING = 0
ASEP_MODEL_TWO_LANE = 1
ASEP_INIT_FLAT = 0
ASEP_INIT_BERNOULLI = 1
ASEP_SCHED_SHIFTED = 0
ASEP_SCHED_SUBLATTICE = 1
ASEP_LOOP_GENERIC = 0
ASEP_LOOP_F5B0 = 1
ASEP_LOOP_F4B1 = 2
ASEP_LOOP_F4B2 = 3
ASEP_LOOP_F1 = 4
ASEP_LOOP_F4B0_LANES = 5
ASEP_LOOP_SUBLATTICE = 6
ASEP_LOOP_H4B0 = 7
ASEP_LOOP_H4B1 = 8


class asep_params(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_uint32),
        ("model", ctypes.c_uint32),
        ("L", ctypes.c_uint64),
        ("samples", ctypes.c_uint32),
        ("sample_offset", ctypes.c_uint32),
        ("init", ctypes.c_uint32),
        ("samples_per_disorder", ctypes.c_uint32),
        ("density", ctypes.c_double),
        ("p", ctypes.c_double),
        ("q", ctypes.c_double),
        ("slow_frac", ctypes.c_double),
        ("slow_factor", ctypes.c_double),
        ("lane_rate", ctypes.c_double),
        ("turn_frac", ctypes.c_double),
        ("seed", ctypes.c_uint32),
        ("stream", ctypes.c_uint32),
        ("cell_log2", ctypes.c_int32),
        ("subsweeps", ctypes.c_int32),
        ("rbits", ctypes.c_int32),
        ("windows", ctypes.c_uint32),
        ("window_sweeps", ctypes.c_uint32),
        ("rings_per_wg", ctypes.c_uint32),
        ("schedule", ctypes.c_uint32),
    ]


class asep_rough(ctypes.Structure):
    _fields_ = [
        ("sum_h", ctypes.c_int64),
        ("sum_h2_lo", ctypes.c_uint64),
        ("sum_h2_hi", ctypes.c_int64),
        ("hops", ctypes.c_int64),
        ("particles", ctypes.c_int64),
        ("w2", ctypes.c_double),
    ]


class asep_plan(ctypes.Structure):
    _fields_ = [
        ("windows", ctypes.c_uint32),
        ("window_sweeps", ctypes.c_uint32),
        ("slots_per_lane", ctypes.c_uint32),
        ("block", ctypes.c_uint32),
        ("lanes_per_ring", ctypes.c_uint32),
        ("rings_per_wg", ctypes.c_uint32),
        ("grid", ctypes.c_uint32),
        ("attempt_loop", ctypes.c_uint32),
        ("backward_hops", ctypes.c_uint32),
        ("packable", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32 * 6),
    ]


class asep_profile_stats(ctypes.Structure):
    _fields_ = [
        ("launches", ctypes.c_uint64),
        ("kernel_ms", ctypes.c_double),
        ("attempts", ctypes.c_uint64),
    ]


class asep_server_cfg(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_uint32),
        ("device", ctypes.c_int32),
        ("hbm_budget_bytes", ctypes.c_uint64),
        ("max_queue", ctypes.c_uint32),
        ("max_active", ctypes.c_uint32),
        ("quantum_mcs", ctypes.c_uint64),
        ("tuning_path", ctypes.c_char_p),
        ("reserved", ctypes.c_uint32 * 4),
    ]


class asep_request(ctypes.Structure):
    _fields_ = [
        ("params", asep_params),
        ("t_max", ctypes.c_uint64),
        ("times", ctypes.POINTER(ctypes.c_uint64)),
        ("n_times", ctypes.c_uint32),
    ]


class asep_result(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("samples", ctypes.c_uint32),
        ("n_times", ctypes.c_uint32),
        ("times", ctypes.POINTER(ctypes.c_uint64)),
        ("rough", ctypes.POINTER(asep_rough)),
        ("t_arrive_ns", ctypes.c_uint64),
        ("t_admit_ns", ctypes.c_uint64),
        ("t_start_ns", ctypes.c_uint64),
        ("t_done_ns", ctypes.c_uint64),
        ("site_updates", ctypes.c_uint64),
        ("params", asep_params),
        ("plan", asep_plan),
        ("quanta", ctypes.c_uint32),
        ("packed_quanta", ctypes.c_uint32),
    ]


_vp = ctypes.c_void_p
_u32 = ctypes.c_uint32
_u64 = ctypes.c_uint64
_i32 = ctypes.c_int32
_sz = ctypes.c_size_t
_P = ctypes.POINTER

# name: (restype, argtypes) -- the declarations of include/asep.h
SIGNATURES = {
    "asep_buffer_sizes": (_i32, [_P(asep_params), _P(_sz), _P(_sz)]),
    "asep_create": (_i32, [_P(asep_params), _P(_vp)]),
    "asep_create_ext": (_i32, [_P(asep_params), _vp, _sz, _vp, _sz, _vp, _P(_vp)]),
    "asep_get_params": (_i32, [_vp, _P(asep_params)]),
    "asep_get_plan": (_i32, [_vp, _P(asep_plan)]),
    "asep_resolve": (_i32, [_P(asep_params), _P(asep_params), _P(asep_plan)]),
    "asep_sweep": (_i32, [_vp, _u64]),
    "asep_roughness": (_i32, [_vp, _P(asep_rough)]),
    "asep_run": (_i32, [_vp, _P(_u64), _u32, _P(asep_rough)]),
    "asep_run_noalloc": (_i32, [_P(asep_params), _vp, ctypes.c_size_t, _vp, _P(_u64), _u32,
                                 _vp]),
    "asep_run_batch": (_i32, [_P(_vp), _u32, _P(_u64), _u32, _P(_P(asep_rough))]),
    "asep_read_state": (_i32, [_vp, _u32, _P(_u64), _u64]),
    "asep_write_state": (_i32, [_vp, _u32, _P(_u64), _u64]),
    "asep_read_mask": (_i32, [_vp, _u32, _u32, _P(_u64), _u64]),
    "asep_current": (_i32, [_vp, _P(ctypes.c_int64)]),
    "asep_set_time": (_i32, [_vp, _u64, _P(ctypes.c_int64)]),
    "asep_reset": (_i32, [_vp]),
    "asep_profile_enable": (_i32, [_vp, _i32]),
    "asep_profile_read": (_i32, [_vp, _P(asep_profile_stats)]),
    "asep_time": (_u64, [_vp]),
    "asep_destroy": (None, [_vp]),
    "asep_ensemble_w2": (_i32, [_P(asep_rough), _u32, _u64, _P(ctypes.c_double)]),
    "asep_sample_times": (_i32, [ctypes.c_double, ctypes.c_double, _u64, _P(_u64), _u32,
                                 _P(_u32)]),
    "asep_strerror": (ctypes.c_char_p, [_i32]),
    "asep_last_device_error": (ctypes.c_char_p, []),
    "asep_tuning_load": (_i32, [ctypes.c_char_p]),
    "asep_server_create": (_i32, [_P(asep_server_cfg), _P(_vp)]),
    "asep_server_destroy": (None, [_vp]),
    "asep_submit": (_i32, [_vp, _P(asep_request), _P(_u64)]),
    "asep_poll": (_i32, [_vp, _u64, _P(asep_result)]),
    "asep_wait": (_i32, [_vp, _u64, _u64, _P(asep_result)]),
    "asep_cancel": (_i32, [_vp, _u64]),
    "asep_result_free": (None, [_P(asep_result)]),
}

_lib = None


def load() -> ctypes.CDLL:
    """Load libasep.so; raises if it is missing (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                "libasep.so is not built (%s); run __graft_entry__.build() or "
                "python -m paper_1012_0385_amd.build" % LIB_PATH)
        # PyTorch ships its own HIP runtime with the same soname as ROCm's;
        # loading torch first makes this library bind to that one, so a
        # process never holds two HIP runtimes (the second sees no device).
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class AsepError(RuntimeError):
    def __init__(self, code: int, where: str):
        lib = load()
        msg = "%s: %s" % (where, lib.asep_strerror(code).decode())
        if code == ASEP_E_DEVICE:
            msg += " [%s]" % lib.asep_last_device_error().decode()
        super().__init__(msg)
        self.code = code


def check(code: int, where: str) -> int:
    if code < 0:
        raise AsepError(code, where)
    return code


def __getattr__(name):
    # module-level access to the C functions under their C names
    if name in SIGNATURES:
        return getattr(load(), name)
    raise AttributeError(name)
