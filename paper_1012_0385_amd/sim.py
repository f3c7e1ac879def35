"""Python front end of the C ABI: one ``Simulation`` per asep_sim handle.

Device buffers come from PyTorch (``torch.empty(..., device="cuda")``) and are
handed to ``asep_create_ext`` together with torch's current HIP stream; every
step of the simulation runs in the HIP library.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import binding as B


def make_params(L: int, samples: int = 1, *, model: int = B.ASEP_MODEL_RING,
                init: int = B.ASEP_INIT_FLAT, density: float = 0.5, p: float = 1.0,
                q: float = 0.0, slow_frac: float = 0.0, slow_factor: float = 1.0,
                samples_per_disorder: int = 1, lane_rate: float = 0.0, turn_frac: float = 0.0,
                seed: int = 1, stream: int = 0, cell_log2: int = 0, subsweeps: int = 0,
                rbits: int = 0, sample_offset: int = 0, windows: int = 0,
                window_sweeps: int = 0, rings_per_wg: int = 0,
                schedule: int = B.ASEP_SCHED_SHIFTED) -> B.asep_params:
    P = B.asep_params()
    P.abi_version = B.ASEP_ABI_VERSION
    P.model = model
    P.L = L
    P.samples = samples
    P.sample_offset = sample_offset
    P.init = init
    P.samples_per_disorder = samples_per_disorder
    P.density = density
    P.p = p
    P.q = q
    P.slow_frac = slow_frac
    P.slow_factor = slow_factor
    P.lane_rate = lane_rate
    P.turn_frac = turn_frac
    P.seed = seed & 0xFFFFFFFF
    P.stream = stream & 0xFFFFFFFF
    P.cell_log2 = cell_log2
    P.subsweeps = subsweeps
    P.rbits = rbits
    P.windows = windows
    P.window_sweeps = window_sweeps
    P.rings_per_wg = rings_per_wg
    P.schedule = schedule
    return P


class Rough:
    """Measurements of one time: per-sample exact sums and W^2.

    S1, J, N are int64 arrays, w2 float64; S2 (the 128-bit sum of squared
    heights) is kept as its two 64-bit halves and formed as Python ints on
    first use."""

    __slots__ = ("S1", "S2_lo", "S2_hi", "J", "N", "w2", "_s2")

    def __init__(self, S1, S2_lo, S2_hi, J, N, w2):
        self.S1, self.S2_lo, self.S2_hi, self.J, self.N, self.w2 = S1, S2_lo, S2_hi, J, N, w2
        self._s2 = None

    @property
    def S2(self) -> list:
        if self._s2 is None:
            self._s2 = [(int(h) << 64) + int(lo) for h, lo in zip(self.S2_hi, self.S2_lo)]
        return self._s2


_ROUGH_DTYPE = np.dtype([("sum_h", "<i8"), ("sum_h2_lo", "<u8"), ("sum_h2_hi", "<i8"),
                         ("hops", "<i8"), ("particles", "<i8"), ("w2", "<f8")])


def _rough_arrays(arr, n: int, first: int = 0) -> Rough:
    """Rough of records first..first+n of a ctypes asep_rough array (copied out)."""
    assert ctypes.sizeof(B.asep_rough) == _ROUGH_DTYPE.itemsize
    a = np.frombuffer(arr, dtype=_ROUGH_DTYPE, count=n,
                      offset=first * _ROUGH_DTYPE.itemsize).copy()
    return Rough(a["sum_h"], a["sum_h2_lo"], a["sum_h2_hi"], a["hops"], a["particles"], a["w2"])


class Simulation:
    """An ensemble of rings on the GPU (asep_create_ext with torch buffers)."""

    def __init__(self, params: B.asep_params, *, buffers: str = "torch", device: int = 0,
                 stream=None):
        lib = B.load()
        self.params_in = params
        self._h = ctypes.c_void_p()
        if buffers == "torch":
            import torch

            sb = ctypes.c_size_t()
            ab = ctypes.c_size_t()
            B.check(lib.asep_buffer_sizes(ctypes.byref(params), ctypes.byref(sb),
                                          ctypes.byref(ab)), "asep_buffer_sizes")
            dev = torch.device("cuda", device)
            self.state_buf = torch.empty(max(sb.value, 8), dtype=torch.uint8, device=dev)
            self.aux_buf = torch.empty(max(ab.value, 8), dtype=torch.uint8, device=dev)
            self.torch_stream = stream if stream is not None else torch.cuda.current_stream(dev)
            B.check(lib.asep_create_ext(ctypes.byref(params), self.state_buf.data_ptr(), sb.value,
                                        self.aux_buf.data_ptr(), ab.value,
                                        self.torch_stream.cuda_stream, ctypes.byref(self._h)),
                    "asep_create_ext")
        elif buffers == "library":
            B.check(lib.asep_create(ctypes.byref(params), ctypes.byref(self._h)), "asep_create")
        else:
            raise ValueError(buffers)
        self.params = B.asep_params()
        B.check(lib.asep_get_params(self._h, ctypes.byref(self.params)), "asep_get_params")
        self.L = int(self.params.L)
        self.samples = int(self.params.samples)
        self.planes = 2 if self.params.model == B.ASEP_MODEL_TWO_LANE else 1

    @property
    def handle(self):
        return self._h

    def plan(self) -> dict:
        """The launch plan (asep_get_plan) as a dict."""
        pl = B.asep_plan()
        B.check(B.load().asep_get_plan(self._h, ctypes.byref(pl)), "asep_get_plan")
        return {n: int(getattr(pl, n)) for n, _ in B.asep_plan._fields_ if n != "reserved"}

    @property
    def time(self) -> int:
        return int(B.load().asep_time(self._h))

    def sweep(self, n_mcs: int) -> None:
        B.check(B.load().asep_sweep(self._h, int(n_mcs)), "asep_sweep")

    def roughness(self) -> Rough:
        arr = (B.asep_rough * self.samples)()
        B.check(B.load().asep_roughness(self._h, arr), "asep_roughness")
        return _rough_arrays(arr, self.samples)

    def run(self, times) -> list:
        times = [int(t) for t in times]
        n = len(times)
        tarr = (ctypes.c_uint64 * max(n, 1))(*times)
        arr = (B.asep_rough * max(n * self.samples, 1))()
        B.check(B.load().asep_run(self._h, tarr, n, arr), "asep_run")
        return [_rough_arrays(arr, self.samples, i * self.samples) for i in range(n)]

    def read_state(self, sample: int) -> np.ndarray:
        n = self.planes * self.L // 64
        out = np.zeros(n, dtype=np.uint64)
        B.check(B.load().asep_read_state(self._h, sample,
                                         out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), n),
                "asep_read_state")
        return out

    def write_state(self, sample: int, words: np.ndarray) -> None:
        w = np.ascontiguousarray(words, dtype=np.uint64)
        B.check(B.load().asep_write_state(self._h, sample,
                                          w.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                          w.size), "asep_write_state")

    def read_mask(self, plane: int, realization: int) -> np.ndarray:
        out = np.zeros(self.L // 64, dtype=np.uint64)
        B.check(B.load().asep_read_mask(self._h, plane, realization,
                                        out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                        out.size), "asep_read_mask")
        return out

    def current(self) -> np.ndarray:
        out = np.zeros(self.samples, dtype=np.int64)
        B.check(B.load().asep_current(self._h,
                                      out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))),
                "asep_current")
        return out

    def set_time(self, t: int, hops=None) -> None:
        ptr = None
        if hops is not None:
            h = np.ascontiguousarray(hops, dtype=np.int64)
            ptr = h.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        B.check(B.load().asep_set_time(self._h, int(t), ptr), "asep_set_time")

    def reset(self) -> None:
        B.check(B.load().asep_reset(self._h), "asep_reset")

    def profile(self, enable: bool = True) -> None:
        B.check(B.load().asep_profile_enable(self._h, 1 if enable else 0), "asep_profile_enable")

    def profile_read(self) -> dict:
        st = B.asep_profile_stats()
        B.check(B.load().asep_profile_read(self._h, ctypes.byref(st)), "asep_profile_read")
        return {"launches": int(st.launches), "kernel_ms": float(st.kernel_ms),
                "attempts": int(st.attempts)}

    def close(self) -> None:
        if self._h:
            B.load().asep_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def run_batch(sims, times) -> list:
    """asep_run_batch: advance several simulations through the same times
    concurrently; returns one list of Rough (per time) per simulation."""
    times = [int(t) for t in times]
    n = len(times)
    tarr = (ctypes.c_uint64 * max(n, 1))(*times)
    handles = (ctypes.c_void_p * len(sims))(*[s.handle.value for s in sims])
    bufs = [(B.asep_rough * max(n * s.samples, 1))() for s in sims]
    outs = (ctypes.POINTER(B.asep_rough) * len(sims))(
        *[ctypes.cast(b, ctypes.POINTER(B.asep_rough)) for b in bufs])
    B.check(B.load().asep_run_batch(handles, len(sims), tarr, n, outs), "asep_run_batch")
    res = []
    for s, buf in zip(sims, bufs):
        res.append([_rough_arrays(buf, s.samples, i * s.samples) for i in range(n)])
    return res


def sample_times(t0: float, factor: float, t_max: int, cap: int = 100000) -> list:
    out = (ctypes.c_uint64 * cap)()
    n = ctypes.c_uint32()
    B.check(B.load().asep_sample_times(float(t0), float(factor), int(t_max), out, cap,
                                       ctypes.byref(n)), "asep_sample_times")
    return [int(out[i]) for i in range(n.value)]


def ensemble_w2(rough_list, L: int) -> float:
    """Order-independent ensemble W^2 from exact sums (asep_ensemble_w2)."""
    n = len(rough_list.S1)
    arr = (B.asep_rough * n)()
    for i in range(n):
        arr[i].sum_h = int(rough_list.S1[i])
        arr[i].sum_h2_lo = int(rough_list.S2_lo[i])
        arr[i].sum_h2_hi = int(rough_list.S2_hi[i])
    out = ctypes.c_double()
    B.check(B.load().asep_ensemble_w2(arr, n, L, ctypes.byref(out)), "asep_ensemble_w2")
    return out.value


def resolve(params: B.asep_params):
    """asep_resolve: (resolved parameters, plan dict) without creating anything."""
    out = B.asep_params()
    pl = B.asep_plan()
    B.check(B.load().asep_resolve(ctypes.byref(params), ctypes.byref(out), ctypes.byref(pl)),
            "asep_resolve")
    return out, {n: int(getattr(pl, n)) for n, _ in B.asep_plan._fields_ if n != "reserved"}


def load_tuning(path) -> None:
    """asep_tuning_load: the process-wide tuning table (None clears it)."""
    B.check(B.load().asep_tuning_load(path.encode() if path else None), "asep_tuning_load")


def _params_dict(P) -> dict:
    return {n: getattr(P, n) for n, _ in B.asep_params._fields_}


class Server:
    """The request loop (asep_server_*): submit ensemble runs, collect results."""

    def __init__(self, *, device: int = 0, hbm_budget_bytes: int = 8 << 30, max_queue: int = 1024,
                 max_active: int = 64, quantum_mcs: int = 1000, tuning_path=None):
        cfg = B.asep_server_cfg()
        cfg.abi_version = B.ASEP_ABI_VERSION
        cfg.device = device
        cfg.hbm_budget_bytes = hbm_budget_bytes
        cfg.max_queue = max_queue
        cfg.max_active = max_active
        cfg.quantum_mcs = quantum_mcs
        cfg.tuning_path = tuning_path.encode() if tuning_path else None
        self._h = ctypes.c_void_p()
        B.check(B.load().asep_server_create(ctypes.byref(cfg), ctypes.byref(self._h)),
                "asep_server_create")

    def submit(self, params: B.asep_params, times, t_max: int) -> int:
        times = [int(t) for t in times]
        tarr = (ctypes.c_uint64 * max(len(times), 1))(*times)
        req = B.asep_request()
        req.params = params
        req.t_max = int(t_max)
        req.times = ctypes.cast(tarr, ctypes.POINTER(ctypes.c_uint64))
        req.n_times = len(times)
        ticket = ctypes.c_uint64()
        B.check(B.load().asep_submit(self._h, ctypes.byref(req), ctypes.byref(ticket)),
                "asep_submit")
        return ticket.value

    def _result(self, res: B.asep_result) -> dict:
        out = {"status": int(res.status), "samples": int(res.samples),
               "n_times": int(res.n_times), "arrive_ns": int(res.t_arrive_ns),
               "admit_ns": int(res.t_admit_ns), "start_ns": int(res.t_start_ns),
               "done_ns": int(res.t_done_ns), "site_updates": int(res.site_updates),
               "params": _params_dict(res.params),
               "plan": {n: int(getattr(res.plan, n)) for n, _ in B.asep_plan._fields_
                        if n != "reserved"},
               "quanta": int(res.quanta), "packed_quanta": int(res.packed_quanta),
               "rough": []}
        if res.status == B.ASEP_OK and res.n_times:
            n, R = res.n_times, res.samples
            for i in range(n):
                sub = (B.asep_rough * R).from_address(
                    ctypes.addressof(res.rough.contents) + i * R * ctypes.sizeof(B.asep_rough))
                out["rough"].append(_rough_arrays(sub, R))
            out["times"] = [int(res.times[i]) for i in range(n)]
        B.load().asep_result_free(ctypes.byref(res))
        return out

    def poll(self, ticket: int):
        res = B.asep_result()
        rc = B.load().asep_poll(self._h, ticket, ctypes.byref(res))
        if rc == B.ASEP_E_PENDING:
            return None
        B.check(rc, "asep_poll")
        return self._result(res)

    def wait(self, ticket: int, timeout_s: float = 600.0) -> dict:
        res = B.asep_result()
        B.check(B.load().asep_wait(self._h, ticket, int(timeout_s * 1e9), ctypes.byref(res)),
                "asep_wait")
        return self._result(res)

    def cancel(self, ticket: int) -> None:
        B.check(B.load().asep_cancel(self._h, ticket), "asep_cancel")

    def close(self) -> None:
        if self._h:
            B.load().asep_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
