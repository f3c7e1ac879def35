"""asep_run_noalloc (the entry point that allocates nothing: its workspace is
one fixed device array per GPU) against the existing entry points
asep_create_ext + asep_run on the same parameters: state words, S1, S2, J, N
exactly, W^2 to 1e-12 relative.  Two calls in a row share the workspace, the
second with a smaller run, so stale contents of the first must not leak."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _noalloc(A, B, torch, params, times):
    lib = B.load()
    sb, ab = ctypes.c_size_t(), ctypes.c_size_t()
    B.check(lib.asep_buffer_sizes(ctypes.byref(params), ctypes.byref(sb), ctypes.byref(ab)),
            "asep_buffer_sizes")
    state = torch.empty(sb.value, dtype=torch.uint8, device="cuda")
    n = len(times)
    R = int(params.samples)
    rec = ctypes.sizeof(B.asep_rough)
    out = torch.empty(max(n * R * rec, 8), dtype=torch.uint8, device="cuda")
    tarr = (ctypes.c_uint64 * max(n, 1))(*times)
    st = torch.cuda.current_stream()
    rc = lib.asep_run_noalloc(ctypes.byref(params), state.data_ptr(), sb.value, st.cuda_stream,
                              tarr, n, out.data_ptr())
    B.check(rc, "asep_run_noalloc")
    torch.cuda.synchronize()
    from paper_1012_0385_amd.sim import _ROUGH_DTYPE

    recs = np.frombuffer(out.cpu().numpy().tobytes(), dtype=_ROUGH_DTYPE, count=n * R)
    words = state.cpu().numpy().view(np.uint64)
    return recs.reshape(n, R), words


def _compare(A, B, torch, kw, samples, times):
    print("case:", kw, "samples", samples, "times", len(times), flush=True)
    P = A.make_params(samples=samples, **kw)
    sim = A.Simulation(P)
    ref = sim.run(times)
    per = sim.planes * sim.L // 64
    ref_words = np.concatenate([sim.read_state(i) for i in range(samples)])
    sim.close()
    got, words = _noalloc(A, B, torch, A.make_params(samples=samples, **kw), times)
    assert np.array_equal(words[: samples * per], ref_words)
    for ti in range(len(times)):
        g, r = got[ti], ref[ti]
        assert np.array_equal(g["sum_h"], r.S1), ("S1", times[ti])
        assert np.array_equal(g["sum_h2_lo"], r.S2_lo), ("S2 lo", times[ti])
        assert np.array_equal(g["sum_h2_hi"], r.S2_hi), ("S2 hi", times[ti])
        assert np.array_equal(g["hops"], r.J), ("J", times[ti])
        assert np.array_equal(g["particles"], r.N), ("N", times[ti])
        rel = np.abs(g["w2"] - r.w2) / np.maximum(np.abs(r.w2), 1e-300)
        assert rel.max() <= 1e-12, ("W2", times[ti], rel.max())


def test_noalloc_equals_run_twice_then_smaller():
    import torch

    import paper_1012_0385_amd as A
    from paper_1012_0385_amd import binding as B

    torch.cuda.set_device(0)
    # 1: windowed rings (second state buffer in the workspace), two quenched
    # planes, backward hops, more than 64 measurement times (two record chunks)
    big = dict(L=1 << 15, p=1.0, q=0.25, slow_frac=0.1, slow_factor=0.5, samples_per_disorder=2,
               seed=3, stream=11, windows=4, window_sweeps=15)
    times = sorted(set([0] + [1 + 3 * i for i in range(70)]))
    _compare(A, B, torch, big, 6, times)
    # 2: a smaller run in the same workspace: whole rings, no quenched planes
    small = dict(L=4096, p=1.0, q=0.0, seed=1, stream=1)
    _compare(A, B, torch, small, 4, [0, 1, 2, 4, 8, 16, 32, 64])


def test_noalloc_two_lanes_and_limits():
    import torch

    import paper_1012_0385_amd as A
    from paper_1012_0385_amd import binding as B

    torch.cuda.set_device(0)
    two = dict(L=2048, model=1, init=1, density=0.3, p=1.0, q=1.0, lane_rate=0.5,
               turn_frac=0.05, seed=1, stream=3)
    _compare(A, B, torch, two, 3, [0, 5, 17, 40])
    # a run whose workspace exceeds the fixed array is refused before any work
    lib = B.load()
    P = A.make_params(L=1 << 22, samples=64)
    sb, ab = ctypes.c_size_t(), ctypes.c_size_t()
    B.check(lib.asep_buffer_sizes(ctypes.byref(P), ctypes.byref(sb), ctypes.byref(ab)),
            "asep_buffer_sizes")
    assert ab.value > B.NOALLOC_SCRATCH_BYTES
    state = torch.empty(sb.value, dtype=torch.uint8, device="cuda")
    out = torch.empty(64 * 48, dtype=torch.uint8, device="cuda")
    tarr = (ctypes.c_uint64 * 1)(0)
    rc = lib.asep_run_noalloc(ctypes.byref(P), state.data_ptr(), sb.value,
                              torch.cuda.current_stream().cuda_stream, tarr, 1, out.data_ptr())
    assert rc == B.ASEP_E_TOO_LARGE
    # a state buffer smaller than the run's state is refused too
    rc = lib.asep_run_noalloc(ctypes.byref(P), state.data_ptr(), sb.value - 8,
                              torch.cuda.current_stream().cuda_stream, tarr, 1, out.data_ptr())
    assert rc == B.ASEP_E_INVAL
