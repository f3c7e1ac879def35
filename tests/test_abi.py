"""The C-ABI library loads and exports every function include/asep.h declares;
host-only entry points behave as documented (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "asep.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(asep_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1012_0385_amd import binding

    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libasep.so not built")
    return binding.load()


def test_exports_every_declared_symbol(lib):
    names = declared()
    assert len(names) >= 20
    from paper_1012_0385_amd import binding

    for n in names:
        assert hasattr(lib, n), n
        assert n in binding.SIGNATURES, n


def test_host_only_entry_points(lib, orc):
    from paper_1012_0385_amd import binding as B
    import paper_1012_0385_amd as A

    assert lib.asep_strerror(B.ASEP_E_INVAL) == b"invalid argument"
    assert A.sample_times(30, 1.05, 10**7) == orc.sample_times(30, 1.05, 10**7)
    # sizes for the LDS-resident workload: 64 rings of 2^17 sites = 1 MiB of state
    P = A.make_params(L=1 << 17, samples=64)
    sb, ab = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.asep_buffer_sizes(ctypes.byref(P), ctypes.byref(sb), ctypes.byref(ab)) == 0
    assert sb.value == 64 * (1 << 17) // 8
    bad = A.make_params(L=1000, samples=1)
    assert lib.asep_buffer_sizes(ctypes.byref(bad), ctypes.byref(sb), ctypes.byref(ab)) == B.ASEP_E_INVAL
    # the sub-lattice schedules: ell = 2, S = 2 (rings) or 4 (two lanes)
    SUB = B.ASEP_SCHED_SUBLATTICE
    for kw, rc in [(dict(L=4096), 0), (dict(L=64), 0), (dict(L=4096, cell_log2=1, subsweeps=2), 0),
                   (dict(L=4096, cell_log2=6), B.ASEP_E_INVAL),
                   (dict(L=4096, subsweeps=4), B.ASEP_E_INVAL),
                   (dict(L=4096, rbits=25), B.ASEP_E_INVAL),
                   (dict(L=4096, p=0.8, rbits=21), B.ASEP_E_INVAL),
                   (dict(L=4096, model=1, slow_frac=0.5, slow_factor=0.25, lane_rate=0.8), 0),
                   (dict(L=4096, model=1, subsweeps=4), 0),
                   (dict(L=4096, model=1, subsweeps=2), B.ASEP_E_INVAL),
                   (dict(L=4096, model=1, turn_frac=0.05), B.ASEP_E_INVAL)]:
        P = A.make_params(samples=2, schedule=SUB, **kw)
        assert lib.asep_buffer_sizes(ctypes.byref(P), ctypes.byref(sb), ctypes.byref(ab)) == rc, kw
    P = A.make_params(L=4096, samples=1, schedule=2)
    assert lib.asep_buffer_sizes(ctypes.byref(P), ctypes.byref(sb), ctypes.byref(ab)) == B.ASEP_E_INVAL
    # ensemble W^2 of two flat rings is the intrinsic width 1/4
    arr = (B.asep_rough * 2)()
    for i in range(2):
        arr[i].sum_h = -2048
        arr[i].sum_h2_lo = 2048
    out = ctypes.c_double()
    assert lib.asep_ensemble_w2(arr, 2, 4096, ctypes.byref(out)) == 0 and out.value == 0.25


def test_documented_zero_initialisation(lib):
    # the header's recipe: zero-initialise, set abi_version and the run's
    # fields; everything left at zero takes its default (rbits 0: the fewest
    # exact bits), so p = 0.5 resolves to one compared bit
    from paper_1012_0385_amd import binding as B

    P = B.asep_params()
    P.abi_version = B.ASEP_ABI_VERSION
    P.L = 4096
    P.samples = 2
    P.p = 0.5
    P.q = 0.5
    out = B.asep_params()
    plan = B.asep_plan()
    assert lib.asep_resolve(ctypes.byref(P), ctypes.byref(out), ctypes.byref(plan)) == 0
    assert (out.cell_log2, out.subsweeps, out.rbits, out.samples_per_disorder) == (6, 4, 1, 1)
    assert plan.attempt_loop == B.ASEP_LOOP_F4B1 and plan.backward_hops == 1
    P.p = 0.8  # 0.8 is exact only at all 26 bits
    assert lib.asep_resolve(ctypes.byref(P), ctypes.byref(out), None) == 0 and out.rbits == 26
    P.rbits = 3  # an explicit count that leaves 0.8 inexact
    assert lib.asep_resolve(ctypes.byref(P), ctypes.byref(out), None) == B.ASEP_E_INVAL
    P.p, P.q, P.rbits = 1.0, 0.0, 0
    assert lib.asep_resolve(ctypes.byref(P), ctypes.byref(out), ctypes.byref(plan)) == 0
    assert out.rbits == 0 and plan.attempt_loop == B.ASEP_LOOP_F5B0 and plan.backward_hops == 0


def test_tuning_table_fills_zero_parameters(lib, tmp_path):
    import paper_1012_0385_amd as A
    from paper_1012_0385_amd import binding as B

    table = tmp_path / "tune.txt"
    table.write_text(
        "# model schedule disorder log2L_lo log2L_hi samples_lo samples_hi "
        "cell_log2 subsweeps windows window_sweeps rings_per_wg\n"
        "0 0 0 16 17 32 128   6 2   4 127 0   # rings of 2^16..2^17\n"
        "0 0 1 16 16 1 100000 0 0   1 0 0     # disorder: launch shape only\n")
    try:
        A.load_tuning(str(table))
        got, plan = A.resolve(A.make_params(L=1 << 17, samples=64, p=1.0))
        assert (got.cell_log2, got.subsweeps, got.windows, got.window_sweeps) == (6, 2, 4, 127)
        assert plan["windows"] == 4 and plan["window_sweeps"] == 127
        # an explicit schedule field keeps the table's schedule out
        got, _ = A.resolve(A.make_params(L=1 << 17, samples=64, p=1.0, subsweeps=4))
        assert (got.cell_log2, got.subsweeps) == (6, 4)
        # an explicit launch field keeps the table's launch shape out
        got, plan = A.resolve(A.make_params(L=1 << 17, samples=64, p=1.0, windows=1))
        assert got.windows == 1 and got.window_sweeps == 0 and plan["windows"] == 1
        # no matching class: defaults
        got, _ = A.resolve(A.make_params(L=1 << 18, samples=64, p=1.0))
        assert (got.cell_log2, got.subsweeps, got.windows) == (6, 4, 0)
        got, plan = A.resolve(A.make_params(L=1 << 16, samples=4096, p=1.0, slow_frac=0.1,
                                            slow_factor=0.5))
        assert (got.cell_log2, got.subsweeps, got.windows) == (6, 4, 1) and plan["windows"] == 1
        # a malformed table is refused and the one in use stays
        bad = tmp_path / "bad.txt"
        bad.write_text("0 0 0 16 17 32 128 6 2 4 127\n")
        assert lib.asep_tuning_load(str(bad).encode()) == B.ASEP_E_INVAL
        assert lib.asep_tuning_load(str(tmp_path / "missing.txt").encode()) == B.ASEP_E_NOTFOUND
        got, _ = A.resolve(A.make_params(L=1 << 17, samples=64, p=1.0))
        assert got.subsweeps == 2
    finally:
        A.load_tuning(None)
    got, _ = A.resolve(A.make_params(L=1 << 17, samples=64, p=1.0))
    assert (got.subsweeps, got.windows) == (4, 0)
