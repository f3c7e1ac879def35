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
