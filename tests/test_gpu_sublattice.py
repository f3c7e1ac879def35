"""Bit-exact parity of the HIP two-sub-lattice update (Sec. 2.1, Fig. parasep)
with the CPU oracle, through the C ABI.

Final state words, and S1, S2, J, N at every measurement time, must be
identical; W^2 must agree to 1e-12 relative.  Cases: the paper's p = 1
degeneracy, one-word and ragged rings, every slot count per lane, dyadic and
general thresholds (the lazily evaluated comparison stops at different bit
planes), forward-only and two-way hopping, columnar disorder on p and q,
windowed (HBM-tier) rings, chunked runs, and prefixes of the L = 2^17
workload at full size.
"""
import numpy as np
import pytest

from tests.test_gpu_parity import compare

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


SUB = 1  # ASEP_SCHED_SUBLATTICE


def test_sublattice_degenerate_p1(orc):
    times = [0, 1, 2, 3, 10, 100]
    got = compare(orc, dict(L=4096, p=1.0, q=0.0, seed=1, stream=1, schedule=SUB), times, 8)
    for ti, t in enumerate(times):
        assert np.all(got[ti].w2 == 0.25) and np.all(got[ti].J == 4096 * t)


@pytest.mark.parametrize("L,p,q,init", [
    (64, 0.8, 0.0, 0),        # one word: the closing pair inside the only slot
    (128, 0.8, 0.3, 1),
    (192, 0.75, 0.25, 1),     # three words, ragged; 2-bit thresholds
    (640, 0.5, 0.5, 1),       # 1-bit thresholds both ways
    (4160, 0.6, 0.45, 1),     # 65 words; 24-bit thresholds
    (4096, 0.3, 0.9, 0),      # drift to the left
    (65600, 0.8, 0.0, 1),     # 1025 words: two slots per lane, ragged last lane
    (1 << 18, 0.8, 0.1, 1),   # 4096 words: eight slots per lane
])
def test_sublattice_shapes(orc, L, p, q, init):
    compare(orc, dict(L=L, p=p, q=q, init=init, density=0.4, seed=7, stream=3, schedule=SUB),
            [0, 1, 4, 11], 3)


def test_sublattice_many_rings_and_offsets(orc):
    compare(orc, dict(L=128, p=0.8, q=0.2, seed=5, stream=9, schedule=SUB), [0, 3, 40], 37)
    compare(orc, dict(L=320, p=0.8, q=0.0, seed=5, stream=9, sample_offset=1000, schedule=SUB),
            [0, 30], 70)


def test_sublattice_explicit_bits(orc):
    compare(orc, dict(L=2048, p=0.8, q=0.0, rbits=24, seed=4, stream=4, schedule=SUB), [0, 7], 2)
    compare(orc, dict(L=2048, p=0.5, q=0.25, rbits=9, seed=4, stream=4, schedule=SUB), [0, 7], 2)


def test_sublattice_disorder(orc):
    kw = dict(L=4096, p=0.8, q=0.0, slow_frac=0.1, slow_factor=0.5, samples_per_disorder=4,
              seed=3, stream=2, schedule=SUB)
    compare(orc, kw, [0, 4, 33], 8)
    kw = dict(L=2048, p=0.75, q=0.5, slow_frac=0.3, slow_factor=0.25, samples_per_disorder=2,
              seed=3, stream=2, sample_offset=5, init=1, schedule=SUB)
    compare(orc, kw, [0, 9, 20], 5)


@pytest.mark.parametrize("L,windows,K", [(4096, 2, 3), (65536, 4, 15), (1 << 17, 4, 63)])
def test_sublattice_windowed(orc, L, windows, K):
    compare(orc, dict(L=L, p=0.8, q=0.1, init=1, density=0.5, seed=6, stream=1, schedule=SUB,
                      windows=windows, window_sweeps=K), [0, 2, 9, 40], 2)


def test_sublattice_windowed_disorder(orc):
    compare(orc, dict(L=16384, p=0.8, q=0.2, slow_frac=0.2, slow_factor=0.3, seed=3, stream=2,
                      schedule=SUB, windows=3, window_sweeps=9), [0, 5, 14], 2)


def test_sublattice_chunks(orc):
    import paper_1012_0385_amd as A

    kw = dict(L=8192, p=0.8, q=0.1, init=1, seed=8, stream=8, schedule=SUB)
    whole = compare(orc, kw, [0, 50], 2)
    sim = A.Simulation(A.make_params(samples=2, **kw))
    for t in (7, 19, 33, 50):
        sim.sweep(t - sim.time)
    r = sim.roughness()
    assert np.array_equal(r.S1, whole[-1].S1) and r.S2 == whole[-1].S2
    assert np.array_equal(r.J, whole[-1].J)
    sim.close()


def test_sublattice_2p17_prefix(orc):
    # the full-size ring of the benchmark: two samples, 200 MCS
    compare(orc, dict(L=1 << 17, p=0.8, q=0.0, seed=1, stream=11, schedule=SUB),
            [0, 31, 200], 2)


# --------------------------------------------------------------------------- two lanes
def _two(**kw):
    base = dict(model=1, init=1, density=0.5, p=0.5, q=0.5, lane_rate=0.8, slow_frac=0.5,
                slow_factor=0.25, seed=2, stream=6, schedule=SUB)
    base.update(kw)
    return base


@pytest.mark.parametrize("L,kw", [
    (64, {}),                                        # one word
    (192, dict(p=0.75, q=0.25)),                     # ragged
    (4096, {}),                                      # the paper's bimodal 0.8 / 0.2 rates
    (4160, dict(lane_rate=0.5, slow_frac=0.0)),      # no marks, dyadic rates
    (65600, dict(p=1.0, q=1.0, lane_rate=1.0, slow_factor=0.5, init=0)),
    (1 << 18, dict(density=0.3)),                    # eight slots per lane
])
def test_two_lane_sublattice_shapes(orc, L, kw):
    compare(orc, _two(L=L, **kw), [0, 1, 3, 9], 3)


def test_two_lane_sublattice_realisations(orc):
    compare(orc, _two(L=2048, samples_per_disorder=2, sample_offset=3), [0, 5, 17], 5)
    compare(orc, _two(L=128), [0, 2, 30], 37)


def test_two_lane_sublattice_windowed(orc):
    compare(orc, _two(L=16384, windows=3, window_sweeps=9), [0, 4, 13], 2)
    compare(orc, _two(L=1 << 17, windows=4, window_sweeps=63), [0, 2, 40], 2)


def test_two_lane_sublattice_paper_sizes(orc):
    # Sec. 3: L = 2^9 ... 2^12 from half-filled random starts
    for L in (512, 4096):
        compare(orc, _two(L=L, stream=L), [0, 30, 100], 4)


def test_two_lane_sublattice_long_ring(orc):
    # 2^19 sites per lane: past the register tier of two lanes, automatic windows
    compare(orc, _two(L=1 << 19), [0, 1, 3], 1)
