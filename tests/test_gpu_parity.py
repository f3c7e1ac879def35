"""Bit-exact parity of the HIP path (through the C ABI) with the CPU oracle.

Words of the final state, and S1, S2, J, N at every measurement time, must
be identical; W^2 formed from them must agree to 1e-12 relative.  Cases span
several workgroup tiles, ragged ring lengths and packings, every cell size
and sub-sweep count the kernels accept, the dyadic (packed) and general
threshold encodings, quenched disorder, two lanes, and prefixes of the
benchmark workloads at their full ring sizes.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


import paper_1012_0385_amd as A  # noqa: E402
from paper_1012_0385_amd import binding as B  # noqa: E402


def oracle_params(orc, kw):
    """The same run parameters in the oracle's own structure."""
    return orc.Params(
        L=kw["L"], model=kw.get("model", 0), init=kw.get("init", 0),
        density=kw.get("density", 0.5), p=kw.get("p", 1.0), q=kw.get("q", 0.0),
        slow_frac=kw.get("slow_frac", 0.0), slow_factor=kw.get("slow_factor", 1.0),
        samples_per_disorder=kw.get("samples_per_disorder", 1),
        lane_rate=kw.get("lane_rate", 0.0), turn_frac=kw.get("turn_frac", 0.0),
        seed=kw.get("seed", 1), stream=kw.get("stream", 0),
        cell_log2=kw.get("cell_log2", 6) or 6, subsweeps=kw.get("subsweeps", 4) or 4,
        rbits=kw.get("rbits", -1), schedule=kw.get("schedule", 0))


def compare(orc, kw, times, samples, check_states=True, buffers="torch"):
    print("case:", kw, "times", times[:4], "...", len(times), "samples", samples, flush=True)
    P = A.make_params(samples=samples, **kw)
    sim = A.Simulation(P, buffers=buffers)
    got = sim.run(times)
    OP = oracle_params(orc, kw)
    off = kw.get("sample_offset", 0)
    for i in range(samples):
        ref = orc.run(OP, off + i, times)
        for ti in range(len(times)):
            g = got[ti]
            assert g.S1[i] == ref.S1[ti], ("S1", i, times[ti])
            assert g.S2[i] == ref.S2[ti], ("S2", i, times[ti])
            assert g.J[i] == ref.J[ti], ("J", i, times[ti])
            assert g.N[i] == ref.N[ti], ("N", i, times[ti])
            w = orc.w2(kw["L"], int(ref.S1[ti]), ref.S2[ti])
            assert abs(g.w2[i] - w) <= 1e-12 * max(abs(w), 1e-300)
        if check_states:
            words = sim.read_state(i)
            assert np.array_equal(words, orc.pack_words(ref.state)), ("state", i)
    sim.close()
    return got


def test_flat_start_and_config1(orc):
    # plain ring, L = 4096, 8 samples, p = 1, q = 0, flat start, 1000 MCS,
    # measured at t = 0 and powers of two
    times = [0] + [2**k for k in range(10)] + [1000]
    got = compare(orc, dict(L=4096, p=1.0, q=0.0, seed=1, stream=1), times, 8)
    assert np.all(got[0].w2 == 0.25)


@pytest.mark.parametrize("L,cell_log2,S,p,q", [
    (128, 6, 4, 1.0, 0.0),       # two cells, one word per lane
    (192, 6, 1, 0.5, 0.5),       # three words, ragged
    (640, 6, 16, 0.8, 0.1),      # general thresholds (one attempt per 32 bits)
    (4160, 6, 64, 0.75, 0.25),   # ragged 65-word ring
    (64, 5, 2, 1.0, 0.0),        # one word: a lane is its own neighbour
    (1024, 5, 8, 0.6, 0.3),
    (2048, 4, 4, 1.0, 0.5),
    (512, 3, 1, 0.9, 0.0),
    (256, 1, 2, 0.7, 0.2),       # two-site cells
    (65600, 6, 4, 1.0, 0.0),     # 1025 words: C = 2 with a ragged last lane
])
def test_plain_shapes(orc, L, cell_log2, S, p, q):
    compare(orc, dict(L=L, cell_log2=cell_log2, subsweeps=S, p=p, q=q, seed=7, stream=3,
                      init=1, density=0.4), [0, 1, 5, 12], 3)


@pytest.mark.parametrize("kw", [
    dict(L=64000, p=1.0, q=0.0),                                        # 1000 lanes
    dict(L=64000, p=0.5, q=0.5, init=1, density=0.4),
    dict(L=64000, p=1.0, q=0.0, slow_frac=0.1, slow_factor=0.5),
    dict(L=64000, model=1, init=1, density=0.3, p=1.0, q=1.0, lane_rate=0.1, turn_frac=0.05),
    dict(L=96000, p=0.75, q=0.25, init=1),                              # 2 slots, 750 lanes
])
def test_whole_ring_partial_last_wave(orc, kw):
    # one ring per workgroup whose lanes end inside a wave: the last wave's
    # remaining lanes belong to no ring, so every wave still serves one ring
    compare(orc, dict(seed=8, stream=4, windows=1, **kw), [0, 1, 6, 13], 2)


def test_many_rings_per_workgroup(orc):
    # 37 rings of 2 words: packed 128 per workgroup, last workgroup partial
    compare(orc, dict(L=128, p=0.8, q=0.3, seed=5, stream=9), [0, 3, 40], 37)
    compare(orc, dict(L=320, p=1.0, q=0.0, seed=5, stream=9, sample_offset=1000), [0, 30], 70)


@pytest.mark.parametrize("kw", [
    dict(L=64, p=1.0, q=0.0, cell_log2=5, subsweeps=2),                 # byte fields, q = 0
    dict(L=64, p=0.5, q=0.5, cell_log2=5, subsweeps=2, init=1),         # byte fields, one bit
    dict(L=64, p=0.8, q=0.3, cell_log2=4, subsweeps=4),                 # generic loop
    dict(L=64, p=1.0, q=0.25, cell_log2=5, subsweeps=2, slow_frac=0.3, slow_factor=0.5),
    dict(L=64, model=1, init=1, density=0.4, p=1.0, q=1.0, lane_rate=0.5, turn_frac=0.3,
         cell_log2=5, subsweeps=8),                                     # two lanes
    dict(L=128, p=0.5, q=0.5, cell_log2=5, subsweeps=2, init=1),
])
def test_one_and_two_word_rings(orc, kw):
    # every frame puts the closing bond (L-1, 0) inside the ring's last slot,
    # which here is also its first: the hop count taken at that bond and from
    # the position sums must still equal the oracle's count of hops
    compare(orc, dict(seed=12, stream=3, **kw), [0, 1, 2, 7, 50, 333], 70)


def test_disorder(orc):
    kw = dict(L=4096, p=1.0, q=0.0, slow_frac=0.1, slow_factor=0.5, samples_per_disorder=4,
              seed=3, stream=2)
    compare(orc, kw, [0, 4, 33], 8)
    kw = dict(L=2048, p=0.75, q=0.5, slow_frac=0.3, slow_factor=0.25, samples_per_disorder=2,
              seed=3, stream=2, sample_offset=5, subsweeps=16)
    compare(orc, kw, [0, 9, 20], 5)


@pytest.mark.parametrize("rates", [
    dict(p=1.0, q=1.0, slow_factor=0.5),    # 1 compared bit, marks of both directions
    dict(p=1.0, q=0.0, slow_factor=0.25),   # 2 compared bits, forward marks only
    dict(p=0.5, q=0.0, slow_factor=0.5),    # 2 compared bits
    dict(p=1.0, q=1.0, slow_factor=0.0),    # 0 compared bits: slow bonds closed
    dict(p=0.5, q=0.5, slow_factor=1.0),    # marks present, rates equal
])
def test_disorder_outcome_bits(orc, rates):
    # rates on a grid of 1/2 or 1/4: the attempt reads its outcome from one
    # bit indexed by the pair, the compared bits and the marks
    kw = dict(L=4096, slow_frac=0.3, samples_per_disorder=2, seed=8, stream=5, **rates)
    compare(orc, kw, [0, 5, 21], 5)
    compare(orc, dict(kw, windows=3, window_sweeps=7), [0, 5, 21], 5)


def test_disorder_masks_match_oracle(orc):
    kw = dict(L=4096, p=0.75, q=0.5, slow_frac=0.1, slow_factor=0.5, samples_per_disorder=4,
              seed=3, stream=2, sample_offset=6)
    sim = A.Simulation(A.make_params(samples=7, **kw))
    OP = oracle_params(orc, kw)
    for real in (1, 2, 3):
        sp, sq, _ = orc.init_masks(OP, real)
        assert np.array_equal(sim.read_mask(0, real), orc.pack_words(sp))
        assert np.array_equal(sim.read_mask(1, real), orc.pack_words(sq))
    sim.close()


@pytest.mark.parametrize("L,S,lane_rate,turn", [(1024, 4, 0.1, 0.05), (256, 16, 0.25, 0.5),
                                                 (4160, 1, 0.5, 0.3)])
def test_two_lane(orc, L, S, lane_rate, turn):
    kw = dict(L=L, model=1, init=1, density=0.3, p=1.0, q=1.0, lane_rate=lane_rate,
              turn_frac=turn, subsweeps=S, seed=11, stream=4)
    compare(orc, kw, [0, 2, 15], 5)


@pytest.mark.parametrize("rates", [
    dict(p=1.0, q=0.0), dict(p=0.5, q=0.5, init=1, density=0.4),
    dict(p=1.0, q=0.0, slow_frac=0.1, slow_factor=0.5, samples_per_disorder=2),
    dict(p=0.5, q=0.5, slow_frac=0.3, slow_factor=0.0, init=1, density=0.4),
], ids=["kpz", "ew", "kpz-disorder", "ew-disorder-closed"])
@pytest.mark.parametrize("shape", [dict(L=4096), dict(L=4160, windows=1),
                                   dict(L=1 << 17, windows=4, window_sweeps=255),
                                   dict(L=1 << 15, windows=3, window_sweeps=31)],
                         ids=["small-packed", "ragged", "windows-K255", "windows-K31"])
def test_half_word_cells(orc, rates, shape):
    # cells of 32 sites with two sub-sweeps per MCS: the attempt loop that
    # updates a slot's two halves as two cells, in small rings packed several
    # per workgroup, a ragged ring, and windows (several launches)
    kw = dict(dict(cell_log2=5, subsweeps=2, seed=21, stream=6), **rates, **shape)
    sim = A.Simulation(A.make_params(samples=1, **kw))
    loop = sim.plan()["attempt_loop"]
    sim.close()
    nbits = 1 if rates["p"] < 1 or rates.get("slow_factor", 0) > 0 else 0
    assert loop == (B.ASEP_LOOP_H4B0 if nbits == 0 else B.ASEP_LOOP_H4B1)
    compare(orc, kw, [0, 1, 7, 130, 300], 3)


@pytest.mark.parametrize("kw", [
    dict(L=4096 + 64, p=0.875, q=0.25, init=1),                 # 3 compared bits: generic loop
    dict(L=4096, p=1.0, q=0.0, subsweeps=1),                     # 32 attempts: two blocks per cell
    dict(L=4096, p=0.9375, q=0.0),                               # 9-bit fields: packed, not bytes
    dict(L=2048, model=1, init=1, density=0.3, p=1.0, q=1.0, lane_rate=0.1,
         turn_frac=0.05),                                        # two lanes, 7-bit fields: bytes
], ids=["b3-ragged", "S1", "b4-packed", "two-lane"])
def test_byte_fields_in_generic_loops(orc, kw):
    # cells of 32 sites outside the fast loop: the generic loops read the
    # fields' offsets from the schedule (bytes with the position low, or
    # packed fields with the position on top)
    kw = dict(dict(cell_log2=5, subsweeps=2, seed=13, stream=9), **kw)
    compare(orc, kw, [0, 1, 6, 40], 3)


@pytest.mark.parametrize("kw,samples", [
    (dict(L=64 * 67, model=1, init=1, density=0.3, p=1.0, q=1.0, lane_rate=0.1,
          turn_frac=0.05), 3),                                   # odd word count, two planes
    (dict(L=64 * 33331, init=1, density=0.45, p=0.5, q=0.5), 2),  # many segments per ring
    (dict(L=4096, init=1, density=0.5), 70),                      # one segment per ring
], ids=["two-lane-odd", "long-odd", "many-rings"])
def test_roughness_of_any_layout(orc, kw, samples):
    # the measurement of rings in HBM (segments summed per wave, combined per
    # ring in 128 bits) against the oracle's sums of the words read back
    sim = A.Simulation(A.make_params(samples=samples, seed=4, stream=2, **kw))
    sim.sweep(3)
    r = sim.roughness()
    L = kw["L"]
    for i in range(samples):
        st = orc.unpack_words(sim.read_state(i))
        S1, S2, N = orc.sums(st, L)
        if kw.get("model", 0) == 1:
            N += int(st[L:].sum())
        assert (r.S1[i], r.S2[i], r.N[i]) == (S1, S2, N), i
        assert abs(r.w2[i] - orc.w2(L, S1, S2)) <= 1e-12 * orc.w2(L, S1, S2)
    sim.close()


@pytest.mark.parametrize("lane_rate", [0.5, 0.1, 1.0])
def test_two_lane_many_lane_changes(orc, lane_rate):
    # every site a turning point, half filled lanes: most cells meet more
    # than four lane-change candidates per sub-sweep, the case the fast loop
    # hands to its exact replay; lane_rate 1 changes lanes without a draw
    kw = dict(L=4096, model=1, init=1, density=0.5, p=1.0, q=1.0, lane_rate=lane_rate,
              turn_frac=1.0, seed=5, stream=9)
    compare(orc, kw, [0, 1, 4, 9], 3)
    # the same with cells of 32 sites (the generic loop, byte fields)
    compare(orc, dict(kw, cell_log2=5, subsweeps=2), [0, 1, 4, 9], 3)


def test_two_lane_general_rates(orc):
    kw = dict(L=512, model=1, init=1, density=0.5, p=0.7, q=0.4, lane_rate=0.1,
              turn_frac=0.2, seed=2, stream=8)
    compare(orc, kw, [0, 6], 4)


def test_chunks_and_roughness_agree(orc):
    kw = dict(L=2048, p=0.5, q=0.5, seed=9, stream=1)
    P = A.make_params(samples=4, **kw)
    s1 = A.Simulation(P)
    s1.sweep(5)
    s1.sweep(7)
    r1 = s1.roughness()
    s2 = A.Simulation(P)
    r2 = s2.run([12])[0]
    assert np.array_equal(r1.S1, r2.S1) and r1.S2 == r2.S2 and np.array_equal(r1.J, r2.J)
    for i in range(4):
        assert np.array_equal(s1.read_state(i), s2.read_state(i))
    s1.close()
    s2.close()


def test_library_buffers_equal_borrowed(orc):
    kw = dict(L=1024, p=0.9, q=0.2, seed=4, stream=4)
    a = compare(orc, kw, [0, 10], 3, buffers="library")
    b = compare(orc, kw, [0, 10], 3, buffers="torch")
    assert np.array_equal(a[1].S1, b[1].S1)


def test_checkpoint_resume(orc):
    kw = dict(L=1024, p=0.8, q=0.1, seed=6, stream=2)
    P = A.make_params(samples=2, **kw)
    sim = A.Simulation(P)
    sim.sweep(9)
    words = [sim.read_state(i) for i in range(2)]
    hops = sim.current()
    sim.sweep(6)
    want = [sim.read_state(i) for i in range(2)]
    sim2 = A.Simulation(P)
    for i in range(2):
        sim2.write_state(i, words[i])
    sim2.set_time(9, hops)
    sim2.sweep(6)
    for i in range(2):
        assert np.array_equal(sim2.read_state(i), want[i])
    assert np.array_equal(sim2.current(), sim.current())
    # a state written from the host continues like the oracle from that state
    OP = oracle_params(orc, kw)
    st = orc.unpack_words(words[1])
    J = orc.advance(OP, 1, st, 9, 6, int(hops[1]))
    assert np.array_equal(orc.pack_words(st), want[1]) and J == sim.current()[1]
    sim.close()
    sim2.close()


def test_sampling_times_match_oracle(orc):
    assert A.sample_times(30, 1.05, 10**7) == orc.sample_times(30, 1.05, 10**7)
    assert A.sample_times(30, 1.05, 10**5) == orc.sample_times(30, 1.05, 10**5)


def test_ensemble_w2_matches_mean():
    P = A.make_params(samples=6, L=1024, p=1.0, q=0.0)
    sim = A.Simulation(P)
    r = sim.run([0, 50])[1]
    ens = A.ensemble_w2(r, 1024)
    assert abs(ens - r.w2.mean()) <= 1e-12 * ens
    sim.close()


# --------------------------------------------------------------------------- workload prefixes
def test_kpz_ew_rings_2p17_prefix(orc):
    # the LDS-resident workload's ring size: L = 2^17, flat start, KPZ and EW
    for stream, (p, q) in ((0, (1.0, 0.0)), (1, (0.5, 0.5))):
        compare(orc, dict(L=1 << 17, p=p, q=q, seed=1, stream=stream), [0, 1, 8, 20], 3)


def test_columnar_disorder_2p16_prefix(orc):
    kw = dict(L=1 << 16, p=1.0, q=0.0, slow_frac=0.1, slow_factor=0.5, samples_per_disorder=4,
              seed=1, stream=2)
    compare(orc, kw, [0, 5, 12], 8)


def test_two_lane_2p16_prefix(orc):
    kw = dict(L=1 << 16, model=1, init=1, density=0.3, p=1.0, q=1.0, lane_rate=0.1,
              turn_frac=0.05, seed=1, stream=3)
    compare(orc, kw, [0, 3, 6], 3)


def test_largest_register_ring(orc):
    # 2^19 sites: 16 slots per lane, 512 lanes
    compare(orc, dict(L=1 << 19, p=1.0, q=0.0, seed=2, stream=5), [0, 2], 1)


@pytest.mark.parametrize("kw", [
    dict(p=0.5, q=0.5),                                   # 4 fields, one compared bit
    dict(p=0.75, q=0.25, init=1, density=0.4),            # 4 fields, two compared bits
    dict(p=1.0, q=0.0, slow_frac=0.1, slow_factor=0.5),   # disorder, outcome bits with marks
    dict(p=0.8, q=0.1, init=1),                           # general rates: the generic loop
])
def test_sixteen_slot_loops(orc, kw):
    # whole rings of 2^19 sites hold 16 slots per lane: the packed attempt
    # loops with measurements inside the launch, then without (a bare sweep)
    kw = dict(L=1 << 19, seed=2, stream=6, windows=1, **kw)
    compare(orc, kw, [0, 1, 3], 2)
    sim = A.Simulation(A.make_params(samples=2, **kw))
    sim.sweep(2)
    OP = oracle_params(orc, kw)
    for i in range(2):
        st = orc.init_state(OP, i)
        orc.advance(OP, i, st, 0, 2)
        assert np.array_equal(sim.read_state(i), orc.pack_words(st)), i
    sim.close()


# --------------------------------------------------------------------------- windows (HBM tier)
@pytest.mark.parametrize("L,windows,K,S,p,q", [
    (4096, 2, 3, 4, 1.0, 0.0),     # 64 words in 2 windows, 3 sub-sweeps per launch
    (4096, 3, 7, 4, 0.5, 0.5),     # ragged last window
    (8192, 4, 13, 16, 0.8, 0.1),   # general thresholds, launches end mid-MCS
    (6400, 5, 1, 1, 0.75, 0.25),   # one sub-sweep per launch
    (16384, 2, 63, 4, 1.0, 0.0),   # default launch length
])
def test_windowed_rings(orc, L, windows, K, S, p, q):
    kw = dict(L=L, p=p, q=q, subsweeps=S, seed=3, stream=7, init=1, density=0.45,
              windows=windows, window_sweeps=K)
    compare(orc, kw, [0, 1, 3, 10, 11], 3)


def test_windowed_disorder_and_two_lane(orc):
    kw = dict(L=8192, p=0.75, q=0.5, slow_frac=0.2, slow_factor=0.5, samples_per_disorder=2,
              seed=3, stream=2, windows=3, window_sweeps=9)
    compare(orc, kw, [0, 7, 15], 4)
    kw = dict(L=4096, model=1, init=1, density=0.3, p=1.0, q=1.0, lane_rate=0.1,
              turn_frac=0.05, seed=1, stream=3, windows=2, window_sweeps=5)
    compare(orc, kw, [0, 3, 8], 3)


def test_windowed_equals_whole(orc):
    # the launch shape never changes a result
    base = dict(L=32768, p=1.0, q=0.0, seed=4, stream=1)
    a = compare(orc, dict(base, windows=1), [0, 5, 9], 2)
    b = compare(orc, dict(base, windows=4, window_sweeps=11), [0, 5, 9], 2)
    for x, y in zip(a, b):
        assert np.array_equal(x.S1, y.S1) and x.S2 == y.S2 and np.array_equal(x.J, y.J)


def test_hbm_ring_2p21(orc):
    # a ring too long for one workgroup: 2^21 sites, automatic windows
    compare(orc, dict(L=1 << 21, p=1.0, q=0.0, seed=2, stream=5), [0, 1, 3], 1)


def test_largest_served_ring(orc):
    # the longest ring of the served mix: 2^26 sites (2^20 words, 8 MiB per
    # ring), automatic windows, random start so the heights are large
    kw = dict(L=1 << 26, p=0.8, q=0.2, init=1, density=0.5, seed=3, stream=9)
    compare(orc, kw, [0, 1, 2], 1)


@pytest.mark.parametrize("shape", [dict(windows=1), dict(windows=2, window_sweeps=7)])
@pytest.mark.parametrize("kw", [
    dict(init=1, density=0.0, p=0.7, q=0.3),                    # empty ring
    dict(init=1, density=1.0, p=0.7, q=0.3),                    # full ring
    dict(init=1, density=0.5, p=0.0, q=0.0),                    # no hops at all
    dict(init=1, density=0.4, p=0.0, q=0.0, slow_frac=0.5, slow_factor=0.5),
    dict(model=1, init=1, density=0.0, p=1.0, q=1.0, lane_rate=0.1, turn_frac=0.05),
])
def test_degenerate_cases(orc, kw, shape):
    # nothing can move: every record equals the oracle's, no hop is counted,
    # and the final words are the initial ones
    kw = dict(L=8192, seed=4, stream=11, **kw, **shape)
    got = compare(orc, kw, [0, 2, 9], 2)
    assert all(int(j) == 0 for r in got for j in r.J)
    OP = oracle_params(orc, kw)
    sim = A.Simulation(A.make_params(samples=2, **kw))
    sim.sweep(9)
    for i in range(2):
        assert np.array_equal(sim.read_state(i), orc.pack_words(orc.init_state(OP, i))), i
    sim.close()


def test_run_batch_equals_alone(orc):
    kws = [dict(L=4096, p=1.0, q=0.0, seed=1, stream=0), dict(L=4096, p=0.5, q=0.5, seed=1, stream=1),
           dict(L=65536, p=1.0, q=0.0, seed=2, stream=2, windows=2, window_sweeps=17)]
    times = [0, 2, 9, 30]
    sims = [A.Simulation(A.make_params(samples=3, **kw), stream=torch.cuda.Stream()) for kw in kws]
    got = A.run_batch(sims, times)
    for kw, g in zip(kws, got):
        alone = compare(orc, kw, times, 3)
        for x, y in zip(g, alone):
            assert np.array_equal(x.S1, y.S1) and x.S2 == y.S2 and np.array_equal(x.J, y.J)
    for s in sims:
        s.close()


def _site_bits(words):
    return np.unpackbits(np.asarray(words, dtype="<u8").view(np.uint8), bitorder="little")


def test_benchmark_configuration(orc):
    # the benchmark exactly: 64 KPZ and 64 EW rings of 2^17 sites from the flat
    # start, at the tuned launch shape and cell schedule of the shipped table,
    # both ensembles advanced together; sampled rings against the oracle (with
    # the schedule the library resolved), every ring against the conservation
    # law and the hop-count identity (J = change of the position sum modulo L)
    from concurrent.futures import ThreadPoolExecutor

    from paper_1012_0385_amd import tune
    from parity_util import oracle_params_from

    L, R, times = 1 << 17, 64, [0, 1, 8, 64, 200]
    kws = [dict(L=L, p=1.0, q=0.0, seed=1, stream=0), dict(L=L, p=0.5, q=0.5, seed=1, stream=1)]
    sims = []
    try:
        A.load_tuning(tune.DEFAULT_TABLE)
        for kw in kws:
            sims.append(A.Simulation(A.make_params(samples=R, **kw), stream=torch.cuda.Stream()))
            print("case: benchmark ensemble", kw, sims[-1].plan(), "cell", 1 << sims[-1].params.cell_log2,
                  "S", sims[-1].params.subsweeps, flush=True)
    finally:
        A.load_tuning(None)
    got = A.run_batch(sims, times)
    pos = np.arange(L, dtype=np.int64)
    P0 = int(pos[::2].sum())
    picks = (0, 37, R - 1)
    with ThreadPoolExecutor(6) as ex:
        refs = {(m, i): ex.submit(orc.run, oracle_params_from(orc, sims[m].params), i, times)
                for m, kw in enumerate(kws) for i in picks}
        for m, (kw, sim, g) in enumerate(zip(kws, sims, got)):
            for i in range(R):
                bits = _site_bits(sim.read_state(i))
                assert int(bits.sum()) == L // 2 and all(int(r.N[i]) == L // 2 for r in g), (m, i)
                dP = int((pos * bits).sum()) - P0
                assert (int(g[-1].J[i]) - dP) % L == 0, (m, i)
            for i in picks:
                ref = refs[(m, i)].result()
                for ti in range(len(times)):
                    assert g[ti].S1[i] == ref.S1[ti] and g[ti].S2[i] == ref.S2[ti], (m, i, times[ti])
                    assert g[ti].J[i] == ref.J[ti], (m, i, times[ti])
                    w = orc.w2(L, int(ref.S1[ti]), ref.S2[ti])
                    assert abs(g[ti].w2[i] - w) <= 1e-12 * max(abs(w), 1e-300)
                assert np.array_equal(sim.read_state(i), orc.pack_words(ref.state)), (m, i)
    for s in sims:
        s.close()


def test_invalid_parameters_rejected():
    lib = B.load()
    bad = [dict(L=100), dict(L=64, cell_log2=6), dict(L=1024, p=1.5), dict(L=1024, subsweeps=3),
           dict(L=1024, model=1, slow_frac=0.1)]
    for kw in bad:
        P = A.make_params(samples=1, **kw)
        import ctypes
        h = ctypes.c_void_p()
        assert lib.asep_create(ctypes.byref(P), ctypes.byref(h)) < 0
        assert not h.value


def _records_and_states(kw, times, samples):
    sim = A.Simulation(A.make_params(samples=samples, **kw))
    rec = sim.run(times)
    states = [sim.read_state(i) for i in range(samples)]
    sim.close()
    return rec, states


@pytest.mark.parametrize("base", [
    dict(L=8192, p=0.75, q=0.25, init=1, seed=4, stream=4),
    dict(L=8192, p=0.8, q=0.1, init=1, seed=4, stream=5, schedule=1),
    dict(L=4096, model=1, init=1, p=0.5, q=0.5, lane_rate=0.8, slow_frac=0.5, slow_factor=0.25,
         seed=4, stream=6, schedule=1),
])
def test_launch_shape_invariance(base):
    # rings per workgroup, whole rings vs windows of several sizes and reaches:
    # launch shape only, so every record and every final word is identical
    times = [0, 3, 10, 31]
    ref, ref_states = _records_and_states(dict(base, windows=1, rings_per_wg=1), times, 6)
    for shape in [dict(windows=1, rings_per_wg=2), dict(windows=1, rings_per_wg=6),
                  dict(windows=2, window_sweeps=5), dict(windows=3, window_sweeps=13),
                  dict(windows=4, window_sweeps=2)]:
        got, states = _records_and_states(dict(base, **shape), times, 6)
        for x, y in zip(got, ref):
            assert np.array_equal(x.S1, y.S1) and x.S2 == y.S2, shape
            assert np.array_equal(x.J, y.J) and np.array_equal(x.N, y.N), shape
        for a, b in zip(states, ref_states):
            assert np.array_equal(a, b), shape


@pytest.mark.parametrize("base", [
    dict(L=8192, p=1.0, q=0.0, init=1, seed=6, stream=1),
    dict(L=1024, p=0.5, q=0.5, init=1, seed=6, stream=2),
    dict(L=4096, init=1, p=0.75, q=0.25, slow_frac=0.5, slow_factor=0.5, seed=6, stream=3),
    dict(L=4096, model=1, init=1, density=0.3, p=1.0, q=1.0, lane_rate=0.1, turn_frac=0.05,
         seed=6, stream=4),
])
def test_whole_ring_launch_split(base, monkeypatch):
    # a whole-ring run cut into launches of at most 37 sub-sweeps (measurement
    # times inside, at and between the cuts) is the same run, word for word
    times = [0, 3, 9, 10, 31, 40]
    ref, ref_states = _records_and_states(dict(base, windows=1), times, 5)
    monkeypatch.setenv("ASEP_MAX_LAUNCH_SUBSWEEPS", "37")
    got, states = _records_and_states(dict(base, windows=1), times, 5)
    for x, y in zip(got, ref):
        assert np.array_equal(x.S1, y.S1) and x.S2 == y.S2
        assert np.array_equal(x.J, y.J) and np.array_equal(x.N, y.N)
    for a, b in zip(states, ref_states):
        assert np.array_equal(a, b)
