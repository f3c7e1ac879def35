"""Pins of the CPU oracle against facts fixed outside it.

Each check ties a part of the oracle to something it does not compute itself:
published Philox known answers and an independent library implementation,
exact threshold values, the paper's printed numbers (intrinsic width, number of
sampling events), closed forms, Python brute force on tiny inputs, exact laws
from the master equation of tiny rings, and the growth exponents.
"""
import json
import os
import shutil
import subprocess
import tempfile
from math import comb

import numpy as np
import pytest

from oracle import master_equation as me

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# --------------------------------------------------------------------------- Philox
def test_philox_known_answers(orc):
    for v in _gold("philox4x32_10_kat.json")["vectors"]:
        ctr = [int(x, 16) for x in v["ctr"]]
        key = [int(x, 16) for x in v["key"]]
        out = [int(x, 16) for x in v["out"]]
        assert list(orc.philox(ctr, key)) == out


@pytest.fixture(scope="module")
def rocrand_probe():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND probe")
    d = tempfile.mkdtemp()
    exe = os.path.join(d, "rkat")
    src = os.path.join(os.path.dirname(__file__), "helpers", "rocrand_philox_kat.cpp")
    subprocess.check_call([hipcc, "-O1", "-std=c++17", src, "-o", exe],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    yield exe
    shutil.rmtree(d, ignore_errors=True)


def test_philox_matches_rocrand(orc, rocrand_probe):
    rng = np.random.default_rng(12345)
    rows = rng.integers(0, 2**32, size=(300, 6), dtype=np.uint64)
    rows[:8, :] = 0
    rows[8:16, 4:] = 0xFFFFFFFF
    text = "\n".join(" ".join(str(int(v)) for v in r) for r in rows) + "\n"
    res = subprocess.run([rocrand_probe], input=text.encode(), capture_output=True, check=True)
    got = [list(map(int, line.split())) for line in res.stdout.decode().strip().splitlines()]
    assert len(got) == len(rows)
    for r, g in zip(rows, got):
        assert list(orc.philox(r[:4], r[4:])) == g


# --------------------------------------------------------------------------- thresholds
def test_threshold_exact_values(orc):
    assert orc.threshold(0.5, 26) == 2**25
    assert orc.threshold(1.0, 26) == 2**26
    assert orc.threshold(0.0, 26) == 0
    assert orc.threshold(0.1, 32) == (2**32) // 10  # floor(0.1 * 2^32) = 429496729
    assert orc.threshold(0.8, 26) == int(np.floor(0.8 * 2**26))
    assert orc.threshold(1.0, 32) == 2**32


@pytest.mark.parametrize("p,q,b,A", [(1.0, 0.0, 0, 5), (0.5, 0.5, 1, 4), (0.75, 0.25, 2, 4),
                                     (0.8, 0.0, 26, 1)])
def test_draw_packing(orc, p, q, b, A):
    s = orc.lower(orc.Params(L=4096, p=p, q=q))
    assert s["B"] == 26 and s["b"] == b and s["A"] == A
    assert s["w"] == 6 + b
    # the acceptance probability realised at b bits equals the one at B bits
    for tb, t in zip(s["TB"][:2], s["T"][:2]):
        assert t * 2 ** (s["B"] - b) == tb


@pytest.mark.parametrize("kw,jlow,A", [
    (dict(cell_log2=5, subsweeps=2, p=1.0, q=0.0), 1, 4),                 # b = 0
    (dict(cell_log2=5, subsweeps=2, p=0.5, q=0.5), 1, 4),                 # b = 1
    (dict(cell_log2=5, subsweeps=2, p=0.875, q=0.25), 1, 4),              # b = 3: 8 bits
    (dict(cell_log2=5, subsweeps=2, p=0.9375, q=0.0), 0, 3),              # b = 4: 9 bits
    (dict(cell_log2=4, subsweeps=1, p=1.0, q=0.0), 0, 8),                 # 16-site cells
    (dict(cell_log2=6, subsweeps=4, p=1.0, q=0.0), 0, 5),                 # 64-site cells
    (dict(cell_log2=5, subsweeps=2, model=1, p=1.0, q=1.0, lane_rate=0.5), 1, 4),  # 7 bits
    (dict(cell_log2=5, subsweeps=2, model=1, p=0.75, q=1.0, lane_rate=0.5), 0, 3),  # 9 bits
])
def test_byte_fields_for_32_site_cells(orc, kw, jlow, A):
    # cells of 32 sites whose field fits in 8 bits take the four bytes of a
    # word as fields (the position in the low bits); every other schedule
    # packs fields of lam + ebits + b bits
    s = orc.lower(orc.Params(L=4096, **kw))
    assert s["jlow"] == jlow and s["A"] == A
    ebits = 2 if kw.get("model", 0) == 1 else 0
    assert s["w"] == (8 if jlow else kw["cell_log2"] + ebits + s["b"])
    assert s["per_block"] == 4 * A


# --------------------------------------------------------------------------- init, heights
@pytest.mark.parametrize("L", [128, 4096, 2**17])
def test_flat_start_intrinsic_width(orc, L):
    facts = _gold("paper_facts.json")
    P = orc.Params(L=L)
    st = orc.init_state(P, 0)
    words = orc.pack_words(st)
    assert np.all(words == np.uint64(0x5555555555555555))
    S1, S2, N = orc.sums(st, L)
    assert (S1, S2, N) == (-L // 2, L // 2, L // 2)
    assert orc.w2(L, S1, S2) == facts["intrinsic_width"]["value"]


def _brute_sums(bits):
    h, s1, s2 = 0, 0, 0
    for b in bits:
        s1 += h
        s2 += h * h
        h += 1 - 2 * int(b)
    return s1, s2


def test_sums_brute_force(orc):
    rng = np.random.default_rng(7)
    for L in (64, 128, 640, 4096):
        for dens in (0.1, 0.5, 0.9):
            st = (rng.random(L) < dens).astype(np.uint8)
            S1, S2, N = orc.sums(st, L)
            assert (S1, S2) == _brute_sums(st)
            assert N == int(st.sum())


def test_sums_step_closed_form(orc):
    # 1^N 0^(L-N): h_x = -x for x <= N, then h_x = x - 2N
    for L, N in ((64, 32), (1024, 100), (1 << 20, 1 << 19)):
        st = np.zeros(L, np.uint8)
        st[:N] = 1
        S1, S2, _ = orc.sums(st, L)
        e1 = -N * (N + 1) // 2 + sum_range(N + 1, L - 1, lambda x: x - 2 * N)
        e2 = sum_sq(N) + sum_range_sq(N + 1, L - 1, -2 * N)
        assert S1 == e1 and S2 == e2


def sum_range(a, b, f):
    # sum of f over a..b for linear f(x) = x + c
    n = b - a + 1
    c = f(0)
    return (a + b) * n // 2 + c * n


def sum_sq(n):
    return n * (n + 1) * (2 * n + 1) // 6


def sum_range_sq(a, b, c):
    # sum_{x=a}^{b} (x + c)^2 = sum_{y=a+c}^{b+c} y^2
    lo, hi = a + c, b + c
    def S(m):
        if m >= 0:
            return sum_sq(m)
        return sum_sq(-m)
    if lo >= 0:
        return S(hi) - S(lo - 1)
    if hi <= 0:
        return S(lo) - S(hi + 1)
    return S(lo) + S(hi)


def test_w2_big_ring_exact(orc):
    # L = 2^26 half filled with a single step: S2 needs more than 64 bits
    L, N = 1 << 26, 1 << 25
    S1 = -N * (N + 1) // 2 + sum_range(N + 1, L - 1, lambda x: x - 2 * N)
    S2 = sum_sq(N) + sum_range_sq(N + 1, L - 1, -2 * N)
    assert S2 >= 1 << 64
    w = orc.w2(L, S1, S2)
    exact = (L * S2 - S1 * S1) / (L * L)
    assert abs(w - exact) <= 1e-12 * exact


# --------------------------------------------------------------------------- sampling
def test_sampling_events_match_paper(orc):
    f = _gold("paper_facts.json")["sampling"]
    t = orc.sample_times(f["t0"], f["factor"], f["t_max"])
    assert t[0] == 0 and t[1] == 30
    assert len(t) - 2 == f["events"]  # t=0 aside, 261 sampling times = 260 gaps
    assert all(b > a for a, b in zip(t, t[1:]))
    assert len(orc.sample_times(30, 1.05, 10**5)) == 1 + 167
    assert len(orc.sample_times(30, 1.05, 10**6)) == 1 + 214


# --------------------------------------------------------------------------- invariants
@pytest.mark.parametrize("S", [1, 4, 16])
def test_conservation_and_chunks(orc, S):
    P = orc.Params(L=1024, p=0.8, q=0.1, subsweeps=S, init=orc.INIT_BERNOULLI, density=0.3)
    full = orc.run(P, 3, [0, 7, 20])
    assert len(set(full.N.tolist())) == 1
    st = orc.init_state(P, 3)
    J = orc.advance(P, 3, st, 0, 5)
    J = orc.advance(P, 3, st, 5, 2, J)
    J = orc.advance(P, 3, st, 7, 13, J)
    assert J == full.J[-1]
    assert np.array_equal(st, full.state)


def test_zero_rates_freeze(orc):
    P = orc.Params(L=512, p=0.0, q=0.0, init=orc.INIT_BERNOULLI, density=0.5)
    r = orc.run(P, 0, [0, 50])
    assert r.J[-1] == 0
    assert np.array_equal(r.state, orc.init_state(P, 0))


def test_disorder_special_cases(orc):
    base = dict(L=2048, p=0.75, q=0.25, subsweeps=4, rbits=26)
    plain = orc.run(orc.Params(**base), 5, [0, 40])
    c0 = orc.run(orc.Params(**base, slow_frac=0.0, slow_factor=0.5), 5, [0, 40])
    assert np.array_equal(plain.state, c0.state) and plain.J[-1] == c0.J[-1]
    c1 = orc.run(orc.Params(**base, slow_frac=1.0, slow_factor=0.5), 5, [0, 40])
    scaled = orc.run(orc.Params(**dict(base, p=0.375, q=0.125)), 5, [0, 40])
    assert np.array_equal(scaled.state, c1.state) and scaled.J[-1] == c1.J[-1]
    # masks: fraction near c, and keyed by realization only
    P = orc.Params(L=1 << 16, slow_frac=0.1, slow_factor=0.5, samples_per_disorder=4)
    sp, sq, _ = orc.init_masks(P, 0)
    assert sq is None and abs(sp.mean() - 0.1) < 0.005


@pytest.mark.parametrize("sched", [(6, 4), (5, 2)], ids=["64-site", "32-site"])
def test_two_lane_conservation_and_decoupling(orc, sched):
    P = orc.Params(L=1024, model=orc.TWO_LANE, init=orc.INIT_BERNOULLI, density=0.3, p=1.0,
                   q=1.0, lane_rate=0.1, turn_frac=0.05, cell_log2=sched[0], subsweeps=sched[1])
    r = orc.run(P, 2, [0, 10, 30])
    assert len(set(r.N.tolist())) == 1
    # no lane changes: each lane keeps its particle number
    P0 = orc.Params(**{**P.__dict__, "lane_rate": 0.0})
    st0 = orc.init_state(P0, 2)
    r0 = orc.run(P0, 2, [0, 30])
    assert r0.state[:1024].sum() == st0[:1024].sum()
    assert r0.state[1024:].sum() == st0[1024:].sum()


# --------------------------------------------------------------------------- exact laws
def _histogram(orc, P, t, n_samples):
    counts = {}
    for s in range(n_samples):
        st = orc.init_state(P, s)
        orc.advance(P, s, st, 0, t)
        k = me.state_index(st)
        counts[k] = counts.get(k, 0) + 1
    return counts


def _chi2_pvalue(counts, probs, n):
    from scipy.stats import chi2

    keys = [k for k in range(len(probs)) if probs[k] > 1e-12]
    stat = 0.0
    for k in keys:
        e = n * probs[k]
        stat += (counts.get(k, 0) - e) ** 2 / e
    extra = sum(v for k, v in counts.items() if probs[k] <= 1e-12)
    assert extra == 0, "oracle reached a state the exact law forbids"
    return chi2.sf(stat, len(keys) - 1)


@pytest.mark.parametrize("ell,S,p,q", [(4, 1, 0.7, 0.2), (4, 2, 1.0, 0.0), (2, 1, 0.6, 0.3)])
def test_schedule_law_exact_small_ring(orc, ell, S, p, q):
    L, t, n = 8, 3, 6000
    P = orc.Params(L=L, p=p, q=q, cell_log2=ell.bit_length() - 1, subsweeps=S)
    s = orc.lower(P)
    pe = s["T"][0] / 2 ** s["b"]
    qe = s["T"][1] / 2 ** s["b"]
    ring = me.Ring(L, pe, qe)
    v = np.zeros(1 << L)
    v[me.state_index(orc.init_state(P, 0))] = 1.0
    for _ in range(t):
        v = ring.dd_mcs(v, ell, S)
    pval = _chi2_pvalue(_histogram(orc, P, t, n), v, n)
    assert pval > 1e-4


def test_schedule_law_exact_disordered_ring(orc):
    # site-dependent rates: forward from x uses the slow mask at x, backward
    # from x+1 uses the q mask at x+1 (rates of the departure site)
    L, ell, S, t, n = 8, 4, 2, 3, 6000
    P = orc.Params(L=L, p=0.9, q=0.6, slow_frac=0.5, slow_factor=0.25, cell_log2=2,
                   subsweeps=S, seed=11)
    s = orc.lower(P)
    sp, sq, _ = orc.init_masks(P, 0)
    assert sp.any() and (1 - sp).any() and sq.any() and (1 - sq).any()
    den = 2 ** s["b"]
    pe = np.where(sp == 1, s["T"][2] / den, s["T"][0] / den)
    qe = np.where(sq == 1, s["T"][3] / den, s["T"][1] / den)
    ring = me.Ring(L, pe, qe)
    v = np.zeros(1 << L)
    v[me.state_index(orc.init_state(P, 0))] = 1.0
    for _ in range(t):
        v = ring.dd_mcs(v, ell, S)
    # every sample shares realization 0 of the masks
    P.samples_per_disorder = n
    assert _chi2_pvalue(_histogram(orc, P, t, n), v, n) > 1e-4


def test_rsu_law_and_current(orc):
    L, p, q = 8, 0.9, 0.3
    ring = me.Ring(L, p, q)
    v0 = np.zeros(1 << L)
    v0[me.state_index([1, 0] * 4)] = 1.0
    pi = me.stationary(ring.rsu_attempt, v0)
    # uniform over the 70 configurations with N = 4
    nz = pi[pi > 1e-12]
    assert len(nz) == comb(8, 4) and np.allclose(nz, 1 / comb(8, 4), atol=1e-12)
    cur = sum(float(pi @ ring.bond_current(x)) for x in range(L))  # per attempt x L bonds
    N = 4
    assert abs(cur - (p - q) * N * (L - N) / (L - 1)) < 1e-12
    # the oracle's random-sequential simulator reproduces that current
    P = orc.Params(L=L, p=p, q=q)
    js = []
    for smp in range(400):
        st = np.array([1, 0] * 4, np.uint8)
        J0 = orc.rsu(P, smp, st, 0, 20)
        js.append(orc.rsu(P, smp, st, 20, 200, 0) / 200.0)
    js = np.array(js)
    exact = (p - q) * N * (L - N) / (L - 1)
    assert abs(js.mean() - exact) < 5 * js.std() / np.sqrt(len(js))


def test_symmetric_schedule_is_uniform_and_current(orc):
    # at p = q the schedule keeps the uniform law (symmetric bond maps are
    # doubly stochastic); at p != q the exact stationary current of the
    # schedule is reproduced by the oracle
    L, ell, S = 8, 4, 1
    v0 = np.zeros(1 << L)
    v0[me.state_index([1, 0] * 4)] = 1.0
    sym = me.Ring(L, 0.5, 0.5)
    pi = me.stationary(lambda v: sym.subsweep(v, ell, ell // S), v0)
    nz = pi[pi > 1e-12]
    assert len(nz) == comb(8, 4) and np.allclose(nz, 1 / comb(8, 4), atol=1e-10)

    p, q = 1.0, 0.0
    asym = me.Ring(L, p, q)
    pi = me.stationary(lambda v: asym.subsweep(v, ell, ell // S), v0)
    j_exact = asym.dd_subsweep_current(pi, ell, ell // S) * S  # per MCS
    P = orc.Params(L=L, p=p, q=q, cell_log2=2, subsweeps=S)
    js = []
    for smp in range(400):
        st = np.array([1, 0] * 4, np.uint8)
        orc.advance(P, smp, st, 0, 20)
        js.append(orc.advance(P, smp, st, 20, 200, 0) / 200.0)
    js = np.array(js)
    assert abs(js.mean() - j_exact) < 5 * js.std() / np.sqrt(len(js))


def test_two_lane_law_exact(orc):
    L, ell, S, t, n = 4, 2, 2, 2, 6000
    # every sample shares turning-point realization 0; starts are random
    P = orc.Params(L=L, model=orc.TWO_LANE, init=orc.INIT_BERNOULLI, density=0.5, p=0.5,
                   q=0.25, lane_rate=0.25, turn_frac=0.5, cell_log2=1, subsweeps=S,
                   samples_per_disorder=n)
    s = orc.lower(P)
    pa, pb = (s["T"][i] / 2 ** s["b"] for i in range(2))
    om = s["T"][2] / 2 ** s["bc"]
    _, _, turn = orc.init_masks(P, 0)
    tl = me.TwoLane(L, pa, pb, om, turn)
    counts = {}
    probs = np.zeros(1 << (2 * L))
    for smp in range(n):
        st = orc.init_state(P, smp)
        orc.advance(P, smp, st, 0, t)
        k = me.state_index(st)
        counts[k] = counts.get(k, 0) + 1
    # exact law: average over the sample-dependent random starts
    starts = {}
    for smp in range(n):
        k = me.state_index(orc.init_state(P, smp))
        starts[k] = starts.get(k, 0) + 1
    for k0, c in starts.items():
        v = np.zeros(1 << (2 * L))
        v[k0] = 1.0
        for _ in range(t):
            v = tl.dd_mcs(v, ell, S)
        probs += v * c / n
    assert _chi2_pvalue(counts, probs, n) > 1e-4


@pytest.mark.parametrize("lane", [0, 1])
def test_two_lane_lone_particle_current(orc, lane):
    # one particle, no lane changes: it only moves in its lane's direction,
    # and its mean displacement after t MCS equals the exact expectation
    L, ell, S, t, n = 8, 4, 2, 3, 3000
    P = orc.Params(L=L, model=orc.TWO_LANE, p=0.75, q=0.5, lane_rate=0.0, turn_frac=0.0,
                   cell_log2=2, subsweeps=S)
    s = orc.lower(P)
    tl = me.TwoLane(L, s["T"][0] / 2 ** s["b"], s["T"][1] / 2 ** s["b"], 0.0, np.zeros(L))
    start = np.zeros(2 * L, np.uint8)
    start[lane * L + 3] = 1
    v = np.zeros(1 << (2 * L))
    v[me.state_index(start)] = 1.0
    exact = 0.0
    for _ in range(t * S):
        exact += tl.dd_subsweep_current(v, ell, 4 * ell // S)
        v = tl.subsweep(v, ell, 4 * ell // S)
    js, counts = [], {}
    for smp in range(n):
        st = start.copy()
        J = orc.advance(P, smp, st, 0, t)
        assert st.sum() == 1 and st[lane * L:(lane + 1) * L].sum() == 1
        assert (J >= 0) if lane == 0 else (J <= 0)
        js.append(J)
        k = me.state_index(st)
        counts[k] = counts.get(k, 0) + 1
    js = np.array(js, dtype=float)
    assert abs(js.mean() - exact) < 5 * js.std() / np.sqrt(n)
    assert _chi2_pvalue(counts, v, n) > 1e-4


# --------------------------------------------------------------------------- physics
def test_ew_saturation_width(orc):
    # uniform law at half filling: E[W^2] = (L + 1) / 12 exactly
    L = 64
    P = orc.Params(L=L, p=0.5, q=0.5, cell_log2=4, subsweeps=4)
    ts = list(range(6000, 20001, 500))
    vals = []
    for smp in range(12):
        r = orc.run(P, smp, ts)
        vals.append(r.w2(L).mean())
    vals = np.array(vals)
    assert abs(vals.mean() - (L + 1) / 12) < 5 * vals.std() / np.sqrt(len(vals)) + 0.05


def _growth_slope(orc, p, q, L=8192, t_hi=3000, n=16, cell_log2=6, subsweeps=4):
    from concurrent.futures import ThreadPoolExecutor

    times = orc.sample_times(30, 1.05, t_hi)
    P = orc.Params(L=L, p=p, q=q, cell_log2=cell_log2, subsweeps=subsweeps)
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        W = list(ex.map(lambda smp: orc.run(P, smp, times).w2(L), range(n)))
    W = np.mean(W, axis=0) - 0.25  # subtract the intrinsic width (Sec. 2.2)
    t = np.array(times[1:], dtype=float)
    sel = t >= 100
    return np.polyfit(np.log(t[sel]), np.log(W[1:][sel]), 1)[0]


# cells of 64 sites with four sub-sweeps per MCS, and of 32 sites with two
SCHEDULES = [(6, 4), (5, 2)]


@pytest.mark.parametrize("cell_log2,subsweeps", SCHEDULES)
def test_growth_exponent_kpz(orc, cell_log2, subsweeps):
    f = _gold("paper_facts.json")["kpz_exponents"]
    two_beta = 2 * f["alpha"] / f["z"]
    slope = _growth_slope(orc, 1.0, 0.0, cell_log2=cell_log2, subsweeps=subsweeps)
    assert abs(slope - two_beta) < 0.05


@pytest.mark.parametrize("cell_log2,subsweeps", SCHEDULES)
def test_growth_exponent_ew(orc, cell_log2, subsweeps):
    # 1+1 dimensional Edwards-Wilkinson: beta = 1/4
    slope = _growth_slope(orc, 0.5, 0.5, cell_log2=cell_log2, subsweeps=subsweeps)
    assert abs(slope - 0.5) < 0.05


@pytest.mark.parametrize("cell_log2,subsweeps", SCHEDULES)
def test_schedule_matches_random_sequential(orc, cell_log2, subsweeps):
    # W^2(t) of the shifted decomposition and of random-sequential updates agree
    # within error bars once time is rescaled by the bond-attempt rate 1 - 1/ell
    L, n = 1024, 48
    ell = 1 << cell_log2
    P = orc.Params(L=L, p=1.0, q=0.0, cell_log2=cell_log2, subsweeps=subsweeps)
    ts = [64, 128, 256, 512]
    dd, rs = [], []
    for smp in range(n):
        dd.append(orc.run(P, smp, [0] + ts).w2(L)[1:])
        st = orc.init_state(P, smp)
        prev, w = 0, []
        for t in ts:
            tr = t * (ell - 1) // ell
            orc.rsu(P, smp, st, prev, tr - prev)
            prev = tr
            S1, S2, _ = orc.sums(st, L)
            w.append(orc.w2(L, S1, S2))
        rs.append(w)
    dd, rs = np.array(dd), np.array(rs)
    z = (dd.mean(0) - rs.mean(0)) / np.sqrt(dd.var(0) / n + rs.var(0) / n)
    assert np.all(np.abs(z) < 4)


# --------------------------------------------------------------------------- hop count
def _hop_cases(orc):
    two = dict(model=orc.TWO_LANE, lane_rate=0.3, turn_frac=0.2)
    return [
        ("plain", orc.Params(L=512, p=0.8, q=0.3)),
        ("plain-ell4", orc.Params(L=256, p=0.6, q=0.4, cell_log2=2, subsweeps=1)),
        ("disorder", orc.Params(L=1024, p=0.75, q=0.25, slow_frac=0.3, slow_factor=0.5, rbits=26)),
        ("two-lane", orc.Params(L=512, p=0.9, q=0.7, **two)),
        ("sublattice", orc.Params(L=512, p=0.7, q=0.2, schedule=orc.SCHED_SUBLATTICE)),
        ("two-lane sublattice", orc.Params(L=512, model=orc.TWO_LANE, p=0.5, q=0.5,
                                           lane_rate=0.8, slow_frac=0.5, slow_factor=0.25,
                                           schedule=orc.SCHED_SUBLATTICE)),
    ]


@pytest.mark.parametrize("case", range(6))
def test_hops_equal_position_sum_change(orc, case):
    """The hop count J (+1 per hop to the right, -1 per hop to the left; on two
    lanes lane A hops right and lane B left, lane changes count nothing) moves
    the particles' position sum P = sum_y y n_y by J modulo L: a hop within the
    ring changes P by +-1, one across the closing bond by -+(L-1), and a lane
    change keeps it.  The identity ties J to the state alone, so a hop counted
    with the wrong sign, twice, or not at all shows up."""
    name, P = _hop_cases(orc)[case]
    P.init = orc.INIT_BERNOULLI
    P.density = 0.4
    L = P.L
    for sample in (0, 3):
        st0 = orc.init_state(P, sample).astype(np.int64)
        r = orc.run(P, sample, [0, 4, 11])
        st1 = r.state.astype(np.int64)
        pos = np.tile(np.arange(L, dtype=np.int64), len(st0) // L)
        dP = int((pos * (st1 - st0)).sum())
        J = int(r.J[-1])
        assert J != 0, name
        assert (J - dP) % L == 0, (name, sample, J, dP)
