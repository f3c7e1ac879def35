"""Pins of the oracle's two-sub-lattice update (Sec. 2.1, Fig. parasep).

The paper's own parallel schedule: every pair (x, x+1) with x even is tried
once, then every pair with x odd, the ring's closing pair (L-1, 0) last.  The
pins below fix it against facts the oracle's code does not produce itself:
the paper's p = 1 degeneracy, the exact master-equation law of tiny rings
(state histograms by chi-square, mean current by a z-test), and special cases
that reduce the disordered ring to a plain one bit for bit.
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import master_equation as me


def _chi2_pvalue(counts, probs, n):
    """Chi-square p-value of a state histogram against an exact law; a state
    the law forbids fails outright."""
    from scipy.stats import chi2

    keys = [k for k in range(len(probs)) if probs[k] > 1e-12]
    stat = sum((counts.get(k, 0) - n * probs[k]) ** 2 / (n * probs[k]) for k in keys)
    assert sum(v for k, v in counts.items() if probs[k] <= 1e-12) == 0
    return chi2.sf(stat, len(keys) - 1)


def _sca(orc, **kw):
    return orc.Params(schedule=orc.SCHED_SUBLATTICE, **kw)


def test_sublattice_threshold_bits(orc):
    # thresholds at 24 bits, then the fewest bits that keep them exact
    s = orc.lower(_sca(orc, L=256, p=0.8, q=0.0))
    assert s["S"] == 2 and s["B"] == 24
    assert s["TB"][0] == int(0.8 * 2 ** 24) == 0xCCCCCC
    assert s["b"] == 22 and s["T"][0] == 0xCCCCCC >> 2
    s = orc.lower(_sca(orc, L=256, p=0.5, q=0.25))
    assert s["b"] == 2 and s["T"][:2] == [2, 1]
    s = orc.lower(_sca(orc, L=256, p=1.0, q=0.0))
    assert s["b"] == 0 and s["T"][:2] == [1, 0]


def test_sublattice_rejects_other_shapes(orc):
    with pytest.raises(ValueError):
        orc.lower(_sca(orc, L=255))
    with pytest.raises(ValueError):
        orc.lower(_sca(orc, L=256, model=orc.TWO_LANE, turn_frac=0.05))


@pytest.mark.parametrize("L", [8, 256, 4096])
def test_sublattice_degenerate_at_p1(orc, L):
    # Sec. 2.1 / the choice p < 1: at p = 1 a flat start returns to 1010...
    # after every MCS (each particle hops once per phase), so W^2 stays 1/4.
    P = _sca(orc, L=L, p=1.0, q=0.0)
    times = [0, 1, 2, 3, 10, 57]
    r = orc.run(P, 3, times)
    assert np.all(r.w2(L) == 0.25)
    assert list(r.J) == [L * t for t in times]
    assert np.array_equal(r.state, orc.init_state(P, 3))


def test_sublattice_grows_below_p1(orc):
    L = 4096
    P = _sca(orc, L=L, p=0.8, q=0.0)
    w = np.mean([orc.run(P, s, [0, 10, 100]).w2(L) for s in range(4)], axis=0)
    assert w[0] == 0.25 and w[1] > 0.5 and w[2] > 1.5 * w[1]


def _exact(ring, v0, t):
    v = v0
    for _ in range(t):
        v = ring.sca_mcs(v)
    return v


def _bernoulli_law(L, T_init):
    rho = T_init / 2 ** 32
    bits = me.bits_table(L).astype(np.float64)
    return np.prod(np.where(bits == 1, rho, 1 - rho), axis=1)


def _histogram(orc, P, t, n):
    counts = {}
    for s in range(n):
        st = orc.init_state(P, s)
        orc.advance(P, s, st, 0, t)
        k = me.state_index(st)
        counts[k] = counts.get(k, 0) + 1
    return counts


@pytest.mark.parametrize(
    "p,q,init", [(0.8, 0.0, 0), (0.8, 0.3, 0), (0.6, 0.45, 1), (0.75, 0.25, 1)]
)
def test_sublattice_law_exact_small_ring(orc, p, q, init):
    L, t, n = 8, 3, 6000
    P = _sca(orc, L=L, p=p, q=q, init=init, density=0.375, seed=5)
    s = orc.lower(P)
    den = 2 ** s["b"]
    ring = me.Ring(L, s["T"][0] / den, s["T"][1] / den)
    if init == orc.INIT_FLAT:
        v0 = np.zeros(1 << L)
        v0[me.state_index(orc.init_state(P, 0))] = 1.0
    else:
        v0 = _bernoulli_law(L, s["T_init"])
    v = _exact(ring, v0, t)
    assert _chi2_pvalue(_histogram(orc, P, t, n), v, n) > 1e-4


def test_sublattice_law_exact_disordered_ring(orc):
    # forward from x uses the slow mask at x, backward from x+1 the q mask at x+1
    L, t, n = 8, 3, 6000
    P = _sca(orc, L=L, p=0.9, q=0.6, slow_frac=0.5, slow_factor=0.25, seed=11)
    s = orc.lower(P)
    sp, sq, _ = orc.init_masks(P, 0)
    assert sp.any() and (1 - sp).any() and sq.any() and (1 - sq).any()
    assert not np.array_equal(sp, sq)
    den = 2 ** s["b"]
    pe = np.where(sp == 1, s["T"][2] / den, s["T"][0] / den)
    qe = np.where(sq == 1, s["T"][3] / den, s["T"][1] / den)
    v0 = np.zeros(1 << L)
    v0[me.state_index(orc.init_state(P, 0))] = 1.0
    v = _exact(me.Ring(L, pe, qe), v0, t)
    P.samples_per_disorder = n  # every sample shares realisation 0
    assert _chi2_pvalue(_histogram(orc, P, t, n), v, n) > 1e-4


def test_sublattice_current_exact(orc):
    L, t, n = 12, 4, 4000
    P = _sca(orc, L=L, p=0.8, q=0.2, init=orc.INIT_BERNOULLI, density=0.5, seed=2)
    s = orc.lower(P)
    den = 2 ** s["b"]
    ring = me.Ring(L, s["T"][0] / den, s["T"][1] / den)
    v = _bernoulli_law(L, s["T_init"])
    mean = 0.0
    for _ in range(t):
        mean += ring.sca_phase_current(v, 0)
        v = ring.sca_phase(v, 0)
        mean += ring.sca_phase_current(v, 1)
        v = ring.sca_phase(v, 1)
    js = np.array([orc.run(P, k, [t]).J[-1] for k in range(n)], dtype=np.float64)
    z = (js.mean() - mean) / (js.std(ddof=1) / np.sqrt(n))
    assert abs(z) < 4.5, (js.mean(), mean)


def test_sublattice_disorder_special_cases(orc):
    base = dict(L=2048, p=0.75, q=0.25)
    plain = orc.run(_sca(orc, **base), 5, [0, 40])
    c0 = orc.run(_sca(orc, **base, slow_frac=0.0, slow_factor=0.5), 5, [0, 40])
    assert np.array_equal(plain.state, c0.state) and plain.J[-1] == c0.J[-1]
    c1 = orc.run(_sca(orc, **base, slow_frac=1.0, slow_factor=0.5), 5, [0, 40])
    scaled = orc.run(_sca(orc, **dict(base, p=0.375, q=0.125)), 5, [0, 40])
    assert np.array_equal(scaled.state, c1.state) and scaled.J[-1] == c1.J[-1]


def test_sublattice_conservation_and_chunks(orc):
    P = _sca(orc, L=1024, p=0.8, q=0.1, init=orc.INIT_BERNOULLI, density=0.4)
    full = orc.run(P, 7, [0, 9, 25])
    assert len(set(full.N.tolist())) == 1
    st = orc.init_state(P, 7)
    J = orc.advance(P, 7, st, 0, 4)
    J = orc.advance(P, 7, st, 4, 5, J)
    J = orc.advance(P, 7, st, 9, 16, J)
    assert J == full.J[-1] and np.array_equal(st, full.state)


# --------------------------------------------------------------------------- two lanes
def _sca2(orc, **kw):
    base = dict(model=orc.TWO_LANE, init=orc.INIT_BERNOULLI, density=0.5, p=0.5, q=0.5,
                lane_rate=0.8, slow_frac=0.5, slow_factor=0.25)
    base.update(kw)
    return orc.Params(schedule=orc.SCHED_SUBLATTICE, **base)


def test_two_lane_sublattice_lowering(orc):
    # Sec. 3: in-lane 0.5, crossing 0.8 reduced to 0.2 at marked sites
    s = orc.lower(_sca2(orc, L=256))
    assert s["S"] == 4 and s["b"] == 24
    assert s["T"] == [1 << 23, 1 << 23, 0xCCCCCC, int(0.2 * 2 ** 24)]
    with pytest.raises(ValueError):
        orc.lower(_sca2(orc, L=256, turn_frac=0.1))


def test_two_lane_sublattice_invariants(orc):
    P = _sca2(orc, L=1024)
    r = orc.run(P, 3, [0, 5, 20])
    assert len(set(r.N.tolist())) == 1
    # no lane changes: each lane keeps its particle number, and p = q = 1 on
    # lanes started flat is the one-lane degeneracy in both directions
    P0 = _sca2(orc, L=1024, lane_rate=0.0, p=1.0, q=1.0, init=orc.INIT_FLAT)
    st0 = orc.init_state(P0, 3)
    r0 = orc.run(P0, 3, [0, 1, 7])
    assert r0.state[:1024].sum() == st0[:1024].sum() and r0.state[1024:].sum() == st0[1024:].sum()
    # from 1010... in both lanes: A hops at every pair of both phases (+L per
    # MCS); B, hopping left, misses the even phase of the first MCS and then
    # follows A's pattern mirrored (-L/2, then -L per MCS)
    assert list(r0.J) == [0, 512, 512]
    # the marks: two independent planes of density 1/2 keyed by realisation
    sp, sq, tu = orc.init_masks(_sca2(orc, L=1 << 14), 0)
    assert tu is None and abs(sp.mean() - 0.5) < 0.02 and abs(sq.mean() - 0.5) < 0.02
    assert abs((sp & sq).mean() - 0.25) < 0.02


def test_two_lane_sublattice_law_exact(orc):
    L, t, n = 4, 2, 6000
    P = _sca2(orc, L=L, p=0.75, q=0.5, lane_rate=0.8, slow_factor=0.25, seed=9)
    s = orc.lower(P)
    um, vm, _ = orc.init_masks(P, 0)
    assert um.any() or vm.any()
    den = 2 ** s["b"]
    u = np.where(um == 1, s["T"][3] / den, s["T"][2] / den)
    w = np.where(vm == 1, s["T"][3] / den, s["T"][2] / den)
    tl = me.TwoLane(L, s["T"][0] / den, s["T"][1] / den, 0.0, np.zeros(L))
    rho = s["T_init"] / 2 ** 32
    bits = me.bits_table(L, 2).astype(np.float64)
    v = np.prod(np.where(bits == 1, rho, 1 - rho), axis=1)
    for _ in range(t):
        v = tl.sca_mcs(v, u, w)
    P.samples_per_disorder = n
    assert _chi2_pvalue(_histogram(orc, P, t, n), v, n) > 1e-4


def test_two_lane_sublattice_current_exact(orc):
    L, t, n = 4, 3, 6000
    P = _sca2(orc, L=L, p=0.75, q=0.25, lane_rate=0.5, slow_frac=0.0, seed=4)
    s = orc.lower(P)
    den = 2 ** s["b"]
    tl = me.TwoLane(L, s["T"][0] / den, s["T"][1] / den, 0.0, np.zeros(L))
    u = np.full(L, s["T"][2] / den)
    rho = s["T_init"] / 2 ** 32
    bits = me.bits_table(L, 2).astype(np.float64)
    v = np.prod(np.where(bits == 1, rho, 1 - rho), axis=1)
    mean = 0.0
    for _ in range(t):
        mean += tl.sca_inlane_current(v, 0)
        v = tl.lane_change(tl.sca_inlane(v, 0), True, u)
        mean += tl.sca_inlane_current(v, 1)
        v = tl.lane_change(tl.sca_inlane(v, 1), False, u)
    js = np.array([orc.run(P, k, [t]).J[-1] for k in range(n)], dtype=np.float64)
    z = (js.mean() - mean) / (js.std(ddof=1) / np.sqrt(n))
    assert abs(z) < 4.5, (js.mean(), mean)
