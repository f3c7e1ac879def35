"""TEST INFRASTRUCTURE ONLY: exact laws of tiny ASEP rings (L <= 12).

Distributions are vectors over all 2^L (single lane) or 2^(2L) (two lanes)
configurations, index = sum_x s_x 2^x (lane B bits above lane A's).  Every
operator is applied to vectors, never formed as a matrix, so nothing here
shares arithmetic with the simulators it checks.

* random-sequential update (Sec. 2.1's serial dynamics): one attempt picks a
  bond uniformly; one MCS is L attempts;
* the shifted domain decomposition (the parallel schedule): for a shift sigma
  drawn uniformly from [0, ell), every cell of ell sites receives `a` attempts,
  each on a uniformly chosen offset j in [0, ell) with j = ell-1 a no-op; the
  cells act on disjoint sites, so their order does not matter;
* the paper's two-sub-lattice update (Sec. 2.1, Fig. parasep): every pair
  (x, x+1) with x even tried once, then every pair with x odd (the ring's
  closing pair (L-1, 0) among them);
* observables: W^2 per configuration (Eq. W with h_0 = 0, h_{x+1} = h_x + 1 -
  2 s_x) and the expected hop current.

Acceptance probabilities are passed in exactly as the simulators realise them
(threshold / 2^bits), so the laws are exact for the schedule being tested.
"""
from __future__ import annotations

import numpy as np


def bits_table(L: int, planes: int = 1) -> np.ndarray:
    n = 1 << (L * planes)
    idx = np.arange(n, dtype=np.int64)
    return ((idx[:, None] >> np.arange(L * planes)) & 1).astype(np.int8)


def w2_of_states(L: int) -> np.ndarray:
    """W^2 of every single-lane configuration (Eq. W, population variance)."""
    s = bits_table(L)
    h = np.zeros((s.shape[0], L), dtype=np.float64)
    for x in range(1, L):
        h[:, x] = h[:, x - 1] + 1 - 2 * s[:, x - 1]
    return (h * h).mean(axis=1) - h.mean(axis=1) ** 2


class Ring:
    """Single-lane ring of L sites with site-dependent right/left probabilities.

    p[x] is the probability that a particle at x hops to x+1, q[y] that a
    particle at y hops to y-1 (rates belong to the departure site)."""

    def __init__(self, L: int, p, q):
        self.L = L
        self.n = 1 << L
        self.p = np.broadcast_to(np.asarray(p, dtype=np.float64), (L,)).copy()
        self.q = np.broadcast_to(np.asarray(q, dtype=np.float64), (L,)).copy()
        idx = np.arange(self.n, dtype=np.int64)
        self._fwd = []  # per bond x: (sources with "10" at (x,x+1), targets)
        self._bwd = []
        for x in range(L):
            y = (x + 1) % L
            bx = (idx >> x) & 1
            by = (idx >> y) & 1
            flip = (1 << x) | (1 << y)
            f = idx[(bx == 1) & (by == 0)]
            b = idx[(bx == 0) & (by == 1)]
            self._fwd.append((f, f ^ flip))
            self._bwd.append((b, b ^ flip))

    def bond(self, v: np.ndarray, x: int) -> np.ndarray:
        """Distribution after one attempt on bond (x, x+1)."""
        out = v.copy()
        f, ft = self._fwd[x]
        b, bt = self._bwd[x]
        px = self.p[x]
        qy = self.q[(x + 1) % self.L]
        mf = px * v[f]
        mb = qy * v[b]
        out[f] -= mf
        out[ft] += mf
        out[b] -= mb
        out[bt] += mb
        return out

    def bond_current(self, x: int) -> np.ndarray:
        """Expected hop count (+1 right, -1 left) of one attempt on bond x, per state."""
        c = np.zeros(self.n)
        f, _ = self._fwd[x]
        b, _ = self._bwd[x]
        c[f] += self.p[x]
        c[b] -= self.q[(x + 1) % self.L]
        return c

    # --- random-sequential update --------------------------------------------
    def rsu_attempt(self, v):
        return sum(self.bond(v, x) for x in range(self.L)) / self.L

    def rsu_mcs(self, v):
        for _ in range(self.L):
            v = self.rsu_attempt(v)
        return v

    # --- shifted domain decomposition ----------------------------------------
    def cell_attempt(self, v, base: int, ell: int):
        acc = v.copy()  # j = ell-1: the no-op
        for j in range(ell - 1):
            acc += self.bond(v, (base + j) % self.L)
        return acc / ell

    def subsweep(self, v, ell: int, a: int):
        out = np.zeros_like(v)
        for sigma in range(ell):
            u = v
            for k in range(self.L // ell):
                base = (sigma + k * ell) % self.L
                for _ in range(a):
                    u = self.cell_attempt(u, base, ell)
            out += u
        return out / ell

    def dd_mcs(self, v, ell: int, S: int):
        a = ell // S
        for _ in range(S):
            v = self.subsweep(v, ell, a)
        return v

    def dd_subsweep_current(self, v, ell: int, a: int) -> float:
        """Expected hop count of one sub-sweep started from distribution v."""
        total = 0.0
        for sigma in range(ell):
            for k in range(self.L // ell):
                base = (sigma + k * ell) % self.L
                cur = np.zeros(self.n)
                for j in range(ell - 1):
                    cur += self.bond_current((base + j) % self.L)
                cur /= ell
                u = v
                for _ in range(a):
                    total += float(u @ cur) / ell
                    u = self.cell_attempt(u, base, ell)
        return total

    # --- the paper's two-sub-lattice update ----------------------------------
    def sca_phase(self, v, f: int):
        """Every pair (x, x+1) with x = f mod 2 tried once (disjoint pairs)."""
        for x in range(f, self.L, 2):
            v = self.bond(v, x)
        return v

    def sca_mcs(self, v):
        return self.sca_phase(self.sca_phase(v, 0), 1)

    def sca_phase_current(self, v, f: int) -> float:
        """Expected hop count of one phase started from distribution v; the
        pairs of a phase share no site, so each sees the phase's input law."""
        return float(sum(v @ self.bond_current(x) for x in range(f, self.L, 2)))


class TwoLane:
    """Two rings A (hops right w.p. pa) and B (hops left w.p. pb) with lane
    changes w.p. omega at turning sites (turn[x] = 1); index = A | B << L."""

    def __init__(self, L: int, pa: float, pb: float, omega: float, turn):
        self.L = L
        self.n = 1 << (2 * L)
        self.pa, self.pb, self.omega = pa, pb, omega
        self.turn = np.asarray(turn, dtype=np.int8)
        idx = np.arange(self.n, dtype=np.int64)
        A = lambda x: (idx >> x) & 1
        Bq = lambda x: (idx >> (L + x)) & 1
        self._ahop, self._bhop, self._ab, self._ba = [], [], [], []
        for x in range(L):
            y = (x + 1) % L
            s = idx[(A(x) == 1) & (A(y) == 0)]
            self._ahop.append((s, s ^ ((1 << x) | (1 << y))))
            s = idx[(Bq(y) == 1) & (Bq(x) == 0)]
            self._bhop.append((s, s ^ ((1 << (L + x)) | (1 << (L + y)))))
            s = idx[(A(x) == 1) & (Bq(x) == 0)]
            self._ab.append((s, s ^ ((1 << x) | (1 << (L + x)))))
            s = idx[(Bq(x) == 1) & (A(x) == 0)]
            self._ba.append((s, s ^ ((1 << x) | (1 << (L + x)))))

    def _move(self, v, pair, prob):
        out = v.copy()
        s, t = pair
        m = prob * v[s]
        out[s] -= m
        out[t] += m
        return out

    def event(self, v, x: int, e: int, dead: bool):
        if e == 0:
            return v.copy() if dead else self._move(v, self._ahop[x], self.pa)
        if e == 1:
            return v.copy() if dead else self._move(v, self._bhop[x], self.pb)
        if not self.turn[x]:
            return v.copy()
        return self._move(v, self._ab[x] if e == 2 else self._ba[x], self.omega)

    def event_current(self, x: int, e: int, dead: bool) -> np.ndarray:
        c = np.zeros(self.n)
        if dead or e > 1:
            return c
        if e == 0:
            c[self._ahop[x][0]] += self.pa
        else:
            c[self._bhop[x][0]] -= self.pb
        return c

    def cell_attempt(self, v, base: int, ell: int):
        acc = np.zeros_like(v)
        for j in range(ell):
            x = (base + j) % self.L
            for e in range(4):
                acc += self.event(v, x, e, dead=(j == ell - 1))
        return acc / (4 * ell)

    def subsweep(self, v, ell: int, a: int):
        out = np.zeros_like(v)
        for sigma in range(ell):
            u = v
            for k in range(self.L // ell):
                base = (sigma + k * ell) % self.L
                for _ in range(a):
                    u = self.cell_attempt(u, base, ell)
            out += u
        return out / ell

    def dd_mcs(self, v, ell: int, S: int):
        a = 4 * ell // S
        for _ in range(S):
            v = self.subsweep(v, ell, a)
        return v

    def dd_subsweep_current(self, v, ell: int, a: int) -> float:
        """Expected net hop count (A right minus B left) of one sub-sweep from v."""
        total = 0.0
        for sigma in range(ell):
            for k in range(self.L // ell):
                base = (sigma + k * ell) % self.L
                cur = np.zeros(self.n)
                for j in range(ell):
                    x = (base + j) % self.L
                    for e in range(4):
                        cur += self.event_current(x, e, dead=(j == ell - 1))
                cur /= 4 * ell
                u = v
                for _ in range(a):
                    total += float(u @ cur) / ell
                    u = self.cell_attempt(u, base, ell)
        return total


    # --- the paper's two-lane SCA sequence -----------------------------------
    def sca_inlane(self, v, f: int):
        """Pairs (x, x+1), x = f mod 2: A hops right w.p. pa, B hops left w.p.
        pb, each lane's pair tried once (disjoint bits, so the order is free)."""
        for x in range(f, self.L, 2):
            v = self._move(v, self._ahop[x], self.pa)
            v = self._move(v, self._bhop[x], self.pb)
        return v

    def sca_inlane_current(self, v, f: int) -> float:
        return float(sum(v @ self.event_current(x, e, False)
                         for x in range(f, self.L, 2) for e in (0, 1)))

    def lane_change(self, v, to_b: bool, prob):
        """Every site once: A -> B (to_b) or B -> A with probability prob[x]."""
        moves = self._ab if to_b else self._ba
        for x in range(self.L):
            v = self._move(v, moves[x], prob[x])
        return v

    def sca_mcs(self, v, u, w):
        v = self.sca_inlane(v, 0)
        v = self.lane_change(v, True, u)
        v = self.sca_inlane(v, 1)
        return self.lane_change(v, False, w)


def stationary(step, v0: np.ndarray, tol: float = 1e-14, max_iter: int = 200000) -> np.ndarray:
    """Fixed point of a stochastic map by iteration from v0."""
    v = v0.copy()
    for _ in range(max_iter):
        w = step(v)
        if np.abs(w - v).sum() < tol:
            return w
        v = w
    raise RuntimeError("no convergence")


def state_index(bits) -> int:
    return int(sum(int(b) << i for i, b in enumerate(bits)))
