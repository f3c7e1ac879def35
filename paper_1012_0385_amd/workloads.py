"""Seeded synthetic inputs shaped like the paper's workloads.

Parameter sets and request streams only: nothing here simulates, measures or
lowers anything.  Both the benchmark and the tests draw their inputs from this
module.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# ring models of the served mix (Sec. 2.2 KPZ/TASEP, Sec. 2 EW/SSEP, Sec. 2.3
# columnar disorder with slow sites at rate r p)
MODELS = {
    "kpz": dict(p=1.0, q=0.0),
    "ew": dict(p=0.5, q=0.5),
    "disorder": dict(p=1.0, q=0.0, slow_frac=0.1, slow_factor=0.5, samples_per_disorder=4),
}


# Named ensemble workloads (besides the L = 2^17 KPZ + EW pair of the headline
# benchmark): (run parameters, samples, t_max, explicit times or None for the
# geometric schedule, description).
WORKLOADS = {
    "small_L4096": (dict(L=4096, p=1.0, q=0.0, seed=1, stream=1), 8, 1000,
                    [0] + [2 ** k for k in range(10)] + [1000],
                    "8 rings of 4096 sites, KPZ, 1000 MCS (full)"),
    "disorder_L2p16": (dict(L=1 << 16, p=1.0, q=0.0, slow_frac=0.1, slow_factor=0.5,
                            samples_per_disorder=4, seed=1, stream=2), 4096, 10 ** 6, None,
                       "1024 disorder realisations x 4 noise, L=2^16, 10^6 MCS"),
    "two_lane_L2p16": (dict(L=1 << 16, model=1, init=1, density=0.3, p=1.0, q=1.0, lane_rate=0.1,
                            turn_frac=0.05, seed=1, stream=3), 1024, 10 ** 5, None,
                       "1024 two-lane rings of 2^16 per lane, 10^5 MCS"),
    "sca_L2p17": (dict(L=1 << 17, p=0.8, q=0.0, seed=1, stream=4, schedule=1), 64, 10 ** 5, None,
                  "64 rings of 2^17, the paper's two-sub-lattice update at p = 0.8, 10^5 MCS"),
    "qssep_sca_L2p15": (dict(L=1 << 15, p=0.5, q=0.5, slow_frac=0.5, slow_factor=0.2, seed=1,
                             stream=5, schedule=1), 120, 10 ** 6, None,
                        "Q-SSEP (Q = 0.5, r = 0.2, p = q = 0.5), 120 realisations of 2^15, "
                        "two-sub-lattice update, 10^6 MCS"),
    "hbm_L2p26": (dict(L=1 << 26, p=1.0, q=0.0, seed=1, stream=7), 64, 1000, None,
                  "64 KPZ rings of 2^26 sites (512 MiB of state, beyond the 256 MB "
                  "last-level cache: resident in HBM), 1000 MCS"),
    "two_lane_sca_L2p12": (dict(L=1 << 12, model=1, init=1, density=0.5, p=0.5, q=0.5,
                                lane_rate=0.8, slow_frac=0.5, slow_factor=0.25, seed=1, stream=6,
                                schedule=1), 1024, 10 ** 5, None,
                           "the paper's two-lane SCA sequence (in-lane 0.5, crossing 0.8 / 0.2 "
                           "bimodal), 1024 rings of 2^12 per lane, 10^5 MCS"),
}


def geometric_times(t_max: int, t0: float = 30.0, factor: float = 1.05) -> list:
    """t = 0 and ceil(t0 * factor^i) <= t_max (Eq. sampling), plus t_max."""
    out = [0]
    t = t0
    while t <= t_max:
        c = int(math.ceil(t))
        if c > t_max:
            break
        if c != out[-1]:
            out.append(c)
        t *= factor
    if out[-1] != t_max:
        out.append(t_max)
    return out


@dataclass
class Request:
    arrival_s: float
    model: str
    L: int
    samples: int
    t_max: int
    seed: int
    stream: int
    times: list = field(default_factory=list)

    @property
    def attempts(self) -> int:
        return self.L * self.samples * self.t_max

    def kwargs(self) -> dict:
        kw = dict(MODELS[self.model])
        kw.update(L=self.L, seed=self.seed, stream=self.stream)
        return kw


def served_mix(n: int, rate_per_s: float, seed: int = 5, max_attempts: float = 2.0**38,
               log2_L=(10, 26), log10_t=(3, 5), log2_samples=(0, 8)) -> list:
    """Poisson stream of n ensemble requests: L = 64 ceil(2^x / 64) with
    x ~ U[10, 26], model uniform over MODELS, t_max = floor(10^y) with
    y ~ U[3, 5], samples = floor(2^z) with z ~ U[0, 8].  Requests whose work
    L * samples * t_max exceeds max_attempts are redrawn (the uncapped tail
    runs for minutes per request)."""
    rng = np.random.default_rng(seed)
    names = sorted(MODELS)
    t = 0.0
    out = []
    while len(out) < n:
        x = rng.uniform(*log2_L)
        L = 64 * int(math.ceil(2.0**x / 64))
        y = rng.uniform(*log10_t)
        t_max = int(math.floor(10.0**y))
        z = rng.uniform(*log2_samples)
        samples = int(math.floor(2.0**z))
        model = names[int(rng.integers(len(names)))]
        if L * samples * t_max > max_attempts:
            continue
        t += rng.exponential(1.0 / rate_per_s)
        out.append(Request(t, model, L, samples, t_max, seed=1000 + len(out), stream=len(out),
                           times=geometric_times(t_max)))
    return out
