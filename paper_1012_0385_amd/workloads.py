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
