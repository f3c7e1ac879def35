"""Autotuner of launch shapes and of the cell schedule.

For a set of run parameters it times short probe runs of candidate launch
shapes -- whole rings with several rings per workgroup, or rings cut into
windows advanced several sub-sweeps per launch -- and, for single-lane rings
under the shifted schedule whose caller left the cell size and sub-sweeps
open, the candidate cell schedules (64-site cells with four sub-sweeps per
MCS, 32-site cells with two), and keeps the fastest.  Launch shapes never
change results (every shape computes the same bits; the GPU parity tests
check shape invariance); the cell schedule is part of the update rule, so it
is only tuned where the caller left it to the table (cell_log2 = subsweeps =
0), and both candidates are pinned against random-sequential updating and
the growth exponents.

The table is the text file the library loads with asep_tuning_load, one
entry per class of run:
    model schedule disorder log2L_lo log2L_hi samples_lo samples_hi
    cell_log2 subsweeps windows window_sweeps rings_per_wg   # rate ...
A run matches the first entry whose model, schedule, disorder flag, range
of floor(log2 L) and range of samples contain it; parameters it left at 0
take the entry's values (0 in the entry leaves the default).
"""
from __future__ import annotations

import math
import os
import time

from . import binding as B
from .sim import Simulation, make_params, run_batch

DEFAULT_TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.txt")
FIELDS = ("model", "schedule", "disorder", "log2L_lo", "log2L_hi", "samples_lo", "samples_hi",
          "cell_log2", "subsweeps", "windows", "window_sweeps", "rings_per_wg")
HEADER = "# " + " ".join(FIELDS) + "\n"
SCHEDULES = [(6, 4), (5, 2)]  # (cell_log2, subsweeps) tried where the caller left them open


def class_of(kw: dict, samples: int) -> dict:
    """The class of run an entry tuned on (kw, samples) applies to: the same
    model, schedule and disorder flag, the same floor(log2 L), and from half
    to twice the samples."""
    e = int(math.floor(math.log2(kw["L"])))
    return dict(model=kw.get("model", 0), schedule=kw.get("schedule", 0),
                disorder=1 if kw.get("slow_frac", 0) > 0 else 0, log2L_lo=e, log2L_hi=e,
                samples_lo=max(1, (samples + 1) // 2), samples_hi=2 * samples)


def load_entries(path: str = DEFAULT_TABLE) -> list:
    """Entries of a table file as dicts (with the trailing comment, if any)."""
    out = []
    if not os.path.exists(path):
        return out
    with open(path) as f:
        for line in f:
            body, _, note = line.partition("#")
            vals = body.split()
            if not vals:
                continue
            if len(vals) != len(FIELDS):
                raise ValueError("malformed tuning entry: %r" % line)
            d = dict(zip(FIELDS, (int(v) for v in vals)))
            d["note"] = note.strip()
            out.append(d)
    return out


def _matches(e: dict, kw: dict, samples: int) -> bool:
    c = class_of(kw, samples)
    lg = c["log2L_lo"]
    return (e["model"] == c["model"] and e["schedule"] == c["schedule"] and
            e["disorder"] == c["disorder"] and e["log2L_lo"] <= lg <= e["log2L_hi"] and
            e["samples_lo"] <= samples <= e["samples_hi"])


def lookup(kw: dict, samples: int, path: str = DEFAULT_TABLE) -> dict:
    """Values of the first entry matching (kw, samples), or {} (the library's
    own resolution applies the same rule; this is for reports)."""
    for e in load_entries(path):
        if _matches(e, kw, samples):
            return {k: e[k] for k in ("cell_log2", "subsweeps", "windows", "window_sweeps",
                                      "rings_per_wg")}
    return {}


def store(kw: dict, samples: int, best: dict, device: str, path: str = DEFAULT_TABLE) -> None:
    """Write the entry of (kw, samples)'s class, replacing an entry of the same
    class, ahead of the first broader entry that also matches the run (the
    first match wins)."""
    c = class_of(kw, samples)
    entries = [e for e in load_entries(path)
               if any(e[k] != c[k] for k in c)]
    e = dict(c)
    for k in ("cell_log2", "subsweeps", "windows", "window_sweeps", "rings_per_wg"):
        e[k] = int(best.get(k, 0))
    e["note"] = "%.3e site-updates/s on %s" % (best.get("rate", 0.0), device)
    at = next((i for i, x in enumerate(entries) if _matches(x, kw, samples)), len(entries))
    entries.insert(at, e)
    with open(path, "w") as f:
        f.write("# Autotuned launch shapes and cell schedules (python -m paper_1012_0385_amd.tune)\n")
        f.write(HEADER)
        for x in entries:
            f.write(" ".join(str(x[k]) for k in FIELDS) + ("   # " + x["note"] if x["note"] else "")
                    + "\n")


def candidates(L: int, samples: int, cell_log2: int = 6):
    """Launch shapes worth trying for rings of L sites."""
    nw = L // 64
    out = [dict(windows=1, window_sweeps=0, rings_per_wg=0)]
    for w in (2, 3, 4, 6, 8, 16, 32, 64, 128, 256):
        if nw // w < 64:
            break
        for k in (15, 31, 63, 127, 255):
            if nw // w >= 2 * (k + 1):  # output at least twice the reach
                out.append(dict(windows=w, window_sweeps=k, rings_per_wg=0))
    if nw <= 64:
        for g in (1, 2, 4, 8, 16):
            out.append(dict(windows=1, window_sweeps=0, rings_per_wg=g))
    return out


def schedules_for(kw: dict):
    """Cell schedules to try: both candidates where the caller left the cell
    size and sub-sweeps open on a single-lane ring (with or without columnar
    disorder) under the shifted schedule, otherwise the caller's."""
    if (kw.get("model", 0) == 0 and kw.get("schedule", 0) == 0 and not kw.get("cell_log2")
            and not kw.get("subsweeps")):
        return [dict(cell_log2=c, subsweeps=s) for c, s in SCHEDULES]
    return [dict()]


def _probe(kws, samples, shape, times, streams) -> float:
    sims = []
    try:
        for kw, st in zip(kws, streams):
            sims.append(Simulation(make_params(samples=samples, **dict(kw, **shape)), stream=st))
    except B.AsepError:
        for s in sims:
            s.close()
        return 0.0
    import torch

    run_batch(sims, times[:2])  # warm-up launch
    for s in sims:
        s.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run_batch(sims, times)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    work = sum(s.samples * s.L * (4 if s.planes == 2 else 1) for s in sims) * times[-1]
    for s in sims:
        s.close()
    return work / dt


def tune(kws, samples: int, times, shapes=None, verbose: bool = False, refine_times=None,
         top: int = 3) -> dict:
    """Fastest (cell schedule, launch shape) for the simulations `kws` run
    together (each with `samples` rings) through the measurement times
    `times`.  With `refine_times`, the `top` candidates of that first pass
    are timed again over those (longer) times, which decide: short probes run
    at boost clocks and with denser measurements than a long run, so they
    only shortlist."""
    import torch

    streams = [torch.cuda.Stream() for _ in kws]
    scored = []
    for sched in schedules_for(kws[0]):
        for sh in shapes or candidates(kws[0]["L"], samples):
            cand = dict(sh, **sched)
            rate = _probe(kws, samples, cand, times, streams)
            if verbose:
                print("tune", cand, "%.3e" % rate, flush=True)
            if rate > 0:
                scored.append((rate, cand))
    if not scored:
        return None
    scored.sort(key=lambda x: -x[0])
    if refine_times is None:
        return dict(scored[0][1], rate=scored[0][0])
    best = None
    for _, cand in scored[:top]:
        rate = _probe(kws, samples, cand, refine_times, streams)
        if verbose:
            print("refine", cand, "%.3e" % rate, flush=True)
        if best is None or rate > best["rate"]:
            best = dict(cand, rate=rate)
    return best


# Workloads the shipped table is tuned on: (parameter sets run together, samples)
JOBS = [
    # the L = 2^17 KPZ + EW pair (run together)
    ([dict(L=1 << 17, p=1.0, q=0.0, seed=1, stream=0), dict(L=1 << 17, p=0.5, q=0.5, seed=1, stream=1)], 64),
    # columnar disorder: 1024 realisations x 4 noise seeds of 2^16 sites
    ([dict(L=1 << 16, p=1.0, q=0.0, slow_frac=0.1, slow_factor=0.5, samples_per_disorder=4,
           seed=1, stream=2)], 4096),
    # two lanes of 2^16 sites, 1024 samples
    ([dict(L=1 << 16, model=1, init=1, density=0.3, p=1.0, q=1.0, lane_rate=0.1,
           turn_frac=0.05, seed=1, stream=3)], 1024),
    # the paper's two-sub-lattice update, 64 rings of 2^17 at p = 0.8
    ([dict(L=1 << 17, p=0.8, q=0.0, seed=1, stream=4, schedule=1)], 64),
    # Q-SSEP under the two-sub-lattice update: 120 realisations of 2^15
    ([dict(L=1 << 15, p=0.5, q=0.5, slow_frac=0.5, slow_factor=0.2, seed=1, stream=5,
           schedule=1)], 120),
    # the paper's two-lane SCA (bimodal 0.8 / 0.2 crossing), 1024 rings of 2^12
    ([dict(L=1 << 12, model=1, init=1, density=0.5, p=0.5, q=0.5, lane_rate=0.8,
           slow_frac=0.5, slow_factor=0.25, seed=1, stream=6, schedule=1)], 1024),
]


if __name__ == "__main__":
    import argparse

    import torch

    ap = argparse.ArgumentParser(description="tune the benchmark workloads' classes")
    ap.add_argument("--t-max", type=int, default=2000)
    ap.add_argument("--only", type=int, default=-1, help="tune only job i")
    ap.add_argument("--out", default=DEFAULT_TABLE)
    ap.add_argument("--refine-t-max", type=int, default=0,
                    help="re-time the best candidates over a run of this many MCS (0: no); "
                         "the job's own length decides best, since short probes with dense "
                         "measurements favour short launches")
    ap.add_argument("--refine-top", type=int, default=3,
                    help="how many of the probes' best candidates the long run re-times")
    args = ap.parse_args()
    from .sim import load_tuning, sample_times

    load_tuning(None)  # probes must not pick up the table being written
    times = sample_times(30, 1.05, args.t_max)
    if times[-1] != args.t_max:
        times.append(args.t_max)
    dev = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    for i, (kws, samples) in enumerate(JOBS):
        if args.only >= 0 and i != args.only:
            continue
        jt = times if samples <= 256 else [t for t in times if t <= 300] + ([300] if times[-1] > 300 else [])
        rt = None
        if args.refine_t_max and samples <= 256:
            rt = sample_times(30, 1.05, args.refine_t_max)
            if rt[-1] != args.refine_t_max:
                rt.append(args.refine_t_max)
        best = tune(kws, samples, jt, verbose=True, refine_times=rt, top=args.refine_top)
        print("best", best, flush=True)
        if best:
            store(kws[0], samples, best, dev, args.out)
