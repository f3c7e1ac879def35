"""Run one named workload for a span of MCS (for profilers and spot checks).

    python -m paper_1012_0385_amd.run_workload NAME [--mcs N] [--start T]

Runs the workload's ensemble at its tuned launch shape and cell schedule from MCS T (default:
the middle of the job, the clock set with asep_set_time) for N MCS with the
job's own measurement times in that span, after a short warm-up, and prints
one JSON line with the rate.  NAME is a key of workloads.WORKLOADS.
"""
from __future__ import annotations

import argparse
import json
import time


def main() -> None:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("name")
    ap.add_argument("--mcs", type=int, default=2000)
    ap.add_argument("--start", type=int, default=-1, help="first MCS (default: t_max / 2)")
    args = ap.parse_args()

    import torch

    import paper_1012_0385_amd as A
    from paper_1012_0385_amd import tune
    from paper_1012_0385_amd import workloads as W

    kw, samples, t_max, times, desc = W.WORKLOADS[args.name]
    start = t_max // 2 if args.start < 0 else args.start
    full = times if times is not None else W.geometric_times(t_max)
    span = [start] + [t for t in full if start < t < start + args.mcs] + [start + args.mcs]
    A.load_tuning(tune.DEFAULT_TABLE)  # launch shape and cell schedule from the table
    sim = A.Simulation(A.make_params(samples=samples, **kw))
    sim.run([0, 1])  # warm-up
    sim.reset()
    sim.set_time(start)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.run(span)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    per_mcs = samples * kw["L"] * (4 if kw.get("model", 0) == 1 else 1)
    print(json.dumps({"workload": args.name, "desc": desc, "mcs": [start, start + args.mcs],
                      "measurements": len(span), "seconds": dt,
                      "site_updates_per_s": per_mcs * args.mcs / dt}))
    sim.close()


if __name__ == "__main__":
    main()
