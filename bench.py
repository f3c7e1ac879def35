#!/usr/bin/env python
"""Benchmark of the ASEP / KPZ sweep on one MI355X.

Workload (the LDS-resident ring configuration): rings of L = 2^17 sites,
half filled, flat start, KPZ (p = 1, q = 0) and EW (p = q = 1/2) with 64
samples each, 10^5 MCS, W^2 measured at t = 0 and at the geometric times of
Eq. (sampling) (t_0 = 30, factor 1.05: 168 measurements).  One step = one
such job: reset of both ensembles (init kernels) and their full runs.

Two forms are timed: "plain" runs the two ensembles one after the other
(one run per launch sequence); "batched" advances both through
asep_run_batch (each on its own stream, all launches queued before any
wait).  value = elementary update attempts (site updates) per second of
the batched form.

The JSON line also carries the ALU roofline of the dominant kernel (the
sweep kernel: per-launch algorithmic instruction slots over its average
duration from HIP events that the kernel's dispatch itself records on the
sweep's stream (`hipExtLaunchKernel`), taken in the plain form so that no
two launches overlap) and the CPU oracle timed on
the host cores over a bounded prefix of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

L = 1 << 17
SAMPLES = 64
T_MAX = 100_000
MODELS = (("kpz", 1.0, 0.0, 0), ("ew", 0.5, 0.5, 1))  # name, p, q, stream id
PEAK_SLOTS = 256 * 4 * 16 * 2.4e9  # CUs x SIMDs x lanes x clock: 32-bit VALU slots/s
# Algorithmic VALU work, in full-rate lane slots: a Philox4x32-10 block is 10
# rounds x (2 32x32->64 products + 2 three-input XORs), each product one
# v_mad_u64_u32 and each XOR one v_bitop3_b32, counted as one slot apiece
# (a throughput probe puts the product at ~1.35 slots on gfx950, so this
# count is the conservative one); an attempt's update is field extraction,
# pair test, threshold, flip and hop count.
PHILOX_SLOTS = 40
UPDATE_SLOTS = 10

# HBM traffic of one sweep launch at the tuned launch shape: rocprofv3 --pmc
# FETCH_SIZE and WRITE_SIZE (KiB per dispatch, mean over the sweep dispatches
# of `bench.py --t-max 2000 --steps 1 --warmup 0 --no-cpu --mix-requests 0
# --no-others --form plain`), scaled by what the same counters read for a 4 GiB
# device-to-device copy (`bench.py --calibrate-copy-mib 4096`).  They hold
# only for the kernel sources they were taken on (SHA-256 prefix below) and
# for that launch shape; otherwise the bench reports traffic as unknown.
SWEEP_TRAFFIC = {
    "src_sha256": "6ccf0d3e687eaae0",
    "launch_shape": {"windows": 4, "window_sweeps": 255, "rings_per_wg": 0},
    "fetch_kib": 840.48,   # KPZ 839.7, EW 841.25
    "write_kib": 1032.0,
    "fetch_scale": 2.0,    # 4 GiB copy: FETCH_SIZE 2097206 KiB
    "write_scale": 1.0,    # 4 GiB copy: WRITE_SIZE 4194304 KiB
}
SWEEP_SOURCES = ("asep_device.h", "asep_internal.h", "asep_sweep_plain.hip")


def sweep_source_hash() -> str:
    import hashlib

    h = hashlib.sha256()
    for name in SWEEP_SOURCES:
        with open(os.path.join(ROOT, "paper_1012_0385_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def sweep_traffic_bytes(shape):
    """HBM bytes per sweep launch, or None where the counters do not apply."""
    t = SWEEP_TRAFFIC
    if t["src_sha256"] != sweep_source_hash() or t["launch_shape"] != shape:
        return None
    return (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]) * 1024


LDS_PEAK = 128 * 256 * 2.4e9  # B/clk/CU x CUs x clock


def alu_slots_per_attempt(sim):
    """Algorithmic 32-bit VALU slots per attempt for a simulation under the
    shifted schedule (None for the sub-lattice schedules, whose random bits
    per update depend on the state through the lazy comparison)."""
    p = sim.params
    if p.schedule != 0:
        return None
    two = p.model == 1
    ell = 1 << p.cell_log2
    a = (4 * ell if two else ell) // p.subsweeps
    w = p.cell_log2 + (2 if two else 0) + p.rbits
    per_word = 32 // w
    nblk = -(-a // (4 * per_word))
    return PHILOX_SLOTS * nblk / a + UPDATE_SLOTS


def lds_bytes_per_attempt(sim):
    """State bytes per attempt if the ring were read and written through LDS
    once per sub-sweep (the LDS roofline's algorithmic traffic): L/4 bytes per
    ring per sub-sweep (two lanes: twice that) plus L/8 per read-only mask
    plane, over the attempts of a sub-sweep."""
    p = sim.params
    two = p.model == 1
    per_sub = p.L / 4 * (2 if two else 1) + p.L / 8 * (1 if (p.slow_frac > 0 or two) else 0)
    attempts_per_sub = p.L * (4 if two else 1) / p.subsweeps
    return per_sub / attempts_per_sub


def cpu_baseline(times_all, n_rings, t_cut):
    """The oracle on a prefix: n_rings per model for t_cut MCS, on host threads."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle

    oracle.build()
    threads = min(os.cpu_count() or 1, 16)
    times = [t for t in times_all if t <= t_cut]
    if times[-1] != t_cut:
        times.append(t_cut)
    jobs = []
    for name, p, q, sid in MODELS:
        P = oracle.Params(L=L, p=p, q=q, seed=1, stream=sid)
        jobs += [(P, i) for i in range(n_rings)]
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(lambda j: oracle.run(j[0], j[1], times), jobs))
    dt = time.perf_counter() - t0
    attempts = len(jobs) * L * t_cut
    out = {"value": attempts / dt, "unit": "site-updates/s", "cores": threads, "kind": "oracle",
           "sample": "%d rings (KPZ and EW, %d each) of L=2^17 for the first %d of 10^5 MCS "
                     "with the same measurement times; %.1f s wall" % (len(jobs), n_rings, t_cut, dt)}
    # one core: one KPZ ring of the same prefix, and the L = 4096 job in full
    t0 = time.perf_counter()
    oracle.run(jobs[0][0], 0, times)
    d1 = time.perf_counter() - t0
    P1 = oracle.Params(L=4096, p=1.0, q=0.0, seed=1, stream=1)
    t1 = [0] + [2 ** k for k in range(10)] + [1000]
    t0 = time.perf_counter()
    for i in range(8):
        oracle.run(P1, i, t1)
    d2 = time.perf_counter() - t0
    out["single_core"] = {"value": L * t_cut / d1, "sample": "1 KPZ ring of L=2^17, %d MCS" % t_cut,
                          "small_L4096_full": {"value": 8 * 4096 * 1000 / d2, "seconds": d2}}
    return out


def served_mix_leg(A, W, n_req, load, seed=5):
    """The served-mix workload: a Poisson stream of ensemble requests with
    L = 64 ceil(2^x/64), x ~ U[10,26], models KPZ / EW / disorder, t_max =
    10^U[3,5], samples = 2^U[0,8], redrawn above 2^38 attempts.

    capacity: every request available at t = 0, served (continuous batching)
    vs plain (one request after another, each one run per launch sequence).
    latency: arrivals at `load` x the plain capacity; served measured live,
    plain replayed as a FIFO queue from its measured service times."""
    import numpy as np
    import torch

    probe = W.served_mix(n_req, 1.0, seed=seed)
    total = sum(r.attempts for r in probe)

    # plain capacity: one request at a time
    service = []
    t0 = time.perf_counter()
    for r in probe:
        ts = time.perf_counter()
        sim = A.Simulation(A.make_params(samples=r.samples, **r.kwargs()), buffers="library")
        sim.run(r.times)
        sim.close()
        service.append(time.perf_counter() - ts)
    t_plain = time.perf_counter() - t0

    def serve(reqs, live_arrivals):
        srv = A.Server(quantum_mcs=2000, max_active=64)
        tickets = []
        start = time.perf_counter()
        for r in reqs:
            if live_arrivals:
                delay = r.arrival_s - (time.perf_counter() - start)
                if delay > 0:
                    time.sleep(delay)
            tickets.append(srv.submit(A.make_params(samples=r.samples, **r.kwargs()), r.times,
                                      r.t_max))
        res = [srv.wait(t, timeout_s=600) for t in tickets]
        srv.close()
        assert all(x["status"] == 0 for x in res)
        lat = [(x["done_ns"] - x["arrive_ns"]) * 1e-9 for x in res]
        span = (max(x["done_ns"] for x in res) - min(x["arrive_ns"] for x in res)) * 1e-9
        return lat, span

    torch.cuda.synchronize()
    _, t_served = serve(probe, live_arrivals=False)
    cap_plain = total / t_plain
    cap_served = total / t_served
    # Poisson arrivals at `load` x the plain capacity
    rate = load * cap_plain / (total / n_req)
    reqs = W.served_mix(n_req, rate, seed=seed)
    lat_s, span_s = serve(reqs, live_arrivals=True)
    done, lat_p = 0.0, []
    for r, svc in zip(reqs, service):
        done = max(done, r.arrival_s) + svc
        lat_p.append(done - r.arrival_s)
    pct = lambda v, q: float(np.percentile(np.array(v), q))
    return {
        "workload": "served mix: %d Poisson requests, L=64*ceil(2^U[10,26]/64), KPZ/EW/disorder, "
                    "t_max=10^U[3,5], samples=2^U[0,8], capped at 2^38 attempts" % n_req,
        "site_updates": total,
        "capacity": {"served": cap_served, "plain": cap_plain, "unit": "site-updates/s"},
        "load": load, "arrival_rate_per_s": rate,
        "latency_s": {"served": {"p50": pct(lat_s, 50), "p99": pct(lat_s, 99)},
                      "plain": {"p50": pct(lat_p, 50), "p99": pct(lat_p, 99)}},
        "served_throughput_at_load": total / span_s,
    }


def other_workloads(A, t_cut=1000, t_span=2000):
    """Site-updates/s of the other workload shapes, one timed run each after
    a warm-up.  Jobs longer than t_cut MCS are timed twice: over their first
    t_cut MCS ("prefix", with its dense measurement times) and over t_span
    MCS from the middle of the job ("steady": the clock set to t_max/2, the
    job's own measurement times in that span), which is what the bulk of the
    job runs at.  `value` is the steady rate where there is one."""
    import torch

    from paper_1012_0385_amd import tune
    from paper_1012_0385_amd import workloads as W

    out = {}

    def timed_run(sim, times, t_start):
        sim.reset()
        if t_start:
            sim.set_time(t_start)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.run(times)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    for name, (kw, samples, t_max, times, desc) in W.WORKLOADS.items():
        full = A.sample_times(30, 1.05, t_max)
        if full[-1] != t_max:
            full.append(t_max)
        per_mcs = samples * kw["L"] * (4 if kw.get("model", 0) == 1 else 1)
        sim = A.Simulation(A.make_params(samples=samples, **kw, **tune.lookup(kw, samples)))
        sim.run(full[:3])  # warm-up
        entry = {"unit": "site-updates/s", "workload": desc}
        if times is not None:  # whole job
            dt = timed_run(sim, times, 0)
            entry.update(value=per_mcs * times[-1] / dt, seconds=dt)
            # the same rings one per run (each ring its own launch sequence)
            singles = [A.Simulation(A.make_params(samples=1, sample_offset=i, **kw))
                       for i in range(samples)]
            for one in singles:
                one.run(times[:2])
                one.reset()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for one in singles:
                one.run(times)
            torch.cuda.synchronize()
            d1 = time.perf_counter() - t0
            entry["one_ring_per_run"] = {"value": per_mcs * times[-1] / d1, "seconds": d1}
            for one in singles:
                one.close()
        else:
            pre = [t for t in full if t <= t_cut] + ([t_cut] if t_cut not in full else [])
            dt = timed_run(sim, pre, 0)
            entry["prefix"] = {"value": per_mcs * t_cut / dt, "seconds": dt,
                               "mcs": [0, t_cut], "measurements": len(pre)}
            a = t_max // 2
            span = [a] + [t for t in full if a < t < a + t_span] + [a + t_span]
            dt = timed_run(sim, span, a)
            entry["steady"] = {"value": per_mcs * t_span / dt, "seconds": dt,
                               "mcs": [a, a + t_span], "measurements": len(span)}
            entry["value"] = entry["steady"]["value"]
        slots = alu_slots_per_attempt(sim)
        if slots is not None:
            # whole-run rate (launch gaps and measurements included) against
            # the VALU peak: a lower bound of the kernel's own fraction
            entry["alu_frac"] = entry["value"] * slots / PEAK_SLOTS
            entry["slots_per_attempt"] = slots
        out[name] = entry
        sim.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--cpu-rings", type=int, default=16)
    ap.add_argument("--cpu-mcs", type=int, default=1000)
    ap.add_argument("--t-max", type=int, default=T_MAX)
    ap.add_argument("--mix-requests", type=int, default=48, help="served-mix requests (0: skip)")
    ap.add_argument("--mix-load", type=float, default=0.8)
    ap.add_argument("--no-others", action="store_true", help="skip the other workload shapes")
    ap.add_argument("--form", choices=("both", "plain"), default="both",
                    help="plain: time only the one-after-the-other form (value = plain), "
                         "so that a kernel trace holds no overlapped launches")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="only run a device-to-device copy of this many MiB (counter scale)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(replicas would shard with no communication; see the design notes)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1012_0385_amd as A

    torch.cuda.set_device(0)
    if args.calibrate_copy_mib:
        n = args.calibrate_copy_mib << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n}))
        return
    times = A.sample_times(30, 1.05, args.t_max)
    if times[-1] != args.t_max:
        times.append(args.t_max)
    from paper_1012_0385_amd import tune

    streams = [torch.cuda.Stream() for _ in MODELS]
    sims = []
    shapes = []
    for (name, p, q, sid), st in zip(MODELS, streams):
        kw = dict(L=L, p=p, q=q, seed=1, stream=sid)
        shape = tune.lookup(kw, SAMPLES)  # launch shape only; results do not depend on it
        shapes.append(shape)
        sims.append(A.Simulation(A.make_params(samples=SAMPLES, **kw, **shape), stream=st))
    attempts_per_step = sum(s.samples * s.L for s in sims) * args.t_max

    def run_one(sim, out, k):
        sim.reset()
        out[k] = sim.run(times)

    def step_plain():
        out = [None] * len(sims)
        for k, s in enumerate(sims):
            run_one(s, out, k)
        return out

    def step_batched():
        for s in sims:
            s.reset()
        return A.run_batch(sims, times)

    step_s = {"plain": [], "batched": []}

    def timed(step, n, form):
        # every step returns its records, i.e. ends synchronised with the device
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            ts = time.perf_counter()
            step()
            step_s[form].append(time.perf_counter() - ts)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    def step_stats(form):
        v = sorted(step_s[form])
        if not v:
            return None
        return {"median_ms": v[len(v) // 2] * 1e3, "min_ms": v[0] * 1e3, "max_ms": v[-1] * 1e3}

    for _ in range(args.warmup):
        step_batched() if args.form == "both" else step_plain()
    # plain form, with kernel timing on: launches of one ensemble never
    # overlap, so each event pair times one kernel alone
    for s in sims:
        s.profile(True)
    t_plain = timed(step_plain, args.steps, "plain")
    prof = [s.profile_read() for s in sims]
    for s in sims:
        s.profile(False)
    # batched form
    t_batch = timed(step_batched, args.steps, "batched") if args.form == "both" else t_plain
    print("plain %.3f s, batched %.3f s over %d steps" % (t_plain, t_batch, args.steps),
          file=sys.stderr)

    batched_value = attempts_per_step * args.steps / t_batch
    plain_value = attempts_per_step * args.steps / t_plain
    value = batched_value
    launches = sum(p["launches"] for p in prof)
    kernel_ms = sum(p["kernel_ms"] for p in prof)
    slots = sum(p["attempts"] * alu_slots_per_attempt(s) for p, s in zip(prof, sims))
    avg_ms = kernel_ms / launches
    achieved = slots / launches / (avg_ms * 1e-3)
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_SLOTS / 1e12,
                "unit": "TOP/s", "frac": achieved / PEAK_SLOTS,
                "traffic": sweep_traffic_bytes(shapes[0]),
                "kernel": "k_sweep", "avg_launch_ms": avg_ms, "launches": launches}

    # the LDS roofline as the workload statement defines it: the state through
    # LDS once per sub-sweep; here the rings stay in VGPRs and LDS carries one
    # neighbour word per lane and sub-sweep, so this fraction stays small
    lds_bpa = lds_bytes_per_attempt(sims[0])
    lds = {"bytes_per_attempt": lds_bpa, "achieved_GBps": value * lds_bpa / 1e9,
           "peak_GBps": LDS_PEAK / 1e9, "frac": value * lds_bpa / LDS_PEAK,
           "note": "state held in VGPRs; LDS carries 8 B per lane per sub-sweep"}

    others = None if args.no_others else other_workloads(A)
    if others:
        print("other workloads: %s" % json.dumps(others), file=sys.stderr)

    mix = None
    if args.mix_requests > 0:
        from paper_1012_0385_amd import workloads as W

        mix = served_mix_leg(A, W, args.mix_requests, args.mix_load)
        print("served mix: %s" % json.dumps(mix), file=sys.stderr)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(times, args.cpu_rings, args.cpu_mcs)

    line = {
        "metric": "site-updates/s (1 GPU)",
        "value": value,
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_batch / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64 bit planes, u32 Philox",
        "data": "synthetic: flat (1010...) start, Philox4x32-10 noise keyed by (seed=1, stream, sample)",
        "config": {"workload": "LDS-resident rings: L=2^17, half filling, flat start, KPZ (p=1,q=0) "
                               "and EW (p=q=0.5), 64 samples each, 10^5 MCS, W^2 at t=0 and "
                               "ceil(30*1.05^i)",
                   "rings": len(sims) * SAMPLES, "L": L, "t_max": args.t_max,
                   "launch_shape": shapes[0] or "automatic",
                   "measurements": len(times), "parallelism": "1 GPU"},
        "plain": {"value": plain_value, "ms_per_step": t_plain / args.steps * 1e3,
                  "steps": step_stats("plain")},
        "batched": ({"value": batched_value, "ms_per_step": t_batch / args.steps * 1e3,
                     "steps": step_stats("batched")}
                    if args.form == "both" else None),
        "lds_roofline": lds,
        "roofline": roofline,
        "served_mix": mix,
        "other_workloads": others,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
