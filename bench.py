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
# Algorithmic VALU work, in full-rate 32-bit lane slots, kept a lower bound of
# what any bit-packed implementation of an attempt needs: a Philox4x32-10
# block is 10 rounds x (2 32x32->64 products + 2 three-input XORs) = 40 slots
# (a throughput probe puts the product at ~1.35 slots on gfx950, so this is
# the low side), shared by the attempts whose fields its four words hold; an
# attempt's update is the field's offset, the pair read, the outcome, the
# flip of the two 32-bit halves of the word and the hop count (6 slots; a
# cell of at most 32 sites flips within one 32-bit word: 5; byte fields, which
# cells of 32 sites take, hold the offset where the shifts read it: one
# fewer; the hop count comes from the closing bond's flux and the particles'
# position sum, per sub-sweep rather than per attempt: one fewer), plus one slot for extracting compared bits (b > 0), one for a
# quenched mark and two for a second lane (its pair and the event decode).
PHILOX_SLOTS = 40
UPDATE_SLOTS = 6

# HBM traffic of one sweep launch at the tuned launch shape: rocprofv3 --pmc
# FETCH_SIZE and WRITE_SIZE (KiB per dispatch, mean over the sweep dispatches
# of `bench.py --t-max 2000 --steps 1 --warmup 0 --no-cpu --mix-requests 0
# --no-others --form plain`), scaled by what the same counters read for a 4 GiB
# device-to-device copy (`bench.py --calibrate-copy-mib 4096`).  They hold
# only for the kernel sources they were taken on (SHA-256 prefix below) and
# for that launch shape; otherwise the bench reports traffic as unknown.
SWEEP_TRAFFIC = {
    "src_sha256": "b09b9092d30e23f9",
    "launch_shape": {"windows": 4, "window_sweeps": 255, "rings_per_wg": 0},
    "fetch_kib": 858.15,   # KPZ 858.4, EW 857.9
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
    byte_fields = p.cell_log2 == 5 and w <= 8
    per_word = 4 if byte_fields else 32 // w
    nblk = -(-a // (4 * per_word))
    upd = UPDATE_SLOTS + (1 if p.rbits > 0 else 0) + (1 if p.slow_frac > 0 else 0) + (2 if two else 0)
    if p.cell_log2 <= 5 and not two:
        upd -= 1  # a cell of at most 32 sites flips within one 32-bit word
    if byte_fields:
        upd -= 1  # the offset is the low bits of its byte, read by the shifts
    upd -= 1  # no hop count per attempt
    return PHILOX_SLOTS * nblk / a + upd


# Sub-lattice schedules (the paper's SCA): per slot of 32 pairs (two lanes:
# 32 pairs of each lane, or 64 sites for a lane change) the kernel draws
# Philox blocks bit plane by bit plane until every live comparison of the
# slot is decided.  Algorithmic work of one slot = E[blocks] x (40 + planes
# per block x PLANE_OPS) + SLOT_OPS, where E[blocks] follows exactly from the
# thresholds' bits and the number of live pairs in the slot (each live
# comparison is still undecided after n planes with probability 2^-n, and
# is decided once the planes reach its threshold's last 1 bit).  PLANE_OPS:
# the plane's threshold mask and the bit-sliced compare (lt |= und & t & ~u;
# und &= ~(t ^ u)); SLOT_OPS: the pair masks, folding, the flip and the hop
# count.
SCA_PLANE_OPS = 4
SCA_SLOT_OPS = 16


def _sca_depth(T, b):
    """Planes that decide a comparison with threshold T of b bits (0: none needed)."""
    if T == 0 or T >= (1 << b):
        return 0
    return b - ((T & -T).bit_length() - 1)


def _expected_blocks(counts, depths, planes_per_block):
    """E[blocks] for slots with counts[c][slot] live comparisons of class c."""
    import numpy as np

    n_slots = counts[0].shape[0]
    live = np.zeros(n_slots, dtype=bool)
    for c, d in zip(counts, depths):
        if d:
            live |= c > 0
    e = live.astype(np.float64)
    dmax = max(depths) if depths else 0
    B = 1
    while planes_per_block * B < dmax:
        keep = np.ones(n_slots)
        for c, d in zip(counts, depths):
            if d and planes_per_block * B < d:
                keep *= (1.0 - 2.0 ** (-planes_per_block * B)) ** c
        e += 1.0 - keep
        B += 1
    return e


def sca_slots_per_attempt(sim, n_rings=4):
    """Algorithmic VALU slots per update of a sub-lattice simulation, from the
    live pairs of its current state (the first n_rings rings, both phases)."""
    import numpy as np

    P = sim.params
    L = sim.L
    b = int(P.rbits)

    def thr(x):
        return min(1 << 24, int(np.floor(x * (1 << 24)))) >> (24 - b)

    def bits(words):
        return np.unpackbits(words.view(np.uint8), bitorder="little").astype(bool)

    per_slot = []
    for i in range(min(n_rings, sim.samples)):
        w = sim.read_state(i)
        if P.model == 0:
            s = bits(w)
            T = [thr(P.p), thr(P.q), thr(P.slow_factor * P.p), thr(P.slow_factor * P.q)]
            d = [_sca_depth(t, b) for t in T]
            if P.slow_frac > 0:
                real = i // max(int(P.samples_per_disorder), 1)
                m0 = bits(sim.read_mask(0, real))
                m1 = bits(sim.read_mask(1, real)) if P.q > 0 else np.zeros(L, dtype=bool)
            else:
                m0 = m1 = np.zeros(L, dtype=bool)
            for ph in (0, 1):
                left = (np.arange(0, L, 2) + ph) % L
                right = (left + 1) % L
                fw = s[left] & ~s[right]
                bw = ~s[left] & s[right]
                cls = [fw & ~m0[left], bw & ~m1[right], fw & m0[left], bw & m1[right]]
                counts = [c.reshape(-1, 32).sum(axis=1) for c in cls]
                e = _expected_blocks(counts, d, 4)
                per_slot.append((e * (40 + 4 * SCA_PLANE_OPS) + SCA_SLOT_OPS) / 32.0)
        else:
            sa, sb = bits(w[: L // 64]), bits(w[L // 64:])
            T = [thr(P.p), thr(P.q), thr(P.lane_rate), thr(P.slow_factor * P.lane_rate)]
            d = [_sca_depth(t, b) for t in T]
            if P.slow_frac > 0:
                real = i // max(int(P.samples_per_disorder), 1)
                mu, mv = bits(sim.read_mask(0, real)), bits(sim.read_mask(1, real))
            else:
                mu = mv = np.zeros(L, dtype=bool)
            for ph in (0, 1):  # in-lane steps: 32 pairs of each lane per slot
                left = (np.arange(0, L, 2) + ph) % L
                right = (left + 1) % L
                ca = (sa[left] & ~sa[right]).reshape(-1, 32).sum(axis=1)
                cb = (~sb[left] & sb[right]).reshape(-1, 32).sum(axis=1)
                e = _expected_blocks([ca, cb], [d[0], d[1]], 2)
                per_slot.append((e * (40 + 2 * 2 * SCA_PLANE_OPS) + SCA_SLOT_OPS) / 64.0)
            for frm, to, mk in ((sa, sb, mu), (sb, sa, mv)):  # lane changes: 64 sites per slot
                live = frm & ~to
                c0 = (live & ~mk).reshape(-1, 64).sum(axis=1)
                c1 = (live & mk).reshape(-1, 64).sum(axis=1)
                e = _expected_blocks([c0, c1], [d[2], d[3]], 2)
                per_slot.append((e * (40 + 2 * SCA_PLANE_OPS) + SCA_SLOT_OPS) / 64.0)
    return float(np.mean([x.mean() for x in per_slot]))


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


def cpu_baseline(times_all, n_rings, t_cut, full_ring=False, sched=(6, 4)):
    """The oracle (plain C, one ring per host thread) on bounded samples of the
    workloads: the L = 2^17 pair's first t_cut MCS (n_rings per model) on
    every thread, and one core on one ring of it and on the whole L = 4096
    job; the disorder and two-lane workloads' first 1000 MCS on 16 rings
    (every thread) and one ring (one core, two lanes: 500 MCS); the first 8
    requests of the served mix, one ring each, each cut to at most 2^28
    attempts.  With full_ring, also one L = 2^17 KPZ ring over the whole
    10^5 MCS on one core (about four minutes)."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    from paper_1012_0385_amd import workloads as W

    oracle.build()
    threads = min(os.cpu_count() or 1, 16)

    def prefix(ts, cut):
        t = [x for x in ts if x <= cut]
        if t[-1] != cut:
            t.append(cut)
        return t

    def pool_run(jobs):
        t0 = time.perf_counter()
        with ThreadPoolExecutor(max_workers=threads) as ex:
            list(ex.map(lambda j: oracle.run(j[0], j[1], j[2]), jobs))
        return time.perf_counter() - t0

    def one_core(P, sample, times):
        t0 = time.perf_counter()
        oracle.run(P, sample, times)
        return time.perf_counter() - t0

    def as_run(kw, samples):
        # the cell schedule the GPU run takes from the tuning table, where the
        # workload leaves it open
        from paper_1012_0385_amd import tune

        if kw.get("cell_log2") or kw.get("subsweeps") or kw.get("schedule", 0):
            return kw
        e = tune.lookup(kw, samples)
        if e.get("cell_log2") and e.get("subsweeps"):
            return dict(kw, cell_log2=e["cell_log2"], subsweeps=e["subsweeps"])
        return kw

    times = prefix(times_all, t_cut)
    jobs = []
    for name, p, q, sid in MODELS:
        P = oracle.Params(L=L, p=p, q=q, seed=1, stream=sid, cell_log2=sched[0],
                          subsweeps=sched[1])
        jobs += [(P, i, times) for i in range(n_rings)]
    dt = pool_run(jobs)
    attempts = len(jobs) * L * t_cut
    out = {"value": attempts / dt, "unit": "site-updates/s", "cores": threads, "kind": "oracle",
           "sample": "%d rings (KPZ and EW, %d each) of L=2^17 for the first %d of 10^5 MCS "
                     "with the same measurement times; %.1f s wall" % (len(jobs), n_rings, t_cut, dt)}
    # one core: one KPZ ring of the same prefix, and the L = 4096 job in full
    d1 = one_core(jobs[0][0], 0, times)
    P1 = oracle.Params(L=4096, p=1.0, q=0.0, seed=1, stream=1)
    t1 = [0] + [2 ** k for k in range(10)] + [1000]
    t0 = time.perf_counter()
    for i in range(8):
        oracle.run(P1, i, t1)
    d2 = time.perf_counter() - t0
    out["single_core"] = {"value": L * t_cut / d1, "sample": "1 KPZ ring of L=2^17, %d MCS" % t_cut,
                          "small_L4096_full": {"value": 8 * 4096 * 1000 / d2, "seconds": d2}}
    # the disorder and two-lane workloads: prefixes on every thread and on one core
    others = {}
    for name, cut, cut1 in (("disorder_L2p16", 1000, 1000), ("two_lane_L2p16", 1000, 500)):
        kw, samples, t_max, _, desc = W.WORKLOADS[name]
        P = oracle.Params(**as_run(kw, samples))
        per = kw["L"] * (4 if kw.get("model", 0) == 1 else 1)
        full = W.geometric_times(t_max)
        dt = pool_run([(P, i, prefix(full, cut)) for i in range(16)])
        d1 = one_core(P, 0, prefix(full, cut1))
        others[name] = {"value": 16 * per * cut / dt, "cores": threads,
                        "sample": "16 rings, first %d MCS (%s); %.1f s wall" % (cut, desc, dt),
                        "single_core": {"value": per * cut1 / d1,
                                        "sample": "1 ring, first %d MCS" % cut1}}
    # the served mix: one ring of each of the first 8 requests, cut to 2^28 attempts
    reqs = W.served_mix(8, 1.0)
    jobs, work = [], 0
    for r in reqs:
        cut = max(1, min(r.t_max, (1 << 28) // r.L))
        jobs.append((oracle.Params(**as_run(r.kwargs(), r.samples)), 0, prefix(r.times, cut)))
        work += r.L * cut
    dt = pool_run(jobs)
    others["served_mix"] = {"value": work / dt, "cores": min(threads, len(jobs)),
                            "sample": "sample 0 of the first 8 served-mix requests, each cut "
                                      "to min(t_max, 2^28 / L) MCS; %.1f s wall" % dt}
    out["other_workloads"] = others
    if full_ring:
        # the whole 10^5-MCS job of one ring on one core, advanced between
        # its measurement times with a progress line every 10^4 MCS
        P = oracle.Params(L=L, p=1.0, q=0.0, seed=1, stream=0, cell_log2=sched[0],
                          subsweeps=sched[1])
        t0 = time.perf_counter()
        st = oracle.init_state(P, 0)
        J, t, mark = 0, 0, 0
        for tm in times_all:
            J = oracle.advance(P, 0, st, t, tm - t, J)
            oracle.sums(st, L)
            t = tm
            if t >= mark + 10000:
                mark = t
                print("oracle full ring: %d MCS, %.0f s" % (t, time.perf_counter() - t0),
                      file=sys.stderr, flush=True)
        d = time.perf_counter() - t0
        out["single_core"]["full_L2p17_ring"] = {
            "value": L * times_all[-1] / d, "seconds": d,
            "sample": "1 KPZ ring of L=2^17 over all %d MCS with its %d measurements"
                      % (times_all[-1], len(times_all))}
    return out


def served_mix_leg(A, W, n_req, load, n_lat=200, seed=5):
    """The served-mix workload: a Poisson stream of ensemble requests with
    L = 64 ceil(2^x/64), x ~ U[10,26], models KPZ / EW / disorder, t_max =
    10^U[3,5], samples = 2^U[0,8], redrawn above 2^38 attempts.

    capacity: the first n_req requests all available at t = 0, served
    (continuous batching) vs plain (one request after another, each one run
    per launch sequence).
    latency: n_lat requests arriving as a Poisson stream at `load` x the plain
    capacity, measured live both ways: through the request loop, and plain
    (one request at a time, in arrival order, each started when it has
    arrived and the previous one is done)."""
    import numpy as np
    import torch

    from paper_1012_0385_amd import tune

    def run_alone(r):
        sim = A.Simulation(A.make_params(samples=r.samples, **r.kwargs()), buffers="library")
        sim.run(r.times)
        sim.close()

    probe = W.served_mix(n_req, 1.0, seed=seed)
    total = sum(r.attempts for r in probe)

    # plain capacity: one request at a time
    t0 = time.perf_counter()
    for r in probe:
        run_alone(r)
    t_plain = time.perf_counter() - t0

    def serve(reqs, live_arrivals):
        srv = A.Server(quantum_mcs=2000, max_active=64, tuning_path=tune.DEFAULT_TABLE)
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

    def plain_live(reqs):
        lat = []
        start = time.perf_counter()
        for r in reqs:
            delay = r.arrival_s - (time.perf_counter() - start)
            if delay > 0:
                time.sleep(delay)
            run_alone(r)
            lat.append(time.perf_counter() - start - r.arrival_s)
        return lat

    torch.cuda.synchronize()
    _, t_served = serve(probe, live_arrivals=False)
    cap_plain = total / t_plain
    cap_served = total / t_served
    out = {
        "workload": "served mix: Poisson requests, L=64*ceil(2^U[10,26]/64), KPZ/EW/disorder, "
                    "t_max=10^U[3,5], samples=2^U[0,8], capped at 2^38 attempts",
        "capacity": {"served": cap_served, "plain": cap_plain, "unit": "site-updates/s",
                     "requests": n_req, "site_updates": total},
    }
    if n_lat <= 0:
        return out
    # Poisson arrivals at `load` x the plain capacity
    rate = load * cap_plain / (total / n_req)
    reqs = W.served_mix(n_lat, rate, seed=seed)
    work_lat = sum(r.attempts for r in reqs)
    lat_s, span_s = serve(reqs, live_arrivals=True)
    lat_p = plain_live(reqs)
    pct = lambda v, q: float(np.percentile(np.array(v), q))
    out["latency"] = {"requests": n_lat, "load": load, "arrival_rate_per_s": rate,
                      "site_updates": work_lat, "measured": "live, both forms",
                      "served_s": {"p50": pct(lat_s, 50), "p99": pct(lat_s, 99),
                                   "max": max(lat_s)},
                      "plain_s": {"p50": pct(lat_p, 50), "p99": pct(lat_p, 99),
                                  "max": max(lat_p)},
                      "served_throughput_at_load": work_lat / span_s}
    return out


HBM_PEAK = 8.0e12  # B/s


def state_bytes_per_launch(sim):
    """Algorithmic HBM bytes of one window launch: every ring's state read and
    written once, each read-only quenched plane read once."""
    p = sim.params
    words = sim.samples * sim.planes * (sim.L // 64)
    mplanes = 0
    if p.model == 1 and p.schedule == 0:
        mplanes = 1
    elif p.slow_frac > 0:
        mplanes = 2 if (p.q > 0 or p.model == 1) else 1
    n_real = -(-sim.samples // max(int(p.samples_per_disorder), 1))
    return 16 * words + 8 * mplanes * n_real * (sim.L // 64)


def other_workloads(A, t_cut=1000, t_span=2000):
    """Site-updates/s of the other workload shapes, one timed run each after
    a warm-up.  Jobs of at most t_cut MCS are timed whole; longer ones twice:
    over their first t_cut MCS ("prefix", with its dense measurement times)
    and over t_span MCS from the middle of the job ("steady": the clock set to
    t_max/2, the job's own measurement times in that span), which is what the
    bulk of the job runs at.  `value` is the steady rate where there is one.

    Every sweep launch of the whole job (or of the steady span) is timed with
    HIP events that its dispatch records: `kernel` gives the sweep kernel's
    own VALU fraction (algorithmic slots per launch / average launch time),
    and for windowed rings its algorithmic HBM bytes per launch and their
    rate against the 8 TB/s peak."""
    import torch

    from paper_1012_0385_amd import workloads as W

    out = {}

    def timed_run(sim, times, t_start):
        sim.reset()
        if t_start:
            sim.set_time(t_start)
        sim.profile(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.run(times)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        prof = sim.profile_read()
        sim.profile(False)
        return dt, prof

    for name, (kw, samples, t_max, times, desc) in W.WORKLOADS.items():
        full = times if times is not None else W.geometric_times(t_max)
        per_mcs = samples * kw["L"] * (4 if kw.get("model", 0) == 1 else 1)
        sim = A.Simulation(A.make_params(samples=samples, **kw))  # shape from the table
        sim.run(full[:3])  # warm-up
        entry = {"unit": "site-updates/s", "workload": desc, "plan": sim.plan()}
        if t_max <= t_cut:  # whole job
            dt, prof = timed_run(sim, full, 0)
            entry.update(value=per_mcs * t_max / dt, seconds=dt, mcs=[0, t_max],
                         measurements=len(full))
            if samples * kw["L"] <= 1 << 20:
                # the same rings one per run (each ring its own launch sequence)
                singles = [A.Simulation(A.make_params(samples=1, sample_offset=i, **kw))
                           for i in range(samples)]
                for one in singles:
                    one.run(full[:2])
                    one.reset()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for one in singles:
                    one.run(full)
                torch.cuda.synchronize()
                d1 = time.perf_counter() - t0
                entry["one_ring_per_run"] = {"value": per_mcs * t_max / d1, "seconds": d1}
                for one in singles:
                    one.close()
        else:
            pre = [t for t in full if t <= t_cut] + ([t_cut] if t_cut not in full else [])
            dt, _ = timed_run(sim, pre, 0)
            entry["prefix"] = {"value": per_mcs * t_cut / dt, "seconds": dt,
                               "mcs": [0, t_cut], "measurements": len(pre)}
            a = t_max // 2
            span = [a] + [t for t in full if a < t < a + t_span] + [a + t_span]
            dt, prof = timed_run(sim, span, a)
            entry["steady"] = {"value": per_mcs * t_span / dt, "seconds": dt,
                               "mcs": [a, a + t_span], "measurements": len(span)}
            entry["value"] = entry["steady"]["value"]
        slots = alu_slots_per_attempt(sim)
        if slots is None:
            slots = sca_slots_per_attempt(sim)
            entry["slots_note"] = ("sub-lattice schedule: expected Philox blocks per slot from "
                                   "the live pairs of the final state")
        entry["slots_per_attempt"] = slots
        # whole-run rate (launch gaps and measurements included) against the
        # VALU peak: a lower bound of the kernel's own fraction
        entry["alu_frac"] = entry["value"] * slots / PEAK_SLOTS
        if prof["launches"]:
            ks = prof["kernel_ms"] * 1e-3
            kern = {"launches": prof["launches"], "avg_launch_ms": prof["kernel_ms"] / prof["launches"],
                    "attempts_per_s": prof["attempts"] / ks,
                    "alu_frac": prof["attempts"] * slots / ks / PEAK_SLOTS}
            if entry["plan"]["windows"] > 1:
                b = state_bytes_per_launch(sim)
                kern["hbm"] = {"bytes_per_launch": b, "achieved_GBps": b * prof["launches"] / ks / 1e9,
                               "peak_GBps": HBM_PEAK / 1e9,
                               "frac": b * prof["launches"] / ks / HBM_PEAK}
            entry["kernel"] = kern
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
    ap.add_argument("--cpu-full-ring", action="store_true",
                    help="also time one L=2^17 KPZ ring over the whole job on one core (~4 min)")
    ap.add_argument("--t-max", type=int, default=T_MAX)
    ap.add_argument("--mix-requests", type=int, default=48,
                    help="served-mix requests of the capacity runs (0: skip the served mix)")
    ap.add_argument("--mix-latency-requests", type=int, default=200,
                    help="served-mix requests of the live latency runs")
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

    # the autotuner's table fills the launch shape and the cell schedule
    A.load_tuning(tune.DEFAULT_TABLE)
    streams = [torch.cuda.Stream() for _ in MODELS]
    sims = []
    shapes = []
    for (name, p, q, sid), st in zip(MODELS, streams):
        kw = dict(L=L, p=p, q=q, seed=1, stream=sid)
        sims.append(A.Simulation(A.make_params(samples=SAMPLES, **kw), stream=st))
        rp = sims[-1].params
        shapes.append({"windows": int(rp.windows), "window_sweeps": int(rp.window_sweeps),
                       "rings_per_wg": int(rp.rings_per_wg)})
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

        mix = served_mix_leg(A, W, args.mix_requests, args.mix_load, args.mix_latency_requests)
        print("served mix: %s" % json.dumps(mix), file=sys.stderr)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(times, args.cpu_rings, args.cpu_mcs, args.cpu_full_ring,
                           (int(sims[0].params.cell_log2), int(sims[0].params.subsweeps)))

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
                   "launch_shape": shapes[0], "plan": sims[0].plan(),
                   "cell_sites": 1 << int(sims[0].params.cell_log2),
                   "subsweeps_per_mcs": int(sims[0].params.subsweeps),
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
