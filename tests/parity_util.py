"""Helpers of the GPU parity tests: the same run on the HIP library (through
the C ABI) and on the oracle, compared bit for bit.

The oracle's parameters are taken from the library's *resolved* parameters
(asep_get_params: cell size, sub-sweeps and compared bits as the library
used them), so a case checks the schedule that actually ran.
"""
import numpy as np


def oracle_params_from(orc, P):
    """The oracle's structure for resolved library parameters ``P``
    (a binding.asep_params)."""
    return orc.Params(
        L=int(P.L), model=int(P.model), init=int(P.init), density=float(P.density),
        p=float(P.p), q=float(P.q), slow_frac=float(P.slow_frac),
        slow_factor=float(P.slow_factor),
        samples_per_disorder=max(int(P.samples_per_disorder), 1),
        lane_rate=float(P.lane_rate), turn_frac=float(P.turn_frac), seed=int(P.seed),
        stream=int(P.stream), cell_log2=int(P.cell_log2), subsweeps=int(P.subsweeps),
        rbits=int(P.rbits), schedule=int(P.schedule))


def check_records(orc, L, got, ref, i, times, tag=""):
    """Records of sample i (library: list over times of Rough) against one
    oracle run: S1, S2, J, N exact, W^2 to 1e-12 relative."""
    for ti in range(len(times)):
        g = got[ti]
        assert g.S1[i] == ref.S1[ti], ("S1", tag, i, times[ti])
        assert g.S2[i] == ref.S2[ti], ("S2", tag, i, times[ti])
        assert g.J[i] == ref.J[ti], ("J", tag, i, times[ti])
        assert g.N[i] == ref.N[ti], ("N", tag, i, times[ti])
        w = orc.w2(L, int(ref.S1[ti]), ref.S2[ti])
        assert abs(g.w2[i] - w) <= 1e-12 * max(abs(w), 1e-300), ("W2", tag, i, times[ti])


def compare(orc, A, kw, times, samples, check_states=True, buffers="torch", plan=None,
            pool=None):
    """Run ``kw`` on the library and every sample on the oracle; everything
    must agree.  ``plan``: expected entries of the launch plan (asserted
    before any comparison, so a case that no longer reaches its kernel
    fails).  ``pool``: optional executor running the oracle samples in
    parallel."""
    print("case:", kw, "times", times[:4], "...", len(times), "samples", samples, flush=True)
    sim = A.Simulation(A.make_params(samples=samples, **kw), buffers=buffers)
    if plan:
        got_plan = sim.plan()
        for k, v in plan.items():
            assert got_plan[k] == v, ("plan", k, got_plan[k], v, got_plan)
    got = sim.run(times)
    OP = oracle_params_from(orc, sim.params)
    off = int(sim.params.sample_offset)
    if pool is not None:
        refs = [pool.submit(orc.run, OP, off + i, times) for i in range(samples)]
        refs = [r.result() for r in refs]
    else:
        refs = [orc.run(OP, off + i, times) for i in range(samples)]
    for i, ref in enumerate(refs):
        check_records(orc, kw["L"], got, ref, i, times)
        if check_states:
            words = sim.read_state(i)
            assert np.array_equal(words, orc.pack_words(ref.state)), ("state", i)
    sim.close()
    return got


def sweep_and_compare_states(orc, A, kw, n_mcs, samples, plan=None):
    """A bare sweep (no measurement inside the launch) against the oracle's
    advance of every sample; returns the simulation's hop counts."""
    sim = A.Simulation(A.make_params(samples=samples, **kw))
    if plan:
        got_plan = sim.plan()
        for k, v in plan.items():
            assert got_plan[k] == v, ("plan", k, got_plan[k], v, got_plan)
    sim.sweep(n_mcs)
    OP = oracle_params_from(orc, sim.params)
    off = int(sim.params.sample_offset)
    hops = sim.current()
    for i in range(samples):
        st = orc.init_state(OP, off + i)
        J = orc.advance(OP, off + i, st, 0, n_mcs)
        assert np.array_equal(sim.read_state(i), orc.pack_words(st)), ("state", i)
        assert int(hops[i]) == J, ("J", i)
    sim.close()
    return hops
