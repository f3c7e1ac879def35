"""The request loop on the GPU: continuous batching changes no result.

Every request's records equal those of the same request run alone through
asep_run, bit for bit (and the oracle's for the small ones); cancellation,
back-pressure and the memory budget behave as documented."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


import paper_1012_0385_amd as A  # noqa: E402
from paper_1012_0385_amd import binding as B  # noqa: E402
from paper_1012_0385_amd import workloads as W  # noqa: E402


def alone(kw, samples, times):
    sim = A.Simulation(A.make_params(samples=samples, **kw))
    out = sim.run(times)
    sim.close()
    return out


def same(a, b):
    return (np.array_equal(a.S1, b.S1) and a.S2 == b.S2 and np.array_equal(a.J, b.J)
            and np.array_equal(a.N, b.N))


def test_mix_equals_alone(orc):
    reqs = W.served_mix(24, rate_per_s=1e9, seed=11, max_attempts=2.0**31,
                        log2_L=(7, 22), log10_t=(1, 2.5), log2_samples=(0, 5))
    srv = A.Server(quantum_mcs=7, max_active=16)
    tickets = []
    for r in reqs:
        print("submit", r.model, r.L, r.samples, r.t_max, flush=True)
        tickets.append(srv.submit(A.make_params(samples=r.samples, **r.kwargs()), r.times, r.t_max))
    for r, t in zip(reqs, tickets):
        res = srv.wait(t, timeout_s=120)
        assert res["status"] == 0
        ref = alone(r.kwargs(), r.samples, r.times)
        assert len(ref) == len(res["rough"])
        for x, y in zip(res["rough"], ref):
            assert same(x, y), (r.model, r.L, r.samples)
        assert res["site_updates"] == r.attempts
        assert res["arrive_ns"] <= res["admit_ns"] <= res["start_ns"] <= res["done_ns"]
    srv.close()


def test_packed_small_requests_equal_alone():
    # many small rings of one kernel shape: they share launches in the server
    reqs = []
    for i in range(20):
        kw = dict(L=1024 + 64 * (i % 3), p=[1.0, 0.5, 0.75][i % 3], q=[0.0, 0.5, 0.25][i % 3],
                  seed=7 + i, stream=i)
        if i % 5 == 4:
            kw.update(slow_frac=0.2, slow_factor=0.5)
        reqs.append((kw, 1 + i % 4, [0, 3, 17, 40 + i]))
    srv = A.Server(quantum_mcs=11, max_active=32)
    tickets = [srv.submit(A.make_params(samples=n, **kw), times, times[-1]) for kw, n, times in reqs]
    packed = 0
    for (kw, n, times), t in zip(reqs, tickets):
        res = srv.wait(t, timeout_s=120)
        assert res["status"] == 0
        for x, y in zip(res["rough"], alone(kw, n, times)):
            assert same(x, y), kw
        # the result echoes the schedule and plan the request ran with
        sim = A.Simulation(A.make_params(samples=n, **kw))
        assert res["params"]["cell_log2"] == sim.params.cell_log2 == 6
        assert res["params"]["subsweeps"] == sim.params.subsweeps
        assert res["params"]["rbits"] == sim.params.rbits
        assert res["plan"] == sim.plan()
        sim.close()
        assert 1 <= res["quanta"] and res["packed_quanta"] <= res["quanta"]
        packed += res["packed_quanta"]
    assert packed > 0
    srv.close()


def test_sublattice_requests_in_the_mix():
    # the paper's SCA schedules (rings and two lanes) next to shifted ones:
    # packed where shapes agree, every request equal to its run alone
    reqs = []
    for i in range(18):
        if i % 3 == 0:
            kw = dict(L=1024 + 64 * (i % 2), p=0.8, q=0.1 * (i % 2), seed=3 + i, stream=i,
                      schedule=1)
        elif i % 3 == 1:
            kw = dict(L=512 * (1 + i % 2), model=1, init=1, p=0.5, q=0.5, lane_rate=0.8,
                      slow_frac=0.5, slow_factor=0.25, seed=3 + i, stream=i, schedule=1)
        else:
            kw = dict(L=1024, p=1.0, q=0.0, seed=3 + i, stream=i)
        reqs.append((kw, 1 + i % 3, [0, 2, 9, 25 + i]))
    srv = A.Server(quantum_mcs=6, max_active=32)
    tickets = [srv.submit(A.make_params(samples=n, **kw), times, times[-1]) for kw, n, times in reqs]
    for (kw, n, times), t in zip(reqs, tickets):
        res = srv.wait(t, timeout_s=120)
        assert res["status"] == 0
        for x, y in zip(res["rough"], alone(kw, n, times)):
            assert same(x, y), kw
    srv.close()


def test_server_matches_oracle_small(orc):
    kw = dict(L=4096, p=1.0, q=0.0, seed=1, stream=1)
    times = [0, 1, 2, 4, 8, 16, 33]
    srv = A.Server(quantum_mcs=5)
    t = srv.submit(A.make_params(samples=4, **kw), times, 40)
    res = srv.wait(t)
    P = orc.Params(L=4096, p=1.0, q=0.0, seed=1, stream=1)
    for i in range(4):
        ref = orc.run(P, i, times)
        for ti in range(len(times)):
            assert res["rough"][ti].S1[i] == ref.S1[ti] and res["rough"][ti].S2[i] == ref.S2[ti]
            assert res["rough"][ti].J[i] == ref.J[ti]
    srv.close()


def test_cancel_and_unknown_ticket():
    srv = A.Server(quantum_mcs=10, max_active=1)
    big = A.make_params(L=1 << 16, samples=64, p=1.0, q=0.0)
    t1 = srv.submit(big, [0, 100000], 100000)
    t2 = srv.submit(big, [0, 10], 10)  # queued behind t1
    srv.cancel(t2)
    srv.cancel(t1)
    assert srv.wait(t1)["status"] == B.ASEP_E_CANCELLED
    assert srv.wait(t2)["status"] == B.ASEP_E_CANCELLED
    with pytest.raises(A.AsepError):
        srv.poll(999999)
    srv.close()


def test_queue_full_and_budget():
    srv = A.Server(max_queue=2, max_active=1, quantum_mcs=10, hbm_budget_bytes=1 << 22)
    small = A.make_params(L=4096, samples=1)
    t1 = srv.submit(small, [0, 50], 50)
    # a request larger than the whole budget can never be admitted
    huge = A.make_params(L=1 << 20, samples=64)
    t2 = srv.submit(huge, [0], 0)
    codes = []
    for _ in range(6):
        try:
            srv.submit(small, [0], 0)
        except A.AsepError as e:
            codes.append(e.code)
    assert B.ASEP_E_BUSY in codes
    assert srv.wait(t1)["status"] == 0
    assert srv.wait(t2)["status"] == B.ASEP_E_NOMEM
    srv.close()


def test_invalid_request_rejected():
    srv = A.Server()
    with pytest.raises(A.AsepError):
        srv.submit(A.make_params(L=4096, samples=1), [5, 3], 10)  # unsorted times
    with pytest.raises(A.AsepError):
        srv.submit(A.make_params(L=4096, samples=1), [0, 20], 10)  # time past t_max
    srv.close()
