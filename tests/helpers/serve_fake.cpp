// serve_fake.cpp -- TEST ONLY: the request loop's policy core driven by a
// CPU executor that runs every request on the oracle.
//
// The core (paper_1012_0385_amd/csrc/asep_server.cpp) is linked unchanged;
// this executor replaces the device: a memory budget in bytes, quanta run on
// the oracle when first polled (after a pseudo-random number of "still
// running" answers), shared launches sometimes refused.  Each scenario goes
// through the public C calls (asep_submit / asep_wait / asep_poll /
// asep_cancel) and checks every request against the oracle run alone.
// Prints one line per check and exits non-zero on the first failure.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdlib>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "asep_serve.h"

extern "C" {
#include "asep_oracle.h"
}

using asep::serve::Executor;
using asep::serve::Job;

namespace {

orc_params to_orc(const asep_params& p) {
    orc_params o;
    memset(&o, 0, sizeof o);
    o.model = p.model == ASEP_MODEL_TWO_LANE ? ORC_TWO_LANE : ORC_RING;
    o.init = p.init == ASEP_INIT_BERNOULLI ? ORC_INIT_BERNOULLI : ORC_INIT_FLAT;
    o.L = p.L;
    o.density = p.density;
    o.p = p.p;
    o.q = p.q;
    o.slow_frac = p.slow_frac;
    o.slow_factor = p.slow_factor;
    o.samples_per_disorder = p.samples_per_disorder ? p.samples_per_disorder : 1;
    o.lane_rate = p.lane_rate;
    o.turn_frac = p.turn_frac;
    o.seed = p.seed;
    o.stream = p.stream;
    o.cell_log2 = p.cell_log2 ? (uint32_t)p.cell_log2 : 6;
    o.subsweeps = p.subsweeps ? (uint32_t)p.subsweeps : 4;
    o.rbits = p.rbits > 0 ? p.rbits : -1;  // the library's 0 means automatic
    o.schedule = p.schedule == ASEP_SCHED_SUBLATTICE ? ORC_SCHED_SUBLATTICE : ORC_SCHED_SHIFTED;
    return o;
}

asep_rough record_of(const orc_params& P, const uint8_t* s, int64_t J) {
    asep_rough r;
    memset(&r, 0, sizeof r);
    int64_t N = 0;
    orc_sums(s, P.L, &r.sum_h, &r.sum_h2_lo, &r.sum_h2_hi, &N);
    if (P.model == ORC_TWO_LANE)
        for (uint64_t x = 0; x < P.L; ++x) N += s[P.L + x];
    r.particles = N;
    r.hops = J;
    r.w2 = orc_w2(P.L, r.sum_h, r.sum_h2_lo, r.sum_h2_hi);
    return r;
}

struct FakeJob {
    orc_params P;
    uint32_t samples = 0, offset = 0;
    std::vector<std::vector<uint8_t>> state;
    std::vector<int64_t> J;
    uint64_t t = 0;        // queued up to
    uint64_t ran_to = 0;   // the oracle has run up to
    uint64_t q_t1 = 0;     // quantum in flight
    uint32_t q_first = 0, q_n = 0;
    int polls = 0;
    std::vector<asep_rough> staged;
    size_t bytes = 0;
};

class FakeExecutor final : public Executor {
   public:
    FakeExecutor(size_t budget, uint32_t cap, int max_polls, uint32_t refuse_every,
                 uint64_t max_q = ~0ull)
        : budget_(budget), cap_(cap), max_polls_(max_polls), refuse_every_(refuse_every),
          max_q_(max_q) {}

    std::vector<uint64_t> admitted;  // tickets in admission order (read after the run)
    std::atomic<uint64_t> n_admitted{0};
    std::atomic<uint64_t> shared_launches{0};
    std::atomic<uint64_t> longest_quantum{0};

    int init() override { return ASEP_OK; }
    void shutdown() override {}

    int footprint(const asep_params& p, size_t* state_bytes, size_t* aux_bytes) override {
        if (p.abi_version != ASEP_ABI_VERSION || p.samples == 0) return ASEP_E_INVAL;
        orc_params o = to_orc(p);
        orc_sched s;
        if (orc_lower(&o, &s) != 0) return ASEP_E_INVAL;
        *state_bytes = (size_t)p.samples * (p.model == ASEP_MODEL_TWO_LANE ? 2 : 1) * p.L / 8;
        *aux_bytes = 4096;
        return ASEP_OK;
    }

    int admit(Job& j) override {
        const size_t need = j.state_bytes + j.aux_bytes;
        if (used_ + need > budget_) return ASEP_E_NOMEM;
        auto* f = new FakeJob();
        f->P = to_orc(j.params);
        f->samples = j.params.samples;
        f->offset = j.params.sample_offset;
        orc_sched s;
        orc_lower(&f->P, &s);
        const size_t planes = f->P.model == ORC_TWO_LANE ? 2 : 1;
        f->state.assign(f->samples, std::vector<uint8_t>(planes * f->P.L));
        f->J.assign(f->samples, 0);
        for (uint32_t i = 0; i < f->samples; ++i)
            orc_init_state(&f->P, &s, f->offset + i, f->state[i].data());
        f->bytes = need;
        f->polls = next_polls();
        used_ += need;
        j.x = f;
        j.resolved = j.params;
        j.resolved.cell_log2 = (int32_t)f->P.cell_log2;
        j.resolved.subsweeps = (int32_t)f->P.subsweeps;
        j.plan = asep_plan{};
        admitted.push_back(j.ticket);
        n_admitted++;
        return ASEP_OK;
    }

    void release(Job& j) override {
        auto* f = fj(j);
        used_ -= f->bytes;
        delete f;
        j.x = nullptr;
    }

    void wait(Job&) override {}
    uint64_t time(const Job& j) override { return fj(j)->t; }
    uint32_t record_capacity(const Job&) override { return cap_; }
    uint64_t max_quantum_mcs(const Job&) override { return max_q_; }
    uint64_t attempts_per_mcs(const Job& j) override {
        return (uint64_t)j.params.samples * j.params.L *
               (j.params.model == ASEP_MODEL_TWO_LANE ? 4 : 1);
    }

    int query(Job& j) override {
        auto* f = fj(j);
        if (f->polls > 0) {
            --f->polls;
            return ASEP_E_PENDING;
        }
        // run the quantum in flight (if any) on the oracle
        if (f->ran_to < f->q_t1 || f->q_n) {
            f->staged.assign((size_t)f->q_n * f->samples, asep_rough{});
            for (uint32_t i = 0; i < f->samples; ++i) {
                uint64_t t = f->ran_to;
                for (uint32_t k = 0; k < f->q_n; ++k) {
                    const uint64_t tk = j.times[f->q_first + k];
                    orc_advance(&f->P, f->offset + i, f->state[i].data(), t, tk - t, &f->J[i]);
                    t = tk;
                    f->staged[(size_t)k * f->samples + i] = record_of(f->P, f->state[i].data(), f->J[i]);
                }
                orc_advance(&f->P, f->offset + i, f->state[i].data(), t, f->q_t1 - t, &f->J[i]);
            }
            f->ran_to = f->q_t1;
        }
        return ASEP_OK;
    }

    void collect(Job& j) override {
        auto* f = fj(j);
        if (f->q_first != j.staged_first || f->q_n != j.staged_n) {
            fprintf(stderr, "FAIL staged range mismatch\n");
            std::abort();
        }
        for (size_t k = 0; k < f->staged.size(); ++k)
            j.rough[(size_t)j.staged_first * f->samples + k] = f->staged[k];
        f->q_n = 0;
        f->staged.clear();
    }

    bool pack_key(const Job& j, uint64_t* key) override {
        *key = j.params.L * 4 + j.params.model * 2 + j.params.schedule;
        return true;
    }

    bool queue(const std::vector<Job*>& g, const std::vector<uint64_t>& t_end,
               const std::vector<uint32_t>& n, std::vector<int>* rcs,
               std::vector<char>* shared) override {
        if (g.size() > 1) {
            if (refuse_every_ && (++tries_ % refuse_every_) == 0) return false;
            shared_launches++;
        }
        for (size_t i = 0; i < g.size(); ++i) {
            auto* f = fj(*g[i]);
            (*shared)[i] = g.size() > 1;
            const uint64_t len = t_end[i] >= f->t ? t_end[i] - f->t : 0;
            if (len > longest_quantum) longest_quantum = len;
            if (t_end[i] < f->t || f->q_n || n[i] > cap_ || len > max_q_) {
                (*rcs)[i] = ASEP_E_INVAL;
                continue;
            }
            f->q_first = g[i]->next_time;
            f->q_n = n[i];
            f->q_t1 = t_end[i];
            f->t = t_end[i];
            f->polls = next_polls();
            (*rcs)[i] = ASEP_OK;
        }
        return true;
    }

    void sync_all() override {}

   private:
    static FakeJob* fj(const Job& j) { return static_cast<FakeJob*>(j.x); }
    int next_polls() {
        lcg_ = lcg_ * 6364136223846793005ull + 1442695040888963407ull;
        return max_polls_ ? (int)((lcg_ >> 33) % (uint64_t)(max_polls_ + 1)) : 0;
    }

    size_t budget_, used_ = 0;
    uint32_t cap_;
    int max_polls_;
    uint32_t refuse_every_, tries_ = 0;
    uint64_t max_q_;
    uint64_t lcg_ = 12345;
};

int failures = 0;

void check(bool ok, const char* what, long a = 0, long b = 0) {
    printf("%s %s %ld %ld\n", ok ? "OK" : "FAIL", what, a, b);
    fflush(stdout);
    if (!ok) ++failures;
}

struct Req {
    asep_params p;
    uint64_t t_max;
    std::vector<uint64_t> times;
};

asep_params base_params(uint64_t L, uint32_t samples) {
    asep_params p;
    memset(&p, 0, sizeof p);
    p.abi_version = ASEP_ABI_VERSION;
    p.L = L;
    p.samples = samples;
    p.samples_per_disorder = 1;
    p.density = 0.5;
    p.p = 1.0;
    p.rbits = -1;
    p.seed = 1;
    return p;
}

// The request's records equal the oracle's run of each sample alone.
bool equals_alone(const Req& r, const asep_result& res) {
    if (res.status != ASEP_OK || res.n_times != r.times.size() || res.samples != r.p.samples)
        return false;
    orc_params P = to_orc(r.p);
    std::vector<orc_record> rec(r.times.size());
    for (uint32_t i = 0; i < r.p.samples; ++i) {
        if (orc_run(&P, r.p.sample_offset + i, r.times.data(), (uint32_t)r.times.size(),
                    rec.data(), nullptr) != 0)
            return false;
        for (size_t k = 0; k < r.times.size(); ++k) {
            const asep_rough& g = res.rough[k * r.p.samples + i];
            if (g.sum_h != rec[k].S1 || g.sum_h2_lo != rec[k].S2_lo || g.sum_h2_hi != rec[k].S2_hi ||
                g.hops != rec[k].J || g.particles != rec[k].N)
                return false;
            if (g.w2 != orc_w2(P.L, rec[k].S1, rec[k].S2_lo, rec[k].S2_hi)) return false;
        }
    }
    return res.site_updates ==
           r.t_max * r.p.samples * r.p.L * (r.p.model == ASEP_MODEL_TWO_LANE ? 4 : 1);
}

uint64_t rng_state = 99;
uint64_t rnd(uint64_t n) {
    rng_state = rng_state * 6364136223846793005ull + 1442695040888963407ull;
    return (rng_state >> 33) % n;
}

Req random_request(int i) {
    const uint64_t Ls[] = {64, 128, 192, 256, 512};
    Req r;
    r.p = base_params(Ls[rnd(5)], 1 + (uint32_t)rnd(3));
    r.p.seed = 5 + i;
    r.p.stream = (uint32_t)i;
    r.p.sample_offset = (uint32_t)rnd(4);
    switch (i % 5) {
        case 0:  // KPZ, shifted cells of 16
            r.p.cell_log2 = 4;
            break;
        case 1:  // disorder with backward hops
            r.p.p = 0.75;
            r.p.q = 0.25;
            r.p.slow_frac = 0.3;
            r.p.slow_factor = 0.5;
            r.p.init = ASEP_INIT_BERNOULLI;
            r.p.cell_log2 = 3;
            break;
        case 2:  // two lanes, shifted
            r.p.model = ASEP_MODEL_TWO_LANE;
            r.p.init = ASEP_INIT_BERNOULLI;
            r.p.density = 0.3;
            r.p.q = 1.0;
            r.p.lane_rate = 0.5;
            r.p.turn_frac = 0.25;
            r.p.cell_log2 = 3;
            break;
        case 3:  // the sub-lattice ring
            r.p.schedule = ASEP_SCHED_SUBLATTICE;
            r.p.p = 0.75;
            r.p.q = 0.25;
            break;
        default:  // the two-lane SCA sequence
            r.p.model = ASEP_MODEL_TWO_LANE;
            r.p.schedule = ASEP_SCHED_SUBLATTICE;
            r.p.init = ASEP_INIT_BERNOULLI;
            r.p.p = 0.5;
            r.p.q = 0.5;
            r.p.lane_rate = 0.75;
            r.p.slow_frac = 0.5;
            r.p.slow_factor = 0.5;
            break;
    }
    r.t_max = 5 + rnd(30);
    for (uint64_t t = 0; t <= r.t_max; ++t)
        if (t == 0 || t == r.t_max || rnd(3) == 0) r.times.push_back(t);
    return r;
}

asep_server* make_server(FakeExecutor** fx, size_t budget, uint32_t cap, int polls,
                         uint32_t refuse, uint32_t max_active, uint32_t max_queue,
                         uint64_t quantum, uint64_t max_q = ~0ull) {
    asep_server_cfg cfg;
    memset(&cfg, 0, sizeof cfg);
    cfg.abi_version = ASEP_ABI_VERSION;
    cfg.max_active = max_active;
    cfg.max_queue = max_queue;
    cfg.quantum_mcs = quantum;
    cfg.hbm_budget_bytes = budget;
    auto x = std::unique_ptr<Executor>(new FakeExecutor(budget, cap, polls, refuse, max_q));
    *fx = static_cast<FakeExecutor*>(x.get());
    asep_server* S = nullptr;
    if (asep::serve::server_create_with(&cfg, std::move(x), &S) != ASEP_OK) return nullptr;
    return S;
}

uint64_t submit(asep_server* S, const Req& r, int* rc) {
    asep_request q;
    memset(&q, 0, sizeof q);
    q.params = r.p;
    q.t_max = r.t_max;
    q.times = r.times.data();
    q.n_times = (uint32_t)r.times.size();
    uint64_t t = 0;
    *rc = asep_submit(S, &q, &t);
    return t;
}

const uint64_t kWait = 20ull * 1000000000ull;

// Many requests of every model and schedule, small quanta, few records per
// quantum, slow completions and refused shared launches.
void scenario_mix() {
    FakeExecutor* fx;
    asep_server* S = make_server(&fx, 24 * 1024, 4, 3, 3, 6, 64, 7);
    std::vector<Req> reqs;
    std::vector<uint64_t> tickets;
    for (int i = 0; i < 30; ++i) {
        reqs.push_back(random_request(i));
        int rc;
        tickets.push_back(submit(S, reqs.back(), &rc));
        check(rc == ASEP_OK, "mix.submit", i, rc);
    }
    uint64_t packed = 0;
    for (size_t i = 0; i < reqs.size(); ++i) {
        asep_result res;
        int rc = asep_wait(S, tickets[i], kWait, &res);
        check(rc == ASEP_OK && equals_alone(reqs[i], res), "mix.equals_alone", (long)i, rc);
        check(res.quanta >= 1 && res.packed_quanta <= res.quanta, "mix.quanta", (long)res.quanta,
              (long)res.packed_quanta);
        packed += res.packed_quanta;
        check(res.t_arrive_ns <= res.t_admit_ns && res.t_admit_ns <= res.t_start_ns &&
                  res.t_start_ns <= res.t_done_ns,
              "mix.timestamps", (long)i);
        asep_result_free(&res);
    }
    check((fx->shared_launches > 0) == (packed > 0), "mix.shared_counted",
          (long)fx->shared_launches, (long)packed);

    std::vector<uint64_t> order = fx->admitted;
    check(std::is_sorted(order.begin(), order.end()), "mix.admission_in_arrival_order");
    asep_server_destroy(S);
}

// Room for one request at a time: every request still completes, in order.
void scenario_backpressure() {
    FakeExecutor* fx;
    Req r0 = random_request(3);
    r0.p.L = 512;
    r0.p.samples = 2;
    const size_t one = 2 * 512 / 8 + 4096;
    asep_server* S = make_server(&fx, one + 100, 64, 2, 0, 8, 64, 4);
    std::vector<Req> reqs;
    std::vector<uint64_t> tickets;
    for (int i = 0; i < 6; ++i) {
        Req r = r0;
        r.p.seed = 40 + i;
        reqs.push_back(r);
        int rc;
        tickets.push_back(submit(S, r, &rc));
    }
    for (size_t i = 0; i < reqs.size(); ++i) {
        asep_result res;
        int rc = asep_wait(S, tickets[i], kWait, &res);
        check(rc == ASEP_OK && equals_alone(reqs[i], res), "backpressure.equals_alone", (long)i);
        asep_result_free(&res);
    }
    check(fx->admitted == tickets, "backpressure.admission_order");
    asep_server_destroy(S);
}

// Cancel a queued and a resident request; the others are unaffected.
void scenario_cancel() {
    FakeExecutor* fx;
    asep_server* S = make_server(&fx, 1 << 20, 64, 200, 0, 1, 64, 2);
    std::vector<Req> reqs;
    std::vector<uint64_t> tickets;
    for (int i = 0; i < 5; ++i) {
        Req r = random_request(5 * i);  // all of the first model
        r.t_max = 20;
        r.times = {0, 7, 20};
        reqs.push_back(r);
        int rc;
        tickets.push_back(submit(S, r, &rc));
    }
    // the first request is resident (one slot, long quanta), the fourth queued
    while (fx->n_admitted.load() < 1) std::this_thread::sleep_for(std::chrono::microseconds(100));
    check(asep_cancel(S, tickets[3]) == ASEP_OK, "cancel.queued");
    check(asep_cancel(S, tickets[0]) == ASEP_OK, "cancel.resident");
    check(asep_cancel(S, 999999) == ASEP_E_NOTFOUND, "cancel.unknown");
    for (size_t i = 0; i < reqs.size(); ++i) {
        asep_result res;
        int rc = asep_wait(S, tickets[i], kWait, &res);
        if (i == 0 || i == 3)
            check(rc == ASEP_OK && res.status == ASEP_E_CANCELLED, "cancel.status", (long)i,
                  res.status);
        else
            check(rc == ASEP_OK && equals_alone(reqs[i], res), "cancel.others", (long)i);
        asep_result_free(&res);
    }
    asep_result res;
    check(asep_poll(S, tickets[1], &res) == ASEP_E_NOTFOUND, "cancel.collected_once");
    asep_server_destroy(S);
}

// A full queue answers BUSY; a request larger than the budget fails with
// NOMEM; invalid parameters are refused at submission.
void scenario_limits() {
    FakeExecutor* fx;
    asep_server* S = make_server(&fx, 16 * 1024, 64, 1000, 0, 1, 2, 1);
    Req big = random_request(0);
    big.p.L = 1 << 20;
    big.p.samples = 1;
    big.p.cell_log2 = 6;
    Req slow = random_request(0);
    slow.t_max = 30;
    slow.times = {30};
    int rc;
    uint64_t t_slow = submit(S, slow, &rc);
    check(rc == ASEP_OK, "limits.first");
    int busy = 0;
    std::vector<uint64_t> extra;
    for (int i = 0; i < 8; ++i) {
        uint64_t t = submit(S, slow, &rc);
        if (rc == ASEP_E_BUSY)
            ++busy;
        else if (rc == ASEP_OK)
            extra.push_back(t);
    }
    check(busy > 0, "limits.busy", busy);
    Req bad = slow;
    bad.p.p = 1.5;
    submit(S, bad, &rc);
    check(rc == ASEP_E_INVAL, "limits.invalid", rc);
    asep_result res;
    check(asep_wait(S, t_slow, kWait, &res) == ASEP_OK && equals_alone(slow, res), "limits.slow_ok");
    asep_result_free(&res);
    for (uint64_t t : extra) {
        check(asep_wait(S, t, kWait, &res) == ASEP_OK && res.status == ASEP_OK, "limits.extra_ok");
        asep_result_free(&res);
    }
    uint64_t t_big = submit(S, big, &rc);
    check(rc == ASEP_OK, "limits.big_submitted", rc);
    check(asep_wait(S, t_big, kWait, &res) == ASEP_OK && res.status == ASEP_E_NOMEM,
          "limits.nomem", res.status);
    asep_result_free(&res);
    asep_server_destroy(S);
}

// Requests of one kernel shape whose quanta end together share launches,
// and each still equals its run alone.
void scenario_packing() {
    FakeExecutor* fx;
    asep_server* S = make_server(&fx, 1 << 20, 64, 0, 0, 8, 64, 4);
    std::vector<Req> reqs;
    std::vector<uint64_t> tickets;
    for (int i = 0; i < 8; ++i) {
        Req r = random_request(0);  // the first model: shifted cells of 16
        r.p.L = 256;
        r.p.seed = 60 + i;
        r.t_max = 24;
        r.times = {0, 5, 17, 24};
        reqs.push_back(r);
        int rc;
        tickets.push_back(submit(S, r, &rc));
    }
    uint64_t packed = 0;
    for (size_t i = 0; i < reqs.size(); ++i) {
        asep_result res;
        int rc = asep_wait(S, tickets[i], kWait, &res);
        check(rc == ASEP_OK && equals_alone(reqs[i], res), "packing.equals_alone", (long)i);
        packed += res.packed_quanta;
        asep_result_free(&res);
    }
    check(fx->shared_launches > 0 && packed > 0, "packing.shared_launches",
          (long)fx->shared_launches, (long)packed);
    asep_server_destroy(S);
}

// A quantum configured far longer than the executor allows (one launch of a
// whole ring has a sub-sweep cap): every quantum the core queues is cut to
// the executor's limit, and every request still equals its run alone.
void scenario_quantum_clamp() {
    FakeExecutor* fx;
    asep_server* S = make_server(&fx, 1 << 20, 64, 1, 2, 8, 64, 1ull << 40, 3);
    std::vector<Req> reqs;
    std::vector<uint64_t> tickets;
    for (int i = 0; i < 8; ++i) {
        reqs.push_back(random_request(i));
        int rc;
        tickets.push_back(submit(S, reqs.back(), &rc));
    }
    for (size_t i = 0; i < reqs.size(); ++i) {
        asep_result res;
        int rc = asep_wait(S, tickets[i], kWait, &res);
        check(rc == ASEP_OK && equals_alone(reqs[i], res), "quantum.equals_alone", (long)i,
              res.status);
        check(res.quanta >= (reqs[i].t_max + 2) / 3, "quantum.count", (long)res.quanta);
        check(res.params.cell_log2 == (reqs[i].p.cell_log2 ? reqs[i].p.cell_log2 : 6) ||
                  reqs[i].p.schedule == ASEP_SCHED_SUBLATTICE,
              "quantum.schedule_echoed", (long)res.params.cell_log2);
        asep_result_free(&res);
    }
    check(fx->longest_quantum <= 3, "quantum.clamped", (long)fx->longest_quantum);
    asep_server_destroy(S);
}

// Several client threads submit, wait, poll and cancel at once; every
// request that was not cancelled equals its run alone.
void scenario_concurrent_clients() {
    FakeExecutor* fx;
    asep_server* S = make_server(&fx, 64 * 1024, 8, 2, 4, 6, 256, 5);
    std::atomic<int> bad{0}, good{0};
    std::vector<std::vector<Req>> drawn(4);
    for (int c = 0; c < 4; ++c)
        for (int i = 0; i < 6; ++i) drawn[c].push_back(random_request(10 * c + i));
    std::vector<std::thread> th;
    for (int c = 0; c < 4; ++c) {
        th.emplace_back([&, c] {
            std::vector<Req> reqs;
            std::vector<uint64_t> tickets;
            for (int i = 0; i < 6; ++i) {
                const Req& r = drawn[c][i];
                int rc = ASEP_E_BUSY;
                uint64_t t = 0;
                while (rc == ASEP_E_BUSY) t = submit(S, r, &rc);
                if (rc != ASEP_OK) {
                    ++bad;
                    continue;
                }
                reqs.push_back(r);
                tickets.push_back(t);
                if (i == 3) asep_cancel(S, t);
            }
            for (size_t i = 0; i < reqs.size(); ++i) {
                asep_result res;
                int rc = ASEP_E_PENDING;
                if (i % 2) {
                    while ((rc = asep_poll(S, tickets[i], &res)) == ASEP_E_PENDING)
                        std::this_thread::sleep_for(std::chrono::microseconds(200));
                } else {
                    rc = asep_wait(S, tickets[i], kWait, &res);
                }
                if (rc != ASEP_OK) {
                    ++bad;
                    continue;
                }
                if (res.status == ASEP_E_CANCELLED ? i == 3 : equals_alone(reqs[i], res))
                    ++good;
                else
                    ++bad;
                asep_result_free(&res);
            }
        });
    }
    for (auto& t : th) t.join();
    check(bad == 0 && good == 24, "concurrent.all_requests", good.load(), bad.load());
    asep_server_destroy(S);
}

}  // namespace

// The device executor and the host library's tuning table are not part of
// this program.
namespace asep {
namespace serve {
std::unique_ptr<Executor> make_device_executor(const asep_server_cfg&) { return nullptr; }
}  // namespace serve
}  // namespace asep
extern "C" int asep_tuning_load(const char*) { return ASEP_OK; }

int main() {
    scenario_mix();
    scenario_backpressure();
    scenario_cancel();
    scenario_limits();
    scenario_packing();
    scenario_quantum_clamp();
    scenario_concurrent_clients();
    printf("%s %d failures\n", failures ? "FAILED" : "PASSED", failures);
    return failures ? 1 : 0;
}
