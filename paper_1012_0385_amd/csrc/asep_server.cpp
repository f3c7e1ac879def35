// asep_server.cpp -- request loop with continuous batching.
//
// A request is an ensemble run (parameters, ascending measurement times,
// t_max), the unit the paper's host driver loops over (Sec. 2.1: blocks of
// independent realisations, then an outer statistics loop averaging W^2 on
// the CPU).  Here requests arrive at any time: a worker thread admits them
// while device memory (the configured budget) and resident slots allow, gives
// each its own simulation and stream, and advances every resident request by
// one quantum of MCS per round, all rounds' launches queued before the worker
// waits on any of them, so the work of different requests overlaps on the
// GPU.  A request that finishes frees its memory at once and the next
// arrival is admitted in the same round.  Every random number is keyed by the
// request's own (seed, stream, sample), and chunking never changes a result,
// so each request's output is the same alone or in any mix.
#include <hip/hip_runtime.h>
#include <time.h>

#include <algorithm>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "../../include/asep.h"
#include "asep_internal.h"

using namespace asep;

namespace {

uint64_t now_ns() {
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (uint64_t)ts.tv_sec * 1000000000ull + (uint64_t)ts.tv_nsec;
}

struct Job {
    uint64_t ticket = 0;
    asep_params params{};
    uint64_t t_max = 0;
    std::vector<uint64_t> times;
    size_t footprint = 0;
    // progress
    asep_sim* sim = nullptr;
    uint32_t next_time = 0;  // first measurement not yet queued
    std::vector<asep_rough> rough;
    uint64_t* pinned_times = nullptr;  // host-pinned copy of times
    Record* pinned_rec = nullptr;      // host-pinned record staging for one round
    uint32_t staged_first = 0, staged_n = 0;
    bool cancel = false;
    int status = ASEP_E_PENDING;
    uint64_t t_arrive = 0, t_admit = 0, t_start = 0, t_done = 0;
    uint64_t updates = 0;
};

}  // namespace

struct asep_server {
    asep_server_cfg cfg{};
    std::mutex mu;
    std::condition_variable cv_work;  // worker waits for requests
    std::condition_variable cv_done;  // clients wait for results
    std::deque<std::shared_ptr<Job>> queue;
    std::vector<std::shared_ptr<Job>> active;
    std::map<uint64_t, std::shared_ptr<Job>> all;  // every ticket not yet collected
    uint64_t next_ticket = 1;
    size_t in_use = 0;
    bool stop = false;
    std::thread worker;
};

namespace {

void free_job_device(Job& j) {
    if (j.sim) {
        asep_destroy(j.sim);
        j.sim = nullptr;
    }
    if (j.pinned_times) (void)hipHostFree(j.pinned_times);
    if (j.pinned_rec) (void)hipHostFree(j.pinned_rec);
    j.pinned_times = nullptr;
    j.pinned_rec = nullptr;
}

// Create the job's simulation; ASEP_E_NOMEM leaves it queued.
int admit(asep_server* S, Job& j) {
    int rc = asep_create(&j.params, &j.sim);
    if (rc) return rc;
    const uint32_t cap = sim_record_capacity(j.sim);
    const uint32_t R = sim_samples(j.sim);
    if (hipHostMalloc((void**)&j.pinned_times, 8 * std::max<size_t>(j.times.size(), 1)) !=
            hipSuccess ||
        hipHostMalloc((void**)&j.pinned_rec, sizeof(Record) * (size_t)cap * R) != hipSuccess) {
        free_job_device(j);
        return ASEP_E_NOMEM;
    }
    if (!j.times.empty()) std::memcpy(j.pinned_times, j.times.data(), 8 * j.times.size());
    j.rough.assign(j.times.size() * (size_t)R, asep_rough{});
    j.t_admit = now_ns();
    (void)S;
    return ASEP_OK;
}

// Queue one round of work for a job; returns an error code or ASEP_OK.
int queue_round(asep_server* S, Job& j) {
    const uint64_t t = asep_time(j.sim);
    const uint64_t q = std::max<uint64_t>(S->cfg.quantum_mcs, 1);
    uint64_t t_end = std::min(j.t_max, t + q);
    const uint32_t cap = sim_record_capacity(j.sim);
    // measurements due in [t, t_end], at most one launch's worth per round
    uint32_t n = 0;
    while (j.next_time + n < j.times.size() && j.times[j.next_time + n] <= t_end && n < cap) ++n;
    if (n == cap && j.next_time + n < j.times.size() && j.times[j.next_time + n] <= t_end)
        t_end = j.times[j.next_time + n - 1];
    if (!j.t_start) j.t_start = now_ns();
    int rc = sim_run_async(j.sim, j.pinned_times + j.next_time, n, t_end, j.pinned_rec);
    if (rc) return rc;
    j.updates += (t_end - t) * sim_attempts_per_mcs(j.sim);
    j.staged_first = j.next_time;
    j.staged_n = n;
    j.next_time += n;
    return ASEP_OK;
}

void collect_round(Job& j) {
    const uint32_t R = sim_samples(j.sim);
    for (uint32_t i = 0; i < j.staged_n * R; ++i)
        record_to_rough(j.sim, j.pinned_rec[i], &j.rough[(size_t)j.staged_first * R + i]);
    j.staged_n = 0;
}

void finish(asep_server* S, Job& j, int status) {
    j.status = status;
    j.t_done = now_ns();
    free_job_device(j);
    S->in_use -= std::min(S->in_use, j.footprint);
}

void worker_main(asep_server* S) {
    (void)hipSetDevice(S->cfg.device);
    std::unique_lock<std::mutex> lk(S->mu);
    while (!S->stop) {
        // admission: FIFO while slots and the memory budget allow
        while (!S->queue.empty() && S->active.size() < S->cfg.max_active) {
            auto j = S->queue.front();
            if (j->cancel) {
                S->queue.pop_front();
                finish(S, *j, ASEP_E_CANCELLED);
                S->cv_done.notify_all();
                continue;
            }
            if (S->in_use + j->footprint > S->cfg.hbm_budget_bytes && !S->active.empty()) break;
            S->queue.pop_front();
            S->in_use += j->footprint;
            lk.unlock();
            int rc = admit(S, *j);
            lk.lock();
            if (rc == ASEP_E_NOMEM && !S->active.empty()) {
                S->in_use -= j->footprint;
                S->queue.push_front(j);  // back-pressure: retry when memory frees
                break;
            }
            if (rc) {
                finish(S, *j, rc);
                S->cv_done.notify_all();
                continue;
            }
            S->active.push_back(j);
        }
        if (S->active.empty()) {
            S->cv_work.wait_for(lk, std::chrono::milliseconds(50));
            continue;
        }
        // one round: queue every active job's quantum, then wait for all
        std::vector<std::shared_ptr<Job>> round = S->active;
        lk.unlock();
        std::vector<int> rcs(round.size(), ASEP_OK);
        for (size_t i = 0; i < round.size(); ++i)
            if (!round[i]->cancel) rcs[i] = queue_round(S, *round[i]);
        for (size_t i = 0; i < round.size(); ++i) {
            hipError_t e = hipStreamSynchronize(sim_stream(round[i]->sim));
            if (e != hipSuccess && rcs[i] == ASEP_OK) rcs[i] = device_error(e, "round");
            if (rcs[i] == ASEP_OK) collect_round(*round[i]);
        }
        lk.lock();
        std::vector<std::shared_ptr<Job>> still;
        for (size_t i = 0; i < round.size(); ++i) {
            Job& j = *round[i];
            if (j.cancel)
                finish(S, j, ASEP_E_CANCELLED);
            else if (rcs[i] != ASEP_OK)
                finish(S, j, rcs[i]);
            else if (asep_time(j.sim) >= j.t_max && j.next_time >= j.times.size())
                finish(S, j, ASEP_OK);
            else
                still.push_back(round[i]);
        }
        S->active.swap(still);
        S->cv_done.notify_all();
    }
    // shutdown: release everything still held
    for (auto& j : S->active) finish(S, *j, ASEP_E_CANCELLED);
    S->active.clear();
    for (auto& j : S->queue) finish(S, *j, ASEP_E_CANCELLED);
    S->queue.clear();
    S->cv_done.notify_all();
}

int fill_result(const Job& j, asep_result* out) {
    std::memset(out, 0, sizeof *out);
    out->status = j.status;
    out->samples = j.params.samples;
    out->n_times = (uint32_t)j.times.size();
    out->t_arrive_ns = j.t_arrive;
    out->t_admit_ns = j.t_admit;
    out->t_start_ns = j.t_start;
    out->t_done_ns = j.t_done;
    out->site_updates = j.updates;
    if (j.status == ASEP_OK && !j.times.empty()) {
        out->times = (uint64_t*)std::malloc(8 * j.times.size());
        out->rough = (asep_rough*)std::malloc(sizeof(asep_rough) * j.rough.size());
        if (!out->times || !out->rough) {
            std::free(out->times);
            std::free(out->rough);
            out->times = nullptr;
            out->rough = nullptr;
            return ASEP_E_NOMEM;
        }
        std::memcpy(out->times, j.times.data(), 8 * j.times.size());
        std::memcpy(out->rough, j.rough.data(), sizeof(asep_rough) * j.rough.size());
    }
    return ASEP_OK;
}

}  // namespace

extern "C" int asep_server_create(const asep_server_cfg* cfg, asep_server** out) {
    if (!cfg || !out || cfg->abi_version != ASEP_ABI_VERSION) return ASEP_E_INVAL;
    asep_server* S = new (std::nothrow) asep_server();
    if (!S) return ASEP_E_NOMEM;
    S->cfg = *cfg;
    if (!S->cfg.max_queue) S->cfg.max_queue = 1024;
    if (!S->cfg.max_active) S->cfg.max_active = 64;
    if (!S->cfg.quantum_mcs) S->cfg.quantum_mcs = 1000;
    if (!S->cfg.hbm_budget_bytes) S->cfg.hbm_budget_bytes = (uint64_t)64 << 30;
    try {
        S->worker = std::thread(worker_main, S);
    } catch (...) {
        delete S;
        return ASEP_E_NOMEM;
    }
    *out = S;
    return ASEP_OK;
}

extern "C" void asep_server_destroy(asep_server* S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    if (S->worker.joinable()) S->worker.join();
    delete S;
}

extern "C" int asep_submit(asep_server* S, const asep_request* req, uint64_t* ticket) {
    if (!S || !req || !ticket) return ASEP_E_INVAL;
    if (req->n_times && !req->times) return ASEP_E_INVAL;
    for (uint32_t i = 0; i < req->n_times; ++i)
        if (req->times[i] > req->t_max || (i && req->times[i] < req->times[i - 1]))
            return ASEP_E_INVAL;
    size_t sb = 0, ab = 0;
    int rc = asep_buffer_sizes(&req->params, &sb, &ab);
    if (rc) return rc;
    auto j = std::make_shared<Job>();
    j->params = req->params;
    j->t_max = req->t_max;
    j->times.assign(req->times, req->times + req->n_times);
    j->footprint = sb + ab;
    j->t_arrive = now_ns();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->queue.size() >= S->cfg.max_queue) return ASEP_E_BUSY;
        j->ticket = S->next_ticket++;
        S->queue.push_back(j);
        S->all[j->ticket] = j;
        *ticket = j->ticket;
    }
    S->cv_work.notify_all();
    return ASEP_OK;
}

static int take_if_done(asep_server* S, uint64_t ticket, asep_result* out) {
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return ASEP_E_NOTFOUND;
    Job& j = *it->second;
    if (j.status == ASEP_E_PENDING) return ASEP_E_PENDING;
    int rc = fill_result(j, out);
    if (rc) return rc;
    S->all.erase(it);
    return ASEP_OK;
}

extern "C" int asep_poll(asep_server* S, uint64_t ticket, asep_result* out) {
    if (!S || !out) return ASEP_E_INVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    return take_if_done(S, ticket, out);
}

extern "C" int asep_wait(asep_server* S, uint64_t ticket, uint64_t timeout_ns, asep_result* out) {
    if (!S || !out) return ASEP_E_INVAL;
    std::unique_lock<std::mutex> lk(S->mu);
    const auto deadline = std::chrono::steady_clock::now() + std::chrono::nanoseconds(timeout_ns);
    for (;;) {
        int rc = take_if_done(S, ticket, out);
        if (rc != ASEP_E_PENDING) return rc;
        if (S->cv_done.wait_until(lk, deadline) == std::cv_status::timeout) {
            rc = take_if_done(S, ticket, out);
            return rc == ASEP_E_PENDING ? ASEP_E_TIMEOUT : rc;
        }
    }
}

extern "C" int asep_cancel(asep_server* S, uint64_t ticket) {
    if (!S) return ASEP_E_INVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return ASEP_E_NOTFOUND;
    Job& j = *it->second;
    if (j.status != ASEP_E_PENDING) return ASEP_OK;  // already finished
    j.cancel = true;
    auto q = std::find(S->queue.begin(), S->queue.end(), it->second);
    if (q != S->queue.end()) {
        S->queue.erase(q);
        j.status = ASEP_E_CANCELLED;
        j.t_done = now_ns();
        S->cv_done.notify_all();
    }
    S->cv_work.notify_all();
    return ASEP_OK;
}

extern "C" void asep_result_free(asep_result* r) {
    if (!r) return;
    std::free(r->times);
    std::free(r->rough);
    r->times = nullptr;
    r->rough = nullptr;
}
