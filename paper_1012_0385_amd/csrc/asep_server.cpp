// asep_server.cpp -- request loop with continuous batching (policy core).
//
// A request is an ensemble run (parameters, ascending measurement times,
// t_max), the unit the paper's host driver loops over (Sec. 2.1: blocks of
// independent realisations, then an outer statistics loop averaging W^2 on
// the CPU).  Requests arrive at any time.  A worker thread admits them in
// arrival order while the executor has room for their state and the
// resident count allows, and advances every resident request by quanta of
// MCS: as soon as a request's previous quantum has finished, its next one is
// queued, so requests of every size overlap on the device and a request
// that finishes frees its room for the next arrival at once.  Ready requests
// whose work can share a launch are queued together.  Every random number is
// keyed by the request's own (seed, stream, sample), and splitting a run into
// quanta never changes a result, so each request's output is the same alone
// or in any mix.
//
// This file holds the policy only and calls no HIP function: the device side
// is an Executor (asep_serve.h).
#include <time.h>

#include <algorithm>
#include <chrono>
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
#include "asep_serve.h"

using asep::serve::Executor;
using asep::serve::Job;

struct asep_server {
    asep_server_cfg cfg{};
    std::mutex mu;                    // guards queue, all, stop, ready, init_rc, Job::status
    std::condition_variable cv_work;  // worker waits for requests
    std::condition_variable cv_done;  // clients wait for results
    std::deque<std::shared_ptr<Job>> queue;        // submitted, not yet taken by the worker
    std::map<uint64_t, std::shared_ptr<Job>> all;  // every ticket not yet collected
    uint64_t next_ticket = 1;
    bool stop = false;
    bool ready = false;  // the worker finished set-up (init_rc holds its status)
    int init_rc = ASEP_OK;
    std::unique_ptr<Executor> X;
    std::thread worker;
};

namespace asep {
namespace serve {

uint64_t now_ns() {
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (uint64_t)ts.tv_sec * 1000000000ull + (uint64_t)ts.tv_nsec;
}

namespace {

// State of the worker thread only.
struct Worker {
    asep_server* S;
    Executor& X;
    std::vector<std::shared_ptr<Job>> active;  // resident jobs
    std::vector<std::shared_ptr<Job>> done;    // concluded, status not yet published

    // The job is over: free its device state (it has no work in flight) and
    // keep its outcome for publication under the lock.
    void conclude(const std::shared_ptr<Job>& j, int outcome) {
        j->t_done = now_ns();
        if (j->x) X.release(*j);
        j->inflight = false;
        j->outcome = outcome;
        done.push_back(j);
    }

    // The job's next quantum: end time and number of measurements in it.
    void next_quantum(const Job& j, uint64_t* t_end_out, uint32_t* n_out) {
        const uint64_t t = X.time(j);
        const uint64_t q = std::min<uint64_t>(std::max<uint64_t>(S->cfg.quantum_mcs, 1),
                                              std::max<uint64_t>(X.max_quantum_mcs(j), 1));
        uint64_t t_end = (j.t_max - t > q) ? t + q : j.t_max;
        const uint32_t cap = X.record_capacity(j);
        uint32_t n = 0;
        while (j.next_time + n < j.times.size() && j.times[j.next_time + n] <= t_end && n < cap)
            ++n;
        if (n == cap && j.next_time + n < j.times.size() && j.times[j.next_time + n] <= t_end)
            t_end = j.times[j.next_time + n - 1];
        *t_end_out = t_end;
        *n_out = n;
    }

    void mark_queued(Job& j, uint64_t t0, uint64_t t_end, uint32_t n, bool shared) {
        if (!j.t_start) j.t_start = now_ns();
        j.updates += (t_end - t0) * X.attempts_per_mcs(j);
        j.staged_first = j.next_time;
        j.staged_n = n;
        j.next_time += n;
        j.inflight = true;
        j.quanta += 1;
        if (shared) j.packed_quanta += 1;
    }

    // Queue one quantum of each job of the group (one launch if several);
    // false if the executor cannot take a shared launch now.
    bool queue_group(const std::vector<Job*>& g, std::vector<std::pair<Job*, int>>* failed) {
        std::vector<uint64_t> t_end(g.size()), t0(g.size());
        std::vector<uint32_t> n(g.size());
        for (size_t i = 0; i < g.size(); ++i) {
            next_quantum(*g[i], &t_end[i], &n[i]);
            t0[i] = X.time(*g[i]);
        }
        std::vector<int> rcs(g.size(), ASEP_OK);
        std::vector<char> shared(g.size(), 0);
        if (!X.queue(g, t_end, n, &rcs, &shared)) return false;
        for (size_t i = 0; i < g.size(); ++i) {
            if (rcs[i] == ASEP_OK)
                mark_queued(*g[i], t0[i], t_end[i], n[i], shared[i] != 0);
            else
                failed->push_back({g[i], rcs[i]});
        }
        return true;
    }

    bool finished(const Job& j) { return X.time(j) >= j.t_max && j.next_time >= j.times.size(); }

    // Admission of the candidates taken from the queue, in arrival order;
    // those that find no room now go back (returned in order).
    std::vector<std::shared_ptr<Job>> admit(std::vector<std::shared_ptr<Job>>& cand,
                                            bool* progressed) {
        std::vector<std::shared_ptr<Job>> back;
        for (auto& j : cand) {
            if (!back.empty()) {  // an earlier arrival is waiting for room
                back.push_back(j);
                continue;
            }
            if (j->cancel.load()) {
                conclude(j, ASEP_E_CANCELLED);
                *progressed = true;
                continue;
            }
            const int rc = X.admit(*j);
            if (rc == ASEP_E_NOMEM) {
                if (active.empty()) {  // nothing resident: it can never fit
                    conclude(j, ASEP_E_NOMEM);
                    *progressed = true;
                    continue;
                }
                back.push_back(j);  // back-pressure: wait for room
                continue;
            }
            if (rc) {
                conclude(j, rc);
                *progressed = true;
                continue;
            }
            j->rough.assign(j->times.size() * (size_t)j->params.samples, asep_rough{});
            j->t_admit = now_ns();
            j->inflight = true;  // the initialisation is the job's first work
            active.push_back(j);
            *progressed = true;
        }
        return back;
    }

    // Every resident job whose quantum is done gets its next one; jobs that
    // can share a launch go together.
    void advance(bool* progressed) {
        std::vector<std::shared_ptr<Job>> still;
        std::vector<Job*> ready;
        std::vector<std::pair<Job*, int>> failed;
        for (auto& jp : active) {
            Job& j = *jp;
            int rc = ASEP_OK;
            if (j.inflight) {
                const int q = X.query(j);
                if (q == ASEP_E_PENDING) {
                    still.push_back(jp);
                    continue;
                }
                rc = q;
                if (rc == ASEP_OK) {
                    X.collect(j);
                    j.staged_n = 0;
                    j.inflight = false;
                }
                *progressed = true;
            }
            if (rc == ASEP_OK && j.cancel.load()) rc = ASEP_E_CANCELLED;
            if (rc == ASEP_OK && finished(j)) {
                conclude(jp, ASEP_OK);
                continue;
            }
            if (rc) {
                if (j.inflight) X.wait(j);  // a failed query: let its work drain
                conclude(jp, rc);
                continue;
            }
            ready.push_back(&j);
            still.push_back(jp);
        }
        std::map<uint64_t, std::vector<Job*>> groups;
        std::vector<Job*> single;
        for (Job* j : ready) {
            uint64_t key;
            if (X.pack_key(*j, &key))
                groups[key].push_back(j);
            else
                single.push_back(j);
        }
        for (auto& kv : groups) {
            auto& g = kv.second;
            if (g.size() >= 2 && queue_group(g, &failed)) {
                *progressed = true;
                continue;
            }
            for (Job* j : g) single.push_back(j);
        }
        for (Job* j : single) {
            queue_group({j}, &failed);
            *progressed = true;
        }
        if (!failed.empty()) {
            std::vector<std::shared_ptr<Job>> keep;
            for (auto& jp : still) {
                auto it = std::find_if(failed.begin(), failed.end(),
                                       [&](const std::pair<Job*, int>& f) { return f.first == jp.get(); });
                if (it == failed.end()) {
                    keep.push_back(jp);
                } else {
                    X.wait(*jp);  // whatever part of the quantum was queued
                    conclude(jp, it->second);
                }
            }
            still.swap(keep);
        }
        active.swap(still);
    }

    // Under the lock: outcomes become visible to the clients.
    void publish() {
        for (auto& j : done) j->status = j->outcome;
        done.clear();
    }
};

void worker_main(asep_server* S) {
    Worker W{S, *S->X, {}, {}};
    const int rc0 = W.X.init();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->init_rc = rc0;
        S->ready = true;
    }
    S->cv_done.notify_all();
    if (rc0 == ASEP_OK) {
        for (;;) {
            // take the arrivals that may be admitted (under the lock)
            std::vector<std::shared_ptr<Job>> cand;
            {
                std::lock_guard<std::mutex> lk(S->mu);
                if (S->stop) break;
                while (!S->queue.empty() && W.active.size() + cand.size() < S->cfg.max_active) {
                    cand.push_back(S->queue.front());
                    S->queue.pop_front();
                }
            }
            // device work without the lock
            bool progressed = false;
            std::vector<std::shared_ptr<Job>> back = W.admit(cand, &progressed);
            W.advance(&progressed);
            // publish (under the lock), then wait for work or poll again
            std::unique_lock<std::mutex> lk(S->mu);
            for (auto it = back.rbegin(); it != back.rend(); ++it) S->queue.push_front(*it);
            const bool any_done = !W.done.empty();
            W.publish();
            if (progressed || any_done) S->cv_done.notify_all();
            if (S->stop) break;
            if (W.active.empty() && S->queue.empty()) {
                S->cv_work.wait_for(lk, std::chrono::milliseconds(20));
            } else if (!progressed) {
                lk.unlock();
                std::this_thread::sleep_for(std::chrono::microseconds(50));
            }
        }
    }
    // shutdown: wait for work in flight, release everything
    W.X.sync_all();
    for (auto& j : W.active) W.conclude(j, ASEP_E_CANCELLED);
    W.active.clear();
    std::vector<std::shared_ptr<Job>> left;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        left.assign(S->queue.begin(), S->queue.end());
        S->queue.clear();
    }
    for (auto& j : left) W.conclude(j, S->init_rc ? S->init_rc : ASEP_E_CANCELLED);
    W.X.shutdown();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        W.publish();
    }
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
    out->params = j.resolved;
    out->plan = j.plan;
    out->quanta = j.quanta;
    out->packed_quanta = j.packed_quanta;
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

int take_if_done(asep_server* S, uint64_t ticket, asep_result* out) {
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return ASEP_E_NOTFOUND;
    Job& j = *it->second;
    if (j.status == ASEP_E_PENDING) return ASEP_E_PENDING;
    int rc = fill_result(j, out);
    if (rc) return rc;
    S->all.erase(it);
    return ASEP_OK;
}

int server_create_with(const asep_server_cfg* cfg, std::unique_ptr<Executor> x,
                       asep_server** out) {
    if (!cfg || !out || !x || cfg->abi_version != ASEP_ABI_VERSION) return ASEP_E_INVAL;
    asep_server* S = new (std::nothrow) asep_server();
    if (!S) return ASEP_E_NOMEM;
    S->cfg = *cfg;
    if (!S->cfg.max_queue) S->cfg.max_queue = 1024;
    if (!S->cfg.max_active) S->cfg.max_active = 64;
    if (!S->cfg.quantum_mcs) S->cfg.quantum_mcs = 1000;
    if (!S->cfg.hbm_budget_bytes) S->cfg.hbm_budget_bytes = (uint64_t)8 << 30;
    S->X = std::move(x);
    try {
        S->worker = std::thread(worker_main, S);
    } catch (...) {
        delete S;
        return ASEP_E_NOMEM;
    }
    *out = S;
    return ASEP_OK;
}

}  // namespace serve
}  // namespace asep

using asep::serve::now_ns;

extern "C" int asep_server_create(const asep_server_cfg* cfg, asep_server** out) {
    if (!cfg || !out || cfg->abi_version != ASEP_ABI_VERSION) return ASEP_E_INVAL;
    if (cfg->tuning_path) {
        const int rc = asep_tuning_load(cfg->tuning_path);
        if (rc) return rc;
    }
    asep_server_cfg c = *cfg;
    if (!c.max_active) c.max_active = 64;
    if (!c.hbm_budget_bytes) c.hbm_budget_bytes = (uint64_t)8 << 30;
    auto x = asep::serve::make_device_executor(c);
    if (!x) return ASEP_E_NOMEM;
    return asep::serve::server_create_with(cfg, std::move(x), out);
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
    int rc = S->X->footprint(req->params, &sb, &ab);
    if (rc) return rc;
    auto j = std::make_shared<Job>();
    j->params = req->params;
    j->t_max = req->t_max;
    j->times.assign(req->times, req->times + req->n_times);
    j->state_bytes = sb;
    j->aux_bytes = ab;
    j->t_arrive = now_ns();
    {
        std::unique_lock<std::mutex> lk(S->mu);
        S->cv_done.wait(lk, [&] { return S->ready; });
        if (S->init_rc) return S->init_rc;
        if (S->queue.size() >= S->cfg.max_queue) return ASEP_E_BUSY;
        j->ticket = S->next_ticket++;
        S->queue.push_back(j);
        S->all[j->ticket] = j;
        *ticket = j->ticket;
    }
    S->cv_work.notify_all();
    return ASEP_OK;
}

extern "C" int asep_poll(asep_server* S, uint64_t ticket, asep_result* out) {
    if (!S || !out) return ASEP_E_INVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    return asep::serve::take_if_done(S, ticket, out);
}

extern "C" int asep_wait(asep_server* S, uint64_t ticket, uint64_t timeout_ns, asep_result* out) {
    if (!S || !out) return ASEP_E_INVAL;
    std::unique_lock<std::mutex> lk(S->mu);
    const auto deadline = std::chrono::steady_clock::now() + std::chrono::nanoseconds(timeout_ns);
    for (;;) {
        int rc = asep::serve::take_if_done(S, ticket, out);
        if (rc != ASEP_E_PENDING) return rc;
        if (S->cv_done.wait_until(lk, deadline) == std::cv_status::timeout) {
            rc = asep::serve::take_if_done(S, ticket, out);
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
