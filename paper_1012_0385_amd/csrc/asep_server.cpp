// asep_server.cpp -- request loop with continuous batching.
//
// A request is an ensemble run (parameters, ascending measurement times,
// t_max), the unit the paper's host driver loops over (Sec. 2.1: blocks of
// independent realisations, then an outer statistics loop averaging W^2 on
// the CPU).  Requests arrive at any time.  A worker thread admits them in
// arrival order while the device arena (the configured memory budget) has
// room for their state and the resident count allows, places each on one of
// a fixed pool of streams, and advances every resident request by quanta of
// MCS: as soon as a request's previous quantum has finished (an event per
// request), its next one is queued, so requests of every size overlap on the
// GPU and a request that finishes frees its memory for the next arrival at
// once.  Every random number is keyed by the request's own (seed, stream,
// sample), and splitting a run into quanta never changes a result, so each
// request's output is the same alone or in any mix.
#include <hip/hip_runtime.h>
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
#include <tuple>
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

// First-fit allocator over one device buffer; blocks are 256-byte aligned.
class Arena {
   public:
    bool init(size_t bytes) {
        if (hipMalloc(&base_, bytes) != hipSuccess) return false;
        size_ = bytes;
        free_[0] = bytes;
        return true;
    }
    void release() {
        if (base_) (void)hipFree(base_);
        base_ = nullptr;
    }
    void* alloc(size_t bytes) {
        bytes = (bytes + 255) & ~(size_t)255;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                const size_t off = it->first;
                const size_t rest = it->second - bytes;
                free_.erase(it);
                if (rest) free_[off + bytes] = rest;
                used_[off] = bytes;
                return (char*)base_ + off;
            }
        }
        return nullptr;
    }
    void free(void* p) {
        if (!p) return;
        const size_t off = (size_t)((char*)p - (char*)base_);
        auto u = used_.find(off);
        if (u == used_.end()) return;
        size_t len = u->second;
        used_.erase(u);
        size_t start = off;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && next->first == off + len) {
            len += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == start) {
                start = prev->first;
                len += prev->second;
                free_.erase(prev);
            }
        }
        free_[start] = len;
    }
    size_t size() const { return size_; }

   private:
    void* base_ = nullptr;
    size_t size_ = 0;
    std::map<size_t, size_t> free_;  // offset -> length
    std::map<size_t, size_t> used_;
};

struct Job {
    uint64_t ticket = 0;
    asep_params params{};
    uint64_t t_max = 0;
    std::vector<uint64_t> times;
    size_t state_bytes = 0, aux_bytes = 0;
    // resident state
    asep_sim* sim = nullptr;
    void* state = nullptr;
    void* aux = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t done_ev = nullptr;
    Record* pinned_rec = nullptr;
    bool inflight = false;
    uint32_t next_time = 0;  // first measurement not yet queued
    uint32_t staged_first = 0, staged_n = 0;
    std::vector<asep_rough> rough;
    bool cancel = false;
    int status = ASEP_E_PENDING;
    uint64_t t_arrive = 0, t_admit = 0, t_start = 0, t_done = 0;
    uint64_t updates = 0;
};

const uint32_t kStreams = 8;

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
    bool stop = false;
    std::thread worker;
    // worker-owned device resources
    Arena arena;
    hipStream_t streams[kStreams] = {};
    uint32_t next_stream = 0;
    // packed launches: one descriptor buffer per stream
    SimDesc* pack_host[kStreams] = {};
    SimDesc* pack_dev[kStreams] = {};
    hipEvent_t pack_ev[kStreams] = {};
    bool pack_used[kStreams] = {};
    uint64_t packed_launches = 0;
    int init_rc = ASEP_OK;
};

namespace {

void release_job(asep_server* S, Job& j) {
    if (j.sim) {
        asep_destroy(j.sim);  // the job's work is complete (its event was reached)
        j.sim = nullptr;
    }
    S->arena.free(j.state);
    S->arena.free(j.aux);
    j.state = j.aux = nullptr;
    if (j.done_ev) (void)hipEventDestroy(j.done_ev);
    j.done_ev = nullptr;
    if (j.pinned_rec) (void)hipHostFree(j.pinned_rec);
    j.pinned_rec = nullptr;
}

// Place the job in the arena and create its simulation; ASEP_E_NOMEM means
// "not now" (no room yet).
int admit(asep_server* S, Job& j) {
    j.state = S->arena.alloc(j.state_bytes);
    j.aux = j.state ? S->arena.alloc(j.aux_bytes) : nullptr;
    if (!j.state || !j.aux) {
        S->arena.free(j.state);
        j.state = nullptr;
        return ASEP_E_NOMEM;
    }
    j.stream = S->streams[S->next_stream++ % kStreams];
    int rc = asep_create_ext(&j.params, j.state, j.state_bytes, j.aux, j.aux_bytes, j.stream,
                             &j.sim);
    if (rc == ASEP_OK &&
        hipEventCreateWithFlags(&j.done_ev, hipEventDisableTiming) != hipSuccess)
        rc = ASEP_E_DEVICE;
    if (rc == ASEP_OK &&
        hipHostMalloc((void**)&j.pinned_rec,
                      sizeof(Record) * sim_record_capacity(j.sim) * j.params.samples) !=
            hipSuccess) {
        j.pinned_rec = nullptr;
        rc = ASEP_E_NOMEM;
    }
    if (rc) {
        if (j.sim && j.stream) (void)hipStreamSynchronize(j.stream);
        release_job(S, j);
        return rc == ASEP_E_NOMEM ? ASEP_E_DEVICE : rc;
    }
    j.rough.assign(j.times.size() * (size_t)j.params.samples, asep_rough{});
    j.t_admit = now_ns();
    // the initialisation kernels are the job's first work in flight
    if (hipEventRecord(j.done_ev, j.stream) != hipSuccess) {
        (void)hipStreamSynchronize(j.stream);
        release_job(S, j);
        return ASEP_E_DEVICE;
    }
    j.inflight = true;
    return ASEP_OK;
}

// The job's next quantum: end time and number of measurements in it.
void next_quantum(asep_server* S, const Job& j, uint64_t* t_end_out, uint32_t* n_out) {
    const uint64_t t = asep_time(j.sim);
    const uint64_t q = std::max<uint64_t>(S->cfg.quantum_mcs, 1);
    uint64_t t_end = std::min(j.t_max, t + q);
    const uint32_t cap = sim_record_capacity(j.sim);
    uint32_t n = 0;
    while (j.next_time + n < j.times.size() && j.times[j.next_time + n] <= t_end && n < cap) ++n;
    if (n == cap && j.next_time + n < j.times.size() && j.times[j.next_time + n] <= t_end)
        t_end = j.times[j.next_time + n - 1];
    *t_end_out = t_end;
    *n_out = n;
}

void mark_queued(Job& j, uint64_t t0, uint64_t t_end, uint32_t n) {
    if (!j.t_start) j.t_start = now_ns();
    j.updates += (t_end - t0) * sim_attempts_per_mcs(j.sim);
    j.staged_first = j.next_time;
    j.staged_n = n;
    j.next_time += n;
    j.inflight = true;
}

// Queue the job's next quantum on its own stream and record its event.
int queue_quantum(asep_server* S, Job& j) {
    uint64_t t_end;
    uint32_t n;
    next_quantum(S, j, &t_end, &n);
    const uint64_t t0 = asep_time(j.sim);
    if (!j.t_start) j.t_start = now_ns();
    int rc = sim_run_async(j.sim, j.times.data() + j.next_time, n, t_end, j.pinned_rec);
    if (rc) return rc;
    if (hipEventRecord(j.done_ev, j.stream) != hipSuccess) return ASEP_E_DEVICE;
    mark_queued(j, t0, t_end, n);
    return ASEP_OK;
}

// Queue the next quanta of several jobs with the same kernel shape as one
// launch on a free stream of the pool.  Returns false if no stream is free.
bool queue_packed(asep_server* S, const std::vector<Job*>& group, const PackInfo& pi,
                  std::vector<int>* rcs) {
    uint32_t slot = kStreams;
    for (uint32_t k = 0; k < kStreams; ++k) {
        if (!S->pack_used[k] || hipEventQuery(S->pack_ev[k]) == hipSuccess) {
            slot = k;
            break;
        }
    }
    if (slot == kStreams) return false;
    hipStream_t st = S->streams[slot];
    SimDesc* hd = S->pack_host[slot];
    std::vector<uint64_t> t_end(group.size()), t0(group.size());
    std::vector<uint32_t> n(group.size());
    uint32_t wg = 0;
    size_t lds = 0;
    for (size_t i = 0; i < group.size(); ++i) {
        Job& j = *group[i];
        next_quantum(S, j, &t_end[i], &n[i]);
        t0[i] = asep_time(j.sim);
        (*rcs)[i] = sim_pack_prepare(j.sim, t_end[i], j.times.data() + j.next_time, n[i], &hd[i]);
        PackInfo ji;
        sim_pack_info(j.sim, &ji);
        hd[i].wg_begin = wg;
        wg += ji.grid;
        lds = std::max(lds, ji.lds);
    }
    for (int rc : *rcs)
        if (rc) return true;  // reported per job by the caller
    const uint32_t nd = (uint32_t)group.size();
    hipError_t e = hipMemcpyAsync(S->pack_dev[slot], hd, sizeof(SimDesc) * nd,
                                  hipMemcpyHostToDevice, st);
    // the launch measures if any of its simulations does
    SimDesc head = hd[0];
    head.n_rec = 0;
    for (uint32_t i = 0; i < nd; ++i) head.n_rec = std::max(head.n_rec, hd[i].n_rec);
    if (e == hipSuccess) e = launch_sweep(pi.kern, head, S->pack_dev[slot], nd, wg, pi.block, lds, st);
    for (size_t i = 0; i < group.size(); ++i) {
        Job& j = *group[i];
        int rc = (e == hipSuccess) ? ASEP_OK : device_error(e, "packed launch");
        if (rc == ASEP_OK) rc = sim_pack_commit(j.sim, t_end[i], n[i], j.pinned_rec, st);
        if (rc == ASEP_OK && hipEventRecord(j.done_ev, st) != hipSuccess) rc = ASEP_E_DEVICE;
        if (rc == ASEP_OK) mark_queued(j, t0[i], t_end[i], n[i]);
        (*rcs)[i] = rc;
    }
    (void)hipEventRecord(S->pack_ev[slot], st);
    S->pack_used[slot] = true;
    S->packed_launches += 1;
    return true;
}

void collect_quantum(Job& j) {
    const uint32_t R = sim_samples(j.sim);
    for (uint32_t i = 0; i < j.staged_n * R; ++i)
        record_to_rough(j.sim, j.pinned_rec[i], &j.rough[(size_t)j.staged_first * R + i]);
    j.staged_n = 0;
    j.inflight = false;
}

bool finished(const Job& j) {
    return asep_time(j.sim) >= j.t_max && j.next_time >= j.times.size();
}

void finish(asep_server* S, Job& j, int status) {
    j.status = status;
    j.t_done = now_ns();
    release_job(S, j);
}

void worker_main(asep_server* S) {
    if (hipSetDevice(S->cfg.device) != hipSuccess) S->init_rc = ASEP_E_DEVICE;
    for (uint32_t i = 0; i < kStreams && S->init_rc == ASEP_OK; ++i)
        if (hipStreamCreateWithFlags(&S->streams[i], hipStreamNonBlocking) != hipSuccess)
            S->init_rc = ASEP_E_DEVICE;
    if (S->init_rc == ASEP_OK && !S->arena.init(S->cfg.hbm_budget_bytes)) S->init_rc = ASEP_E_NOMEM;
    for (uint32_t i = 0; i < kStreams && S->init_rc == ASEP_OK; ++i) {
        const size_t bytes = sizeof(SimDesc) * S->cfg.max_active;
        if (hipHostMalloc((void**)&S->pack_host[i], bytes) != hipSuccess ||
            hipMalloc((void**)&S->pack_dev[i], bytes) != hipSuccess ||
            hipEventCreateWithFlags(&S->pack_ev[i], hipEventDisableTiming) != hipSuccess)
            S->init_rc = ASEP_E_NOMEM;
    }
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->cv_done.notify_all();
    }
    std::unique_lock<std::mutex> lk(S->mu);
    while (!S->stop && S->init_rc == ASEP_OK) {
        bool progressed = false;
        // admission in arrival order while slots and memory allow
        while (!S->queue.empty() && S->active.size() < S->cfg.max_active) {
            auto j = S->queue.front();
            S->queue.pop_front();
            if (j->cancel) {
                finish(S, *j, ASEP_E_CANCELLED);
                progressed = true;
                continue;
            }
            int rc = admit(S, *j);
            if (rc == ASEP_E_NOMEM) {
                if (S->active.empty()) {
                    finish(S, *j, ASEP_E_NOMEM);  // can never fit
                    progressed = true;
                    continue;
                }
                S->queue.push_front(j);  // back-pressure: wait for memory to free
                break;
            }
            if (rc) {
                finish(S, *j, rc);
                progressed = true;
                continue;
            }
            S->active.push_back(j);
            progressed = true;
        }
        // progress: every request whose quantum is done gets its next one;
        // ready requests of the same small-ring kernel shape share a launch
        std::vector<std::shared_ptr<Job>> still;
        std::vector<Job*> ready;
        for (auto& jp : S->active) {
            Job& j = *jp;
            int rc = ASEP_OK;
            if (j.inflight) {
                const hipError_t q = hipEventQuery(j.done_ev);
                if (q == hipErrorNotReady) {
                    still.push_back(jp);
                    continue;
                }
                if (q != hipSuccess) rc = device_error(q, "request event");
                if (rc == ASEP_OK) collect_quantum(j);
                progressed = true;
            }
            if (rc == ASEP_OK && j.cancel) rc = ASEP_E_CANCELLED;
            if (rc == ASEP_OK && finished(j)) {
                finish(S, j, ASEP_OK);
                continue;
            }
            if (rc) {
                (void)hipStreamSynchronize(j.stream);
                finish(S, j, rc);
                continue;
            }
            ready.push_back(&j);
            still.push_back(jp);
        }
        // group the ready jobs by kernel shape
        std::map<std::tuple<uint32_t, uint32_t, uint32_t, bool, uint32_t>, std::vector<Job*>> groups;
        std::vector<Job*> single;
        for (Job* j : ready) {
            PackInfo pi;
            if (sim_pack_info(j->sim, &pi))
                groups[std::make_tuple(pi.kern.C, pi.kern.model, pi.kern.variant, pi.kern.q0,
                                       pi.block)]
                    .push_back(j);
            else
                single.push_back(j);
        }
        std::vector<std::pair<Job*, int>> failed;
        for (auto& kv : groups) {
            auto& g = kv.second;
            if (g.size() >= 2) {
                PackInfo pi;
                sim_pack_info(g[0]->sim, &pi);
                std::vector<int> rcs(g.size(), ASEP_OK);
                if (queue_packed(S, g, pi, &rcs)) {
                    for (size_t i = 0; i < g.size(); ++i)
                        if (rcs[i]) failed.push_back({g[i], rcs[i]});
                    progressed = true;
                    continue;
                }
            }
            for (Job* j : g) single.push_back(j);
        }
        for (Job* j : single) {
            int rc = queue_quantum(S, *j);
            if (rc) failed.push_back({j, rc});
            progressed = true;
        }
        if (!failed.empty()) {
            std::vector<std::shared_ptr<Job>> keep;
            for (auto& jp : still) {
                auto it = std::find_if(failed.begin(), failed.end(),
                                       [&](const std::pair<Job*, int>& f) { return f.first == jp.get(); });
                if (it == failed.end()) {
                    keep.push_back(jp);
                    continue;
                }
                for (uint32_t k = 0; k < kStreams; ++k) (void)hipStreamSynchronize(S->streams[k]);
                finish(S, *jp, it->second);
            }
            still.swap(keep);
        }
        S->active.swap(still);
        if (progressed) S->cv_done.notify_all();
        if (S->active.empty() && S->queue.empty()) {
            S->cv_work.wait_for(lk, std::chrono::milliseconds(20));
        } else if (!progressed) {
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(50));
            lk.lock();
        }
    }
    // shutdown: wait for work in flight, release everything
    for (uint32_t i = 0; i < kStreams; ++i)
        if (S->streams[i]) (void)hipStreamSynchronize(S->streams[i]);
    for (auto& j : S->active) finish(S, *j, ASEP_E_CANCELLED);
    S->active.clear();
    for (auto& j : S->queue) finish(S, *j, S->init_rc ? S->init_rc : ASEP_E_CANCELLED);
    S->queue.clear();
    S->arena.release();
    for (uint32_t i = 0; i < kStreams; ++i) {
        if (S->pack_host[i]) (void)hipHostFree(S->pack_host[i]);
        if (S->pack_dev[i]) (void)hipFree(S->pack_dev[i]);
        if (S->pack_ev[i]) (void)hipEventDestroy(S->pack_ev[i]);
        if (S->streams[i]) (void)hipStreamDestroy(S->streams[i]);
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
    if (!S->cfg.hbm_budget_bytes) S->cfg.hbm_budget_bytes = (uint64_t)8 << 30;
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
    j->state_bytes = sb;
    j->aux_bytes = ab;
    j->t_arrive = now_ns();
    {
        std::lock_guard<std::mutex> lk(S->mu);
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
