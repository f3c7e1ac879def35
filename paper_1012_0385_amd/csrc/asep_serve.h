// asep_serve.h -- the request loop's policy core and its device interface.
//
// The core (asep_server.cpp) owns the queues, admission order, quanta,
// grouping of requests that may share a launch, cancellation and results;
// it calls no HIP function.  Everything that touches a device goes through
// an Executor: the library's executor (asep_server_hip.cpp) places requests
// in a device arena and runs them on a stream pool; a test executor can run
// them on the CPU, so the same policy code is exercised without a GPU.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <atomic>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/asep.h"

namespace asep {
namespace serve {

uint64_t now_ns();

// One request as the core sees it.  Fields are written by the submitting
// thread before the job is queued, then only by the worker thread, except
// `cancel` (any thread) and `status` (under the server's lock: a job whose
// status is no longer ASEP_E_PENDING is never touched by the worker again).
struct Job {
    uint64_t ticket = 0;
    asep_params params{};
    uint64_t t_max = 0;
    std::vector<uint64_t> times;  // ascending measurement times
    size_t state_bytes = 0, aux_bytes = 0;
    void* x = nullptr;            // executor state while admitted
    bool inflight = false;        // a quantum is queued and not yet collected
    uint32_t next_time = 0;       // first measurement not yet queued
    uint32_t staged_first = 0;    // measurements of the quantum in flight
    uint32_t staged_n = 0;
    std::vector<asep_rough> rough;  // [times][samples]
    std::atomic<bool> cancel{false};
    int status = ASEP_E_PENDING;   // under the server's lock
    int outcome = ASEP_E_PENDING;  // the worker's verdict, published as status
    uint64_t t_arrive = 0, t_admit = 0, t_start = 0, t_done = 0;
    uint64_t updates = 0;
    uint32_t quanta = 0, packed_quanta = 0;
    asep_params resolved{};        // parameters as the executor resolved them
    asep_plan plan{};              // and the launch plan of the rings
};

// Device side of the loop.  Every call except footprint() comes from the
// worker thread, which holds no lock of the server while it makes them;
// footprint() may come from any thread.
class Executor {
   public:
    virtual ~Executor() = default;
    // Device set-up and tear-down (the worker's first and last calls).
    virtual int init() = 0;
    virtual void shutdown() = 0;
    // Validate a request and size its resident state.
    virtual int footprint(const asep_params& p, size_t* state_bytes, size_t* aux_bytes) = 0;
    // Make the job resident and start its initialisation (j.inflight is set
    // by the core); ASEP_E_NOMEM means "no room now".  Fills j.resolved and
    // j.plan.
    virtual int admit(Job& j) = 0;
    // Free what admit took; the job has no work in flight.  Must not wait
    // for other jobs' work.
    virtual void release(Job& j) = 0;
    // Wait until the job's queued work has finished (after a failure).
    virtual void wait(Job& j) = 0;
    // MCS the job has been queued up to.
    virtual uint64_t time(const Job& j) = 0;
    // Measurements one quantum can hold.
    virtual uint32_t record_capacity(const Job& j) = 0;
    // Longest quantum (MCS) the job may be given.
    virtual uint64_t max_quantum_mcs(const Job& j) = 0;
    virtual uint64_t attempts_per_mcs(const Job& j) = 0;
    // ASEP_OK once the job's queued work has finished, ASEP_E_PENDING while
    // it runs, or an error.
    virtual int query(Job& j) = 0;
    // Copy the finished quantum's measurements to j.rough at staged_first.
    virtual void collect(Job& j) = 0;
    // Jobs with equal keys may share one launch.
    virtual bool pack_key(const Job& j, uint64_t* key) = 0;
    // Queue one quantum per job of the group (up to t_end[i], measuring
    // n[i] times from next_time), as one launch when the group has several
    // jobs.  Returns false, queueing nothing, if a shared launch cannot be
    // taken now (the core then queues the jobs one by one); a single job
    // always returns true.  rcs[i] is each job's status, shared[i] whether
    // its quantum went into a launch shared with other jobs.
    virtual bool queue(const std::vector<Job*>& group, const std::vector<uint64_t>& t_end,
                       const std::vector<uint32_t>& n, std::vector<int>* rcs,
                       std::vector<char>* shared) = 0;
    // Wait for all queued work (shutdown).
    virtual void sync_all() = 0;
};

// The executor the public asep_server_create uses (device arena, streams).
std::unique_ptr<Executor> make_device_executor(const asep_server_cfg& cfg);

// A server driving the given executor (asep_server_create with the device
// executor; tests pass their own).
int server_create_with(const asep_server_cfg* cfg, std::unique_ptr<Executor> x,
                       asep_server** out);

}  // namespace serve
}  // namespace asep
