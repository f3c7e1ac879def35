// asep_server_hip.cpp -- the request loop's device executor.
//
// Requests live in one device arena (the configured memory budget, first
// fit), with an event marking the end of their queued work.  A quantum is one
// asynchronous run segment of the request's simulation, queued on the next
// stream of a fixed pool; several small whole-ring requests with the same
// kernel shape share one packed launch on a free pool stream (their
// descriptors in device memory).
//
// Nothing that waits on the device runs while requests come and go: pinned
// record staging and events are taken from pools that grow on demand and
// are freed only at shutdown (freeing pinned host memory waits for the whole
// device), and a finished request's arena range is simply marked free.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <memory>
#include <new>
#include <vector>

#include "../../include/asep.h"
#include "asep_internal.h"
#include "asep_serve.h"

namespace asep {
namespace serve {
namespace {

// First-fit allocator over one device buffer; blocks are 256-byte aligned.
class Arena {
   public:
    bool init(size_t bytes) {
        if (hipMalloc(&base_, bytes) != hipSuccess) {
            base_ = nullptr;
            return false;
        }
        size_ = bytes;
        free_[0] = bytes;
        return true;
    }
    void release() {
        if (base_) (void)hipFree(base_);
        base_ = nullptr;
        free_.clear();
        used_.clear();
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

   private:
    void* base_ = nullptr;
    size_t size_ = 0;
    std::map<size_t, size_t> free_;  // offset -> length
    std::map<size_t, size_t> used_;
};

// Device state of one admitted request.
struct Resident {
    asep_sim* sim = nullptr;
    void* state = nullptr;
    void* aux = nullptr;
    hipStream_t stream = nullptr;
    hipStream_t last = nullptr;  // stream of the request's latest queued work
    hipEvent_t done_ev = nullptr;
    Record* pinned_rec = nullptr;
    size_t pinned_bytes = 0;
};

// Pinned host buffers by capacity (powers of two), reused and freed only at
// shutdown.
class PinnedPool {
   public:
    Record* take(size_t bytes, size_t* cap) {
        size_t c = 4096;
        while (c < bytes) c <<= 1;
        auto it = free_.lower_bound(c);
        if (it != free_.end() && it->first == c) {
            Record* r = it->second;
            free_.erase(it);
            *cap = c;
            return r;
        }
        void* p = nullptr;
        if (hipHostMalloc(&p, c) != hipSuccess) return nullptr;
        all_.push_back(p);
        *cap = c;
        return (Record*)p;
    }
    void give(Record* r, size_t cap) {
        if (r) free_.emplace(cap, r);
    }
    void release() {
        for (void* p : all_) (void)hipHostFree(p);
        all_.clear();
        free_.clear();
    }

   private:
    std::multimap<size_t, Record*> free_;
    std::vector<void*> all_;
};

constexpr uint32_t kStreams = 16;

class DeviceExecutor final : public Executor {
   public:
    explicit DeviceExecutor(const asep_server_cfg& cfg) : cfg_(cfg) {}

    int init() override {
        if (hipSetDevice(cfg_.device) != hipSuccess) return ASEP_E_DEVICE;
        for (uint32_t i = 0; i < kStreams; ++i)
            if (hipStreamCreateWithFlags(&streams_[i], hipStreamNonBlocking) != hipSuccess)
                return ASEP_E_DEVICE;
        if (!arena_.init(cfg_.hbm_budget_bytes)) return ASEP_E_NOMEM;
        for (uint32_t i = 0; i < kStreams; ++i) {
            const size_t bytes = sizeof(SimDesc) * cfg_.max_active;
            if (hipHostMalloc((void**)&pack_host_[i], bytes) != hipSuccess ||
                hipMalloc((void**)&pack_dev_[i], bytes) != hipSuccess ||
                hipEventCreateWithFlags(&pack_ev_[i], hipEventDisableTiming) != hipSuccess)
                return ASEP_E_NOMEM;
        }
        return ASEP_OK;
    }

    void shutdown() override {
        sync_all();
        arena_.release();
        pinned_.release();
        for (hipEvent_t e : events_) (void)hipEventDestroy(e);
        events_.clear();
        for (uint32_t i = 0; i < kStreams; ++i) {
            if (pack_host_[i]) (void)hipHostFree(pack_host_[i]);
            if (pack_dev_[i]) (void)hipFree(pack_dev_[i]);
            if (pack_ev_[i]) (void)hipEventDestroy(pack_ev_[i]);
            if (streams_[i]) (void)hipStreamDestroy(streams_[i]);
            pack_host_[i] = nullptr;
            pack_dev_[i] = nullptr;
            pack_ev_[i] = nullptr;
            streams_[i] = nullptr;
        }
    }

    int footprint(const asep_params& p, size_t* state_bytes, size_t* aux_bytes) override {
        return sim_buffer_sizes_on(&p, cfg_.device, state_bytes, aux_bytes);
    }

    int admit(Job& j) override {
        auto* r = new (std::nothrow) Resident();
        if (!r) return ASEP_E_DEVICE;
        r->state = arena_.alloc(j.state_bytes);
        r->aux = r->state ? arena_.alloc(j.aux_bytes) : nullptr;
        if (!r->state || !r->aux) {
            arena_.free(r->state);
            delete r;
            return ASEP_E_NOMEM;
        }
        j.x = r;
        r->stream = streams_[next_stream_++ % kStreams];
        r->last = r->stream;
        int rc = ASEP_OK;
        r->pinned_rec = pinned_.take(sim_host_rec_bytes(j.params), &r->pinned_bytes);
        if (!r->pinned_rec) rc = ASEP_E_DEVICE;
        if (rc == ASEP_OK) {
            r->done_ev = take_event();
            if (!r->done_ev) rc = ASEP_E_DEVICE;
        }
        if (rc == ASEP_OK)
            rc = sim_create_borrowed(&j.params, r->state, j.state_bytes, r->aux, j.aux_bytes,
                                     r->stream, r->pinned_rec, &r->sim);
        // the initialisation kernels are the job's first work in flight
        if (rc == ASEP_OK && hipEventRecord(r->done_ev, r->stream) != hipSuccess)
            rc = ASEP_E_DEVICE;
        if (rc) {
            if (r->sim) (void)hipStreamSynchronize(r->stream);
            release(j);
            return rc == ASEP_E_NOMEM ? ASEP_E_DEVICE : rc;
        }
        sim_describe(r->sim, &j.resolved, &j.plan);
        return ASEP_OK;
    }

    void release(Job& j) override {
        auto* r = res(j);
        if (!r) return;
        // the job has no work in flight; its simulation borrows stream,
        // buffers and staging, so destroying it waits for nothing
        if (r->sim) asep_destroy(r->sim);
        arena_.free(r->state);
        arena_.free(r->aux);
        if (r->done_ev) events_free_.push_back(r->done_ev);
        pinned_.give(r->pinned_rec, r->pinned_bytes);
        delete r;
        j.x = nullptr;
    }

    void wait(Job& j) override {
        Resident* r = res(j);
        if (r && r->last) (void)hipStreamSynchronize(r->last);
    }

    uint64_t time(const Job& j) override { return asep_time(res(j)->sim); }
    uint32_t record_capacity(const Job& j) override { return sim_record_capacity(res(j)->sim); }
    uint64_t max_quantum_mcs(const Job& j) override { return sim_max_quantum_mcs(res(j)->sim); }
    uint64_t attempts_per_mcs(const Job& j) override { return sim_attempts_per_mcs(res(j)->sim); }

    int query(Job& j) override {
        const hipError_t q = hipEventQuery(res(j)->done_ev);
        if (q == hipErrorNotReady) return ASEP_E_PENDING;
        if (q != hipSuccess) return device_error(q, "request event");
        return ASEP_OK;
    }

    void collect(Job& j) override {
        Resident* r = res(j);
        const uint32_t R = sim_samples(r->sim);
        for (uint32_t i = 0; i < j.staged_n * R; ++i)
            record_to_rough(r->sim, r->pinned_rec[i], &j.rough[(size_t)j.staged_first * R + i]);
    }

    bool pack_key(const Job& j, uint64_t* key) override {
        PackInfo pi;
        if (!sim_pack_info(res(j)->sim, &pi)) return false;
        *key = (uint64_t)pi.kern.C | ((uint64_t)pi.kern.model << 8) |
               ((uint64_t)pi.kern.variant << 16) | ((uint64_t)(pi.kern.q0 ? 1 : 0) << 24) |
               ((uint64_t)pi.block << 32);
        return true;
    }

    bool queue(const std::vector<Job*>& g, const std::vector<uint64_t>& t_end,
               const std::vector<uint32_t>& n, std::vector<int>* rcs,
               std::vector<char>* shared) override {
        if (g.size() == 1) {
            (*rcs)[0] = queue_alone(*g[0], t_end[0], n[0]);
            (*shared)[0] = 0;
            return true;
        }
        return queue_packed(g, t_end, n, rcs, shared);
    }

    void sync_all() override {
        for (uint32_t i = 0; i < kStreams; ++i)
            if (streams_[i]) (void)hipStreamSynchronize(streams_[i]);
    }

   private:
    static Resident* res(const Job& j) { return static_cast<Resident*>(j.x); }

    hipEvent_t take_event() {
        if (!events_free_.empty()) {
            hipEvent_t e = events_free_.back();
            events_free_.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
        events_.push_back(e);
        return e;
    }

    // One quantum of one job (cut into as many launches as the run needs).
    // Quanta take the pool's streams in turn: a job's previous quantum is
    // complete when its next is queued, so it may run on any stream, and
    // turning the streams over spreads long jobs across the hardware queues
    // the streams map to (pinned to one stream, a few long jobs that shared
    // a queue ran one after another while other queues idled).
    int queue_alone(Job& j, uint64_t t_end, uint32_t n) {
        Resident* r = res(j);
        r->stream = streams_[next_stream_++ % kStreams];
        sim_set_stream(r->sim, r->stream);
        r->last = r->stream;
        int rc = sim_run_async(r->sim, j.times.data() + j.next_time, n, t_end, r->pinned_rec);
        if (rc == ASEP_OK && hipEventRecord(r->done_ev, r->stream) != hipSuccess)
            rc = ASEP_E_DEVICE;
        return rc;
    }

    // Several jobs of one kernel shape as one launch on a free pool stream.
    bool queue_packed(const std::vector<Job*>& g, const std::vector<uint64_t>& t_end,
                      const std::vector<uint32_t>& n, std::vector<int>* rcs,
                      std::vector<char>* shared) {
        uint32_t slot = kStreams;
        for (uint32_t k = 0; k < kStreams; ++k) {
            if (!pack_used_[k] || hipEventQuery(pack_ev_[k]) == hipSuccess) {
                slot = k;
                break;
            }
        }
        if (slot == kStreams) return false;
        hipStream_t st = streams_[slot];
        SimDesc* hd = pack_host_[slot];
        PackInfo pi;
        sim_pack_info(res(*g[0])->sim, &pi);
        uint32_t wg = 0;
        size_t lds = 0;
        bool ok = true;
        for (size_t i = 0; i < g.size(); ++i) {
            Job& j = *g[i];
            (*rcs)[i] = sim_pack_prepare(res(j)->sim, t_end[i], j.times.data() + j.next_time,
                                         n[i], &hd[i]);
            if ((*rcs)[i]) ok = false;
            PackInfo ji;
            sim_pack_info(res(j)->sim, &ji);
            hd[i].wg_begin = wg;
            wg += ji.grid;
            lds = std::max(lds, ji.lds);
        }
        if (!ok) {
            // nothing was queued: every job of the group runs its quantum
            // alone (a run too long for one launch is cut there)
            for (size_t i = 0; i < g.size(); ++i) {
                (*rcs)[i] = queue_alone(*g[i], t_end[i], n[i]);
                (*shared)[i] = 0;
            }
            return true;
        }
        const uint32_t nd = (uint32_t)g.size();
        hipError_t e = hipMemcpyAsync(pack_dev_[slot], hd, sizeof(SimDesc) * nd,
                                      hipMemcpyHostToDevice, st);
        // the launch measures if any of its simulations does
        SimDesc head = hd[0];
        head.n_rec = 0;
        for (uint32_t i = 0; i < nd; ++i) head.n_rec = std::max(head.n_rec, hd[i].n_rec);
        if (e == hipSuccess)
            e = launch_sweep(pi.kern, head, pack_dev_[slot], nd, wg, pi.block, lds, st);
        for (size_t i = 0; i < g.size(); ++i) {
            Job& j = *g[i];
            Resident* r = res(j);
            r->last = st;
            int rc = (e == hipSuccess) ? ASEP_OK : device_error(e, "packed launch");
            if (rc == ASEP_OK) rc = sim_pack_commit(r->sim, t_end[i], n[i], r->pinned_rec, st);
            if (rc == ASEP_OK && hipEventRecord(r->done_ev, st) != hipSuccess) rc = ASEP_E_DEVICE;
            (*rcs)[i] = rc;
            (*shared)[i] = 1;
        }
        (void)hipEventRecord(pack_ev_[slot], st);
        pack_used_[slot] = true;
        return true;
    }

    asep_server_cfg cfg_;
    Arena arena_;
    hipStream_t streams_[kStreams] = {};
    uint32_t next_stream_ = 0;
    SimDesc* pack_host_[kStreams] = {};
    SimDesc* pack_dev_[kStreams] = {};
    hipEvent_t pack_ev_[kStreams] = {};
    bool pack_used_[kStreams] = {};
    PinnedPool pinned_;
    std::vector<hipEvent_t> events_;       // every event created
    std::vector<hipEvent_t> events_free_;  // of those, the ones not in use
};

}  // namespace

std::unique_ptr<Executor> make_device_executor(const asep_server_cfg& cfg) {
    return std::unique_ptr<Executor>(new (std::nothrow) DeviceExecutor(cfg));
}

}  // namespace serve
}  // namespace asep
