// asep_host.cpp -- host side of the C ABI declared in include/asep.h:
// parameter validation, probability -> threshold lowering, device buffers,
// launch shapes, and the conversions of exact integer sums to W^2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/asep.h"
#include "asep_internal.h"

using namespace asep;

namespace {

thread_local std::string g_last_device_error;

int device_fail(hipError_t e, const char* where) {
    char buf[256];
    std::snprintf(buf, sizeof buf, "%s: %s (%d)", where, hipGetErrorString(e), (int)e);
    g_last_device_error = buf;
    return ASEP_E_DEVICE;
}

#define HIP_OR_FAIL(expr)                                      \
    do {                                                       \
        hipError_t _e = (expr);                                \
        if (_e != hipSuccess) return device_fail(_e, #expr);   \
    } while (0)

// Threshold at `bits` bits for probability x (Sec. 2.1: an exchange happens
// "with probability p"): min(2^bits, floor(x 2^bits)), exact in binary64.
uint64_t lower_prob(double x, int bits) {
    const double cap = std::ldexp(1.0, bits);
    const double v = std::floor(std::ldexp(x, bits));
    if (v >= cap) return uint64_t(1) << bits;
    if (v <= 0.0) return 0;
    return (uint64_t)v;
}

bool in01(double x) { return x >= 0.0 && x <= 1.0; }

}  // namespace

// Resolved parameters plus the lowered schedule.
struct Resolved {
    asep_params P;
    Sched sc;
    uint32_t planes;      // state planes per ring
    uint32_t mplanes;     // quenched planes per realisation
    uint32_t mtags[2];
    uint64_t T_mask;      // 32-bit threshold of the quenched planes
    uint32_t nw;          // words per plane
    uint32_t n_real;      // realisations held
    uint32_t real0;       // first realisation
    uint32_t spd;
    uint32_t model;       // kernel model
};

static int resolve(const asep_params* in, Resolved* r) {
    if (!in) return ASEP_E_INVAL;
    if (in->abi_version != ASEP_ABI_VERSION) return ASEP_E_INVAL;
    asep_params P = *in;
    if (P.cell_log2 == 0) P.cell_log2 = 6;
    if (P.subsweeps == 0) P.subsweeps = 4;
    if (P.samples_per_disorder == 0) P.samples_per_disorder = 1;
    if (P.model != ASEP_MODEL_RING && P.model != ASEP_MODEL_TWO_LANE) return ASEP_E_INVAL;
    if (P.init != ASEP_INIT_FLAT && P.init != ASEP_INIT_BERNOULLI) return ASEP_E_INVAL;
    if (P.samples == 0) return ASEP_E_INVAL;
    if (!in01(P.p) || !in01(P.q) || !in01(P.density) || !in01(P.slow_frac) ||
        !in01(P.slow_factor) || !in01(P.lane_rate) || !in01(P.turn_frac))
        return ASEP_E_INVAL;
    if (P.cell_log2 < 1 || P.cell_log2 > 6) return ASEP_E_INVAL;
    const uint64_t ell = uint64_t(1) << P.cell_log2;
    if (P.L == 0 || P.L % 64 != 0 || P.L % ell != 0 || P.L / ell < 2) return ASEP_E_INVAL;
    if (P.L / 64 > 0xFFFFFFFFull / 64) return ASEP_E_UNSUPPORTED;
    const bool two = P.model == ASEP_MODEL_TWO_LANE;
    const uint32_t per_mcs = (uint32_t)(two ? 4 * ell : ell);
    if (P.subsweeps < 1 || per_mcs % (uint32_t)P.subsweeps != 0) return ASEP_E_INVAL;
    if (two && P.slow_frac > 0) return ASEP_E_UNSUPPORTED;
    if ((uint64_t)P.sample_offset + P.samples > 0x100000000ull) return ASEP_E_INVAL;

    Sched sc{};
    sc.lam = (uint32_t)P.cell_log2;
    sc.S = (uint32_t)P.subsweeps;
    sc.a = per_mcs / sc.S;
    const int ebits = two ? 2 : 0;
    const int B = 32 - (int)sc.lam - ebits;
    uint64_t TB[4] = {0, 0, 0, 0};
    std::vector<uint64_t> used;
    if (!two) {
        TB[0] = lower_prob(P.p, B);
        TB[1] = lower_prob(P.q, B);
        TB[2] = lower_prob(P.slow_factor * P.p, B);
        TB[3] = lower_prob(P.slow_factor * P.q, B);
        used = {TB[0], TB[1]};
        if (P.slow_frac > 0) {
            used.push_back(TB[2]);
            used.push_back(TB[3]);
        }
    } else {
        TB[0] = lower_prob(P.p, B);
        TB[1] = lower_prob(P.q, B);
        TB[2] = lower_prob(P.lane_rate, B);
        used = {TB[0], TB[1], TB[2]};
    }
    auto exact_at = [&](int b) {
        const uint64_t unit = uint64_t(1) << (B - b);
        for (uint64_t t : used)
            if (t % unit != 0) return false;
        return true;
    };
    int b;
    if (P.rbits < 0) {
        for (b = 0; b < B && !exact_at(b); ++b) {
        }
    } else {
        b = P.rbits;
        if (b > B || !exact_at(b)) return ASEP_E_INVAL;
    }
    P.rbits = b;
    sc.b = (uint32_t)b;
    for (int i = 0; i < 4; ++i) sc.T[i] = (uint32_t)(TB[i] >> (B - b));
    sc.w = sc.lam + (uint32_t)ebits + sc.b;
    sc.A = 32 / sc.w;
    sc.nblk = (sc.a + 4 * sc.A - 1) / (4 * sc.A);
    sc.T_init = lower_prob(P.density, 32);
    sc.T_slow = lower_prob(P.slow_frac, 32);
    sc.T_turn = lower_prob(P.turn_frac, 32);

    r->P = P;
    r->sc = sc;
    r->planes = two ? 2 : 1;
    r->nw = (uint32_t)(P.L / 64);
    r->spd = P.samples_per_disorder;
    if (two) {
        r->model = kTwoLane;
        r->mplanes = 1;
        r->mtags[0] = r->mtags[1] = kTagTurn;
        r->T_mask = sc.T_turn;
    } else if (P.slow_frac > 0) {
        r->model = kDisorder;
        r->mplanes = P.q > 0 ? 2 : 1;
        r->mtags[0] = kTagDisP;
        r->mtags[1] = kTagDisQ;
        r->T_mask = sc.T_slow;
    } else {
        r->model = kPlain;
        r->mplanes = 0;
        r->mtags[0] = r->mtags[1] = 0;
        r->T_mask = 0;
    }
    if (r->mplanes) {
        r->real0 = P.sample_offset / r->spd;
        const uint32_t last = (P.sample_offset + P.samples - 1) / r->spd;
        r->n_real = last - r->real0 + 1;
    } else {
        r->real0 = 0;
        r->n_real = 0;
    }
    return ASEP_OK;
}

struct Shape {
    uint32_t C, lanes_per_ring, rings_per_wg, block, grid;
    size_t lds;
};

static size_t lds_limit() {
    static size_t lim = 0;
    if (!lim) {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
            lim = prop.sharedMemPerBlock;
        if (!lim) lim = 65536;
    }
    return lim;
}

// Launch shape of the register-resident ring kernel.
static int choose_shape(const Resolved& r, Shape* s) {
    const uint32_t nw = r.nw;
    const uint32_t R = r.P.samples;
    static const uint32_t Cs[] = {1, 2, 4, 8, 16};
    for (uint32_t C : Cs) {
        const uint32_t lim = ring_block_limit(C);
        const uint32_t Tr = (nw + C - 1) / C;
        if (Tr > lim) continue;
        // small rings: pack several per workgroup, up to 256 lanes
        uint32_t G = 1;
        if (Tr < 256) G = std::max(1u, std::min(256u / Tr, R));
        const uint32_t lanes = G * Tr;
        const uint32_t block = std::min(lim, (lanes + 63) / 64 * 64);
        if (block < lanes) continue;
        const size_t lds = ring_lds_bytes(block, r.planes, G, r.mplanes, nw);
        if (lds > lds_limit()) continue;
        s->C = C;
        s->lanes_per_ring = Tr;
        s->rings_per_wg = G;
        s->block = block;
        s->grid = (R + G - 1) / G;
        s->lds = lds;
        return ASEP_OK;
    }
    return ASEP_E_UNSUPPORTED;
}

struct asep_sim {
    Resolved r;
    Shape shape;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    uint64_t* words = nullptr;
    uint64_t* masks = nullptr;
    int64_t* hops = nullptr;
    Record* rec = nullptr;     // device staging
    uint64_t* rec_t = nullptr; // device copy of measurement times
    uint32_t rec_cap = 0;      // records per ring the staging holds
    void* own_state = nullptr;
    void* own_aux = nullptr;
    uint64_t t = 0;
    std::vector<Record> host_rec;
    // sweep-launch timing
    bool prof = false;
    std::vector<hipEvent_t> ev;     // pairs (start, stop)
    std::vector<uint64_t> ev_att;   // attempts of each pending pair
    size_t ev_pending = 0;
    asep_profile_stats prof_acc{};
};

static const size_t kEvPairs = 64;

// Add the durations of every recorded (start, stop) pair (waits for them).
static int harvest_events(asep_sim* s) {
    for (size_t i = 0; i < s->ev_pending; ++i) {
        HIP_OR_FAIL(hipEventSynchronize(s->ev[2 * i + 1]));
        float ms = 0.f;
        HIP_OR_FAIL(hipEventElapsedTime(&ms, s->ev[2 * i], s->ev[2 * i + 1]));
        s->prof_acc.launches += 1;
        s->prof_acc.kernel_ms += ms;
        s->prof_acc.attempts += s->ev_att[i];
    }
    s->ev_pending = 0;
    return ASEP_OK;
}

static const uint32_t kRecCap = 64;  // measurement times per launch

static void aux_layout(const Resolved& r, size_t* o_masks, size_t* o_hops, size_t* o_rec,
                       size_t* o_rect, size_t* total) {
    size_t off = 0;
    *o_masks = off;
    off += (size_t)r.n_real * r.mplanes * r.nw * 8;
    off = (off + 255) & ~(size_t)255;
    *o_hops = off;
    off += (size_t)r.P.samples * 8;
    off = (off + 255) & ~(size_t)255;
    *o_rec = off;
    off += (size_t)kRecCap * r.P.samples * sizeof(Record);
    off = (off + 255) & ~(size_t)255;
    *o_rect = off;
    off += (size_t)kRecCap * 8;
    *total = (off + 255) & ~(size_t)255;
}

extern "C" int asep_buffer_sizes(const asep_params* p, size_t* state_bytes, size_t* aux_bytes) {
    Resolved r;
    int rc = resolve(p, &r);
    if (rc) return rc;
    size_t a, b, c, d, tot;
    aux_layout(r, &a, &b, &c, &d, &tot);
    if (state_bytes) *state_bytes = (size_t)r.P.samples * r.planes * r.nw * 8;
    if (aux_bytes) *aux_bytes = tot;
    return ASEP_OK;
}

static int sim_init(asep_sim* s) {
    const Resolved& r = s->r;
    HIP_OR_FAIL(launch_init_state(s->words, r.P.samples, r.planes, r.nw, r.P.init, r.sc.T_init,
                                  r.P.seed, r.P.stream, r.P.sample_offset, s->stream));
    if (r.mplanes)
        HIP_OR_FAIL(launch_init_masks(s->masks, r.n_real, r.mplanes, r.mtags, r.nw, r.T_mask,
                                      r.P.seed, r.P.stream, r.real0, s->stream));
    HIP_OR_FAIL(hipMemsetAsync(s->hops, 0, (size_t)r.P.samples * 8, s->stream));
    return ASEP_OK;
}

static int create_common(const asep_params* p, void* state, size_t state_bytes, void* aux,
                         size_t aux_bytes, void* stream, bool borrowed, asep_sim** out) {
    if (!out) return ASEP_E_INVAL;
    asep_sim* s = new (std::nothrow) asep_sim();
    if (!s) return ASEP_E_NOMEM;
    int rc = resolve(p, &s->r);
    if (rc == ASEP_OK) rc = choose_shape(s->r, &s->shape);
    if (rc) {
        delete s;
        return rc;
    }
    size_t need_state, need_aux;
    asep_buffer_sizes(p, &need_state, &need_aux);
    size_t o_masks, o_hops, o_rec, o_rect, tot;
    aux_layout(s->r, &o_masks, &o_hops, &o_rec, &o_rect, &tot);
    if (borrowed) {
        if (!state || !aux || state_bytes < need_state || aux_bytes < need_aux) {
            delete s;
            return ASEP_E_INVAL;
        }
        s->stream = (hipStream_t)stream;
    } else {
        hipError_t e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete s;
            return device_fail(e, "hipStreamCreateWithFlags");
        }
        s->own_stream = true;
        if (hipMalloc(&s->own_state, need_state) != hipSuccess ||
            hipMalloc(&s->own_aux, need_aux) != hipSuccess) {
            asep_destroy(s);
            return ASEP_E_NOMEM;
        }
        state = s->own_state;
        aux = s->own_aux;
    }
    unsigned char* a = (unsigned char*)aux;
    s->words = (uint64_t*)state;
    s->masks = s->r.mplanes ? (uint64_t*)(a + o_masks) : nullptr;
    s->hops = (int64_t*)(a + o_hops);
    s->rec = (Record*)(a + o_rec);
    s->rec_t = (uint64_t*)(a + o_rect);
    s->rec_cap = kRecCap;
    rc = sim_init(s);
    if (rc) {
        asep_destroy(s);
        return rc;
    }
    *out = s;
    return ASEP_OK;
}

extern "C" int asep_create(const asep_params* p, asep_sim** out) {
    return create_common(p, nullptr, 0, nullptr, 0, nullptr, false, out);
}

extern "C" int asep_create_ext(const asep_params* p, void* state_dev, size_t state_bytes,
                               void* aux_dev, size_t aux_bytes, void* hip_stream,
                               asep_sim** out) {
    return create_common(p, state_dev, state_bytes, aux_dev, aux_bytes, hip_stream, true, out);
}

extern "C" int asep_get_params(const asep_sim* s, asep_params* out) {
    if (!s || !out) return ASEP_E_INVAL;
    *out = s->r.P;
    return ASEP_OK;
}

extern "C" void asep_destroy(asep_sim* s) {
    if (!s) return;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    for (hipEvent_t e : s->ev) (void)hipEventDestroy(e);
    if (s->own_state) (void)hipFree(s->own_state);
    if (s->own_aux) (void)hipFree(s->own_aux);
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

// One launch of the ring kernel from s->t to t1, measuring at rec_t[0..n).
static int ring_launch(asep_sim* s, uint64_t t1, const uint64_t* rec_t_dev, uint32_t n_rec) {
    const Resolved& r = s->r;
    RingArgs a{};
    a.words = s->words;
    a.masks = s->masks;
    a.hops = s->hops;
    a.rec = s->rec;
    a.rec_t = rec_t_dev;
    a.n_rec = n_rec;
    a.t0 = s->t;
    a.t1 = t1;
    a.R = r.P.samples;
    a.nw = r.nw;
    a.planes = r.planes;
    a.mplanes = r.mplanes;
    a.lanes_per_ring = s->shape.lanes_per_ring;
    a.rings_per_wg = s->shape.rings_per_wg;
    a.key0 = r.P.seed;
    a.key1 = r.P.stream;
    a.sample0 = r.P.sample_offset;
    a.spd = r.spd;
    a.real0 = r.real0;
    a.sc = r.sc;
    const bool prof = s->prof;
    if (prof) {
        if (s->ev_pending == kEvPairs) {
            int rc = harvest_events(s);
            if (rc) return rc;
        }
        HIP_OR_FAIL(hipEventRecord(s->ev[2 * s->ev_pending], s->stream));
    }
    HIP_OR_FAIL(launch_ring(a, s->shape.C, r.model, s->shape.block, s->shape.grid, s->shape.lds,
                            s->stream));
    if (prof) {
        HIP_OR_FAIL(hipEventRecord(s->ev[2 * s->ev_pending + 1], s->stream));
        s->ev_att[s->ev_pending] = (t1 - s->t) * (uint64_t)r.P.samples * r.P.L * (r.planes == 2 ? 4 : 1);
        s->ev_pending += 1;
    }
    s->t = t1;
    return ASEP_OK;
}

extern "C" int asep_profile_enable(asep_sim* s, int enable) {
    if (!s) return ASEP_E_INVAL;
    if (enable && s->ev.empty()) {
        s->ev.resize(2 * kEvPairs);
        s->ev_att.resize(kEvPairs);
        for (auto& e : s->ev) HIP_OR_FAIL(hipEventCreate(&e));
    }
    if (!enable) {
        int rc = harvest_events(s);
        if (rc) return rc;
    }
    s->prof = enable != 0;
    s->prof_acc = asep_profile_stats{};
    return ASEP_OK;
}

extern "C" int asep_profile_read(asep_sim* s, asep_profile_stats* out) {
    if (!s || !out) return ASEP_E_INVAL;
    int rc = harvest_events(s);
    if (rc) return rc;
    *out = s->prof_acc;
    return ASEP_OK;
}

extern "C" int asep_reset(asep_sim* s) {
    if (!s) return ASEP_E_INVAL;
    int rc = sim_init(s);
    if (rc) return rc;
    s->t = 0;
    return ASEP_OK;
}

static const uint64_t kMaxG = (uint64_t(1) << 48) - 1;

extern "C" int asep_sweep(asep_sim* s, uint64_t n_mcs) {
    if (!s) return ASEP_E_INVAL;
    if (n_mcs == 0) return ASEP_OK;
    const uint64_t t1 = s->t + n_mcs;
    if (t1 < s->t || t1 > kMaxG / s->r.sc.S) return ASEP_E_INVAL;
    return ring_launch(s, t1, nullptr, 0);
}

static void fill_rough(const Resolved& r, const Record& rc, asep_rough* o) {
    o->sum_h = rc.s1;
    o->sum_h2_lo = rc.s2lo;
    o->sum_h2_hi = rc.s2hi;
    o->hops = rc.hops;
    o->particles = rc.n;
    const __int128 s2 = ((__int128)rc.s2hi << 64) | (__int128)rc.s2lo;
    const __int128 L = (__int128)r.P.L;
    const __int128 num = L * s2 - (__int128)rc.s1 * rc.s1;
    o->w2 = (double)num / ((double)r.P.L * (double)r.P.L);
}

extern "C" int asep_roughness(asep_sim* s, asep_rough* out) {
    if (!s || !out) return ASEP_E_INVAL;
    const Resolved& r = s->r;
    HIP_OR_FAIL(launch_rough(s->words, s->hops, s->rec, r.P.samples, r.planes, r.nw, s->stream));
    s->host_rec.resize(r.P.samples);
    HIP_OR_FAIL(hipMemcpyAsync(s->host_rec.data(), s->rec, sizeof(Record) * r.P.samples,
                               hipMemcpyDeviceToHost, s->stream));
    HIP_OR_FAIL(hipStreamSynchronize(s->stream));
    for (uint32_t i = 0; i < r.P.samples; ++i) fill_rough(r, s->host_rec[i], &out[i]);
    return ASEP_OK;
}

extern "C" int asep_run(asep_sim* s, const uint64_t* times, uint32_t n_times, asep_rough* out) {
    if (!s || (n_times && (!times || !out))) return ASEP_E_INVAL;
    for (uint32_t i = 0; i < n_times; ++i) {
        if (times[i] < s->t || (i && times[i] < times[i - 1])) return ASEP_E_INVAL;
        if (times[i] > kMaxG / s->r.sc.S) return ASEP_E_INVAL;
    }
    const Resolved& r = s->r;
    const uint32_t R = r.P.samples;
    s->host_rec.resize((size_t)s->rec_cap * R);
    uint32_t done = 0;
    while (done < n_times) {
        const uint32_t n = std::min(s->rec_cap, n_times - done);
        HIP_OR_FAIL(hipMemcpyAsync(s->rec_t, times + done, 8 * n, hipMemcpyHostToDevice,
                                   s->stream));
        int rc = ring_launch(s, times[done + n - 1], s->rec_t, n);
        if (rc) return rc;
        HIP_OR_FAIL(hipMemcpyAsync(s->host_rec.data(), s->rec, sizeof(Record) * n * R,
                                   hipMemcpyDeviceToHost, s->stream));
        HIP_OR_FAIL(hipStreamSynchronize(s->stream));
        for (uint32_t i = 0; i < n * R; ++i)
            fill_rough(r, s->host_rec[i], &out[(size_t)done * R + i]);
        done += n;
    }
    return ASEP_OK;
}

// ---- internal entry points used by the request loop (asep_server.cpp) ----
namespace asep {

uint32_t sim_record_capacity(const asep_sim* s) { return s->rec_cap; }
hipStream_t sim_stream(const asep_sim* s) { return s->stream; }
uint32_t sim_samples(const asep_sim* s) { return s->r.P.samples; }
uint64_t sim_attempts_per_mcs(const asep_sim* s) {
    return (uint64_t)s->r.P.samples * s->r.P.L * (s->r.planes == 2 ? 4 : 1);
}

// Queue one launch advancing to t_end and measuring at times[0..n) (n <= the
// record capacity, every time in [asep_time, t_end]); the records are copied
// asynchronously to host_out (n x samples).
int sim_run_async(asep_sim* s, const uint64_t* times_pinned, uint32_t n, uint64_t t_end,
                  Record* host_out) {
    if (n > s->rec_cap || t_end < s->t) return ASEP_E_INVAL;
    if (n) {
        HIP_OR_FAIL(hipMemcpyAsync(s->rec_t, times_pinned, 8 * n, hipMemcpyHostToDevice,
                                   s->stream));
    }
    int rc = ring_launch(s, t_end, s->rec_t, n);
    if (rc) return rc;
    if (n)
        HIP_OR_FAIL(hipMemcpyAsync(host_out, s->rec, sizeof(Record) * n * s->r.P.samples,
                                   hipMemcpyDeviceToHost, s->stream));
    return ASEP_OK;
}

void record_to_rough(const asep_sim* s, const Record& rc, asep_rough* o) { fill_rough(s->r, rc, o); }

int device_error(hipError_t e, const char* where) { return device_fail(e, where); }

}  // namespace asep

extern "C" int asep_read_state(asep_sim* s, uint32_t sample, uint64_t* words, uint64_t n_words) {
    if (!s || !words || sample >= s->r.P.samples) return ASEP_E_INVAL;
    const uint64_t per = (uint64_t)s->r.planes * s->r.nw;
    if (n_words != per) return ASEP_E_INVAL;
    HIP_OR_FAIL(hipMemcpyAsync(words, s->words + per * sample, per * 8, hipMemcpyDeviceToHost,
                               s->stream));
    HIP_OR_FAIL(hipStreamSynchronize(s->stream));
    return ASEP_OK;
}

extern "C" int asep_write_state(asep_sim* s, uint32_t sample, const uint64_t* words,
                                uint64_t n_words) {
    if (!s || !words || sample >= s->r.P.samples) return ASEP_E_INVAL;
    const uint64_t per = (uint64_t)s->r.planes * s->r.nw;
    if (n_words != per) return ASEP_E_INVAL;
    HIP_OR_FAIL(hipMemcpyAsync(s->words + per * sample, words, per * 8, hipMemcpyHostToDevice,
                               s->stream));
    HIP_OR_FAIL(hipStreamSynchronize(s->stream));
    return ASEP_OK;
}

extern "C" int asep_read_mask(asep_sim* s, uint32_t plane, uint32_t realization,
                              uint64_t* words, uint64_t n_words) {
    if (!s || !words) return ASEP_E_INVAL;
    const Resolved& r = s->r;
    if (plane >= r.mplanes || realization < r.real0 || realization >= r.real0 + r.n_real)
        return ASEP_E_INVAL;
    if (n_words != r.nw) return ASEP_E_INVAL;
    const uint64_t* src = s->masks + ((size_t)(realization - r.real0) * r.mplanes + plane) * r.nw;
    HIP_OR_FAIL(hipMemcpyAsync(words, src, 8 * (size_t)r.nw, hipMemcpyDeviceToHost, s->stream));
    HIP_OR_FAIL(hipStreamSynchronize(s->stream));
    return ASEP_OK;
}

extern "C" int asep_current(asep_sim* s, int64_t* hops) {
    if (!s || !hops) return ASEP_E_INVAL;
    HIP_OR_FAIL(hipMemcpyAsync(hops, s->hops, 8 * (size_t)s->r.P.samples, hipMemcpyDeviceToHost,
                               s->stream));
    HIP_OR_FAIL(hipStreamSynchronize(s->stream));
    return ASEP_OK;
}

extern "C" int asep_set_time(asep_sim* s, uint64_t t, const int64_t* hops) {
    if (!s || t > kMaxG / s->r.sc.S) return ASEP_E_INVAL;
    const size_t n = (size_t)s->r.P.samples * 8;
    if (hops)
        HIP_OR_FAIL(hipMemcpyAsync(s->hops, hops, n, hipMemcpyHostToDevice, s->stream));
    else
        HIP_OR_FAIL(hipMemsetAsync(s->hops, 0, n, s->stream));
    HIP_OR_FAIL(hipStreamSynchronize(s->stream));
    s->t = t;
    return ASEP_OK;
}

extern "C" uint64_t asep_time(const asep_sim* s) { return s ? s->t : 0; }

extern "C" int asep_ensemble_w2(const asep_rough* r, uint32_t n, uint64_t L, double* w2_mean) {
    if (!r || !w2_mean || n == 0 || L == 0) return ASEP_E_INVAL;
    __int128 acc = 0;
    for (uint32_t i = 0; i < n; ++i) {
        const __int128 s2 = ((__int128)r[i].sum_h2_hi << 64) | (__int128)r[i].sum_h2_lo;
        acc += (__int128)L * s2 - (__int128)r[i].sum_h * r[i].sum_h;
    }
    *w2_mean = (double)acc / ((double)n * (double)L * (double)L);
    return ASEP_OK;
}

extern "C" int asep_sample_times(double t0, double factor, uint64_t t_max, uint64_t* out,
                                 uint32_t cap, uint32_t* n) {
    if (!out || !n || !(t0 > 0) || !(factor > 1.0)) return ASEP_E_INVAL;
    uint32_t k = 0;
    if (cap == 0) {
        *n = 0;
        return ASEP_OK;
    }
    out[k++] = 0;
    for (double t = t0; t <= (double)t_max; t *= factor) {
        const uint64_t c = (uint64_t)std::ceil(t);
        if (c > t_max) break;
        if (out[k - 1] == c) continue;
        if (k >= cap) break;
        out[k++] = c;
    }
    *n = k;
    return ASEP_OK;
}

extern "C" const char* asep_strerror(int code) {
    switch (code) {
        case ASEP_OK: return "ok";
        case ASEP_E_INVAL: return "invalid argument";
        case ASEP_E_UNSUPPORTED: return "unsupported configuration";
        case ASEP_E_NOMEM: return "out of memory";
        case ASEP_E_DEVICE: return "HIP device error";
        case ASEP_E_BUSY: return "queue full";
        case ASEP_E_PENDING: return "pending";
        case ASEP_E_CANCELLED: return "cancelled";
        case ASEP_E_TIMEOUT: return "timed out";
        case ASEP_E_NOTFOUND: return "unknown ticket";
        default: return "unknown error";
    }
}

extern "C" const char* asep_last_device_error(void) { return g_last_device_error.c_str(); }
