// asep_host.cpp -- host side of the C ABI declared in include/asep.h:
// parameter validation, probability -> threshold lowering, device buffers,
// launch shapes, and the conversions of exact integer sums to W^2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <new>
#include <sstream>
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

// ---------------------------------------------------------------------------
// Tuning table (process-wide): per class of run (model, schedule, disorder,
// range of log2 L, range of samples) the launch shape and, for the shifted
// schedule, the cell size and sub-sweeps the autotuner chose.  Parameters
// left at 0 are filled from the first matching entry.
// ---------------------------------------------------------------------------
namespace {

struct TuneEntry {
    uint32_t model, schedule, disorder;
    uint32_t l2_lo, l2_hi;
    uint64_t s_lo, s_hi;
    int32_t cell_log2, subsweeps;
    uint32_t windows, window_sweeps, rings_per_wg;
};

std::mutex g_tune_mu;
std::vector<TuneEntry> g_tune;

uint32_t floor_log2(uint64_t v) {
    uint32_t e = 0;
    while (v >>= 1) ++e;
    return e;
}

bool tune_match(const asep_params& P, TuneEntry* out) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const uint32_t e = floor_log2(P.L);
    const uint32_t dis = P.slow_frac > 0 ? 1u : 0u;
    for (const TuneEntry& t : g_tune) {
        if (t.model == P.model && t.schedule == P.schedule && t.disorder == dis && e >= t.l2_lo &&
            e <= t.l2_hi && P.samples >= t.s_lo && P.samples <= t.s_hi) {
            *out = t;
            return true;
        }
    }
    return false;
}

}  // namespace

extern "C" int asep_tuning_load(const char* path) {
    std::vector<TuneEntry> tab;
    if (path && *path) {
        std::ifstream f(path);
        if (!f) return ASEP_E_NOTFOUND;
        std::string line;
        while (std::getline(f, line)) {
            const size_t h = line.find('#');
            if (h != std::string::npos) line.resize(h);
            std::istringstream in(line);
            TuneEntry t{};
            long long v[12];
            int n = 0;
            while (n < 12 && (in >> v[n])) ++n;
            if (n == 0 && in.eof()) continue;  // blank or comment
            std::string rest;
            if (n != 12 || (in >> rest)) return ASEP_E_INVAL;
            for (int i = 0; i < 12; ++i)
                if (v[i] < 0 || v[i] > 0xFFFFFFFFll) return ASEP_E_INVAL;
            t.model = (uint32_t)v[0];
            t.schedule = (uint32_t)v[1];
            t.disorder = (uint32_t)v[2];
            t.l2_lo = (uint32_t)v[3];
            t.l2_hi = (uint32_t)v[4];
            t.s_lo = (uint64_t)v[5];
            t.s_hi = (uint64_t)v[6];
            t.cell_log2 = (int32_t)v[7];
            t.subsweeps = (int32_t)v[8];
            t.windows = (uint32_t)v[9];
            t.window_sweeps = (uint32_t)v[10];
            t.rings_per_wg = (uint32_t)v[11];
            if (t.model > 1 || t.schedule > 1 || t.disorder > 1 || t.l2_lo > t.l2_hi ||
                t.l2_hi > 63 || t.s_lo > t.s_hi || t.cell_log2 > 6 || t.subsweeps > 256 ||
                t.window_sweeps > 4096)
                return ASEP_E_INVAL;
            tab.push_back(t);
        }
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.swap(tab);
    return ASEP_OK;
}

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
    int dev;              // device whose limits the plan follows
};

static int resolve(const asep_params* in, int dev, Resolved* r) {
    if (!in) return ASEP_E_INVAL;
    if (in->abi_version != ASEP_ABI_VERSION) return ASEP_E_INVAL;
    asep_params P = *in;
    if (P.schedule != ASEP_SCHED_SHIFTED && P.schedule != ASEP_SCHED_SUBLATTICE)
        return ASEP_E_INVAL;
    const bool sca = P.schedule == ASEP_SCHED_SUBLATTICE;
    // parameters left at 0 take the tuning table's values: the update
    // schedule (shifted cells only) as one unit when neither is given, the
    // launch shape as one unit when none of its fields is given
    TuneEntry te;
    if (P.samples && tune_match(P, &te)) {
        if (!sca && P.cell_log2 == 0 && P.subsweeps == 0 && te.cell_log2 && te.subsweeps) {
            P.cell_log2 = te.cell_log2;
            P.subsweeps = te.subsweeps;
        }
        if (P.windows == 0 && P.window_sweeps == 0 && P.rings_per_wg == 0) {
            P.windows = te.windows;
            P.window_sweeps = te.window_sweeps;
            P.rings_per_wg = te.rings_per_wg;
        }
    }
    if (sca) {
        // pairs of two sites; single lane: even pairs, odd pairs (S = 2);
        // two lanes: even pairs, A -> B, odd pairs, B -> A (S = 4)
        const int32_t S_sca = P.model == ASEP_MODEL_TWO_LANE ? 4 : 2;
        if ((P.cell_log2 != 0 && P.cell_log2 != 1) || (P.subsweeps != 0 && P.subsweeps != S_sca))
            return ASEP_E_INVAL;
        // the two-lane sequence changes lanes at every site (bimodal rates
        // through the slow marks), so there is no turning-point plane
        if (P.model == ASEP_MODEL_TWO_LANE && P.turn_frac != 0) return ASEP_E_INVAL;
        P.cell_log2 = 1;
        P.subsweeps = S_sca;
    }
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
    if (two && !sca && P.slow_frac > 0) return ASEP_E_UNSUPPORTED;
    if ((uint64_t)P.sample_offset + P.samples > 0x100000000ull) return ASEP_E_INVAL;

    Sched sc{};
    sc.lam = (uint32_t)P.cell_log2;
    sc.S = (uint32_t)P.subsweeps;
    sc.a = per_mcs / sc.S;
    const int ebits = two ? 2 : 0;
    // draw width: the shifted schedule packs [j | e | r] into 32 bits; the
    // two-sub-lattice update compares a 24-bit uniform per pair
    const int B = sca ? 24 : 32 - (int)sc.lam - ebits;
    uint64_t TB[4] = {0, 0, 0, 0};
    uint32_t n_used;  // thresholds in use: TB[0 .. n_used)
    if (!two) {
        TB[0] = lower_prob(P.p, B);
        TB[1] = lower_prob(P.q, B);
        TB[2] = lower_prob(P.slow_factor * P.p, B);
        TB[3] = lower_prob(P.slow_factor * P.q, B);
        n_used = P.slow_frac > 0 ? 4 : 2;
    } else if (sca) {
        TB[0] = lower_prob(P.p, B);
        TB[1] = lower_prob(P.q, B);
        TB[2] = lower_prob(P.lane_rate, B);
        TB[3] = lower_prob(P.slow_factor * P.lane_rate, B);  // marked sites
        n_used = P.slow_frac > 0 ? 4 : 3;
    } else {
        // hops compare the attempt field's bits; a lane change draws a 32-bit
        // word of its own per candidate (below)
        TB[0] = lower_prob(P.p, B);
        TB[1] = lower_prob(P.q, B);
        n_used = 2;
    }
    auto exact_at = [&](int b) {
        const uint64_t unit = uint64_t(1) << (B - b);
        for (uint32_t i = 0; i < n_used; ++i)
            if (TB[i] % unit != 0) return false;
        return true;
    };
    int b;
    if (P.rbits <= 0) {
        for (b = 0; b < B && !exact_at(b); ++b) {
        }
    } else {
        b = P.rbits;
        if (b > B || !exact_at(b)) return ASEP_E_INVAL;
    }
    P.rbits = b;
    sc.b = (uint32_t)b;
    for (int i = 0; i < 4; ++i) sc.T[i] = (uint32_t)(TB[i] >> (B - b));
    if (two && !sca) {
        // lane change: threshold at 32 bits, compared at its fewest exact bits
        const uint64_t tc = lower_prob(P.lane_rate, 32);
        uint32_t c = 0;
        while (c < 32 && tc % (uint64_t(1) << (32 - c)) != 0) ++c;
        sc.bc = c;
        sc.T[2] = (uint32_t)(tc >> (32 - c));
    }
    if (sca) {
        sc.w = 0;
        sc.A = 0;
        // one random bit plane per compared bit: 32 pairs or sites per word;
        // two lanes draw two words per plane (A and B pairs, or 64 sites)
        sc.nblk = two ? (sc.b + 1) / 2 : (sc.b + 3) / 4;
    } else {
        // cells of 32 sites whose field fits a byte take the four bytes of a
        // word as fields, the position in the low bits (read straight from
        // the byte by the shifts that use it); other schedules pack fields of
        // lam + ebits + b bits with the position on top
        sc.jlow = (sc.lam == 5 && sc.lam + (uint32_t)ebits + sc.b <= 8) ? 1u : 0u;
        sc.w = sc.jlow ? 8u : sc.lam + (uint32_t)ebits + sc.b;
        sc.A = 32 / sc.w;
        sc.nblk = (sc.a + 4 * sc.A - 1) / (4 * sc.A);
    }
    sc.T_init = lower_prob(P.density, 32);
    sc.T_slow = lower_prob(P.slow_frac, 32);
    sc.T_turn = lower_prob(P.turn_frac, 32);

    r->P = P;
    r->sc = sc;
    r->dev = dev;
    r->planes = two ? 2 : 1;
    r->nw = (uint32_t)(P.L / 64);
    r->spd = P.samples_per_disorder;
    if (two && sca) {
        r->model = kTwoLane;  // u (A -> B) and v (B -> A) marks, if any
        r->mplanes = P.slow_frac > 0 ? 2 : 0;
        r->mtags[0] = kTagDisP;
        r->mtags[1] = kTagDisQ;
        r->T_mask = sc.T_slow;
    } else if (two) {
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

// ---------------------------------------------------------------------------
// Launch plans.  A ring is either held whole by one workgroup (periodic,
// measurements inside the launch) or cut into windows of seg_n output words
// plus a halo, one workgroup each, advanced K <= halo-1 sub-sweeps per launch
// between two state buffers.  Windows are used when the ring does not fit a
// workgroup, or when whole rings would leave compute units idle.
// ---------------------------------------------------------------------------
struct Plan {
    bool seg = false;
    uint32_t C = 1, block = 64, lanes_per_ring = 1, rings_per_wg = 1, grid = 1;
    uint32_t segs = 1, seg_n = 0, halo = 0, nslot = 0, K = 0;
    size_t lds = 0;
    SweepKernel kern{};
};

// LDS per workgroup and compute units of a device, looked up once per
// device (any thread may plan: the request loop sizes requests on the
// submitting thread).
static void device_limits(int dev, size_t* lds, uint32_t* cus) {
    static std::mutex mu;
    static std::map<int, std::pair<size_t, uint32_t>> cache;
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(dev);
    if (it == cache.end()) {
        size_t lim = 0;
        uint32_t ncu = 0;
        hipDeviceProp_t prop;
        if (dev >= 0 && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
            lim = prop.sharedMemPerBlock;
            ncu = (uint32_t)prop.multiProcessorCount;
        }
        // no device visible (host-only planning): gfx950's limits
        if (!lim) lim = 160 * 1024;
        if (!ncu) ncu = 256;
        it = cache.emplace(dev, std::make_pair(lim, ncu)).first;
    }
    *lds = it->second.first;
    *cus = it->second.second;
}

static int current_device() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    return dev;
}

// Attempt-loop variant: the specialised ones need ell = 64 and the default
// four sub-sweeps per MCS (16 attempts per cell and sub-sweep; 64 on two
// lanes); they differ in fields per 32-bit word and compared bits.
static SweepKernel pick_kernel(const Resolved& r, uint32_t C) {
    SweepKernel k{};
    k.C = C;
    k.model = r.model;
    k.variant = 0;
    const Sched& sc = r.sc;
    const bool two = r.model == kTwoLane;
    if (r.P.schedule == ASEP_SCHED_SUBLATTICE) {
        k.variant = 6;  // the paper's sub-lattice updates
    } else if (sc.lam == 6 && sc.a == (two ? 64u : 16u)) {
        uint32_t v = 0;
        if (!two) {
            if (sc.A == 5 && sc.b == 0) v = 1;
            if (sc.A == 4 && sc.b == 1) v = 2;
            if (sc.A == 4 && sc.b == 2) v = 3;
            if (sc.A == 1) v = 4;
        } else {
            if (sc.A == 4 && sc.b == 0) v = 5;
            if (sc.A == 1) v = 4;
        }
        if (v && sweep_variant_compiled(C, r.model, v)) k.variant = v;
    } else if (sc.lam == 5 && sc.a == 16 && r.model != kTwoLane) {
        // cells of 32 sites, two sub-sweeps: the slot's halves are two cells
        uint32_t v = 0;
        if (sc.jlow && sc.b == 0) v = 7;
        if (sc.jlow && sc.b == 1) v = 8;
        if (v && sweep_variant_compiled(C, r.model, v)) k.variant = v;
    }
    k.q0 = !two && sc.T[1] == 0 && (r.model != kDisorder || sc.T[3] == 0);
    return k;
}

static bool plan_whole(const Resolved& r, Plan* p) {
    size_t lim;
    uint32_t ncu;
    device_limits(r.dev, &lim, &ncu);
    const uint32_t nw = r.nw, R = r.P.samples;
    static const uint32_t Cs[] = {1, 2, 4, 8, 16};
    for (uint32_t C : Cs) {
        if (!sweep_variant_compiled(C, r.model, pick_kernel(r, C).variant)) continue;
        const uint32_t maxb = sweep_block_limit(C, r.model);
        uint32_t Tr = (nw + C - 1) / C;
        if (Tr > maxb) continue;
        // rings of at most one wave get a power-of-two lane count, so none
        // straddles two waves and the kernel exchanges across lanes
        if (Tr < 64) {
            uint32_t t = 1;
            while (t < Tr) t <<= 1;
            Tr = t;
        }
        uint32_t G = 1;
        if (r.P.rings_per_wg)
            G = std::min(r.P.rings_per_wg, R);
        else if (Tr < 256)
            G = std::max(1u, std::min(256u / Tr, R));
        if ((uint64_t)G * Tr > maxb) continue;
        const uint32_t block = std::min(maxb, (G * Tr + 63) / 64 * 64);
        if (block < G * Tr) continue;
        const size_t lds = sweep_lds_bytes(block, r.planes, G, r.mplanes, nw);
        if (lds > lim) continue;
        p->seg = false;
        p->C = C;
        p->block = block;
        p->lanes_per_ring = Tr;
        p->rings_per_wg = G;
        p->grid = (R + G - 1) / G;
        p->segs = 1;
        p->lds = lds;
        p->kern = pick_kernel(r, C);
        return true;
    }
    return false;
}

static bool plan_windows(const Resolved& r, uint32_t segs, uint32_t K, Plan* p) {
    size_t lim;
    uint32_t ncu;
    device_limits(r.dev, &lim, &ncu);
    const uint32_t nw = r.nw;
    if (segs < 2 || segs > nw) return false;
    const uint32_t seg_n = (nw + segs - 1) / segs;
    // windows of seg_n words: as many as it takes (every window owns words;
    // a count whose last window would be empty becomes the next smaller one)
    segs = (nw + seg_n - 1) / seg_n;
    if (segs < 2) return false;
    // the window starts exactly its drift (at most K+1 words) before its
    // output and reaches K+1 words past it (the garbage depth)
    const uint32_t halo = K + 1;
    const uint32_t nslot = seg_n + halo;
    if (nslot + halo + 2 > 4 * (uint64_t)nw) return false;
    static const uint32_t Cs[] = {1, 2, 4, 8};
    for (uint32_t C : Cs) {
        if (!sweep_variant_compiled(C, r.model, pick_kernel(r, C).variant)) continue;
        const uint32_t maxb = sweep_block_limit(C, r.model);
        const uint32_t Tr = (nslot + C - 1) / C;
        if (Tr > maxb) continue;
        const uint32_t block = (Tr + 63) / 64 * 64;
        if (block > maxb) continue;
        const size_t lds = sweep_lds_bytes(block, r.planes, 1, r.mplanes, nslot + halo + 2);
        if (lds > lim) continue;
        p->seg = true;
        p->C = C;
        p->block = block;
        p->lanes_per_ring = Tr;
        p->rings_per_wg = 1;
        p->segs = segs;
        p->seg_n = seg_n;
        p->halo = halo;
        p->nslot = nslot;
        p->K = K;
        p->grid = r.P.samples * segs;
        p->lds = lds;
        p->kern = pick_kernel(r, C);
        return true;
    }
    return false;
}

static int choose_plan(const Resolved& r, Plan* p) {
    size_t lim;
    uint32_t ncu;
    device_limits(r.dev, &lim, &ncu);
    const uint32_t want = r.P.windows;  // windows per ring (0 = auto)
    // sub-sweeps per window launch: given, else 63 (longer launches need
    // longer windows, i.e. fewer of them per ring: on the served mix that
    // parallelism was worth more than the launches saved)
    const uint32_t K = r.P.window_sweeps ? r.P.window_sweeps : 63;
    if (K > 4096) return ASEP_E_INVAL;
    if (want == 1) return plan_whole(r, p) ? ASEP_OK : ASEP_E_UNSUPPORTED;
    if (want >= 2) return plan_windows(r, want, K, p) ? ASEP_OK : ASEP_E_UNSUPPORTED;
    Plan whole;
    const bool have_whole = plan_whole(r, &whole);
    const uint32_t R = r.P.samples;
    // Whole rings when they fill the compute units or are too short for
    // windows.  Otherwise windows: as many as it takes to give each compute
    // unit a workgroup, but no more than keep every window's output at least
    // twice its reach (K + 1 words), and at least as many as fit a workgroup
    // -- a few long rings in a few workgroups would hold a handful of CUs
    // for the whole run (and a served request's launch shares the GPU with
    // at most three others, one per hardware queue).
    if (have_whole && (whole.grid >= ncu || r.nw < 4 * (K + 1))) {
        *p = whole;
        return ASEP_OK;
    }
    const uint32_t fill = (ncu + R - 1) / R;
    const uint32_t cap = std::max(2u, r.nw / (2 * (K + 1)));
    for (uint32_t segs = std::max(2u, std::min(fill, cap)); segs <= r.nw;
         segs = segs + (segs >> 2) + 1)
        if (plan_windows(r, segs, K, p)) return ASEP_OK;
    if (have_whole) {
        *p = whole;
        return ASEP_OK;
    }
    return ASEP_E_UNSUPPORTED;
}

struct asep_sim {
    Resolved r;
    Plan plan;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    uint64_t* words = nullptr;  // the state buffer (caller-visible)
    uint64_t* alt = nullptr;    // second state buffer of windowed plans
    uint64_t* masks = nullptr;
    int64_t* hops = nullptr;
    Record* rec = nullptr;      // device staging
    SegRec* segs = nullptr;     // measurement segments
    uint32_t rec_cap = 0;       // records per ring the staging holds
    void* own_state = nullptr;
    void* own_aux = nullptr;
    uint64_t t = 0;
    Record* host_rec = nullptr;  // pinned staging of rec_cap x samples records
    bool own_host_rec = false;   // allocated here (else borrowed from the caller)
    // sweep-launch timing
    bool prof = false;
    std::vector<hipEvent_t> ev;    // pairs (start, stop), ring buffer
    std::vector<uint64_t> ev_att;  // attempts of each recorded pair
    size_t ev_head = 0, ev_count = 0;
    asep_profile_stats prof_acc{};
};

static const size_t kEvPairs = 4096;

// Add the durations of the oldest `n` recorded pairs (waits for them).
static int harvest_events(asep_sim* s, size_t n) {
    n = std::min(n, s->ev_count);
    for (size_t q = 0; q < n; ++q) {
        const size_t i = (s->ev_head + kEvPairs - s->ev_count) % kEvPairs;
        HIP_OR_FAIL(hipEventSynchronize(s->ev[2 * i + 1]));
        float ms = 0.f;
        HIP_OR_FAIL(hipEventElapsedTime(&ms, s->ev[2 * i], s->ev[2 * i + 1]));
        s->prof_acc.launches += 1;
        s->prof_acc.kernel_ms += ms;
        s->prof_acc.attempts += s->ev_att[i];
        s->ev_count -= 1;
    }
    return ASEP_OK;
}

static const uint32_t kRecCap = 64;  // measurement times per chunk

static void aux_layout(const Resolved& r, const Plan& pl, size_t* o_masks, size_t* o_hops,
                       size_t* o_rec, size_t* o_recg, size_t* o_alt, size_t* total) {
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
    *o_recg = off;
    off += (size_t)kRecCap * 8;
    off = (off + 255) & ~(size_t)255;
    *o_alt = off;
    if (pl.seg) off += (size_t)r.P.samples * r.planes * r.nw * 8;
    off = (off + 255) & ~(size_t)255;
    off += rough_seg_bytes(r.P.samples, r.nw);  // measurement segments (last)
    *total = (off + 255) & ~(size_t)255;
}

// Offset of the measurement segments: after the second state buffer.
static size_t seg_offset(const Resolved& r, const Plan& pl, size_t o_alt) {
    size_t off = o_alt;
    if (pl.seg) off += (size_t)r.P.samples * r.planes * r.nw * 8;
    return (off + 255) & ~(size_t)255;
}

static int buffer_sizes_on(const asep_params* p, int dev, size_t* state_bytes,
                           size_t* aux_bytes) {
    Resolved r;
    int rc = resolve(p, dev, &r);
    if (rc) return rc;
    Plan pl;
    rc = choose_plan(r, &pl);
    if (rc) return rc;
    size_t a, b, c, d, e, tot;
    aux_layout(r, pl, &a, &b, &c, &d, &e, &tot);
    if (state_bytes) *state_bytes = (size_t)r.P.samples * r.planes * r.nw * 8;
    if (aux_bytes) *aux_bytes = tot;
    return ASEP_OK;
}

extern "C" int asep_buffer_sizes(const asep_params* p, size_t* state_bytes, size_t* aux_bytes) {
    return buffer_sizes_on(p, current_device(), state_bytes, aux_bytes);
}

static int sim_init(asep_sim* s) {
    const Resolved& r = s->r;
    HIP_OR_FAIL(launch_init_state(s->words, r.P.samples, r.planes, r.nw, r.P.init, r.sc.T_init,
                                  r.P.seed, r.P.stream, r.P.sample_offset, s->stream));
    if (r.mplanes)
        HIP_OR_FAIL(launch_init_masks(s->masks, r.n_real, r.mplanes, r.mtags, r.nw, r.T_mask,
                                      r.P.seed, r.P.stream, r.real0, s->stream));
    // a fill kernel rather than a memset node, so that the work can be captured
    HIP_OR_FAIL(launch_zero_u64((uint64_t*)s->hops, r.P.samples, s->stream));
    return ASEP_OK;
}

static int create_common(const asep_params* p, void* state, size_t state_bytes, void* aux,
                         size_t aux_bytes, void* stream, bool borrowed, Record* host_rec,
                         asep_sim** out) {
    if (!out) return ASEP_E_INVAL;
    asep_sim* s = new (std::nothrow) asep_sim();
    if (!s) return ASEP_E_NOMEM;
    int rc = resolve(p, current_device(), &s->r);
    if (rc == ASEP_OK) rc = choose_plan(s->r, &s->plan);
    if (rc) {
        delete s;
        return rc;
    }
    const size_t need_state = (size_t)s->r.P.samples * s->r.planes * s->r.nw * 8;
    size_t o_masks, o_hops, o_rec, o_recg, o_alt, need_aux;
    aux_layout(s->r, s->plan, &o_masks, &o_hops, &o_rec, &o_recg, &o_alt, &need_aux);
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
    (void)o_recg;
    if (host_rec) {
        s->host_rec = host_rec;  // borrowed pinned staging
    } else if (hipHostMalloc((void**)&s->host_rec,
                             sizeof(Record) * (size_t)kRecCap * s->r.P.samples) != hipSuccess) {
        s->host_rec = nullptr;
        asep_destroy(s);
        return ASEP_E_NOMEM;
    } else {
        s->own_host_rec = true;
    }
    s->alt = s->plan.seg ? (uint64_t*)(a + o_alt) : nullptr;
    s->segs = (SegRec*)(a + seg_offset(s->r, s->plan, o_alt));
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
    return create_common(p, nullptr, 0, nullptr, 0, nullptr, false, nullptr, out);
}

extern "C" int asep_create_ext(const asep_params* p, void* state_dev, size_t state_bytes,
                               void* aux_dev, size_t aux_bytes, void* hip_stream,
                               asep_sim** out) {
    return create_common(p, state_dev, state_bytes, aux_dev, aux_bytes, hip_stream, true,
                         nullptr, out);
}

extern "C" int asep_get_params(const asep_sim* s, asep_params* out) {
    if (!s || !out) return ASEP_E_INVAL;
    *out = s->r.P;
    return ASEP_OK;
}

static void fill_plan(const Plan& pl, asep_plan* o) {
    std::memset(o, 0, sizeof *o);
    o->windows = pl.seg ? pl.segs : 1;
    o->window_sweeps = pl.seg ? pl.K : 0;
    o->slots_per_lane = pl.kern.C;
    o->block = pl.block;
    o->lanes_per_ring = pl.lanes_per_ring;
    o->rings_per_wg = pl.rings_per_wg;
    o->grid = pl.grid;
    o->attempt_loop = pl.kern.variant;
    o->backward_hops = pl.kern.q0 ? 0u : 1u;
    o->packable = (!pl.seg && pl.kern.C <= 4) ? 1u : 0u;
}

extern "C" int asep_get_plan(const asep_sim* s, asep_plan* out) {
    if (!s || !out) return ASEP_E_INVAL;
    fill_plan(s->plan, out);
    return ASEP_OK;
}

extern "C" int asep_resolve(const asep_params* p, asep_params* resolved, asep_plan* plan) {
    if (!resolved) return ASEP_E_INVAL;
    Resolved r;
    int rc = resolve(p, current_device(), &r);
    if (rc) return rc;
    Plan pl;
    rc = choose_plan(r, &pl);
    if (rc) return rc;
    *resolved = r.P;
    if (plan) fill_plan(pl, plan);
    return ASEP_OK;
}

extern "C" void asep_destroy(asep_sim* s) {
    if (!s) return;
    // work queued on a borrowed stream is the caller's to wait for
    if (s->own_stream && s->stream) (void)hipStreamSynchronize(s->stream);
    if (s->host_rec && s->own_host_rec) (void)hipHostFree(s->host_rec);
    for (hipEvent_t e : s->ev) (void)hipEventDestroy(e);
    if (s->own_state) (void)hipFree(s->own_state);
    if (s->own_aux) (void)hipFree(s->own_aux);
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

static SimDesc make_desc(const asep_sim* s) {
    const Resolved& r = s->r;
    const Plan& pl = s->plan;
    SimDesc d{};
    d.words_in = s->words;
    d.words_out = s->words;
    d.masks = s->masks;
    d.hops = s->hops;
    d.rec = s->rec;
    d.R = r.P.samples;
    d.nw = r.nw;
    d.planes = r.planes;
    d.mplanes = r.mplanes;
    d.lanes_per_ring = pl.lanes_per_ring;
    d.rings_per_wg = pl.rings_per_wg;
    d.segs = pl.segs;
    d.seg_n = pl.seg_n;
    d.halo = pl.halo;
    d.nslot = pl.nslot;
    d.key0 = r.P.seed;
    d.key1 = r.P.stream;
    d.sample0 = r.P.sample_offset;
    d.spd = r.spd;
    d.real0 = r.real0;
    d.wg_begin = 0;
    d.sc = r.sc;
    return d;
}

// One sweep launch on the simulation's stream (timed when profiling).
static int sweep_launch(asep_sim* s, const SimDesc& d) {
    const Plan& pl = s->plan;
    const bool prof = s->prof;
    size_t slot = 0;
    if (prof) {
        if (s->ev_count == kEvPairs) {
            int rc = harvest_events(s, kEvPairs / 2);
            if (rc) return rc;
        }
        slot = s->ev_head;
    }
    // timing: the dispatch records the kernel's own start and end
    HIP_OR_FAIL(launch_sweep(pl.kern, d, nullptr, 0, pl.grid, pl.block, pl.lds, s->stream,
                             prof ? s->ev[2 * slot] : nullptr,
                             prof ? s->ev[2 * slot + 1] : nullptr));
    if (prof) {
        const Resolved& r = s->r;
        s->ev_att[slot] = (d.g1 - d.g0) * (uint64_t)r.P.samples * r.P.L * (r.planes == 2 ? 4 : 1) /
                          r.sc.S;
        s->ev_head = (s->ev_head + 1) % kEvPairs;
        s->ev_count += 1;
    }
    return ASEP_OK;
}

// Queue the work from the current time to t_end (MCS), measuring at
// times[0..n) (ascending, within [t, t_end], n <= rec_cap) into the device
// staging; the records are copied to host_out (n x samples) asynchronously.
// Sub-sweeps of one whole-ring launch at most (the kernel counts them in 32 bits).
// ASEP_MAX_LAUNCH_SUBSWEEPS (1 .. 2^30) lowers it, so that tests can run the
// split of long runs at small sizes.
static const uint64_t kMaxLaunchSub = 1ull << 30;

static uint64_t max_launch_sub() {
    const char* e = std::getenv("ASEP_MAX_LAUNCH_SUBSWEEPS");
    if (e && *e) {
        char* end = nullptr;
        const unsigned long long v = std::strtoull(e, &end, 10);
        if (end && *end == '\0' && v >= 1 && v <= kMaxLaunchSub) return v;
    }
    return kMaxLaunchSub;
}

static int enqueue_to(asep_sim* s, uint64_t t_end, const uint64_t* times, uint32_t n,
                      Record* host_out) {
    const Resolved& r = s->r;
    const uint32_t S = r.sc.S;
    SimDesc d = make_desc(s);
    if (!s->plan.seg) {
        // whole rings: one launch per at most kMaxLaunchSub sub-sweeps, each
        // with the measurements in [g0, g1) (the last one also at g1)
        uint64_t g = s->t * S;
        const uint64_t g_end = t_end * S;
        const uint64_t cap = max_launch_sub();
        uint32_t ri = 0;
        do {
            const uint64_t gl = std::min<uint64_t>(g_end, g + cap);
            uint32_t nr = 0;
            while (ri + nr < n && (times[ri + nr] * S < gl || (gl == g_end && times[ri + nr] * S == gl))) {
                d.rec_g[nr] = times[ri + nr] * S;
                ++nr;
            }
            d.g0 = g;
            d.g1 = gl;
            d.n_rec = nr;
            d.rec = s->rec + (size_t)ri * r.P.samples;
            int rc = sweep_launch(s, d);
            if (rc) return rc;
            ri += nr;
            g = gl;
        } while (g < g_end);
    } else {
        // windows: launches of at most K sub-sweeps between the two buffers,
        // measurements from the words of whole rings between launches
        uint64_t* cur = s->words;
        uint64_t* oth = s->alt;
        uint64_t g = s->t * S;
        const uint64_t g_end = t_end * S;
        uint32_t ri = 0;
        for (;;) {
            while (ri < n && times[ri] * S == g) {
                HIP_OR_FAIL(launch_rough(cur, s->hops, s->rec + (size_t)ri * r.P.samples,
                                         r.P.samples, r.planes, r.nw, s->segs, s->stream));
                ++ri;
            }
            if (g >= g_end) break;
            uint64_t gl = std::min<uint64_t>(g + s->plan.K, g_end);
            if (ri < n) gl = std::min<uint64_t>(gl, times[ri] * S);
            d.words_in = cur;
            d.words_out = oth;
            d.g0 = g;
            d.g1 = gl;
            d.n_rec = 0;
            int rc = sweep_launch(s, d);
            if (rc) return rc;
            std::swap(cur, oth);
            g = gl;
        }
        if (cur != s->words)
            HIP_OR_FAIL(hipMemcpyAsync(s->words, cur, (size_t)r.P.samples * r.planes * r.nw * 8,
                                       hipMemcpyDeviceToDevice, s->stream));
    }
    s->t = t_end;
    if (n && host_out)
        HIP_OR_FAIL(hipMemcpyAsync(host_out, s->rec, sizeof(Record) * n * r.P.samples,
                                   hipMemcpyDeviceToHost, s->stream));
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
        int rc = harvest_events(s, s->ev_count);
        if (rc) return rc;
    }
    s->prof = enable != 0;
    s->prof_acc = asep_profile_stats{};
    return ASEP_OK;
}

extern "C" int asep_profile_read(asep_sim* s, asep_profile_stats* out) {
    if (!s || !out) return ASEP_E_INVAL;
    int rc = harvest_events(s, s->ev_count);
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
    return enqueue_to(s, t1, nullptr, 0, nullptr);
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
    HIP_OR_FAIL(launch_rough(s->words, s->hops, s->rec, r.P.samples, r.planes, r.nw, s->segs,
                             s->stream));
    HIP_OR_FAIL(hipMemcpyAsync(s->host_rec, s->rec, sizeof(Record) * r.P.samples,
                               hipMemcpyDeviceToHost, s->stream));
    HIP_OR_FAIL(hipStreamSynchronize(s->stream));
    for (uint32_t i = 0; i < r.P.samples; ++i) fill_rough(r, s->host_rec[i], &out[i]);
    return ASEP_OK;
}

static int check_times(const asep_sim* s, const uint64_t* times, uint32_t n_times) {
    for (uint32_t i = 0; i < n_times; ++i) {
        if (times[i] < s->t || (i && times[i] < times[i - 1])) return ASEP_E_INVAL;
        if (times[i] > kMaxG / s->r.sc.S) return ASEP_E_INVAL;
    }
    return ASEP_OK;
}

extern "C" int asep_run(asep_sim* s, const uint64_t* times, uint32_t n_times, asep_rough* out) {
    asep_sim* one[1] = {s};
    asep_rough* outs[1] = {out};
    return asep_run_batch(one, 1, times, n_times, outs);
}

extern "C" int asep_run_batch(asep_sim* const* sims, uint32_t n_sims, const uint64_t* times,
                              uint32_t n_times, asep_rough* const* outs) {
    if (!sims || n_sims == 0 || (n_times && (!times || !outs))) return ASEP_E_INVAL;
    for (uint32_t k = 0; k < n_sims; ++k) {
        if (!sims[k] || (n_times && !outs[k])) return ASEP_E_INVAL;
        for (uint32_t j = 0; j < k; ++j)
            if (sims[j] == sims[k]) return ASEP_E_INVAL;
        int rc = check_times(sims[k], times, n_times);
        if (rc) return rc;
    }
    uint32_t done = 0;
    while (done < n_times) {
        const uint32_t n = std::min(kRecCap, n_times - done);
        // queue every simulation's chunk before waiting on any of them
        for (uint32_t k = 0; k < n_sims; ++k) {
            int rc = enqueue_to(sims[k], times[done + n - 1], times + done, n,
                                sims[k]->host_rec);
            if (rc) return rc;
        }
        for (uint32_t k = 0; k < n_sims; ++k) {
            asep_sim* s = sims[k];
            HIP_OR_FAIL(hipStreamSynchronize(s->stream));
            const uint32_t R = s->r.P.samples;
            for (uint32_t i = 0; i < n * R; ++i)
                fill_rough(s->r, s->host_rec[i], &outs[k][(size_t)done * R + i]);
        }
        done += n;
    }
    return ASEP_OK;
}

// ---- internal entry points used by the request loop (asep_server.cpp) ----
namespace asep {

uint32_t sim_record_capacity(const asep_sim* s) { return s->rec_cap; }

size_t sim_host_rec_bytes(const asep_params& p) {
    return sizeof(Record) * (size_t)kRecCap * p.samples;
}

int sim_buffer_sizes_on(const asep_params* p, int dev, size_t* state_bytes, size_t* aux_bytes) {
    return buffer_sizes_on(p, dev, state_bytes, aux_bytes);
}

// asep_create_ext with a borrowed pinned staging buffer of at least
// sim_host_rec_bytes(*p) bytes, which the simulation never frees.
int sim_create_borrowed(const asep_params* p, void* state, size_t state_bytes, void* aux,
                        size_t aux_bytes, hipStream_t st, Record* host_rec, asep_sim** out) {
    if (!host_rec) return ASEP_E_INVAL;
    return create_common(p, state, state_bytes, aux, aux_bytes, st, true, host_rec, out);
}

// Longest run one quantum of the request loop may take: whole rings may be
// packed into one launch, whose sub-sweep count is 32 bits wide; windowed
// rings are cut into launches of K sub-sweeps anyway.
uint64_t sim_max_quantum_mcs(const asep_sim* s) {
    if (s->plan.seg) return ~0ull;
    return std::max<uint64_t>(1, kMaxLaunchSub / s->r.sc.S);
}

void sim_describe(const asep_sim* s, asep_params* resolved, asep_plan* plan) {
    *resolved = s->r.P;
    fill_plan(s->plan, plan);
}
hipStream_t sim_stream(const asep_sim* s) { return s->stream; }
void sim_set_stream(asep_sim* s, hipStream_t st) {
    if (!s->own_stream) s->stream = st;
}
uint32_t sim_samples(const asep_sim* s) { return s->r.P.samples; }
uint64_t sim_attempts_per_mcs(const asep_sim* s) {
    return (uint64_t)s->r.P.samples * s->r.P.L * (s->r.planes == 2 ? 4 : 1);
}

// Queue the work advancing to t_end and measuring at times[0..n) (n <= the
// record capacity, every time in [asep_time, t_end]); the records are copied
// asynchronously to host_out (n x samples).
int sim_run_async(asep_sim* s, const uint64_t* times, uint32_t n, uint64_t t_end,
                  Record* host_out) {
    if (n > s->rec_cap || t_end < s->t) return ASEP_E_INVAL;
    return enqueue_to(s, t_end, times, n, host_out);
}

void record_to_rough(const asep_sim* s, const Record& rc, asep_rough* o) { fill_rough(s->r, rc, o); }

// Packing: whole-ring simulations of the small shapes can share a launch
// with other simulations of the same kernel and workgroup size.
bool sim_pack_info(const asep_sim* s, PackInfo* pi) {
    const Plan& pl = s->plan;
    pi->kern = pl.kern;
    pi->block = pl.block;
    pi->lds = pl.lds;
    pi->grid = pl.grid;
    return !pl.seg && pl.kern.C <= 4;
}

// Descriptor advancing the simulation to t_end with measurements at
// times[0..n) (n <= the record capacity); wg_begin is left to the caller.
int sim_pack_prepare(asep_sim* s, uint64_t t_end, const uint64_t* times, uint32_t n,
                     SimDesc* d) {
    if (s->plan.seg || n > s->rec_cap || t_end < s->t) return ASEP_E_INVAL;
    const uint32_t S = s->r.sc.S;
    if ((t_end - s->t) * S > kMaxLaunchSub) return ASEP_E_INVAL;  // one launch
    *d = make_desc(s);
    for (uint32_t i = 0; i < n; ++i) d->rec_g[i] = times[i] * S;
    d->g0 = s->t * S;
    d->g1 = t_end * S;
    d->n_rec = n;
    return ASEP_OK;
}

// After the packed launch: the clock moves to t_end and the records are
// copied to host_out on the launch's stream.
int sim_pack_commit(asep_sim* s, uint64_t t_end, uint32_t n, Record* host_out, hipStream_t st) {
    s->t = t_end;
    if (n && host_out)
        HIP_OR_FAIL(hipMemcpyAsync(host_out, s->rec, sizeof(Record) * n * s->r.P.samples,
                                   hipMemcpyDeviceToHost, st));
    return ASEP_OK;
}

int device_error(hipError_t e, const char* where) { return device_fail(e, where); }

int sim_run_scratch(const asep_params* p, uint64_t* state, size_t state_bytes, hipStream_t st,
                    void* scratch, size_t scratch_bytes, const uint64_t* times, uint32_t n,
                    asep_rough* out_dev, RoughOut to_rough) {
    if (!state || !scratch || !to_rough || (n && (!times || !out_dev))) return ASEP_E_INVAL;
    asep_sim s;  // on this frame; its vectors stay empty (profiling is off)
    int rc = resolve(p, current_device(), &s.r);
    if (rc == ASEP_OK) rc = choose_plan(s.r, &s.plan);
    if (rc) return rc;
    const size_t need_state = (size_t)s.r.P.samples * s.r.planes * s.r.nw * 8;
    size_t o_masks, o_hops, o_rec, o_recg, o_alt, need_aux;
    aux_layout(s.r, s.plan, &o_masks, &o_hops, &o_rec, &o_recg, &o_alt, &need_aux);
    if (state_bytes < need_state) return ASEP_E_INVAL;
    if (need_aux > scratch_bytes) return ASEP_E_TOO_LARGE;
    unsigned char* a = (unsigned char*)scratch;
    s.stream = st;
    s.words = state;
    s.masks = s.r.mplanes ? (uint64_t*)(a + o_masks) : nullptr;
    s.hops = (int64_t*)(a + o_hops);
    s.rec = (Record*)(a + o_rec);
    s.alt = s.plan.seg ? (uint64_t*)(a + o_alt) : nullptr;
    s.segs = (SegRec*)(a + seg_offset(s.r, s.plan, o_alt));
    s.rec_cap = kRecCap;
    rc = check_times(&s, times, n);
    if (rc) return rc;
    // every scratch region is rewritten before it is read: the quenched
    // planes and hop counters by the initialisation, the records by the
    // measurements, the second state buffer by the first window launch
    rc = sim_init(&s);
    if (rc) return rc;
    const uint32_t R = s.r.P.samples;
    for (uint32_t done = 0; done < n;) {
        const uint32_t m = std::min(kRecCap, n - done);
        rc = enqueue_to(&s, times[done + m - 1], times + done, m, nullptr);
        if (rc) return rc;
        HIP_OR_FAIL(to_rough(s.rec, out_dev + (size_t)done * R, m * R, s.r.P.L, st));
        done += m;
    }
    return ASEP_OK;
}

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
        case ASEP_E_TOO_LARGE:
            return "run needs more scratch than the fixed no-allocation workspace holds";
        default: return "unknown error";
    }
}

extern "C" const char* asep_last_device_error(void) { return g_last_device_error.c_str(); }
