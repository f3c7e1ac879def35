// asep_internal.h -- structures shared by the host library and the gfx950
// kernels of the ASEP engine (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace asep {

// Counter tags, top nibble of Philox counter word 2.
enum : uint32_t {
    kTagAttempt = 1,
    kTagShift = 2,
    kTagInit = 3,
    kTagDisP = 4,
    kTagDisQ = 5,
    kTagTurn = 6,
    kTagSublattice = 8,
    kTagChange = 9,
};

// One measurement of one ring (exact integers; W^2 is formed on the host).
struct Record {
    int64_t s1;
    uint64_t s2lo;
    int64_t s2hi;
    int64_t hops;
    int64_t n;
};

// Measurement of rings held in HBM: each ring is cut into segments of
// `seg` words, each summed by one wave relative to its own start height
// (d = height change, s1 and s2 = sums of heights and squared heights,
// n = particles), then combined per ring in exact 128-bit arithmetic.
struct SegRec {
    int64_t d;
    int64_t s1;
    uint64_t s2;
    int64_t n;
};

// Segment length in words: a power of two from 128 to 16384, the smallest
// that keeps the segments of all rings at most 4096 (enough waves to keep
// HBM busy, few enough for the per-ring combine).
inline uint32_t rough_seg_words(uint32_t R, uint32_t nw) {
    uint32_t seg = 128;
    while (seg < 16384 && (uint64_t)R * ((nw + seg - 1) / seg) > 4096) seg <<= 1;
    return seg;
}
inline size_t rough_seg_bytes(uint32_t R, uint32_t nw) {
    const uint32_t seg = rough_seg_words(R, nw);
    return sizeof(SegRec) * (size_t)R * ((nw + seg - 1) / seg);
}

// The lowered update rule: cell size, sub-sweeps, draw packing, thresholds.
struct Sched {
    uint32_t lam;   // log2 of the cell size ell
    uint32_t S;     // sub-sweeps per MCS
    uint32_t a;     // attempts per cell per sub-sweep
    uint32_t b;     // bits compared with a threshold
    uint32_t w;     // bits per attempt field
    uint32_t A;     // attempt fields per 32-bit word
    uint32_t nblk;  // Philox blocks per cell per sub-sweep
    uint32_t T[4];  // ring {p, q, r p, r q}; two lanes {A hop, B hop, lane change}
    uint32_t bc;    // two lanes, shifted schedule: bits of a lane-change draw compared
                    // with T[2] (0: T[2] is 0 = never or 1 = always)
    uint32_t jlow;  // fields are the bytes of a word, position in the low bits
                    // (cells of 32 sites whose field fits in 8 bits)
    uint64_t T_init, T_slow, T_turn;  // 32-bit-draw thresholds (may equal 2^32)
};

enum Model : uint32_t { kPlain = 0, kDisorder = 1, kTwoLane = 2 };

// Measurement points one launch can hold (they travel in the kernel arguments).
constexpr uint32_t kRecPerLaunch = 64;

// Work of one simulation inside one sweep launch.
struct SimDesc {
    uint64_t* words_in;       // [R][planes][nw] state read by the launch
    uint64_t* words_out;      // state written (== words_in for whole rings)
    const uint64_t* masks;    // [realisations][mplanes][nw], first = real0
    int64_t* hops;            // [R]
    Record* rec;              // [n_rec][R] (whole rings only)
    uint64_t g0, g1;          // sub-sweeps [g0, g1) of this launch
    uint32_t n_rec;
    uint32_t R, nw, planes, mplanes;
    uint32_t lanes_per_ring;  // lanes serving one ring (whole rings) or one window
    uint32_t rings_per_wg;    // whole rings packed per workgroup (1 for windows)
    uint32_t segs;            // windows per ring (1 = whole ring, periodic)
    uint32_t seg_n;           // output words per window
    uint32_t halo;            // words of context on each side of a window
    uint32_t nslot;           // slots of a window (seg_n + 2 halo)
    uint32_t key0, key1, sample0, spd, real0;
    uint32_t wg_begin;        // first workgroup of this simulation in a batched launch
    Sched sc;
    uint64_t rec_g[kRecPerLaunch];  // sub-sweep indices of the measurements, in [g0, g1]
};

// Host-side launch helpers implemented in the .hip translation units.
hipError_t launch_init_state(uint64_t* words, uint32_t R, uint32_t planes, uint32_t nw,
                             uint32_t init, uint64_t T_init, uint32_t key0, uint32_t key1,
                             uint32_t sample0, hipStream_t st);
hipError_t launch_init_masks(uint64_t* masks, uint32_t n_real, uint32_t mplanes,
                             const uint32_t* tags, uint32_t nw, uint64_t T, uint32_t key0,
                             uint32_t key1, uint32_t real0, hipStream_t st);
hipError_t launch_rough(const uint64_t* words, const int64_t* hops, Record* rec, uint32_t R,
                        uint32_t planes, uint32_t nw, SegRec* segs, hipStream_t st);
// words[0 .. n) = 0 (a kernel, not a memset node).
hipError_t launch_zero_u64(uint64_t* words, uint64_t n, hipStream_t st);

// Sweep launch: `one` describes the whole launch when descs == nullptr;
// otherwise descs[0..n_desc) (device memory, sorted by wg_begin) do.  With
// ev0 and ev1 (single-simulation launches only) the dispatch itself records
// the kernel's start and end in them.
struct SweepKernel {
    uint32_t C, model, variant;
    bool q0;
};
hipError_t launch_sweep(const SweepKernel& k, const SimDesc& one, const SimDesc* descs,
                        uint32_t n_desc, uint32_t grid, uint32_t block, size_t lds,
                        hipStream_t st, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
hipError_t launch_sweep_plain(const SweepKernel& k, const SimDesc& one, const SimDesc* descs,
                              uint32_t n_desc, uint32_t grid, uint32_t block, size_t lds,
                              hipStream_t st, hipEvent_t ev0, hipEvent_t ev1);
hipError_t launch_sweep_disorder(const SweepKernel& k, const SimDesc& one, const SimDesc* descs,
                                 uint32_t n_desc, uint32_t grid, uint32_t block, size_t lds,
                                 hipStream_t st, hipEvent_t ev0, hipEvent_t ev1);
hipError_t launch_sweep_two_lane(const SweepKernel& k, const SimDesc& one, const SimDesc* descs,
                                 uint32_t n_desc, uint32_t grid, uint32_t block, size_t lds,
                                 hipStream_t st, hipEvent_t ev0, hipEvent_t ev1);
uint32_t sweep_block_limit(uint32_t C, uint32_t model);
size_t sweep_lds_bytes(uint32_t block, uint32_t planes, uint32_t rings_per_wg, uint32_t mplanes,
                       uint32_t mwords);
bool sweep_variant_compiled(uint32_t C, uint32_t model, uint32_t variant);

}  // namespace asep

// Internal hooks of the host library used by the request loop.
struct asep_sim;
struct asep_rough;
struct asep_params;
struct asep_plan;
namespace asep {
uint32_t sim_record_capacity(const asep_sim* s);
size_t sim_host_rec_bytes(const asep_params& p);
int sim_buffer_sizes_on(const asep_params* p, int dev, size_t* state_bytes, size_t* aux_bytes);
int sim_create_borrowed(const asep_params* p, void* state, size_t state_bytes, void* aux,
                        size_t aux_bytes, hipStream_t st, Record* host_rec, asep_sim** out);
uint64_t sim_max_quantum_mcs(const asep_sim* s);
void sim_describe(const asep_sim* s, asep_params* resolved, asep_plan* plan);
hipStream_t sim_stream(const asep_sim* s);
// A borrowed simulation's next work goes to `st` (its earlier work must be
// complete: nothing orders the two streams).
void sim_set_stream(asep_sim* s, hipStream_t st);
uint32_t sim_samples(const asep_sim* s);
uint64_t sim_attempts_per_mcs(const asep_sim* s);
int sim_run_async(asep_sim* s, const uint64_t* times_pinned, uint32_t n, uint64_t t_end,
                  Record* host_out);
void record_to_rough(const asep_sim* s, const Record& rc, asep_rough* o);
struct PackInfo {
    SweepKernel kern;
    uint32_t block, grid;
    size_t lds;
};
bool sim_pack_info(const asep_sim* s, PackInfo* pi);
int sim_pack_prepare(asep_sim* s, uint64_t t_end, const uint64_t* times, uint32_t n,
                     SimDesc* d);
int sim_pack_commit(asep_sim* s, uint64_t t_end, uint32_t n, Record* host_out, hipStream_t st);
int device_error(hipError_t e, const char* where);
// A whole run (initialisation, then advance and measure through times[0..n))
// on the caller's state buffer and stream, with every other buffer carved
// from `scratch` (scratch_bytes long); nothing is allocated.  Records go to
// `out_dev` (device memory, n x samples asep_rough) through the device
// conversion `to_rough`.  ASEP_E_TOO_LARGE if the run needs more scratch.
typedef hipError_t (*RoughOut)(const Record* rec, asep_rough* out, uint32_t n, uint64_t L,
                               hipStream_t st);
int sim_run_scratch(const asep_params* p, uint64_t* state, size_t state_bytes, hipStream_t st,
                    void* scratch, size_t scratch_bytes, const uint64_t* times, uint32_t n,
                    asep_rough* out_dev, RoughOut to_rough);
}  // namespace asep
