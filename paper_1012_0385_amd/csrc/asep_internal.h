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
};

// One measurement of one ring (exact integers; W^2 is formed on the host).
struct Record {
    int64_t s1;
    uint64_t s2lo;
    int64_t s2hi;
    int64_t hops;
    int64_t n;
};

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
    uint64_t T_init, T_slow, T_turn;  // 32-bit-draw thresholds (may equal 2^32)
};

enum Model : uint32_t { kPlain = 0, kDisorder = 1, kTwoLane = 2 };

// Arguments of the register-resident ring kernel.
struct RingArgs {
    uint64_t* words;          // [R][planes][nw]
    const uint64_t* masks;    // [realizations][mplanes][nw] or null
    int64_t* hops;            // [R]
    Record* rec;              // [n_rec][R] or null
    const uint64_t* rec_t;    // [n_rec] absolute MCS, ascending, in [t0, t1]
    uint32_t n_rec;
    uint64_t t0, t1;
    uint32_t R, nw, planes, mplanes;
    uint32_t lanes_per_ring;  // lanes serving one ring
    uint32_t rings_per_wg;
    uint32_t key0, key1, sample0, spd;
    uint32_t real0;           // first realisation held in masks
    Sched sc;
};

// Host-side launch helpers implemented in asep_kernels.hip.
hipError_t launch_init_state(uint64_t* words, uint32_t R, uint32_t planes, uint32_t nw,
                             uint32_t init, uint64_t T_init, uint32_t key0, uint32_t key1,
                             uint32_t sample0, hipStream_t st);
hipError_t launch_init_masks(uint64_t* masks, uint32_t n_real, uint32_t mplanes,
                             const uint32_t* tags, uint32_t nw, uint64_t T, uint32_t key0,
                             uint32_t key1, uint32_t real0, hipStream_t st);
// C slots (64-bit words) per lane, model; dynamic LDS bytes in *lds.
hipError_t launch_ring(const RingArgs& a, uint32_t C, uint32_t model, uint32_t block,
                       uint32_t grid, size_t lds, hipStream_t st);
uint32_t ring_block_limit(uint32_t C);
size_t ring_lds_bytes(uint32_t block, uint32_t planes, uint32_t rings_per_wg, uint32_t mplanes,
                      uint32_t nw);
hipError_t launch_rough(const uint64_t* words, const int64_t* hops, Record* rec, uint32_t R,
                        uint32_t planes, uint32_t nw, hipStream_t st);

}  // namespace asep

// Internal hooks of the host library used by the request loop.
struct asep_sim;
struct asep_rough;
namespace asep {
uint32_t sim_record_capacity(const asep_sim* s);
hipStream_t sim_stream(const asep_sim* s);
uint32_t sim_samples(const asep_sim* s);
uint64_t sim_attempts_per_mcs(const asep_sim* s);
int sim_run_async(asep_sim* s, const uint64_t* times_pinned, uint32_t n, uint64_t t_end,
                  Record* host_out);
void record_to_rough(const asep_sim* s, const Record& rc, asep_rough* o);
int device_error(hipError_t e, const char* where);
}  // namespace asep
