// asep_kernels.hip -- gfx950 kernels of the ASEP / KPZ lattice-gas engine.
//
// State layout in HBM: uint64 words, site 64w+b at bit b of word w, planes
// (lane A, lane B) contiguous per ring, rings contiguous:
//   words[(ring * planes + plane) * nw + w].
//
// Initialisation and measurement kernels, and the dispatch of the sweep
// kernel (asep_device.h, instantiated per model in asep_sweep_*.hip).
//
// The sweep kernel keeps each ring resident in VGPRs for the whole launch:
// lane t of a ring owns C consecutive 64-bit "slots".  A slot is 64
// consecutive sites starting at sig + 64 (off + index) (mod L), where sig is
// the shift of the current sub-sweep (Sec. 2.1's sub-lattice split, here a
// randomly shifted decomposition into cells of ell <= 64 sites).  Moving to
// the next sub-sweep's shift only needs each slot's successor, so a lane
// trades one word with its neighbour per sub-sweep through LDS; all attempts
// then run in registers on cells that never straddle two slots.  Quenched
// planes (Eq. bimodal slow sites, Sec. 3 turning points) are read-only and
// staged whole in LDS.  Heights and the exact sums of Eq. W are formed at
// the measurement times inside the same launch.
//
// Random numbers: Philox4x32-10 (Salmon et al., SC'11) keyed by (seed,
// stream); counters:
//   attempt: (cell k, lo32(g), 1<<28 | blk<<16 | hi16(g), sample)
//   shift:   (0, lo32(g/4), 2<<28 | hi16(g/4), sample), word g mod 4
//   init:    (site/4, lane, 3<<28, sample), word site mod 4
//   masks:   (site/4, 0, tag<<28, realization), word site mod 4
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "asep_device.h"

namespace asep {

namespace {

using dev::Blk;
using dev::build_byte_tables;
using dev::philox;
using dev::word_moments;

// Word of 64 per-site Bernoulli draws: site 64w+i uses word i%4 of the block
// at counter (16w + i/4, c1, tag << 28, c3).
__device__ __forceinline__ uint64_t bernoulli_word(uint32_t w, uint32_t c1, uint32_t tag,
                                                   uint32_t c3, uint64_t T, uint32_t k0,
                                                   uint32_t k1) {
    uint64_t v = 0;
    for (uint32_t blk = 0; blk < 16; ++blk) {
        const Blk r = philox(w * 16u + blk, c1, tag << 28, c3, k0, k1);
#pragma unroll
        for (int i = 0; i < 4; ++i)
            v |= (uint64_t)((uint64_t)r.v[i] < T) << (blk * 4u + (uint32_t)i);
    }
    return v;
}

__global__ void k_init_state(uint64_t* __restrict__ words, uint32_t R, uint32_t planes,
                             uint32_t nw, uint32_t init, uint64_t T, uint32_t k0, uint32_t k1,
                             uint32_t sample0) {
    const uint64_t total = (uint64_t)R * planes * nw;
    for (uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; gid < total;
         gid += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t w = (uint32_t)(gid % nw);
        const uint32_t plane = (uint32_t)((gid / nw) % planes);
        const uint32_t ring = (uint32_t)(gid / ((uint64_t)nw * planes));
        uint64_t v;
        if (init == 0)
            v = 0x5555555555555555ull;  // flat: site x occupied iff x is even
        else
            v = bernoulli_word(w, plane, kTagInit, sample0 + ring, T, k0, k1);
        words[gid] = v;
    }
}

__global__ void k_init_masks(uint64_t* __restrict__ masks, uint32_t n_real, uint32_t mplanes,
                             uint32_t tag0, uint32_t tag1, uint32_t nw, uint64_t T, uint32_t k0,
                             uint32_t k1, uint32_t real0) {
    const uint64_t total = (uint64_t)n_real * mplanes * nw;
    for (uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; gid < total;
         gid += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t w = (uint32_t)(gid % nw);
        const uint32_t plane = (uint32_t)((gid / nw) % mplanes);
        const uint32_t real = (uint32_t)(gid / ((uint64_t)nw * mplanes));
        masks[gid] = bernoulli_word(w, 0, plane == 0 ? tag0 : tag1, real0 + real, T, k0, k1);
    }
}

// Measurement of rings resident in HBM: one workgroup per ring.  Each lane
// takes a contiguous run of words; an exclusive scan of the per-word height
// steps 64 - 2 popcount gives the height at every word start, then the byte
// tables give the in-word sums.  S2 is accumulated in 128 bits.
__global__ __launch_bounds__(256) void k_rough(const uint64_t* __restrict__ words,
                                               const int64_t* __restrict__ hops,
                                               Record* __restrict__ rec, uint32_t planes,
                                               uint32_t nw) {
    __shared__ int32_t tab1[256], tab2[256];
    __shared__ int64_t sc[256];
    __shared__ unsigned long long rlo[256], rhi[256];
    __shared__ long long rs1[256], rn[256];
    const uint32_t ring = blockIdx.x;
    const uint32_t tid = threadIdx.x;
    build_byte_tables(tab1, tab2);
    const uint64_t* wa = words + (size_t)ring * planes * nw;
    const uint32_t per = (nw + blockDim.x - 1) / blockDim.x;
    const uint32_t w0 = min(nw, tid * per), w1 = min(nw, w0 + per);
    int64_t dsum = 0, n = 0;
    for (uint32_t w = w0; w < w1; ++w) {
        const uint64_t x = wa[w];
        dsum += 64 - 2 * (int64_t)__popcll(x);
        n += __popcll(x);
        if (planes > 1) n += __popcll(wa[nw + w]);
    }
    sc[tid] = dsum;
    __syncthreads();
    for (uint32_t d = 1; d < blockDim.x; d <<= 1) {
        const int64_t v = sc[tid] + (tid >= d ? sc[tid - d] : 0);
        __syncthreads();
        sc[tid] = v;
        __syncthreads();
    }
    int64_t H = sc[tid] - dsum;
    int64_t s1 = 0;
    unsigned long long lo = 0, hi = 0;
    for (uint32_t w = w0; w < w1; ++w) {
        const uint64_t x = wa[w];
        int64_t e1, e2;
        word_moments(x, tab1, tab2, e1, e2);
        s1 += 64 * H + e1;
        const uint64_t add = (uint64_t)(64 * H * H + 2 * H * e1 + e2);
        lo += add;
        hi += (lo < add) ? 1u : 0u;
        H += 64 - 2 * (int64_t)__popcll(x);
    }
    rlo[tid] = lo;
    rhi[tid] = hi;
    rs1[tid] = s1;
    rn[tid] = n;
    __syncthreads();
    for (uint32_t d = blockDim.x / 2; d > 0; d >>= 1) {
        if (tid < d) {
            const unsigned long long a = rlo[tid], b = rlo[tid + d];
            const unsigned long long s = a + b;
            rlo[tid] = s;
            rhi[tid] = rhi[tid] + rhi[tid + d] + (s < a ? 1u : 0u);
            rs1[tid] += rs1[tid + d];
            rn[tid] += rn[tid + d];
        }
        __syncthreads();
    }
    if (tid == 0) {
        Record r;
        r.s1 = rs1[0];
        r.s2lo = rlo[0];
        r.s2hi = (int64_t)rhi[0];
        r.hops = hops[ring];
        r.n = rn[0];
        rec[ring] = r;
    }
}

__global__ void k_zero_u64(uint64_t* __restrict__ words, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        words[i] = 0;
}

}  // namespace

hipError_t launch_zero_u64(uint64_t* words, uint64_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    const uint32_t block = 256;
    const uint64_t want = (n + block - 1) / block;
    const uint32_t grid = (uint32_t)(want < 4096 ? want : 4096);
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_zero_u64, dim3(grid), dim3(block), 0, st, words, n);
    return hipGetLastError();
}

hipError_t launch_init_state(uint64_t* words, uint32_t R, uint32_t planes, uint32_t nw,
                             uint32_t init, uint64_t T_init, uint32_t key0, uint32_t key1,
                             uint32_t sample0, hipStream_t st) {
    const uint64_t total = (uint64_t)R * planes * nw;
    const uint32_t block = 256;
    const uint64_t want = (total + block - 1) / block;
    const uint32_t grid = (uint32_t)(want < 65536 ? (want ? want : 1) : 65536);
    (void)hipGetLastError();  // drop errors left by earlier, unrelated calls
    hipLaunchKernelGGL(k_init_state, dim3(grid), dim3(block), 0, st, words, R, planes, nw, init,
                       T_init, key0, key1, sample0);
    return hipGetLastError();
}

hipError_t launch_init_masks(uint64_t* masks, uint32_t n_real, uint32_t mplanes,
                             const uint32_t* tags, uint32_t nw, uint64_t T, uint32_t key0,
                             uint32_t key1, uint32_t real0, hipStream_t st) {
    const uint64_t total = (uint64_t)n_real * mplanes * nw;
    const uint32_t block = 256;
    const uint64_t want = (total + block - 1) / block;
    const uint32_t grid = (uint32_t)(want < 65536 ? (want ? want : 1) : 65536);
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_init_masks, dim3(grid), dim3(block), 0, st, masks, n_real, mplanes,
                       tags[0], mplanes > 1 ? tags[1] : tags[0], nw, T, key0, key1, real0);
    return hipGetLastError();
}

uint32_t sweep_block_limit(uint32_t C, uint32_t model) {
    return dev::sweep_max_block((int)C, (int)model);
}

size_t sweep_lds_bytes(uint32_t block, uint32_t planes, uint32_t G, uint32_t mplanes,
                       uint32_t mwords) {
    size_t a, b, c, d, e;
    return dev::sweep_lds_layout(block, planes, G, mplanes, mwords, &a, &b, &c, &d, &e);
}

bool sweep_variant_compiled(uint32_t C, uint32_t model, uint32_t variant) {
    return dev::variant_compiled(C, model, variant);
}

hipError_t launch_sweep(const SweepKernel& k, const SimDesc& one, const SimDesc* descs,
                        uint32_t n_desc, uint32_t grid, uint32_t block, size_t lds,
                        hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
    switch (k.model) {
        case kPlain:
            return launch_sweep_plain(k, one, descs, n_desc, grid, block, lds, st, ev0, ev1);
        case kDisorder:
            return launch_sweep_disorder(k, one, descs, n_desc, grid, block, lds, st, ev0, ev1);
        case kTwoLane:
            return launch_sweep_two_lane(k, one, descs, n_desc, grid, block, lds, st, ev0, ev1);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_rough(const uint64_t* words, const int64_t* hops, Record* rec, uint32_t R,
                        uint32_t planes, uint32_t nw, hipStream_t st) {
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_rough, dim3(R), dim3(256), 0, st, words, hops, rec, planes, nw);
    return hipGetLastError();
}

}  // namespace asep
