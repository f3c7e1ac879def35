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

// Sums of heights inside one word relative to the height at its first site
// (as word_moments), in 32-bit arithmetic: |d| <= 64, |e1| <= 2016,
// e2 <= 64^3.
__device__ __forceinline__ void word_moments32(uint64_t word, const int32_t* tab1,
                                               const int32_t* tab2, int32_t& e1, int32_t& e2) {
    int32_t d = 0;
    e1 = 0;
    e2 = 0;
#pragma unroll
    for (int by = 0; by < 8; ++by) {
        const uint32_t byte = (uint32_t)(word >> (8 * by)) & 255u;
        const int32_t t1 = tab1[byte];
        e1 += 8 * d + t1;
        e2 += 8 * d * d + 2 * d * t1 + tab2[byte];
        d += 8 - 2 * __popc(byte);
    }
}

// Measurement of rings held in HBM, pass 1: one wave per segment of `seg`
// words (segment s of ring r is words [s seg, (s+1) seg) of the ring).  The
// wave walks its segment in slabs of 128 words, each lane loading two
// consecutive words with one 16-byte load (coalesced), a wave scan of the
// per-word height steps 64 - 2 popcount giving each word's start height;
// the byte tables give the in-word sums.  Heights are relative to the
// segment's start, so a segment's S2 stays below 2^60 (2^20 sites of height
// below 2^20).
__global__ __launch_bounds__(256) void k_rough_seg(const uint64_t* __restrict__ words,
                                                   uint32_t planes, uint32_t nw, uint32_t seg,
                                                   uint32_t nseg, uint32_t total,
                                                   SegRec* __restrict__ out) {
    __shared__ int32_t tab1[256], tab2[256];
    build_byte_tables(tab1, tab2);
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t gs = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (gs >= total) return;  // whole waves; no barrier follows
    const uint32_t ring = gs / nseg, sg = gs - ring * nseg;
    const uint32_t w0 = sg * seg, w1 = min(nw, w0 + seg);
    const uint64_t* wa = words + (size_t)ring * planes * nw;
    int32_t carry = 0;
    int64_t s1 = 0, n = 0;
    uint64_t s2 = 0;
    for (uint32_t b = w0; b < w1; b += 128) {
        const uint32_t i0 = b + 2u * lane;
        const bool v0 = i0 < w1, v1 = i0 + 1 < w1;
        uint64_t x0 = 0, x1 = 0;
        if (v1 && ((((size_t)ring * planes * nw + i0) & 1u) == 0)) {
            const ulonglong2 q = *reinterpret_cast<const ulonglong2*>(wa + i0);
            x0 = q.x;
            x1 = q.y;
        } else {
            if (v0) x0 = wa[i0];
            if (v1) x1 = wa[i0 + 1];
        }
        n += __popcll(x0) + __popcll(x1);
        if (planes > 1) {
            if (v0) n += __popcll(wa[nw + i0]);
            if (v1) n += __popcll(wa[nw + i0 + 1]);
        }
        const int32_t d0 = v0 ? 64 - 2 * (int32_t)__popcll(x0) : 0;
        const int32_t d1 = v1 ? 64 - 2 * (int32_t)__popcll(x1) : 0;
        // inclusive wave scan of the lane's two steps
        const int32_t t = d0 + d1;
        int32_t inc = t;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int32_t y = __shfl_up(inc, o, 64);
            if ((int)lane >= o) inc += y;
        }
        const int32_t h0 = carry + inc - t, h1 = h0 + d0;
        int32_t e1, e2;
        if (v0) {
            word_moments32(x0, tab1, tab2, e1, e2);
            s1 += 64 * (int64_t)h0 + e1;
            s2 += (uint64_t)(64 * (int64_t)h0 * h0 + 2 * (int64_t)h0 * e1 + e2);
        }
        if (v1) {
            word_moments32(x1, tab1, tab2, e1, e2);
            s1 += 64 * (int64_t)h1 + e1;
            s2 += (uint64_t)(64 * (int64_t)h1 * h1 + 2 * (int64_t)h1 * e1 + e2);
        }
        carry += __shfl(inc, 63, 64);
    }
    // wave sums (every lane ends with the totals)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        s1 += (int64_t)__shfl_xor((long long)s1, o, 64);
        s2 += (uint64_t)__shfl_xor((unsigned long long)s2, o, 64);
        n += (int64_t)__shfl_xor((long long)n, o, 64);
    }
    if (lane == 0) {
        SegRec r;
        r.d = carry;
        r.s1 = s1;
        r.s2 = s2;
        r.n = n;
        out[gs] = r;
    }
}

// Pass 2, one workgroup per ring: segment start heights from an exclusive
// scan of the segments' height changes, then the exact ring sums
//   S1 = sum (s1 + M H),  S2 = sum (s2 + 2 H s1 + M H^2)
// (M sites in a segment starting at height H), S2 in 128 bits.
__global__ __launch_bounds__(256) void k_rough_combine(const SegRec* __restrict__ segs,
                                                       uint32_t nseg, uint32_t seg, uint32_t nw,
                                                       const int64_t* __restrict__ hops,
                                                       Record* __restrict__ rec) {
    __shared__ int64_t sc[256];
    __shared__ unsigned long long rlo[256];
    __shared__ long long rhi[256], rs1[256], rn[256];
    const uint32_t ring = blockIdx.x, tid = threadIdx.x;
    const SegRec* sr = segs + (size_t)ring * nseg;
    const uint32_t per = (nseg + blockDim.x - 1) / blockDim.x;
    const uint32_t a = min(nseg, tid * per), z = min(nseg, a + per);
    int64_t dsum = 0;
    for (uint32_t i = a; i < z; ++i) dsum += sr[i].d;
    sc[tid] = dsum;
    __syncthreads();
    for (uint32_t o = 1; o < blockDim.x; o <<= 1) {
        const int64_t v = sc[tid] + (tid >= o ? sc[tid - o] : 0);
        __syncthreads();
        sc[tid] = v;
        __syncthreads();
    }
    int64_t H = sc[tid] - dsum;
    __int128 S2 = 0;
    int64_t S1 = 0, N = 0;
    for (uint32_t i = a; i < z; ++i) {
        const SegRec r = sr[i];
        const int64_t M = 64 * (int64_t)(min(nw, (i + 1) * seg) - i * seg);
        S1 += r.s1 + M * H;
        S2 += (__int128)r.s2 + 2 * (__int128)H * r.s1 + (__int128)M * H * H;
        N += r.n;
        H += r.d;
    }
    rlo[tid] = (unsigned long long)(uint64_t)S2;
    rhi[tid] = (long long)(int64_t)(S2 >> 64);
    rs1[tid] = S1;
    rn[tid] = N;
    __syncthreads();
    for (uint32_t o = blockDim.x / 2; o > 0; o >>= 1) {
        if (tid < o) {
            const unsigned long long x = rlo[tid], y = rlo[tid + o];
            const unsigned long long t = x + y;
            rlo[tid] = t;
            rhi[tid] = rhi[tid] + rhi[tid + o] + (t < x ? 1 : 0);
            rs1[tid] += rs1[tid + o];
            rn[tid] += rn[tid + o];
        }
        __syncthreads();
    }
    if (tid == 0) {
        Record r;
        r.s1 = rs1[0];
        r.s2lo = rlo[0];
        r.s2hi = rhi[0];
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
                        uint32_t planes, uint32_t nw, SegRec* segs, hipStream_t st) {
    const uint32_t seg = rough_seg_words(R, nw);
    const uint32_t nseg = (nw + seg - 1) / seg;
    const uint32_t total = R * nseg;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_rough_seg, dim3((total + 3) / 4), dim3(256), 0, st, words, planes, nw,
                       seg, nseg, total, segs);
    hipLaunchKernelGGL(k_rough_combine, dim3(R), dim3(256), 0, st, segs, nseg, seg, nw, hops,
                       rec);
    return hipGetLastError();
}

}  // namespace asep
