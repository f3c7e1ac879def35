// asep_kernels.hip -- gfx950 kernels of the ASEP / KPZ lattice-gas engine.
//
// State layout in HBM: uint64 words, site 64w+b at bit b of word w, planes
// (lane A, lane B) contiguous per ring, rings contiguous:
//   words[(ring * planes + plane) * nw + w].
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

#include "asep_internal.h"

namespace asep {

namespace {

constexpr uint32_t kMulA = 0xD2511F53u;
constexpr uint32_t kMulB = 0xCD9E8D57u;
constexpr uint32_t kWeylA = 0x9E3779B9u;
constexpr uint32_t kWeylB = 0xBB67AE85u;

struct Blk {
    uint32_t v[4];
};

// Ten Philox rounds: products of counter words 0 and 2, high halves mixed
// with the other two words and the round key, Weyl key schedule.
__device__ __forceinline__ Blk philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                      uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        const uint64_t pa = (uint64_t)kMulA * (uint64_t)c0;
        const uint64_t pb = (uint64_t)kMulB * (uint64_t)c2;
        const uint32_t n0 = (uint32_t)(pb >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(pa >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)pb;
        c3 = (uint32_t)pa;
        c0 = n0;
        c2 = n2;
        k0 += kWeylA;
        k1 += kWeylB;
    }
    Blk b;
    b.v[0] = c0;
    b.v[1] = c1;
    b.v[2] = c2;
    b.v[3] = c3;
    return b;
}

// 64 sites starting `sh` bits into `lo`, continuing into `hi`; sh in [0, 63].
__device__ __forceinline__ uint64_t funnel(uint64_t lo, uint64_t hi, uint32_t sh) {
    return (lo >> sh) | ((hi << 1) << (63u - sh));
}

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

// Sums of heights inside one word, relative to the height at its first site:
// E1 = sum_q d_q, E2 = sum_q d_q^2 with d_0 = 0, d_{q+1} = d_q + 1 - 2 n_q.
// tab1/tab2 hold the same sums for single bytes.
__device__ __forceinline__ void word_moments(uint64_t word, const int32_t* tab1,
                                             const int32_t* tab2, int64_t& e1, int64_t& e2) {
    int64_t d = 0;
    e1 = 0;
    e2 = 0;
#pragma unroll
    for (int by = 0; by < 8; ++by) {
        const uint32_t byte = (uint32_t)(word >> (8 * by)) & 255u;
        const int64_t t1 = tab1[byte];
        e1 += 8 * d + t1;
        e2 += 8 * d * d + 2 * d * t1 + tab2[byte];
        d += 8 - 2 * (int64_t)__popc(byte);
    }
}

__device__ void build_byte_tables(int32_t* tab1, int32_t* tab2) {
    for (uint32_t v = threadIdx.x; v < 256; v += blockDim.x) {
        int32_t e = 0, s = 0, s2 = 0;
        for (int q = 0; q < 8; ++q) {
            s += e;
            s2 += e * e;
            e += 1 - 2 * (int32_t)((v >> q) & 1u);
        }
        tab1[v] = s;
        tab2[v] = s2;
    }
}

// Dynamic LDS of the ring kernel, in this order:
//   xch   [2][block][planes] uint64  neighbour exchange, double-buffered
//   mask  [rings_per_wg][mplanes][nw] uint64
//   red   [rings_per_wg][4] uint64     per-ring reductions
//   scan  [2][block] int32
//   tab   [2][256] int32
//   g0    [rings_per_wg] int32
__host__ __device__ inline size_t lds_layout(uint32_t block, uint32_t planes, uint32_t G,
                                             uint32_t mplanes, uint32_t nw, size_t* o_mask,
                                             size_t* o_red, size_t* o_scan, size_t* o_tab,
                                             size_t* o_g0) {
    size_t off = (size_t)2 * block * planes * 8;
    *o_mask = off;
    off += (size_t)G * mplanes * nw * 8;
    *o_red = off;
    off += (size_t)G * 4 * 8;
    *o_scan = off;
    off += (size_t)2 * block * 4;
    *o_tab = off;
    off += 2 * 256 * 4;
    *o_g0 = off;
    off += (size_t)G * 4;
    return (off + 15) & ~(size_t)15;
}

// Largest workgroup for C slots per lane: more slots need more VGPRs.
// (gfx950: 512 VGPRs per SIMD lane; a 512-lane workgroup is 2 waves per SIMD,
// so C = 8 and 16 may use up to 256 VGPRs.)
__host__ __device__ constexpr uint32_t ring_max_block(int C) {
    return C <= 2 ? 1024u : 512u;
}

template <int C, int MODEL>
__global__ __launch_bounds__(ring_max_block(C)) void k_ring(RingArgs P) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int NPL = (MODEL == kTwoLane) ? 2 : 1;

    const uint32_t tid = threadIdx.x;
    const uint32_t block = blockDim.x;
    const uint32_t Tr = P.lanes_per_ring;
    const uint32_t G = P.rings_per_wg;
    const uint32_t gi = tid / Tr;
    const uint32_t lt = tid - gi * Tr;
    const uint32_t ring = blockIdx.x * G + gi;
    const bool ring_ok = (gi < G) && (ring < P.R);
    const uint32_t nw = P.nw;
    const uint32_t nact = (nw + C - 1) / C;
    const bool act = ring_ok && lt < nact;
    const uint32_t base_slot = lt * C;
    const int cnt = act ? (int)min((uint32_t)C, nw - base_slot) : 0;
    const uint32_t sample = P.sample0 + (ring_ok ? ring : 0);
    const uint32_t lane0 = gi * Tr;  // first lane of this ring in the block
    const uint32_t nxt = lane0 + ((lt + 1 < nact) ? lt + 1 : 0);

    size_t o_mask, o_red, o_scan, o_tab, o_g0;
    lds_layout(block, NPL, G, P.mplanes, nw, &o_mask, &o_red, &o_scan, &o_tab, &o_g0);
    uint64_t* xch = reinterpret_cast<uint64_t*>(smem);
    uint64_t* lmask = reinterpret_cast<uint64_t*>(smem + o_mask) +
                      (size_t)(gi < G ? gi : 0) * P.mplanes * nw;
    unsigned long long* red = reinterpret_cast<unsigned long long*>(smem + o_red);
    int32_t* scan = reinterpret_cast<int32_t*>(smem + o_scan);
    int32_t* tab1 = reinterpret_cast<int32_t*>(smem + o_tab);
    int32_t* tab2 = tab1 + 256;
    int32_t* g0s = reinterpret_cast<int32_t*>(smem + o_g0);

    const uint32_t lam = P.sc.lam;
    const uint32_t cmask = (1u << lam) - 1u;
    const uint32_t cps = 64u >> lam;  // cells per slot
    const uint32_t rb = P.sc.b;
    const uint32_t rmask = (rb >= 32) ? 0xFFFFFFFFu : ((1u << rb) - 1u);
    const uint32_t fw = P.sc.w;
    const uint32_t Aw = P.sc.A;
    const uint32_t na = P.sc.a;
    const uint32_t nblk = P.sc.nblk;
    const uint32_t T0 = P.sc.T[0], T1 = P.sc.T[1], T2 = P.sc.T[2], T3 = P.sc.T[3];
    const uint32_t k0 = P.key0, k1 = P.key1;

    uint64_t sa[C];
    uint64_t sb[C];
#pragma unroll
    for (int i = 0; i < C; ++i) {
        sa[i] = 0;
        sb[i] = 0;
        if (i < cnt) {
            const uint64_t* src = P.words + (size_t)ring * NPL * nw;
            sa[i] = src[base_slot + i];
            if (MODEL == kTwoLane) sb[i] = src[nw + base_slot + i];
        }
    }
    if (MODEL != kPlain && ring_ok) {
        const uint32_t real = sample / P.spd - P.real0;
        const uint64_t* msrc = P.masks + (size_t)real * P.mplanes * nw;
        for (uint32_t idx = lt; idx < P.mplanes * nw; idx += Tr) lmask[idx] = msrc[idx];
    }
    if (P.n_rec) build_byte_tables(tab1, tab2);
    __syncthreads();

    uint32_t sig = 0, off = 0, buf = 0;
    int64_t J = 0;
    const int64_t hops0 = ring_ok ? P.hops[ring] : 0;

    // Move every slot to the shift sig_new (neighbour exchange through LDS).
    auto shift_to = [&](uint32_t sig_new) {
        const uint32_t delta = (sig_new - sig) & 63u;
        const bool wrap = sig_new < sig;
        uint64_t* xb = xch + (size_t)buf * block * NPL;
        if (act) {
            xb[tid * NPL] = sa[0];
            if (MODEL == kTwoLane) xb[tid * NPL + 1] = sb[0];
        }
        __syncthreads();
        if (act) {
            const uint64_t na_ = xb[nxt * NPL];
            const uint64_t nb_ = (MODEL == kTwoLane) ? xb[nxt * NPL + 1] : 0;
#pragma unroll
            for (int i = 0; i < C; ++i) {
                if (i < cnt) {
                    uint64_t ha = na_, hb = nb_;
                    if (i + 1 < C && i + 1 < cnt) {
                        ha = sa[i + 1 < C ? i + 1 : i];
                        hb = sb[i + 1 < C ? i + 1 : i];
                    }
                    sa[i] = funnel(sa[i], ha, delta);
                    if (MODEL == kTwoLane) sb[i] = funnel(sb[i], hb, delta);
                }
            }
        }
        if (wrap) off = (off + 1 == nw) ? 0 : off + 1;
        sig = sig_new;
        buf ^= 1u;
    };

    // Heights and exact sums at the current time (slots must be at shift 0).
    auto measure = [&](uint32_t ri) {
        // slot base_slot+i holds word (off + base_slot + i) mod nw
        int32_t dl = 0;
#pragma unroll
        for (int i = 0; i < C; ++i)
            if (i < cnt) dl += 64 - 2 * (int32_t)__popcll(sa[i]);
        int32_t* s0 = scan;
        int32_t* s1 = scan + block;
        s0[tid] = dl;
        if (lt == 0 && gi < G) {
            red[gi * 4 + 0] = 0;
            red[gi * 4 + 1] = 0;
            red[gi * 4 + 2] = 0;
            red[gi * 4 + 3] = 0;
        }
        __syncthreads();
        for (uint32_t d = 1; d < block; d <<= 1) {
            const int32_t v = s0[tid] + (tid >= d ? s0[tid - d] : 0);
            __syncthreads();
            s1[tid] = v;
            __syncthreads();
            int32_t* t = s0;
            s0 = s1;
            s1 = t;
        }
        const int32_t before = (lane0 > 0) ? s0[lane0 - 1] : 0;
        const int32_t excl = s0[tid] - dl - before;
        const int32_t last = lane0 + Tr - 1 < block ? lane0 + Tr - 1 : block - 1;
        const int32_t gtot = s0[last] - before;
        const uint32_t i0 = (nw - off) % nw;  // slot holding word 0
        if (act && i0 >= base_slot && i0 < base_slot + (uint32_t)cnt) {
            int32_t g = excl;
#pragma unroll
            for (int i = 0; i < C; ++i)
                if ((uint32_t)i < i0 - base_slot) g += 64 - 2 * (int32_t)__popcll(sa[i]);
            g0s[gi] = g;
        }
        __syncthreads();
        int64_t ls1 = 0;
        uint64_t ls2 = 0;
        int64_t ln = 0;
        if (act) {
            const int32_t gz = g0s[gi];
            int32_t g = excl;
#pragma unroll
            for (int i = 0; i < C; ++i) {
                if (i < cnt) {
                    const uint32_t idx = base_slot + i;
                    const int64_t H = (idx >= i0) ? (int64_t)(g - gz) : (int64_t)(g + gtot - gz);
                    int64_t e1, e2;
                    word_moments(sa[i], tab1, tab2, e1, e2);
                    ls1 += 64 * H + e1;
                    ls2 += (uint64_t)(64 * H * H + 2 * H * e1 + e2);
                    ln += __popcll(sa[i]);
                    if (MODEL == kTwoLane) ln += __popcll(sb[i]);
                    g += 64 - 2 * (int32_t)__popcll(sa[i]);
                }
            }
        }
        if (act) {
            atomicAdd(&red[gi * 4 + 0], (unsigned long long)ls1);
            atomicAdd(&red[gi * 4 + 1], (unsigned long long)ls2);
            atomicAdd(&red[gi * 4 + 2], (unsigned long long)J);
            atomicAdd(&red[gi * 4 + 3], (unsigned long long)ln);
        }
        __syncthreads();
        if (ring_ok && lt == 0) {
            Record rc;
            rc.s1 = (int64_t)red[gi * 4 + 0];
            rc.s2lo = (uint64_t)red[gi * 4 + 1];
            rc.s2hi = 0;
            rc.hops = hops0 + (int64_t)red[gi * 4 + 2];
            rc.n = (int64_t)red[gi * 4 + 3];
            P.rec[(size_t)ri * P.R + ring] = rc;
        }
        __syncthreads();
    };

    uint32_t shblk[4] = {0, 0, 0, 0};
    uint64_t shq = ~0ull;
    const uint32_t S = P.sc.S;
    uint64_t t = P.t0;
    uint32_t ri = 0;
    for (;;) {
        while (ri < P.n_rec && P.rec_t[ri] == t) {
            shift_to(0);  // uniform call: rings of one workgroup may differ in sig
            measure(ri);
            ++ri;
        }
        if (t >= P.t1) break;
        uint64_t tn = P.t1;
        if (ri < P.n_rec && P.rec_t[ri] < tn) tn = P.rec_t[ri];
        for (; t < tn; ++t) {
            for (uint32_t s = 0; s < S; ++s) {
                const uint64_t g = t * S + s;
                const uint64_t quad = g >> 2;
                if (quad != shq) {
                    const Blk r = philox(0u, (uint32_t)quad,
                                         (kTagShift << 28) | (uint32_t)((quad >> 32) & 0xFFFFu),
                                         sample, k0, k1);
                    shblk[0] = r.v[0];
                    shblk[1] = r.v[1];
                    shblk[2] = r.v[2];
                    shblk[3] = r.v[3];
                    shq = quad;
                }
                const uint32_t gq = (uint32_t)(g & 3u);
                const uint32_t sw = gq == 0 ? shblk[0] : gq == 1 ? shblk[1] : gq == 2 ? shblk[2]
                                                                                     : shblk[3];
                shift_to(sw & cmask);

                const uint32_t glo = (uint32_t)g;
                const uint32_t c2b = (kTagAttempt << 28) | (uint32_t)((g >> 32) & 0xFFFFu);
                int32_t dj = 0;
#pragma unroll
                for (int i = 0; i < C; ++i) {
                    if (i < cnt) {
                        uint32_t slot = base_slot + (uint32_t)i + off;
                        if (slot >= nw) slot -= nw;
                        uint64_t xa = sa[i];
                        uint64_t xb = sb[i];
                        uint64_t m0 = 0, m1 = 0;
                        if (MODEL != kPlain) {
                            const uint32_t sn = (slot + 1 == nw) ? 0 : slot + 1;
                            m0 = funnel(lmask[slot], lmask[sn], sig);
                            if (P.mplanes > 1) m1 = funnel(lmask[nw + slot], lmask[nw + sn], sig);
                        }
                        for (uint32_t cq = 0; cq < cps; ++cq) {
                            const uint32_t k = slot * cps + cq;
                            const uint32_t bb = cq << lam;
                            uint32_t m = 0;
                            for (uint32_t blk = 0; blk < nblk; ++blk) {
                                const Blk r = philox(k, glo, c2b | (blk << 16), sample, k0, k1);
#pragma unroll
                                for (int wd = 0; wd < 4; ++wd) {
                                    const uint32_t u = r.v[wd];
                                    for (uint32_t sl = 0; sl < Aw && m < na; ++sl, ++m) {
                                        const uint32_t sh = sl * fw;
                                        const uint32_t rv = (u >> sh) & rmask;
                                        if (MODEL != kTwoLane) {
                                            const uint32_t j = (u >> (sh + rb)) & cmask;
                                            const uint32_t pos = bb + j;
                                            const uint32_t pr = (uint32_t)(xa >> pos) & 3u;
                                            uint32_t tp = T0, tq = T1;
                                            if (MODEL == kDisorder) {
                                                if ((m0 >> pos) & 1u) tp = T2;
                                                if (((m1 >> pos) >> 1) & 1u) tq = T3;
                                            }
                                            const bool live = j != cmask;
                                            const bool fwd = live && pr == 1u && rv < tp;
                                            const bool bwd = live && pr == 2u && rv < tq;
                                            xa ^= (uint64_t)((fwd || bwd) ? 3u : 0u) << pos;
                                            dj += (int32_t)fwd - (int32_t)bwd;
                                        } else {
                                            const uint32_t e = (u >> (sh + rb)) & 3u;
                                            const uint32_t j = (u >> (sh + rb + 2)) & cmask;
                                            const uint32_t pos = bb + j;
                                            const uint32_t pa2 = (uint32_t)(xa >> pos) & 3u;
                                            const uint32_t pb2 = (uint32_t)(xb >> pos) & 3u;
                                            const uint32_t tt = (uint32_t)(m0 >> pos) & 1u;
                                            const bool live = j != cmask;
                                            const bool hopA = e == 0 && live && pa2 == 1u && rv < T0;
                                            const bool hopB = e == 1 && live && pb2 == 2u && rv < T1;
                                            const uint32_t a0 = pa2 & 1u, b0 = pb2 & 1u;
                                            const bool ab = e == 2 && tt && a0 == 1u && b0 == 0u && rv < T2;
                                            const bool ba = e == 3 && tt && b0 == 1u && a0 == 0u && rv < T2;
                                            const uint32_t ch = (ab || ba) ? 1u : 0u;
                                            xa ^= (uint64_t)(hopA ? 3u : ch) << pos;
                                            xb ^= (uint64_t)(hopB ? 3u : ch) << pos;
                                            dj += (int32_t)hopA - (int32_t)hopB;
                                        }
                                    }
                                }
                            }
                        }
                        sa[i] = xa;
                        if (MODEL == kTwoLane) sb[i] = xb;
                    }
                }
                J += dj;
            }
        }
    }
    shift_to(0);
#pragma unroll
    for (int i = 0; i < C; ++i) {
        if (i < cnt) {
            uint32_t wdx = base_slot + (uint32_t)i + off;
            if (wdx >= nw) wdx -= nw;
            uint64_t* dst = P.words + (size_t)ring * NPL * nw;
            dst[wdx] = sa[i];
            if (MODEL == kTwoLane) dst[nw + wdx] = sb[i];
        }
    }
    // total hops of the ring
    if (lt == 0 && gi < G) red[gi * 4 + 2] = 0;
    __syncthreads();
    if (act) atomicAdd(&red[gi * 4 + 2], (unsigned long long)J);
    __syncthreads();
    if (ring_ok && lt == 0) P.hops[ring] = hops0 + (int64_t)red[gi * 4 + 2];
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

}  // namespace

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

uint32_t ring_block_limit(uint32_t C) { return ring_max_block((int)C); }

size_t ring_lds_bytes(uint32_t block, uint32_t planes, uint32_t G, uint32_t mplanes,
                      uint32_t nw) {
    size_t a, b, c, d, e;
    return lds_layout(block, planes, G, mplanes, nw, &a, &b, &c, &d, &e);
}

template <int MODEL>
static hipError_t launch_ring_model(const RingArgs& a, uint32_t C, uint32_t block, uint32_t grid,
                                    size_t lds, hipStream_t st) {
    (void)hipGetLastError();
    switch (C) {
        case 1: hipLaunchKernelGGL((k_ring<1, MODEL>), dim3(grid), dim3(block), lds, st, a); break;
        case 2: hipLaunchKernelGGL((k_ring<2, MODEL>), dim3(grid), dim3(block), lds, st, a); break;
        case 4: hipLaunchKernelGGL((k_ring<4, MODEL>), dim3(grid), dim3(block), lds, st, a); break;
        case 8: hipLaunchKernelGGL((k_ring<8, MODEL>), dim3(grid), dim3(block), lds, st, a); break;
        case 16: hipLaunchKernelGGL((k_ring<16, MODEL>), dim3(grid), dim3(block), lds, st, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_ring(const RingArgs& a, uint32_t C, uint32_t model, uint32_t block,
                       uint32_t grid, size_t lds, hipStream_t st) {
    switch (model) {
        case kPlain: return launch_ring_model<kPlain>(a, C, block, grid, lds, st);
        case kDisorder: return launch_ring_model<kDisorder>(a, C, block, grid, lds, st);
        case kTwoLane: return launch_ring_model<kTwoLane>(a, C, block, grid, lds, st);
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
