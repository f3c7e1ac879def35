// asep_device.h -- device code shared by the gfx950 kernel translation units:
// Philox4x32-10, bit helpers, height-moment tables, the per-cell attempt
// loops and the sweep kernel template.  Included only by .hip files.
//
// Random numbers: Philox4x32-10 (Salmon et al., SC'11) keyed by (seed,
// stream); counters
//   attempt: (cell k, lo32(g), 1<<28 | blk<<16 | hi16(g), sample)
//   shift:   (0, lo32(g/4), 2<<28 | hi16(g/4), sample), word g mod 4
//   init:    (site/4, lane, 3<<28, sample), word site mod 4
//   masks:   (site/4, 0, tag<<28, realisation), word site mod 4
//   two-sub-lattice update: (slot w, lo32(g), 8<<28 | blk<<16 | hi16(g), sample)
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "asep_internal.h"

namespace asep {
namespace dev {

constexpr uint32_t kMulA = 0xD2511F53u;
constexpr uint32_t kMulB = 0xCD9E8D57u;
constexpr uint32_t kWeylA = 0x9E3779B9u;
constexpr uint32_t kWeylB = 0xBB67AE85u;

struct Blk {
    uint32_t v[4];
};

// a ^ b ^ k in one VALU instruction (gfx950's three-input bitwise op with
// the XOR truth table 0x96), k wave-uniform (an SGPR operand).
__device__ __forceinline__ uint32_t xor3_uniform(uint32_t a, uint32_t b, uint32_t k) {
    uint32_t r;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "s"(k), "v"(b));
    return r;
}

// x ^ (m & f) in one VALU instruction (three-input bitwise op, truth table
// 0x78 with the inputs in the order x, m, f).
__device__ __forceinline__ uint32_t xor_masked(uint32_t x, uint32_t m, uint32_t f) {
    uint32_t r;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x78" : "=v"(r) : "v"(x), "v"(m), "v"(f));
    return r;
}

// (a & 3) | (b & ~3): the low two bits of a below the rest of b.
__device__ __forceinline__ uint32_t insert_low2(uint32_t a, uint32_t b) {
    uint32_t r;
    asm("v_bfi_b32 %0, 3, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// Ten Philox rounds: products of counter words 0 and 2, high halves mixed
// with the other two words and the round key, Weyl key schedule.  The key
// must be wave-uniform.  With FUSE, from the third round on (where every
// counter word varies across lanes) each mix is one three-input XOR; the
// first two rounds are left to the compiler, which keeps their uniform parts
// scalar.  FUSE is off where the compiler's own schedule measured faster
// (the attempt loop with quenched-rate lookups).
template <bool FUSE = true>
__device__ __forceinline__ Blk philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                      uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        const uint64_t pa = (uint64_t)kMulA * (uint64_t)c0;
        const uint64_t pb = (uint64_t)kMulB * (uint64_t)c2;
        uint32_t n0, n2;
        if (FUSE && i >= 2) {
            n0 = xor3_uniform((uint32_t)(pb >> 32), c1, k0);
            n2 = xor3_uniform((uint32_t)(pa >> 32), c3, k1);
        } else {
            n0 = (uint32_t)(pb >> 32) ^ c1 ^ k0;
            n2 = (uint32_t)(pa >> 32) ^ c3 ^ k1;
        }
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

// Value of `v` in lane `src` of the wave (two 32-bit lane permutes); every
// lane of the wave must execute it.
__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src) {
    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, src, 64);
    const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), src, 64);
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

__device__ __forceinline__ uint32_t bfe(uint32_t v, uint32_t off, uint32_t width) {
    return __builtin_amdgcn_ubfe(v, off, width);
}

// Sums of heights inside one word relative to the height at its first site:
// E1 = sum_q d_q, E2 = sum_q d_q^2 with d_0 = 0, d_{q+1} = d_q + 1 - 2 n_q
// (Eq. W's h restricted to one word); tab1/tab2 hold the same sums per byte.
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

__device__ inline void build_byte_tables(int32_t* tab1, int32_t* tab2) {
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

// ---------------------------------------------------------------------------
// Attempt loops.  One call runs the `na` attempts of one cell in one
// sub-sweep (Sec. 2.1's exchange rules under the shifted decomposition):
// attempt m takes field (m mod A) of word ((m / A) mod 4) of Philox block
// m / 4A; a field is [j | e | r] from the top (e only for two lanes), or,
// for cells of 32 sites whose field fits a byte, the fields are the bytes of
// the word and each is [r | e | j] from the top (j in the low five bits, where
// a shift by j reads it straight from the byte).
// ---------------------------------------------------------------------------
struct CellCtx {
    uint32_t k;       // cell index
    uint32_t glo;     // lo32(g)
    uint32_t c2b;     // attempt tag | hi16(g)
    uint32_t sample;
    uint32_t k0, k1;  // key
    uint32_t na, nblk, b, w, A;
    uint32_t oj, oe, orr;  // bit offsets of j, e and r in a field
    uint32_t T0, T1, T2, T3;
    // With at most 2 compared bits: bit o says whether pair o mod 4 with
    // compared bits (o >> 2) mod 2^b hops (the pattern repeats every 2^(2+b)
    // bits, so any higher bits of the offset select the same outcome).
    uint32_t lutP;
    // Columnar disorder, when the offset fits five bits: bit o says whether
    // pair o mod 4, compared bits (o >> 2) mod 2^b, the forward mark at bit
    // 2+b and (with backward hops) the backward mark at bit 3+b hop;
    // repeated likewise above the bits in use.
    uint32_t lutD;
    // Two lanes: lane-change draws (tag | hi16(g)), their compared bits,
    // and the outcome table of the fast loop: bit 32 e1 + 16 e0 + [a_x
    // a_x+1 b_x b_x+1] (bit 0 first) says, for events e = 2 e1 + e0 0 and 1,
    // whether the hop (A right, B left) fires, and for events 2 and 3
    // whether the lane change (A -> B, B -> A) finds a particle on its side
    // and a hole on the other.
    uint32_t c2c, bc;
    uint64_t lut2;
};

// Generic single-lane cell: any cell size ell <= 64 located at bit `bb` of
// the slot; the attempt count per word is a runtime value.
template <bool DIS>
__device__ __forceinline__ int32_t cell_ring_generic(uint64_t& x, uint64_t m0, uint64_t m1,
                                                      uint32_t bb, uint32_t lam,
                                                      const CellCtx& c) {
    const uint32_t cmask = (1u << lam) - 1u;
    const uint32_t rmask = (c.b >= 32) ? 0xFFFFFFFFu : ((1u << c.b) - 1u);
    int32_t dj = 0;
    uint32_t m = 0;
    for (uint32_t blk = 0; blk < c.nblk; ++blk) {
        const Blk r = philox<!DIS>(c.k, c.glo, c.c2b | (blk << 16), c.sample, c.k0, c.k1);
#pragma unroll
        for (int wd = 0; wd < 4; ++wd) {
            const uint32_t u = r.v[wd];
            for (uint32_t sl = 0; sl < c.A && m < c.na; ++sl, ++m) {
                const uint32_t sh = sl * c.w;
                const uint32_t rv = (u >> (sh + c.orr)) & rmask;
                const uint32_t j = (u >> (sh + c.oj)) & cmask;
                const uint32_t pos = bb + j;
                const uint32_t pr = (uint32_t)(x >> pos) & 3u;
                uint32_t tp = c.T0, tq = c.T1;
                if (DIS) {
                    if ((m0 >> pos) & 1u) tp = c.T2;
                    if (((m1 >> pos) >> 1) & 1u) tq = c.T3;
                }
                const bool live = j != cmask;
                const bool fwd = live && pr == 1u && rv < tp;
                const bool bwd = live && pr == 2u && rv < tq;
                x ^= (uint64_t)((fwd || bwd) ? 3u : 0u) << pos;
                dj += (int32_t)fwd - (int32_t)bwd;
            }
        }
    }
    return dj;
}

// Single lane, ell = 64 (one cell per slot), default schedule: NA attempts
// per cell per sub-sweep, A fields per 32-bit word and BB compared bits known
// at compile time (BB < 0: runtime).  The pair (x, x+1) is read with an
// arithmetic shift: at j = 63 the top bit is replicated, the pair is 00 or
// 11 and nothing can hop, which is exactly the no-op of the bond leaving the
// cell.  With at most two compared bits (p, q multiples of 1/4) the pair and
// those bits index one 32-bit pattern of outcomes (lutP), and the hop is an
// XOR with 3 << j under the all-ones-or-zero outcome.  Q0: no backward hops
// (q = 0): every flip is a right hop.
template <int A, int BB, bool Q0, bool DIS, int NA>
__device__ __forceinline__ int32_t cell_ring_fast(uint64_t& x, uint64_t m0, uint64_t m1,
                                                   const CellCtx& c) {
    constexpr int PER = 4 * A;
    constexpr int NB = (NA + PER - 1) / PER;
    int32_t dj = 0;
#pragma unroll
    for (int blk = 0; blk < NB; ++blk) {
        const Blk r =
            philox<!DIS>(c.k, c.glo, c.c2b | ((uint32_t)blk << 16), c.sample, c.k0, c.k1);
#pragma unroll
        for (int wd = 0; wd < 4; ++wd) {
#pragma unroll
            for (int sl = 0; sl < A; ++sl) {
                if (blk * PER + wd * A + sl >= NA) continue;
                const uint32_t u = r.v[wd];
                const uint32_t b = BB >= 0 ? (uint32_t)BB : c.b;
                const uint32_t sh = BB >= 0 ? (uint32_t)(sl * (6 + BB)) : (uint32_t)sl * c.w;
                const uint32_t j = bfe(u, sh + b, 6);
                const int64_t sx = (int64_t)x >> j;
                const uint32_t pr = (uint32_t)sx & 3u;
                uint32_t f;
                constexpr bool DTAB = DIS && BB >= 0 && 3 + BB + (Q0 ? 0 : 1) <= 5;
                if (DTAB) {
                    // pair, compared bits and the marks of the bond index
                    // one outcome bit (lutD); then as below
                    uint32_t hi = (uint32_t)(m0 >> j);  // bit 0: forward mark at j
                    if (!Q0)  // bit 1: backward mark at j+1
                        hi = __builtin_amdgcn_bitop3_b32(hi, (uint32_t)(m1 >> j), 1u, 0xE4);
                    uint32_t off;
                    if (BB > 0) {
                        const uint32_t rs = sh >= 2 ? u >> (sh - 2) : u << (2 - sh);
                        off = __builtin_amdgcn_bitop3_b32(insert_low2((uint32_t)sx, rs),
                                                          hi << (2 + BB), (1u << (2 + BB)) - 1u,
                                                          0xE4);
                    } else {
                        off = insert_low2((uint32_t)sx, hi << 2);
                    }
                    const uint32_t F = (uint32_t)__builtin_amdgcn_sbfe((int32_t)c.lutD, off, 1);
                    const uint64_t M = 3ull << j;
                    const uint32_t lo = xor_masked((uint32_t)x, (uint32_t)M, F);
                    const uint32_t hw = xor_masked((uint32_t)(x >> 32), (uint32_t)(M >> 32), F);
                    x = ((uint64_t)hw << 32) | lo;
                    dj += (int32_t)F;
                    if (!Q0) dj += (int32_t)(F & ~(uint32_t)sx & 2u);
                    continue;
                } else if (BB >= 0 && BB <= 2 && !DIS) {
                    // Offset into lutP: the pair in bits 0-1, the compared
                    // bits above it (v_bfe takes the offset mod 32, so the
                    // sites beyond the pair only repeat the pattern).  F is
                    // all ones when the pair hops; the flip mask 3 << j does
                    // not wait for the state.
                    uint32_t off = (uint32_t)sx;
                    if (BB > 0) {
                        const uint32_t rs = sh >= 2 ? u >> (sh - 2) : u << (2 - sh);
                        off = insert_low2(off, rs);
                    }
                    const uint32_t F = (uint32_t)__builtin_amdgcn_sbfe((int32_t)c.lutP, off, 1);
                    const uint64_t M = 3ull << j;
                    const uint32_t lo = xor_masked((uint32_t)x, (uint32_t)M, F);
                    const uint32_t hi = xor_masked((uint32_t)(x >> 32), (uint32_t)(M >> 32), F);
                    x = ((uint64_t)hi << 32) | lo;
                    // Q0: minus one per (right) hop; otherwise a hop adds
                    // F = -1 plus 2 when site j+1 was empty, i.e. it went right
                    dj += (int32_t)F;
                    if (!Q0) dj += (int32_t)(F & ~(uint32_t)sx & 2u);
                    continue;
                } else {
                    const uint32_t rv = (BB == 0) ? 0u : bfe(u, sh, b);
                    uint32_t tsel;
                    if (DIS) {
                        const uint32_t tp = ((m0 >> j) & 1u) ? c.T2 : c.T0;
                        uint32_t tq = 0;
                        if (!Q0) tq = (((m1 >> j) >> 1) & 1u) ? c.T3 : c.T1;
                        tsel = pr == 1u ? tp : (pr == 2u ? tq : 0u);
                    } else {
                        tsel = pr == 1u ? c.T0 : (pr == 2u ? c.T1 : 0u);
                    }
                    f = (rv < tsel) ? 3u : 0u;
                }
                x ^= (uint64_t)f << j;
                if (Q0)
                    dj += (int32_t)f;  // 3 per right hop
                else
                    dj += f ? (int32_t)(3u - 2u * pr) : 0;
            }
        }
    }
    if (BB >= 0 && BB <= 2 && (!DIS || 3 + BB + (Q0 ? 0 : 1) <= 5)) return Q0 ? -dj : dj;
    return Q0 ? dj / 3 : dj;
}

// Single lane, ell = 32, two sub-sweeps per MCS (16 attempts per cell per
// sub-sweep): the slot's two cells are its 32-bit halves (cells 2w and
// 2w + 1), each updated with 32-bit operations, and their attempt chains
// are independent, so one lane runs two of them side by side.  The 16 fields
// of a cell are the bytes of its Philox block, j in the low five bits of the
// byte and BB (<= 2) compared bits above it: the shifts by j read it straight
// from the byte (a byte operand select), so no instruction extracts it.  The
// outcome is one bit of lutP indexed by the pair and the compared bits, and
// the arithmetic shift makes j = 31 (the bond leaving the cell) a no-op, as
// in cell_ring_fast.  With columnar disorder (DIS) the forward mark at j,
// and with backward hops the backward mark at j + 1, join the pair and the
// compared bits in the offset of lutD, as in cell_ring_fast; the marks come
// from the same half of the slot's mark words.
template <int BB, bool Q0, bool DIS>
__device__ __forceinline__ int32_t cell_half_apply(uint64_t& x, uint64_t m0, uint64_t m1,
                                                    const CellCtx& c, const Blk& r0,
                                                    const Blk& r1) {
    static_assert(BB >= 0 && BB <= 2, "field layout");
    static_assert(!DIS || 3 + BB + (Q0 ? 0 : 1) <= 5, "marks in the offset");
    uint32_t h0 = (uint32_t)x, h1 = (uint32_t)(x >> 32);
    const uint32_t f0 = (uint32_t)m0, f1 = (uint32_t)(m0 >> 32);
    const uint32_t g0 = (uint32_t)m1, g1 = (uint32_t)(m1 >> 32);
    int32_t d0 = 0, d1 = 0;
#pragma unroll
    for (int wd = 0; wd < 4; ++wd) {
#pragma unroll
        for (int sl = 0; sl < 4; ++sl) {
            const uint32_t sh = (uint32_t)sl * 8u;
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const uint32_t u = q ? r1.v[wd] : r0.v[wd];
                uint32_t& h = q ? h1 : h0;
                int32_t& d = q ? d1 : d0;
                // the byte holding j (its low five bits are what a shift
                // uses; written as a byte extract so that the compiler folds
                // it into the shifts' operand select)
                const uint32_t jb = sl == 0 ? u : __builtin_amdgcn_ubfe(u, sh, 8);
                const uint32_t j = jb & 31u;
                const uint32_t sx = (uint32_t)((int32_t)h >> j);
                uint32_t off = sx;
                if (BB > 0) off = insert_low2(sx, u >> (sh + 3u));  // compared bits at 2
                if (DIS) {
                    // bit 0: forward mark at j; bit 1: backward mark at j+1
                    uint32_t mk = (q ? f1 : f0) >> j;
                    if (!Q0) mk = __builtin_amdgcn_bitop3_b32(mk, (q ? g1 : g0) >> j, 1u, 0xE4);
                    off = __builtin_amdgcn_bitop3_b32(off, mk << (2 + BB), (1u << (2 + BB)) - 1u,
                                                      0xE4);
                }
                const uint32_t F =
                    (uint32_t)__builtin_amdgcn_sbfe((int32_t)(DIS ? c.lutD : c.lutP), off, 1);
                h = xor_masked(h, 3u << j, F);
                d += (int32_t)F;
                if (!Q0) d += (int32_t)(F & ~sx & 2u);
            }
        }
    }
    x = (uint64_t)h0 | ((uint64_t)h1 << 32);
    return Q0 ? -(d0 + d1) : d0 + d1;
}

// Draws of cells k and k+1 in the sub-sweep of c, then their attempts.
template <int BB, bool Q0, bool DIS>
__device__ __forceinline__ int32_t cell_half_fast(uint64_t& x, uint64_t m0, uint64_t m1,
                                                   const CellCtx& c) {
    const Blk r0 = philox(c.k, c.glo, c.c2b, c.sample, c.k0, c.k1);
    const Blk r1 = philox(c.k + 1u, c.glo, c.c2b, c.sample, c.k0, c.k1);
    return cell_half_apply<BB, Q0, DIS>(x, m0, m1, c, r0, r1);
}

// Two lanes (Sec. 3): events 0 = A hops right on (x, x+1), 1 = B hops left
// from x+1 to x, 2 = A->B at x, 3 = B->A at x (turning point, other lane
// empty).  Bond events at j = ell-1 are no-ops; site events use every j.
//
// A lane change is decided by a 32-bit draw of its own: the cell's c-th
// candidate of the sub-sweep (a lane-change attempt at a turning point with
// a particle on its side and a hole on the other, counted from 0 in attempt
// order) takes word c mod 4 of Philox block (k, lo32(g), change tag |
// (c / 4) << 16 | hi16(g), sample) and moves when the word's top bc bits are
// below T2.  Candidates are rare (a fraction of a percent of the attempts in
// the two-lane workload): a cell draws its first block up front, the fast
// loop decides at most four candidates from it, and a lane whose cell meets
// a fifth redoes the cell's sub-sweep with the generic loop, which draws
// every further block as it needs it.
struct ChangeDraws {
    uint32_t u0, u1, u2, u3;
    uint32_t n;  // candidates so far
    // fast loops: acceptance of the first four candidates (bit i for
    // candidate i, taken from bit 0 and shifted out) above a sentinel at
    // bit 4, which reaches bit 0 exactly when a fifth candidate comes.  With
    // no compared bit (bc = 0) every decision is T2 != 0: all ones or zero,
    // which the arithmetic shift keeps and which never equals the sentinel.
    int32_t m;
};

// The fast loops' form of the cell's four up-front lane-change draws: their
// decisions as bits (the same comparisons change_accept makes).
__device__ __forceinline__ void change_begin_bits(ChangeDraws& d, const CellCtx& c) {
    if (c.bc) {
        const Blk r = philox(c.k, c.glo, c.c2c, c.sample, c.k0, c.k1);
        const uint32_t sh = 32u - c.bc;
        d.m = (int32_t)(0x10u | ((r.v[0] >> sh) < c.T2 ? 1u : 0u) |
                        ((r.v[1] >> sh) < c.T2 ? 2u : 0u) | ((r.v[2] >> sh) < c.T2 ? 4u : 0u) |
                        ((r.v[3] >> sh) < c.T2 ? 8u : 0u));
    } else {
        d.m = c.T2 != 0 ? -1 : 0;
    }
}

__device__ __forceinline__ void change_begin(ChangeDraws& d, const CellCtx& c) {
    d.n = 0;
    d.u0 = d.u1 = d.u2 = d.u3 = 0;
    if (c.bc) {
        const Blk r = philox(c.k, c.glo, c.c2c, c.sample, c.k0, c.k1);
        d.u0 = r.v[0];
        d.u1 = r.v[1];
        d.u2 = r.v[2];
        d.u3 = r.v[3];
    }
}

// Decision of the next candidate.  LATE: draw blocks past the first as
// needed; otherwise a fifth candidate sets `over` (its outcome is not used).
template <bool LATE>
__device__ __forceinline__ bool change_accept(ChangeDraws& d, const CellCtx& c, bool& over) {
    if constexpr (!LATE) {
        // decisions of change_begin_bits; the sentinel at bit 0 marks a
        // fifth candidate
        over |= d.m == 1;
        const bool a = (d.m & 1) != 0;
        d.m >>= 1;
        return a;
    }
    if (c.bc == 0) return c.T2 != 0;
    const uint32_t n = d.n++;
    uint32_t u;
    if (n < 4) {
        u = n == 0 ? d.u0 : n == 1 ? d.u1 : n == 2 ? d.u2 : d.u3;
    } else if (LATE) {
        const Blk r = philox(c.k, c.glo, c.c2c | ((n >> 2) << 16), c.sample, c.k0, c.k1);
        const uint32_t q = n & 3u;
        u = q == 0 ? r.v[0] : q == 1 ? r.v[1] : q == 2 ? r.v[2] : r.v[3];
    } else {
        over = true;
        return false;
    }
    return (u >> (32u - c.bc)) < c.T2;
}

template <bool LATE>
__device__ __forceinline__ void two_lane_event(uint64_t& xa, uint64_t& xb, uint32_t pa,
                                               uint32_t pb, uint32_t tt, uint32_t e, uint32_t rv,
                                               bool live, uint32_t pos, const CellCtx& c,
                                               ChangeDraws& cd, bool& over, int32_t& dj) {
    const bool hopA = e == 0u && live && pa == 1u && rv < c.T0;
    const bool hopB = e == 1u && live && pb == 2u && rv < c.T1;
    const uint32_t a0 = pa & 1u, b0 = pb & 1u;
    const bool cand = e >= 2u && tt && a0 != b0 && a0 == (e == 2u ? 1u : 0u);
    bool chg = false;
    if (cand) chg = change_accept<LATE>(cd, c, over);
    const uint32_t ch = chg ? 1u : 0u;
    xa ^= (uint64_t)(hopA ? 3u : ch) << pos;
    xb ^= (uint64_t)(hopB ? 3u : ch) << pos;
    dj += (int32_t)hopA - (int32_t)hopB;
}

// Any cell size ell <= 64 at bit `bb` of the slot, runtime fields per word.
__device__ __forceinline__ int32_t cell_two_lane_generic(uint64_t& xa, uint64_t& xb, uint64_t tm,
                                                          uint32_t bb, uint32_t lam,
                                                          const CellCtx& c) {
    const uint32_t cmask = (1u << lam) - 1u;
    const uint32_t rmask = (c.b >= 32) ? 0xFFFFFFFFu : ((1u << c.b) - 1u);
    int32_t dj = 0;
    uint32_t m = 0;
    ChangeDraws cd;
    change_begin(cd, c);
    bool over = false;  // never set: every block is drawn as needed
    for (uint32_t blk = 0; blk < c.nblk; ++blk) {
        const Blk r = philox(c.k, c.glo, c.c2b | (blk << 16), c.sample, c.k0, c.k1);
        for (int wd = 0; wd < 4; ++wd) {
            const uint32_t u = r.v[wd];
            for (uint32_t sl = 0; sl < c.A && m < c.na; ++sl, ++m) {
                const uint32_t sh = sl * c.w;
                const uint32_t rv = (u >> (sh + c.orr)) & rmask;
                const uint32_t e = (u >> (sh + c.oe)) & 3u;
                const uint32_t j = (u >> (sh + c.oj)) & cmask;
                const uint32_t pos = bb + j;
                const uint32_t pa = (uint32_t)(xa >> pos) & 3u;
                const uint32_t pb = (uint32_t)(xb >> pos) & 3u;
                const uint32_t tt = (uint32_t)(tm >> pos) & 1u;
                two_lane_event<true>(xa, xb, pa, pb, tt, e, rv, j != cmask, pos, c, cd, over, dj);
            }
        }
    }
    return dj;
}

// ell = 64, default schedule (NA attempts per cell per sub-sweep), A fields
// per word and BB compared bits known at compile time (BB < 0: runtime); the
// arithmetic-shift pair read makes bond events at j = 63 no-ops while site
// events there stay live.  With no compared bit (hop rates 0 or 1) the
// pairs of both lanes and the event's low bit index the outcome tables:
// the hop is one masked XOR per half of the hopping lane's word, and only
// lane-change candidates (rare) take a branch for their draw.
template <int A, int BB, int NA>
__device__ __forceinline__ void cell_two_lane_fast(uint64_t& xa, uint64_t& xb, uint64_t tm,
                                                    const CellCtx& c) {
    constexpr int PER = 4 * A;
    constexpr int NB = (NA + PER - 1) / PER;
    int32_t dj = 0;  // not returned: the sweep counts hops at the closing bond
    ChangeDraws cd;
    change_begin_bits(cd, c);
    bool over = false;
    const uint64_t xa0 = xa, xb0 = xb;
    // the outcome table's low half in a vector register for the select
    // below (two scalar operands do not fit one instruction; held here, it
    // is not copied again for every attempt)
    uint32_t lut_lo = (uint32_t)c.lut2;
    asm volatile("" : "+v"(lut_lo));
#pragma unroll
    for (int blk = 0; blk < NB; ++blk) {
        const Blk r = philox(c.k, c.glo, c.c2b | ((uint32_t)blk << 16), c.sample, c.k0, c.k1);
#pragma unroll
        for (int wd = 0; wd < 4; ++wd) {
#pragma unroll
            for (int sl = 0; sl < A; ++sl) {
                if (blk * PER + wd * A + sl >= NA) continue;
                const uint32_t u = r.v[wd];
                if constexpr (BB == 0) {
                    const uint32_t sh = (uint32_t)sl * 8u;  // field [j(6) | e(2)]
                    const uint32_t j = bfe(u, sh + 2u, 6);
                    // state-independent: event bits as masks, the table half
                    // of e1, the turning bit at j, the pair mask
                    const uint32_t E0 = (uint32_t)__builtin_amdgcn_sbfe((int32_t)u, sh, 1);
                    const uint32_t E1 = (uint32_t)__builtin_amdgcn_sbfe((int32_t)u, sh + 1u, 1);
                    // E1 ? high half : low half (truth table 0xCA: src0 selects)
                    const uint32_t lw = __builtin_amdgcn_bitop3_b32(
                        E1, (uint32_t)(c.lut2 >> 32), lut_lo, 0xCA);
                    const uint32_t TT =
                        (uint32_t)__builtin_amdgcn_sbfe((int32_t)(uint32_t)(tm >> j), 0, 1);
                    const uint64_t M = 3ull << j;
                    // the state chain: both lanes' pairs, then one table bit
                    // (offset bits 0-3 the pairs, bit 4 the event's low bit
                    // from the mask E0; v_bfe reads five offset bits)
                    const int64_t sa = (int64_t)xa >> j;
                    const int64_t sb = (int64_t)xb >> j;
                    const uint32_t v = insert_low2((uint32_t)sa, (uint32_t)sb << 2);
                    const uint32_t idx = __builtin_amdgcn_bitop3_b32(v, E0, 0xFu, 0xE4);
                    const uint32_t F = (uint32_t)__builtin_amdgcn_sbfe((int32_t)lw, idx, 1);
                    // F & ~E0 & ~E1, F & E0 & ~E1, F & E1 & TT (the table
                    // index of a three-input op is src0 << 2 | src1 << 1 | src2)
                    const uint32_t FA = __builtin_amdgcn_bitop3_b32(F, E0, E1, 0x10);
                    const uint32_t FB = __builtin_amdgcn_bitop3_b32(F, E0, E1, 0x40);
                    const uint32_t FC = __builtin_amdgcn_bitop3_b32(F, E1, TT, 0x80);
                    xa = ((uint64_t)xor_masked((uint32_t)(xa >> 32), (uint32_t)(M >> 32), FA) << 32) |
                         xor_masked((uint32_t)xa, (uint32_t)M, FA);
                    xb = ((uint64_t)xor_masked((uint32_t)(xb >> 32), (uint32_t)(M >> 32), FB) << 32) |
                         xor_masked((uint32_t)xb, (uint32_t)M, FB);
                    if (FC) {
                        // the next of the four decisions made up front as
                        // a mask (a fifth candidate finds the sentinel and
                        // sends the cell to the replay), then the site's
                        // bit flips in both lanes under it
                        over |= cd.m == 1;
                        const uint32_t am = (uint32_t)__builtin_amdgcn_sbfe(cd.m, 0, 1);
                        cd.m >>= 1;
                        const uint64_t B = 1ull << j;
                        xa = ((uint64_t)xor_masked((uint32_t)(xa >> 32), (uint32_t)(B >> 32), am) << 32) |
                             xor_masked((uint32_t)xa, (uint32_t)B, am);
                        xb = ((uint64_t)xor_masked((uint32_t)(xb >> 32), (uint32_t)(B >> 32), am) << 32) |
                             xor_masked((uint32_t)xb, (uint32_t)B, am);
                    }
                } else {
                    const uint32_t b = BB >= 0 ? (uint32_t)BB : c.b;
                    const uint32_t sh = BB >= 0 ? (uint32_t)(sl * (8 + BB)) : (uint32_t)sl * c.w;
                    const uint32_t rv = bfe(u, sh, b);
                    const uint32_t e = bfe(u, sh + b, 2);
                    const uint32_t j = bfe(u, sh + b + 2, 6);
                    const uint32_t pa = (uint32_t)((int64_t)xa >> j) & 3u;
                    const uint32_t pb = (uint32_t)((int64_t)xb >> j) & 3u;
                    const uint32_t tt = (uint32_t)(tm >> j) & 1u;
                    two_lane_event<false>(xa, xb, pa, pb, tt, e, rv, true, j, c, cd, over, dj);
                }
            }
        }
    }
    if (over) {  // a fifth lane-change candidate: redo the cell exactly
        xa = xa0;
        xb = xb0;
        cell_two_lane_generic(xa, xb, tm, 0, 6, c);
    }
}

// The paper's two-sub-lattice update (Sec. 2.1, Fig. parasep) on one slot:
// the slot holds the 64 sites starting at an even site (phase 0) or an odd
// one (phase 1), so the 32 pairs of the phase sit at bits (2m, 2m+1) and the
// ring's closing pair is the top pair of the last slot.  Every pair is tried
// once: "10" hops right if U < T_p of its left site, "01" hops left if
// U < T_q of its right site, with U a b-bit number per pair.  The pairs are
// handled bit-parallel: pair m takes bit c(m) = 2 (m mod 16) + m / 16 of the
// random words, so the pair masks fold into 32 bits with one shift and one
// or (the left-site bits of the high half move next to those of the low
// half).  Random word n holds bit b-1-n of every U (most significant first);
// word n of the comparison is word n mod 4 of Philox block n / 4.  The
// comparison runs from the top bit and stops, block by block, as soon as
// every live pair of the slot is decided; a pair still equal to its
// threshold once the threshold's remaining bits are all zero is decided too
// (U >= T).  The result is that of the full b-bit comparison, with most of
// the blocks never drawn.
__device__ __forceinline__ uint32_t fold_pairs(uint64_t m) {
    return (uint32_t)m | ((uint32_t)(m >> 32) << 1);
}

__device__ __forceinline__ uint64_t unfold_pairs(uint32_t a) {
    return (uint64_t)(a & 0x55555555u) | ((uint64_t)((a >> 1) & 0x55555555u) << 32);
}

// One bit plane of a lazy bit-sliced comparison U < T from the top bit:
// `t` marks the pairs (sites) whose threshold has a 1 at this bit, `u` holds
// this bit of their U.  Pairs where u < t become accepted, pairs where they
// differ leave the undecided set.
template <typename W>
__device__ __forceinline__ void cmp_plane(W& lt, W& und, W t, W u) {
    lt |= und & t & ~u;
    und &= ~(t ^ u);
}

template <bool Q0, bool DIS>
__device__ __forceinline__ int32_t sca_slot(uint64_t& x, uint64_t m0, uint64_t m1,
                                            const CellCtx& c) {
    constexpr uint64_t kEven = 0x5555555555555555ull;
    const uint64_t l = x & kEven;
    const uint64_t r = (x >> 1) & kEven;
    const uint32_t fw = fold_pairs(l & ~r);
    const uint32_t bw = Q0 ? 0u : fold_pairs(r & ~l);
    // pair classes: forward at a fast/slow left site, backward at a fast/slow right site
    const uint32_t sp = DIS ? fold_pairs(m0 & kEven) : 0u;
    const uint32_t sq = (DIS && !Q0) ? fold_pairs((m1 >> 1) & kEven) : 0u;
    const uint32_t cls[4] = {fw & ~sp, Q0 ? 0u : (bw & ~sq), fw & sp, Q0 ? 0u : (bw & sq)};
    const uint32_t thr[4] = {c.T0, c.T1, c.T2, c.T3};
    const uint32_t full = 1u << c.b;
    uint32_t acc = 0, und = 0;
    uint32_t depth[4];  // leading bits that decide a comparison with thr[i]
    uint32_t ta[4];     // thresholds left-aligned: plane n reads bit 31 - n
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        depth[i] = 0;
        ta[i] = 0;
        if (thr[i] >= full) {
            acc |= cls[i];
        } else if (thr[i] != 0) {
            und |= cls[i];
            depth[i] = c.b - (uint32_t)__builtin_ctz(thr[i]);
            ta[i] = thr[i] << (32u - c.b);  // 1 <= b <= 24 here
        }
    }
    // Planes past a class's depth carry threshold bit 0, so its pairs can
    // only leave the undecided set there (as rejections); cutting the class
    // at the end of the block that reaches its depth decides the same.
    uint32_t lt = 0;
    for (uint32_t blk = 0; und != 0u && blk < c.nblk; ++blk) {
        const Blk rb = philox(c.k, c.glo, c.c2b | (blk << 16), c.sample, c.k0, c.k1);
#pragma unroll
        for (int wd = 0; wd < 4; ++wd) {
            const uint32_t sh = 31u - (blk * 4u + (uint32_t)wd);  // >= 8: at most 6 blocks
            uint32_t t = 0;
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (!(Q0 && (i & 1)) && (DIS || i < 2))
                    t |= cls[i] & (0u - ((ta[i] >> sh) & 1u));
            cmp_plane(lt, und, t, rb.v[wd]);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (!(Q0 && (i & 1)) && (DIS || i < 2))
                if (4u * (blk + 1u) >= depth[i]) und &= ~cls[i];
    }
    acc |= lt;
    const uint64_t a64 = unfold_pairs(acc);
    x ^= a64 | (a64 << 1);
    if (Q0) return __popc(acc);
    return __popc(acc & fw) - __popc(acc & bw);
}

// Accept-all / undecided split of one threshold class, and the number of
// leading bits that decide it (the bits below its lowest 1 are all zero).
template <typename W>
__device__ __forceinline__ uint32_t sca_class(W cls, uint32_t thr, uint32_t b, W& acc, W& und) {
    if (thr >= (1u << b)) {
        acc |= cls;
        return 0;
    }
    if (thr == 0) return 0;
    und |= cls;
    return b - (uint32_t)__builtin_ctz(thr);
}

// Two lanes, the paper's SCA sequence (Sec. 3), in-lane step on the pairs
// at bits (2m, 2m+1) of the slot: A's "10" hops right if U_A < T0, B's "01"
// hops left if U_B < T1.  Bit b-1-n of U_A is bit c(m) of the step's word
// 2n, of U_B of word 2n+1 (Philox block n / 2 gives A's planes in words 0
// and 2, B's in words 1 and 3).  Returns A hops minus B hops.
__device__ __forceinline__ int32_t sca_two_inlane(uint64_t& xa, uint64_t& xb, const CellCtx& c) {
    constexpr uint64_t kEven = 0x5555555555555555ull;
    const uint64_t la = xa & kEven, ra = (xa >> 1) & kEven;
    const uint64_t lb = xb & kEven, rb = (xb >> 1) & kEven;
    const uint32_t fa = fold_pairs(la & ~ra);
    const uint32_t fb = fold_pairs(rb & ~lb);
    uint32_t acc_a = 0, acc_b = 0, und_a = 0, und_b = 0, lt_a = 0, lt_b = 0;
    const uint32_t da = sca_class(fa, c.T0, c.b, acc_a, und_a);
    const uint32_t db = sca_class(fb, c.T1, c.b, acc_b, und_b);
    // left-aligned thresholds (plane n reads bit 31 - n; bits past b are 0),
    // classes cut at the end of the block reaching their depth (as sca_slot)
    const uint32_t ta0 = c.b ? c.T0 << (32u - c.b) : 0u;
    const uint32_t ta1 = c.b ? c.T1 << (32u - c.b) : 0u;
    for (uint32_t blk = 0; (und_a | und_b) != 0u && blk < c.nblk; ++blk) {
        const Blk r = philox(c.k, c.glo, c.c2b | (blk << 16), c.sample, c.k0, c.k1);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const uint32_t sh = 31u - (2u * blk + (uint32_t)j);  // >= 8: at most 12 blocks
            cmp_plane(lt_a, und_a, fa & (0u - ((ta0 >> sh) & 1u)), r.v[2 * j]);
            cmp_plane(lt_b, und_b, fb & (0u - ((ta1 >> sh) & 1u)), r.v[2 * j + 1]);
        }
        if (2u * (blk + 1u) >= da) und_a = 0;
        if (2u * (blk + 1u) >= db) und_b = 0;
    }
    acc_a |= lt_a;
    acc_b |= lt_b;
    const uint64_t ma = unfold_pairs(acc_a), mb = unfold_pairs(acc_b);
    xa ^= ma | (ma << 1);
    xb ^= mb | (mb << 1);
    return __popc(acc_a) - __popc(acc_b);
}

// Two lanes, lane-change step: every site with a particle in `from` and a
// hole in `to` moves across if U < T2 (T3 where `mark` is set).  Bit b-1-n
// of a site's U is bit (s mod 32) of the step's word 2n + s / 32, s the
// site's bit in the slot (Philox block n / 2 holds planes 2 blk, 2 blk + 1).
__device__ __forceinline__ void sca_two_change(uint64_t& from, uint64_t& to, uint64_t mark,
                                               const CellCtx& c) {
    const uint64_t live = from & ~to;
    const uint64_t c0 = live & ~mark, c1 = live & mark;
    uint64_t acc = 0, und = 0, lt = 0;
    const uint32_t d0 = sca_class(c0, c.T2, c.b, acc, und);
    const uint32_t d1 = sca_class(c1, c.T3, c.b, acc, und);
    const uint32_t ta2 = c.b ? c.T2 << (32u - c.b) : 0u;
    const uint32_t ta3 = c.b ? c.T3 << (32u - c.b) : 0u;
    for (uint32_t blk = 0; und != 0u && blk < c.nblk; ++blk) {
        const Blk r = philox(c.k, c.glo, c.c2b | (blk << 16), c.sample, c.k0, c.k1);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const uint32_t sh = 31u - (2u * blk + (uint32_t)j);
            const uint64_t u = (uint64_t)r.v[2 * j] | ((uint64_t)r.v[2 * j + 1] << 32);
            const uint64_t t = (c0 & (0ull - ((ta2 >> sh) & 1u))) |
                               (c1 & (0ull - ((ta3 >> sh) & 1u)));
            cmp_plane(lt, und, t, u);
        }
        if (2u * (blk + 1u) >= d0) und &= ~c0;
        if (2u * (blk + 1u) >= d1) und &= ~c1;
    }
    const uint64_t flip = acc | lt;
    from ^= flip;
    to ^= flip;
}

// Variants of the attempt loop.  The fast ones need ell = 64 and the default
// four sub-sweeps per MCS (16 attempts per cell and sub-sweep on one lane,
// 64 on two lanes).
enum Variant : int {
    kGeneric = 0,
    kF5B0 = 1,  // 5 fields per word, no threshold bits (p, q in {0, 1})
    kF4B1 = 2,  // 4 fields per word, 1 threshold bit (e.g. p = q = 1/2)
    kF4B2 = 3,  // 4 fields per word, 2 threshold bits
    kF1 = 4,    // 1 field per word, threshold bits at run time
    kF4B0 = 5,  // two lanes: 4 fields per word, no threshold bits
    kSca = 6,   // the paper's sub-lattice updates (both models, every slot shape)
    kH4B0 = 7,  // ell = 32, two sub-sweeps: 4 byte fields per word, no threshold bits
    kH4B1 = 8,  // ell = 32, two sub-sweeps: 4 byte fields per word, 1 threshold bit
};

template <int V>
struct VarInfo {
    static constexpr int A = 0, BB = -1;
};
template <>
struct VarInfo<kF5B0> {
    static constexpr int A = 5, BB = 0;
};
template <>
struct VarInfo<kF4B1> {
    static constexpr int A = 4, BB = 1;
};
template <>
struct VarInfo<kF4B2> {
    static constexpr int A = 4, BB = 2;
};
template <>
struct VarInfo<kF1> {
    static constexpr int A = 1, BB = -1;
};
template <>
struct VarInfo<kF4B0> {
    static constexpr int A = 4, BB = 0;
};
template <>
struct VarInfo<kH4B0> {
    static constexpr int A = 4, BB = 0;
};
template <>
struct VarInfo<kH4B1> {
    static constexpr int A = 4, BB = 1;
};

// Dynamic LDS of the sweep kernel, in this order:
//   xch   [2][block][planes] uint64  neighbour exchange, double-buffered
//   mask  [rings_per_wg][mplanes][mwords] uint64
//   red   [rings_per_wg][4] uint64     per-ring reductions
//   scan  [2][block] int32
//   tab   [2][256] int32
//   g0    [rings_per_wg] int32
__host__ __device__ inline size_t sweep_lds_layout(uint32_t block, uint32_t planes, uint32_t G,
                                                   uint32_t mplanes, uint32_t mwords,
                                                   size_t* o_mask, size_t* o_red, size_t* o_scan,
                                                   size_t* o_tab, size_t* o_g0) {
    size_t off = (size_t)2 * block * planes * 8;
    *o_mask = off;
    off += (size_t)G * mplanes * mwords * 8;
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

// Largest workgroup for C slots per lane: more slots need more VGPRs
// (gfx950: 512 VGPRs per SIMD lane; a 512-lane workgroup is 2 waves per SIMD).
__host__ __device__ constexpr uint32_t sweep_max_block(int C, int model = kPlain) {
    return (C == 1 || (C == 2 && model != kTwoLane)) ? 1024u : 512u;
}

// Slot drift of a window over the launch's sub-sweeps [g0, g1): the number
// of times the cell frame wraps (its start moves back below the previous
// one), including the return to frame 0 at the end.  Each wrap moves the
// slot labels one word to the right.  The shifted schedule's frames are the
// Philox shift draws of the ring (lane l of the wave draws quad g0/4 + l, a
// shuffle hands each quad the last frame of the one before); the sub-lattice
// schedules' frames are fixed.  Every lane of the wave must call this (the
// loop bounds are uniform); every lane gets the total.
template <int MODEL, int V>
__device__ uint32_t window_drift(const SimDesc& P, uint32_t sample, uint32_t cmask) {
    const uint64_t g0 = P.g0, g1 = P.g1;
    if (g1 <= g0) return 0;
    if constexpr (V == kSca) {
        // single lane: frames 0,1,0,1,... wrap at every even g; two lanes:
        // frames 0,0,1,0 wrap at g = 3 mod 4; plus the return to frame 0
        if constexpr (MODEL == kTwoLane)
            return (uint32_t)(g1 / 4 - (g0 + 1) / 4) + (((g1 - 1) & 3u) == 2u ? 1u : 0u);
        else
            return (uint32_t)((g1 - 1) / 2 - g0 / 2) + (uint32_t)((g1 - 1) & 1u);
    } else {
        const uint32_t lane = threadIdx.x & 63u;
        const uint64_t qlast = (g1 - 1) >> 2;
        uint32_t carry = 0, total = 0;
        for (uint64_t qb = g0 >> 2; qb <= qlast; qb += 64) {
            const uint64_t q = qb + lane;
            const Blk r = philox(0u, (uint32_t)q, (kTagShift << 28) | (uint32_t)((q >> 32) & 0xFFFFu),
                                 sample, P.key0, P.key1);
            uint32_t sg[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) sg[j] = r.v[j] & cmask;
            uint32_t prev = (uint32_t)__shfl_up((int)sg[3], 1, 64);
            if (lane == 0) prev = carry;
            uint32_t c = 0;
            if (q <= qlast) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const uint64_t g = 4 * q + (uint64_t)j;
                    const uint32_t p = j == 0 ? prev : sg[j - 1];
                    if (g > g0 && g < g1 && sg[j] < p) ++c;
                    if (g + 1 == g1 && sg[j] != 0u) ++c;
                }
            }
#pragma unroll
            for (int m = 32; m >= 1; m >>= 1) c += (uint32_t)__shfl_xor((int)c, m, 64);
            total += c;
            carry = (uint32_t)__shfl((int)sg[3], 63, 64);
        }
        return total;
    }
}

// Sum of the positions 64 w + b of the particles (set bits b) of word w.
__device__ __forceinline__ int64_t position_sum(uint64_t x, uint32_t w) {
    const uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
    uint32_t s = __popc(lo & 0xAAAAAAAAu) + __popc(hi & 0xAAAAAAAAu);
    s += 2u * (__popc(lo & 0xCCCCCCCCu) + __popc(hi & 0xCCCCCCCCu));
    s += 4u * (__popc(lo & 0xF0F0F0F0u) + __popc(hi & 0xF0F0F0F0u));
    s += 8u * (__popc(lo & 0xFF00FF00u) + __popc(hi & 0xFF00FF00u));
    s += 16u * (__popc(lo & 0xFFFF0000u) + __popc(hi & 0xFFFF0000u));
    s += 32u * __popc(hi);
    return (int64_t)s + 64 * (int64_t)w * (int64_t)__popcll(x);
}

// ---------------------------------------------------------------------------
// The sweep kernel.  A workgroup serves either G whole rings (segs == 1:
// the ring is periodic, measurements may be taken inside the launch) or one
// window of one ring (segs > 1): output words [s0, s0+n) plus the next
// K+1 words, with the window's start placed d words before s0, d being the
// exact slot drift of this launch (window_drift).  Garbage enters a window
// only from its right end, at most one slot per frame change (K sub-sweeps
// plus the return to frame 0), and the slot labels move right by exactly d,
// so the output words are exact.
// Lane lt owns window slots [lt*C, lt*C+C); slot i holds the 64 sites
// starting at sig + 64*(base + off + i) (mod L).
// WU: every active lane of a wave serves the same ring (windows, or rings of
// a whole number of waves), so the ring's sample, shift draws, frame and
// drift are wave-uniform and live in scalar registers.
// ---------------------------------------------------------------------------
template <int C, int MODEL, int V, bool Q0, bool MEAS, bool WU>
__device__ __forceinline__ void sweep_body(const SimDesc& P) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int NPL = (MODEL == kTwoLane) ? 2 : 1;
    constexpr bool HALF = V == kH4B0 || V == kH4B1;
    constexpr bool FAST = V != kGeneric && V != kSca && !HALF;
    constexpr int AV = VarInfo<V>::A;
    constexpr int BV = VarInfo<V>::BB;
    // Hop count of the cell loops (all but the sub-lattice update): a hop
    // moves the particles' position sum M = sum_y y n_y by one in its
    // direction, except a hop over the closing bond (L-1, 0), which moves
    // it by -(L-1) (right) or L-1 (left).  So J = M(end) - M(start) + L X,
    // with X the net right crossings of the closing bond.  Two lanes: J
    // (A hops right minus B hops left) is the displacement of all
    // particles, M and X summed over both lanes; a lane change keeps the
    // sum.  Cells are closed within a sub-sweep (their last bond is never
    // tried), so X grows by the change in the particles the closing
    // bond's slot holds to its right (sites 0 .. sig-1, its top sig bits):
    // no work per attempt.  J below then counts X, and each lane adds the
    // change in M of the words it owns.
    constexpr bool WRAPJ = V != kSca;

    const uint32_t lb = blockIdx.x - P.wg_begin;

    const uint32_t tid = threadIdx.x;
    const uint32_t block = blockDim.x;
    const uint32_t Tr = P.lanes_per_ring;
    const uint32_t G = P.rings_per_wg;
    const bool seg = P.segs > 1;
    const uint32_t gi = tid / Tr;
    const uint32_t lt = tid - gi * Tr;
    const uint32_t ring = seg ? lb / P.segs : lb * G + gi;
    const uint32_t sidx = seg ? lb % P.segs : 0;
    const bool ring_ok = (gi < G) && (ring < P.R);
    const uint32_t nw = P.nw;
    const uint32_t nslot = seg ? P.nslot : nw;
    const uint32_t nact = (nslot + C - 1) / C;
    const bool act = ring_ok && lt < nact;
    const uint32_t base_slot = lt * C;
    const int cnt = act ? (int)min((uint32_t)C, nslot - base_slot) : 0;
    uint32_t sample = P.sample0 + (ring_ok ? ring : 0);
    // lanes past the last ring of a window's workgroup are inactive; they
    // take the wave's first lane's sample like the rest of the wave
    if constexpr (WU) sample = __builtin_amdgcn_readfirstlane(sample);
    const uint32_t lane0 = gi * Tr;
    const uint32_t nxt = lane0 + ((lt + 1 < nact) ? lt + 1 : 0);
    // window origin (whole ring: 0) and the output range in window positions
    const uint32_t s0 = sidx * P.seg_n;
    const uint32_t nout = seg ? min(P.seg_n, nw - s0) : nw;
    // left margin: the exact drift of this launch (windows), 0 for whole rings
    uint32_t lm =
        seg ? window_drift<MODEL, V>(P, P.sample0 + lb / P.segs, (1u << P.sc.lam) - 1u) : 0;
    if constexpr (WU) lm = __builtin_amdgcn_readfirstlane(lm);  // every lane holds the total
    const uint32_t base = seg ? (s0 + nw - lm) % nw : 0;
    // mask words staged: every position a slot can reach, plus one
    const uint32_t mwords = seg ? nslot + P.halo + 2 : nw;

    size_t o_mask, o_red, o_scan, o_tab, o_g0;
    sweep_lds_layout(block, NPL, G, P.mplanes, mwords, &o_mask, &o_red, &o_scan, &o_tab, &o_g0);
    uint64_t* xch = reinterpret_cast<uint64_t*>(smem);
    uint64_t* lmask = reinterpret_cast<uint64_t*>(smem + o_mask) +
                      (size_t)(gi < G ? gi : 0) * P.mplanes * mwords;
    unsigned long long* red = reinterpret_cast<unsigned long long*>(smem + o_red);
    int32_t* scan = reinterpret_cast<int32_t*>(smem + o_scan);
    int32_t* tab1 = reinterpret_cast<int32_t*>(smem + o_tab);
    int32_t* tab2 = tab1 + 256;
    int32_t* g0s = reinterpret_cast<int32_t*>(smem + o_g0);

    const uint32_t lam = P.sc.lam;
    const uint32_t cmask = (1u << lam) - 1u;
    const uint32_t cps = 64u >> lam;

    CellCtx cc;
    cc.sample = sample;
    cc.k0 = P.key0;
    cc.k1 = P.key1;
    cc.na = P.sc.a;
    cc.nblk = P.sc.nblk;
    cc.b = P.sc.b;
    cc.w = P.sc.w;
    cc.A = P.sc.A;
    {
        const uint32_t eb = MODEL == kTwoLane ? 2u : 0u;
        cc.oj = P.sc.jlow ? 0u : P.sc.b + eb;
        cc.oe = P.sc.jlow ? P.sc.lam : P.sc.b;
        cc.orr = P.sc.jlow ? P.sc.lam + eb : 0u;
    }
    cc.T0 = P.sc.T[0];
    cc.T1 = P.sc.T[1];
    cc.T2 = P.sc.T[2];
    cc.T3 = P.sc.T[3];
    cc.lutP = 0;
    cc.lutD = 0;
    cc.c2c = 0;
    cc.bc = P.sc.bc;
    cc.lut2 = 0;
    if (MODEL == kTwoLane) {
        for (uint32_t o = 0; o < 32; ++o) {
            const uint32_t a0 = o & 1u, a1 = (o >> 1) & 1u, b0 = (o >> 2) & 1u,
                           b1 = (o >> 3) & 1u, e0 = (o >> 4) & 1u;
            const bool hop = e0 == 0 ? (a0 == 1u && a1 == 0u && P.sc.T[0] != 0)
                                     : (b0 == 0u && b1 == 1u && P.sc.T[1] != 0);
            const bool cand = e0 == 0 ? (a0 == 1u && b0 == 0u) : (a0 == 0u && b0 == 1u);
            cc.lut2 |= (uint64_t)(hop ? 1u : 0u) << o;
            cc.lut2 |= (uint64_t)(cand ? 1u : 0u) << (32 + o);
        }
    }
    if (P.sc.b <= 2) {
        const uint32_t b = P.sc.b;
        for (uint32_t o = 0; o < 32; ++o) {
            const uint32_t pr = o & 3u, rv = (o >> 2) & ((1u << b) - 1u);
            const bool hop = (pr == 1u && rv < P.sc.T[0]) || (pr == 2u && rv < P.sc.T[1]);
            cc.lutP |= (hop ? 1u : 0u) << o;
            const uint32_t mp = (o >> (2 + b)) & 1u, mq = Q0 ? 0u : (o >> (3 + b)) & 1u;
            const bool hopd = (pr == 1u && rv < (mp ? P.sc.T[2] : P.sc.T[0])) ||
                              (pr == 2u && rv < (mq ? P.sc.T[3] : P.sc.T[1]));
            cc.lutD |= (hopd ? 1u : 0u) << o;
        }
    }

    // load the window (whole ring: every word)
    uint64_t sa[C];
    uint64_t sb[C];
#pragma unroll
    for (int i = 0; i < C; ++i) {
        sa[i] = 0;
        sb[i] = 0;
        if (i < cnt) {
            uint32_t w = base + base_slot + (uint32_t)i;
            if (w >= nw) w -= nw;
            const uint64_t* src = P.words_in + (size_t)ring * NPL * nw;
            sa[i] = src[w];
            if (MODEL == kTwoLane) sb[i] = src[nw + w];
        }
    }
    // position sum of the lane's own words at the start (frame 0)
    int64_t Ms = 0;
    if constexpr (WRAPJ) {
#pragma unroll
        for (int i = 0; i < C; ++i) {
            const uint32_t pos = base_slot + (uint32_t)i;
            if (i < cnt && (!seg || pos - lm < nout)) {
                uint32_t w = base + pos;
                if (w >= nw) w -= nw;
                Ms += position_sum(sa[i], w);
                if (MODEL == kTwoLane) Ms += position_sum(sb[i], w);
            }
        }
    }
    if (MODEL != kPlain && ring_ok) {
        const uint32_t real = sample / P.spd - P.real0;
        const uint64_t* msrc = P.masks + (size_t)real * P.mplanes * nw;
        for (uint32_t pl = 0; pl < P.mplanes; ++pl)
            for (uint32_t idx = lt; idx < mwords; idx += Tr) {
                uint32_t w = base + idx;
                while (w >= nw) w -= nw;
                lmask[pl * mwords + idx] = msrc[(size_t)pl * nw + w];
            }
    }
    if (MEAS && P.n_rec) build_byte_tables(tab1, tab2);
    __syncthreads();

    // whole rings of at most one wave each (lanes_per_ring a power of two
    // up to 64, so no ring straddles two waves) exchange across lanes
    const bool wsync = !seg && Tr <= 64u && (64u % Tr) == 0u;
    // bo: word offset of this sub-sweep's half of the double-buffered
    // exchange area (toggles between 0 and block * NPL)
    uint32_t sig = 0, off = 0, bo = 0;
    const uint32_t bstride = block * NPL;
    // word held by this lane's slot 0: (base + off + base_slot) mod nw
    uint32_t wb = (uint32_t)(((uint64_t)base + base_slot) % nw);
    int64_t J = 0;
    const int64_t hops0 = (ring_ok && !seg) ? P.hops[ring] : 0;

    // Move every slot to the shift sig_new (neighbour exchange through LDS).
    // Every lane shifts, inactive ones and unused slots included: what they
    // hold is never read by an active slot (the last active slot takes the
    // lane nxt's first slot), measured or stored.
    uint64_t* const xw = xch + (size_t)tid * NPL;
    uint64_t* const xr = xch + (size_t)nxt * NPL;
    // LAY: 0 = windows or whole rings as `seg` says, 1 = windows, 2 = whole
    // rings (the sub-sweep loop runs in the form of its launch, so that the
    // bookkeeping of the other form drops out)
    auto shift_to = [&](uint32_t sig_new, auto lay) {
        constexpr int LAY = decltype(lay)::value;
        const bool sg = LAY == 0 ? seg : LAY == 1;
        const uint32_t delta = (sig_new + 64u - sig) & 63u;
        // frames are below 64: the start moved back (wrapped) exactly when
        // sig + delta overshoots sig_new (written so that a wave-uniform frame
        // keeps both in scalar registers)
        const bool wrap = sig + delta != sig_new;
        uint64_t na_ = 0, nb_ = 0;
        if (!sg && wsync) {
            // the ring lies inside one wave: read the neighbour lane's first
            // slot across lanes (every lane takes part), no barrier
            const int src = (int)(nxt & 63u);
            na_ = shfl_u64(sa[0], src);
            if (MODEL == kTwoLane) nb_ = shfl_u64(sb[0], src);
        } else {
            xw[bo] = sa[0];
            if (MODEL == kTwoLane) xw[bo + 1] = sb[0];
            __syncthreads();
            na_ = xr[bo];
            if (MODEL == kTwoLane) nb_ = xr[bo + 1];
        }
#pragma unroll
        for (int i = 0; i < C; ++i) {
            uint64_t ha = na_, hb = nb_;
            if (i + 1 < C && i + 1 < cnt) {
                ha = sa[i + 1 < C ? i + 1 : i];
                hb = sb[i + 1 < C ? i + 1 : i];
            }
            sa[i] = funnel(sa[i], ha, delta);
            if (MODEL == kTwoLane) sb[i] = funnel(sb[i], hb, delta);
        }
        if (wrap) {
            off += 1;
            wb = (wb + 1 == nw) ? 0u : wb + 1;
            if (!sg && off == nw) off = 0;
        }
        sig = sig_new;
        bo ^= bstride;
    };

    // Heights and exact sums of a whole ring (slots at shift 0).
    auto measure = [&](uint32_t ri) {
        // slot base_slot+i holds word (off + base_slot + i) mod nw
        int32_t dl = 0;
#pragma unroll
        for (int i = 0; i < C; ++i)
            if (i < cnt) dl += 64 - 2 * (int32_t)__popcll(sa[i]);
        // inclusive prefix sum of the height steps over the workgroup: within
        // each wave by lane permutes (every lane takes part), then the wave
        // totals through LDS
        const uint32_t lane = tid & 63u, wv = tid >> 6;
        int32_t v = dl;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int32_t up = __shfl_up(v, (unsigned)d, 64);
            if (lane >= (uint32_t)d) v += up;
        }
        int32_t* s0p = scan;
        int32_t* wsum = scan + block;
        if (lane == 63u) wsum[wv] = v;
        if (lt == 0 && gi < G) {
            red[gi * 4 + 0] = 0;
            red[gi * 4 + 1] = 0;
            red[gi * 4 + 2] = 0;
            red[gi * 4 + 3] = 0;
        }
        __syncthreads();
        for (uint32_t w = 0; w < wv; ++w) v += wsum[w];
        s0p[tid] = v;
        __syncthreads();
        const int32_t before = (lane0 > 0) ? s0p[lane0 - 1] : 0;
        const int32_t excl = s0p[tid] - dl - before;
        const int32_t last = lane0 + Tr - 1 < block ? lane0 + Tr - 1 : block - 1;
        const int32_t gtot = s0p[last] - before;
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
            int64_t Jm = J;
            if constexpr (WRAPJ) {
                int64_t Mn = 0;
#pragma unroll
                for (int i = 0; i < C; ++i) {
                    if (i < cnt) {
                        uint32_t w = off + base_slot + (uint32_t)i;
                        if (w >= nw) w -= nw;
                        Mn += position_sum(sa[i], w);
                        if (MODEL == kTwoLane) Mn += position_sum(sb[i], w);
                    }
                }
                Jm = (int64_t)(64ull * nw) * J + Mn - Ms;
            }
            atomicAdd(&red[gi * 4 + 0], (unsigned long long)ls1);
            atomicAdd(&red[gi * 4 + 1], (unsigned long long)ls2);
            atomicAdd(&red[gi * 4 + 2], (unsigned long long)Jm);
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
    uint32_t shv = 0;
    uint32_t ri = 0;
    // sub-sweeps of this launch (at most 2^30: the host splits longer runs);
    // the hops of the lane's own cells add into the 64-bit J every
    // sub-sweep (one sign extension and one 64-bit add)
    const uint32_t nsub = (uint32_t)(P.g1 - P.g0);
    // first slot of this lane's wave (windows: one ring per workgroup, lt = tid)
    const uint32_t wave_slot0 = __builtin_amdgcn_readfirstlane(lt & ~63u) * (uint32_t)C;
    // sub-sweeps in which this wave's slots can still reach the output
    // (windows; whole rings: all)
    const uint32_t tlive =
        !seg ? 0xFFFFFFFFu : (nout + nsub > wave_slot0 ? nout + nsub - wave_slot0 : 0u);
    auto sub_sweeps = [&](auto lay) {
    constexpr int LAY = decltype(lay)::value;
    const bool sg = LAY == 0 ? seg : LAY == 1;
    for (uint32_t t = 0;; ++t) {
        const uint64_t g = P.g0 + t;
        if constexpr (MEAS) {
            while (ri < P.n_rec && P.rec_g[ri] == g) {
                shift_to(0, lay);  // uniform call: rings of one workgroup may differ in sig
                measure(ri);
                ++ri;
            }
        }
        if (t >= nsub) break;
        // SCA step: single lane even / odd pairs; two lanes even pairs,
        // A -> B, odd pairs, B -> A.  g is the same for the whole workgroup,
        // so skipping the exchange when the frame stays is a uniform branch.
        const uint32_t step = (MODEL == kTwoLane) ? (uint32_t)(g & 3u) : (uint32_t)(g & 1u);
        if constexpr (V == kSca) {
            // the odd pairs are the only step in the frame starting at odd
            // sites; lane changes draw their bits in the even frame
            const uint32_t frame = (MODEL == kTwoLane) ? (step == 2u ? 1u : 0u) : step;
            if (frame != sig) shift_to(frame, lay);
            cc.c2b = (kTagSublattice << 28) | (uint32_t)((g >> 32) & 0xFFFFu);
        } else {
            uint32_t sw;
            if constexpr (WU) {
                // lane l holds the draw of sub-sweep g + l from the last
                // multiple of 64 sub-sweeps into the launch (its quad's
                // block, word (g + l) mod 4): one vector Philox per 64
                // sub-sweeps, then one lane read each
                if ((t & 63u) == 0) {
                    const uint64_t gl = g + (threadIdx.x & 63u);
                    const uint64_t q = gl >> 2;
                    const Blk r = philox(0u, (uint32_t)q,
                                         (kTagShift << 28) | (uint32_t)((q >> 32) & 0xFFFFu),
                                         sample, cc.k0, cc.k1);
                    const uint32_t wq = (uint32_t)(gl & 3u);
                    shv = wq == 0 ? r.v[0] : wq == 1 ? r.v[1] : wq == 2 ? r.v[2] : r.v[3];
                }
                sw = (uint32_t)__builtin_amdgcn_readlane((int)shv, (int)(t & 63u));
            } else {
                const uint64_t quad = g >> 2;
                if (quad != shq) {
                    const Blk r = philox(0u, (uint32_t)quad,
                                         (kTagShift << 28) | (uint32_t)((quad >> 32) & 0xFFFFu),
                                         sample, cc.k0, cc.k1);
                    shblk[0] = r.v[0];
                    shblk[1] = r.v[1];
                    shblk[2] = r.v[2];
                    shblk[3] = r.v[3];
                    shq = quad;
                }
                const uint32_t gq = (uint32_t)(g & 3u);
                sw = gq == 0 ? shblk[0] : gq == 1 ? shblk[1] : gq == 2 ? shblk[2] : shblk[3];
            }
            shift_to(sw & cmask, lay);
            cc.c2b = (kTagAttempt << 28) | (uint32_t)((g >> 32) & 0xFFFFu);
            cc.c2c = (kTagChange << 28) | (uint32_t)((g >> 32) & 0xFFFFu);
        }
        cc.glo = (uint32_t)g;
        int32_t dj = 0;
        // Windows: content moves at most one slot to the left per frame
        // change, and nsub - t of them follow this sub-sweep, so slots at or
        // past nout + nsub - t can no longer reach the output (nor are they
        // owned).  A wave whose first slot is there skips its attempts.
        const bool live = !sg || t < tlive;
        // Wave-uniform rings, several slots per lane: whether this wave's
        // slots (words wb of its first lane onwards, 64 C of them) hold the
        // ring's last word, one scalar test per sub-sweep instead of one per
        // slot (with one slot per lane the test would only add work)
        bool wrap_wave = true;
        if constexpr (WRAPJ && WU && C > 1) {
            const uint32_t wbw = __builtin_amdgcn_readfirstlane(wb);
            wrap_wave = nw - 1u - wbw < 64u * (uint32_t)C;
        }
#pragma unroll
        for (int i = 0; i < C; ++i) {
            if (live && i < cnt) {
                uint32_t w = wb + (uint32_t)i;
                if (w >= nw) w -= nw;
                const uint32_t pos = off + base_slot + (uint32_t)i;  // window position
                uint64_t xa = sa[i];
                uint64_t xb = sb[i];
                uint64_t m0 = 0, m1 = 0;
                if (MODEL != kPlain && P.mplanes > 0) {
                    uint32_t ia, ib;
                    if (sg) {
                        ia = min(pos, mwords - 2);
                        ib = ia + 1;
                    } else {
                        ia = w;
                        ib = (w + 1 == nw) ? 0 : w + 1;
                    }
                    m0 = funnel(lmask[ia], lmask[ib], sig);
                    if ((MODEL == kDisorder || V == kSca) && P.mplanes > 1)
                        m1 = funnel(lmask[mwords + ia], lmask[mwords + ib], sig);
                }
                int32_t d = 0;
                if constexpr (V == kSca) {
                    cc.k = w;
                    if constexpr (MODEL == kTwoLane) {
                        if ((step & 1u) == 0)
                            d = sca_two_inlane(xa, xb, cc);
                        else if (step == 1)
                            sca_two_change(xa, xb, m0, cc);  // A -> B, u marks
                        else
                            sca_two_change(xb, xa, m1, cc);  // B -> A, v marks
                    } else {
                        d = sca_slot<Q0, MODEL == kDisorder>(xa, m0, m1, cc);
                    }
                } else if constexpr (HALF) {
                    cc.k = 2u * w;
                    d = cell_half_fast<BV, Q0, MODEL == kDisorder>(xa, m0, m1, cc);
                } else if constexpr (FAST) {
                    cc.k = w;
                    if (MODEL == kTwoLane)
                        cell_two_lane_fast<AV, BV, 64>(xa, xb, m0, cc);
                    else
                        d = cell_ring_fast<AV, BV, Q0, MODEL == kDisorder, 16>(xa, m0, m1, cc);
                } else {
                    for (uint32_t cq = 0; cq < cps; ++cq) {
                        cc.k = w * cps + cq;
                        const uint32_t bb = cq << lam;
                        if (MODEL == kTwoLane)
                            d += cell_two_lane_generic(xa, xb, m0, bb, lam, cc);
                        else
                            d += cell_ring_generic<MODEL == kDisorder>(xa, m0, m1, bb, lam, cc);
                    }
                }
                if constexpr (WRAPJ) {
                    // the closing bond's slot (owned by exactly one window)
                    if (wrap_wave) {
                        if (w == nw - 1u && (!sg || pos - lm < nout)) {
                            const uint64_t top = sig ? ~0ull << (64u - sig) : 0ull;
                            dj += (int32_t)__popcll(xa & top) - (int32_t)__popcll(sa[i] & top);
                            if (MODEL == kTwoLane)
                                dj += (int32_t)__popcll(xb & top) - (int32_t)__popcll(sb[i] & top);
                        }
                    }
                } else if (!sg || pos - lm < nout) {
                    // a window counts the hops of the cells it owns
                    dj += d;
                }
                sa[i] = xa;
                if (MODEL == kTwoLane) sb[i] = xb;
            }
        }
        J += dj;
    }
    };
    // measuring kernels run whole rings only; launches without measurements
    // take the loop of their form
    if constexpr (MEAS) {
        sub_sweeps(std::integral_constant<int, 0>{});
    } else if (seg) {
        sub_sweeps(std::integral_constant<int, 1>{});
    } else {
        sub_sweeps(std::integral_constant<int, 2>{});
    }
    shift_to(0, std::integral_constant<int, 0>{});
    int64_t Me = 0;  // position sum of the lane's own words at the end
#pragma unroll
    for (int i = 0; i < C; ++i) {
        if (i < cnt) {
            const uint32_t pos = off + base_slot + (uint32_t)i;
            if (!seg || pos - lm < nout) {
                uint32_t w = base + pos;
                while (w >= nw) w -= nw;
                uint64_t* dst = P.words_out + (size_t)ring * NPL * nw;
                dst[w] = sa[i];
                if (MODEL == kTwoLane) dst[nw + w] = sb[i];
                if constexpr (WRAPJ) {
                    Me += position_sum(sa[i], w);
                    if (MODEL == kTwoLane) Me += position_sum(sb[i], w);
                }
            }
        }
    }
    if constexpr (WRAPJ) J = (int64_t)(64ull * nw) * J + Me - Ms;
    // hops of the ring (whole ring) or of the window's own cells (segments)
    if (lt == 0 && gi < G) red[gi * 4 + 2] = 0;
    __syncthreads();
    if (act) atomicAdd(&red[gi * 4 + 2], (unsigned long long)J);
    __syncthreads();
    if (ring_ok && lt == 0) {
        if (seg)
            atomicAdd((unsigned long long*)&P.hops[ring], (unsigned long long)red[gi * 4 + 2]);
        else
            P.hops[ring] = hops0 + (int64_t)red[gi * 4 + 2];
    }
}

// Workgroup -> simulation of a packed launch (descriptors sorted by wg_begin).
__device__ __forceinline__ uint32_t find_desc(const SimDesc* __restrict__ d, uint32_t n,
                                              uint32_t wg) {
    uint32_t lo = 0, hi = n;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (d[mid].wg_begin <= wg)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// One simulation per launch: the descriptor travels in the kernel arguments.
template <int C, int MODEL, int V, bool Q0, bool MEAS, bool WU>
__global__ __launch_bounds__(sweep_max_block(C, MODEL)) void k_sweep(const SimDesc P) {
    sweep_body<C, MODEL, V, Q0, MEAS, WU>(P);
}

// Packed launch: workgroups of several simulations (requests) in one grid,
// each finding its descriptor in device memory.
template <int C, int MODEL, int V, bool Q0, bool MEAS>
__global__ __launch_bounds__(sweep_max_block(C, MODEL)) void k_sweep_packed(
    const SimDesc* __restrict__ descs, uint32_t n_desc) {
    sweep_body<C, MODEL, V, Q0, MEAS, false>(descs[find_desc(descs, n_desc, blockIdx.x)]);
}

// Dispatch of one model's kernels over (C, variant, q0).  Compiled variants:
// generic for every C; fast (ell = 64) for C <= 8 -- single lane with 5, 4 or
// 1 fields per word, each with and without backward hops; two lanes with 4 or
// 1 fields per word.
// Packed launches are compiled for the small-ring shapes (C <= 4).
// Measurement code is compiled in only where a launch measures (it costs
// registers, hence waves per SIMD).  A packed launch measures if any of its
// simulations does (`one` then carries n_rec > 0).
template <int MODEL, int C, int V, bool Q>
inline void launch_one(const SimDesc& one, const SimDesc* descs, uint32_t n_desc, uint32_t grid,
                       uint32_t block, size_t lds, hipStream_t st, hipEvent_t ev0,
                       hipEvent_t ev1) {
    const bool meas = one.n_rec > 0;
    if constexpr (C <= 4) {
        if (descs) {
            if (meas)
                hipLaunchKernelGGL((k_sweep_packed<C, MODEL, V, Q, true>), dim3(grid), dim3(block),
                                   lds, st, descs, n_desc);
            else
                hipLaunchKernelGGL((k_sweep_packed<C, MODEL, V, Q, false>), dim3(grid),
                                   dim3(block), lds, st, descs, n_desc);
            return;
        }
    }
    // one ring per wave: windows, whole rings of whole waves, or one whole
    // ring per workgroup (the lanes past it belong to no ring); the dispatch
    // records the kernel's own start and end in ev0 / ev1 if given
    const bool wu = one.segs > 1 || one.lanes_per_ring % 64u == 0 ||
                    (one.rings_per_wg == 1 && one.lanes_per_ring > 64u);
    if (meas) {
        if (wu)
            hipExtLaunchKernelGGL((k_sweep<C, MODEL, V, Q, true, true>), dim3(grid), dim3(block),
                                  (uint32_t)lds, st, ev0, ev1, 0u, one);
        else
            hipExtLaunchKernelGGL((k_sweep<C, MODEL, V, Q, true, false>), dim3(grid), dim3(block),
                                  (uint32_t)lds, st, ev0, ev1, 0u, one);
    } else {
        if (wu)
            hipExtLaunchKernelGGL((k_sweep<C, MODEL, V, Q, false, true>), dim3(grid), dim3(block),
                                  (uint32_t)lds, st, ev0, ev1, 0u, one);
        else
            hipExtLaunchKernelGGL((k_sweep<C, MODEL, V, Q, false, false>), dim3(grid),
                                  dim3(block), (uint32_t)lds, st, ev0, ev1, 0u, one);
    }
}

template <int MODEL, int C, int V>
inline void launch_q(const SweepKernel& k, const SimDesc& one, const SimDesc* descs,
                     uint32_t n_desc, uint32_t grid, uint32_t block, size_t lds, hipStream_t st,
                     hipEvent_t ev0, hipEvent_t ev1) {
    if constexpr (MODEL == kTwoLane) {
        launch_one<MODEL, C, V, false>(one, descs, n_desc, grid, block, lds, st, ev0, ev1);
    } else {
        if (k.q0)
            launch_one<MODEL, C, V, true>(one, descs, n_desc, grid, block, lds, st, ev0, ev1);
        else
            launch_one<MODEL, C, V, false>(one, descs, n_desc, grid, block, lds, st, ev0, ev1);
    }
}

template <int MODEL, int C>
inline hipError_t launch_c(const SweepKernel& k, const SimDesc& one, const SimDesc* descs,
                           uint32_t n_desc, uint32_t grid, uint32_t block, size_t lds,
                           hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
    if (descs && C > 4) return hipErrorInvalidValue;
    if (k.variant == kSca) {
        // two lanes hold twice the state: 16 slots per lane would spill
        if constexpr (MODEL != kTwoLane || C <= 8) {
            launch_q<MODEL, C, kSca>(k, one, descs, n_desc, grid, block, lds, st, ev0, ev1);
            return hipSuccess;
        }
        return hipErrorInvalidValue;
    }
    if (k.variant == kGeneric) {
        launch_one<MODEL, C, kGeneric, false>(one, descs, n_desc, grid, block, lds, st, ev0, ev1);
        return hipSuccess;
    }
    // two lanes hold twice the state: their specialised loops stop at 8 slots
    if constexpr (MODEL != kTwoLane || C <= 8) {
        if constexpr (MODEL == kTwoLane) {
            switch (k.variant) {
                case kF4B0: launch_one<MODEL, C, kF4B0, false>(one, descs, n_desc, grid, block, lds, st, ev0, ev1); return hipSuccess;
                case kF1: launch_one<MODEL, C, kF1, false>(one, descs, n_desc, grid, block, lds, st, ev0, ev1); return hipSuccess;
                default: return hipErrorInvalidValue;
            }
        } else {
            switch (k.variant) {
                case kF5B0: launch_q<MODEL, C, kF5B0>(k, one, descs, n_desc, grid, block, lds, st, ev0, ev1); return hipSuccess;
                case kF4B1: launch_q<MODEL, C, kF4B1>(k, one, descs, n_desc, grid, block, lds, st, ev0, ev1); return hipSuccess;
                case kF4B2: launch_q<MODEL, C, kF4B2>(k, one, descs, n_desc, grid, block, lds, st, ev0, ev1); return hipSuccess;
                case kH4B0:
                case kH4B1:
                    if constexpr ((MODEL == kPlain || MODEL == kDisorder) && C <= 8) {
                        if (k.variant == kH4B0)
                            launch_q<MODEL, C, kH4B0>(k, one, descs, n_desc, grid, block, lds, st, ev0, ev1);
                        else
                            launch_q<MODEL, C, kH4B1>(k, one, descs, n_desc, grid, block, lds, st, ev0, ev1);
                        return hipSuccess;
                    }
                    return hipErrorInvalidValue;
                case kF1:
                    if constexpr (C <= 8) {
                        launch_q<MODEL, C, kF1>(k, one, descs, n_desc, grid, block, lds, st, ev0, ev1);
                        return hipSuccess;
                    }
                    return hipErrorInvalidValue;
                default: return hipErrorInvalidValue;
            }
        }
    }
    return hipErrorInvalidValue;
}

template <int MODEL>
inline hipError_t launch_model(const SweepKernel& k, const SimDesc& one, const SimDesc* descs,
                               uint32_t n_desc, uint32_t grid, uint32_t block, size_t lds,
                               hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
    (void)hipGetLastError();  // drop errors left by earlier, unrelated calls
    hipError_t e;
    switch (k.C) {
        case 1: e = launch_c<MODEL, 1>(k, one, descs, n_desc, grid, block, lds, st, ev0, ev1); break;
        case 2: e = launch_c<MODEL, 2>(k, one, descs, n_desc, grid, block, lds, st, ev0, ev1); break;
        case 4: e = launch_c<MODEL, 4>(k, one, descs, n_desc, grid, block, lds, st, ev0, ev1); break;
        case 8: e = launch_c<MODEL, 8>(k, one, descs, n_desc, grid, block, lds, st, ev0, ev1); break;
        case 16: e = launch_c<MODEL, 16>(k, one, descs, n_desc, grid, block, lds, st, ev0, ev1); break;
        default: e = hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

// Whether launch_model has a kernel for (C, model, variant).
inline bool variant_compiled(uint32_t C, uint32_t model, uint32_t variant) {
    if (C != 1 && C != 2 && C != 4 && C != 8 && C != 16) return false;
    if (variant == kGeneric) return true;
    if (variant == kSca) return model != kTwoLane || C <= 8;
    if (model == kTwoLane) return C <= 8 && (variant == kF4B0 || variant == kF1);
    if (variant == kF1) return C <= 8;  // one field per draw: 16 slots would spill
    if (variant == kH4B0 || variant == kH4B1) return (model == kPlain || model == kDisorder) && C <= 8;
    return variant == kF5B0 || variant == kF4B1 || variant == kF4B2;
}

}  // namespace dev
}  // namespace asep
