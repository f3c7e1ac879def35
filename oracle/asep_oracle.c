/*
 * asep_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU reference for the ASEP / KPZ lattice-gas
 * Monte Carlo of Schulz, Odor, Odor and Nagy, "Simulation of 1+1 dimensional
 * surface growth and lattice gases using GPUs".  Only tests/, the smoke check
 * and the cpu_baseline leg of bench.py may load this file.  It shares no code,
 * header, table or constant generator with the HIP library: every routine is
 * written here from the paper and from the published Philox definition.
 *
 * Storage is one byte per site (0 = hole, 1 = particle); nothing is bit-packed,
 * blocked or reordered.  Each function names the passage it follows:
 *
 *   Sec. 2, Fig. kpzasep      RSOS <-> ASEP mapping: a particle hops to an empty
 *                             neighbour, right with probability p, left with q.
 *   Sec. 2.1 (CUDA)           flat start = alternating 1010...; one MCS = every
 *                             site updated once; parallel sub-lattice updates
 *                             replace random-sequential ones.  Here the parallel
 *                             schedule is a randomly shifted domain decomposition
 *                             (cells of ell sites, random-sequential attempts in
 *                             each cell, a fresh random shift per sub-sweep).
 *   Sec. 2.1, Eq. (W)         W^2 = (1/L) sum h^2 - ((1/L) sum h)^2.
 *   Sec. 2.2, Eq. (sampling)  t_{i+1} = 1.05 t_i, t_0 = 30.
 *   Sec. 2.3, Eq. (bimodal)   quenched slow sites with p_i = r p (and q_i = r q).
 *   Sec. 3                    two TASEP lanes with opposite drift and lane
 *                             changes at randomly chosen turning points.
 *   Salmon et al., SC'11      Philox4x32-10 counter-based generator.
 *
 * The schedule, the Philox counter layout and the threshold lowering are the
 * readings written down in the design notes; they are restated next to each
 * routine below.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "asep_oracle.h"

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11, Sec. 3 "Philox").        */
/* Round: two 32x32->64 products of counter words 0 and 2 with the           */
/* multipliers; the high halves are xored with the other counter words and   */
/* the key; the key is bumped by the Weyl constants between rounds.          */
/* ------------------------------------------------------------------------- */
#define PHX_MUL_A 0xD2511F53u
#define PHX_MUL_B 0xCD9E8D57u
#define PHX_WEYL_A 0x9E3779B9u
#define PHX_WEYL_B 0xBB67AE85u

void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHX_WEYL_A;
            k1 += PHX_WEYL_B;
        }
        uint64_t prod_a = (uint64_t)PHX_MUL_A * (uint64_t)c0;
        uint64_t prod_b = (uint64_t)PHX_MUL_B * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(prod_b >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)prod_b;
        uint32_t n2 = (uint32_t)(prod_a >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)prod_a;
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* Counter tags (top nibble of counter word 2). */
#define TAG_ATTEMPT 1u
#define TAG_SHIFT 2u
#define TAG_INIT 3u
#define TAG_DIS_P 4u
#define TAG_DIS_Q 5u
#define TAG_TURN 6u
#define TAG_RSU 7u
#define TAG_CHANGE 9u

static void draw(const orc_params *P, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                 uint32_t out[4]) {
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t key[2] = {P->seed, P->stream};
    orc_philox(ctr, key, out);
}

/* ------------------------------------------------------------------------- */
/* Probability -> integer threshold.  "with probability p" (Sec. 2.1) is     */
/* realised as r < T with r uniform on [0, 2^B):  T(x) = min(2^B,            */
/* floor(x 2^B)), computed in binary64 (scaling by 2^B and floor are exact). */
/* ------------------------------------------------------------------------- */
uint64_t orc_threshold(double x, int bits) {
    double scaled = floor(ldexp(x, bits));
    double cap = ldexp(1.0, bits);
    if (scaled >= cap) return (uint64_t)1 << bits;
    if (scaled <= 0.0) return 0;
    return (uint64_t)scaled;
}

static int is_pow2_log(uint32_t v) { return v >= 1 && v <= 30; }

/* The paper's two-sub-lattice update (Sec. 2.1, Fig. parasep) has no cells:
 * every pair of a sub-lattice is tried once per MCS with its own uniform
 * B-bit number, B at most 24. */
/* Two lanes (Sec. 3, the SCA sequence): in-lane hops of A (right, p) and B   */
/* (left, q) on the sub-lattices, lane changes at every site with u_x (A to   */
/* B) and v_x (B to A) equal to the lane rate, times the slow factor where    */
/* the site's u (v) mark is set; T = {p, q, lane rate, slow factor x lane     */
/* rate}.  Four steps per MCS (see sweep_two_lane_sublattice).               */
static int lower_sublattice(const orc_params *P, orc_sched *S) {
    const int two = P->model == ORC_TWO_LANE;
    if (P->model != ORC_RING && !two) return -1;
    if (two && P->turn_frac != 0) return -1;
    if (P->L < 4 || P->L % 2 != 0) return -1;
    if (!(P->p >= 0 && P->p <= 1 && P->q >= 0 && P->q <= 1)) return -1;
    const int BMAX = 24;
    uint64_t t[4];
    int nt = 0;
    S->TB[0] = orc_threshold(P->p, BMAX);
    S->TB[1] = orc_threshold(P->q, BMAX);
    if (two) {
        S->TB[2] = orc_threshold(P->lane_rate, BMAX);
        S->TB[3] = orc_threshold(P->slow_factor * P->lane_rate, BMAX);
    } else {
        S->TB[2] = orc_threshold(P->slow_factor * P->p, BMAX);
        S->TB[3] = orc_threshold(P->slow_factor * P->q, BMAX);
    }
    t[nt++] = S->TB[0];
    t[nt++] = S->TB[1];
    if (two) t[nt++] = S->TB[2];
    if (P->slow_frac > 0) {
        if (!two) t[nt++] = S->TB[2];
        t[nt++] = S->TB[3];
    }
    int b;
    if (P->rbits < 0) {
        for (b = 0; b <= BMAX; ++b) {
            int ok = 1;
            for (int i = 0; i < nt; ++i)
                if (t[i] % ((uint64_t)1 << (BMAX - b)) != 0) ok = 0;
            if (ok) break;
        }
    } else {
        b = P->rbits;
        if (b > BMAX) return -1;
        for (int i = 0; i < nt; ++i)
            if (t[i] % ((uint64_t)1 << (BMAX - b)) != 0) return -1;
    }
    S->B = BMAX;
    S->b = (uint32_t)b;
    for (int i = 0; i < 4; ++i) S->T[i] = S->TB[i] >> (BMAX - b);
    S->S = two ? 4 : 2;
    S->ell = 2;
    S->T_init = orc_threshold(P->density, 32);
    S->T_slow = orc_threshold(P->slow_frac, 32);
    S->T_turn = 0;
    return 0;
}

int orc_lower(const orc_params *P, orc_sched *S) {
    memset(S, 0, sizeof(*S));
    if (P->schedule == ORC_SCHED_SUBLATTICE) return lower_sublattice(P, S);
    if (P->schedule != ORC_SCHED_SHIFTED) return -1;
    if (!is_pow2_log(P->cell_log2)) return -1;
    uint32_t ell = 1u << P->cell_log2;
    int two = (P->model == ORC_TWO_LANE);
    if (P->L < 2 * (uint64_t)ell || P->L % ell != 0) return -1;
    if (P->subsweeps == 0) return -1;
    uint32_t per_mcs = two ? 4u * ell : ell; /* attempts per cell per MCS */
    if (per_mcs % P->subsweeps != 0) return -1;
    if (!(P->p >= 0 && P->p <= 1 && P->q >= 0 && P->q <= 1)) return -1;

    S->ell = ell;
    S->lam = P->cell_log2;
    S->ebits = two ? 2 : 0;
    S->B = 32 - S->lam - S->ebits;
    S->a = per_mcs / P->subsweeps;
    S->S = P->subsweeps;

    /* thresholds at B bits */
    uint64_t t[5];
    int nt = 0;
    if (!two) {
        S->TB[0] = orc_threshold(P->p, S->B);
        S->TB[1] = orc_threshold(P->q, S->B);
        S->TB[2] = orc_threshold(P->slow_factor * P->p, S->B);
        S->TB[3] = orc_threshold(P->slow_factor * P->q, S->B);
        t[nt++] = S->TB[0];
        t[nt++] = S->TB[1];
        if (P->slow_frac > 0) {
            t[nt++] = S->TB[2];
            t[nt++] = S->TB[3];
        }
    } else {
        S->TB[0] = orc_threshold(P->p, S->B); /* lane A hop right */
        S->TB[1] = orc_threshold(P->q, S->B); /* lane B hop left  */
        t[nt++] = S->TB[0];
        t[nt++] = S->TB[1];
        /* A lane change is decided by a 32-bit draw of its own (see
         * subsweep_two_lane), compared at the fewest bits that keep its
         * threshold exact. */
        S->TB[2] = orc_threshold(P->lane_rate, 32);
        uint32_t c = 0;
        while (c < 32 && S->TB[2] % ((uint64_t)1 << (32 - c)) != 0) ++c;
        S->bc = c;
    }
    /* precision b: the fewest low-order bits such that every threshold in use
     * is an exact multiple of 2^(B-b); then r < T at b bits has the same law. */
    int b;
    if (P->rbits < 0) {
        for (b = 0; b <= (int)S->B; ++b) {
            int ok = 1;
            for (int i = 0; i < nt; ++i)
                if (t[i] % ((uint64_t)1 << (S->B - b)) != 0) ok = 0;
            if (ok) break;
        }
    } else {
        b = P->rbits;
        if (b > (int)S->B) return -1;
        for (int i = 0; i < nt; ++i)
            if (t[i] % ((uint64_t)1 << (S->B - b)) != 0) return -1;
    }
    S->b = (uint32_t)b;
    for (int i = 0; i < 4; ++i) S->T[i] = S->TB[i] >> (S->B - b);
    if (two) S->T[2] = S->TB[2] >> (32 - S->bc);
    /* Cells of 32 sites whose field (position, event, compared bits) fits
     * in 8 bits take the four bytes of a word as fields, the position in
     * the low bits of its byte; every other schedule packs fields of
     * lam + ebits + b bits with the position on top. */
    S->jlow = (S->lam == 5 && S->lam + S->ebits + S->b <= 8) ? 1u : 0u;
    S->w = S->jlow ? 8u : S->lam + S->ebits + S->b;
    S->A = 32 / S->w;
    S->per_block = 4 * S->A;
    S->T_init = orc_threshold(P->density, 32);
    S->T_slow = orc_threshold(P->slow_frac, 32);
    S->T_turn = orc_threshold(P->turn_frac, 32);
    return 0;
}

/* Attempt m of cell k in sub-sweep g: block floor(m / 4A), word, slot, then
 * the field of w bits is split into (j | e | r) from the top, or, with byte
 * fields (jlow), into (r | e | j) from the top with j in the low lam bits. */
static void attempt_fields(const orc_params *P, const orc_sched *S, uint32_t sample, uint64_t k,
                           uint64_t g, uint32_t m, uint32_t blockbuf[4], uint32_t *cached_blk,
                           uint32_t *j, uint32_t *e, uint32_t *r) {
    uint32_t blk = m / S->per_block;
    uint32_t q = m % S->per_block;
    uint32_t wd = q / S->A;
    uint32_t sl = q % S->A;
    if (*cached_blk != blk) {
        uint32_t c2 = (TAG_ATTEMPT << 28) | (blk << 16) | (uint32_t)((g >> 32) & 0xFFFFu);
        draw(P, (uint32_t)k, (uint32_t)(g & 0xFFFFFFFFu), c2, sample, blockbuf);
        *cached_blk = blk;
    }
    uint32_t u = blockbuf[wd];
    uint64_t field = ((uint64_t)u >> (sl * S->w)) & ((((uint64_t)1) << S->w) - 1);
    if (S->jlow) {
        *j = (uint32_t)(field & ((1u << S->lam) - 1));
        *e = (uint32_t)((field >> S->lam) & ((1u << S->ebits) - 1));
        *r = (uint32_t)((field >> (S->lam + S->ebits)) & ((1u << S->b) - 1));
        return;
    }
    *r = (uint32_t)(field & ((((uint64_t)1) << S->b) - 1));
    *e = (uint32_t)((field >> S->b) & ((1u << S->ebits) - 1));
    *j = (uint32_t)(field >> (S->b + S->ebits));
}

/* The shift of sub-sweep g is word (g mod 4) of the block at counter
 * (0, lo32(g/4), SHIFT << 28 | hi16(g/4), sample), reduced mod ell. */
static uint32_t shift_draw(const orc_params *P, const orc_sched *S, uint32_t sample, uint64_t g) {
    uint32_t out[4];
    uint64_t quad = g / 4;
    uint32_t c2 = (TAG_SHIFT << 28) | (uint32_t)((quad >> 32) & 0xFFFFu);
    draw(P, 0, (uint32_t)(quad & 0xFFFFFFFFu), c2, sample, out);
    return out[g % 4] % S->ell;
}

/* ------------------------------------------------------------------------- */
/* Initial state and quenched planes (Sec. 2.1 flat start; Eq. bimodal;      */
/* Sec. 3 turning points).  A per-site draw uses word (x mod 4) of the block  */
/* at counter (x / 4, lane, tag << 28, sample or realization).               */
/* ------------------------------------------------------------------------- */
static uint32_t site_word(const orc_params *P, uint32_t tag, uint64_t x, uint32_t c1,
                          uint32_t c3) {
    uint32_t out[4];
    draw(P, (uint32_t)(x / 4), c1, tag << 28, c3, out);
    return out[x % 4];
}

void orc_init_state(const orc_params *P, const orc_sched *S, uint32_t sample, uint8_t *s) {
    int planes = P->model == ORC_TWO_LANE ? 2 : 1;
    for (int lane = 0; lane < planes; ++lane) {
        uint8_t *st = s + (uint64_t)lane * P->L;
        for (uint64_t x = 0; x < P->L; ++x) {
            if (P->init == ORC_INIT_FLAT) {
                st[x] = (x % 2 == 0) ? 1 : 0;
            } else {
                uint32_t u = site_word(P, TAG_INIT, x, (uint32_t)lane, sample);
                st[x] = ((uint64_t)u < S->T_init) ? 1 : 0;
            }
        }
    }
}

void orc_init_masks(const orc_params *P, const orc_sched *S, uint32_t realization,
                    uint8_t *slow_p, uint8_t *slow_q, uint8_t *turn) {
    for (uint64_t x = 0; x < P->L; ++x) {
        if (slow_p) slow_p[x] = ((uint64_t)site_word(P, TAG_DIS_P, x, 0, realization) < S->T_slow);
        if (slow_q) slow_q[x] = ((uint64_t)site_word(P, TAG_DIS_Q, x, 0, realization) < S->T_slow);
        if (turn) turn[x] = ((uint64_t)site_word(P, TAG_TURN, x, 0, realization) < S->T_turn);
    }
}

/* ------------------------------------------------------------------------- */
/* One sub-sweep g of the shifted domain decomposition.                      */
/* sigma = shift draw mod ell; cell k covers sites (sigma + k ell + j) mod L, */
/* j = 0..ell-1; each cell receives `a` random-sequential attempts.  An      */
/* attempt picks j; j = ell-1 (the bond leaving the cell) is a no-op.        */
/* Single lane: "10" at (x, x+1) hops right if r < T_p[x]; "01" hops left if */
/* r < T_q[x+1] (rates belong to the departure site).                         */
/* ------------------------------------------------------------------------- */
static void subsweep_ring(const orc_params *P, const orc_sched *S, uint32_t sample, uint64_t g,
                          uint8_t *s, const uint8_t *slow_p, const uint8_t *slow_q, int64_t *J) {
    const uint64_t L = P->L;
    const uint64_t ncell = L / S->ell;
    const uint32_t sigma = shift_draw(P, S, sample, g);
    for (uint64_t k = 0; k < ncell; ++k) {
        const uint64_t base = (sigma + k * S->ell) % L;
        uint32_t blockbuf[4];
        uint32_t cached = 0xFFFFFFFFu;
        for (uint32_t m = 0; m < S->a; ++m) {
            uint32_t j, e, r;
            attempt_fields(P, S, sample, k, g, m, blockbuf, &cached, &j, &e, &r);
            (void)e;
            if (j == S->ell - 1) continue;
            uint64_t x = (base + j) % L;
            uint64_t y = (x + 1) % L;
            uint64_t tp = (slow_p && slow_p[x]) ? S->T[2] : S->T[0];
            uint64_t tq = (slow_q && slow_q[y]) ? S->T[3] : S->T[1];
            if (s[x] == 1 && s[y] == 0 && (uint64_t)r < tp) {
                s[x] = 0;
                s[y] = 1;
                *J += 1;
            } else if (s[x] == 0 && s[y] == 1 && (uint64_t)r < tq) {
                s[x] = 1;
                s[y] = 0;
                *J -= 1;
            }
        }
    }
}

/* Two lanes (Sec. 3): lane A hops right, lane B hops left, and a particle may
 * change lane at a turning point when the other lane's site is empty.  The
 * event e of each attempt is 0: A hop on bond (x,x+1); 1: B hop on bond
 * (x,x+1) from x+1 to x; 2: A->B at x; 3: B->A at x.  Bond events with
 * j = ell-1 are no-ops; site events use every j.  Hops compare the field's r
 * with their thresholds.  A lane-change attempt that finds a turning point,
 * a particle on its side and a hole on the other is the cell's c-th
 * candidate of the sub-sweep (counted from 0 in attempt order); it draws the
 * 32-bit word c mod 4 of the block at counter (k, lo32(g), CHANGE << 28 |
 * (c / 4) << 16 | hi16(g), sample) and moves if the word's top bc bits are
 * below the lane-change threshold. */
static uint32_t change_word(const orc_params *P, uint32_t sample, uint64_t k, uint64_t g,
                            uint32_t c) {
    uint32_t out[4];
    uint32_t c2 = (TAG_CHANGE << 28) | ((c / 4) << 16) | (uint32_t)((g >> 32) & 0xFFFFu);
    draw(P, (uint32_t)k, (uint32_t)(g & 0xFFFFFFFFu), c2, sample, out);
    return out[c % 4];
}

static void subsweep_two_lane(const orc_params *P, const orc_sched *S, uint32_t sample, uint64_t g,
                              uint8_t *s, const uint8_t *turn, int64_t *J) {
    const uint64_t L = P->L;
    uint8_t *A = s;
    uint8_t *Bl = s + L;
    const uint64_t ncell = L / S->ell;
    const uint32_t sigma = shift_draw(P, S, sample, g);
    for (uint64_t k = 0; k < ncell; ++k) {
        const uint64_t base = (sigma + k * S->ell) % L;
        uint32_t blockbuf[4];
        uint32_t cached = 0xFFFFFFFFu;
        uint32_t cand = 0; /* lane-change candidates of this cell so far */
        for (uint32_t m = 0; m < S->a; ++m) {
            uint32_t j, e, r;
            attempt_fields(P, S, sample, k, g, m, blockbuf, &cached, &j, &e, &r);
            uint64_t x = (base + j) % L;
            uint64_t y = (x + 1) % L;
            if (e == 0) {
                if (j != S->ell - 1 && A[x] == 1 && A[y] == 0 && (uint64_t)r < S->T[0]) {
                    A[x] = 0;
                    A[y] = 1;
                    *J += 1;
                }
            } else if (e == 1) {
                if (j != S->ell - 1 && Bl[y] == 1 && Bl[x] == 0 && (uint64_t)r < S->T[1]) {
                    Bl[y] = 0;
                    Bl[x] = 1;
                    *J -= 1;
                }
            } else {
                uint8_t *from = (e == 2) ? A : Bl;
                uint8_t *to = (e == 2) ? Bl : A;
                if (turn[x] && from[x] == 1 && to[x] == 0) {
                    uint32_t u = change_word(P, sample, k, g, cand++);
                    uint64_t rc = S->bc ? ((uint64_t)u >> (32 - S->bc)) : 0;
                    if (rc < S->T[2]) {
                        from[x] = 0;
                        to[x] = 1;
                    }
                }
            }
        }
    }
}

/* ------------------------------------------------------------------------- */
/* The paper's two-sub-lattice update (Sec. 2.1, Fig. parasep).  One MCS:    */
/* phase 0 tries every pair (x, x+1) with x even, phase 1 every pair with x   */
/* odd.  Pairs of one phase share no site, so their order is free; in phase  */
/* 1 the pair (L-1, 0) that closes the ring is tried after the others, as in */
/* the paper.  A tried pair "10" hops right if U < T_p[x], a pair "01" hops   */
/* left if U < T_q[x+1] (rates of the departure site).                        */
/*                                                                            */
/* U is b bits.  Pair i of phase f (left site x = 2 i + f) belongs to group   */
/* w = i / 32 at position m = i mod 32; bit (b-1-n) of U, n = 0..b-1 from the */
/* top, is bit ((m mod 16) * 2 + m / 16) of random word n of group w, and     */
/* random word n is word (n mod 4) of the Philox block at counter            */
/* (w, lo32(g), 8 << 28 | (n / 4) << 16 | hi16(g), sample) with g = 2 t + f. */
/* ------------------------------------------------------------------------- */
#define TAG_SUBLATTICE 8u

static void phase_sublattice(const orc_params *P, const orc_sched *S, uint32_t sample, uint64_t g,
                             uint8_t *s, const uint8_t *slow_p, const uint8_t *slow_q, int64_t *J) {
    const uint64_t L = P->L;
    const uint64_t f = g % 2;
    const uint64_t npairs = L / 2;
    uint32_t words[24];
    for (uint64_t i = 0; i < npairs; ++i) {
        const uint64_t w = i / 32;
        const uint32_t m = (uint32_t)(i % 32);
        if (m == 0) {
            for (uint32_t n = 0; n < S->b; n += 4) {
                uint32_t out[4];
                uint32_t c2 = (TAG_SUBLATTICE << 28) | ((n / 4) << 16) |
                              (uint32_t)((g >> 32) & 0xFFFFu);
                draw(P, (uint32_t)w, (uint32_t)(g & 0xFFFFFFFFu), c2, sample, out);
                for (uint32_t k = 0; k < 4 && n + k < S->b; ++k) words[n + k] = out[k];
            }
        }
        const uint32_t bit = (m % 16) * 2 + m / 16;
        uint64_t u = 0;
        for (uint32_t n = 0; n < S->b; ++n) u = (u << 1) | ((words[n] >> bit) & 1u);
        const uint64_t x = 2 * i + f;
        const uint64_t y = (x + 1) % L;
        const uint64_t tp = (slow_p && slow_p[x]) ? S->T[2] : S->T[0];
        const uint64_t tq = (slow_q && slow_q[y]) ? S->T[3] : S->T[1];
        if (s[x] == 1 && s[y] == 0 && u < tp) {
            s[x] = 0;
            s[y] = 1;
            *J += 1;
        } else if (s[x] == 0 && s[y] == 1 && u < tq) {
            s[x] = 1;
            s[y] = 0;
            *J -= 1;
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Two lanes under the paper's SCA sequence (Sec. 3): one MCS is             */
/*   g = 4t:   even pairs of A (hop right, p) and of B (hop left, q);        */
/*   g = 4t+1: A -> B at every site (A occupied, B empty) with u_x;          */
/*   g = 4t+2: odd pairs of A and B, the closing pair (L-1, 0) among them    */
/*             (the paper's steps 3 and 4, disjoint pairs);                  */
/*   g = 4t+3: B -> A at every site (B occupied, A empty) with v_x.          */
/* J counts A hops minus B hops.  Random numbers: Philox blocks at counter   */
/* (w, lo32(g), 8 << 28 | blk << 16 | hi16(g), sample), word k of the step  */
/* being word k mod 4 of block k / 4.  In-lane: pair i (left site 2i + f)    */
/* is in group w = i / 32 at m = i mod 32, and bit b-1-n of lane A's U is    */
/* bit (m mod 16) * 2 + m / 16 of word 2n, of lane B's U the same bit of     */
/* word 2n+1.  Lane changes: site x is in group w = x / 64 at s = x mod 64,  */
/* and bit b-1-n of its U is bit s mod 32 of word 2n + s / 32.               */
/* ------------------------------------------------------------------------- */
static void draw_words(const orc_params *P, uint32_t sample, uint64_t g, uint64_t w, uint32_t n,
                       uint32_t *words) {
    for (uint32_t k = 0; k < n; k += 4) {
        uint32_t out[4];
        uint32_t c2 = (TAG_SUBLATTICE << 28) | ((k / 4) << 16) | (uint32_t)((g >> 32) & 0xFFFFu);
        draw(P, (uint32_t)w, (uint32_t)(g & 0xFFFFFFFFu), c2, sample, out);
        for (uint32_t i = 0; i < 4 && k + i < n; ++i) words[k + i] = out[i];
    }
}

static void inlane_two(const orc_params *P, const orc_sched *S, uint32_t sample, uint64_t g,
                       uint64_t f, uint8_t *a, uint8_t *b, int64_t *J) {
    const uint64_t L = P->L;
    uint32_t words[48];
    for (uint64_t i = 0; i < L / 2; ++i) {
        const uint32_t m = (uint32_t)(i % 32);
        if (m == 0) draw_words(P, sample, g, i / 32, 2 * S->b, words);
        const uint32_t bit = (m % 16) * 2 + m / 16;
        uint64_t ua = 0, ub = 0;
        for (uint32_t n = 0; n < S->b; ++n) {
            ua = (ua << 1) | ((words[2 * n] >> bit) & 1u);
            ub = (ub << 1) | ((words[2 * n + 1] >> bit) & 1u);
        }
        const uint64_t x = 2 * i + f;
        const uint64_t y = (x + 1) % L;
        if (a[x] == 1 && a[y] == 0 && ua < S->T[0]) {
            a[x] = 0;
            a[y] = 1;
            *J += 1;
        }
        if (b[y] == 1 && b[x] == 0 && ub < S->T[1]) {
            b[y] = 0;
            b[x] = 1;
            *J -= 1;
        }
    }
}

static void lane_change_two(const orc_params *P, const orc_sched *S, uint32_t sample, uint64_t g,
                            uint8_t *from, uint8_t *to, const uint8_t *mark) {
    const uint64_t L = P->L;
    uint32_t words[48];
    for (uint64_t x = 0; x < L; ++x) {
        const uint32_t sx = (uint32_t)(x % 64);
        if (sx == 0) draw_words(P, sample, g, x / 64, 2 * S->b, words);
        uint64_t u = 0;
        for (uint32_t n = 0; n < S->b; ++n)
            u = (u << 1) | ((words[2 * n + sx / 32] >> (sx % 32)) & 1u);
        const uint64_t thr = (mark && mark[x]) ? S->T[3] : S->T[2];
        if (from[x] == 1 && to[x] == 0 && u < thr) {
            from[x] = 0;
            to[x] = 1;
        }
    }
}

static void sweep_two_lane_sublattice(const orc_params *P, const orc_sched *S, uint32_t sample,
                                      uint8_t *s, const uint8_t *umark, const uint8_t *vmark,
                                      uint64_t t0, uint64_t n_mcs, int64_t *J) {
    uint8_t *a = s, *b = s + P->L;
    for (uint64_t t = t0; t < t0 + n_mcs; ++t) {
        inlane_two(P, S, sample, 4 * t, 0, a, b, J);
        lane_change_two(P, S, sample, 4 * t + 1, a, b, umark);
        inlane_two(P, S, sample, 4 * t + 2, 1, a, b, J);
        lane_change_two(P, S, sample, 4 * t + 3, b, a, vmark);
    }
}

void orc_sweep(const orc_params *P, const orc_sched *S, uint32_t sample, uint8_t *s,
               const uint8_t *mask_a, const uint8_t *mask_b, uint64_t t0, uint64_t n_mcs,
               int64_t *J) {
    if (P->schedule == ORC_SCHED_SUBLATTICE && P->model == ORC_TWO_LANE) {
        sweep_two_lane_sublattice(P, S, sample, s, mask_a, mask_b, t0, n_mcs, J);
        return;
    }
    if (P->schedule == ORC_SCHED_SUBLATTICE) {
        for (uint64_t t = t0; t < t0 + n_mcs; ++t)
            for (uint64_t phase = 0; phase < 2; ++phase)
                phase_sublattice(P, S, sample, 2 * t + phase, s, mask_a, mask_b, J);
        return;
    }
    for (uint64_t t = t0; t < t0 + n_mcs; ++t) {
        for (uint32_t sub = 0; sub < S->S; ++sub) {
            uint64_t g = t * S->S + sub;
            if (P->model == ORC_TWO_LANE)
                subsweep_two_lane(P, S, sample, g, s, mask_a, J);
            else
                subsweep_ring(P, S, sample, g, s, mask_a, mask_b, J);
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Heights and roughness (Sec. 2.1, Eq. W).  h_0 = 0 and                      */
/* h_{x+1} = h_x + 1 - 2 s_x, so "10" is a local minimum and a right hop      */
/* deposits.  S1 = sum_x h_x and S2 = sum_x h_x^2 over x = 0..L-1, exact.     */
/* ------------------------------------------------------------------------- */
void orc_sums(const uint8_t *s, uint64_t L, int64_t *S1, uint64_t *S2_lo, int64_t *S2_hi,
              int64_t *N) {
    __int128 s1 = 0, s2 = 0;
    int64_t h = 0, n = 0;
    for (uint64_t x = 0; x < L; ++x) {
        s1 += h;
        s2 += (__int128)h * h;
        h += 1 - 2 * (int64_t)s[x];
        n += s[x];
    }
    *S1 = (int64_t)s1;
    *S2_lo = (uint64_t)(unsigned __int128)s2;
    *S2_hi = (int64_t)(s2 >> 64);
    *N = n;
}

/* W^2 = (L S2 - S1^2) / L^2: the numerator is exact in 128-bit integers and
 * converted once. */
double orc_w2(uint64_t L, int64_t S1, uint64_t S2_lo, int64_t S2_hi) {
    __int128 s2 = ((__int128)S2_hi << 64) | (__int128)S2_lo;
    __int128 num = (__int128)L * s2 - (__int128)S1 * S1;
    return (double)num / ((double)L * (double)L);
}

/* Quenched planes of one realisation: the turning plane of the shifted     */
/* two-lane model; the slow-p (u) and slow-q (v) planes of a disordered ring */
/* (q plane only if q > 0) or of the two-lane SCA.                           */
static void alloc_masks(const orc_params *P, const orc_sched *S, uint32_t realization,
                        uint8_t **ma, uint8_t **mb) {
    const int sca_two = P->model == ORC_TWO_LANE && P->schedule == ORC_SCHED_SUBLATTICE;
    if (P->model == ORC_TWO_LANE && !sca_two) {
        *ma = (uint8_t *)calloc(P->L, 1);
        orc_init_masks(P, S, realization, NULL, NULL, *ma);
    } else if (P->slow_frac > 0) {
        *ma = (uint8_t *)calloc(P->L, 1);
        if (P->q > 0 || sca_two) *mb = (uint8_t *)calloc(P->L, 1);
        orc_init_masks(P, S, realization, *ma, *mb, NULL);
    }
}

/* Full run of one sample: init, then for each requested time t (ascending,
 * t = 0 meaning the initial state) advance to t and record (S1, S2, J, N). */
int orc_run(const orc_params *P, uint32_t sample, const uint64_t *times, uint32_t n_times,
            orc_record *rec, uint8_t *final_state) {
    orc_sched S;
    if (orc_lower(P, &S) != 0) return -1;
    int planes = P->model == ORC_TWO_LANE ? 2 : 1;
    uint8_t *s = (uint8_t *)calloc((size_t)P->L * planes, 1);
    uint8_t *ma = NULL, *mb = NULL;
    uint32_t spd = P->samples_per_disorder ? P->samples_per_disorder : 1;
    uint32_t realization = sample / spd;
    if (!s) return -2;
    orc_init_state(P, &S, sample, s);
    alloc_masks(P, &S, realization, &ma, &mb);
    int64_t J = 0;
    uint64_t t = 0;
    for (uint32_t i = 0; i < n_times; ++i) {
        if (times[i] < t) {
            free(s);
            free(ma);
            free(mb);
            return -1;
        }
        orc_sweep(P, &S, sample, s, ma, mb, t, times[i] - t, &J);
        t = times[i];
        orc_sums(s, P->L, &rec[i].S1, &rec[i].S2_lo, &rec[i].S2_hi, &rec[i].N);
        if (P->model == ORC_TWO_LANE) {
            int64_t nb = 0;
            for (uint64_t x = 0; x < P->L; ++x) nb += s[P->L + x];
            rec[i].N += nb;
        }
        rec[i].J = J;
    }
    if (final_state) memcpy(final_state, s, (size_t)P->L * planes);
    free(s);
    free(ma);
    free(mb);
    return 0;
}

/* Continue a run from a given state (checkpoint/resume and chunk checks). */
int orc_advance(const orc_params *P, uint32_t sample, uint8_t *s, uint64_t t0, uint64_t n_mcs,
                int64_t *J) {
    orc_sched S;
    if (orc_lower(P, &S) != 0) return -1;
    uint8_t *ma = NULL, *mb = NULL;
    uint32_t spd = P->samples_per_disorder ? P->samples_per_disorder : 1;
    uint32_t realization = sample / spd;
    alloc_masks(P, &S, realization, &ma, &mb);
    orc_sweep(P, &S, sample, s, ma, mb, t0, n_mcs, J);
    free(ma);
    free(mb);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Random-sequential update (Sec. 2.1: the serial dynamics the parallel       */
/* update is compared with).  One MCS = L attempts; each picks a bond         */
/* (x, x+1) uniformly (word 0 of its own Philox block, x = floor(u L / 2^32)) */
/* and accepts with 32-bit thresholds from word 1.                           */
/* ------------------------------------------------------------------------- */
int orc_rsu(const orc_params *P, uint32_t sample, uint8_t *s, uint64_t t0, uint64_t n_mcs,
            int64_t *J) {
    uint64_t L = P->L;
    uint64_t tp = orc_threshold(P->p, 32), tq = orc_threshold(P->q, 32);
    for (uint64_t t = t0; t < t0 + n_mcs; ++t) {
        for (uint64_t i = 0; i < L; ++i) {
            uint64_t n = t * L + i;
            uint32_t out[4];
            draw(P, (uint32_t)n, (uint32_t)(n >> 32), TAG_RSU << 28, sample, out);
            uint64_t x = ((uint64_t)out[0] * L) >> 32;
            uint64_t y = (x + 1) % L;
            if (s[x] == 1 && s[y] == 0 && (uint64_t)out[1] < tp) {
                s[x] = 0;
                s[y] = 1;
                *J += 1;
            } else if (s[x] == 0 && s[y] == 1 && (uint64_t)out[1] < tq) {
                s[x] = 1;
                s[y] = 0;
                *J -= 1;
            }
        }
    }
    return 0;
}

/* Sampling times of Eq. (sampling): t_0 = 30, t_{i+1} = 1.05 t_i with real t;
 * a sample is taken at ceil(t_i) for every t_i <= t_max, preceded by t = 0. */
uint32_t orc_sample_times(double t0, double factor, uint64_t t_max, uint64_t *out, uint32_t cap) {
    uint32_t n = 0;
    if (cap > 0) out[n++] = 0;
    double t = t0;
    while (t <= (double)t_max) {
        uint64_t c = (uint64_t)ceil(t);
        if (c > t_max) break;
        if (n == 0 || out[n - 1] != c) {
            if (n >= cap) break;
            out[n++] = c;
        }
        t = t * factor;
    }
    return n;
}
