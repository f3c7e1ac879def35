/*
 * asep_oracle.h -- TEST INFRASTRUCTURE ONLY (see asep_oracle.c).
 * Declarations of the plain CPU reference.  Not included by, and not sharing
 * anything with, the HIP library.
 */
#ifndef ASEP_ORACLE_H
#define ASEP_ORACLE_H

#include <stdint.h>

#define ORC_RING 0
#define ORC_TWO_LANE 1
#define ORC_INIT_FLAT 0
#define ORC_INIT_BERNOULLI 1
#define ORC_SCHED_SHIFTED 0
#define ORC_SCHED_SUBLATTICE 1

typedef struct {
    uint32_t model;     /* ORC_RING or ORC_TWO_LANE */
    uint32_t init;      /* ORC_INIT_FLAT or ORC_INIT_BERNOULLI */
    uint64_t L;         /* sites per ring (per lane) */
    double density;     /* Bernoulli start */
    double p;           /* ring: right hop; two-lane: lane A hop right */
    double q;           /* ring: left hop;  two-lane: lane B hop left */
    double slow_frac;   /* ring: fraction c of slow sites (Eq. bimodal's Q) */
    double slow_factor; /* ring: slow-site factor r */
    uint32_t samples_per_disorder;
    double lane_rate;   /* two-lane: lane-change probability at turning points */
    double turn_frac;   /* two-lane: fraction of turning points */
    uint32_t seed;      /* Philox key word 0 */
    uint32_t stream;    /* Philox key word 1 */
    uint32_t cell_log2; /* ell = 2^cell_log2 */
    uint32_t subsweeps; /* S */
    int32_t rbits;      /* -1: fewest exact bits; else explicit */
    uint32_t schedule;  /* ORC_SCHED_SHIFTED or ORC_SCHED_SUBLATTICE */
} orc_params;

typedef struct {
    uint32_t ell, lam, ebits, B, b, w, A, per_block, a, S;
    uint64_t TB[4]; /* thresholds at B bits */
    uint64_t T[4];  /* thresholds at b bits: ring {p, q, r p, r q}; two-lane {A, B, lane} */
    uint64_t T_init, T_slow, T_turn; /* 32-bit thresholds */
    uint32_t bc;    /* two lanes, shifted schedule: bits compared for a lane change
                       (T[2] is the lane-change threshold at bc bits) */
    uint32_t jlow;  /* cells of 32 sites whose field fits a byte: fields are the
                       four bytes of a word, position in the low bits */
} orc_sched;

typedef struct {
    int64_t S1;
    uint64_t S2_lo;
    int64_t S2_hi;
    int64_t J;
    int64_t N;
} orc_record;

void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
uint64_t orc_threshold(double x, int bits);
int orc_lower(const orc_params *P, orc_sched *S);
void orc_init_state(const orc_params *P, const orc_sched *S, uint32_t sample, uint8_t *s);
void orc_init_masks(const orc_params *P, const orc_sched *S, uint32_t realization,
                    uint8_t *slow_p, uint8_t *slow_q, uint8_t *turn);
void orc_sweep(const orc_params *P, const orc_sched *S, uint32_t sample, uint8_t *s,
               const uint8_t *mask_a, const uint8_t *mask_b, uint64_t t0, uint64_t n_mcs,
               int64_t *J);
void orc_sums(const uint8_t *s, uint64_t L, int64_t *S1, uint64_t *S2_lo, int64_t *S2_hi,
              int64_t *N);
double orc_w2(uint64_t L, int64_t S1, uint64_t S2_lo, int64_t S2_hi);
int orc_run(const orc_params *P, uint32_t sample, const uint64_t *times, uint32_t n_times,
            orc_record *rec, uint8_t *final_state);
int orc_advance(const orc_params *P, uint32_t sample, uint8_t *s, uint64_t t0, uint64_t n_mcs,
                int64_t *J);
int orc_rsu(const orc_params *P, uint32_t sample, uint8_t *s, uint64_t t0, uint64_t n_mcs,
            int64_t *J);
uint32_t orc_sample_times(double t0, double factor, uint64_t t_max, uint64_t *out, uint32_t cap);

#endif
