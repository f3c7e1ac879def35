/*
 * asep.h -- C ABI of the MI355X (gfx950) ASEP / KPZ lattice-gas engine.
 *
 * The engine simulates the one-dimensional binary lattice gas that encodes
 * restricted solid-on-solid KPZ growth (Schulz, Odor, Odor, Nagy,
 * "Simulation of 1+1 dimensional surface growth and lattice gases using GPUs"):
 *
 *   - Sec. 2, Fig. kpzasep: periodic rings of L sites, n_i in {0,1}; a particle
 *     hops right onto an empty site with probability p and left with q; up to
 *     the height convention a right hop of "10" is a deposition on a local
 *     minimum, a left hop of "01" an evaporation.
 *   - Sec. 2.1: flat start 1010..., one Monte Carlo step (MCS) updates every
 *     site once on average, W^2(L,t) measured from the heights at chosen times
 *     and averaged over independent samples (Eq. W).
 *   - Sec. 2.2, Eq. (sampling): geometric sampling times t_{i+1} = 1.05 t_i.
 *   - Sec. 2.3, Eq. (bimodal): quenched columnar disorder, a fraction Q of
 *     sites with p_i = r p (and q_i = r q).
 *   - Sec. 3: two lanes with opposite drift and lane changes at turning points.
 *
 * Parallel update rule.  Each MCS is S sub-sweeps.  Sub-sweep g = t*S + s
 * draws a shift sigma in [0, ell) and cuts the ring into cells of ell sites
 * starting at sigma; every cell receives ell/S (two lanes: 4 ell/S)
 * random-sequential attempts on a uniformly chosen offset j, the offset
 * j = ell-1 (the bond leaving the cell) being a no-op.  Cells are disjoint,
 * so all of them are updated at once.  The paper's own two-sub-lattice
 * update (Sec. 2.1, Fig. parasep) is the second schedule (asep_params.schedule):
 * S = 2 sub-sweeps, the first trying every pair (x, x+1) with x even once,
 * the second every pair with x odd.  Random numbers are Philox4x32-10
 * blocks keyed by (seed, stream) with counters built from (cell, g, sample),
 * so a result depends only on the parameters, never on how the work is
 * batched, chunked or laid out on the device.
 *
 * Conventions:
 *   - every call returns 0 (ASEP_OK) or a negative ASEP_E_* code; out
 *     parameters are untouched on error; no exception crosses the ABI;
 *   - device pointers are HIP device addresses on the simulation's device;
 *     host pointers are ordinary process memory; output arrays are owned by
 *     the caller, handles by the library;
 *   - an asep_sim is used from one thread at a time; the server calls
 *     (asep_submit, asep_poll, asep_wait, asep_cancel) are thread-safe.
 */
#ifndef ASEP_H
#define ASEP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ASEP_ABI_VERSION 3u

enum {
    ASEP_OK = 0,
    ASEP_E_INVAL = -1,       /* a parameter is out of its documented range */
    ASEP_E_UNSUPPORTED = -2, /* valid, but not handled by this build */
    ASEP_E_NOMEM = -3,       /* device or host allocation failed */
    ASEP_E_DEVICE = -4,      /* a HIP call failed; see asep_last_device_error() */
    ASEP_E_BUSY = -5,        /* the server queue is full */
    ASEP_E_PENDING = -6,     /* the request has not finished yet */
    ASEP_E_CANCELLED = -7,   /* the request was cancelled */
    ASEP_E_TIMEOUT = -8,     /* asep_wait ran out of time */
    ASEP_E_NOTFOUND = -9,    /* unknown ticket */
    ASEP_E_TOO_LARGE = -10   /* larger than the fixed workspace of asep_run_noalloc */
};

enum { ASEP_MODEL_RING = 0, ASEP_MODEL_TWO_LANE = 1 };
enum { ASEP_INIT_FLAT = 0, ASEP_INIT_BERNOULLI = 1 };
enum { ASEP_SCHED_SHIFTED = 0, ASEP_SCHED_SUBLATTICE = 1 };

/* Run parameters.  Zero-initialise, then set abi_version = ASEP_ABI_VERSION
 * and the fields of the run; every field left at zero takes its default. */
typedef struct asep_params {
    uint32_t abi_version;
    uint32_t model;    /* ASEP_MODEL_RING | ASEP_MODEL_TWO_LANE */
    uint64_t L;        /* sites per ring (per lane); multiple of 64 and of 2^cell_log2,
                          at least two cells */
    uint32_t samples;  /* independent rings (>= 1) */
    uint32_t sample_offset; /* index of the first sample: sample i of this run is
                               realisation sample_offset + i of the ensemble */
    uint32_t init;     /* ASEP_INIT_FLAT (1010...) | ASEP_INIT_BERNOULLI(density) */
    uint32_t samples_per_disorder; /* samples sharing one quenched realisation
                                      (realisation = sample / this); 0 means 1 */
    double density;    /* Bernoulli start, in [0,1] */
    double p;          /* ring: right-hop probability; two lanes: lane A (rightward) */
    double q;          /* ring: left-hop probability;  two lanes: lane B (leftward) */
    double slow_frac;  /* ring: fraction of slow sites (Eq. bimodal's Q), [0,1];
                          two lanes under ASEP_SCHED_SUBLATTICE: fraction of
                          marked sites in each of the u and v planes */
    double slow_factor;/* ring: rate factor r of slow sites; two-lane SCA:
                          lane-change factor at marked sites; [0,1] */
    double lane_rate;  /* two lanes: lane-change probability at a turning point */
    double turn_frac;  /* two lanes: fraction of turning points, [0,1] */
    uint32_t seed;     /* Philox key word 0 */
    uint32_t stream;   /* Philox key word 1 (the caller's request identity) */
    int32_t cell_log2; /* ell = 2^cell_log2 in [1,6]; 0 = from the tuning table
                          (asep_tuning_load) if an entry matches, else 6 */
    int32_t subsweeps; /* S, dividing ell (two lanes: 4 ell); 0 = from the
                          tuning table if an entry matches, else 4 */
    int32_t rbits;     /* bits compared against each acceptance threshold:
                          0 (or negative) = the fewest that keep every threshold
                          exact, n >= 1 = exactly n (ASEP_E_INVAL if a threshold
                          is not exact at n bits); an explicit 0 would always
                          equal the automatic choice, so 0 means automatic.
                          Two lanes under the shifted schedule: the hop
                          thresholds only; a lane change compares its own
                          32-bit draw at the fewest bits that keep the lane
                          rate exact */
    uint32_t windows;  /* launch shape only, never results: 0 = from the tuning
                          table, else automatic; 1 = each ring whole in one
                          workgroup, n >= 2 = each ring cut into n windows */
    uint32_t window_sweeps; /* sub-sweeps per launch of a windowed ring; 0 = from
                               the tuning table, else 63 */
    uint32_t rings_per_wg;  /* launch shape only: whole rings packed per
                               workgroup; 0 = from the tuning table, else
                               automatic */
    uint32_t schedule; /* ASEP_SCHED_SHIFTED (the shifted cells above) or
                          ASEP_SCHED_SUBLATTICE, the paper's SCA:
                          rings (Sec. 2.1, Fig. parasep): every pair (x, x+1)
                          with x even tried once, then every pair with x odd,
                          the closing pair (L-1, 0) among them; cell_log2 and
                          subsweeps must be 0 or 1 and 2;
                          two lanes (Sec. 3's sequence): even pairs of A and B,
                          A -> B at every site with u_x, odd pairs, B -> A with
                          v_x; u_x = v_x = lane_rate, times slow_factor where
                          the site's u (v) mark is set (marks: independent
                          Bernoulli(slow_frac) planes); turn_frac must be 0,
                          cell_log2 and subsweeps 0 or 1 and 4.
                          Each tried pair or site compares a 24-bit uniform
                          with its threshold (rbits as above, at most 24) */
} asep_params;

/* Roughness and current of one sample at one time (Sec. 2.1, Eq. W).
 * Heights: h_0 = 0, h_{x+1} = h_x + 1 - 2 n_x (two lanes: lane A).
 * sum_h = S1 = sum_x h_x, sum_h2 = S2 = sum_x h_x^2 as a 128-bit value
 * (hi:lo), hops = J = cumulative right hops minus left hops (two lanes: lane A
 * hops minus lane B hops), particles = N (two lanes: both lanes),
 * w2 = (L S2 - S1^2) / L^2 formed once in binary64 from the exact integers. */
typedef struct asep_rough {
    int64_t sum_h;
    uint64_t sum_h2_lo;
    int64_t sum_h2_hi;
    int64_t hops;
    int64_t particles;
    double w2;
} asep_rough;

typedef struct asep_sim asep_sim;

/* Size in bytes of the two device buffers a simulation needs (Sec. 2.1: the
 * ring's sites, one bit each here; Sec. 2.3 and 3: the quenched planes):
 * state: samples x planes x L/64 words (uint64, bit b of word w = site 64w+b);
 * aux:   quenched planes, hop counters and record staging. */
int asep_buffer_sizes(const asep_params* p, size_t* state_bytes, size_t* aux_bytes);

/* Sec. 2.1 (flat start, exchange probabilities), Sec. 2.3, Sec. 3:
 * validate, lower probabilities to integer thresholds, allocate the device
 * buffers (library-owned) on the current HIP device, create a stream and
 * initialise the state and the quenched planes.  *out receives the handle;
 * p->cell_log2, p->subsweeps and p->rbits as used are readable through
 * asep_get_params. */
int asep_create(const asep_params* p, asep_sim** out);

/* As asep_create, but the state and aux buffers are borrowed device memory
 * (e.g. torch tensors) of at least asep_buffer_sizes() bytes, and all work is
 * queued on the borrowed hip_stream (hipStream_t; NULL = the null stream).
 * The caller keeps the buffers and the stream alive until asep_destroy. */
int asep_create_ext(const asep_params* p, void* state_dev, size_t state_bytes, void* aux_dev,
                    size_t aux_bytes, void* hip_stream, asep_sim** out);

/* Parameters as resolved at creation: defaults and tuning-table values
 * filled in (cell_log2, subsweeps, rbits, samples_per_disorder, and the
 * launch-shape fields as used). */
int asep_get_params(const asep_sim* s, asep_params* out);

/* Launch plan of a simulation: how its rings are laid out on the device
 * (Sec. 2.1: independent rings per block, one ring held on chip; Sec. 2.4:
 * rings longer than on-chip memory pass through device memory).  The plan is
 * launch shape only and never changes a result. */
enum {
    ASEP_LOOP_GENERIC = 0,   /* any cell size and attempt count */
    ASEP_LOOP_F5B0 = 1,      /* ell = 64, 16 attempts: 5 per 32-bit draw, no compared bit */
    ASEP_LOOP_F4B1 = 2,      /* 4 per draw, 1 compared bit */
    ASEP_LOOP_F4B2 = 3,      /* 4 per draw, 2 compared bits */
    ASEP_LOOP_F1 = 4,        /* 1 per draw, compared bits at run time */
    ASEP_LOOP_F4B0_LANES = 5,/* two lanes, 64 attempts: 4 per draw, no compared bit */
    ASEP_LOOP_SUBLATTICE = 6,/* the paper's two-sub-lattice update */
    ASEP_LOOP_H4B0 = 7,      /* ell = 32, 2 sub-sweeps: a slot's halves are two cells,
                                4 byte fields per draw, no compared bit */
    ASEP_LOOP_H4B1 = 8       /* ell = 32, 2 sub-sweeps: 4 byte fields per draw, 1 compared bit */
};
typedef struct asep_plan {
    uint32_t windows;        /* 1: each ring whole in one workgroup; n >= 2: windows per ring */
    uint32_t window_sweeps;  /* sub-sweeps per launch of a windowed ring (0: whole rings) */
    uint32_t slots_per_lane; /* 64-site words held by each lane: 1, 2, 4, 8 or 16 */
    uint32_t block;          /* lanes per workgroup */
    uint32_t lanes_per_ring; /* lanes serving one ring (whole rings) or one window */
    uint32_t rings_per_wg;   /* whole rings per workgroup */
    uint32_t grid;           /* workgroups per sweep launch */
    uint32_t attempt_loop;   /* ASEP_LOOP_* */
    uint32_t backward_hops;  /* 0 when no backward hop can happen (q = 0 and r q = 0) */
    uint32_t packable;       /* 1 when the request loop may share a launch with others */
    uint32_t reserved[6];
} asep_plan;
int asep_get_plan(const asep_sim* s, asep_plan* out);

/* What asep_create would resolve, without creating anything (host only, no
 * device memory or work): *resolved receives the parameters with defaults
 * and tuning-table values filled in, *plan (may be NULL) the launch plan for
 * the current HIP device (gfx950's limits if none is visible).  Same
 * validation and error codes as asep_create. */
int asep_resolve(const asep_params* p, asep_params* resolved, asep_plan* plan);

/* Sec. 2.1 (one MCS: every site updated once on average; here S sub-sweeps
 * of the parallel update): advance every sample by n_mcs Monte Carlo steps; asynchronous on the
 * simulation's stream.  Splitting n_mcs into several calls gives bit-identical
 * results. */
int asep_sweep(asep_sim* s, uint64_t n_mcs);

/* Sec. 2.1, Eq. W: measure the current state (heights, their exact sums,
 * W^2): out[samples] (host array).  Synchronises. */
int asep_roughness(asep_sim* s, asep_rough* out);

/* Sec. 2.2, Eq. (sampling): W^2 recorded at chosen times while the run
 * advances.  Advance through ascending absolute times (MCS, each >= asep_time()) and
 * measure at each: out[n_times * samples] (host array, time-major).  Equal to
 * asep_sweep + asep_roughness at each time, bit for bit.  Synchronises. */
int asep_run(asep_sim* s, const uint64_t* times, uint32_t n_times, asep_rough* out);

/* Sec. 2.1 (independent realisations advanced together on the device):
 * asep_run for several simulations at once: every simulation advances
 * through the same times, each on its own stream, their launches queued
 * before the call waits on any of them so that they overlap on the GPU.
 * outs[k] receives simulation k's n_times x samples records.  Each result
 * equals that simulation's asep_run alone.  The simulations must be distinct
 * and all at or before times[0]. */
int asep_run_batch(asep_sim* const* sims, uint32_t n_sims, const uint64_t* times,
                   uint32_t n_times, asep_rough* const* outs);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): a whole
 * run -- asep_create_ext on state_dev, asep_run through times[0..n_times),
 * asep_destroy -- that allocates nothing, host or device.
 *   state_dev: the samples x planes x L/64 state words (at least
 *     state_bytes >= that many bytes, asep_buffer_sizes' state size); the call
 *     initialises them from p and leaves the state at times[n_times-1] there.
 *   times: host array, ascending absolute MCS (n_times may be 0: only the
 *     initialisation runs).
 *   out_dev: device array of n_times x samples asep_rough (time-major), the
 *     same values asep_run returns (integers exact, w2 formed on the device
 *     from the exact numerator).
 * Everything else the run needs (quenched planes, hop counters, record
 * staging, the second state buffer of windowed plans) lives in one fixed
 * device workspace of ASEP_NOALLOC_SCRATCH_BYTES per GPU, held from the
 * first call on that GPU until the process ends; a run needing more returns
 * ASEP_E_TOO_LARGE.  All work is queued on hip_stream (NULL = the null
 * stream) and the call returns without waiting for it.  Calls on one GPU share
 * the workspace: calls whose work overlaps on the device (other streams or
 * threads, before the previous call's work has finished) race and give
 * undefined results; calls queued on one stream are ordered and safe. */
#define ASEP_NOALLOC_SCRATCH_BYTES (32u << 20)
int asep_run_noalloc(const asep_params* p, uint64_t* state_dev, size_t state_bytes,
                     void* hip_stream, const uint64_t* times, uint32_t n_times,
                     asep_rough* out_dev);

/* Sec. 2.1 (the ring's occupation numbers n_i): copy one sample's state words (planes x L/64 uint64, lane A first) to or
 * from host memory; n_words must equal planes x L/64.  Synchronises. */
int asep_read_state(asep_sim* s, uint32_t sample, uint64_t* words, uint64_t n_words);
int asep_write_state(asep_sim* s, uint32_t sample, const uint64_t* words, uint64_t n_words);

/* Sec. 2.3, Eq. (bimodal) slow sites; Sec. 3 turning points.
 * Quenched plane `plane` (ring: 0 = slow-p, 1 = slow-q; two lanes: 0 = turning
 * points) of one realisation, L/64 words.  ASEP_E_INVAL if the model has none. */
int asep_read_mask(asep_sim* s, uint32_t plane, uint32_t realization, uint64_t* words,
                   uint64_t n_words);

/* Sec. 3 (the current, c = J/L): cumulative hop counters J of all samples
 * (host array[samples]); synchronises. */
int asep_current(asep_sim* s, int64_t* hops);

/* Sec. 2.1 (time in MCS): set the MCS clock and hop counters, e.g. after
 * asep_write_state from a
 * checkpoint.  hops may be NULL (zeros). */
int asep_set_time(asep_sim* s, uint64_t t, const int64_t* hops);

/* Sec. 2.1 (flat start), Sec. 2.3 / 3 (quenched planes): re-run the
 * initialisation (state, quenched planes), set the clock and the
 * hop counters to zero; no allocation.  Asynchronous on the stream. */
int asep_reset(asep_sim* s);

/* Kernel timing of the sweep launches (HIP events on the simulation's
 * stream, taken only while enabled).  asep_profile_read synchronises and
 * returns the number of sweep launches, their summed duration in ms and the
 * elementary attempts they performed since enabling. */
typedef struct asep_profile_stats {
    uint64_t launches;
    double kernel_ms;
    uint64_t attempts;
} asep_profile_stats;
int asep_profile_enable(asep_sim* s, int enable);
int asep_profile_read(asep_sim* s, asep_profile_stats* out);

/* Sec. 2.1 (time in MCS): MCS completed so far (0 for a NULL handle). */
uint64_t asep_time(const asep_sim* s);

/* Free library-owned memory and the library-owned stream; borrowed buffers
 * and streams are left alone.  With a library-owned stream the call first
 * waits for the simulation's work; with a borrowed stream the caller must
 * have synchronised it (or an event after the last call) before freeing the
 * borrowed buffers.  NULL is ignored. */
void asep_destroy(asep_sim* s);

/* Sec. 2.1, Eq. W averaged over samples: ensemble mean of W^2 over n records
 * of one time: sum of the exact numerators
 * L S2 - S1^2 in 128-bit integers, one conversion, independent of order. */
int asep_ensemble_w2(const asep_rough* r, uint32_t n, uint64_t L, double* w2_mean);

/* Sec. 2.2, geometric sampling times of Eq. (sampling): 0, then ceil(t_i) for real
 * t_0 = t0, t_{i+1} = factor t_i while ceil(t_i) <= t_max, duplicates dropped.
 * Writes at most cap values; *n receives the count written. */
int asep_sample_times(double t0, double factor, uint64_t t_max, uint64_t* out, uint32_t cap,
                      uint32_t* n);

/* Static description of an error code, and the last HIP error seen by this
 * thread (empty string if none). */
const char* asep_strerror(int code);
const char* asep_last_device_error(void);

/* ---------------------------------------------------------------------------
 * Request loop with continuous batching (serving).  A request is an ensemble
 * run: parameters, ascending measurement times and t_max.  Requests are
 * admitted as device memory and ring slots free up, their rings advance
 * together in shared launches, and each request's results equal those of the
 * same request run alone, bit for bit.
 * ------------------------------------------------------------------------- */
typedef struct asep_server_cfg {
    uint32_t abi_version;
    int32_t device;            /* HIP device ordinal */
    uint64_t hbm_budget_bytes; /* device memory the server may hold for state */
    uint32_t max_queue;        /* pending requests before ASEP_E_BUSY */
    uint32_t max_active;       /* requests resident at once */
    uint64_t quantum_mcs;      /* MCS a resident request advances per round
                                  (0: 1000); a whole-ring request's quantum is
                                  further cut to one launch (2^30 sub-sweeps) */
    const char* tuning_path;   /* tuning table loaded at creation with
                                  asep_tuning_load; NULL: the process's table
                                  as it is */
    uint32_t reserved[4];
} asep_server_cfg;

typedef struct asep_request {
    asep_params params;
    uint64_t t_max;        /* final time (MCS) */
    const uint64_t* times; /* ascending measurement times <= t_max (copied) */
    uint32_t n_times;
} asep_request;

typedef struct asep_result {
    int32_t status;         /* ASEP_OK, ASEP_E_CANCELLED or an error code */
    uint32_t samples;
    uint32_t n_times;
    uint64_t* times;        /* [n_times] */
    asep_rough* rough;      /* [n_times * samples], time-major */
    uint64_t t_arrive_ns, t_admit_ns, t_start_ns, t_done_ns; /* CLOCK_MONOTONIC */
    uint64_t site_updates;  /* elementary attempts performed */
    asep_params params;     /* the request's parameters as resolved (the
                               schedule used: cell size, sub-sweeps, compared
                               bits); zero if it never became resident */
    asep_plan plan;         /* launch plan of its rings (zero likewise) */
    uint32_t quanta;        /* work segments it was advanced in */
    uint32_t packed_quanta; /* of those, the ones that shared a launch */
} asep_result;

typedef struct asep_server asep_server;

/* Tuning table: launch shapes and, optionally, the update schedule (cell
 * size, sub-sweeps per MCS) chosen by the autotuner per class of run.  Text,
 * one entry per line, '#' comments:
 *   model schedule disorder log2L_min log2L_max samples_min samples_max
 *   cell_log2 subsweeps windows window_sweeps rings_per_wg
 * (disorder: 1 if slow_frac > 0; L and samples ranges inclusive; a value 0
 * leaves that field to its default).  asep_create and asep_buffer_sizes fill
 * every parameter left at 0 from the first matching entry.  The table is
 * process-wide: loading replaces it, NULL or "" clears it.  ASEP_E_INVAL on a
 * malformed line (the table in use is then unchanged), ASEP_E_NOTFOUND if the
 * file cannot be read. */
int asep_tuning_load(const char* path);

int asep_server_create(const asep_server_cfg* cfg, asep_server** out);
void asep_server_destroy(asep_server* s);
/* Non-blocking; copies the request.  *ticket identifies it. */
int asep_submit(asep_server* s, const asep_request* req, uint64_t* ticket);
/* ASEP_E_PENDING until done; then fills *out (free with asep_result_free). */
int asep_poll(asep_server* s, uint64_t ticket, asep_result* out);
int asep_wait(asep_server* s, uint64_t ticket, uint64_t timeout_ns, asep_result* out);
int asep_cancel(asep_server* s, uint64_t ticket);
void asep_result_free(asep_result* r);

#ifdef __cplusplus
}
#endif

#endif /* ASEP_H */
