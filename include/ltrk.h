/*
 * ltrk.h - C ABI of the MI355X longitudinal macro-particle tracker.
 *
 * The method (Oeftiger 2014, "Parallelisation of PyHEADTAIL", section 1.1.2):
 * each macro-particle's longitudinal coordinates (z, delta) are integrated
 * turn by turn through the RF bucket, independently per particle, by an
 * Euler-Cromer, leap-frog (Verlet) or fourth-order Ruth / Runge-Kutta scheme.
 * Particles are independent and turns are sequential (section 2.3). The map
 * of one step of weight w (one turn = weight 1) is the single-harmonic
 * stationary bucket:
 *
 *   drift:  z     <- z - w * eta * C * delta,      eta = 1/gamma_t^2 - 1/gamma^2
 *   kick:   delta <- delta + w * (q V / (beta p0 c)) * sin(2 pi h z / C)
 *
 * After every turn the library can reduce the bunch to its population moments
 * (mean and rms of z and delta, rms emittance), accumulated in FP64.
 *
 * Conventions for every entry point:
 *   - Arrays named z, dp, z_comp, dp_comp, moments are DEVICE pointers owned
 *     by the caller; the library never frees them. Arrays are contiguous
 *     structure-of-arrays, one element per particle. A pointer that is not
 *     device memory, or whose device allocation (the hipMalloc block it lies
 *     in; for sub-allocating allocators such as PyTorch's caching allocator,
 *     that block is the allocator's segment) ends before the stated length,
 *     is rejected with LTRK_EINVAL before anything is enqueued.
 *   - `stream` is a hipStream_t (NULL = the null stream). Calls are
 *     asynchronous: they return after enqueueing; device faults surface at the
 *     caller's next synchronisation.
 *   - Return 0 (LTRK_OK) or a negative code below; ltrk_last_error() gives a
 *     thread-local message for the last failure. No C++ exception crosses
 *     the ABI.
 *   - n = 0 or turns = 0 is a successful no-op, except that with n = 0 and
 *     turns > 0 the moment rows (if requested) are filled with NaN.
 *   - A caller may capture a call into a graph of its own (stream capture):
 *     the call then enqueues its kernels into the capture instead of
 *     replaying a cached graph. Run the same call once on that stream before
 *     capturing, so that its scratch exists and the captured call allocates
 *     nothing: a captured call that would need more moment-partial scratch
 *     than its stream has returns EUNSUPPORTED before enqueueing anything.
 *     When an uncaptured call grows a stream's scratch, the old buffer stays
 *     allocated until ltrk_shutdown, so graphs captured before stay valid.
 *     The programme, wake and batched entry points refuse capture
 *     (EUNSUPPORTED: they upload tables).
 */
#ifndef LTRK_H
#define LTRK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LTRK_ABI_VERSION 1

/* Return codes. */
#define LTRK_OK 0
#define LTRK_EINVAL (-1)      /* invalid argument (sizes, pointers, ring, enums) */
#define LTRK_ENOMEM (-2)      /* device or host allocation failed */
#define LTRK_EDEVICE (-3)     /* a HIP runtime error; message holds hipGetErrorString */
#define LTRK_EAGAIN (-4)      /* engine: no free slot or not enough budget right now */
#define LTRK_EUNSUPPORTED (-5)

/* Integration schemes (section 1.1.2). One scheme step per turn. */
#define LTRK_EULER_CROMER 0   /* first order: drift(1), kick(1) */
#define LTRK_LEAPFROG 1       /* second order: drift(1/2), kick(1), drift(1/2) */
#define LTRK_RUTH4 2          /* fourth-order Forest-Ruth composition, 3 kicks */
#define LTRK_RK4 3            /* classical Runge-Kutta, 4 force evaluations */

/* State precisions. */
#define LTRK_F64 0            /* z, dp in FP64 */
#define LTRK_F32C 1           /* z, dp as FP32 hi plus FP32 Kahan compensation;
                                 value = hi - comp. RF phase reduction and moments
                                 in FP64; the sine of the reduced phase in FP32
                                 (kick relative error <= 1.7e-7; RK4: FP64 sine) */

/* Ring and beam parameters: circumference [m], harmonic number (integer
 * valued, > 0), RF voltage [V], reference momentum p0 c [eV], rest energy
 * m c^2 [eV] (>= 0), transition gamma (> 0), particle charge [e]. The sign of
 * the voltage selects the stable phase: V > 0 is stable at z = 0 above
 * transition (eta > 0); below transition pass a negated voltage. */
typedef struct ltrk_ring {
    double circumference_m;
    double harmonic;
    double voltage_V;
    double p0c_eV;
    double mass_eV;
    double gamma_t;
    double charge_e;
} ltrk_ring;

/* One moments row (40 bytes): population statistics (1/n) of the bunch.
 * emit_rms = sqrt(max(0, rms_z^2 rms_dp^2 - cov(z,dp)^2)) in metres. */
typedef struct ltrk_moments {
    double mean_z;
    double rms_z;
    double mean_dp;
    double rms_dp;
    double emit_rms;
} ltrk_moments;

/* Derived constants of a ring, FP64. kick_amplitude A = q V / (beta p0 c);
 * wavenumber k = 2 pi h / C [1/m]; slip_length D = eta C [m];
 * omega_s = sqrt(A k D) [rad/turn] and q_s = omega_s / 2 pi (smooth motion);
 * q_leapfrog solves cos(2 pi Q) = 1 - omega_s^2 / 2 (linearised leap-frog
 * map); bucket_half_length = C / (2h); bucket_height = 2 sqrt(A / (k D));
 * h_separatrix = -2 A / k for H = -(D/2) dp^2 + (A/k)(cos kz - 1).
 * omega_s, q_s, q_leapfrog, bucket_height are NaN when A k D <= 0 (no
 * stable bucket at z = 0). */
typedef struct ltrk_derived {
    double gamma;
    double beta;
    double eta;
    double kick_amplitude;
    double wavenumber;
    double slip_length;
    double omega_s;
    double q_s;
    double q_leapfrog;
    double bucket_half_length;
    double bucket_height;
    double h_separatrix;
} ltrk_derived;

/* Host-only derivation of the ring constants above. EINVAL for a
 * non-finite parameter, C <= 0, harmonic <= 0 or not integer valued,
 * p0c <= 0, mass < 0 or gamma_t <= 0. */
int ltrk_derive(const ltrk_ring* ring, ltrk_derived* out);

/* Track n particles for `turns` turns in place (FP64 state).
 * z, dp: device arrays of n doubles, updated in place.
 * moments: device array of `turns` rows or NULL; row t receives the moments
 *   after turn t+1 (turn-0 moments: ltrk_moments_f64). The sums behind them
 *   are taken about a centre fixed for the call (the mean of an evenly
 *   strided sample of up to 1024 particles of the initial state where it
 *   lies more than 4 sample rms from zero, else zero), so a bunch far from
 *   the origin keeps its accuracy; a centroid that moves by A rms away from
 *   that centre during the call loses about (A^2) ulp of the variance.
 * integrator: LTRK_EULER_CROMER .. LTRK_RK4.
 * Any finite z is valid (no aperture, no wrapping): the RF phase 2hz/C is
 * reduced to [-1/2, 1/2] exactly, from the unrounded product while every
 * particle of a 64 x ppl tile stays below 2^50 C/(2h) in magnitude for the
 * launch, else from its FP64 rounding; a non-finite z gives NaN momenta. */
int ltrk_track_f64(double* z, double* dp, int64_t n, int64_t turns, const ltrk_ring* ring,
                   int integrator, ltrk_moments* moments, void* stream);

/* For callers that cannot allocate (code under graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): ltrk_track_f64 with the same
 * arguments, plan and results (bit for bit), whose moment partials live in a
 * fixed array of LTRK_NOALLOC_SCRATCH_BYTES on each device, held from the
 * first such call on that device (which looks up the array's address) until
 * the process ends. It allocates no device or host memory, builds no graph and
 * is not timed by ltrk_timing_enable; its launches go directly onto `stream`
 * in chunks of turns whose partials fit the array. EINVAL, before anything is
 * enqueued, for arguments ltrk_track_f64 rejects and when moments are
 * requested for a bunch whose partials of one turn exceed the array (beyond
 * about 8.5e8 particles at 8 per lane, 1.7e9 at 16). All calls on one device share its array: calls that
 * overlap on that device (other streams or threads) race and give wrong
 * moments; the array's contents between calls are unspecified (every row a
 * call reads is written by that call first). */
#define LTRK_NOALLOC_SCRATCH_BYTES (64u << 20)
int ltrk_track_f64_noalloc(double* z, double* dp, int64_t n, int64_t turns,
                           const ltrk_ring* ring, int integrator, ltrk_moments* moments,
                           void* stream);

/* Same with the FP32 + Kahan-compensation state (LTRK_F32C). The four arrays
 * of n floats are all state: z = z_hi - z_comp, dp = dp_hi - dp_comp. Start
 * from comp = fl32(hi - value) (or zero); keep them between calls. */
int ltrk_track_f32c(float* z, float* dp, float* z_comp, float* dp_comp, int64_t n,
                    int64_t turns, const ltrk_ring* ring, int integrator,
                    ltrk_moments* moments, void* stream);

/* Extended RF and slippage: a second RF harmonic, RF phase offsets and a slip
 * factor expanded in delta. The paper's hollow-bunch study (section 2.2,
 * profile) applies two RF kicks and re-evaluates eta and the RF phase every
 * step; this is the stationary form of that map:
 *   drift:  z     <- z - w * C * (eta0 + eta1 delta + eta2 delta^2) * delta
 *   kick:   delta <- delta + w * sum_i (q V_i / (beta p0 c)) sin(2 pi h_i z / C + phi_i)
 * with eta0 = 1/gamma_t^2 - 1/gamma^2 from `ring`, i = 1 from `ring`
 * (harmonic, voltage_V) and i = 2 from the fields below (voltage2_V = 0: no
 * second harmonic). phi_i in radians; harmonic2 integer valued and > 0 when
 * voltage2_V != 0; eta1, eta2 dimensionless and finite. */
typedef struct ltrk_rf2 {
    ltrk_ring ring;
    double phi1_rad;
    double harmonic2;
    double voltage2_V;
    double phi2_rad;
    double eta1;
    double eta2;
} ltrk_rf2;

/* As ltrk_track_f64 (FP64 state, same arrays, moments and stream rules) for
 * the extended map. EINVAL for an invalid ring or extension field. */
int ltrk_track_rf2_f64(double* z, double* dp, int64_t n, int64_t turns, const ltrk_rf2* rf,
                       int integrator, ltrk_moments* moments, void* stream);

/* One turn of an RF programme: the RF settings of that turn and the reference
 * momentum after it. The paper's hollow-bunch run changes the machine
 * settings while it tracks (section 2.2); this is the per-turn form. */
typedef struct ltrk_rf_turn {
    double voltage_V;   /* V1 during the turn */
    double phi1_rad;    /* phase of harmonic 1 */
    double voltage2_V;  /* V2 during the turn (0: no second harmonic) */
    double phi2_rad;    /* phase of harmonic 2 */
    double p0c_eV;      /* reference momentum after the turn, > 0 */
} ltrk_rf_turn;

/* The extended map with per-turn settings (FP64 state; arrays, moments and
 * stream rules as ltrk_track_f64). `rf` gives what stays fixed: the ring
 * (its p0c_eV is the reference momentum before the first turn; its voltage_V
 * and rf's phi1_rad, voltage2_V, phi2_rad are not used), harmonic2, eta1,
 * eta2. `program`: host array of `turns` entries, entry t for turn t, read
 * before the call returns.
 * Turn t runs the reference from p_a (the previous entry's p0c_eV, or the
 * ring's) to p_b (entry t's). The RF gives a particle the energy
 * E_t(z) = q sum_i V_i sin(2 pi h_i z / C + phi_i), a momentum E_t(z) / beta_a
 * with beta_a the reference beta at p_a. A kick of weight w (the scheme's
 * kick weights sum to one) carries the share w of that gain and of the
 * reference step: with the reference moving p -> p' = p + w (p_b - p_a),
 *   delta <- (p / p') delta + (p - p') / p' + w E_t(z) / (beta_a p').
 * A drift uses eta0 at the reference momentum current at that point of the
 * turn. With a constant momentum and constant settings this is
 * ltrk_track_rf2_f64. EINVAL for an invalid ring, extension field or
 * programme entry (non-finite, p0c_eV <= 0, voltage2_V != 0 without a valid
 * harmonic2); EUNSUPPORTED for RK4 with a changing momentum and for a stream
 * that is being captured into a graph (the programme is uploaded by a copy
 * that a graph would replay from reused host memory). */
int ltrk_track_program_f64(double* z, double* dp, int64_t n, int64_t turns,
                           const ltrk_rf2* rf, const ltrk_rf_turn* program, int integrator,
                           ltrk_moments* moments, void* stream);

/* Twiss parameters and tunes of the two transverse planes at the
 * observation point (section 1.1.1: one linear transfer matrix per turn). */
typedef struct ltrk_twiss {
    double q_x;      /* tune (its integer part does not matter) */
    double qp_x;     /* chromaticity: tune shift per unit delta */
    double alpha_x;
    double beta_x;   /* metres, > 0 */
    double q_y;
    double qp_y;
    double alpha_y;
    double beta_y;
} ltrk_twiss;

/* Track n particles with a 6-D FP64 state (device arrays of n doubles each,
 * updated in place; x, y in metres, xp, yp in radians) for `turns` turns.
 * One turn: per plane u the Twiss rotation by phi = 2 pi (Q + Q' delta) with
 * the turn's starting delta,
 *   u  <- (cos phi + alpha sin phi) u + beta sin phi u'
 *   u' <- -gamma sin phi u + (cos phi - alpha sin phi) u',  gamma = (1 + alpha^2) / beta,
 * then one step of the extended longitudinal map (as ltrk_track_rf2_f64).
 * moments: device array of 3 * turns rows or NULL; rows 3t, 3t + 1, 3t + 2
 * hold the moments of (z, dp), (x, xp), (y, yp) after turn t + 1 (means,
 * rms and rms emittance of each pair). EINVAL for an invalid ring, extension
 * or Twiss field (non-finite, beta <= 0). */
int ltrk_track_6d_f64(double* z, double* dp, double* x, double* xp, double* y, double* yp,
                      int64_t n, int64_t turns, const ltrk_rf2* rf, const ltrk_twiss* twiss,
                      int integrator, ltrk_moments* moments, void* stream);

/* Longitudinal wake: the impedance effects the paper's conclusion (section 3)
 * names as the memory-bound next step. */
#define LTRK_WAKE_RESONATOR 0 /* W(tau) = 2 a R e^{-a tau} (cos w' tau - (a/w') sin w' tau),
                                 a = w_r / (2 Q), w' = sqrt(w_r^2 - a^2); W(0) = a R */
#define LTRK_WAKE_CONSTANT 1  /* W(tau > 0) = R (V/C), W(0) = R/2: the potential is the
                                 charge ahead */
#define LTRK_WAKE_MAX_SLICES 4096

typedef struct ltrk_wake {
    int32_t model;        /* LTRK_WAKE_RESONATOR or LTRK_WAKE_CONSTANT */
    int32_t n_slices;     /* 1 .. LTRK_WAKE_MAX_SLICES */
    double shunt;         /* resonator: shunt impedance R (ohm); constant: R (V/C) */
    double freq_hz;       /* resonator: f_r = w_r / 2 pi, > 0 */
    double quality;       /* resonator: Q > 1/2 */
    double intensity;     /* particles in the bunch (each macro-particle carries
                             q e intensity / n), >= 0 */
    double z_lo;          /* sliced range [z_lo, z_hi) in metres, z toward the head */
    double z_hi;
} ltrk_wake;

/* The extended map (as ltrk_track_rf2_f64) with a wake kick after every
 * step: the bunch is cut into n_slices equal slices over [z_lo, z_hi)
 * (particles outside are neither counted nor kicked; the slice coordinate of
 * z is u = (z - z_lo) * (n_slices / (z_hi - z_lo)), each operation rounded
 * once, and slice k holds u in [k, k + 1)), the potential at slice
 * centre k is V_k = Q_mp sum_{j >= k} count_j W((j - k) dz / (beta c)) with
 * Q_mp = q e intensity / n, and a particle at z gets
 *   delta <- delta - q V(z) / (beta p0 c),
 * V(z) interpolated linearly between slice centres (constant beyond the first
 * and last centre). Row t of `moments` holds the moments after turn t's kick.
 * Same arrays and stream rules as ltrk_track_f64. EINVAL for an invalid ring,
 * extension or wake field; EUNSUPPORTED for a stream being captured into a
 * graph (the wake table is uploaded by a copy from reused host memory). */
int ltrk_track_wake_f64(double* z, double* dp, int64_t n, int64_t turns, const ltrk_rf2* rf,
                        const ltrk_wake* wake, int integrator, ltrk_moments* moments,
                        void* stream);

/* Moments of the current state (one row) into the device row `out`. */
int ltrk_moments_f64(const double* z, const double* dp, int64_t n, ltrk_moments* out,
                     void* stream);
int ltrk_moments_f32c(const float* z, const float* dp, const float* z_comp,
                      const float* dp_comp, int64_t n, ltrk_moments* out, void* stream);

/* One bunch of a batched call: its own arrays (z_comp/dp_comp only for
 * LTRK_F32C, else ignored), size, ring (own V and h) and moment rows
 * (device, `turns` rows, or NULL). */
typedef struct ltrk_bunch {
    void* z;
    void* dp;
    void* z_comp;
    void* dp_comp;
    int64_t n;
    ltrk_ring ring;
    ltrk_moments* moments;
} ltrk_bunch;

/* Advance nb bunches of uneven size by `turns` turns with one scheme and one
 * state precision: each launch sweeps a tile table covering every bunch, so
 * all bunches move together. `bunches` is a HOST array of nb descriptors;
 * the arrays it names are device memory. Results per bunch are those of
 * ltrk_track_f64/f32c on that bunch with the same plan. EUNSUPPORTED, before
 * anything is enqueued, for a stream that is being captured into a graph (the
 * bunch and tile tables are uploaded per call). */
int ltrk_track_batched(const ltrk_bunch* bunches, int nb, int64_t turns, int integrator,
                       int dtype, void* stream);

/* Launch plan. turns_per_launch K: turns fused per kernel launch (1 = one
 * launch per turn, the unfused form); block: threads per block (64, 128 or
 * 256); ppl: particles per lane (1, 2, 4, 8 or 16; extended-map and wake
 * calls take 4 or 8, the nearest of the two, with the same results as at that
 * value); use_graph: replay the launch
 * sequence from a cached hipGraph (streams other than NULL only). A call of
 * more launches than the environment variable LTRK_MAX_GRAPH_LAUNCHES (read
 * at every call; default 32768, at least 16) is never captured: its launches
 * are enqueued as they are generated, in pieces of that length, with the same
 * results. The moment partials of one call take at most LTRK_SCRATCH_MB MiB
 * (read at every call; default 192, at least 16); longer runs are finalized
 * in chunks of turns, with the same results. */
typedef struct ltrk_plan {
    int32_t turns_per_launch;
    int32_t block;
    int32_t ppl;
    int32_t use_graph;
} ltrk_plan;

/* Force one plan for all following calls of this process (NULL: back to
 * automatic plans from the tuning cache or the built-in default). EINVAL for
 * values outside the ranges above. Forced and tuned plans are used as given;
 * the built-in default (1024 turns per launch; 8 particles per lane from
 * ~1e5 particles, 16 for FP64 calls and F32C Euler-Cromer and leap-frog
 * calls where the waves then fill the device's wave slots in fewer rounds,
 * e.g. from 6e6 particles in all) is
 * lowered, for calls that compute moments, to the largest power of two (at
 * least 64) whose moment partials of one launch stay within 192 MiB, e.g.
 * 512 turns at 1e7 particles (16 per lane). */
int ltrk_set_plan(const ltrk_plan* plan);

/* The plan a call with these parameters would use now (particles per lane
 * as the call takes them for this dtype; turns per launch before the limit
 * for calls that compute moments). */
int ltrk_get_plan(int integrator, int dtype, int64_t n, ltrk_plan* out);

/* Time candidate plans on scratch particles of size n (on `stream`,
 * synchronising it): every combination of 32, 128, 256, 512, 1024 and 2048
 * turns per launch, 64, 128 and 256 threads per block and 1, 2, 4, 8 and 16
 * particles per lane, with moments. Cache the fastest
 * for single-bunch calls
 * of (device, integrator, dtype, floor(log2 n)). `best` (host, may be NULL)
 * receives it. */
int ltrk_autotune(int integrator, int dtype, int64_t n, void* stream, ltrk_plan* best);

/* The plan a batched call over bunches of total_n particles would use now. */
int ltrk_get_plan_batched(int integrator, int dtype, int64_t total_n, ltrk_plan* out);

/* Tune the batched launch (the paper's sweep of turns per kernel call,
 * section 2.3) for a bunch table like `bunches` (HOST array of nb
 * descriptors; only each bunch's n, ring and whether it has moments are read,
 * its arrays are not touched): probe bunches of those sizes and rings are
 * tracked on `stream` (synchronised) with every combination of 128, 256, 512
 * and 1024 turns per launch, 64, 128 and 256 threads per block and 2, 4, 8
 * and 16 particles per lane, and the fastest plan is cached for
 * batched calls of
 * (device, integrator, dtype, floor(log2 of the total particles)). Needs
 * device memory for the probes' state and 4096 moment rows per bunch with
 * moments. `best` (host, may be NULL) receives the plan. */
int ltrk_autotune_batched(const ltrk_bunch* bunches, int nb, int integrator, int dtype,
                          void* stream, ltrk_plan* best);

/* Save / load the tuning cache as text, one entry per line: arch integrator
 * dtype log2(n) batched K block ppl graph. Loading merges the file's valid
 * entries into the cache and skips lines that do not parse; EINVAL if the
 * file cannot be opened. */
int ltrk_tune_cache_save(const char* path);
int ltrk_tune_cache_load(const char* path);

/* Per-launch timing with HIP events. While enabled, every tracking and
 * finalize launch is timed by events on its stream: eager launches are
 * bracketed by an event pair; a plan with use_graph replays a timed graph
 * (cached apart from the untimed one) with event-record nodes between its
 * segments of consecutive tracking or finalize launches, fresh events at
 * every replay: a segment's time covers its launches and the short gaps
 * between them, and the graph keeps its own launch cadence. A call with
 * moments counts two kinds of moment launches as finalize launches: the one
 * that fixes the centre of its moment sums before its first turn, and the
 * finalize after every chunk of turns. ltrk_timing_take synchronises the
 * recorded events, returns the totals and clears them. */
typedef struct ltrk_timing {
    int64_t track_launches;
    double track_ms;
    int64_t finalize_launches;
    double finalize_ms;
} ltrk_timing;

int ltrk_timing_enable(int on);
int ltrk_timing_take(ltrk_timing* out);

/* ---- Serving engine: continuous batching of tracking jobs ----
 * The engine owns a device arena of `hbm_budget_bytes` for job state and
 * moment rows, and `max_slots` job slots. A job is admitted when a slot is
 * free and its footprint fits in the arena; its state then stays on the device
 * until it is retired. Each ltrk_engine_step is one launch over a tile table
 * of every active job (mixed schemes and precisions, 8 particles per lane,
 * heaviest schemes first) advancing each by min(k, turns left, what the
 * moment-partial scratch holds), plus one moments finalize launch; the step's
 * tables are uploaded on a copy stream of the engine. The partial scratch is
 * 1 GiB beside the arena (LTRK_ENGINE_PARTIALS_MB sets another size in MiB).
 * Jobs admitted between steps join the next step. Results equal those of
 * ltrk_track_f64/f32c on the same job with 8 particles per lane. Not
 * thread-safe: one host thread drives an engine. */
typedef struct ltrk_engine ltrk_engine;

/* A job. z0/dp0 (and z0_comp/dp0_comp for LTRK_F32C) are HOST arrays of the
 * initial state in the job's precision (double for F64, float for F32C),
 * copied at admission. */
typedef struct ltrk_job {
    int64_t n;
    int64_t turns;
    ltrk_ring ring;
    int32_t integrator;
    int32_t dtype;
    const void* z0;
    const void* dp0;
    const void* z0_comp;
    const void* dp0_comp;
} ltrk_job;

typedef struct ltrk_engine_stats {
    int32_t active_slots;
    int32_t max_slots;
    int64_t arena_bytes;
    int64_t arena_free_bytes;
    int64_t largest_free_block;
    int64_t steps;
    int64_t particle_turns;
} ltrk_engine_stats;

int ltrk_engine_create(int device, int64_t hbm_budget_bytes, int max_slots, ltrk_engine** out);
/* Bytes of arena a job needs: state (16 B per particle) + moment rows (40 B
 * per turn), each rounded up to 256 B, + 256 B for the centre of its moment
 * sums. */
int ltrk_engine_footprint(const ltrk_job* job, int64_t* bytes);
/* Admit a job: LTRK_EAGAIN if no slot is free, the arena has no block large
 * enough now, or the running jobs and this one would need more moment-partial
 * columns (one per 512 particles) than the partial scratch holds; EINVAL if
 * the job can never fit (arena or partial scratch alone) or is malformed. */
int ltrk_engine_admit(ltrk_engine* e, const ltrk_job* job, int* slot);
/* Advance every active job by up to k turns (1 <= k <= 4096). `stream` NULL
 * uses the engine's own stream; otherwise the step is ordered after prior
 * work on `stream` and `stream` waits for it. *advanced (may be NULL)
 * receives the particle-turns enqueued. */
int ltrk_engine_step(ltrk_engine* e, int k, void* stream, int64_t* advanced);
/* done = 1 when all of the job's turns have been computed on the device. */
int ltrk_engine_poll(ltrk_engine* e, int slot, int* done);
/* Copy a finished job's final state and moment rows to HOST buffers (any may
 * be NULL; comp arrays only for F32C), blocking until they are there. */
int ltrk_engine_result(ltrk_engine* e, int slot, void* z, void* dp, void* z_comp,
                       void* dp_comp, ltrk_moments* moments);
/* Free a slot and its arena block (finished or not). */
int ltrk_engine_retire(ltrk_engine* e, int slot);
/* Stop a job: it takes no further turns; its slot stays until retired. */
int ltrk_engine_cancel(ltrk_engine* e, int slot);
int ltrk_engine_stats_get(ltrk_engine* e, ltrk_engine_stats* out);
int ltrk_engine_destroy(ltrk_engine* e);

/* Errors and lifetime. */
const char* ltrk_strerror(int code);
/* Copy the calling thread's last error message into buf (NUL terminated);
 * returns the code of that error (0 if none). */
int ltrk_last_error(char* buf, size_t len);
/* Release per-device scratch, cached graphs and streams of this process. */
int ltrk_shutdown(void);
int ltrk_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LTRK_H */
