/*
 * ssa.h -- C ABI of libssa: many independent Gillespie direct-method trajectories of a
 * mass-action reaction network on one MI355X (gfx950), aligned on a time grid and reduced
 * across trajectories into per-grid-point mean and variance, with a likelihood-ratio
 * gradient and a batched many-network form.
 *
 * Paper: Aldinucci, Bracciali, Lio, Sorathiya, Torquati, "StochKit-FF: Efficient Systems
 * Biology on Multicore Architectures" (2010).
 *   - Section 2: the stochastic simulation of a CTMC by Gillespie's algorithm (one
 *     trajectory per realisation, exact exponential waiting times).
 *   - Section 3.2: a model is an integer state vector, an integer stoichiometric matrix,
 *     mass-action propensities and a simulated duration; StochRxn_ff runs copies of one
 *     simulation or parameter-swept simulations.
 *   - Section 3.2.1: "selective memory" aligns the trajectories' points by simulation time
 *     and reduces them online with associative, commutative functions (mean, variance).
 *
 * Arithmetic contract shared (as prose, not code) with the CPU oracle:
 *   propensity  a_j = c_j * h_j(x), h exact in 64-bit integers then rounded once:
 *               1 | x_A | x_A x_B | x_A (x_A - 1) / 2 for 2A
 *   sums        a model attribute (ssa_sum_order), a0 = S_{M-1}:
 *               SSA_SUM_SEQ      S_0 = a_0, S_j = S_{j-1} + a_j (left to right)
 *               SSA_SUM_BLOCK64  64 chunks of q = ceil(M/64) consecutive reactions; L_j the
 *                                left-to-right sum inside chunk l; chunk totals scanned
 *                                inclusively in steps d = 1, 2, ..., 32 (v_l += v_{l-d} for
 *                                l >= d, from the previous step's values); E_l = scanned
 *                                value of chunk l-1 (E_0 = 0); S_j = E_l + L_j
 *   random      Philox4x32-10, key = (seed lo, seed hi), counter = (k lo, k hi, i lo, i hi)
 *               for draw k (0-based) of trajectory i (0-based within its network)
 *   uniforms    r1 = (((o1<<32|o0) >> 11) + 1) 2^-53 in (0,1],  r2 = ((o3<<32|o2) >> 11) 2^-53
 *   time        tau = neglog(r1) / a0; neglog is the atanh-series -ln with fixed roundings
 *   selection   u = r2 * a0; smallest j with S_j > u, else the largest j with a_j > 0
 *   horizon     events with t_next > t_end are not applied; a0 == 0 is absorbing (no draw)
 *   alignment   right-continuous: x(t_g) includes every event with t_e <= t_g
 *   reduction   unbiased variance (divide by N - 1; 0 when N == 1)
 *
 * Conventions:
 *   - Every function returns an ssa_status; on failure ssa_last_error() (thread-local)
 *     describes it.  No C++ exception crosses this boundary.
 *   - The caller owns every buffer it passes.  The library owns model and batch handles,
 *     released by the matching *_destroy (NULL is accepted and ignored).
 *   - Host pointers ("host") are read or written synchronously.  Device pointers ("device")
 *     must be device memory on the current HIP device; *_device calls are asynchronous on
 *     the given hipStream_t (NULL = the null stream) unless stats is non-NULL, in which case
 *     the call waits for the stream and fills stats.
 *   - Layouts are row-major: [G*S] means index g*S + s.
 *   - Graph capture: ssa_run_device, ssa_run_device_static, ssa_backward_device,
 *     ssa_backward_moments_device, ssa_run_jacobian_device, ssa_run_cov_device,
 *     ssa_rates_from_log and ssa_jacobian_vjp may be called on a stream that is being
 *     captured into a HIP graph (hipStreamBeginCapture, torch.cuda.graph), and the graph
 *     replayed any number of times with the results of the same call made directly.  Under
 *     capture a call (1) takes no statistics (stats must be NULL, else SSA_E_INVALID);
 *     (2) compiles nothing: the network's specialised kernels of that launch size must exist
 *     from an earlier call on the device (else SSA_E_INVALID); (3) allocates its scratch with
 *     hipMalloc, this thread's capture mode relaxed for the call, and hands it to the model,
 *     which keeps it until ssa_model_destroy: replay graphs only while their model lives, and
 *     expect each capture to hold its scratch until then.  A refused call returns before its
 *     first stream operation, so the capture stays usable.  Replays of one graph on two
 *     streams at once share that scratch and race.
 *   - Environment variables (read at each call; none changes a result bit, only which
 *     kernel, launch form or buffer size computes it, except where stated):
 *       SSA_KERNEL=generic        the table-driven kernels instead of the specialised ones
 *       SSA_LAUNCH_FORM=two_wave|generations|refill   the specialised kernels' launch form
 *       SSA_DRAW_WAVE=0           no drawing-wave (two-wave) blocks for small launches
 *       SSA_DRAW_WAVE_BLOCKS=n    at most n two-wave blocks
 *       SSA_WIN_BYTES=n           LDS bytes of a selective-memory window (512 .. 16384)
 *       SSA_FWD_FLUSH=slab        windows flushed into wave-private slabs, not by atomics,
 *       SSA_SLAB_BYTES=n            when the slabs fit in n bytes (default 1 GiB)
 *       SSA_FWD_ORDER=0           forwards ignore recorded event counts (index order)
 *       SSA_WIDE_DEPG=0           many-reaction kernels re-evaluate every propensity
 *       SSA_JAC_BYTES=n           scratch budget of ssa_run_jacobian_device (default 4 GiB)
 *       SSA_SORT_BINS=n           bins of the adaptive memory's time order
 *       SSA_ADAPTIVE_RECORDS=n    event-log records per epoch of ssa_adaptive_device
 *       SSA_BATCH_GRAPH=0         ssa_batch_run launches directly instead of replaying a graph
 *       SSA_TUNE_FILE=path        autotuner choices kept in and read from a JSON file
 */
#ifndef SSA_H
#define SSA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SSA_OK = 0,
    SSA_E_INVALID = 1,      /* bad argument: sizes, coefficients, rates, grid, NULL pointer */
    SSA_E_NOMEM = 2,        /* device or host allocation failed */
    SSA_E_DEVICE = 3,       /* a HIP call failed (message in ssa_last_error) */
    SSA_E_OVERFLOW = 4,     /* a species count left the int32 range in some trajectory */
    SSA_E_EVENT_LIMIT = 5,  /* a trajectory reached max_events before t_end */
    SSA_E_UNSUPPORTED = 6   /* valid request outside what the library implements */
} ssa_status;

typedef struct ssa_model ssa_model;
typedef struct ssa_batch ssa_batch;

/* Order of the propensity sums (the paper leaves it open; results differ only in
 * rounding).  SEQ runs one trajectory per lane; BLOCK64 runs one trajectory per wave with
 * a wave-wide prefix scan, for networks with many reactions. */
typedef enum {
    SSA_SUM_SEQ = 0,
    SSA_SUM_BLOCK64 = 1
} ssa_sum_order;

/* Optional per-grid-point histogram of one species: bin = clamp((x - lo) div width, 0,
 * nbins - 1); counts are exact.  Output layout [G*nbins] uint32. */
typedef struct {
    int32_t species;
    int32_t lo;
    int32_t width;   /* > 0 */
    int32_t nbins;   /* 1..4096 */
} ssa_hist_spec;

/* How the simulation kernel of a call was launched (reported in ssa_stats.form).  Every
 * form gives the same bits; they differ in how lanes get their next trajectory. */
typedef enum {
    SSA_FORM_NONE = 0,
    SSA_FORM_TWO_WAVE = 1,     /* blocks of a simulating wave and a wave computing its draws,
                                  one generation of 64 trajectories at a time */
    SSA_FORM_GENERATIONS = 2,  /* persistent blocks; a wave takes its next 64 trajectories once
                                  all of its lanes are done */
    SSA_FORM_REFILL = 3,       /* persistent blocks; a lane takes the next trajectory as soon as
                                  its own ends */
    SSA_FORM_TABLE = 4,        /* the table-driven kernel (sequential order, any network) */
    SSA_FORM_WAVE = 5          /* one trajectory per wave (64-chunk order) */
} ssa_launch_form;

/* Filled when a non-NULL pointer is passed (the call then synchronises). */
typedef struct {
    uint64_t events;      /* events applied with t <= t_end, summed over trajectories */
    uint64_t max_steps;   /* largest per-trajectory event count */
    uint32_t flags;       /* bit 0: overflow seen, bit 1: event limit reached */
    float kernel_ms;      /* device time of the simulation kernel(s) */
    uint32_t form;        /* ssa_launch_form of the simulation kernel */
    uint32_t blocks;      /* its grid size in blocks */
    uint32_t ordered;     /* 1 when the trajectories ran longest first, in the order of the event
                             counts an earlier forward over the same trajectories recorded */
} ssa_stats;

/* Model (Section 3.2 model format).
 *   n_species S >= 1, n_reactions M >= 1 (M <= 4096, S <= 1024)
 *   reactants [M*S] host: coefficients >= 0, sum per reaction <= 2 (order <= 2)
 *   products  [M*S] host: coefficients >= 0 (e.g. 200), each <= 2^19 - 4
 *   rates     [M]   host: stochastic rate constants c_j, finite, >= 0
 *   x0        [S]   host: initial counts >= 0
 *   sum_order ssa_sum_order (either for any M up to 4096)
 * What runs where:
 *   SEQ, M <= 32 and S <= 64: kernels specialised to the network at first use (run-time
 *     compilation, cached per device), every entry point;
 *   SEQ otherwise: the table-driven kernel, which changes at most 4 species per reaction;
 *     record and backward need M <= 32 (SSA_E_UNSUPPORTED beyond);
 *   BLOCK64: one trajectory per wave, at most 4 changed species per reaction; up to 512
 *     reactions the chunk lives in registers, above that in LDS, where an event
 *     re-evaluates only the propensities that read a species it changed (a dependency
 *     graph built here; same results as re-evaluating all, which SSA_WIDE_DEPG=0 selects);
 *     not accepted by ssa_batch_create.
 * The arrays are copied (to the current device); the handle is immutable and may be shared
 * by threads that use the same device.  Errors: SSA_E_INVALID, SSA_E_UNSUPPORTED,
 * SSA_E_NOMEM, SSA_E_DEVICE. */
ssa_status ssa_model_create(int32_t n_species, int32_t n_reactions, const int32_t *reactants,
                            const int32_t *products, const double *rates, const int32_t *x0,
                            int32_t sum_order, ssa_model **out);

/* Rate law of one reaction (Section 2.1's infectivities beta_R5 = beta - K F with
 * 0 <= beta_R5 <= beta, beta_X4 = beta + K F, gamma likewise): with species >= 0 the rate
 * constant of reaction j is
 *     c_j(x) = min(max(c_j + slope * x_species, lo), hi)
 * (one product and one sum in binary64, then the bounds), c_j being the model's or the
 * run's rate; species < 0 keeps mass action.  lo >= 0, lo <= hi (hi may be +inf). */
typedef struct {
    int32_t species;
    double slope;
    double lo;
    double hi;
} ssa_rate_law;

/* ssa_model_create with optional rate laws (laws: host [M], NULL = mass action).  Networks
 * with a rate law run only in the specialised kernels: SSA_SUM_SEQ, M <= 32, S <= 64
 * (SSA_E_UNSUPPORTED otherwise); the gradient, the Jacobian and batches refuse them (the
 * score of a modulated rate is not n_j - A_j). */
ssa_status ssa_model_create_laws(int32_t n_species, int32_t n_reactions, const int32_t *reactants,
                                 const int32_t *products, const double *rates, const int32_t *x0,
                                 int32_t sum_order, const ssa_rate_law *laws, ssa_model **out);
/* Releases a model handle, its device copies and the scratch of every call captured into a
 * graph with it (NULL is ignored). */
void ssa_model_destroy(ssa_model *model);

/* Host convenience (synchronous).  Section 2: n_traj independent Gillespie trajectories
 * 0..n_traj-1 of the model on [0, t_end]; Section 3.2.1: their states aligned on the time
 * grid and reduced across trajectories; Section 4: mean and variance at every grid point.
 *   grid [n_grid] host: non-decreasing, inside [0, t_end] (checked: SSA_E_INVALID)
 *   mean, var [G*S] host outputs (caller-owned); stats may be NULL.
 * Errors: SSA_E_INVALID, SSA_E_NOMEM, SSA_E_DEVICE, SSA_E_OVERFLOW, SSA_E_EVENT_LIMIT
 * (outputs undefined on error). */
ssa_status ssa_run(const ssa_model *model, int64_t n_traj, double t_end, const double *grid,
                   int32_t n_grid, uint64_t seed, double *mean, double *var, ssa_stats *stats);

/* Rate constants from log rate constants (the parameters theta_j = ln c_j of the gradient
 * below; Section 4's sensitivity analysis varies such parameters): rates[j] = e^theta_j for
 * j < n, both device arrays, asynchronous on stream, with fixed roundings the CPU oracle
 * reproduces bit for bit:
 *   theta < -708 (also -inf): 0;   theta > 709 or NaN: NaN (an invalid rate);
 *   else k = rint(fl(theta * INV_LN2)) (ties to even, INV_LN2 = 0x1.71547652b82fep0),
 *   r = fma(-k, LN2_LO, fma(-k, LN2_HI, theta)) (LN2_HI = 0x1.62e42fee00000p-1,
 *   LN2_LO = 0x1.a39ef35793c76p-33), p = E_13 then p = fma(p, r, E_n) for n = 12 .. 0 with
 *   E_n = fl(1/n!), and the result p * 2^k (exact).  Within 2 ulp of e^theta. */
ssa_status ssa_rates_from_log(const double *log_rates, int32_t n, double *rates, void *stream);

/* Device form of ssa_run (Sections 2, 3.2.1 and 4 as above), with an optional histogram
 * of one species at every grid point (a further recombining function, Section 5).
 *   rates [M] device: rate constants for this run (NULL = the model's), or
 *   log_rates [M] device: theta_j = ln c_j, turned into c_j by ssa_rates_from_log's formula
 *     on the device (NULL = none); at most one of the two.
 *   grid [G] device; mean, var [G*S] device outputs; hist + d_hist [G*nbins] device (both
 *   NULL for none).  max_events: per-trajectory cap (0 = 2^62).
 * Device inputs are checked on the device: a grid that is not non-decreasing inside
 * [0, t_end] (NaN included) or a log rate that is NaN or above 709 refuses the run -- no
 * trajectory is simulated, mean and var are NaN and the histogram counts 0xffffffff -- and
 * the call returns SSA_E_INVALID when stats is given.  Asynchronous on stream when stats is
 * NULL: a refusal, an overflow or an event-limit condition is then not reported by the
 * status, so pass stats when the inputs or the model may fail.
 * A run of the specialised kernels (sequential order, M <= 32, S <= 64, n_traj <= 2^27) also
 * records each trajectory's event count into a device buffer of the model (4 bytes per
 * trajectory, grown as needed, released by ssa_model_destroy), for ssa_backward_device.
 * When the record is that of a run with the same n_traj, t_end, seed and max_events (the
 * rates may differ: a fit's previous step), a forward in generations takes its trajectories
 * longest first by it (stats->ordered); the sums are exact integers, so the order changes
 * the time, never a bit of the outputs.
 * Errors: SSA_E_INVALID, SSA_E_NOMEM, SSA_E_DEVICE, SSA_E_OVERFLOW, SSA_E_EVENT_LIMIT,
 * SSA_E_UNSUPPORTED. */
ssa_status ssa_run_device(const ssa_model *model, const double *rates, const double *log_rates,
                          int64_t n_traj, double t_end, const double *grid, int32_t n_grid,
                          uint64_t seed, uint64_t max_events, double *mean, double *var,
                          const ssa_hist_spec *hist, uint32_t *d_hist, void *stream, ssa_stats *stats);

/* ssa_run_device for callers that cannot allocate device memory (code being captured into
 * a HIP graph, tight serving loops, hosts that forbid allocation during a run): the same
 * arguments, results and device-side checks, but every piece of scratch (the grid-point
 * sums, the histogram differences, the status words, rates formed from log_rates) comes
 * from one static device area of 8 MiB that the library holds on each GPU it runs on until
 * the process ends, and the call makes no allocation of its own.  Limits:
 *   about 24 G S + 4 G nbins bytes (256-byte pieces), plus 16 bytes per reaction when
 *   rates or log_rates are given (8 per dependency-list entry for a 64-chunk network above
 *   512 reactions), must fit in the 8 MiB (the large workload, 10^4 points x 4 species
 *   with a 64-bin histogram, takes 3.5 MiB); larger calls get SSA_E_INVALID before anything
 *   runs;
 *   the network's specialised kernels are used only if this device has them compiled
 *   already (by an earlier ssa_run_device call); otherwise the table-driven kernel runs,
 *   with the same results (a network with rate laws then gets SSA_E_UNSUPPORTED);
 *   stats->kernel_ms is 0 (no timing events).
 * Calls on one GPU share its area and find the last call's contents (the call clears what
 * must start at zero): two calls that overlap in time on one GPU, on different streams or
 * threads, race and give undefined results. */
ssa_status ssa_run_device_static(const ssa_model *model, const double *rates, const double *log_rates,
                                 int64_t n_traj, double t_end, const double *grid, int32_t n_grid,
                                 uint64_t seed, uint64_t max_events, double *mean, double *var,
                                 const ssa_hist_spec *hist, uint32_t *d_hist, void *stream, ssa_stats *stats);

/* A run taken in epochs of simulation time, for horizons too long for one launch (Section
 * 4's HIV runs cover 4000 simulated days, about 1.5e8 events per trajectory): the same
 * trajectories, alignment and reduction as ssa_run_device, with the same results bit for
 * bit, but the caller advances the run to successive times and may act (report progress,
 * stop) in between.  Each advance simulates every trajectory up to its last event at or
 * before t_until and saves its state; the next one resumes from there with the draw the
 * trajectory did not use.  The specialised kernels only (sequential order, M <= 32, S <= 64;
 * SSA_E_UNSUPPORTED otherwise).
 *   ssa_run_begin: grid [n_grid] host (checked as in ssa_run), rates [M] host or NULL (the
 *     model's), hist as in ssa_run_device or NULL.  The handle owns its device memory
 *     (about 2 x (4 S + 24) bytes per trajectory plus the grid sums).
 *   ssa_run_advance: up to min(t_until, t_end) (a time at or before the last one does
 *     nothing); synchronous; stats (may be NULL) receive this advance's events (those
 *     applied in it), largest step count so far, flags and kernel time.  Errors as
 *     ssa_run_device; a run past 2^39 events gets SSA_E_UNSUPPORTED.
 *   ssa_run_finish: after the run reached t_end, mean, var [G*S] and d_hist [G*nbins] (iff
 *     the run has a histogram) device outputs; stats receive the run's totals.
 *     SSA_E_INVALID before t_end.
 *   ssa_run_destroy: releases the handle (NULL is ignored). */
typedef struct ssa_run_state ssa_run_state;
ssa_status ssa_run_begin(const ssa_model *model, const double *rates, int64_t n_traj, double t_end,
                         const double *grid, int32_t n_grid, uint64_t seed, uint64_t max_events,
                         const ssa_hist_spec *hist, ssa_run_state **out);
ssa_status ssa_run_advance(ssa_run_state *run, double t_until, void *stream, ssa_stats *stats);
ssa_status ssa_run_finish(ssa_run_state *run, double *mean, double *var, uint32_t *d_hist, void *stream,
                          ssa_stats *stats);
void ssa_run_destroy(ssa_run_state *run);

/* Likelihood-ratio gradient of a loss L(mean) with respect to theta_j = ln c_j (the local
 * form of Section 4's sensitivity analysis of the mean trajectories), by re-simulating the
 * same trajectories (same seed, same Philox counters):
 *   grad_j = sum_{g,s} w_{g,s} (1/N) sum_i (X^i_s(t_g) - mhat_{g,s}) (n^i_j(t_g) - A^i_j(t_g))
 * with n_j the firing count and A_j the integrated propensity.  All pointers device:
 * rates or log_rates [M] as in ssa_run_device (the forward's), grid [G], w [G*S]
 * (dL/dmean), mhat [G*S] (centring, usually the forward mean), grad [M] output.  The
 * per-trajectory sums are reduced in a fixed pairwise order, so the result is
 * deterministic.  Device inputs are checked as in ssa_run_device (a refused run gives a
 * NaN gradient and, with stats, SSA_E_INVALID).  When the model's last ssa_run_device call
 * was the same run (same n_traj, t_end, seed, max_events, n_grid and the same grid, rates
 * and log_rates pointers) and recorded event counts, the trajectories are taken longest
 * first (stats->ordered); the order changes the time, never a bit of grad, so arrays whose
 * contents changed since only lose the speed-up.  Same status codes as ssa_run_device
 * (SSA_E_UNSUPPORTED for a SEQ model with more than 32 reactions or with rate laws). */
ssa_status ssa_backward_device(const ssa_model *model, const double *rates, const double *log_rates,
                               int64_t n_traj, double t_end, const double *grid, int32_t n_grid,
                               uint64_t seed, uint64_t max_events, const double *w, const double *mhat,
                               double *grad, void *stream, ssa_stats *stats);

/* The same gradient for a loss on the grid means and variances (Section 4 reduces runs to
 * average and variance): with wv [G*S] = dL/dvar and the centring vhat [G*S] (usually the
 * forward variance; both device) every crossing adds
 *   wv_{g,s} ((X_s(t_g) - mhat_{g,s})^2 - vhat_{g,s}) z_j(t_g)
 * to the mean term, the score-function derivative of the variance (d E[(X - mu)^2] / d theta
 * = E[(X - mu)^2 z] since E[X - mu] = 0; E[z] = 0 makes the centring unbiased).  The weights
 * are folded into prefix tables of w - 2 wv mhat, wv and their constants, evaluated as a
 * polynomial in x per interval, so the rounding error scales with wv (x^2 + mhat^2 + |vhat|)
 * rather than with the centred square.  wv == NULL gives ssa_backward_device.  Arguments,
 * limits and codes as ssa_backward_device. */
ssa_status ssa_backward_moments_device(const ssa_model *model, const double *rates, const double *log_rates,
                                       int64_t n_traj, double t_end, const double *grid, int32_t n_grid,
                                       uint64_t seed, uint64_t max_events, const double *w, const double *mhat,
                                       const double *wv, const double *vhat, double *grad, void *stream,
                                       ssa_stats *stats);

/* Autotuning of the forward launch (the forward of ssa_run_device, Sections 2 and 3.2.1;
 * the search itself is no step of the paper's method) for this model and problem size: every candidate
 * configuration is timed on the caller's problem (grid [n_grid] device, the same outputs for
 * all: results never depend on the configuration) by the device time of everything the call
 * launches (fills, slabs and their reduction included), the best of two calls after a
 * warm-up, each in index order as a run's first forward: first the LDS window bytes 2048 .. 16384
 * with the windows flushed by atomics or through wave-private slabs, then, with the best
 * window, the launch form of the specialised kernels (two-wave blocks or generations) and
 * its block count (the default and smaller grids).  The fastest is remembered for (device
 * architecture, kernel kind, network, G and N rounded up to powers of two) and used by
 * later ssa_run_device / ssa_run calls in this process, and written to the JSON file named
 * by SSA_TUNE_FILE when set (read back at the first lookup of a later process).  result may
 * be NULL.  Synchronous.  win_bytes 0 / slab -1 / form 0 / blocks 0 denote the built-in
 * choices (form by launch size, grid at the occupancy limit). */
typedef struct {
    int32_t win_bytes;
    int32_t slab;
    float best_ms;      /* device time of a call with the chosen configuration */
    float default_ms;   /* device time of a call with the built-in choices */
    int32_t form;       /* ssa_launch_form chosen (0: by launch size) */
    int32_t blocks;     /* grid size chosen (0: the default) */
} ssa_tune_result;

ssa_status ssa_autotune_forward(const ssa_model *model, const double *rates, int64_t n_traj, double t_end,
                                const double *grid, int32_t n_grid, uint64_t seed, void *stream,
                                ssa_tune_result *result);

/* Autotuning of the backward launch (the re-simulation of ssa_backward_device, the
 * gradient of Section 4's sensitivity; no step of the paper's method itself): the launch
 * forms of the specialised kernels (two-wave blocks, generations, refilled lanes) at their
 * default grids and at smaller ones are timed on the caller's problem with unit weights
 * (results never depend on the choice), after one forward of the same run (so that the
 * backward takes the order of the lengths it records, as after a forward in use), by the
 * device time of everything a call launches, and the fastest is remembered per (architecture,
 * kernel kind, network, G and N rounded up to powers of two) for later ssa_backward_device
 * / ssa_backward_moments_device calls, and in SSA_TUNE_FILE.  Other kernels keep their
 * single form.  result may be NULL (win_bytes 0, slab -1).  Synchronous. */
ssa_status ssa_autotune_backward(const ssa_model *model, const double *rates, int64_t n_traj, double t_end,
                                 const double *grid, int32_t n_grid, uint64_t seed, void *stream,
                                 ssa_tune_result *result);

/* Forward pass that also returns the likelihood-ratio Jacobian of the grid means with
 * respect to theta_j = ln c_j (every local sensitivity of Section 4's mean trajectories),
 * from the same single simulation pass:
 *   jac[g][s][j] = (1/N) sum_i (X^i_s(t_g) - mean_{g,s}) (n^i_j(t_g) - A^i_j(t_g))
 * (the estimator of ssa_backward_device before it is contracted with w, centred on this
 * run's own mean).  Arguments as ssa_run_device (rates or log_rates, no histogram); jac [G*S*M] device.  The
 * item sums are reduced in a fixed order, so the Jacobian is deterministic.  Needs a
 * SSA_SUM_SEQ model with M <= 32 and S <= 64 and ceil(N/64) * G * (S+1) * M * 8 bytes of
 * scratch (at most 4 GiB, or SSA_JAC_BYTES); SSA_E_UNSUPPORTED otherwise (use
 * ssa_backward_device). */
ssa_status ssa_run_jacobian_device(const ssa_model *model, const double *rates, const double *log_rates,
                                   int64_t n_traj, double t_end, const double *grid, int32_t n_grid,
                                   uint64_t seed, uint64_t max_events, double *mean, double *var, double *jac,
                                   void *stream, ssa_stats *stats);

/* Forward pass returning the species covariance matrix at every grid point (a further
 * recombining function over the time-aligned states, Sections 3.2.1 and 5): cov [G*S*S] device,
 *   cov[g][s][r] = (N sum X_s X_r - sum X_s sum X_r) / (N (N - 1))   (0 when N == 1)
 * from exact integer sums, rounded once, so cov[g][s][s] is the variance of ssa_run_device;
 * mean [G*S] device.  Arguments as ssa_run_device (no histogram).  Needs a SSA_SUM_SEQ
 * model with M <= 32 and S <= 64 (SSA_E_UNSUPPORTED otherwise). */
ssa_status ssa_run_cov_device(const ssa_model *model, const double *rates, int64_t n_traj, double t_end,
                              const double *grid, int32_t n_grid, uint64_t seed, uint64_t max_events, double *mean,
                              double *cov, void *stream, ssa_stats *stats);

/* Adaptive selective memory (Section 3.2.1, Figure 3): the time alignment without a caller
 * grid.
 *   Avg-Y: the points are time 0 and every distinct time at which some trajectory applies an
 *     event (t <= t_end); at each point every trajectory contributes its state after its
 *     own events up to that time (sample and hold).  Mean and variance per species from
 *     exact integer sums, rounded once (the formulas of ssa_run_device).
 *   Avg-XY: consecutive groups of k Avg-Y points (the last may be shorter, k' points) each
 *     give one point: time = (t_1 + ... + t_k') / k', and likewise the means and the
 *     variances (sums left to right in binary64, one division).
 * Every applied event is logged (time, species, change, previous count), the log is sorted
 * by time on the device, and the moments are prefix sums over the distinct times.
 * Arguments: rates [M] device or NULL; k >= 1; outputs device: xy_time [xy_cap],
 * xy_mean / xy_var [xy_cap*S]; optional Avg-Y y_time [y_cap], y_mean / y_var [y_cap*S]
 * (NULL to skip).  n_points (host, [2]) receives U (Avg-Y points) and P = ceil(U / k).
 * With xy_time and y_time both NULL the call only sizes (the simulation still runs).
 * Capacities below U / P give SSA_E_INVALID with n_points filled.  Scratch: about
 * 40 bytes per logged species change plus 40 S bytes per Avg-Y point.  Synchronises the
 * stream.  Needs at most 4 changed species per reaction and, in the sequential order,
 * M <= 32 (SSA_E_UNSUPPORTED otherwise); n_traj <= 2^30. */
ssa_status ssa_adaptive_device(const ssa_model *model, const double *rates, int64_t n_traj, double t_end,
                               uint64_t seed, uint64_t max_events, int64_t k, double *xy_time, double *xy_mean,
                               double *xy_var, int64_t xy_cap, double *y_time, double *y_mean, double *y_var,
                               int64_t y_cap, int64_t *n_points, void *stream, ssa_stats *stats);

/* Quantiles per grid point (one of the more informative recombining functions Section 5
 * asks for) from a histogram of ssa_run_device (spec as used there):
 * for each q in qs (0 < q <= 1) the rank k = max(1, ceil(q N)) in binary64 and the result
 * is lo + b width for the first bin b whose cumulative count reaches k (with width 1 and
 * no clamping in the top bin, the k-th smallest count).  hist [G*nbins], qs [nq], out
 * [G*nq] int32, all device; asynchronous on stream. */
ssa_status ssa_hist_quantiles(const uint32_t *hist, int32_t n_grid, const ssa_hist_spec *spec, int64_t n_traj,
                              const double *qs, int32_t nq, int32_t *out, void *stream);

/* grad[j] = sum_{g,s} w[g][s] jac[g][s][j] on the device (fixed summation order; Section 4's
 * sensitivity of the means, contracted with a loss gradient): the
 * vector-Jacobian product that turns the forward Jacobian into d loss / d ln c for
 * w = d loss / d mean.  jac [G*S*M], w [G*S], grad [M], all device; asynchronous on stream. */
ssa_status ssa_jacobian_vjp(const double *jac, const double *w, int32_t n_grid, int32_t n_species,
                            int32_t n_reactions, double *grad, void *stream);

/* Per-trajectory record (Section 2: one trajectory, one realisation of the CTMC; Section
 * 3.2's workers can write whole trajectories out) of trajectories traj_begin .. traj_begin+count-1 (synchronous, all
 * pointers host): states [count*G*S] int32 at the grid points, events [count], draws
 * [count] (Philox blocks consumed), t_last [count] (time of the last applied event, 0 if
 * none), n_fired [count*M] and a_int [count*M] (integral of a_j over [0, t_end]) may be
 * NULL.  rates [M] host or NULL.  For the parity tests against the CPU oracle. */
ssa_status ssa_record(const ssa_model *model, const double *rates, int64_t traj_begin, int64_t count,
                      double t_end, const double *grid, int32_t n_grid, uint64_t seed, uint64_t max_events,
                      int32_t *states, uint64_t *events, uint64_t *draws, double *t_last,
                      int64_t *n_fired, double *a_int);

/* Batched form (Section 3.2, parameter-swept simulations in one call): n_models networks,
 * each with its own trajectory count, horizon, grid (host [n_grid[b]]) and seed; trajectory
 * i of network b uses the same counters as ssa_run on that network alone, so the results
 * equal the per-network runs bit for bit.  All networks run in one persistent
 * work-stealing launch of the table-driven kernel (SEQ models with at most 4 changed
 * species per reaction).  The handle owns the device copies of the grids and its scratch
 * memory. */
ssa_status ssa_batch_create(int32_t n_models, const ssa_model *const *models, const int64_t *n_traj,
                            const double *t_end, const double *const *grids, const int32_t *n_grid,
                            const uint64_t *seeds, ssa_batch **out);
/* One run of a batch (Section 3.2's parameter-swept simulations, reduced per network as in
 * Sections 3.2.1 and 4): means[b], vars[b]: device pointers [G_b * S_b] (caller-owned);
 * the launch sequence is captured as a hipGraph at the first call and replayed after.
 * Asynchronous unless stats != NULL.  Errors: SSA_E_INVALID, SSA_E_DEVICE, SSA_E_OVERFLOW,
 * SSA_E_EVENT_LIMIT. */
ssa_status ssa_batch_run(ssa_batch *batch, double *const *means, double *const *vars, void *stream,
                         ssa_stats *stats);
void ssa_batch_destroy(ssa_batch *batch);

/* Autotuning of a batch (the launch of ssa_batch_run; no step of the paper's method): times the batched launch with each LDS window size (the
 * built-in default, 2048 .. 16384 bytes; sizes that do not fit the LDS are skipped; results
 * never depend on the choice) and keeps the fastest for this handle's later runs (the
 * captured graph is rebuilt).  The trial runs write scratch outputs, not the caller's.
 * result may be NULL (slab is always -1).  Synchronous. */
ssa_status ssa_batch_autotune(ssa_batch *batch, void *stream, ssa_tune_result *result);

/* Thread-local description of the last failure on this thread ("" if none). */
const char *ssa_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SSA_H */
