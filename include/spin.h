/*
 * spin.h -- C ABI of the MI355X random-phase ensemble spin-dynamics library.
 *
 * The method (Alvarez, Danieli, Levstein & Pastawski, "Quantum parallelism
 * as a tool for ensemble spin dynamics calculations", arXiv:0710.3747):
 * instead of evolving each of the 2^(M-1) members of the infinite-
 * temperature ensemble with site n up (Eq. (1)), evolve ONE pure state, the
 * superposition of all members with random phases (section "Ensemble vs.
 * pure entangled state", Eq. (2); the entangled state of section "Testing
 * the quantum parallelism"), under a Trotter-Suzuki product of two-spin
 * propagators, and read the local polarisation P(t) = 2 <psi(t)| I^z_n' |psi(t)>
 * after every step.
 *
 * Conventions shared by every entry point:
 *  - Sites are 0-based (the paper's site 1 is site 0).
 *  - State layout: a contiguous vector of 2^M complex amplitudes in device
 *    memory, interleaved (re, im); complex64 (float2) for SPIN_C64,
 *    complex128 (double2) for SPIN_C128.  Basis index x: bit s of x is site
 *    s; bit value 0 = spin up (I^z = +1/2).  This layout holds at every
 *    return; internal relabelling, if any, is undone before a call returns.
 *  - Couplings: spin_coupling {i, j, a, b} is the two-spin term of the
 *    section "Spin systems with different coupling networks":
 *        H_ij = a I^z_i I^z_j + (b/2)(I^+_i I^-_j + I^-_i I^+_j),  hbar = 1.
 *    a = 0 is the XY family, b = 0 Ising, a = b isotropic, a = -2b dipolar.
 *  - One Trotter step (the paper names the Trotter-Suzuki decomposition but
 *    fixes no scheme; this library takes the symmetric Strang split):
 *        exp(-i dt/2 H_0) ... exp(-i dt/2 H_{K-1}) exp(-i dt/2 H_{K-1}) ... exp(-i dt/2 H_0)
 *    applied right-to-left, i.e. the couplings in list order, then in reverse
 *    order.  Each factor is the exact two-spin propagator.  The library may
 *    reorder factors with disjoint sites and merge adjacent factors on the
 *    same pair (exact identities); the product is unchanged up to rounding.
 *  - Observable: P[k] = sum_x (1 - 2 bit_n'(x)) |psi_x|^2 and
 *    N[k] = sum_x |psi_x|^2 after k steps, both accumulated in FP64 whatever
 *    the state precision; P is not divided by N.
 *  - Ownership: the caller owns every device buffer (state, P, N); host
 *    arrays (couplings, problem lists) are read during the call only.  The
 *    library owns only its plan caches and workspaces (released by
 *    spin_release_caches).  It never frees or reallocates caller memory.
 *  - Streams: `stream` is a hipStream_t (NULL = the null stream).  Work is
 *    enqueued and the call returns without synchronising; outputs are valid
 *    once the stream has reached that point.  Argument errors are detected
 *    on the host and returned before anything is enqueued.
 *  - Errors: every call returns a spin_status; on failure a message is kept
 *    in thread-local storage (spin_last_error).  No C++ exception crosses
 *    this boundary.  Calls are thread-safe; calls that overlap on the same
 *    state buffer race.
 */
#ifndef SPIN_H_
#define SPIN_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SPIN_OK = 0,
    SPIN_EINVAL = -1,        /* bad argument (range, null pointer, non-finite value) */
    SPIN_ENOMEM = -2,        /* workspace allocation failed */
    SPIN_EHIP = -3,          /* HIP runtime error (message in spin_last_error) */
    SPIN_EUNSUPPORTED = -4,  /* valid request the library cannot serve */
    SPIN_ENOTFOUND = -5      /* no autotuned entry for these arguments */
} spin_status;

typedef enum { SPIN_C64 = 1, SPIN_C128 = 2 } spin_prec;

#define SPIN_MAX_M_C64 34
#define SPIN_MAX_M_C128 33

typedef struct {
    int32_t i, j;   /* distinct sites, 0 <= i, j < M */
    double a, b;    /* I^z I^z and flip-flop strengths (finite) */
} spin_coupling;

/*
 * spin_init_random_phase -- write the random-phase state.
 * Section "Ensemble vs. pure entangled state" (alpha_i = sqrt(p_i) e^{i phi_i},
 * p_i = 1/2^(M-1), the infinite-temperature weights of section "Spin
 * systems with different coupling networks") and the entangled state of
 * section "Testing the quantum parallelism":
 *   psi[x] = exp(+i phi_r) / sqrt(2^(M-1))  if bit `polarized_site` of x is 0,
 *   psi[x] = 0                               otherwise,
 * with r = x with bit `polarized_site` deleted, phi_r = 2 pi u(seed, r), and
 * u(seed, r) = (z >> 11) 2^-53 where z is output r+1 of the SplitMix64
 * stream started at state `seed` (Steele, Lea & Flood, OOPSLA 2014).
 *   psi  : device buffer of 2^M amplitudes of `prec` (overwritten).
 *   M    : 1..SPIN_MAX_M_C64 (c64) or 1..SPIN_MAX_M_C128 (c128).
 * Errors: SPIN_EINVAL for a null psi, bad prec, M or site out of range.
 */
int spin_init_random_phase(void *psi, int32_t prec, int32_t M, int32_t polarized_site,
                           uint64_t seed, void *stream);

/*
 * spin_init_product -- writes the product (unentangled) initial state of the
 * section "Testing the quantum parallelism": site `polarized_site` up and
 * every other site l in (|down> + exp(-i phi_l)|up>)/sqrt(2), i.e.
 *   psi[x] = exp(-i sum_{l != n, bit l of x = 0} phi_l) / sqrt(2^(M-1))
 *            if bit n of x is 0, else 0,
 * with only M-1 independent phases phi_l = 2 pi u(seed, l) (u as above, at
 * counter l).  Averages over N_alpha such draws approach the ensemble only
 * for N_alpha (M-1) ~ 2^(M-1) (Fig. 3(a) discussion).
 * Arguments, layout and errors as spin_init_random_phase.
 */
int spin_init_product(void *psi, int32_t prec, int32_t M, int32_t polarized_site,
                      uint64_t seed, void *stream);

/*
 * spin_trotter_evolve -- n_steps symmetric Trotter steps in place, with the
 * observable after every step.  Trotter-Suzuki route of the introduction and
 * summary (wave functions of size 2^M); observable of Eq. (2) with
 * P = 2(W_11 - 1/2) (section "Testing the quantum parallelism").
 *   psi      : device state, 2^M amplitudes of `prec` (in/out).
 *   J, K     : host array of K >= 0 couplings (copied during the call).
 *   dt       : time step (finite; negative runs time backwards).
 *   n_steps  : >= 0.
 *   observed_site : n', 0 <= n' < M.
 *   P_dev    : device FP64 array of n_steps+1 entries; P_dev[0] is the value
 *              at entry, P_dev[k] after k steps.  Required.
 *   N_dev    : device FP64 array of n_steps+1 entries for the norm, or NULL.
 * Errors: SPIN_EINVAL (null psi/P_dev, M, sites, i == j, non-finite a/b/dt,
 * K < 0, n_steps < 0), SPIN_ENOMEM, SPIN_EHIP.
 */
int spin_trotter_evolve(void *psi, int32_t prec, int32_t M, const spin_coupling *J,
                        int32_t K, double dt, int64_t n_steps, int32_t observed_site,
                        double *P_dev, double *N_dev, void *stream);

/* Execution options for spin_trotter_evolve_ex (zero-initialise = defaults). */
typedef struct {
    int32_t schedule;     /* 0 = fused tiles (default); 1 = one full pass per factor
                             (the plain, unfused schedule, kept as a cross-check) */
    int32_t tile_bits;    /* k of the 2^k-amplitude tiles; 0 = default (14 for
                             complex64, 13 for complex128; complex128 also takes 14,
                             with half tiles and one workgroup per CU) */
    int32_t reg_bits;     /* amplitudes per lane = 2^reg_bits; 0 = default */
    int32_t coalesce_bits;/* low address bits every tile keeps; 0 = default (4) */
    int32_t engine;       /* 0 = VALU butterflies (default); 1 = each register stage's
                             factors as one dense 32 x 32 complex matrix on FP32 MFMA
                             (complex64, tile_bits 14, reg_bits 5; tiled path only:
                             states held by one workgroup ignore it) */
    int32_t no_merge;     /* 1 = do not merge adjacent same-pair factors */
    int32_t use_graph;    /* 1 = tiled path: the call's launch sequence is captured
                             into a hipGraph once per (plan, state, P, N, workspace)
                             and replayed on a library stream ordered after `stream`
                             (for calls that repeat); ignored by states held by one
                             workgroup and by the unfused schedule */
    int32_t exchange;     /* tiled path, stage exchanges through LDS: 0 = default (half
                             tiles where the shape has such a kernel, else whole tiles);
                             1 = whole tiles (one workgroup per CU, the next tile
                             prefetched into registers); 2 = half tiles (one tile
                             position stays in registers in every stage, the tile moves
                             through LDS in two halves, two workgroups share a CU, one
                             for complex128 tiles of 2^14) */
    int32_t reserved[8];
} spin_options;

/* As spin_trotter_evolve with explicit options (NULL = defaults). */
int spin_trotter_evolve_ex(void *psi, int32_t prec, int32_t M, const spin_coupling *J,
                           int32_t K, double dt, int64_t n_steps, int32_t observed_site,
                           double *P_dev, double *N_dev, const spin_options *opt,
                           void *stream);

/*
 * spin_trotter_evolve_noalloc -- spin_trotter_evolve_ex for callers that
 * cannot allocate device memory: code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation.  Same arguments, results and
 * stream semantics; it calls no device allocation.
 *  - The plan for these arguments must already be cached on the current
 *    device (spin_prepare_plan with the same prec, M, J, K, dt, n_steps,
 *    observed_site and options); otherwise SPIN_EUNSUPPORTED, nothing
 *    enqueued.
 *  - The per-workgroup partial sums of the observable live in a fixed
 *    device array of SPIN_NOALLOC_SCRATCH_BYTES per GPU, held by the library
 *    until the process ends and shared by every such call on that GPU: calls
 *    that overlap on one GPU (other streams, other threads) race.  The array
 *    needs no clearing between calls; a call that needs more step slots than
 *    it holds for its workgroups gets SPIN_EUNSUPPORTED.
 *  - use_graph is refused (SPIN_EUNSUPPORTED); the unfused schedule
 *    (schedule = 1) is served.
 */
#define SPIN_NOALLOC_SCRATCH_BYTES (1u << 20)
int spin_trotter_evolve_noalloc(void *psi, int32_t prec, int32_t M, const spin_coupling *J,
                                int32_t K, double dt, int64_t n_steps, int32_t observed_site,
                                double *P_dev, double *N_dev, const spin_options *opt,
                                void *stream);

/*
 * observed_site value that selects the all-site profile's plan in
 * spin_prepare_plan, spin_describe_plan and spin_plan_trace.
 */
#define SPIN_ALL_SITES (-1)

/*
 * spin_trotter_evolve_profile -- as spin_trotter_evolve_ex, but the local
 * polarisation of Eq. (2) is read at EVERY site n' = 0..M-1 after every step
 * (the polarisation profile of the chain, not one site), in the same launches
 * that apply the propagators.
 *   Pall_dev : device FP64 array of (n_steps+1) * M entries, row-major:
 *              Pall_dev[k*M + n'] = sum_x (1 - 2 bit_n'(x)) |psi_x|^2 after k
 *              steps.  Required.
 *   N_dev    : device FP64 array of n_steps+1 entries for the norm, or NULL.
 *   opt      : as spin_trotter_evolve_ex; the matrix engine (engine = 1) is
 *              refused with SPIN_EUNSUPPORTED.
 * The factor order, merging and final state are those of spin_trotter_evolve_ex;
 * the tiled plan differs only in where the M observables of each step are
 * taken (spin_plan_trace with observed_site = SPIN_ALL_SITES lists them).
 * Errors as spin_trotter_evolve_ex.
 */
int spin_trotter_evolve_profile(void *psi, int32_t prec, int32_t M, const spin_coupling *J,
                                int32_t K, double dt, int64_t n_steps, double *Pall_dev,
                                double *N_dev, const spin_options *opt, void *stream);

/*
 * spin_local_polarization -- P = sum_x (1 - 2 bit_site(x)) |psi_x|^2, FP64,
 * of the state as it is (Eq. (2), P = 2(W - 1/2); not divided by the norm).
 *   psi   : device state, 2^M amplitudes of `prec` (read only).
 *   site  : 0 <= site < M.
 *   P_dev : device FP64 array of 1 entry, receives P.
 * Errors: SPIN_EINVAL (null psi/P_dev, prec, M, site), SPIN_ENOMEM, SPIN_EHIP.
 */
int spin_local_polarization(const void *psi, int32_t prec, int32_t M, int32_t site,
                            double *P_dev, void *stream);

/*
 * spin_local_polarization_ex -- as spin_local_polarization, and the norm
 * N = sum_x |psi_x|^2 (FP64) into N_dev[0] when N_dev is not NULL.
 */
int spin_local_polarization_ex(const void *psi, int32_t prec, int32_t M, int32_t site,
                               double *P_dev, double *N_dev, void *stream);

/*
 * Batched evolution of independent problems of uneven size (disorder
 * realisations, independent phase draws whose mean is Eq. (4), or the
 * 2^(M-1) basis-state members of the ensemble average of Eq. (1)), in ONE
 * persistent launch.  Every problem uses the same prec, dt and n_steps.
 */
typedef struct {
    void *psi;               /* device state of this problem, 2^M amplitudes */
    int32_t M, K;            /* size and number of couplings */
    int64_t coupling_offset; /* index of its first coupling in J_all */
    int32_t polarized_site;  /* used with SPIN_INIT_RANDOM_PHASE and SPIN_INIT_PRODUCT */
    int32_t observed_site;
    uint64_t seed;           /* phase seed (SPIN_INIT_RANDOM_PHASE, SPIN_INIT_PRODUCT) or basis
                                index (SPIN_INIT_BASIS) */
    double *P_dev;           /* n_steps+1 FP64 entries (required) */
    double *N_dev;           /* n_steps+1 FP64 entries or NULL */
} spin_problem;

/* Initial state written inside the batched launch. */
enum {
    SPIN_INIT_NONE = 0,          /* evolve the states as given */
    SPIN_INIT_RANDOM_PHASE = 1,  /* as spin_init_random_phase(polarized_site, seed) */
    SPIN_INIT_BASIS = 2,         /* the basis state |seed> (0 <= seed < 2^M): one member
                                    |Psi_i> of the ensemble of Eq. (1) */
    SPIN_INIT_PRODUCT = 3        /* as spin_init_product(polarized_site, seed) */
};

/*
 * spin_trotter_evolve_batch -- for every problem, optionally write its
 * initial state (`init`, one of SPIN_INIT_*), then evolve it n_steps steps
 * (as spin_trotter_evolve) writing its P and N.
 *   probs, n       : host array of n >= 0 problems (read during the call).
 *   J_all, K_total : host array holding every problem's couplings; K_total
 *                    bounds each problem's [coupling_offset, +K) range.
 *   init           : SPIN_INIT_* (one initial state for every problem).
 * The states must not overlap.  The work is enqueued on `stream` and the
 * call returns without synchronising (the first call with a new problem set
 * plans and uploads its tables synchronously; later equal calls reuse them
 * until spin_release_caches).  Problems larger than one workgroup's tile run
 * as gangs of workgroups that meet at bounded device-wide barriers; if a
 * barrier times out, the problem's P is set to NaN and spin_batch_status
 * reports it.  Errors as spin_trotter_evolve (plus SPIN_EINVAL for a bad
 * init or a basis index >= 2^M), reported for the first offending problem.
 */
int spin_trotter_evolve_batch(const spin_problem *probs, int32_t n, const spin_coupling *J_all,
                              int64_t K_total, int32_t prec, double dt, int64_t n_steps,
                              int32_t init, void *stream);

/*
 * spin_batch_status -- synchronises `stream`, then reports whether any
 * batched launch on the current device that has completed timed out at a
 * gang barrier since the previous query (SPIN_EHIP with a message) or not
 * (SPIN_OK), and clears that status.
 */
int spin_batch_status(void *stream);

/*
 * spin_ensemble_evolve -- the ensemble average of Eq. (1) taken literally
 * (section "Ensemble vs. pure entangled state"), the computation the
 * random-phase state replaces: at infinite temperature with site
 * `polarized_site` up, the ensemble is the 2^(M-1) Zeeman basis states |x>
 * whose bit `polarized_site` is 0 (bit value 0 is spin up), each of weight
 * 1/2^(M-1).  Every member is evolved on its own (n_steps Strang steps, as
 * spin_trotter_evolve) and, for every step k, the mean over the members of
 * their local polarization P = 2(W - 1/2) at `observed_site` is written to
 * P_dev[k] (FP64).  Over the whole ensemble this is P^ens(t_k).
 *   members : member r (0 <= r < 2^(M-1)) is the basis state whose bits on
 *             the sites other than polarized_site are the bits of r, in
 *             site order; the call averages members first_member ..
 *             first_member + n_members - 1 (n_members >= 1; the whole
 *             ensemble is 0, 2^(M-1)).
 *   work, work_amplitudes : the caller's device buffer of work_amplitudes
 *             amplitudes of `prec` (16-byte aligned, contents overwritten).
 *             2^c members are evolved at once as one state of M + c sites
 *             whose top c (uncoupled) sites hold the member index, with 2^c
 *             the largest power of two that fits the buffer
 *             (2^(M+c) <= work_amplitudes), does not exceed n_members
 *             rounded up to a power of two, and keeps M + c within
 *             SPIN_MAX_M_*; a buffer of 2^M amplitudes evolves one member at
 *             a time.  Unused member slots of the last evolution hold zeros.
 *   P_dev   : n_steps + 1 doubles (device), (1/n_members) sum_r P_r[k].
 *   N_dev   : n_steps + 1 doubles (device), the mean norm, or NULL.
 *   opt     : launch options of the (M + c)-site evolutions, as
 *             spin_trotter_evolve_ex; may be NULL.
 * The member sums are taken on the device in a fixed order (within one
 * evolution by the fused observable's reduction, then evolutions in member
 * order, then the division by n_members), so equal calls give equal bits.
 * The work is enqueued on `stream` and the call returns without
 * synchronising (the first call for new arguments plans synchronously).
 * Errors: SPIN_EINVAL (prec, M, sites, member range, a null or misaligned
 * work buffer, work_amplitudes < 2^M, null P_dev, couplings, dt, n_steps),
 * SPIN_ENOMEM, SPIN_EHIP, SPIN_EUNSUPPORTED as spin_trotter_evolve_ex.
 */
int spin_ensemble_evolve(int32_t prec, int32_t M, const spin_coupling *J, int32_t K, double dt,
                         int64_t n_steps, int32_t polarized_site, int32_t observed_site,
                         int64_t first_member, int64_t n_members, void *work,
                         int64_t work_amplitudes, double *P_dev, double *N_dev,
                         const spin_options *opt, void *stream);

/*
 * spin_prepare_plan -- plans the call spin_trotter_evolve_ex would make with
 * the same arguments (prec, M, J, K, dt, n_steps, observed_site, opt) and
 * uploads the plan tables to the current device, where they stay cached
 * until spin_release_caches.  A later evolve call with equal arguments then
 * does no host planning and no table upload.  No state is touched; the
 * upload is synchronous.  observed_site = SPIN_ALL_SITES prepares the plan
 * of spin_trotter_evolve_profile.  Errors as spin_trotter_evolve_ex (argument
 * checks), SPIN_ENOMEM if the tables cannot be allocated.
 */
int spin_prepare_plan(int32_t prec, int32_t M, const spin_coupling *J, int32_t K, double dt,
                      int64_t n_steps, int32_t observed_site, const spin_options *opt);

/*
 * Autotuner (for callers that run the same problem many times, e.g. long or
 * repeated evolutions).  spin_autotune times trial evolutions of
 * `trial_steps` steps for a set of launch shapes of the tiled path (tile
 * bits, register bits, lanes, coalescing bits; VALU butterflies -- the MFMA
 * matrix engine is selectable through spin_options only) and keeps the
 * fastest:
 *   - key: device architecture and CU count, prec, M, observed_site, dt and
 *     the coupling list (order and values);
 *   - the trials run on a scratch state the call allocates (2^M amplitudes)
 *     and frees; no caller buffer is touched;
 *   - the call enqueues on `stream` and synchronises it before returning;
 *   - best: the chosen options (other fields zero), may be NULL;
 *   - results, cap, n_results: per-candidate outcomes (host array of cap
 *     records, may be NULL with cap = 0; *n_results = number of candidates);
 *   - cache_path: if not NULL, a JSON file that receives the choice (created,
 *     or updated keeping other entries; written atomically by rename).
 * States small enough for one workgroup have a single shape (one trial).
 * A trial of a few steps runs on a short plan whose passes per step differ
 * from a long run's (the plan repeats in blocks of tens of steps), so the
 * candidates within 20% of the fastest trial (at most five) are ranked by
 * their trial time per pass launch times the passes per step of their plan
 * for a 1000-step run (or trial_steps, if longer); the others keep their
 * trial time per step.
 * Planning is done before each timed trial and is not part of the times.
 * Errors as spin_trotter_evolve_ex; SPIN_ENOMEM if the scratch state cannot
 * be allocated; SPIN_EUNSUPPORTED if no candidate ran.
 *
 * spin_tuned_options returns the stored choice for the same key, from the
 * process cache or else from cache_path (may be NULL); SPIN_ENOTFOUND if
 * there is none.  Host only.
 */
typedef struct {
    spin_options opt;          /* the candidate */
    double ms_per_step;        /* ranking: for the refined candidates, trial time per
                                  pass launch x passes_per_step; otherwise the trial
                                  time per step; -1 if the candidate failed */
    double trial_ms_per_step;  /* measured time per step of the trial itself */
    double passes_per_step;    /* of the 1000-step plan (refined candidates), else of
                                  the trial's plan */
    int32_t status;            /* spin_status of the candidate's trial */
    int32_t reserved_;
} spin_tune_result;

int spin_autotune(int32_t prec, int32_t M, const spin_coupling *J, int32_t K, double dt,
                  int32_t observed_site, int64_t trial_steps, const char *cache_path,
                  spin_options *best, spin_tune_result *results, int32_t cap,
                  int32_t *n_results, void *stream);

int spin_tuned_options(int32_t prec, int32_t M, const spin_coupling *J, int32_t K, double dt,
                       int32_t observed_site, const char *cache_path, spin_options *best);

/*
 * Introspection of the execution plan (host only: no device work, usable
 * without a GPU).  The plan is what spin_trotter_evolve_ex would run for the
 * same arguments, or spin_trotter_evolve_profile with observed_site =
 * SPIN_ALL_SITES.
 */
typedef struct {
    int32_t path;           /* 0 = one pass per factor, 1 = whole state in one workgroup,
                               2 = tiled passes */
    int32_t tile_bits;      /* k (path 2), M (path 1) */
    int32_t reg_bits;       /* amplitudes per lane = 2^reg_bits */
    int32_t lanes;          /* lanes per workgroup */
    int32_t coalesce_bits;  /* low address bits in every tile (path 2) */
    int32_t templates;      /* distinct pass templates (path 2) */
    int32_t period_steps, period_passes;  /* repeating block of the plan (path 2) */
    int32_t stages_total;   /* register stages over all templates */
    int32_t engine;         /* stage arithmetic of path 2: 0 VALU butterflies, 1 MFMA matrices */
    int32_t exchange;       /* stage exchanges of path 2: 1 whole tiles, 2 half tiles */
    int32_t reserved_;
    int64_t launches;       /* pass-kernel launches for the whole call */
    int64_t factor_ops;     /* two-spin factor applications after merging, whole call */
    double passes_per_step; /* launches / n_steps (path 2) */
    int64_t exchanges;      /* stage exchanges through LDS over the whole call: each
                               writes and reads every amplitude once (path 2: register
                               stages after the first of each launch; path 1: every
                               stage, the state lives in LDS) */
} spin_plan_info;

int spin_describe_plan(int32_t prec, int32_t M, const spin_coupling *J, int32_t K, double dt,
                       int64_t n_steps, int32_t observed_site, const spin_options *opt,
                       spin_plan_info *info);

/*
 * spin_plan_trace -- the op sequence the plan applies, in execution order,
 * as records of 5 doubles: a factor exp(-i(A I^z_i I^z_j + (B/2)(I^+_i I^-_j +
 * I^-_i I^+_j))) is (0, i, j, A, B) (A, B = strengths times time, merged
 * factors summed); an observable of site n' after step k is (1, k, n', 0, 0).
 *   buf, cap : host buffer of cap records (may be NULL with cap = 0).
 *   len      : number of records of the full trace (always written).
 * Returns SPIN_OK even when cap < *len (the buffer then holds a prefix).
 * Host only; no device work.
 */
int spin_plan_trace(int32_t prec, int32_t M, const spin_coupling *J, int32_t K, double dt,
                    int64_t n_steps, int32_t observed_site, const spin_options *opt,
                    double *buf, int64_t cap, int64_t *len);

/* Thread-local message of the last failed call on this thread ("" if none). */
const char *spin_last_error(void);

/* Frees plan caches, captured graphs, workspaces and the process cache of
 * autotuned choices (files are kept).  Not concurrent-safe with in-flight
 * calls; synchronise the streams used first. */
void spin_release_caches(void);

/* Library version string. */
const char *spin_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SPIN_H_ */
