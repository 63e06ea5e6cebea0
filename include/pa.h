/*
 * pa.h -- C ABI of libpa: the data-parallel hot path of population annealing
 * (PA) for the 3D Edwards-Anderson spin glass, with +-J couplings or Gaussian
 * couplings rounded to multiples of 1/16, on one AMD MI355X (gfx950).
 *
 * Method: C. Amey and J. Machta, "Analysis and Optimization of Population
 * Annealing", arXiv:1711.02146.
 *   Sec. II       the annealing loop: a population of R replicas is cooled
 *                 through a schedule of inverse temperatures; at each step the
 *                 replicas are resampled (Eq. 1 resampling factor, Eq. 2
 *                 normaliser Q, nearest-integer copy counts, family labels
 *                 passed to the copies) and then decorrelated by MCMC sweeps.
 *   Sec. II.A     the model H = -sum J_nm s_n s_m on the periodic cubic
 *                 lattice, the population averages, the spin overlap q, the
 *                 link overlap q_l, and the free-energy estimator (Eq. 9).
 *   Sec. III.A    the family statistic rho_t.
 *   Sec. III.C    the culling fraction and the constant-culling step size.
 *
 * Conventions shared with every caller:
 *   - N = L^3 sites, site = x + L*(y + L*z); bond b = d*N + site joins site and
 *     site + e_d (d = 0,1,2 for x,y,z); couplings J[b] are +1 or -1
 *     (PA_MODEL_PM) or the integers k = 16 J in [-127, 127] (PA_MODEL_GAUSS16).
 *   - The energy word U of a replica: PA_MODEL_PM, the number of unsatisfied
 *     bonds (J_b s_i s_j = -1), E = 2U - 3N; PA_MODEL_GAUSS16, E16 = 16 E =
 *     -sum_b k_b s_i s_j as a two's-complement int32.
 *   - The canonical host spin layout is int8 +-1, [replica][site].
 *   - Every random number is a word of Philox4x32-10 (Salmon et al., SC'11)
 *     keyed by the population seed, addressed by (slot, sweep or step, site
 *     group, stream tag); results are therefore reproducible bit for bit and
 *     do not depend on launch shape or on batching.
 *
 * Ownership: the caller owns the device workspace (one allocation per
 * instance, size from pa_workspace_bytes; it must outlive the instance) and
 * the HIP stream.  libpa never allocates device memory; it allocates a little
 * pinned host memory per instance for staging, released by pa_free.
 * Ordering: calls on one instance are stream-ordered; pa_resample,
 * pa_choose_beta, pa_observables, the two overlap calls and the export/import calls
 * synchronise the instance's stream before they return.  One host thread per
 * instance at a time.
 * Errors: every call returns a status; nothing aborts.  After PA_EDEVICE the
 * instance is unusable (free it).  PA_ECAPACITY leaves the population as it
 * was before the failing resampling step.
 */
#ifndef PA_H_
#define PA_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  PA_OK = 0,
  PA_EINVAL = -1,     /* bad argument (sizes, null pointers, odd L, ...) */
  PA_ENOMEM = -2,     /* workspace smaller than pa_workspace_bytes */
  PA_ECAPACITY = -3,  /* resampled population would exceed the capacity */
  PA_EDEVICE = -4,    /* a HIP call failed; the instance is now unusable */
  PA_ESTATE = -5,     /* call out of order (e.g. a failed instance) */
  PA_ESCHEDULE = -6,  /* constant-culling step impossible: eps(0) > target */
  PA_ECHECK = -7      /* PA_FLAG_CHECK_ENERGY: a stored energy word differs from the energy
                         recomputed from the spins; the instance is now unusable */
};

/* pa_params.flags bits (debugging aids; 0 for production runs). */
enum {
  PA_FLAG_CHECK_ENERGY = 1u, /* after every sweep launch, and before every call that reads the
                                energy histogram (pa_resample, pa_choose_beta, pa_observables),
                                recompute each replica's energy word from its spins and the
                                couplings (the Sec. II.A Hamiltonian) and compare it with the
                                stored word; any difference is PA_ECHECK.  Costs one extra
                                kernel and one synchronisation per checked call. */
  PA_FLAG_FAULT_HOOK = 2u,   /* allow pa_debug_inject on this instance */
  PA_FLAG_TIME_SWEEPS = 4u   /* bracket every sweep launch with HIP events on the instance's
                                stream; pa_obs.sweep_ms reports the last one's duration */
};

enum {
  PA_LAYOUT_AUTO = 0,      /* library's choice, resolved when the instance is created (and by
                              pa_workspace_bytes): the layout the autotuner measured or was
                              given for (model, L, size class of R) in this process
                              (pa_autotune_layout, pa_autotune_set_layout), else
                              PA_LAYOUT_BITPACK64.  pa_layout_choice tells which. */
  PA_LAYOUT_INT8 = 1,      /* one byte per spin: tiles of 64 replicas, [tile][site][64] */
  PA_LAYOUT_BITPACK64 = 2  /* one bit per spin: tiles of 64 replicas, [tile][site] u64,
                              bit (r & 63) of word [r >> 6][site] is replica r, 1 <=> s = -1 */
};

enum {
  PA_MODEL_PM = 0,      /* J = +1 or -1 (J_host holds +-1); energy levels U = 0..3N, E = 2U - 3N */
  PA_MODEL_GAUSS16 = 1, /* Gaussian couplings (Sec. II.A) rounded to multiples of 1/16: J_host
                           holds k = 16 J in [-127, 127]; energies are integers E16 = 16 E.
                           Single-instance calls only (batches and steppers take PA_MODEL_PM). */
  PA_MODEL_GAUSS = 2    /* Gaussian couplings (Sec. II.A) as real numbers: created by
                           pa_init_instance_real from FP64 couplings, each rounded to the
                           nearest multiple of 2^-32 (ties to even), |J| < 8; every energy is
                           then exact (a multiple of 2^-32 below 2^17 in size).  Resampling
                           works on per-replica weights (no energy levels); see
                           pa_init_instance_real.  Single-instance calls only. */
};

typedef struct pa_instance pa_instance;

typedef struct {
  uint32_t L;        /* linear size; even, 4 <= L <= 16 (checkerboard needs even L) */
  uint32_t R;        /* target population size (constant over the run), >= 1 */
  uint32_t capacity; /* max population held; 0 selects R + 16*isqrt(R) + 256 */
  uint32_t layout;   /* PA_LAYOUT_* */
  uint64_t seed;     /* population seed: Philox key of every draw of this population */
  uint32_t flags;    /* PA_FLAG_* bits; any other bit is PA_EINVAL */
  uint32_t model;    /* PA_MODEL_*: the coupling distribution J_host is drawn from */
} pa_params;

/* Scalars of one population after a step (Sec. II.A averages, Eq. 9, Sec. III.A). */
typedef struct {
  double beta;         /* current inverse temperature */
  double dbeta;        /* size of the last resampling step */
  double lnQ;          /* ln Q of the last resampling step (Eq. 2) */
  double beta_F;       /* beta F~ = -(N ln 2 + sum of ln Q) (Eq. 9, Omega = 2^N) */
  double mean_E;       /* population average of E */
  double rho_t;        /* (sum over families of eta^2) / R (Sec. III.A) */
  double eps_expected; /* culling fraction of the last step (Sec. III.C) */
  uint32_t R_tilde;    /* current population size */
  uint32_t n_culled;   /* replicas with zero copies in the last step */
  int32_t E_min;       /* lowest energy in the current population (PA_MODEL_GAUSS16: in
                          quanta 1/16, i.e. the lowest E16; mean_E is in units of J) */
  uint32_t step;       /* number of resampling steps done */
  uint64_t sum_eta2;   /* sum over families of eta^2 */
  uint64_t sweeps_done;/* population sweep counter */
  uint32_t n_at_E_min; /* replicas at E_min (ground-state estimators, Sec. II.A); 0 in the
                          record pa_resample returns (it is taken before the sweeps) */
  uint32_t reserved;
  double sum_lnQ;      /* sum of ln Q over the steps so far (Eq. 9: beta F = -(N ln 2 +
                          sum_lnQ)); with the exported spins, family labels, R_tilde,
                          sweeps_done, step and beta it is the whole state a checkpoint
                          needs (pa_import_state) */
  double sweep_ms;     /* PA_FLAG_TIME_SWEEPS: duration of the last sweep launch on the
                          device (HIP events around it), ms; 0 otherwise */
  double E_lowest;     /* lowest energy in the current population in units of J, every model
                          (PA_MODEL_GAUSS: E_min above is 0; this is the exact value); 0 in
                          the record pa_resample returns */
} pa_obs;

/* Bytes of device workspace an instance with these parameters needs. 0 on bad params. */
size_t pa_workspace_bytes(const pa_params* p);

/* Create a population of R replicas at beta = 0 (Sec. II): spin of replica r
 * at site = bit 31 of word (site & 3) of Philox(seed; r, site >> 2, 0, INIT)
 * (bit 1 <=> s = -1); family label r; U computed from the spins.
 * J_host: 3*L^3 couplings, +1/-1 (PA_MODEL_PM) or k in [-127, 127]
 * (PA_MODEL_GAUSS16), copied; any other value is PA_EINVAL.  d_workspace: device memory of at
 * least pa_workspace_bytes(p) bytes, owned by the caller.  hip_stream: the
 * hipStream_t all work of this instance is queued on (NULL = default stream).
 * On success *out holds the new instance. */
int pa_init_instance(const pa_params* p, const int8_t* J_host, void* d_workspace, size_t ws_bytes,
                     void* hip_stream, pa_instance** out);

/* The same for Gaussian couplings as real numbers (Sec. II.A), p->model =
 * PA_MODEL_GAUSS: J_host holds 3*L^3 FP64 couplings in bond order (bond
 * d*N + site joins site and its +d neighbour), each finite with |J| < 8
 * (PA_EINVAL otherwise), rounded to the nearest multiple of 2^-32.  The
 * model's readings (the paper fixes no arithmetic):
 *   - energies are exact: the int64 word E 2^32 per replica;
 *   - a move raising E by dE > 0 is taken iff its draw is below
 *     floor(2^32 e(-beta dE)), where e(x) is exp evaluated by Cody and Waite's
 *     reduction (x = k ln 2 + r, k the nearest integer to x log2(e), r by two
 *     fused multiply-adds with ln 2 split into its FP64 rounding and the
 *     rounded remainder) and the Taylor polynomial of degree 13 in r by
 *     Horner's rule, one fused multiply-add per degree, times 2^k; e(x) = 0
 *     below x = -708;
 *   - a resampling step weighs replica i by w_i = e(-(dbeta (E_i - E_min)));
 *     the normaliser S = sum w_i (Eq. 2 times R~) and the culled mass
 *     sum_{tau_i < 1} (1 - tau_i) (Sec. III.C) are sums of terms truncated to
 *     multiples of 2^-96, added exactly and rounded once to FP64 (nearest,
 *     ties to even), so they do not depend on the order of addition;
 *     tau_i = (R w_i) / S and the copy counts follow the rule of every model;
 *     ln Q = ln S - ln R~ - dbeta E_min;
 *   - <E> = (the exact sum of the energy words rounded once to FP64) / R~ 2^-32.
 * pa_choose_beta runs the constant-culling bisection on the device.  U_host
 * of pa_export_state must be NULL (pa_export_energies gives the energies).
 * Other errors as pa_init_instance. */
int pa_init_instance_real(const pa_params* p, const double* J_host, void* d_workspace,
                          size_t ws_bytes, void* hip_stream, pa_instance** out);

/* n_sweeps Metropolis sweeps at beta (the MCMC step of Sec. II): colour 0
 * then colour 1 of the checkerboard; a move raising the energy by dE > 0 is
 * accepted iff word (cm & 3) of Philox(seed; slot, t, cm >> 2, MET) is below
 * floor(2^32 exp(-beta dE)), cm being the site's colour-major index and t the
 * population's sweep counter (advanced by one per sweep).  Fuses the gather
 * of a preceding pa_resample.  Asynchronous. */
int pa_sweep(pa_instance* in, double beta, uint32_t n_sweeps);

/* Resampling step beta -> beta_next (Sec. II, Eqs. 1-2): energy histogram,
 * FP64 normaliser and free-energy increment, nearest-integer copy counts
 * (the extra copy iff a 53-bit Philox integer is below ceil(frac(tau) 2^53)),
 * exclusive scan, and an order-preserving copy of the survivors with their
 * family labels (the copy itself is done by the next pa_sweep, or on demand).
 * Synchronises.  step_out (nullable) receives beta, dbeta, lnQ, beta_F,
 * R_tilde (new), n_culled, eps_expected, step. */
int pa_resample(pa_instance* in, double beta_next, pa_obs* step_out);

/* One whole temperature step of the anneal (Sec. II loop) with a single
 * host synchronisation: with eps_target >= 0, the constant-culling step of
 * pa_choose_beta (target eps_target, at most beta_max); with eps_target < 0,
 * the caller's *beta_next (finite, >= 0; beta_max is ignored).  Then the
 * resampling step to it (pa_resample), n_sweeps (>= 1) sweeps there (pa_sweep)
 * and the observables (pa_observables) into out (nullable).  *beta_next
 * receives the new inverse temperature.  Every bit equals that sequence of
 * calls.  PA_ECAPACITY leaves the population as it was (nothing after the
 * capacity check runs); PA_ESCHEDULE as pa_choose_beta. */
int pa_anneal_step(pa_instance* in, double eps_target, double beta_max, uint32_t n_sweeps,
                   double* beta_next, pa_obs* out);

/* Up to max_steps steps of the constant-culling anneal (Sec. II loop with the
 * Sec. III.C step choice, target eps_target >= 0), stopping when beta_max is
 * reached: each step is exactly pa_anneal_step(in, eps_target, beta_max,
 * n_sweeps, ...), bit for bit.  For +-J populations the steps are queued so
 * that the device computes one step's family sums while the host chooses the
 * next step, with one synchronisation per step.  obs (nullable, max_steps
 * entries) receives each step's scalars; *steps_done the number of steps
 * taken.  On an error (PA_ECAPACITY, PA_ESCHEDULE, ...) the steps before it
 * stand and *steps_done counts them; PA_ECAPACITY leaves the population as it
 * was after the last of them. */
int pa_anneal_run(pa_instance* in, double eps_target, double beta_max, uint32_t n_sweeps,
                  uint32_t max_steps, pa_obs* obs, uint32_t* steps_done);

/* Constant-culling step (Sec. III.C): the beta_next in (beta, beta_max] whose
 * culling fraction eps = sum_{tau<1}(1 - tau) / R is eps_target, by 64
 * bisection halvings on [0, beta_max - beta] (mid = lo + (hi - lo)/2) keeping
 * the lower end, so eps <= eps_target; beta_max itself when the whole range
 * culls no more.  PA_ESCHEDULE if eps(0) already exceeds eps_target.
 * Synchronises. */
int pa_choose_beta(pa_instance* in, double eps_target, double beta_max, double* beta_next);

/* Current scalars (Sec. II.A averages, Eq. 9, Sec. III.A).  Synchronises. */
int pa_observables(pa_instance* in, pa_obs* out);

/* Spin-overlap histogram between slot i of population a and slot i of
 * population b, i < min(R~_a, R~_b) (Sec. II.A spin overlap; the two
 * populations must share L and couplings).  With d = number of differing
 * sites, bin = (128 (N - d) + N) / (2N) (round-half-up of 64 (1+q)/2).
 * nbins must be 65; hist_out receives 65 counts.  Synchronises. */
int pa_overlap_hist(pa_instance* a, pa_instance* b, uint32_t nbins, uint64_t* hist_out);

/* Link-overlap histogram between slot i of population a and slot i of
 * population b, i < min(R~_a, R~_b) (Sec. II.A link overlap q_l over the
 * N_b = 3N bonds; the two populations must share L, layout and couplings;
 * either model).  With x_n = s^a_n s^b_n, a bond <n,m> contributes
 * x_n x_m, so q_l = 1 - 2 D / N_b where D counts the bonds whose two ends
 * have different x.  nbins must be 3N + 1; hist_out (caller-owned, nbins
 * entries) receives hist_out[D] = the number of pairs with that D.
 * PA_EINVAL for a == b, different L or layout, a wrong nbins or a null
 * hist_out; PA_ESTATE for an unusable instance.  Synchronises. */
int pa_link_overlap_hist(pa_instance* a, pa_instance* b, uint32_t nbins, uint64_t* hist_out);

/* pa_link_overlap_hist for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the partial and the final counts live in a fixed scratch array
 * of the library in each GPU's memory (PA_NOALLOC_SCRATCH_BYTES, held from the
 * first instance created on that GPU until the process ends), not in the
 * workspace of instance a.  Same arguments, result and errors as
 * pa_link_overlap_hist, and in addition: PA_ENOMEM when nbins exceeds
 * PA_NOALLOC_MAX_BINS (the array holds the counts of lattices up to L = 12);
 * PA_EINVAL unless both instances were created on the current device;
 * PA_EDEVICE if the array's address could not be obtained.  Allocates
 * nothing.  Every call on one GPU uses that GPU's one array: calls that
 * overlap in time on one GPU (from other host threads, on other streams) race
 * and must not be made.  Synchronises. */
#define PA_NOALLOC_MAX_BINS 5185u
#define PA_NOALLOC_SCRATCH_BYTES (32u * PA_NOALLOC_MAX_BINS * 4u + PA_NOALLOC_MAX_BINS * 8u)
int pa_link_overlap_hist_noalloc(pa_instance* a, pa_instance* b, uint32_t nbins,
                                 uint64_t* hist_out);

/* Copy the current population to the host in the canonical layout.
 * spins_host: R~ * N int8 (+1/-1), [replica][site]; U_host, family_host: R~
 * entries each (U_host: the energy word, for PA_MODEL_GAUSS16 the bits of the
 * int32 E16); any of the three may be NULL.  *R_tilde receives R~ (call
 * once with all arrays NULL to size them).  Synchronises. */
int pa_export_state(pa_instance* in, int8_t* spins_host, uint32_t* U_host, uint32_t* family_host,
                    uint32_t* R_tilde);

/* Copy counts n_i and offsets (exclusive scan) of the last resampling step,
 * R~_old entries each (R~ before that step: *n_old receives it).  For tests
 * and diagnostics.  Synchronises. */
int pa_export_counts(pa_instance* in, uint32_t* counts_host, uint32_t* offsets_host,
                     uint32_t* n_old);

/* Energies of the current population in units of J, one FP64 per replica
 * (exact for every model: E = 2U - 3N for PA_MODEL_PM, E16 / 16 for
 * PA_MODEL_GAUSS16, E32 2^-32 for PA_MODEL_GAUSS).  E_host: R~ doubles
 * (pa_observables tells R~).  Synchronises. */
int pa_export_energies(pa_instance* in, double* E_host);

/* Replace the population (checkpoint restore, or tests feeding a state in):
 * R_tilde replicas, spins [replica][site] int8 +-1, family labels (< R), the
 * sweep counter t, the step index k, the current beta and the accumulated
 * sum of ln Q.  U is recomputed from the spins.  Synchronises. */
int pa_import_state(pa_instance* in, const int8_t* spins_host, const uint32_t* family_host,
                    uint32_t R_tilde, uint64_t sweeps_done, uint32_t step, double beta,
                    double sum_lnQ);

/* Release the host-side handle (the caller frees the workspace afterwards). */
int pa_free(pa_instance* in);

/* Fault injection for tests of callers' error handling (instances created
 * with PA_FLAG_FAULT_HOOK only; PA_EINVAL otherwise or for an unknown `what`).
 * Everything is done on the host: no kernel is made to fail.
 *   PA_INJECT_FAIL_AFTER: after `arg` more calls on this instance return
 *     normally, the next one returns PA_EDEVICE without queuing any work and
 *     the instance becomes unusable, as after a real HIP error.  Calls that
 *     count: pa_sweep, pa_resample, pa_choose_beta, pa_observables, the two
 *     overlap calls (for either instance), the export/import calls,
 *     pa_autotune_sweep and pa_stepper_step (per instance in its set).
 *   PA_INJECT_ENERGY: add 1 to the stored energy word of replica `arg`
 *     (< R~) with a host-to-device copy, so that a PA_FLAG_CHECK_ENERGY
 *     check finds it.  Synchronises. */
enum { PA_INJECT_FAIL_AFTER = 1, PA_INJECT_ENERGY = 2 };
int pa_debug_inject(pa_instance* in, uint32_t what, uint32_t arg);

/* +-J couplings of one disorder sample (Sec. II.A model with couplings +-1 of
 * probability 1/2), on the host: J_out[b] = +1 if bit 31 of word (b & 3) of
 * Philox4x32-10(key = coupling_seed; counter = (b >> 2, 0, 0, TAG_J)) is 0,
 * else -1, for the 3 L^3 bonds b (TAG_J = 0x434F5550).  J_out: 3 L^3 int8,
 * caller-owned.  PA_EINVAL for a null J_out or L outside [2, 64].  Callers
 * may pass any other couplings to pa_init_instance instead. */
int pa_make_couplings_pm(uint64_t coupling_seed, uint32_t L, int8_t* J_out);

/* ------------------------------------------------------------------------ */
/* Batches: many populations (PA_MODEL_PM instances of any L, R and layout)  */
/* together through one temperature schedule (Sec. II loop), each step being */
/* one replay of a captured HIP graph: device-side FP64 resampling tables    */
/* (the exp weights come from the host's exp, one row per step), copy        */
/* counts, scans, fused copy + sweeps for all populations, and the per-step  */
/* records (sum of E, lowest E, size, sum of eta^2, ln Q inputs) and overlap */
/* histograms of chosen population pairs.  Each population draws exactly the */
/* numbers it would draw alone, so every result equals the result of the     */
/* same calls made on the instance by itself (pa_resample + pa_sweep +       */
/* pa_observables), bit for bit.                                             */
/* ------------------------------------------------------------------------ */
typedef struct pa_batch pa_batch;

/* Device workspace for a batch of n_pops populations (largest L max_L),
 * n_pairs overlap pairs and n_steps temperature steps.  0 on bad sizes. */
size_t pa_batch_workspace_bytes(uint32_t n_pops, uint32_t n_pairs, uint32_t n_steps,
                                uint32_t max_L);

/* Build a batch over existing instances (all on the same HIP stream, none
 * already in a batch, none with a pending copy step; their current beta must
 * equal betas[0]).  betas: n_steps + 1 inverse temperatures, betas[0] the
 * current one; each step resamples to betas[s] and runs n_sweeps sweeps there.
 * A PA_MODEL_GAUSS16 instance is PA_EINVAL.
 * pairs: 2 * n_pairs instance indices (same L and layout within a pair) whose
 * overlap histogram (pa_overlap_hist's binning) is recorded after every step;
 * may be NULL when n_pairs = 0.  The caller owns d_workspace
 * (pa_batch_workspace_bytes bytes) until pa_batch_free.  Synchronises. */
int pa_batch_create(pa_instance* const* pops, uint32_t n_pops, const uint32_t* pairs,
                    uint32_t n_pairs, const double* betas, uint32_t n_steps, uint32_t n_sweeps,
                    void* d_workspace, size_t ws_bytes, pa_batch** out);

/* Run the next n_steps steps of the schedule (asynchronous: graph replays). */
int pa_batch_run(pa_batch* b, uint32_t n_steps);

/* Wait for the batch and fetch its results.  obs: [steps_done][n_pops]
 * pa_obs records (nullable); qhist: [steps_done][n_pairs][65] counts
 * (nullable); status: per population 0, or PA_ECAPACITY if a step would have
 * overflowed its capacity (that population stopped before that step).
 * *steps_done receives the number of steps run.  Afterwards each instance is
 * at its last completed step and usable on its own again. */
int pa_batch_results(pa_batch* b, pa_obs* obs, uint64_t* qhist, int32_t* status,
                     uint32_t* steps_done);

/* Release a batch (its instances stay valid). */
int pa_batch_free(pa_batch* b);

/* ------------------------------------------------------------------------ */
/* Stepper: continuous batching.  One call advances any set of resident      */
/* instances by one temperature step each (Sec. II loop: resample to the     */
/* instance's next beta with Eqs. 1-2, then its n_sweeps sweeps there), all  */
/* in one set of launches; the set, the temperatures and the sweep counts    */
/* may differ from call to call, so requests can join and leave between      */
/* steps.  Each instance draws exactly the numbers it would draw alone, so    */
/* every result equals that of pa_resample + pa_sweep + pa_observables on    */
/* the instance by itself, bit for bit.                                      */
/* ------------------------------------------------------------------------ */
typedef struct pa_stepper pa_stepper;

/* Device workspace of a stepper for sets of up to max_pops instances of
 * linear size <= max_L.  0 on bad sizes. */
size_t pa_stepper_workspace_bytes(uint32_t max_pops, uint32_t max_L);

/* Create a stepper that launches on hip_stream (every instance it steps must
 * have been created on that stream).  The caller owns d_workspace
 * (pa_stepper_workspace_bytes bytes, 256-byte aligned) until pa_stepper_free.
 * libpa allocates a pinned host staging image of the same size. */
int pa_stepper_create(uint32_t max_pops, uint32_t max_L, void* d_workspace, size_t ws_bytes,
                      void* hip_stream, pa_stepper** out);

/* One step for n instances (distinct, usable, not in a batch, no pending copy
 * step): instance p resamples from its current beta to beta_next[p] and runs
 * n_sweeps[p] sweeps at beta_next[p].  obs[p] (nullable array) receives its
 * scalars after the step, as pa_observables would report them; status[p]
 * (nullable array) PA_OK, or PA_ECAPACITY when the copy step would exceed the
 * capacity (that instance is left as it was).  PA_MODEL_GAUSS16 instances are
 * PA_EINVAL.  Synchronises the stream. */
int pa_stepper_step(pa_stepper* s, pa_instance* const* pops, uint32_t n, const double* beta_next,
                    const uint32_t* n_sweeps, pa_obs* obs, int32_t* status);

/* pa_stepper_step is also the batch step to caller-given temperatures (the
 * "batch step with beta_next per instance" of a batch interface): a stepper
 * over the batch's instances, called with one beta_next per instance, advances
 * them all by one step in one set of launches.  pa_batch_run replays steps whose
 * temperatures were fixed at creation, as captured graphs. */

/* Release a stepper (its instances stay valid). */
int pa_stepper_free(pa_stepper* s);

/* ------------------------------------------------------------------------ */
/* Autotuner.  The sweep kernel (Sec. II MCMC sweeps, Sec. II.A model) runs   */
/* one 64-replica tile per workgroup with 4 or 8 waves sharing it; which is   */
/* faster depends on L, the number of tiles in the launch and the device.     */
/* Both give the same bits.  A built-in rule measured on MI355X is used until */
/* the autotuner has timed a shape in this process.                          */
/* ------------------------------------------------------------------------ */

/* Time n_sweeps-sweep launches of both forms on the instance (repeats times
 * each, at inverse temperature beta >= 0: the regime the caller will run in;
 * at beta = 0 no draw is made) and remember the faster for launches of the same
 * coupling model, spin layout, L and size class (floor(log2(tiles))), in this
 * process, for single instances, batches and steppers alike.  The population, its counters and
 * its results are not changed (the trial sweeps write only the spare buffer).
 * split_out (nullable): the chosen waves per tile; ms_out (nullable, 2
 * floats): average launch time of the 4- and 8-wave forms.  Needs no pending
 * copy step (PA_ESTATE).  Synchronises. */
int pa_autotune_sweep(pa_instance* in, double beta, uint32_t n_sweeps, uint32_t repeats,
                      uint32_t* split_out, float* ms_out);

/* Forget every autotuned choice, sweep forms and layouts (back to the built-in
 * rules). */
int pa_autotune_reset(void);

/* Spin layout (Sec. II state of a replica; both layouts hold the same spins and
 * every result is the same in either).  Which one sweeps faster depends on L,
 * the population size and the device: the autotuner times both on a shape and
 * PA_LAYOUT_AUTO then resolves to the faster for every population of that
 * coupling model, L and size class (floor(log2(ceil(R / 64)))) created later
 * in this process, single instances and the members of batches and steppers
 * alike.  Because the choice is process-wide, a caller that sizes a workspace
 * with PA_LAYOUT_AUTO and creates the instance later should resolve the layout
 * once (pa_layout_choice) and pass it explicitly, or a choice recorded in
 * between may make the workspace too small (PA_ENOMEM). */

/* Device workspace pa_autotune_layout needs for params p (the larger of the
 * two layouts' pa_workspace_bytes; p->layout and p->flags are ignored); 0 on bad
 * params. */
size_t pa_autotune_layout_workspace_bytes(const pa_params* p);

/* Time both layouts on the shape of p: for each, create a population (p with
 * that layout and flags 0; J_host as for pa_init_instance) in d_workspace (at
 * least pa_autotune_layout_workspace_bytes(p) bytes, caller-owned, 256-byte
 * aligned) on hip_stream, time its sweep forms as pa_autotune_sweep does at
 * (beta, n_sweeps, repeats) and record the faster form for that layout, then
 * free it.  The layout whose faster form is faster is recorded for
 * (p->model, p->L, size class of p->R).  layout_out (nullable): the chosen
 * PA_LAYOUT_*; ms_out (nullable, 2 floats): the best launch time of the int8
 * and the bit-packed layout.  PA_EINVAL on bad params or arguments, PA_ENOMEM
 * on a small workspace, PA_EDEVICE on a HIP error.  Synchronises; the workspace
 * holds nothing of value afterwards. */
int pa_autotune_layout(const pa_params* p, const int8_t* J_host, void* d_workspace,
                       size_t ws_bytes, void* hip_stream, double beta, uint32_t n_sweeps,
                       uint32_t repeats, uint32_t* layout_out, float* ms_out);

/* The layout PA_LAYOUT_AUTO resolves to now for (model, L, size class of R):
 * *layout_out = PA_LAYOUT_INT8 or PA_LAYOUT_BITPACK64.  Host only (no device
 * call).  PA_EINVAL on an unknown model, L outside [4, 16] or odd, R = 0 or a
 * null layout_out. */
int pa_layout_choice(uint32_t model, uint32_t L, uint32_t R, uint32_t* layout_out);

/* Pin the layout for a shape instead of timing it: populations of the coupling
 * model, L and size class of `tiles` (floor(log2(tiles)), tiles = ceil(R / 64))
 * created with PA_LAYOUT_AUTO get `layout` (PA_LAYOUT_INT8 or
 * PA_LAYOUT_BITPACK64), until pa_autotune_reset or another choice for the shape.
 * PA_EINVAL on an unknown model or layout, L outside [4, 16] or odd, or
 * tiles = 0. */
int pa_autotune_set_layout(uint32_t model, uint32_t L, uint64_t tiles, uint32_t layout);

/* Pin the sweep form for a shape instead of timing it: launches of the
 * coupling model (PA_MODEL_*), spin layout (PA_LAYOUT_INT8 or
 * PA_LAYOUT_BITPACK64), L and size class of `tiles` (floor(log2(tiles)),
 * tiles = ceil(R~ / 64)) use `split` waves per tile (4 or 8) in this process,
 * until pa_autotune_reset or another choice for the same shape.  The results
 * do not depend on it.  PA_EINVAL on an unknown model or layout, L outside
 * [4, 16] or odd, tiles = 0, or another split. */
int pa_autotune_set(uint32_t model, uint32_t layout, uint32_t L, uint64_t tiles, uint32_t split);

/* ------------------------------------------------------------------------ */
/* Diagnostics: this device's ceilings for the sweep's roofline.             */
/* ------------------------------------------------------------------------ */
typedef struct {
  double valu_lane_ops_per_s;  /* sustained issue rate of v_add_u32 (two register
                                  sources), lane-operations per second */
  double valu3_lane_ops_per_s; /* the same for v_bfe_u32 (three sources), the rate
                                  of bit-field extracts and three-input adds */
  double philox_draws_per_s;   /* Metropolis Philox4x32-10 draws per second with
                                  nothing else computed (the sweep's counter layout) */
} pa_ceilings;

/* Device bytes pa_probe_ceilings needs as scratch (one word per probe lane). */
size_t pa_probe_scratch_bytes(void);

/* Time three probe kernels on hip_stream (null: the default stream) with HIP
 * events, two untimed launches then five timed ones each, and report their
 * average rates: independent v_add_u32 chains and v_bfe_u32 chains over a grid
 * that fills every SIMD, and the sweep's Philox calls alone.  d_scratch: caller-owned device
 * memory of at least pa_probe_scratch_bytes() bytes, 4-byte aligned; its
 * contents are overwritten.  PA_EINVAL on a null or short buffer or a null
 * out; PA_EDEVICE on a HIP error.  Synchronises. */
int pa_probe_ceilings(void* d_scratch, size_t bytes, void* hip_stream, pa_ceilings* out);

/* Static description of a status code. */
const char* pa_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* PA_H_ */
