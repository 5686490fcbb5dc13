/*
 * abcsmc.h -- C ABI of the MI355X (gfx950) implementation of ABC-SMC with
 * Beta-distributed step sizes ("P-ABC-SMC BDSS", Kulkarni & Moritz,
 * arXiv 2106.15508).
 *
 * One SMC round ("stage") over N particles runs on the GPU as hand-written
 * HIP kernels: categorical resampling of the previous stage (eqs. 9-11),
 * per-particle Beta step sizes (eq. 16) and Gaussian perturbation (eq. 17),
 * forward simulation of the stochastic epidemic model (§II-B, eqs. 3-5),
 * Euclidean distance to the observations (§II-C), acceptance dist <= eps
 * (§II-C), importance weights against the previous stage, and the next
 * tolerance as the survival-ratio percentile (eq. 8).
 *
 * Conventions
 *  - Plain C99 types only.  Every pointer argument is HOST memory unless the
 *    comment says "device".  Input buffers are read during the call and not
 *    retained; output buffers are written before the call returns.
 *  - Return value: 0 (ABCSMC_OK) or a negative ABCSMC_E* code.  On error the
 *    context keeps the state of the last completed round; abcsmc_last_error
 *    describes the failure.  After ABCSMC_EDEVICE a context accepts only
 *    abcsmc_free / abcsmc_last_error (further calls return ABCSMC_ESTATE).
 *  - A context is not thread-safe; distinct contexts are independent.
 *  - Results depend only on (config, obs): batch size, launch shapes and the
 *    stream do not change any bit of the trajectories, distances,
 *    acceptances or tolerances.  Importance weights agree with the exact sum
 *    to about 1e-13 relative (summation order is the only freedom).
 *  - Random numbers: Philox4x32-10 keyed by the 64-bit seed, counter
 *    (particle index, round, purpose<<24 | step, block).
 */
#ifndef ABCSMC_H
#define ABCSMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ABCSMC_ABI_VERSION 1
#define ABCSMC_NPAR 8

enum {
    ABCSMC_OK = 0,
    ABCSMC_EINVAL = -1,      /* bad config, observations or argument */
    ABCSMC_ENOMEM = -2,      /* device allocation failed or workspace too small */
    ABCSMC_EDEVICE = -3,     /* a HIP call failed; the context is unusable */
    ABCSMC_EBUDGET = -4,     /* a round did not reach N acceptances within its budget */
    ABCSMC_ESTATE = -5,      /* call not valid in the context's state */
    ABCSMC_EDEGENERATE = -6  /* previous population has no particle to resample */
};

/* Step-size law of the perturbation kernel. */
enum {
    ABCSMC_STEP_PAPER = 0, /* eq. 16: s ~ Beta(eps_i / eps_1, 2 i) in stage i >= 1 */
    ABCSMC_STEP_FIXED = 1  /* s ~ Beta(beta_a, beta_b) in every stage */
};

/* Transition sampler of the simulator (§II-B). */
enum {
    ABCSMC_SAMPLER_BINOMIAL = 0,    /* Bin(n, 1 - exp(-rate)) from the source count */
    ABCSMC_SAMPLER_NORMAL_FLOOR = 1 /* floor(N(h, sqrt(h))) clamped to the source count */
};

enum {
    ABCSMC_F_EARLY_EXIT = 1,      /* stop simulating a proposal once its partial distance exceeds eps
                                     (acceptances unchanged; rejected proposals report d = +inf) */
    ABCSMC_F_STEP_IS_VARIANCE = 2 /* eq. 12 calls s a variance: perturb with sigma = sqrt(s) */
};

/*
 * Problem statement (§II, §IV-A): prior box pi(theta) (eq. 2), observed
 * series D_o of (A, R, D), N accepted samples per stage, survival ratio
 * alpha (eq. 8), step-size law (eq. 16), simulations per batch.
 */
typedef struct {
    int32_t abi_version;          /* must be ABCSMC_ABI_VERSION */
    int32_t n_params;             /* must be 8 */
    double prior_lo[ABCSMC_NPAR]; /* uniform prior box, parameter order of eq. 1: */
    double prior_hi[ABCSMC_NPAR]; /* [alpha0, alpha, n, beta, gamma, delta, eta, kappa]; lo <= hi */
    int64_t population;           /* P, 1 <= P < 2^53, P >= A0 + R0 + D0 */
    int32_t n_days;               /* T, 1 <= T <= 4096 */
    int64_t n_particles;          /* N accepted per stage, 2 <= N <= 2^22 */
    int64_t batch;                /* proposals per batch; 0 = chosen by the library. Results do not depend on it */
    double surv_ratio;            /* alpha of eq. 8, in (0, 1); the paper uses 0.5 */
    int32_t step_schedule;        /* ABCSMC_STEP_* */
    double beta_a;                /* FIXED: Beta shape a > 0 */
    int32_t beta_b;               /* FIXED: integer shape 1 <= b <= 64 */
    int32_t sampler;              /* ABCSMC_SAMPLER_* */
    int32_t flags;                /* ABCSMC_F_* */
    int32_t max_attempts;         /* perturbation redraws before a proposal is void; 0 = 256; <= 4096 */
    uint64_t seed;                /* run seed */
    int64_t max_proposals;        /* per-round budget of proposals; 0 = 4096 * N */
    void* stream;                 /* hipStream_t to run on, or NULL for a library-owned stream */
    void* workspace;              /* optional caller device buffer (e.g. a torch tensor), or NULL */
    size_t workspace_bytes;       /* its size; see abcsmc_workspace_size */
} abcsmc_config;

typedef struct {
    int32_t round;                /* stage index i (0 = prior stage) */
    int32_t beta_b;               /* Beta shape b used in this stage (0 in stage 0) */
    double eps;                   /* tolerance eps^i this stage accepted against (+inf in stage 0) */
    double eps_next;              /* eps^{i+1} = alpha-percentile of the accepted distances (eq. 8) */
    double beta_a;                /* Beta shape a used in this stage */
    double ess;                   /* effective sample size of the importance weights */
    int64_t proposals;            /* proposals up to and including the N-th acceptance */
    int64_t simulated;            /* proposals simulated (whole batches, incl. past the N-th acceptance) */
    int64_t invalid;              /* void proposals (no in-cube perturbation) among `simulated` */
    int64_t attempts;             /* perturbation attempts over `simulated` */
    int64_t survivors;            /* previous-stage particles with resampling weight > 0 (eqs. 9-10) */
    int64_t batches;              /* batches launched */
    double ms_resample, ms_simulate, ms_weights, ms_select, ms_total; /* device time per phase */
    double ms_k_propose;          /* summed device time of the proposal kernel launches */
    double ms_k_weights;          /* device time of the importance-weight kernel */
    int64_t n_k_propose;          /* proposal kernel launches (= batches) */
    int64_t sim_days;             /* proposal-days simulated (early exit stops counting) */
    int64_t weight_pairs;         /* N x survivors terms of the importance-weight sums */
    int64_t weight_terms;         /* terms actually evaluated (the rest lie outside every window and
                                     are exactly zero) */
} abcsmc_round_info;

typedef struct abcsmc_ctx abcsmc_ctx;

/* Device bytes a context needs for cfg (the workspace, if supplied, must be
 * at least this large). */
int abcsmc_workspace_size(const abcsmc_config* cfg, size_t* bytes);

/* Create a context.  obs: (T+1) x 3 int64, row t = (A, R, D) on day t, row 0
 * the initial state; copied.  *out receives the context. */
int abcsmc_init(const abcsmc_config* cfg, const int64_t* obs, abcsmc_ctx** out);

/* Run the next stage (stage 0 is the prior stage with eps^0 = +inf).
 * info may be NULL.  Returns ABCSMC_EBUDGET (context unchanged) when the
 * stage cannot reach N acceptances within max_proposals. */
int abcsmc_round(abcsmc_ctx* ctx, abcsmc_round_info* info);

/* Population of the last completed stage, copied to host buffers (any may
 * be NULL): theta N x 8 in prior units, dist N, weight N (normalised
 * importance weights, sum 1; uniform in stage 0). */
int abcsmc_weights(const abcsmc_ctx* ctx, double* theta, double* dist, double* weight);

/* Per-particle detail of the last completed stage (any may be NULL):
 * u N x 8 unit-cube coordinates, sigma N step sizes, parent N (index into the
 * previous stage, -1 in stage 0), index N proposal indices, attempts N,
 * logw N unnormalised log-weights (8 log sigma - log sum_k q_k N-kernel). */
int abcsmc_population(const abcsmc_ctx* ctx, double* u, double* sigma, int64_t* parent,
                      int64_t* index, int32_t* attempts, double* logw);

/* Integer resampling law the last stage drew its parents from (eqs. 9-11):
 * q N (quantised weights of the previous stage), cdf N (inclusive prefix sum).
 * ABCSMC_ESTATE before stage 1. */
int abcsmc_resampling(const abcsmc_ctx* ctx, uint64_t* q, uint64_t* cdf);

/* Restart the context at stage 0 with the same configuration and seed
 * (the workspace and observations stay resident).  The next abcsmc_round
 * repeats the run bit for bit. */
int abcsmc_reset(abcsmc_ctx* ctx);

/* Stages completed so far. */
int abcsmc_rounds_done(const abcsmc_ctx* ctx);

/* init + n_rounds x round + weights + free.  infos: n_rounds entries or NULL. */
int abcsmc_run(const abcsmc_config* cfg, const int64_t* obs, int32_t n_rounds, double* theta,
               double* dist, double* weight, abcsmc_round_info* infos);

/* Forward-simulate n parameter vectors theta (n x 8, prior units) on the
 * GPU; vector k uses the stream of particle index0 + k in `round` under
 * `seed`.  traj: n x (T+1) x 6 int64 [S, I, A, R, D, Ru] (eq. 3).  obs0 =
 * (A0, R0, D0).  Used for synthetic observations and tests. */
int abcsmc_simulate(const abcsmc_config* cfg, int64_t n, const double* theta, const int64_t* obs0,
                    uint64_t seed, uint32_t round, uint32_t index0, int64_t* traj);

/* Test hook: evaluate a device primitive on n inputs (host buffers).
 *  fn 0..5: exp, expm1, log, log1p, cos 2 pi x, sin 2 pi x   (in: double[n], out: double[n])
 *  fn 6: sqrt, fn 7: x / y                                  (in: double[2n] pairs for 7)
 *  fn 8: Philox4x32-10                                      (in: uint32[6n] ctr0..3,key0..1; out: uint32[4n])
 *  fn 9: Box-Muller pair                                    (in: uint64[n]; out: double[2n])
 *  fn 10: binomial draw                                     (in: {int64 n, double p, uint64 w}[n] as 3 x 8 bytes; out: int64[n])
 *  fn 11: Beta(a, b) draw, a = param_a, b = param_b          (in: uint64[n*b]; out: double[n])
 *  fn 12: floor-normal draw                                 (in: {int64 n, double h, uint64 w}[n]; out: int64[n]) */
int abcsmc_debug_eval(int32_t fn, int64_t n, const void* in, void* out, double param_a, int32_t param_b);

/* ---------------------------------------------------------------------------
 * Batched mode: many independent runs (own population, horizon, particle
 * count, seed, observations, step law) advanced one stage at a time by one
 * captured graph per stage: segmented resampling, one persistent proposal
 * kernel that hands out (run, 256-proposal chunk) work items to every
 * workgroup, per-run ordered compaction, segmented importance weights,
 * per-run percentile.  Each run's trajectories, distances, acceptances and
 * tolerances are bit-identical to the same run alone (abcsmc_init/round);
 * weights agree to 1e-12.  A run that exhausts its per-stage proposal capacity
 * (cfg.max_proposals, default max(4 N, 16384)) stops with ABCSMC_EBUDGET and
 * keeps its last completed stage while the others continue.
 * Stream and workspace come from cfgs[0]; cfgs[r].batch is ignored.
 * ------------------------------------------------------------------------- */
typedef struct abcsmc_batch abcsmc_batch;

/* Launch schedule of the batched mode (no result depends on it). */
typedef struct {
    int32_t propose_blocks;  /* workgroups of the persistent proposal kernel; 0 = 2 per CU */
    int32_t run_order;       /* order runs are offered to workgroups: 0 index, 1 largest N*T first,
                                2 largest/smallest interleaved */
    int32_t weight_cols;     /* target columns per weight-kernel workgroup (0 = 4096) */
    double issue_margin;     /* chunk budget N / (rate * 256) x margin before over-issue (0 = 1.1) */
} abcsmc_schedule;

int abcsmc_batch_workspace_size(const abcsmc_config* cfgs, int32_t n_runs, size_t* bytes);
/* obs[r]: (T_r+1) x 3 int64 of run r; copied.  1 <= n_runs <= 4096, N_r <= 2^20. */
int abcsmc_batch_init(const abcsmc_config* cfgs, int32_t n_runs, const int64_t* const* obs, abcsmc_batch** out);
int abcsmc_batch_set_schedule(abcsmc_batch* b, const abcsmc_schedule* s);
int abcsmc_batch_get_schedule(const abcsmc_batch* b, abcsmc_schedule* s);
/* Time schedule variants (coordinate descent over the four knobs, each trial
 * = stage 0 plus `stages` stages from a reset) and keep the fastest; a line
 * per batch shape is appended to / looked up in cache_path (NULL: no cache).
 * Leaves the batch reset at stage 0. */
int abcsmc_batch_autotune(abcsmc_batch* b, int32_t stages, const char* cache_path, abcsmc_schedule* chosen);
/* Next stage of every run (one graph replay).  infos: n_runs entries or NULL. */
int abcsmc_batch_round(abcsmc_batch* b, abcsmc_round_info* infos);
/* n_rounds stages; infos: n_rounds x n_runs entries (stage-major) or NULL. */
int abcsmc_batch_run(abcsmc_batch* b, int32_t n_rounds, abcsmc_round_info* infos);
int abcsmc_batch_reset(abcsmc_batch* b);
/* 0, or ABCSMC_EBUDGET once run r has stopped. */
int abcsmc_batch_status(const abcsmc_batch* b, int32_t run);
int abcsmc_batch_rounds_done(const abcsmc_batch* b, int32_t run);
/* Last completed stage of run r (any pointer may be NULL); layouts as abcsmc_population /
 * abcsmc_weights (u in unit-cube coordinates). */
int abcsmc_batch_population(const abcsmc_batch* b, int32_t run, double* u, double* sigma, int64_t* parent,
                            int64_t* index, int32_t* attempts, double* logw, double* dist, double* weight);
void abcsmc_batch_free(abcsmc_batch* b); /* NULL-safe */
const char* abcsmc_batch_last_error(const abcsmc_batch* b);

void abcsmc_free(abcsmc_ctx* ctx); /* NULL-safe */
const char* abcsmc_strerror(int code);
const char* abcsmc_last_error(const abcsmc_ctx* ctx); /* NULL ctx: last error of a context-less call */
int abcsmc_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* ABCSMC_H */
