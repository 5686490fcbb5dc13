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

#define ABCSMC_ABI_VERSION 4
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
    ABCSMC_STEP_FIXED = 1, /* s ~ Beta(beta_a, beta_b) in every stage */
    ABCSMC_STEP_MCMC = 2,  /* the paper's baseline (§II-D, eqs. 12-15): one step size s for every
                              proposal of a batch ("run"); after each of the first mcmc_tune batches
                              of stages >= 1, s <- s (1 + (A - 0.234) / (0.766 (n_acc + 1))) with A =
                              accepted / valid proposals of the batch and n_acc the acceptances of
                              all tuned batches so far; needs batch > 0 (whole batches are simulated,
                              so results depend on it); single-run contexts only */
    ABCSMC_STEP_MEANVAR = 3,   /* alternative Beta parameterisation (§III-B), mean and variance from the
                                  same two quantities as eq. 16: mean mu = (eps_i/eps_1)/3, variance
                                  mu (1 - mu) / (3 i + 1); real shapes, gamma-ratio sampler */
    ABCSMC_STEP_MODECONC = 4   /* mode-concentration: mode (eps_i/eps_1)/4, concentration 2 i + 2 */
};

/* Transition sampler of the simulator (§II-B). */
enum {
    ABCSMC_SAMPLER_BINOMIAL = 0,    /* Bin(n, 1 - exp(-rate)) from the source count */
    ABCSMC_SAMPLER_NORMAL_FLOOR = 1 /* floor(N(h, sqrt(h))) clamped to the source count */
};

enum {
    ABCSMC_F_EARLY_EXIT = 1,      /* stop simulating a proposal once its partial distance exceeds eps
                                     (acceptances unchanged; rejected proposals report d = +inf) */
    ABCSMC_F_STEP_IS_VARIANCE = 2, /* eq. 12 calls s a variance: perturb with sigma = sqrt(s) */
    ABCSMC_F_SKIP_WEIGHTS = 4      /* no importance weights: every stage reports W = 1/N, log-weights 0
                                      and ESS = N (simulation-only runs; trajectories, acceptances and
                                      tolerances never depend on the weights) */
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
    double mcmc_s0;               /* STEP_MCMC: initial step size s > 0 */
    int32_t mcmc_tune;            /* STEP_MCMC: number of tuned batches (>= 0) */
    int32_t n_eps_schedule;       /* 0..4096 tolerances to replay (single-run contexts only) */
    const double* eps_schedule;   /* host array (copied at init): stage i = 1..n_eps_schedule accepts
                                     against eps_schedule[i-1] (finite, >= 0) instead of eq. 8's
                                     percentile of stage i-1; later stages use eq. 8 again.  eq. 16's
                                     eps_1 is then eps_schedule[0].  NULL when n_eps_schedule = 0 */
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
    double ms_k_weights;          /* device time of the importance-weight sum kernel (without the window
                                     pass before it and the merge of chunk sums after it) */
    int64_t n_k_propose;          /* proposal kernel launches (= batches) */
    int64_t sim_days;             /* proposal-days simulated (early exit stops counting) */
    int64_t weight_pairs;         /* N x survivors terms of the importance-weight sums */
    int64_t weight_terms;         /* terms actually evaluated (the rest lie outside every row's window,
                                     which bounds their total by 2^-53 of the row sum) */
    double mcmc_s;                /* STEP_MCMC: step size after this stage (0 otherwise) */
    double beta_b_real;           /* Beta shape b as a real number (STEP_MEANVAR / STEP_MODECONC) */
    int64_t weight_window_terms;  /* sum over the N rows of the columns inside the row's own window (the
                                     terms the row sums need; weight_terms - this = terms evaluated
                                     because another row of the same wave needed them) */
} abcsmc_round_info;

typedef struct abcsmc_ctx abcsmc_ctx;

/* Device bytes a context needs for cfg (the workspace, if supplied, must be
 * at least this large, 256-byte aligned, and left to the context until
 * abcsmc_free: it holds the populations between stages and tables written
 * once at abcsmc_init). */
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

/* Posterior predictive simulation (§IV-B, Fig. 7): every particle j of the
 * last completed stage (theta_j = lo + u_j (hi - lo)) is simulated for
 * n_days days from the observed day-0 state with the random stream (seed,
 * particle j, round 0xFFFE); for each day t = 0..n_days and series c = A, R,
 * D the type-7 quantiles (numpy "linear") of the N simulated counts at the
 * n_quant levels quant[] (in [0, 1], 1 <= n_quant <= 64) are written to
 * bands[(3 t + c) n_quant + k].  n_days may exceed the fitted horizon (the
 * days after it are the prediction).  Allocates (n_days+1) x 3 x N doubles of
 * device memory for the duration of the call (ABCSMC_ENOMEM if it cannot). */
int abcsmc_predict(const abcsmc_ctx* ctx, int32_t n_days, uint64_t seed, int32_t n_quant, const double* quant,
                   double* bands);

/* Restart the context at stage 0 with the same configuration and seed
 * (the workspace and observations stay resident).  The next abcsmc_round
 * repeats the run bit for bit. */
int abcsmc_reset(abcsmc_ctx* ctx);

/* Stages completed so far. */
int abcsmc_rounds_done(const abcsmc_ctx* ctx);

/* Checkpoint and resume.  A snapshot holds what the next stage reads from
 * the last completed one: the population (u, d, sigma, parent, index,
 * attempts, log-weights, weights; eqs. 9-11 resample it), the stage count,
 * eps^{i+1} (eq. 8) and eps_1 (eq. 16), the batch-sizing rate and the MCMC
 * step-size state, plus a fingerprint of the configuration and the
 * observations.  abcsmc_snapshot with buf == NULL stores the size in *bytes;
 * otherwise *bytes is the capacity of buf (host memory, caller-owned) and is
 * set to the bytes written (EINVAL if too small).  ESTATE before the first
 * stage or while the learned screen is enabled.
 * abcsmc_restore creates a context as abcsmc_init(cfg, obs) does and loads
 * the snapshot; EINVAL if the buffer is malformed or was taken under another
 * configuration (seed, sizes, model, schedule) or other observations.  The
 * restored context continues the run bit for bit (its own abcsmc_reset goes
 * back to stage 0). */
int abcsmc_snapshot(const abcsmc_ctx* ctx, void* buf, size_t* bytes);
int abcsmc_restore(const abcsmc_config* cfg, const int64_t* obs, const void* buf, size_t bytes, abcsmc_ctx** out);

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
 *  fn 12: floor-normal draw                                 (in: {int64 n, double h, uint64 w}[n]; out: int64[n])
 *  fn 13: real-shape Beta draw (gamma ratio)                 (in: double[2] = {a, b}; out: double[n]; draw i
 *         uses stream (seed = param_a, particle i, round = param_b, PERTURB, attempt 0))
 *  fn 14: importance-weight term q_k exp(-|u_j - u_k|^2 / (2 sigma_j^2)) as the weight kernels
 *         evaluate it (table exponential)       (in: double[18n] records {u_j[8], sigma_j, u_k[8], q_k};
 *                                                out: double[n]) */
int abcsmc_debug_eval(int32_t fn, int64_t n, const void* in, void* out, double param_a, int32_t param_b);

/* Measurement helper (not part of the method): what the current device
 * sustains, as context for the roofline fractions, which are taken against
 * the published peaks.  fp64_tflops: FP64 vector fma throughput (2 flops per
 * fma) of eight independent chains per lane at eight waves per SIMD;
 * clock_mhz: the shader clock during that launch (its cycle counter against
 * the 100 MHz constant counter); copy_gbs: device-to-device copy of 1 GiB
 * (bytes read + bytes written per second).  Each the best of `repeats`
 * (1..100) timed launches after one untimed one.  Allocates 2 GiB + 4 MiB of
 * device memory for the duration of the call (ABCSMC_ENOMEM if it cannot);
 * runs on the null stream of the current device and waits for it. */
int abcsmc_measure_peaks(int32_t repeats, double* fp64_tflops, double* clock_mhz, double* copy_gbs);

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
/* obs[r]: (T_r+1) x 3 int64 of run r; copied.  1 <= n_runs <= 4096, N_r <= 2^20, sum of N_r <= 2^26. */
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

/* ---------------------------------------------------------------------------
 * Learned surrogate screen (an extension; the paper simulates every
 * proposal).  A multilayer perceptron 8 -> 256 -> 256 -> 256 -> 3 with
 * tanh-GELU activations maps a proposal's unit-cube coordinates (as 2u - 1)
 * to y_c = log1p(sqrt(S_c)), where S_A, S_R, S_D are the per-series sums of
 * squared differences whose total is the distance of §II-C; the score
 * sum_c expm1(y_c)^2 predicts d^2.  Matrix products use bfloat16 operands
 * (round to nearest even) on the matrix cores with FP32 accumulation; weights,
 * gradients and Adam state (0.9, 0.999, 1e-8) are FP32.
 *
 * abcsmc_surrogate_enable fits the network on the GPU to n_train prior
 * simulations (the stage-0 streams of indices 0 .. n_train-1; minibatches in
 * index order).  In every later stage each batch of proposals is perturbed
 * exactly as in the plain stage (same per-index streams), scored, and only
 * proposals with score <= tau, or that pass an audit draw U < rho from their
 * own AUDIT stream (purpose 4), are simulated; tau is the keep_frac
 * percentile of the stage's first batch.  Acceptance is d <= eps on the exact
 * FP64 simulation, first N in index order.  The stage's proposal density is
 * q(u) (1{score <= tau} + rho 1{score > tau}) / Z, so an acceptance kept only
 * by the audit gets log-weight - log rho.  The kept proposals of the first
 * batch (up to tune_rows) are simulated in full and the network is trained
 * on them for tune_epochs after the stage.  When a stage's audit estimate of
 * the accepted mass with score > tau exceeds fn_max, later stages run plain.
 * The state lives in its own device allocation (not the workspace);
 * abcsmc_reset restores the network of the initial fit.
 * ------------------------------------------------------------------------- */
typedef struct {
    int64_t n_train;     /* prior simulations of the initial fit; 0 = 2^20; <= 2^24 */
    int32_t epochs;      /* passes over them; 0 = 4; < 0: none (random network) */
    int32_t batch;       /* minibatch rows; 0 = 8192; <= 65536 */
    double lr;           /* Adam step; 0 = 1e-3 */
    double keep_frac;    /* fraction of the first batch kept by score (sets tau); 0 = 0.1; in (0, 1] */
    double audit_rho;    /* audit probability of a proposal with score > tau; 0 = 0.01; in (0, 1] */
    int64_t pool;        /* proposals per batch at most; 0 = 2^22; in [1024, 2^22] */
    int64_t tune_rows;   /* fine-tune rows per stage (rounded down to 256); 0 = min(65536, pool); < 0: none */
    int32_t tune_epochs; /* fine-tune passes; 0 = 2; < 0: none */
    double fn_max;       /* false-negative mass that ends screening; 0 = 0.05 */
    uint64_t seed;       /* network initialisation: N(0, 1/fan_in) weights from the MLP stream (purpose 5) */
} abcsmc_surrogate_config;

typedef struct {
    double loss_first;        /* mean squared error per output over the first epoch of the initial fit */
    double loss_last;         /* ... and over its last epoch */
    int64_t train_steps;      /* Adam steps so far */
    double ms_train;          /* device time of the initial fit's training steps */
    int32_t active;           /* 1 while stages are screened */
    int32_t round;            /* last screened stage (-1: none yet) */
    double tau;               /* its score threshold */
    int64_t kept_screen;      /* proposals kept with score <= tau (over its whole batches) */
    int64_t kept_audit;       /* proposals kept only by the audit */
    int64_t accepted_screen;  /* acceptances among kept_screen */
    int64_t accepted_audit;   /* acceptances among kept_audit */
    double enrichment;        /* acceptance rate of kept_screen / estimated acceptance rate of all proposals */
    double fn_mass;           /* audit estimate of the accepted mass with score > tau */
    double ms_score;          /* device time of perturbation + network + keep decision in the stage */
    double ms_tune;           /* device time of the fine-tune after the stage */
    double ms_data;           /* device time of the initial fit's data simulation (ms_train: its training) */
    int64_t train_flops;      /* matrix-product flops of the initial fit (2 per multiply-add, 3 products per
                                 layer and sample: forward, data gradient, weight gradient) */
} abcsmc_surrogate_info;

/* Allocate, fit and switch on the screen for the following stages (scfg may
 * be NULL: all defaults).  Replaces an earlier network. */
int abcsmc_surrogate_enable(abcsmc_ctx* ctx, const abcsmc_surrogate_config* scfg);
/* Free the surrogate state; later stages run plain.  NULL-safe surrogate. */
int abcsmc_surrogate_disable(abcsmc_ctx* ctx);
int abcsmc_surrogate_info_get(const abcsmc_ctx* ctx, abcsmc_surrogate_info* info);
/* Current network, abcsmc_mlp_param_count() floats: W1[256][8] b1[256]
 * W2[256][256] b2[256] W3[256][256] b3[256] W4[3][256] b4[3] (y = W h + b). */
int abcsmc_surrogate_params(const abcsmc_ctx* ctx, float* params);
/* First n rows of the initial fit's data: x n x 8, y n x 3 (either may be NULL). */
int abcsmc_surrogate_data(const abcsmc_ctx* ctx, int64_t n, float* x, float* y);
/* audit[j] = 1 if particle j of the last completed stage was accepted through
 * the audit only (its log-weight carries - log rho), else 0. */
int abcsmc_surrogate_audit(const abcsmc_ctx* ctx, uint8_t* audit);

/* Network test hooks (host buffers, no context; each call allocates device memory). */
int64_t abcsmc_mlp_param_count(void); /* 134659 */
/* The initialisation of abcsmc_surrogate_enable for `seed`. */
int abcsmc_mlp_init(uint64_t seed, float* params);
/* out n x 3 = network(x n x 8); 1 <= n <= 65536. */
int abcsmc_mlp_forward(const float* params, int64_t n, const float* x, float* out);
/* Allocation-free variant of abcsmc_mlp_forward, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  params (abcsmc_mlp_param_count()
 * floats), x (n x 8) and out (n x 3) are DEVICE pointers owned by the
 * caller; 1 <= n <= 65536, else ABCSMC_EINVAL.  The work is enqueued on
 * `stream` (a hipStream_t of the current device; NULL = the null stream) and
 * the call returns without waiting.  The bfloat16 copy of the network that
 * the kernels read is kept in a fixed device array of the library (269,568
 * bytes, one per GPU, held until the process ends; its address is looked up
 * once per device), so the call allocates nothing.  Every call on one GPU
 * shares that array: calls that overlap on one GPU race (order them on one
 * stream).  Results are bit-identical to abcsmc_mlp_forward's. */
int abcsmc_mlp_forward_noalloc(const float* params, int64_t n, const float* x, float* out, void* stream);
/* Gradient of the loss mean over n x 3 of (out - y)^2 with respect to the
 * parameters (same layout), and the loss; 1 <= n <= 65536. */
int abcsmc_mlp_gradients(const float* params, int64_t n, const float* x, const float* y, float* grad,
                         double* loss);
/* epochs passes of minibatch Adam (fresh state) over (x, y) in row order,
 * updating params in place; losses: epochs entries (mean squared error per
 * output over each pass, before each step's update) or NULL. */
int abcsmc_mlp_train(float* params, int64_t n, const float* x, const float* y, int32_t batch, int32_t epochs,
                     double lr, double* losses);

void abcsmc_free(abcsmc_ctx* ctx); /* NULL-safe */
const char* abcsmc_strerror(int code);
const char* abcsmc_last_error(const abcsmc_ctx* ctx); /* NULL ctx: last error of a context-less call */
int abcsmc_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* ABCSMC_H */
