/*
 * abcsmc_demo.c -- the C ABI from plain C99, no Python: synthetic
 * observations of a known parameter vector (one trajectory of the model,
 * §II-B), then an ABC-SMC run with eq. 16 step sizes, printing each stage's
 * tolerance (eq. 8) and proposal count and the importance-weighted mean of
 * the last stage.  Floating-point values are printed exactly (%a).
 *
 *   abcsmc_demo [N] [T] [P] [stages] [seed] [obs_seed]
 *
 * Built by paper_2106_15508_amd/build.py next to the library it links.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "abcsmc.h"

static int check(int rc, const char* what, const abcsmc_ctx* ctx)
{
    if (rc != ABCSMC_OK) {
        fprintf(stderr, "%s: %s (%s)\n", what, abcsmc_strerror(rc), abcsmc_last_error(ctx));
        return 1;
    }
    return 0;
}

int main(int argc, char** argv)
{
    const int64_t N = argc > 1 ? atoll(argv[1]) : 1024;
    const int32_t T = argc > 2 ? atoi(argv[2]) : 50;
    const int64_t P = argc > 3 ? atoll(argv[3]) : 100000;
    const int stages = argc > 4 ? atoi(argv[4]) : 4;
    const uint64_t seed = argc > 5 ? strtoull(argv[5], NULL, 10) : 1;
    const uint64_t obs_seed = argc > 6 ? strtoull(argv[6], NULL, 10) : 210615508;
    /* prior box and generating vector, parameter order of eq. 1 */
    static const double lo[ABCSMC_NPAR] = {0.0, 1.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    static const double hi[ABCSMC_NPAR] = {1.0, 100.0, 1.0, 1.0, 0.5, 0.5, 0.5, 2.0};
    static const double theta_true[ABCSMC_NPAR] = {0.3, 2.0, 0.5, 0.05, 0.1, 0.005, 0.2, 1.0};
    if (N < 2 || T < 1 || P < 1 || stages < 1) {
        fprintf(stderr, "usage: abcsmc_demo [N] [T] [P] [stages] [seed] [obs_seed]\n");
        return 2;
    }

    abcsmc_config c = {0};
    c.abi_version = ABCSMC_ABI_VERSION;
    c.n_params = ABCSMC_NPAR;
    for (int k = 0; k < ABCSMC_NPAR; ++k) {
        c.prior_lo[k] = lo[k];
        c.prior_hi[k] = hi[k];
    }
    c.population = P;
    c.n_days = T;
    c.n_particles = N;
    c.surv_ratio = 0.5;
    c.step_schedule = ABCSMC_STEP_PAPER;
    c.sampler = ABCSMC_SAMPLER_BINOMIAL;
    c.flags = ABCSMC_F_EARLY_EXIT;
    c.seed = seed;

    /* observations: day-0 state (A0, 0, 0) with A0 = max(10, floor(1e-5 P)),
     * then one trajectory of theta_true from the observation stream (round
     * 0xFFFF, distinct from every SMC stage) */
    int64_t a0 = (int64_t)floor(1e-5 * (double)P);
    if (a0 < 10) a0 = 10;
    const int64_t obs0[3] = {a0, 0, 0};
    int64_t* traj = malloc(sizeof(int64_t) * 6 * (size_t)(T + 1));
    int64_t* obs = malloc(sizeof(int64_t) * 3 * (size_t)(T + 1));
    double* theta = malloc(sizeof(double) * ABCSMC_NPAR * (size_t)N);
    double* w = malloc(sizeof(double) * (size_t)N);
    if (!traj || !obs || !theta || !w) return 3;
    if (check(abcsmc_simulate(&c, 1, theta_true, obs0, obs_seed, 0xFFFFu, 0, traj), "abcsmc_simulate", NULL))
        return 1;
    for (int t = 0; t <= T; ++t)
        for (int k = 0; k < 3; ++k) obs[3 * t + k] = traj[6 * t + 2 + k];  /* A, R, D */

    abcsmc_ctx* ctx = NULL;
    if (check(abcsmc_init(&c, obs, &ctx), "abcsmc_init", NULL)) return 1;
    for (int r = 0; r < stages; ++r) {
        abcsmc_round_info info;
        if (check(abcsmc_round(ctx, &info), "abcsmc_round", ctx)) {
            abcsmc_free(ctx);
            return 1;
        }
        printf("stage %d eps %a eps_next %a proposals %lld ess %.3f\n", info.round, info.eps, info.eps_next,
               (long long)info.proposals, info.ess);
    }
    if (check(abcsmc_weights(ctx, theta, NULL, w), "abcsmc_weights", ctx)) {
        abcsmc_free(ctx);
        return 1;
    }
    printf("weighted mean");
    for (int k = 0; k < ABCSMC_NPAR; ++k) {
        double m = 0.0;
        for (int64_t j = 0; j < N; ++j) m += w[j] * theta[j * ABCSMC_NPAR + k];
        printf(" %.6g", m);
    }
    printf("\n");
    abcsmc_free(ctx);
    free(traj);
    free(obs);
    free(theta);
    free(w);
    return 0;
}
