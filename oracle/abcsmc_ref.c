/*
 * abcsmc_ref.c -- CPU ORACLE for P-ABC-SMC with Beta-distributed step sizes
 * (Kulkarni & Moritz, "Efficient State-space Exploration in Massively Parallel
 * Simulation Based Inference", arXiv 2106.15508).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, single-threaded
 * statement of what the GPU path computes.  Only the test-suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it.  It shares no
 * code, header, table or constant with the HIP library: every constant below
 * is written out here from its mathematical definition.
 *
 * Build: gcc -O2 -std=c11 -fPIC -shared -ffp-contract=off -fno-fast-math
 *        (no contraction: every rounding below is the one written).
 *
 * Arithmetic conventions (shared *specification*, not shared code):
 *   - IEEE-754 binary64 with round-to-nearest-even; +,-,*,/,sqrt are the
 *     correctly rounded operations; fma() is used only where written.
 *   - exp/expm1/log/log1p/sin/cos are evaluated by the methods spelled out
 *     below (Cody-Waite reduction plus Taylor series; atanh series), whose
 *     coefficients are the nearest doubles to 1/k! and 1/(2k+1).
 *   - Counts are exact integers (int64 here).
 *
 * Functions whose result has no independent pin are marked "parity unpinned"
 * at their definition.  At present every function is pinned by the tests
 * (library routine, closed form, brute force or invariant).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define REF_NPAR 8

/* ------------------------------------------------------------------ */
/* Counter-based random numbers: Philox4x32-10 (Salmon, Moraes, Dror,  */
/* Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11).        */
/* The paper draws every random quantity from U(0,1) and transforms it  */
/* ("reparameterization", §III-A); a counter-based generator makes the  */
/* draw for (seed, round, particle, purpose, step) a pure function.     */
/* ------------------------------------------------------------------ */

void ref_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { /* Weyl key schedule between rounds */
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Purposes of a draw (third counter word, high byte). */
enum { REF_PRIOR = 1, REF_PERTURB = 2, REF_SIM = 3 };

/* 64-bit word number w of the stream (seed; index, round, purpose, sub):
 * counter = (index, round, purpose<<24 | sub, w/2); word = (x1<<32|x0) for
 * even w and (x3<<32|x2) for odd w. */
uint64_t ref_word(uint64_t seed, uint32_t index, uint32_t round, uint32_t purpose,
                  uint32_t sub, uint32_t w)
{
    uint32_t ctr[4] = { index, round, (purpose << 24) | (sub & 0xFFFFFFu), w / 2u };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint32_t o[4];
    ref_philox4x32_10(ctr, key, o);
    if ((w & 1u) == 0u) return ((uint64_t)o[1] << 32) | o[0];
    return ((uint64_t)o[3] << 32) | o[2];
}

/* Uniform on the open interval (0,1) with 52 random bits:
 * ((w >> 12) + 1/2) * 2^-52.  Exact; 1-u is exact too. */
double ref_u01(uint64_t w)
{
    double m = (double)(w >> 12);
    return (m + 0.5) * 0x1p-52;
}

/* ------------------------------------------------------------------ */
/* Elementary functions, from their series (no libm transcendental).   */
/* ------------------------------------------------------------------ */

/* ln 2 split: LN2_HI = ln 2 truncated to 32 significant bits (so k*LN2_HI
 * is exact for |k| < 2^21), LN2_LO = nearest double to ln 2 - LN2_HI. */
static const double LN2_HI = 0x1.62e42feep-1;
static const double LN2_LO = 0x1.a39ef35793c76p-33;
static const double LOG2E = 1.4426950408889634;   /* nearest double to 1/ln 2 */
static const double SQRT1_2 = 0.70710678118654757; /* nearest double to 1/sqrt 2 */
static const double PI_2 = 1.5707963267948966;     /* nearest double to pi/2 */
static const double SQRT1_2_M1 = -0.2928932188134524; /* SQRT1_2 - 1, exact (Sterbenz) */

/* nearest double to 1/k!, k = 0..18: each a correctly rounded quotient of
 * two exact doubles (k! < 2^53 for k <= 18), evaluated by the compiler */
static const double INV_FACT[19] = {
    1.0 / 1.0,
    1.0 / 1.0,
    1.0 / 2.0,
    1.0 / 6.0,
    1.0 / 24.0,
    1.0 / 120.0,
    1.0 / 720.0,
    1.0 / 5040.0,
    1.0 / 40320.0,
    1.0 / 362880.0,
    1.0 / 3628800.0,
    1.0 / 39916800.0,
    1.0 / 479001600.0,
    1.0 / 6227020800.0,
    1.0 / 87178291200.0,
    1.0 / 1307674368000.0,
    1.0 / 20922789888000.0,
    1.0 / 355687428096000.0,
    1.0 / 6402373705728000.0
};
static double inv_fact(int k) { return INV_FACT[k]; }

/* exp(x): k = rint(x/ln2), r = x - k ln2 (two-part, Cody & Waite),
 * exp(r) = sum_{i=0}^{13} r^i/i! by Horner with fma, result 2^k exp(r).
 * Results below e^-708 are returned as 0 (no subnormal outputs);
 * x > 709.782712893384 gives +inf. */
double ref_exp(double x)
{
    if (x != x) return x;
    if (x > 709.782712893384) return INFINITY;
    if (x < -708.0) return 0.0;
    double k = rint(x * LOG2E);
    double t = x - k * LN2_HI;            /* exact */
    double r = fma(-k, LN2_LO, t);
    double p = inv_fact(13);
    for (int i = 12; i >= 0; --i) p = fma(p, r, inv_fact(i));
    return ldexp(p, (int)k);
}

/* nearest doubles to 1/(2j+1), j = 0..11 (correctly rounded quotients,
 * evaluated by the compiler) */
static const double INV_ODD[12] = {
    1.0 / 1.0,
    1.0 / 3.0,
    1.0 / 5.0,
    1.0 / 7.0,
    1.0 / 9.0,
    1.0 / 11.0,
    1.0 / 13.0,
    1.0 / 15.0,
    1.0 / 17.0,
    1.0 / 19.0,
    1.0 / 21.0,
    1.0 / 23.0
};

/* atanh series tail: R(z) = z/3 + z^2/5 + ... + z^11/23, z = s^2, so that
 * 2 atanh(s) = 2 (s + s R(z)). */
static double atanh_tail(double z)
{
    double q = INV_ODD[11];
    for (int j = 10; j >= 1; --j) q = fma(q, z, INV_ODD[j]);
    return z * q;
}

/* log(x), x > 0 finite: x = f 2^e with f in [1/sqrt2, sqrt2); with a = f-1
 * (exact) and s = a/(2+a): log f = 2 atanh(s).  log x = e ln2 + log f. */
double ref_log(double x)
{
    if (x != x) return x;
    if (x < 0.0) return NAN;
    if (x == 0.0) return -INFINITY;
    if (x == INFINITY) return INFINITY;
    int e;
    double f = frexp(x, &e); /* f in [0.5, 1) */
    if (f < SQRT1_2) { f = f * 2.0; e = e - 1; }
    double a = f - 1.0;
    double s = a / (2.0 + a);
    double R = atanh_tail(s * s);
    double lf = 2.0 * (s + s * R);
    double de = (double)e;
    return de * LN2_HI + (de * LN2_LO + lf);
}

/* log1p(x), x > -1: in [1/sqrt2 - 1, sqrt2 - 1] the identity
 * log(1+x) = 2 atanh(x/(2+x)); elsewhere log(u) + (x - (u-1))/u, u = 1+x,
 * where x - (u-1) is the exact rounding error of 1+x. */
double ref_log1p(double x)
{
    if (x != x) return x;
    if (x == -1.0) return -INFINITY;
    if (x < -1.0) return NAN;
    if (x >= SQRT1_2_M1 && x <= 0.41421356237309515) {
        double s = x / (2.0 + x);
        double R = atanh_tail(s * s);
        return 2.0 * (s + s * R);
    }
    double u = 1.0 + x;
    return ref_log(u) + (x - (u - 1.0)) / u;
}

/* expm1(x): for |x| <= ln2/2 the Taylor series x + x^2 (1/2! + x/3! + ... +
 * x^12/14!); otherwise exp(x) - 1. */
double ref_expm1(double x)
{
    if (x != x) return x;
    if (fabs(x) <= 0.34657359027997264) {
        double p = inv_fact(14);
        for (int i = 13; i >= 2; --i) p = fma(p, x, inv_fact(i));
        return fma(x * x, p, x);
    }
    return ref_exp(x) - 1.0;
}

/* cos(2 pi t), sin(2 pi t) for t in [0,1): quadrant q = floor(4t),
 * f = 4t - q (both exact), fold f > 1/2 to 1-f, y = (pi/2) g in [0, pi/4],
 * Taylor series sin y = y sum (-1)^i y^2i/(2i+1)!  (i <= 8) and
 * cos y = sum (-1)^i y^2i/(2i)!  (i <= 9). */
void ref_sincos2pi(double t, double* c_out, double* s_out)
{
    double t4 = t * 4.0;
    double q = floor(t4);
    double f = t4 - q;
    int fold = f > 0.5;
    double g = fold ? 1.0 - f : f;
    double y = g * PI_2;
    double y2 = y * y;
    double ps = inv_fact(17);
    for (int i = 7; i >= 0; --i) ps = fma(ps, -y2, inv_fact(2 * i + 1));
    double sy = y * ps;
    double pc = inv_fact(18);
    for (int i = 8; i >= 0; --i) pc = fma(pc, -y2, inv_fact(2 * i));
    double cy = pc;
    double cf = fold ? sy : cy; /* cos(pi f / 2) */
    double sf = fold ? cy : sy; /* sin(pi f / 2) */
    int iq = (int)q;
    double c, s;
    if (iq == 0)      { c = cf;  s = sf;  }
    else if (iq == 1) { c = -sf; s = cf;  }
    else if (iq == 2) { c = -cf; s = -sf; }
    else              { c = sf;  s = -cf; }
    *c_out = c;
    *s_out = s;
}

/* Box & Muller (1958) pair from one 64-bit word: u1 from the low 32 bits,
 * u2 from the high 32 bits, both ((h + 1/2) 2^-32); rho = sqrt(-2 log u1);
 * z0 = rho cos(2 pi u2), z1 = rho sin(2 pi u2). */
void ref_box_muller(uint64_t w, double* z0, double* z1)
{
    double u1 = ((double)(uint32_t)w + 0.5) * 0x1p-32;
    double u2 = ((double)(uint32_t)(w >> 32) + 0.5) * 0x1p-32;
    double rho = sqrt(-2.0 * ref_log(u1));
    double c, s;
    ref_sincos2pi(u2, &c, &s);
    *z0 = rho * c;
    *z1 = rho * s;
}

/* ------------------------------------------------------------------ */
/* Binomial draw with one random word.                                 */
/* The model's transitions (§II-B, eq. 5) are Poisson tau-leap counts;  */
/* here each is drawn as Bin(n, p), p = 1 - exp(-rate), from the count  */
/* it leaves (so no compartment goes negative).                         */
/* ------------------------------------------------------------------ */
#define REF_T_SWITCH 10.0
#define REF_BINV_CAP 128

/* 1/j for j = 1..REF_BINV_CAP, each the correctly rounded double */
static double binv_recip(int64_t j)
{
    static double tab[REF_BINV_CAP + 1];
    static int ready = 0;
    if (!ready) {
        for (int i = 1; i <= REF_BINV_CAP; ++i) tab[i] = 1.0 / (double)i;
        ready = 1;
    }
    return tab[j];
}

/* Bin(n, p) with the inversion uniform from word wu and, in the normal
 * branch, the deviate from the Box-Muller pair of word wz (half 0: the
 * cosine deviate, half 1: the sine deviate). */
static int64_t binomial_core(int64_t n, double p, uint64_t wu, uint64_t wz, int half)
{
    if (n <= 0 || p <= 0.0) return 0;
    if (p >= 1.0) return n;
    int flip = p > 0.5;
    double q = flip ? 1.0 - p : p;
    double dn = (double)n;
    double m = dn * q;
    int64_t x;
    if (m < REF_T_SWITCH) {
        /* inversion by sequential search (BINV): F(k) accumulates the pmf,
         * f(k+1) = f(k) (n - k) r / (k + 1) with the division taken as a
         * product with the rounded reciprocal 1/(k+1) */
        double u = ref_u01(wu);
        double f = ref_exp(dn * ref_log1p(-q));
        double F = f;
        double r = q / (1.0 - q);
        int64_t k = 0;
        while (u > F && k < n && k < REF_BINV_CAP) {
            f = f * (((double)(n - k) * r) * binv_recip(k + 1));
            k = k + 1;
            F = F + f;
        }
        x = k;
    } else {
        /* normal approximation with continuity correction */
        double z0, z1;
        ref_box_muller(wz, &z0, &z1);
        double z = half ? z1 : z0;
        double sd = sqrt(m * (1.0 - q));
        double y = (m + 0.5) + sd * z;
        double fl = floor(y);
        if (fl < 0.0) fl = 0.0;
        if (fl > dn) fl = dn;
        x = (int64_t)fl;
    }
    return flip ? n - x : x;
}

/* One draw from one word: the uniform and the cosine deviate of the same word. */
int64_t ref_binomial(int64_t n, double p, uint64_t w)
{
    return binomial_core(n, p, w, w, 0);
}

/* The paper's own transition sampler (§II-B): floor of a normal with mean
 * h and spread sqrt(h) (read as standard deviation sqrt(h), matching the
 * Poisson it approximates), clamped to [0, n] so the source compartment
 * cannot go negative.  Uses the Box-Muller cosine of the draw's word. */
int64_t ref_normal_floor(int64_t n, double h, uint64_t w)
{
    if (n <= 0 || !(h > 0.0)) return 0;
    double z, z_unused;
    ref_box_muller(w, &z, &z_unused);
    double y = h + sqrt(h) * z;
    double fl = floor(y);
    if (fl < 0.0) fl = 0.0;
    if (fl > (double)n) fl = (double)n;
    return (int64_t)fl;
}

/* ------------------------------------------------------------------ */
/* Beta(a, b) for integer b >= 1 (step-size law of eq. 16):            */
/* Beta(a,b) = prod_{m=0}^{b-1} Beta(a+m, 1), each factor U^(1/(a+m))   */
/* by inversion, so s = exp( sum_m log(U_m) / (a+m) ), summed in m order.*/
/* ------------------------------------------------------------------ */
double ref_beta_int(double a, int b, const uint64_t* words)
{
    double L = 0.0;
    for (int m = 0; m < b; ++m) L = L + ref_log(ref_u01(words[m])) / (a + (double)m);
    return ref_exp(L);
}

/* Gamma(k) by Marsaglia & Tsang (ACM TOMS 2000): for k >= 1, d = k - 1/3,
 * c = 1/sqrt(9 d); iteration m takes z from word w0 + 2m (first Box-Muller
 * normal) and U from word w0 + 2m + 1; v = (1 + c z)^3; accept d v when
 * v > 0 and log U < z^2/2 + d - d v + d log v.  After 32 rejections (chance
 * below 1e-40) the value is d.  For k < 1: Gamma(k + 1) U^(1/k) with U from
 * word w0 + 64.  Words are those of stream (seed, index, round, PERTURB,
 * sub). */
double ref_gamma_mt(double k, uint64_t seed, uint32_t index, uint32_t round, uint32_t sub, uint32_t w0)
{
    const double kk = k < 1.0 ? k + 1.0 : k;
    const double d = kk - 1.0 / 3.0;
    const double c = 1.0 / sqrt(9.0 * d);
    double g = d;
    for (uint32_t m = 0; m < 32; ++m) {
        double z, z_unused;
        ref_box_muller(ref_word(seed, index, round, REF_PERTURB, sub, w0 + 2 * m), &z, &z_unused);
        const double t = 1.0 + c * z;
        if (!(t > 0.0)) continue;
        const double v = t * t * t;
        const double U = ref_u01(ref_word(seed, index, round, REF_PERTURB, sub, w0 + 2 * m + 1));
        if (ref_log(U) < 0.5 * (z * z) + d - d * v + d * ref_log(v)) {
            g = d * v;
            break;
        }
    }
    if (k < 1.0) g = g * ref_exp(ref_log(ref_u01(ref_word(seed, index, round, REF_PERTURB, sub, w0 + 64))) / k);
    return g;
}

/* Beta(a, b) for real shapes: X / (X + Y) with X ~ Gamma(a) from words 5..,
 * Y ~ Gamma(b) from words 70.. of the attempt's stream; 0 if both vanish. */
double ref_beta_general(double a, double b, uint64_t seed, uint32_t index, uint32_t round, uint32_t sub)
{
    const double X = ref_gamma_mt(a, seed, index, round, sub, 5);
    const double Y = ref_gamma_mt(b, seed, index, round, sub, 70);
    const double s = X + Y;
    return s > 0.0 ? X / s : 0.0;
}

/* ------------------------------------------------------------------ */
/* Stochastic epidemic model (§II-B, eqs. 1-5)                          */
/* ------------------------------------------------------------------ */
typedef struct {
    double lo[REF_NPAR], hi[REF_NPAR]; /* prior box, paper order (eq. 1) */
    int64_t population;                /* P */
    int32_t n_days;                    /* T */
    int64_t n_particles;               /* N accepted per round */
    double surv_ratio;                 /* alpha of eq. 8 */
    int32_t step_schedule;             /* 0: eq. 16, 1: fixed Beta(beta_a, beta_b), 2: MCMC-tuned s (eqs. 12-15) */
    double beta_a;
    int32_t beta_b;
    int32_t step_is_variance;          /* eq. 12 calls s a variance: sigma = sqrt(s) */
    int32_t sampler;                   /* 0: chain binomial, 1: floor-normal of §II-B */
    int32_t max_attempts;              /* perturbation redraws before a proposal is void */
    uint64_t seed;
    int64_t max_proposals;             /* per-round budget */
    int64_t batch;                     /* simulations per run (schedule 2: one s per batch) */
    double mcmc_s0;                    /* schedule 2: initial step size s */
    int32_t mcmc_tune;                 /* schedule 2: batches of stages >= 1 after which s is adapted */
    double beta_b_real;                /* schedules 3, 4: the stage's real Beta shape b (set by ref_run) */
    int32_t n_eps_schedule;            /* stages 1..n accept against eps_schedule[i-1] instead of */
    const double* eps_schedule;        /* eq. 8's percentile of stage i-1 (a replayed schedule) */
} ref_config;

enum { REF_S = 0, REF_I, REF_A, REF_R, REF_D, REF_RU };

/* Forward simulation of one parameter vector theta = [alpha0, alpha, n,
 * beta, gamma, delta, eta, kappa] (eq. 1) for T days.  obs0 = (A0, R0, D0)
 * is day 0 of the observed series.  traj receives (T+1) x 6 counts
 * [S, I, A, R, D, Ru] (eq. 3).  Step 1 (initialisation): Ru = 0,
 * I0 = floor(kappa A0) (capped so S >= 0), S = P - (A0+R0+D0+I0).  Steps
 * 2-4 per day: hazards h of eq. 5 with g of eq. 4 from start-of-day state;
 * transitions drawn in h order S->I, I->A, A->R, A->D, I->Ru, each from
 * what is left of its source compartment; apply. */
void ref_simulate(const ref_config* cfg, const double theta[REF_NPAR], const int64_t obs0[3],
                  uint64_t seed, uint32_t round, uint32_t index, int64_t* traj)
{
    const double alpha0 = theta[0], alpha_c = theta[1], n_exp = theta[2], beta = theta[3];
    const double gamma = theta[4], delta = theta[5], eta = theta[6], kappa = theta[7];
    const int64_t P = cfg->population;
    int64_t A = obs0[0], R = obs0[1], D = obs0[2];
    int64_t I = (int64_t)floor(kappa * (double)A);
    int64_t room = P - (A + R + D);
    if (I > room) I = room;
    if (I < 0) I = 0;
    int64_t S = P - (A + R + D + I);
    int64_t Ru = 0;
    const double invP = 1.0 / (double)P;
    double pIA = 0, pAR = 0, pAD = 0, pIRu = 0;
    if (cfg->sampler == 0) {
        pIA = -ref_expm1(-gamma);
        pAR = -ref_expm1(-beta);
        pAD = -ref_expm1(-delta);
        pIRu = -ref_expm1(-(beta * eta));
    }
    int64_t* row = traj;
    row[REF_S] = S; row[REF_I] = I; row[REF_A] = A; row[REF_R] = R; row[REF_D] = D; row[REF_RU] = Ru;
    for (int32_t t = 0; t < cfg->n_days; ++t) {
        /* eq. 4: g = alpha0 + alpha / (1 + (A+R+D)^n) */
        double C = (double)(A + R + D);
        double pw;
        if (C == 0.0) pw = (n_exp == 0.0) ? 1.0 : 0.0;
        else pw = ref_exp(n_exp * ref_log(C));
        double g = alpha0 + alpha_c / (1.0 + pw);
        double rate_si = (g * (double)I) * invP; /* per-susceptible rate g I / P */
        /* draw k: inversion uniform from word k; normal deviates in Box-Muller
         * pairs: draws 0, 1 from word 5, draws 2, 3 from word 6, draw 4 from
         * word 7 (the floor-normal sampler: the cosine deviate of word k) */
        uint64_t w[8];
        for (uint32_t k = 0; k < 8; ++k) w[k] = ref_word(seed, index, round, REF_SIM, (uint32_t)t, k);
        int64_t n1, n2, n3, n4, n5;
        if (cfg->sampler == 0) {
            double pSI = -ref_expm1(-rate_si);
            n1 = binomial_core(S, pSI, w[0], w[5], 0);
            n2 = binomial_core(I, pIA, w[1], w[5], 1);
            n3 = binomial_core(A, pAR, w[2], w[6], 0);
            n4 = binomial_core(A - n3, pAD, w[3], w[6], 1);
            n5 = binomial_core(I - n2, pIRu, w[4], w[7], 0);
        } else {
            /* eq. 5 hazards h = (g S I/P, gamma I, beta A, delta A, beta eta I) */
            n1 = ref_normal_floor(S, rate_si * (double)S, w[0]);
            n2 = ref_normal_floor(I, gamma * (double)I, w[1]);
            n3 = ref_normal_floor(A, beta * (double)A, w[2]);
            n4 = ref_normal_floor(A - n3, delta * (double)A, w[3]);
            n5 = ref_normal_floor(I - n2, (beta * eta) * (double)I, w[4]);
        }
        S = S - n1;
        I = I + n1 - n2 - n5;
        A = A + n2 - n3 - n4;
        R = R + n3;
        D = D + n4;
        Ru = Ru + n5;
        row = traj + (size_t)(t + 1) * 6;
        row[REF_S] = S; row[REF_I] = I; row[REF_A] = A; row[REF_R] = R; row[REF_D] = D; row[REF_RU] = Ru;
    }
}

/* Euclidean distance between simulated and observed (A, R, D) over days
 * 1..T (§II-C).  Sum in day order, A then R then D, each term the square of
 * an exact integer difference; d = sqrt(sum). */
double ref_distance(int32_t T, const int64_t* traj, const int64_t* obs)
{
    double acc = 0.0;
    for (int32_t t = 1; t <= T; ++t) {
        const int64_t* s = traj + (size_t)t * 6;
        const int64_t* o = obs + (size_t)t * 3;
        double dA = (double)(s[REF_A] - o[0]);
        double dR = (double)(s[REF_R] - o[1]);
        double dD = (double)(s[REF_D] - o[2]);
        acc = acc + dA * dA;
        acc = acc + dR * dR;
        acc = acc + dD * dD;
    }
    return sqrt(acc);
}

/* ------------------------------------------------------------------ */
/* SMC stage machinery (§II-D)                                          */
/* ------------------------------------------------------------------ */

static int cmp_double(const void* a, const void* b)
{
    double x = *(const double*)a, y = *(const double*)b;
    return (x > y) - (x < y);
}

/* eq. 8: the alpha-percentile of the accepted distances, with linear
 * interpolation between order statistics (Hyndman & Fan type 7), in the
 * arithmetic numpy uses for method "linear": virtual index v = (n-1) a,
 * g = v - floor(v), lerp a + (b-a) g, or b - (b-a)(1-g) when g >= 1/2. */
double ref_quantile(const double* x, int64_t n, double alpha)
{
    double* s = (double*)malloc((size_t)n * sizeof(double));
    memcpy(s, x, (size_t)n * sizeof(double));
    qsort(s, (size_t)n, sizeof(double), cmp_double);
    double dn = (double)n;
    double v = (dn - 1.0) * alpha;
    double res;
    if (v >= dn - 1.0) res = s[n - 1];
    else if (v < 0.0) res = s[0];
    else {
        double fl = floor(v);
        int64_t i = (int64_t)fl;
        double g = v - fl;
        double a = s[i], b = s[i + 1];
        double diff = b - a;
        if (g >= 0.5) res = b - diff * (1.0 - g);
        else res = a + diff * g;
    }
    free(s);
    return res;
}

/* eqs. 9-10: prior set of stage i = previous particles with d < eps
 * (if none, d <= eps), weight eps - d.  The categorical law of eq. 11 is
 * realised on integers: q_k = floor((w_k / w_max) 2^40), C = inclusive
 * prefix sum of q (exact in uint64).  Particles outside the set get q = 0.
 * If every survivor has w = 0 the survivors are weighted equally (q = 1).
 * Returns the number of survivors. */
int64_t ref_resample_weights(const double* d, int64_t n, double eps, uint64_t* q, uint64_t* C)
{
    int64_t nsurv = 0;
    for (int64_t k = 0; k < n; ++k) nsurv += (d[k] < eps);
    int strict = nsurv > 0;
    if (!strict) {
        for (int64_t k = 0; k < n; ++k) nsurv += (d[k] <= eps);
    }
    double wmax = 0.0;
    for (int64_t k = 0; k < n; ++k) {
        int in = strict ? (d[k] < eps) : (d[k] <= eps);
        if (in) {
            double w = eps - d[k];
            if (w > wmax) wmax = w;
        }
    }
    uint64_t run = 0;
    for (int64_t k = 0; k < n; ++k) {
        int in = strict ? (d[k] < eps) : (d[k] <= eps);
        uint64_t qk = 0;
        if (in) {
            if (wmax > 0.0) qk = (uint64_t)floor(((eps - d[k]) / wmax) * 0x1p40);
            else qk = 1;
        }
        q[k] = qk;
        run += qk;
        C[k] = run;
    }
    return nsurv;
}

/* eq. 11 categorical draw from one 64-bit word R: r = floor(R Q / 2^64),
 * parent = first k with C[k] > r. */
int64_t ref_parent(const uint64_t* C, int64_t n, uint64_t R)
{
    uint64_t Q = C[n - 1];
    uint64_t r = (uint64_t)(((unsigned __int128)R * (unsigned __int128)Q) >> 64);
    int64_t lo = 0, hi = n - 1; /* C[hi] = Q > r */
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (C[mid] > r) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

/* eq. 16 step-size law for stage i >= 1: Beta(eps_i/eps_1, 2i); or a fixed
 * Beta(a, b). */
/* Alternative parameterisations of the step-size Beta (§III-B, stated
 * without formulas): the two tuned quantities of eq. 16 -- the tolerance
 * ratio r = eps_i / eps_1 and the stage i -- set
 *   schedule 3, mean-variance: mean mu = r / 3 (at least 1e-12), variance mu (1 - mu) / (3 i + 1)
 *     -> a = mu k, b = (1 - mu) k with k = mu (1 - mu) / variance - 1 = 3 i
 *   schedule 4, mode-concentration: mode w = r / 4, concentration k = 2 i + 2
 *     -> a = w (k - 2) + 1, b = (1 - w) (k - 2) + 1
 * (both give the stage-1 shape a mean near that of eq. 16's Beta(1, 2)). */
void ref_beta_shape_real(const ref_config* cfg, int32_t round, double eps_i, double eps_1, double* a, double* b)
{
    const double r = eps_i / eps_1;
    if (cfg->step_schedule == 3) {
        double mu = r / 3.0;
        if (mu < 1e-12) mu = 1e-12; /* a stage with eps_i = 0 */
        const double var = mu * (1.0 - mu) / (3.0 * (double)round + 1.0);
        const double k = mu * (1.0 - mu) / var - 1.0;
        *a = mu * k;
        *b = (1.0 - mu) * k;
    } else {
        const double w = r / 4.0;
        const double k = 2.0 * (double)round + 2.0;
        *a = w * (k - 2.0) + 1.0;
        *b = (1.0 - w) * (k - 2.0) + 1.0;
    }
}

void ref_beta_shape(const ref_config* cfg, int32_t round, double eps_i, double eps_1,
                    double* a, int32_t* b)
{
    if (cfg->step_schedule == 2) { /* no Beta: the MCMC variant's s is carried separately */
        *a = 0.0;
        *b = 0;
    } else if (cfg->step_schedule == 1) {
        *a = cfg->beta_a;
        *b = cfg->beta_b;
    } else {
        *a = eps_i / eps_1;
        *b = 2 * round;
    }
}

/* One proposal of stage i >= 1 (eqs. 11, 16, 17 in the unit cube of the
 * reparameterisation, §III-A): for attempt = 0, 1, ...: parent k from the
 * categorical law, s ~ Beta(a, b), sigma = s (or sqrt(s) when s is read as a
 * variance) floored at 1e-8, z ~ N(0, I_8), u = u_k + sigma z; stop at the
 * first u inside [0,1]^8.  Returns the number of attempts used, or
 * -attempts if none landed inside (a void proposal). */
int32_t ref_perturb(const ref_config* cfg, uint32_t round, uint32_t index, const double* u_prev,
                    const uint64_t* C, int64_t n_prev, double beta_a, int32_t beta_b,
                    double u_out[REF_NPAR], double* sigma_out, int64_t* parent_out)
{
    uint64_t words[5 + 128];
    const int fixed_s = cfg->step_schedule == 2; /* MCMC variant: s = beta_a, no Beta words */
    const int general = cfg->step_schedule >= 3; /* real shapes: beta_a and beta_b_real */
    for (int32_t att = 0; att < cfg->max_attempts; ++att) {
        int nw = 5 + ((fixed_s || general) ? 0 : beta_b);
        for (int k = 0; k < nw; ++k)
            words[k] = ref_word(cfg->seed, index, round, REF_PERTURB, (uint32_t)att, (uint32_t)k);
        int64_t parent = ref_parent(C, n_prev, words[0]);
        double s = fixed_s ? beta_a
                 : general ? ref_beta_general(beta_a, cfg->beta_b_real, cfg->seed, index, round, (uint32_t)att)
                           : ref_beta_int(beta_a, beta_b, words + 5);
        double sigma = cfg->step_is_variance ? sqrt(s) : s;
        if (sigma < 1e-8) sigma = 1e-8;
        double z[REF_NPAR];
        for (int p = 0; p < 4; ++p) ref_box_muller(words[1 + p], &z[2 * p], &z[2 * p + 1]);
        int inside = 1;
        for (int d = 0; d < REF_NPAR; ++d) {
            double v = u_prev[(size_t)parent * REF_NPAR + d] + sigma * z[d];
            u_out[d] = v;
            if (!(v >= 0.0 && v <= 1.0)) inside = 0;
        }
        *sigma_out = sigma;
        *parent_out = parent;
        if (inside) return att + 1;
    }
    return -cfg->max_attempts;
}

/* Prior draw for stage 0: u ~ U(0,1)^8 (reparameterised uniform prior of
 * eq. 2). */
void ref_prior_draw(const ref_config* cfg, uint32_t index, double u_out[REF_NPAR])
{
    for (uint32_t d = 0; d < REF_NPAR; ++d) u_out[d] = ref_u01(ref_word(cfg->seed, index, 0, REF_PRIOR, 0, d));
}

/* theta_d = lo_d + u_d (hi_d - lo_d) */
void ref_to_theta(const ref_config* cfg, const double u[REF_NPAR], double theta[REF_NPAR])
{
    for (int d = 0; d < REF_NPAR; ++d) theta[d] = cfg->lo[d] + u[d] * (cfg->hi[d] - cfg->lo[d]);
}

/* Simulate the proposal with unit-cube coordinates u; return its distance. */
double ref_sim_distance(const ref_config* cfg, const int64_t* obs, const double u[REF_NPAR],
                        uint32_t round, uint32_t index, int64_t* traj_scratch)
{
    double theta[REF_NPAR];
    ref_to_theta(cfg, u, theta);
    ref_simulate(cfg, theta, obs, cfg->seed, round, index, traj_scratch);
    return ref_distance(cfg->n_days, traj_scratch, obs);
}

/* Importance weight row sum of particle j against the stage's proposal
 * mixture: L_j = sum_k q_k exp(-|u_j - u_k|^2 / (2 sigma_j^2)) over the
 * previous particles with q_k > 0, summed with Neumaier compensation.
 * log-weight l_j = 8 log sigma_j - log L_j (the Gaussian normaliser and the
 * total Q are constants that cancel on normalisation). */
double ref_log_weight(const double u_j[REF_NPAR], double sigma_j, const double* u_prev,
                      const uint64_t* q, int64_t n_prev)
{
    double sum = 0.0, comp = 0.0;
    double two_s2 = 2.0 * (sigma_j * sigma_j);
    for (int64_t k = 0; k < n_prev; ++k) {
        if (q[k] == 0) continue;
        double D = 0.0;
        for (int d = 0; d < REF_NPAR; ++d) {
            double diff = u_j[d] - u_prev[(size_t)k * REF_NPAR + d];
            D = D + diff * diff;
        }
        double term = (double)q[k] * ref_exp(-(D / two_s2));
        double t = sum + term;
        if (fabs(sum) >= fabs(term)) comp += (sum - t) + term;
        else comp += (term - t) + sum;
        sum = t;
    }
    double L = sum + comp;
    return 8.0 * ref_log(sigma_j) - ref_log(L);
}

/* Normalise log-weights: W_j = exp(l_j - max l) / sum; returns ESS = 1/sum W^2. */
double ref_normalise(const double* l, int64_t n, double* W)
{
    double mx = -INFINITY;
    for (int64_t j = 0; j < n; ++j) if (l[j] > mx) mx = l[j];
    double sum = 0.0, comp = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        W[j] = ref_exp(l[j] - mx);
        double t = sum + W[j];
        if (fabs(sum) >= fabs(W[j])) comp += (sum - t) + W[j];
        else comp += (W[j] - t) + sum;
        sum = t;
    }
    sum = sum + comp;
    double s2 = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        W[j] = W[j] / sum;
        s2 += W[j] * W[j];
    }
    return 1.0 / s2;
}

/* ------------------------------------------------------------------ */
/* MCMC variant (§II-D, eqs. 12-15): after a batch ("run") of proposals
 * with acc of its valid proposals accepted (eq. 14, A = acc / valid), the
 * step size moves toward the target acceptance A_T = 0.234 by
 *   s_new = s_old (1 + (A - A_T) / ((1 - A_T) (n_acc + 1)))
 * where n_acc counts every acceptance of the tuned batches so far, this one
 * included.  (Eq. 15 as printed multiplies s by (A - A_T) itself, which turns
 * s negative whenever A < A_T; the relative-change reading keeps its sign
 * and its 1 / (n_acc + 1) gain.) */
double ref_mcmc_update(double s, int64_t acc, int64_t valid, int64_t n_acc)
{
    const double A_T = 0.234;
    const double A = valid > 0 ? (double)acc / (double)valid : 0.0;
    return s * (1.0 + (A - A_T) / ((1.0 - A_T) * ((double)n_acc + 1.0)));
}

/* Whole run: stage 0 (ABC with eps^0 = +inf, §II-D) then stages        */
/* 1..R-1 (eqs. 8-11, 16-17).                                           */
/* ------------------------------------------------------------------ */
typedef struct {
    /* per round r (arrays of n_rounds * N or n_rounds) */
    double* u;        /* N x 8 unit-cube coordinates of the accepted particles */
    double* dist;     /* N */
    double* sigma;    /* N (0 in stage 0) */
    int64_t* parent;  /* N (-1 in stage 0) */
    int64_t* index;   /* N proposal index j */
    int32_t* attempts;/* N attempts used */
    double* logw;     /* N unnormalised log-weight (0 in stage 0) */
    double* W;        /* N normalised weight */
    double* eps;      /* tolerance eps^r used by stage r (inf for r = 0) */
    double* eps_next; /* eps^{r+1} */
    double* beta_a;   /* Beta shape used by stage r (0 for r = 0) */
    int32_t* beta_b;
    int64_t* proposals; /* proposals examined: index of the N-th acceptance + 1 */
    int64_t* invalid;   /* void proposals among them */
    int64_t* attempts_total;
    double* ess;
    double* mcmc_s;   /* schedule 2: step size after stage r (its starting value for stage 0) */
    double* beta_b_real; /* Beta shape b of stage r as a real number (schedules 3, 4: not an integer) */
    int64_t* simulated; /* proposals simulated: whole batches for schedule 2, else = proposals */
} ref_result;

/* Returns 0 on success, -4 if a round exhausted max_proposals (result
 * holds the completed rounds), -1 on bad arguments. */
int ref_run(const ref_config* cfg, const int64_t* obs, int32_t n_rounds, ref_result* out)
{
    const int64_t N = cfg->n_particles;
    const int32_t T = cfg->n_days;
    if (N < 2 || T < 1 || n_rounds < 1) return -1;
    int64_t* traj = (int64_t*)malloc((size_t)(T + 1) * 6 * sizeof(int64_t));
    uint64_t* q = (uint64_t*)malloc((size_t)N * sizeof(uint64_t));
    uint64_t* C = (uint64_t*)malloc((size_t)N * sizeof(uint64_t));
    int rc = 0;
    double eps1 = INFINITY;
    ref_config stage_cfg = *cfg;   /* schedules 3, 4: carries the stage's real shape b */
    double s_mcmc = cfg->mcmc_s0;  /* schedule 2 state, carried across stages */
    int32_t tunes = 0;
    int64_t n_acc = 0;
    for (int32_t r = 0; r < n_rounds; ++r) {
        double* u = out->u + (size_t)r * N * REF_NPAR;
        double* dist = out->dist + (size_t)r * N;
        double* sig = out->sigma + (size_t)r * N;
        int64_t* par = out->parent + (size_t)r * N;
        int64_t* idx = out->index + (size_t)r * N;
        int32_t* att = out->attempts + (size_t)r * N;
        double* lw = out->logw + (size_t)r * N;
        double* W = out->W + (size_t)r * N;
        int64_t accepted = 0, j = 0, invalid = 0, att_total = 0;
        if (r == 0) {
            out->eps[0] = INFINITY;
            out->beta_a[0] = 0.0;
            out->beta_b[0] = 0;
            for (j = 0; j < N; ++j) {
                double uj[REF_NPAR];
                ref_prior_draw(cfg, (uint32_t)j, uj);
                double d = ref_sim_distance(cfg, obs, uj, 0, (uint32_t)j, traj);
                memcpy(u + (size_t)j * REF_NPAR, uj, sizeof uj);
                dist[j] = d; sig[j] = 0.0; par[j] = -1; idx[j] = j; att[j] = 1;
                lw[j] = 0.0; W[j] = 1.0 / (double)N;
                ++att_total;
            }
            accepted = N;
        } else {
            const double* u_prev = out->u + (size_t)(r - 1) * N * REF_NPAR;
            const double* d_prev = out->dist + (size_t)(r - 1) * N;
            double eps = r <= cfg->n_eps_schedule ? cfg->eps_schedule[r - 1] : out->eps_next[r - 1];
            out->eps[r] = eps;
            if (r == 1) eps1 = eps;
            double ba; int32_t bb;
            ref_beta_shape(cfg, r, eps, eps1, &ba, &bb);
            if (cfg->step_schedule >= 3) {
                ref_beta_shape_real(cfg, r, eps, eps1, &ba, &stage_cfg.beta_b_real);
                bb = 0;
            }
            out->beta_a[r] = ba;
            out->beta_b[r] = bb;
            out->beta_b_real[r] = cfg->step_schedule >= 3 ? stage_cfg.beta_b_real : (double)bb;
            ref_resample_weights(d_prev, N, eps, q, C);
            if (cfg->step_schedule != 2) {
                while (accepted < N) {
                    if (j >= cfg->max_proposals) { rc = -4; break; }
                    double uj[REF_NPAR], s; int64_t parent;
                    int32_t a = ref_perturb(&stage_cfg, (uint32_t)r, (uint32_t)j, u_prev, C, N, ba, bb, uj, &s, &parent);
                    att_total += a > 0 ? a : -a;
                    if (a < 0) { ++invalid; ++j; continue; }
                    double d = ref_sim_distance(cfg, obs, uj, (uint32_t)r, (uint32_t)j, traj);
                    if (d <= eps) { /* accept: dist <= eps (§II-C) */
                        memcpy(u + (size_t)accepted * REF_NPAR, uj, sizeof uj);
                        dist[accepted] = d; sig[accepted] = s; par[accepted] = parent;
                        idx[accepted] = j; att[accepted] = a;
                        ++accepted;
                    }
                    ++j;
                }
                out->simulated[r] = j;
            } else {
                /* MCMC variant: batches of cfg->batch proposals, one s per batch;
                 * a batch is simulated whole, acceptances past the N-th are
                 * counted for eq. 14 but not kept */
                int64_t base = 0, proposals = -1, inval_all = 0, att_all = 0;
                while (accepted < N) {
                    if (base >= cfg->max_proposals) { rc = -4; break; }
                    int64_t B = cfg->batch;
                    if (base + B > cfg->max_proposals) B = cfg->max_proposals - base;
                    int64_t acc_b = 0, valid_b = 0;
                    for (j = base; j < base + B; ++j) {
                        double uj[REF_NPAR], s; int64_t parent;
                        int32_t a = ref_perturb(cfg, (uint32_t)r, (uint32_t)j, u_prev, C, N, s_mcmc, 0, uj, &s,
                                                &parent);
                        att_all += a > 0 ? a : -a;
                        if (a < 0) { ++inval_all; continue; }
                        ++valid_b;
                        double d = ref_sim_distance(cfg, obs, uj, (uint32_t)r, (uint32_t)j, traj);
                        if (d <= eps) {
                            ++acc_b;
                            if (accepted < N) {
                                memcpy(u + (size_t)accepted * REF_NPAR, uj, sizeof uj);
                                dist[accepted] = d; sig[accepted] = s; par[accepted] = parent;
                                idx[accepted] = j; att[accepted] = a;
                                ++accepted;
                                if (accepted == N) proposals = j + 1;
                            }
                        }
                    }
                    base += B;
                    if (tunes < cfg->mcmc_tune) {
                        n_acc += acc_b;
                        s_mcmc = ref_mcmc_update(s_mcmc, acc_b, valid_b, n_acc);
                        ++tunes;
                    }
                }
                if (rc != 0) break;
                j = proposals;
                invalid = inval_all;
                att_total = att_all;
                out->simulated[r] = base;
            }
            if (rc != 0) break;
            for (int64_t k = 0; k < N; ++k)
                lw[k] = ref_log_weight(u + (size_t)k * REF_NPAR, sig[k], u_prev, q, N);
            out->ess[r] = ref_normalise(lw, N, W);
        }
        if (r == 0) { out->ess[0] = (double)N; out->simulated[0] = N; out->beta_b_real[0] = 0.0; }
        out->mcmc_s[r] = s_mcmc;
        out->proposals[r] = j;
        out->invalid[r] = invalid;
        out->attempts_total[r] = att_total;
        out->eps_next[r] = ref_quantile(dist, N, cfg->surv_ratio);
    }
    free(traj); free(q); free(C);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Array helpers for the tests (no new arithmetic).                     */
/* ------------------------------------------------------------------ */
void ref_map(int32_t fn, const double* x, double* y, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) {
        switch (fn) {
        case 0: y[i] = ref_exp(x[i]); break;
        case 1: y[i] = ref_expm1(x[i]); break;
        case 2: y[i] = ref_log(x[i]); break;
        case 3: y[i] = ref_log1p(x[i]); break;
        case 4: { double c, s; ref_sincos2pi(x[i], &c, &s); y[i] = c; } break;
        case 5: { double c, s; ref_sincos2pi(x[i], &c, &s); y[i] = s; } break;
        default: y[i] = NAN;
        }
    }
}

void ref_words(uint64_t seed, uint32_t index, uint32_t round, uint32_t purpose, uint32_t sub,
               uint32_t nwords, uint64_t* out)
{
    for (uint32_t w = 0; w < nwords; ++w) out[w] = ref_word(seed, index, round, purpose, sub, w);
}

/* Number of the n simulations of u on streams index0 .. index0+n-1 of
 * `round` whose distance is at most eps (acceptance of §II-C). */
int64_t ref_accept_count(const ref_config* cfg, const int64_t* obs, const double u[REF_NPAR], double eps,
                         uint32_t round, uint32_t index0, int64_t n)
{
    int64_t* traj = (int64_t*)malloc((size_t)(cfg->n_days + 1) * 6 * sizeof(int64_t));
    int64_t acc = 0;
    for (int64_t i = 0; i < n; ++i)
        acc += ref_sim_distance(cfg, obs, u, round, index0 + (uint32_t)i, traj) <= eps;
    free(traj);
    return acc;
}

void ref_binomial_many(const int64_t* n, const double* p, const uint64_t* w, int64_t* out, int64_t cnt)
{
    for (int64_t i = 0; i < cnt; ++i) out[i] = ref_binomial(n[i], p[i], w[i]);
}

void ref_box_muller_many(const uint64_t* w, double* z, int64_t cnt)
{
    for (int64_t i = 0; i < cnt; ++i) ref_box_muller(w[i], &z[2 * i], &z[2 * i + 1]);
}

void ref_beta_many(double a, int32_t b, const uint64_t* words, double* out, int64_t cnt)
{
    for (int64_t i = 0; i < cnt; ++i) out[i] = ref_beta_int(a, b, words + (size_t)i * b);
}

/* n general Beta(a, b) draws: draw i uses stream (seed, index0 + i, round, PERTURB, sub) */
void ref_beta_general_many(double a, double b, uint64_t seed, uint32_t index0, uint32_t round, uint32_t sub,
                           double* out, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) out[i] = ref_beta_general(a, b, seed, index0 + (uint32_t)i, round, sub);
}

void ref_gamma_many(double k, uint64_t seed, uint32_t index0, uint32_t round, uint32_t sub, double* out, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) out[i] = ref_gamma_mt(k, seed, index0 + (uint32_t)i, round, sub, 5);
}

