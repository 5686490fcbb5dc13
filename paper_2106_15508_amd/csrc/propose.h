// propose.h -- per-lane device code of one proposal: perturbation (or prior
// draw), forward simulation, distance and acceptance.  Shared by the plain
// batch kernel and the persistent batched-runs kernel.
#pragma once

#include "dmath.h"
#include "kernels.h"

namespace abcsmc {
namespace lane {

// ---------------------------------------------------------------------------
// One trajectory of the epidemic model (§II-B, eqs. 3-5) with the running
// Euclidean distance to the observed (A, R, D) (§II-C).
//   init   Ru = 0, I = floor(kappa A0) (capped so S >= 0), S = P - (A0+R0+D0+I)
//   day t  g = alpha0 + alpha / (1 + (A+R+D)^n)          (eq. 4)
//          transitions in the order of h (eq. 5): S->I, I->A, A->R, A->D, I->Ru,
//          each drawn from what is left of its source compartment
//   dist   sum over days 1..T of dA^2, dR^2, dD^2 in that order; sqrt at the end
// Returns +inf as soon as the partial sum exceeds exit_thr (the final
// distance would exceed eps).  Stream (index, round, SIM, t) of day t: draw k
// takes its inversion uniform from word k and its normal deviate from the
// Box-Muller pairs of words 5 (draws 0, 1), 6 (draws 2, 3) and 7 (draw 4);
// the floor-normal sampler uses the cosine deviate of word k.
// ---------------------------------------------------------------------------
// With kSplit the three series' sums of squares also go to split[0..2]
// (no early exit; the surrogate's training targets); the returned distance
// is the same as without.
// With kTraj and series != null the trajectory's (A, R, D) go to
// series[(3 t + c) * sstride] (day t = 0..T) instead of traj.
template <int kSampler, bool kTraj, bool kSplit = false>
__device__ __forceinline__ double simulate_distance(const Model& m, const double* th,
                                                    const double* __restrict__ obs, uint32_t round,
                                                    uint32_t index, double exit_thr, int64_t* traj,
                                                    int32_t& days, double* split = nullptr,
                                                    double* series = nullptr, int64_t sstride = 0)
{
    const double alpha0 = th[0], alpha_c = th[1], n_exp = th[2], beta = th[3];
    const double gamma = th[4], delta = th[5], eta = th[6], kappa = th[7];
    double A = m.A0, R = m.R0, D = m.D0;
    double I = __builtin_floor(kappa * A);
    const double room = m.P - (A + R + D);
    if (I > room) I = room;
    if (I < 0.0) I = 0.0;
    double S = m.P - (A + R + D + I);
    double Ru = 0.0;
    double pIA = 0.0, pAR = 0.0, pAD = 0.0, pIRu = 0.0;
    if (kSampler == 0) {
        pIA = -dm::expm1(-gamma);
        pAR = -dm::expm1(-beta);
        pAD = -dm::expm1(-delta);
        pIRu = -dm::expm1(-(beta * eta));
    }
    if (kTraj) {
        if (series) {
            series[0] = A;
            series[sstride] = R;
            series[2 * sstride] = D;
        } else {
            traj[0] = (int64_t)S; traj[1] = (int64_t)I; traj[2] = (int64_t)A;
            traj[3] = (int64_t)R; traj[4] = (int64_t)D; traj[5] = (int64_t)Ru;
        }
    }
    double acc = 0.0;
    for (int32_t t = 0; t < m.T; ++t) {
        const double C = A + R + D;
        double pw;
        if (C == 0.0) pw = (n_exp == 0.0) ? 1.0 : 0.0;
        else pw = dm::exp(n_exp * dm::log(C));
        const double g = alpha0 + alpha_c / (1.0 + pw);
        const double rate = (g * I) * m.invP;
        const dm::w2 b0 = dm::block_words(m.seed, index, round, dm::kSim, (uint32_t)t, 0);
        const dm::w2 b1 = dm::block_words(m.seed, index, round, dm::kSim, (uint32_t)t, 1);
        const dm::w2 b2 = dm::block_words(m.seed, index, round, dm::kSim, (uint32_t)t, 2);
        double n1, n2, n3, n4, n5;
        if (kSampler == 0) {
            const double pSI = -dm::expm1(-rate);
            const dm::w2 b3 = dm::block_words(m.seed, index, round, dm::kSim, (uint32_t)t, 3);
            bool h01 = false, h23 = false, h4 = false;
            double z0, z1, z2, z3, z4, z5;
            n1 = dm::binomial_pair(S, pSI, b0.a, b2.b, 0, h01, z0, z1);
            n2 = dm::binomial_pair(I, pIA, b0.b, b2.b, 1, h01, z0, z1);
            n3 = dm::binomial_pair(A, pAR, b1.a, b3.a, 0, h23, z2, z3);
            n4 = dm::binomial_pair(A - n3, pAD, b1.b, b3.a, 1, h23, z2, z3);
            n5 = dm::binomial_pair(I - n2, pIRu, b2.a, b3.b, 0, h4, z4, z5);
        } else {
            n1 = dm::normal_floor(S, rate * S, b0.a);
            n2 = dm::normal_floor(I, gamma * I, b0.b);
            n3 = dm::normal_floor(A, beta * A, b1.a);
            n4 = dm::normal_floor(A - n3, delta * A, b1.b);
            n5 = dm::normal_floor(I - n2, (beta * eta) * I, b2.a);
        }
        S = S - n1;
        I = I + n1 - n2 - n5;
        A = A + n2 - n3 - n4;
        R = R + n3;
        D = D + n4;
        Ru = Ru + n5;
        if (kTraj) {
            if (series) {
                double* col = series + (size_t)(3 * (t + 1)) * sstride;
                col[0] = A;
                col[sstride] = R;
                col[2 * sstride] = D;
            } else {
                int64_t* row = traj + (size_t)(t + 1) * 6;
                row[0] = (int64_t)S; row[1] = (int64_t)I; row[2] = (int64_t)A;
                row[3] = (int64_t)R; row[4] = (int64_t)D; row[5] = (int64_t)Ru;
            }
        }
        if (kSplit) {
            const double* o = obs + (size_t)(t + 1) * 3;
            const double dA = A - o[0];
            const double dR = R - o[1];
            const double dD = D - o[2];
            split[0] = split[0] + dA * dA;
            split[1] = split[1] + dR * dR;
            split[2] = split[2] + dD * dD;
            acc = acc + dA * dA;
            acc = acc + dR * dR;
            acc = acc + dD * dD;
        } else if (!kTraj) {
            const double* o = obs + (size_t)(t + 1) * 3;
            const double dA = A - o[0];
            const double dR = R - o[1];
            const double dD = D - o[2];
            acc = acc + dA * dA;
            acc = acc + dR * dR;
            acc = acc + dD * dD;
            if (acc > exit_thr) {
                days = t + 1;
                return __builtin_inf();
            }
        }
    }
    days = m.T;
    return __builtin_sqrt(acc);
}

// First k with cdf[k] > r (cdf non-decreasing, cdf[n-1] > r).
__device__ __forceinline__ int32_t upper_bound_u64(const uint64_t* __restrict__ cdf, int32_t n, uint64_t r)
{
    int32_t lo = 0, hi = n - 1;
    while (lo < hi) {
        const int32_t mid = lo + ((hi - lo) >> 1);
        if (cdf[mid] > r) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}


// Inputs of one proposal beyond the model.
struct ProposalIn {
    const double* obs;       // (T+1) x 3
    uint32_t round;
    int32_t max_attempts;
    double eps;              // accept iff d <= eps
    double exit_thr;         // early-exit threshold on the partial sum of squares
    const double* u_prev;    // previous population, n_prev x 8
    const uint64_t* cdf;     // its integer CDF
    int32_t n_prev;
    double beta_a;
    int32_t beta_b;
    int32_t step_is_variance;
    double s_fixed;          // >= 0: step size of every proposal (MCMC variant); < 0: Beta draw
    double beta_b_real;      // > 0: real Beta shape b (general sampler; beta_b unused)
};

struct ProposalOut {
    double u[kNP];
    double sigma;
    int32_t parent;
    int32_t att;             // attempts used; -max_attempts for a void proposal
    double d;
    bool valid;
    bool acc;
    int32_t days;            // days simulated
};

// ---------------------------------------------------------------------------
// One proposal j.  Stage 0: u ~ U(0,1)^8 (prior of eq. 2 in the unit cube).
// Stage i >= 1, attempt a = 1, 2, ...: parent k ~ Categorical(q) (eq. 11) from
// word 0; s ~ Beta(a_i, b_i) (eq. 16) from words 5..5+b-1; z ~ N(0, I_8) from
// the Box-Muller pairs of words 1..4; u = u_k + sigma z (eq. 17); stop at the
// first u inside [0,1]^8.  Then simulate, distance, accept iff d <= eps.
// ---------------------------------------------------------------------------
// Stage-0 prior draw (kRound0) or the perturbation attempts of stage >= 1:
// fills o.u, o.sigma, o.parent, o.att and o.valid.
template <bool kRound0>
__device__ __forceinline__ void perturb_one(const Model& m, const ProposalIn& a, uint32_t j, ProposalOut& o)
{
    double* u = o.u;
    double sigma = 0.0;
    int32_t parent = -1;
    int32_t att = 1;
    bool valid = true;
    {
        if (kRound0) {
#pragma unroll
            for (uint32_t blk = 0; blk < 4; ++blk) {
                const dm::w2 w = dm::block_words(m.seed, j, 0, dm::kPrior, 0, blk);
                u[2 * blk] = dm::u01(w.a);
                u[2 * blk + 1] = dm::u01(w.b);
            }
        } else {
            const uint64_t Q = a.cdf[a.n_prev - 1];
            valid = false;
            for (att = 1; att <= a.max_attempts; ++att) {
                const uint32_t sub = (uint32_t)(att - 1);
                const dm::w2 b0 = dm::block_words(m.seed, j, a.round, dm::kPerturb, sub, 0);
                const dm::w2 b1 = dm::block_words(m.seed, j, a.round, dm::kPerturb, sub, 1);
                const dm::w2 b2 = dm::block_words(m.seed, j, a.round, dm::kPerturb, sub, 2);
                const uint64_t r = __umul64hi(b0.a, Q);
                const int32_t k = upper_bound_u64(a.cdf, a.n_prev, r);
                // Beta(a, b), b integer: exp( sum_m log U_m / (a + m) )
                double L = 0.0;
                uint64_t hold = 0;
                const int32_t nb = (a.s_fixed >= 0.0 || a.beta_b_real > 0.0) ? 0 : a.beta_b;
                for (int32_t mm = 0; mm < nb; ++mm) {
                    uint64_t w;
                    if (mm == 0) {
                        w = b2.b;
                    } else if (mm & 1) {
                        const dm::w2 nb = dm::block_words(m.seed, j, a.round, dm::kPerturb, sub,
                                                          2u + (uint32_t)((mm + 1) >> 1));
                        w = nb.a;
                        hold = nb.b;
                    } else {
                        w = hold;
                    }
                    L = L + dm::log(dm::u01(w)) / (a.beta_a + (double)mm);
                }
                const double s = a.s_fixed >= 0.0       ? a.s_fixed
                                 : a.beta_b_real > 0.0 ? dm::beta_general(a.beta_a, a.beta_b_real, m.seed, j,
                                                                          a.round, sub)
                                                       : dm::exp(L);
                double sg = a.step_is_variance ? __builtin_sqrt(s) : s;
                if (sg < 1e-8) sg = 1e-8;
                double z[kNP];
                dm::normal_pair(b0.b, z[0], z[1]);
                dm::normal_pair(b1.a, z[2], z[3]);
                dm::normal_pair(b1.b, z[4], z[5]);
                dm::normal_pair(b2.a, z[6], z[7]);
                const double* up = a.u_prev + (size_t)k * kNP;
                bool inside = true;
#pragma unroll
                for (int d = 0; d < kNP; ++d) {
                    const double v = up[d] + sg * z[d];
                    u[d] = v;
                    inside = inside && (v >= 0.0 && v <= 1.0);
                }
                sigma = sg;
                parent = k;
                if (inside) {
                    valid = true;
                    break;
                }
            }
            if (!valid) att = -a.max_attempts;
        }
    }
    o.sigma = sigma;
    o.parent = parent;
    o.att = att;
    o.valid = valid;
}

template <bool kRound0, int kSampler>
__device__ __forceinline__ void propose_one(const Model& m, const ProposalIn& a, uint32_t j, ProposalOut& o)
{
    perturb_one<kRound0>(m, a, j, o);
    double d = __builtin_inf();
    bool acc = false;
    int32_t days = 0;
    if (o.valid) {
        double th[kNP];
#pragma unroll
        for (int q = 0; q < kNP; ++q) th[q] = m.lo[q] + o.u[q] * m.width[q];
        d = simulate_distance<kSampler, false>(m, th, a.obs, a.round, j, a.exit_thr, nullptr, days);
        acc = d <= a.eps;
    }
    o.d = d;
    o.acc = acc;
    o.days = days;
}

}  // namespace lane
}  // namespace abcsmc
