// sim.hip -- proposal kernel (perturb + simulate + distance + accept, one
// wave64 lane per proposal), ordered compaction of acceptances, trajectory
// kernel and the primitive test hook.
#include "dmath.h"
#include "kernels.h"

namespace abcsmc {

namespace {

// ---------------------------------------------------------------------------
// One trajectory of the epidemic model (§II-B, eqs. 3-5) with the running
// Euclidean distance to the observed (A, R, D) (§II-C).
//   init   Ru = 0, I = floor(kappa A0) (capped so S >= 0), S = P - (A0+R0+D0+I)
//   day t  g = alpha0 + alpha / (1 + (A+R+D)^n)          (eq. 4)
//          transitions in the order of h (eq. 5): S->I, I->A, A->R, A->D, I->Ru,
//          each drawn from what is left of its source compartment
//   dist   sum over days 1..T of dA^2, dR^2, dD^2 in that order; sqrt at the end
// Returns +inf as soon as the partial sum exceeds exit_thr (the final
// distance would exceed eps).  Draw k of day t is word k of the stream
// (index, round, SIM, t): blocks 0, 0, 1, 1, 2.
// ---------------------------------------------------------------------------
template <int kSampler, bool kTraj>
__device__ __forceinline__ double simulate_distance(const Model& m, const double* th,
                                                    const double* __restrict__ obs, uint32_t round,
                                                    uint32_t index, double exit_thr, int64_t* traj,
                                                    int32_t& days)
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
        traj[0] = (int64_t)S; traj[1] = (int64_t)I; traj[2] = (int64_t)A;
        traj[3] = (int64_t)R; traj[4] = (int64_t)D; traj[5] = (int64_t)Ru;
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
            n1 = dm::binomial(S, pSI, b0.a);
            n2 = dm::binomial(I, pIA, b0.b);
            n3 = dm::binomial(A, pAR, b1.a);
            n4 = dm::binomial(A - n3, pAD, b1.b);
            n5 = dm::binomial(I - n2, pIRu, b2.a);
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
            int64_t* row = traj + (size_t)(t + 1) * 6;
            row[0] = (int64_t)S; row[1] = (int64_t)I; row[2] = (int64_t)A;
            row[3] = (int64_t)R; row[4] = (int64_t)D; row[5] = (int64_t)Ru;
        }
        if (!kTraj) {
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

// ---------------------------------------------------------------------------
// Proposal kernel.  Stage 0: u ~ U(0,1)^8 (prior of eq. 2 in the unit cube).
// Stage i >= 1, attempt a = 1, 2, ...: parent k ~ Categorical(q) (eq. 11) from
// word 0; s ~ Beta(a_i, b_i) (eq. 16) from words 5..5+b-1; z ~ N(0, I_8) from
// the Box-Muller pairs of words 1..4; u = u_k + sigma z (eq. 17); stop at the
// first u inside [0,1]^8.  Then simulate, distance, accept iff d <= eps, and
// publish the wave's acceptance ballot for the ordered compaction.
// ---------------------------------------------------------------------------
template <bool kRound0, int kSampler>
__global__ __launch_bounds__(kBlock) void propose_kernel(ProposeArgs a)
{
    const uint32_t p = blockIdx.x * kBlock + threadIdx.x;
    const bool active = p < a.count;
    const uint32_t j = a.base + p;
    double u[kNP];
    double sigma = 0.0;
    int32_t parent = -1;
    int32_t att = 1;
    bool valid = active;
    if (active) {
        if (kRound0) {
#pragma unroll
            for (uint32_t blk = 0; blk < 4; ++blk) {
                const dm::w2 w = dm::block_words(a.m.seed, j, 0, dm::kPrior, 0, blk);
                u[2 * blk] = dm::u01(w.a);
                u[2 * blk + 1] = dm::u01(w.b);
            }
        } else {
            const uint64_t Q = a.cdf[a.n_prev - 1];
            valid = false;
            for (att = 1; att <= a.max_attempts; ++att) {
                const uint32_t sub = (uint32_t)(att - 1);
                const dm::w2 b0 = dm::block_words(a.m.seed, j, a.round, dm::kPerturb, sub, 0);
                const dm::w2 b1 = dm::block_words(a.m.seed, j, a.round, dm::kPerturb, sub, 1);
                const dm::w2 b2 = dm::block_words(a.m.seed, j, a.round, dm::kPerturb, sub, 2);
                const uint64_t r = __umul64hi(b0.a, Q);
                const int32_t k = upper_bound_u64(a.cdf, a.n_prev, r);
                // Beta(a, b), b integer: exp( sum_m log U_m / (a + m) )
                double L = 0.0;
                uint64_t hold = 0;
                for (int32_t mm = 0; mm < a.beta_b; ++mm) {
                    uint64_t w;
                    if (mm == 0) {
                        w = b2.b;
                    } else if (mm & 1) {
                        const dm::w2 nb = dm::block_words(a.m.seed, j, a.round, dm::kPerturb, sub,
                                                          2u + (uint32_t)((mm + 1) >> 1));
                        w = nb.a;
                        hold = nb.b;
                    } else {
                        w = hold;
                    }
                    L = L + dm::log(dm::u01(w)) / (a.beta_a + (double)mm);
                }
                const double s = dm::exp(L);
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
    double d = __builtin_inf();
    bool acc = false;
    int32_t days = 0;
    if (valid) {
        double th[kNP];
#pragma unroll
        for (int q = 0; q < kNP; ++q) th[q] = a.m.lo[q] + u[q] * a.m.width[q];
        d = simulate_distance<kSampler, false>(a.m, th, a.obs, a.round, j, a.exit_thr, nullptr, days);
        acc = d <= a.eps;
    }
    if (active) {
        double* su = a.st_u + (size_t)p * kNP;
#pragma unroll
        for (int q = 0; q < kNP; ++q) su[q] = u[q];
        a.st_d[p] = d;
        a.st_sigma[p] = sigma;
        a.st_parent[p] = parent;
        a.st_att[p] = att;
    }
    const unsigned long long mask = __ballot(acc);
    const unsigned long long inv = wave_sum_u64((active && !valid) ? 1ull : 0ull);
    const unsigned long long natt = wave_sum_u64(active ? (unsigned long long)(att < 0 ? -att : att) : 0ull);
    const unsigned long long ndays = wave_sum_u64((unsigned long long)days);
    if ((threadIdx.x & (kWave - 1)) == 0) {
        a.wave_mask[p / kWave] = mask;
        if (inv) atomicAdd(&a.ctr->invalid, inv);
        if (natt) atomicAdd(&a.ctr->attempts, natt);
        if (ndays) atomicAdd(&a.ctr->days, ndays);
    }
}

// Exclusive prefix of the per-wave acceptance counts (one workgroup) and the
// batch's starting rank.
constexpr int kScanThreads = 1024;

__global__ __launch_bounds__(kScanThreads) void compact_scan_kernel(CompactArgs a)
{
    __shared__ unsigned long long part[kScanThreads];
    const uint32_t nW = (a.count + kWave - 1) / kWave;
    const uint32_t per = (nW + kScanThreads - 1) / kScanThreads;
    const uint32_t t = threadIdx.x;
    const uint32_t b0 = t * per, b1 = min(nW, b0 + per);
    unsigned long long s = 0;
    for (uint32_t w = b0; w < b1; ++w) s += __popcll(a.wave_mask[w]);
    part[t] = s;
    __syncthreads();
    // Hillis-Steele inclusive scan over 1024 partial sums
    for (int off = 1; off < kScanThreads; off <<= 1) {
        const unsigned long long v = (t >= (uint32_t)off) ? part[t - off] : 0ull;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    unsigned long long run = part[t] - s;
    for (uint32_t w = b0; w < b1; ++w) {
        a.wave_off[w] = (uint32_t)run;
        run += __popcll(a.wave_mask[w]);
    }
    if (t == kScanThreads - 1) {
        const unsigned long long before = a.ctr->accepted;
        a.ctr->base_rank = before;
        a.ctr->accepted = before + part[t];
    }
}

// Scatter the acceptances of the batch into population slots in proposal
// order; slots >= N are dropped (the stage keeps its first N acceptances).
__global__ __launch_bounds__(kBlock) void compact_scatter_kernel(CompactArgs a)
{
    const uint32_t p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= a.count) return;
    const uint32_t w = p / kWave, lane = p % kWave;
    const unsigned long long mask = a.wave_mask[w];
    if (!((mask >> lane) & 1ull)) return;
    const unsigned long long below = lane ? (mask & ((1ull << lane) - 1ull)) : 0ull;
    const unsigned long long gr = a.ctr->base_rank + a.wave_off[w] + (unsigned long long)__popcll(below);
    if (gr >= (unsigned long long)a.N) return;
    const double* su = a.st_u + (size_t)p * kNP;
    double* du = a.pop.u + (size_t)gr * kNP;
#pragma unroll
    for (int q = 0; q < kNP; ++q) du[q] = su[q];
    a.pop.d[gr] = a.st_d[p];
    a.pop.sigma[gr] = a.st_sigma[p];
    a.pop.parent[gr] = a.st_parent[p];
    a.pop.index[gr] = a.base + p;
    a.pop.att[gr] = a.st_att[p];
    if (gr == (unsigned long long)(a.N - 1)) a.ctr->proposals = (unsigned long long)a.base + p + 1ull;
}

template <int kSampler>
__global__ __launch_bounds__(kBlock) void simulate_traj_kernel(TrajArgs a)
{
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= a.n) return;
    double th[kNP];
#pragma unroll
    for (int q = 0; q < kNP; ++q) th[q] = a.theta[k * kNP + q];
    int64_t* traj = a.traj + (size_t)k * (size_t)(a.m.T + 1) * 6;
    // a bare trajectory: no observations, no distance
    int32_t days = 0;
    simulate_distance<kSampler, true>(a.m, th, nullptr, a.round, a.index0 + (uint32_t)k,
                                      __builtin_inf(), traj, days);
}

__global__ __launch_bounds__(kBlock) void debug_eval_kernel(int32_t fn, int64_t n, const void* in,
                                                            void* out, double pa, int32_t pb)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const double* x = (const double*)in;
    double* y = (double*)out;
    switch (fn) {
    case 0: y[i] = dm::exp(x[i]); break;
    case 1: y[i] = dm::expm1(x[i]); break;
    case 2: y[i] = dm::log(x[i]); break;
    case 3: y[i] = dm::log1p(x[i]); break;
    case 4: { double c, s; dm::sincos2pi(x[i], c, s); y[i] = c; } break;
    case 5: { double c, s; dm::sincos2pi(x[i], c, s); y[i] = s; } break;
    case 6: y[i] = __builtin_sqrt(x[i]); break;
    case 7: y[i] = x[2 * i] / x[2 * i + 1]; break;
    case 8: {
        const uint32_t* c = (const uint32_t*)in + 6 * i;
        dm::u4 o = dm::philox10(dm::u4{c[0], c[1], c[2], c[3]}, c[4], c[5]);
        uint32_t* r = (uint32_t*)out + 4 * i;
        r[0] = o.x; r[1] = o.y; r[2] = o.z; r[3] = o.w;
    } break;
    case 9: {
        const uint64_t w = ((const uint64_t*)in)[i];
        dm::normal_pair(w, y[2 * i], y[2 * i + 1]);
    } break;
    case 10:
    case 12: {
        const int64_t nn = ((const int64_t*)in)[3 * i];
        const double pp = ((const double*)in)[3 * i + 1];
        const uint64_t w = ((const uint64_t*)in)[3 * i + 2];
        const double r = fn == 10 ? dm::binomial((double)nn, pp, w) : dm::normal_floor((double)nn, pp, w);
        ((int64_t*)out)[i] = (int64_t)r;
    } break;
    case 11: {
        const uint64_t* w = (const uint64_t*)in + (size_t)i * pb;
        double L = 0.0;
        for (int32_t mm = 0; mm < pb; ++mm) L = L + dm::log(dm::u01(w[mm])) / (pa + (double)mm);
        y[i] = dm::exp(L);
    } break;
    default: break;
    }
}

inline unsigned grid_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

void launch_propose(const ProposeArgs& a, bool round0, hipStream_t s)
{
    const dim3 g(grid_for(a.count)), b(kBlock);
    if (round0) {
        if (a.m.sampler == 0) hipLaunchKernelGGL((propose_kernel<true, 0>), g, b, 0, s, a);
        else hipLaunchKernelGGL((propose_kernel<true, 1>), g, b, 0, s, a);
    } else {
        if (a.m.sampler == 0) hipLaunchKernelGGL((propose_kernel<false, 0>), g, b, 0, s, a);
        else hipLaunchKernelGGL((propose_kernel<false, 1>), g, b, 0, s, a);
    }
}

void launch_compact(const CompactArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(compact_scan_kernel, dim3(1), dim3(kScanThreads), 0, s, a);
    hipLaunchKernelGGL(compact_scatter_kernel, dim3(grid_for(a.count)), dim3(kBlock), 0, s, a);
}

void launch_simulate_traj(const TrajArgs& a, hipStream_t s)
{
    if (a.m.sampler == 0)
        hipLaunchKernelGGL((simulate_traj_kernel<0>), dim3(grid_for(a.n)), dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL((simulate_traj_kernel<1>), dim3(grid_for(a.n)), dim3(kBlock), 0, s, a);
}

void launch_debug_eval(int32_t fn, int64_t n, const void* in, void* out, double pa, int32_t pb,
                       hipStream_t s)
{
    hipLaunchKernelGGL(debug_eval_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, fn, n, in, out, pa, pb);
}

}  // namespace abcsmc
