// screen.hip -- kernels of the surrogate-screened stage and of the
// surrogate's training data.
//
// Screened stage (i >= 1), per pool batch of proposal indices [base, base+count):
//   perturb   the same per-index perturbation as the plain stage (eqs. 11, 16, 17)
//   score     network prediction of the squared distance (mlp.hip)
//   keep      score <= tau (fixed per stage) or an audit draw u < rho from
//             the proposal's own AUDIT stream
//   simulate  exact FP64 simulation and distance of the kept proposals only,
//             acceptance d <= eps, first N acceptances in index order
// The screened proposal density is q(u) [1{score <= tau} + rho 1{score > tau}]
// up to a constant, so an acceptance kept only by the audit carries an
// importance weight 1/rho times that of the plain stage.
#include "dmath.h"
#include "mlp.h"
#include "propose.h"

namespace abcsmc {

namespace {

constexpr uint32_t kAudit = 4;
constexpr uint32_t kMlpInit = 5;

__global__ __launch_bounds__(kBlock) void perturb_only_kernel(PerturbArgs a)
{
    const uint32_t p = blockIdx.x * kBlock + threadIdx.x;
    const bool active = p < a.count;
    int32_t att = 0;
    bool valid = false;
    if (active) {
        const lane::ProposalIn in{nullptr, a.round, a.max_attempts, 0.0, 0.0, a.u_prev, a.cdf, a.n_prev,
                                  a.beta_a, a.beta_b, a.step_is_variance, -1.0, a.beta_b_real};
        lane::ProposalOut o;
        lane::perturb_one<false>(a.m, in, a.base + p, o);
        double* u = a.pu + (size_t)p * kNP;
        float* x = a.x + (size_t)p * kNP;
#pragma unroll
        for (int d = 0; d < kNP; ++d) {
            u[d] = o.u[d];
            x[d] = o.valid ? (float)(2.0 * o.u[d] - 1.0) : 0.f;
        }
        a.psigma[p] = o.sigma;
        a.pparent[p] = o.parent;
        a.patt[p] = o.att;
        att = o.att < 0 ? -o.att : o.att;
        valid = o.valid;
    }
    const unsigned long long inv = lane::wave_sum_u64((active && !valid) ? 1ull : 0ull);
    const unsigned long long natt = lane::wave_sum_u64((unsigned long long)att);
    if ((threadIdx.x & (kWave - 1)) == 0) {
        if (inv) atomicAdd(&a.ctr->invalid, inv);
        if (natt) atomicAdd(&a.ctr->attempts, natt);
    }
}

__global__ __launch_bounds__(kBlock) void keep_kernel(KeepArgs a)
{
    const uint32_t p = blockIdx.x * kBlock + threadIdx.x;
    const bool active = p < a.count;
    bool screen = false, audit_only = false;
    if (active && a.patt[p] > 0) {
        screen = a.score[p] <= *a.tau;
        const dm::w2 w = dm::block_words(a.seed, a.base + p, a.round, kAudit, 0, 0);
        audit_only = !screen && dm::u01(w.a) < a.rho;
    }
    if (active) a.audit[p] = audit_only ? 1 : 0;
    const unsigned long long mask = __ballot(screen || audit_only);
    const unsigned long long ns = lane::wave_sum_u64(screen ? 1ull : 0ull);
    const unsigned long long na = lane::wave_sum_u64(audit_only ? 1ull : 0ull);
    if ((threadIdx.x & (kWave - 1)) == 0) {
        a.wave_mask[p / kWave] = mask;
        if (ns) atomicAdd(&a.sc->kept_screen, ns);
        if (na) atomicAdd(&a.sc->kept_audit, na);
    }
}

template <bool kTune>
__global__ __launch_bounds__(kBlock) void sim_kept_kernel(SimKeptArgs a)
{
    const uint32_t t = blockIdx.x * kBlock + threadIdx.x;
    const uint32_t i = a.first + t;
    const bool active = t < a.n;
    bool acc = false, aud = false;
    int32_t days = 0;
    if (active) {
        const uint32_t pos = a.kept[i];
        const double* u = a.pu + (size_t)pos * kNP;
        double th[kNP];
#pragma unroll
        for (int q = 0; q < kNP; ++q) th[q] = a.m.lo[q] + u[q] * a.m.width[q];
        double d;
        if (kTune) {
            double split[3] = {0.0, 0.0, 0.0};
            if (a.m.sampler == 0)
                d = lane::simulate_distance<0, false, true>(a.m, th, a.obs, a.round, a.base + pos, __builtin_inf(),
                                                            nullptr, days, split);
            else
                d = lane::simulate_distance<1, false, true>(a.m, th, a.obs, a.round, a.base + pos, __builtin_inf(),
                                                            nullptr, days, split);
#pragma unroll
            for (int q = 0; q < kNP; ++q) a.tune_x[(size_t)t * kNP + q] = (float)(2.0 * u[q] - 1.0);
            for (int c = 0; c < 3; ++c) a.tune_y[(size_t)t * 3 + c] = (float)log1p(sqrt(split[c]));
        } else if (a.m.sampler == 0) {
            d = lane::simulate_distance<0, false>(a.m, th, a.obs, a.round, a.base + pos, a.exit_thr, nullptr, days);
        } else {
            d = lane::simulate_distance<1, false>(a.m, th, a.obs, a.round, a.base + pos, a.exit_thr, nullptr, days);
        }
        a.kd[i] = d;
        acc = d <= a.eps;
        aud = a.paudit[pos] != 0;
    }
    const unsigned long long mask = __ballot(acc);
    const unsigned long long nd = lane::wave_sum_u64((unsigned long long)days);
    const unsigned long long na = lane::wave_sum_u64((acc && aud) ? 1ull : 0ull);
    const unsigned long long ns = lane::wave_sum_u64((acc && !aud) ? 1ull : 0ull);
    if ((threadIdx.x & (kWave - 1)) == 0) {
        a.wave_mask[i / kWave] = mask;
        if (nd) atomicAdd(&a.ctr->days, nd);
        if (na) atomicAdd(&a.sc->acc_audit, na);
        if (ns) atomicAdd(&a.sc->acc_screen, ns);
    }
}

__global__ __launch_bounds__(kBlock) void train_data_kernel(TrainDataArgs a)
{
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= a.n) return;
    const lane::ProposalIn in{};
    lane::ProposalOut o;
    lane::perturb_one<true>(a.m, in, (uint32_t)j, o);
    double th[kNP];
#pragma unroll
    for (int q = 0; q < kNP; ++q) th[q] = a.m.lo[q] + o.u[q] * a.m.width[q];
    double split[3] = {0.0, 0.0, 0.0};
    int32_t days = 0;
    if (a.m.sampler == 0)
        lane::simulate_distance<0, false, true>(a.m, th, a.obs, 0, (uint32_t)j, __builtin_inf(), nullptr, days, split);
    else
        lane::simulate_distance<1, false, true>(a.m, th, a.obs, 0, (uint32_t)j, __builtin_inf(), nullptr, days, split);
#pragma unroll
    for (int q = 0; q < kNP; ++q) a.x[j * kNP + q] = (float)(2.0 * o.u[q] - 1.0);
    for (int c = 0; c < 3; ++c) a.y[j * 3 + c] = (float)log1p(sqrt(split[c]));
}

// Weights ~ N(0, 1/fan_in) (first Box-Muller normal of word 0 of the
// parameter's MLP stream, computed in FP64 and rounded once), biases 0.
__global__ __launch_bounds__(kBlock) void mlp_init_kernel(float* p, uint64_t seed)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= kMlpParams) return;
    const int o1 = kH * kIn, o2 = o1 + kH, o3 = o2 + kH * kH, o4 = o3 + kH, o5 = o4 + kH * kH, o6 = o5 + kH,
              o7 = o6 + kOut * kH;
    int fan = 0;
    if (i < o1) fan = kIn;
    else if (i >= o2 && i < o3) fan = kH;
    else if (i >= o4 && i < o5) fan = kH;
    else if (i >= o6 && i < o7) fan = kH;
    if (fan == 0) {
        p[i] = 0.f;
        return;
    }
    const dm::w2 w = dm::block_words(seed, (uint32_t)i, 0, kMlpInit, 0, 0);
    double z0, z1;
    dm::normal_pair(w.a, z0, z1);
    p[i] = (float)(z0 / __builtin_sqrt((double)fan));
}

constexpr int kScan = 1024;

// One workgroup: exclusive prefix of the per-wave popcounts.
__global__ __launch_bounds__(kScan) void mask_scan_kernel(MaskArgs a)
{
    __shared__ unsigned long long part[kScan];
    const uint32_t nW = (a.count + kWave - 1) / kWave;
    const uint32_t per = (nW + kScan - 1) / kScan;
    const uint32_t t = threadIdx.x;
    const uint32_t w0 = min(nW, t * per), w1 = min(nW, w0 + per);
    unsigned long long s = 0;
    for (uint32_t w = w0; w < w1; ++w) s += __popcll(a.wave_mask[w]);
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < kScan; off <<= 1) {
        const unsigned long long v = t >= (uint32_t)off ? part[t - off] : 0ull;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    unsigned long long run = part[t] - s;
    for (uint32_t w = w0; w < w1; ++w) {
        a.wave_off[w] = (uint32_t)run;
        run += __popcll(a.wave_mask[w]);
    }
    if (t == kScan - 1) *a.total = part[t];
}

__global__ __launch_bounds__(kBlock) void mask_list_kernel(MaskArgs a)
{
    const uint32_t p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= a.count) return;
    const unsigned long long mask = a.wave_mask[p / kWave];
    const uint32_t lane = p % kWave;
    if (!((mask >> lane) & 1ull)) return;
    const unsigned long long below = lane ? (mask & ((1ull << lane) - 1ull)) : 0ull;
    a.list[a.wave_off[p / kWave] + (uint32_t)__popcll(below)] = p;
}

__global__ __launch_bounds__(kBlock) void screen_scatter_kernel(ScreenScatterArgs a)
{
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= a.nkept) return;
    const unsigned long long mask = a.wave_mask[i / kWave];
    const uint32_t lane = i % kWave;
    if (!((mask >> lane) & 1ull)) return;
    const unsigned long long below = lane ? (mask & ((1ull << lane) - 1ull)) : 0ull;
    const unsigned long long gr = a.base_rank + a.wave_off[i / kWave] + (unsigned long long)__popcll(below);
    if (gr >= (unsigned long long)a.N) return;
    const uint32_t pos = a.kept[i];
    const double* su = a.pu + (size_t)pos * kNP;
    double* du = a.pop.u + (size_t)gr * kNP;
#pragma unroll
    for (int q = 0; q < kNP; ++q) du[q] = su[q];
    a.pop.d[gr] = a.kd[i];
    a.pop.sigma[gr] = a.psigma[pos];
    a.pop.parent[gr] = a.pparent[pos];
    a.pop.index[gr] = a.base + pos;
    a.pop.att[gr] = a.patt[pos];
    a.pop_audit[gr] = a.paudit[pos];
    if (gr == (unsigned long long)(a.N - 1)) a.ctr->proposals = (unsigned long long)a.base + pos + 1ull;
}

__global__ __launch_bounds__(kBlock) void audit_weight_kernel(double* logw, const unsigned char* audit, int32_t N,
                                                              double add)
{
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j < N && audit[j]) logw[j] += add;
}

__global__ __launch_bounds__(kBlock) void fill_u8_kernel(unsigned char* p, uint8_t v, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace

void launch_mask_list(const MaskArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(mask_scan_kernel, dim3(1), dim3(kScan), 0, s, a);
    if (a.list && a.count)
        hipLaunchKernelGGL(mask_list_kernel, dim3((a.count + kBlock - 1) / kBlock), dim3(kBlock), 0, s, a);
}

void launch_screen_scatter(const ScreenScatterArgs& a, hipStream_t s)
{
    if (a.nkept == 0) return;
    hipLaunchKernelGGL(screen_scatter_kernel, dim3((a.nkept + kBlock - 1) / kBlock), dim3(kBlock), 0, s, a);
}

void launch_audit_weight(double* logw, const unsigned char* audit, int32_t N, double add, hipStream_t s)
{
    hipLaunchKernelGGL(audit_weight_kernel, dim3((N + kBlock - 1) / kBlock), dim3(kBlock), 0, s, logw, audit, N, add);
}

void launch_perturb_only(const PerturbArgs& a, hipStream_t s)
{
    if (a.count == 0) return;
    hipLaunchKernelGGL(perturb_only_kernel, dim3((a.count + kBlock - 1) / kBlock), dim3(kBlock), 0, s, a);
}

void launch_keep(const KeepArgs& a, hipStream_t s)
{
    if (a.count == 0) return;
    hipLaunchKernelGGL(keep_kernel, dim3((a.count + kBlock - 1) / kBlock), dim3(kBlock), 0, s, a);
}

void launch_sim_kept(const SimKeptArgs& a, hipStream_t s)
{
    if (a.n == 0) return;
    const dim3 grid((a.n + kBlock - 1) / kBlock);
    if (a.tune_x)
        hipLaunchKernelGGL(sim_kept_kernel<true>, grid, dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL(sim_kept_kernel<false>, grid, dim3(kBlock), 0, s, a);
}

void launch_train_data(const TrainDataArgs& a, hipStream_t s)
{
    if (a.n == 0) return;
    hipLaunchKernelGGL(train_data_kernel, dim3((unsigned)((a.n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, a);
}

void launch_mlp_init(float* p, uint64_t seed, hipStream_t s)
{
    hipLaunchKernelGGL(mlp_init_kernel, dim3((kMlpParams + kBlock - 1) / kBlock), dim3(kBlock), 0, s, p, seed);
}

void launch_fill_u8(unsigned char* p, uint8_t v, int64_t n, hipStream_t s)
{
    if (n == 0) return;
    hipLaunchKernelGGL(fill_u8_kernel, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, p, v, n);
}

}  // namespace abcsmc
