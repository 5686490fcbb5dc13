// sim.hip -- proposal kernel (perturb + simulate + distance + accept, one
// wave64 lane per proposal), ordered compaction of acceptances, trajectory
// kernel and the primitive test hook.
#include "dmath.h"
#include "kernels.h"
#include "propose.h"

namespace abcsmc {

namespace {

// ---------------------------------------------------------------------------
// Proposal kernel of one batch: lane p makes proposal j = base + p and
// publishes the wave's acceptance ballot for the ordered compaction.
// ---------------------------------------------------------------------------
// Waves per SIMD the register allocation aims for.  The kernel needs 156
// VGPRs, so three waves per SIMD are resident whether two or three are asked
// for; asking for two gave a slightly different instruction schedule that ran
// 1.8% faster, and asking for four (128 VGPRs) was 6% slower.
#ifndef ABCSMC_PROPOSE_WAVES
#define ABCSMC_PROPOSE_WAVES 2
#endif

template <bool kRound0, int kSampler>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(ABCSMC_PROPOSE_WAVES)))
void propose_kernel(ProposeArgs a)
{
    const uint32_t p = blockIdx.x * kBlock + threadIdx.x;
    const bool active = p < a.count;
    const uint32_t j = a.base + p;
    const lane::ProposalIn in{a.obs,    a.round,  a.max_attempts, a.eps,   a.exit_thr,          a.u_prev,
                              a.cdf,    a.n_prev, a.beta_a,       a.beta_b, a.step_is_variance, a.s_fixed, a.beta_b_real};
    lane::ProposalOut o;
    o.valid = false;
    o.acc = false;
    o.days = 0;
    o.att = 0;
    if (active) lane::propose_one<kRound0, kSampler>(a.m, in, j, o);
    if (active) {
        double* su = a.st_u + (size_t)p * kNP;
#pragma unroll
        for (int q = 0; q < kNP; ++q) su[q] = o.u[q];
        a.st_d[p] = o.d;
        a.st_sigma[p] = o.sigma;
        a.st_parent[p] = o.parent;
        a.st_att[p] = o.att;
    }
    const unsigned long long mask = __ballot(o.acc);
    const unsigned long long inv = lane::wave_sum_u64((active && !o.valid) ? 1ull : 0ull);
    const unsigned long long natt = lane::wave_sum_u64(active ? (unsigned long long)(o.att < 0 ? -o.att : o.att) : 0ull);
    const unsigned long long ndays = lane::wave_sum_u64((unsigned long long)o.days);
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
    lane::simulate_distance<kSampler, true>(a.m, th, nullptr, a.round, a.index0 + (uint32_t)k,
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
    case 13: {
        const double* ab = (const double*)in;
        y[i] = dm::beta_general(ab[0], ab[1], (uint64_t)pa, (uint32_t)i, (uint32_t)pb, 0);
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

int64_t propose_first_batch_lanes()
{
    int dev = 0, cus = 0, blocks = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, propose_kernel<false, 0>, kBlock, 0) != hipSuccess ||
        blocks < 1) {
        (void)hipGetLastError();
        return 0;
    }
    return (int64_t)cus * blocks * kBlock;
}

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
    if (fn == 14) {
        launch_wterm_debug(n, (const double*)in, (double*)out, s);
        return;
    }
    hipLaunchKernelGGL(debug_eval_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, fn, n, in, out, pa, pb);
}

}  // namespace abcsmc
