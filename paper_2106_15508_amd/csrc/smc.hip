// smc.hip -- SMC stage machinery around the proposal kernel:
//   resample   prior set, eq. 10 weights and the integer CDF of eq. 11
//   weights    N x M importance-weight row sums, LDS-tiled, FP64
//   normalise  W = softmax(log-weights), effective sample size
//   select     exact type-7 percentile of eq. 8 by radix select
#include "dmath.h"
#include "kernels.h"

namespace abcsmc {

namespace {

constexpr int kOne = 1024;  // threads of the single-workgroup kernels

template <typename T>
__device__ __forceinline__ T block_reduce_sum(T v, T* sh)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = kOne / 2; off > 0; off >>= 1) {
        if (t < off) sh[t] += sh[t + off];
        __syncthreads();
    }
    const T r = sh[0];
    __syncthreads();
    return r;
}

__device__ __forceinline__ double block_reduce_max(double v, double* sh)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = kOne / 2; off > 0; off >>= 1) {
        if (t < off) sh[t] = sh[t] > sh[t + off] ? sh[t] : sh[t + off];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// Inclusive scan of one value per thread (Hillis-Steele in LDS).
template <typename T>
__device__ __forceinline__ T block_scan_incl(T v, T* sh)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < kOne; off <<= 1) {
        const T x = t >= off ? sh[t - off] : (T)0;
        __syncthreads();
        sh[t] += x;
        __syncthreads();
    }
    const T r = sh[t];
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------------------
// Prior set of the stage (eq. 9): particles of the previous stage with
// d < eps (d <= eps when none is strictly below); weight eps - d (eq. 10),
// quantised q_k = floor((w_k / w_max) 2^40) (all survivors q = 1 when
// w_max = 0); cdf = inclusive prefix sum of q, exact in uint64 (eq. 11 draws
// r uniform in [0, cdf[N-1]) and takes the first k with cdf[k] > r).  Also
// packs (u_k, q_k) of every q_k > 0 in index order for the weight kernel.
// One workgroup, contiguous chunks per thread.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kOne) void resample_kernel(ResampleArgs a)
{
    __shared__ unsigned long long shu[kOne];
    __shared__ double shd[kOne];
    const int t = threadIdx.x;
    const int N = a.N;
    const double eps = a.eps;
    unsigned long long ns = 0, nle = 0;
    double wmx = 0.0;
    for (int k = t; k < N; k += kOne) {
        const double d = a.d_prev[k];
        if (d < eps) {
            ++ns;
            const double w = eps - d;
            wmx = w > wmx ? w : wmx;
        }
        nle += d <= eps;
    }
    ns = block_reduce_sum(ns, shu);
    nle = block_reduce_sum(nle, shu);
    wmx = block_reduce_max(wmx, shd);
    const bool strict = ns > 0;
    const double wmax = strict ? wmx : 0.0;

    const int chunk = (N + kOne - 1) / kOne;
    const int k0 = min(N, t * chunk), k1 = min(N, k0 + chunk);
    unsigned long long sq = 0, sc = 0;
    for (int k = k0; k < k1; ++k) {
        const double d = a.d_prev[k];
        const bool in = strict ? (d < eps) : (d <= eps);
        unsigned long long q = 0;
        if (in) q = wmax > 0.0 ? (unsigned long long)__builtin_floor(((eps - d) / wmax) * 0x1p40) : 1ull;
        sq += q;
        sc += q > 0;
    }
    const unsigned long long qi = block_scan_incl(sq, shu);
    const unsigned long long ci = block_scan_incl(sc, shu);
    unsigned long long run = qi - sq, col = ci - sc;
    for (int k = k0; k < k1; ++k) {
        const double d = a.d_prev[k];
        const bool in = strict ? (d < eps) : (d <= eps);
        unsigned long long q = 0;
        if (in) q = wmax > 0.0 ? (unsigned long long)__builtin_floor(((eps - d) / wmax) * 0x1p40) : 1ull;
        run += q;
        a.q[k] = q;
        a.cdf[k] = run;
        if (q > 0) {
            double* c = a.cols + (size_t)col * 9;
            const double* up = a.u_prev + (size_t)k * kNP;
#pragma unroll
            for (int dd = 0; dd < kNP; ++dd) c[dd] = up[dd];
            c[8] = (double)q;
            ++col;
        }
    }
    if (t == kOne - 1) {
        a.ctr->survivors = ci;
        a.ctr->fallback = strict ? 0ull : 1ull;
    }
    (void)nle;
}

// ---------------------------------------------------------------------------
// Importance weights.  Row j (an accepted particle with step sigma_j) gets
//   L_j = sum_k q_k exp(-|u_j - u_k|^2 / (2 sigma_j^2))
// over the previous particles with q_k > 0, and log-weight
//   l_j = 8 log sigma_j - log L_j,
// the log of 1 / (proposal density at u_j given sigma_j) up to a constant
// (prior density 1 on the cube).  One lane per row; column tiles of
// (u_k, q_k) stream through LDS and every lane of the wave reads the same
// column (broadcast).  Terms whose exponent is below -708 are exactly 0 and
// skipped; a wave skips the exponential when all its lanes do.  Partial sums
// per tile are added to the row total (two-level summation).
// ---------------------------------------------------------------------------
constexpr int kTile = 256;

__global__ __launch_bounds__(kBlock) void weights_kernel(WeightArgs a)
{
    __shared__ double tu[kNP][kTile];
    __shared__ double tq[kTile];
    const int j = blockIdx.x * kBlock + threadIdx.x;
    const bool active = j < a.N;
    double uj[kNP];
    double ninv = 0.0, sj = 1.0;
    if (active) {
#pragma unroll
        for (int d = 0; d < kNP; ++d) uj[d] = a.u[(size_t)j * kNP + d];
        sj = a.sigma[j];
        ninv = -1.0 / (2.0 * (sj * sj));
    } else {
#pragma unroll
        for (int d = 0; d < kNP; ++d) uj[d] = 0.0;
    }
    const int M = (int)*a.M;
    double total = 0.0;
    for (int c0 = 0; c0 < M; c0 += kTile) {
        const int n = min(kTile, M - c0);
        __syncthreads();
        if (threadIdx.x < n) {
            const double* c = a.cols + (size_t)(c0 + threadIdx.x) * 9;
#pragma unroll
            for (int d = 0; d < kNP; ++d) tu[d][threadIdx.x] = c[d];
            tq[threadIdx.x] = c[8];
        }
        __syncthreads();
        double part = 0.0;
        for (int c = 0; c < n; ++c) {
            double D = 0.0;
#pragma unroll
            for (int d = 0; d < kNP; ++d) {
                const double df = uj[d] - tu[d][c];
                D = __builtin_fma(df, df, D);
            }
            const double arg = D * ninv;
            if (arg >= dm::kExpLo) part = __builtin_fma(tq[c], dm::exp_core(arg), part);
        }
        total += part;
    }
    if (active) a.logw[j] = 8.0 * dm::log(sj) - dm::log(total);
}

// ---------------------------------------------------------------------------
// W_j = exp(l_j - max l) / sum; ESS = 1 / sum W^2.  One workgroup, fixed
// reduction order (deterministic).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kOne) void normalise_kernel(NormArgs a)
{
    __shared__ double sh[kOne];
    const int t = threadIdx.x;
    double mx = -__builtin_inf();
    for (int j = t; j < a.N; j += kOne) mx = a.logw[j] > mx ? a.logw[j] : mx;
    mx = block_reduce_max(mx, sh);
    double s = 0.0;
    for (int j = t; j < a.N; j += kOne) {
        const double e = dm::exp(a.logw[j] - mx);
        a.W[j] = e;
        s += e;
    }
    s = block_reduce_sum(s, sh);
    double s2 = 0.0;
    for (int j = t; j < a.N; j += kOne) {
        const double w = a.W[j] / s;
        a.W[j] = w;
        s2 += w * w;
    }
    s2 = block_reduce_sum(s2, sh);
    if (t == 0) *a.ess = 1.0 / s2;
}

__global__ __launch_bounds__(kBlock) void uniform_weights_kernel(double* W, double* logw, int32_t N)
{
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j < N) {
        W[j] = 1.0 / (double)N;
        logw[j] = 0.0;
    }
}

// ---------------------------------------------------------------------------
// eq. 8 tolerance: type-7 percentile with numpy's "linear" arithmetic:
// v = (N-1) alpha, order statistics x_(floor v) and x_(floor v + 1) found by a
// radix select on the IEEE bit patterns (non-negative doubles order as
// unsigned integers; digits of 11, 11, 11, 11, 11, 9 bits), then
// a + (b-a) g, or b - (b-a)(1-g) when g >= 1/2.  One workgroup; the two
// ranks are selected together.
// ---------------------------------------------------------------------------
constexpr int kBins = 2048;

__global__ __launch_bounds__(kOne) void select_kernel(SelectArgs a)
{
    __shared__ unsigned int hist[2][kBins];
    __shared__ unsigned long long s_pref[2], s_mask[2], s_rank[2];
    const int t = threadIdx.x;
    const int N = a.N;
    const double v = ((double)N - 1.0) * a.alpha;
    long long r0, r1;
    if (v >= (double)N - 1.0) {
        r0 = r1 = N - 1;
    } else if (v < 0.0) {
        r0 = r1 = 0;
    } else {
        r0 = (long long)__builtin_floor(v);
        r1 = r0 + 1;
    }
    if (t < 2) {
        s_pref[t] = 0;
        s_mask[t] = 0;
        s_rank[t] = (unsigned long long)(t == 0 ? r0 : r1);
    }
    for (int pass = 0; pass < 6; ++pass) {
        for (int b = t; b < 2 * kBins; b += kOne) (&hist[0][0])[b] = 0;
        __syncthreads();
        const int sh = pass < 5 ? 53 - 11 * pass : 0;
        const unsigned long long dmask = (1ull << (pass < 5 ? 11 : 9)) - 1ull;
        const unsigned long long p0 = s_pref[0], m0 = s_mask[0], p1 = s_pref[1], m1 = s_mask[1];
        for (int k = t; k < N; k += kOne) {
            const unsigned long long bits = (unsigned long long)__double_as_longlong(a.x[k]);
            const unsigned int dig = (unsigned int)((bits >> sh) & dmask);
            if ((bits & m0) == p0) atomicAdd(&hist[0][dig], 1u);
            if ((bits & m1) == p1) atomicAdd(&hist[1][dig], 1u);
        }
        __syncthreads();
        if (t < 2) {
            unsigned long long rem = s_rank[t], cum = 0;
            int b = 0;
            for (; b < (int)(dmask + 1); ++b) {
                if (cum + hist[t][b] > rem) break;
                cum += hist[t][b];
            }
            s_rank[t] = rem - cum;
            s_pref[t] |= (unsigned long long)b << sh;
            s_mask[t] |= dmask << sh;
        }
        __syncthreads();
    }
    if (t == 0) {
        const double xa = __longlong_as_double((long long)s_pref[0]);
        const double xb = __longlong_as_double((long long)s_pref[1]);
        double res;
        if (r0 == r1) {
            res = xa;
        } else {
            const double g = v - __builtin_floor(v);
            const double diff = xb - xa;
            res = g >= 0.5 ? xb - diff * (1.0 - g) : xa + diff * g;
        }
        *a.out = res;
    }
}

// theta_d = lo_d + u_d (hi_d - lo_d) for the copy-out of a population.
__global__ __launch_bounds__(kBlock) void to_theta_kernel(const double* u, Model m, double* theta, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n * kNP) return;
    const int d = (int)(i % kNP);
    theta[i] = m.lo[d] + u[i] * m.width[d];
}

}  // namespace

void launch_to_theta(const double* u, const Model& m, double* theta, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(to_theta_kernel, dim3((unsigned)((n * kNP + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                       u, m, theta, n);
}

void launch_resample(const ResampleArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(resample_kernel, dim3(1), dim3(kOne), 0, s, a);
}

void launch_weights(const WeightArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(weights_kernel, dim3((a.N + kBlock - 1) / kBlock), dim3(kBlock), 0, s, a);
}

void launch_normalise(const NormArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(normalise_kernel, dim3(1), dim3(kOne), 0, s, a);
}

void launch_uniform_weights(double* W, double* logw, int32_t N, hipStream_t s)
{
    hipLaunchKernelGGL(uniform_weights_kernel, dim3((N + kBlock - 1) / kBlock), dim3(kBlock), 0, s, W,
                       logw, N);
}

void launch_select(const SelectArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(select_kernel, dim3(1), dim3(kOne), 0, s, a);
}

}  // namespace abcsmc
