// smc.hip -- SMC stage machinery around the proposal kernel:
//   resample   prior set, eq. 10 weights and the integer CDF of eq. 11
//   weights    N x M importance-weight row sums, LDS-tiled, FP64
//   normalise  W = softmax(log-weights), effective sample size
//   select     exact type-7 percentile of eq. 8 by radix select
// All reductions combine per-block partials in a fixed order, so every result
// is bitwise reproducible run to run.
#include "dmath.h"
#include "kernels.h"
#include "wterm.h"

namespace abcsmc {

namespace {

constexpr int kChunk = 1024;            // elements per block of the resample kernels
constexpr int kPer = kChunk / kBlock;   // elements per thread (contiguous)

__device__ __forceinline__ unsigned long long block_sum_u64(unsigned long long v, unsigned long long* sh)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (t < off) sh[t] += sh[t + off];
        __syncthreads();
    }
    const unsigned long long r = sh[0];
    __syncthreads();
    return r;
}

__device__ __forceinline__ double block_sum_f64(double v, double* sh)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (t < off) sh[t] += sh[t + off];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

__device__ __forceinline__ double block_max_f64(double v, double* sh)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (t < off) sh[t] = sh[t] > sh[t + off] ? sh[t] : sh[t + off];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// Exclusive scan of one value per thread (Hillis-Steele in LDS); *total gets the sum.
__device__ __forceinline__ unsigned long long block_excl_scan_u64(unsigned long long v, unsigned long long* sh,
                                                                  unsigned long long* total)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {
        const unsigned long long x = t >= off ? sh[t - off] : 0ull;
        __syncthreads();
        sh[t] += x;
        __syncthreads();
    }
    const unsigned long long incl = sh[t];
    *total = sh[kBlock - 1];
    __syncthreads();
    return incl - v;
}

// ---------------------------------------------------------------------------
// Prior set of the stage (eq. 9): particles of the previous stage with
// d < eps (d <= eps when none is strictly below); weight eps - d (eq. 10),
// quantised q_k = floor((w_k / w_max) 2^40) (all survivors q = 1 when
// w_max = 0); cdf = inclusive prefix sum of q, exact in uint64 (eq. 11 draws
// r uniform in [0, cdf[N-1]) and takes the first k with cdf[k] > r).  Also
// packs (u_k, q_k) of every q_k > 0 in index order for the weight kernel.
// Three passes over blocks of 1024 particles: statistics, per-block sums,
// write-out with the block's exclusive offset.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void resample_stats_kernel(ResampleArgs a)
{
    __shared__ unsigned long long shu[kBlock];
    __shared__ double shd[kBlock];
    const int k0 = blockIdx.x * kChunk;
    unsigned long long ns = 0;
    double wmx = 0.0;
    for (int i = 0; i < kPer; ++i) {
        const int k = k0 + i * kBlock + threadIdx.x;
        if (k < a.N) {
            const double d = a.d_prev[k];
            if (d < a.eps) {
                ++ns;
                const double w = a.eps - d;
                wmx = w > wmx ? w : wmx;
            }
        }
    }
    ns = block_sum_u64(ns, shu);
    wmx = block_max_f64(wmx, shd);
    if (threadIdx.x == 0) {
        a.sc.u0[blockIdx.x] = ns;
        a.sc.d0[blockIdx.x] = wmx;
    }
}

// Global prior-set mode from the per-block statistics (same order in every block).
__device__ __forceinline__ void resample_mode(const ResampleArgs& a, bool& strict, double& wmax,
                                              unsigned long long* shu, double* shd)
{
    const int G = gridDim.x;
    unsigned long long ns = 0;
    double wmx = 0.0;
    for (int b = threadIdx.x; b < G; b += kBlock) {
        ns += a.sc.u0[b];
        wmx = a.sc.d0[b] > wmx ? a.sc.d0[b] : wmx;
    }
    ns = block_sum_u64(ns, shu);
    wmx = block_max_f64(wmx, shd);
    strict = ns > 0;
    wmax = strict ? wmx : 0.0;
}

__device__ __forceinline__ unsigned long long quantise(double d, double eps, bool strict, double wmax)
{
    const bool in = strict ? (d < eps) : (d <= eps);
    if (!in) return 0ull;
    return wmax > 0.0 ? (unsigned long long)__builtin_floor(((eps - d) / wmax) * 0x1p40) : 1ull;
}

__global__ __launch_bounds__(kBlock) void resample_count_kernel(ResampleArgs a)
{
    __shared__ unsigned long long shu[kBlock];
    __shared__ double shd[kBlock];
    bool strict;
    double wmax;
    resample_mode(a, strict, wmax, shu, shd);
    const int k0 = blockIdx.x * kChunk + threadIdx.x * kPer;
    unsigned long long sq = 0, sc = 0;
    for (int i = 0; i < kPer; ++i) {
        const int k = k0 + i;
        if (k < a.N) {
            const unsigned long long q = quantise(a.d_prev[k], a.eps, strict, wmax);
            sq += q;
            sc += q > 0;
        }
    }
    sq = block_sum_u64(sq, shu);
    sc = block_sum_u64(sc, shu);
    if (threadIdx.x == 0) {
        a.sc.u1[blockIdx.x] = sq;
        a.sc.u2[blockIdx.x] = sc;
    }
}

__global__ __launch_bounds__(kBlock) void resample_write_kernel(ResampleArgs a)
{
    __shared__ unsigned long long shu[kBlock];
    __shared__ double shd[kBlock];
    bool strict;
    double wmax;
    resample_mode(a, strict, wmax, shu, shd);
    // exclusive offsets of this block (and the survivor total for the last block)
    const int G = gridDim.x;
    unsigned long long oq = 0, oc = 0, tc = 0;
    for (int b = threadIdx.x; b < G; b += kBlock) {
        const unsigned long long q = a.sc.u1[b], c = a.sc.u2[b];
        if (b < (int)blockIdx.x) {
            oq += q;
            oc += c;
        }
        tc += c;
    }
    oq = block_sum_u64(oq, shu);
    oc = block_sum_u64(oc, shu);
    tc = block_sum_u64(tc, shu);
    const int k0 = blockIdx.x * kChunk + threadIdx.x * kPer;
    unsigned long long q[kPer];
    unsigned long long sq = 0, sc = 0;
    for (int i = 0; i < kPer; ++i) {
        const int k = k0 + i;
        q[i] = k < a.N ? quantise(a.d_prev[k], a.eps, strict, wmax) : 0ull;
        sq += q[i];
        sc += q[i] > 0;
    }
    unsigned long long tot;
    unsigned long long run = oq + block_excl_scan_u64(sq, shu, &tot);
    unsigned long long col = oc + block_excl_scan_u64(sc, shu, &tot);
    for (int i = 0; i < kPer; ++i) {
        const int k = k0 + i;
        if (k >= a.N) break;
        run += q[i];
        a.q[k] = q[i];
        a.cdf[k] = run;
        if (q[i] > 0) {
            double* c = a.cols + (size_t)col * 9;
            const double* up = a.u_prev + (size_t)k * kNP;
#pragma unroll
            for (int dd = 0; dd < kNP; ++dd) c[dd] = up[dd];
            c[8] = (double)q[i];
            ++col;
        }
    }
    if (blockIdx.x == (unsigned)(G - 1) && threadIdx.x == 0) {
        a.ctr->survivors = tc;
        a.ctr->fallback = strict ? 0ull : 1ull;
    }
}

// ---------------------------------------------------------------------------
// Importance weights.  Row j (an accepted particle with step sigma_j) gets
//   L_j = sum_k q_k exp(-|u_j - u_k|^2 / (2 sigma_j^2))
// over the previous particles with q_k > 0, and log-weight
//   l_j = 8 log sigma_j - log L_j,
// the log of 1 / (proposal density at u_j given sigma_j) up to a constant
// (prior density 1 on the cube).  One lane per row; the columns are split in
// `chunks` contiguous ranges (grid y) so the launch fills the chip; every lane
// of a wave reads the same column through scalar loads.  Four columns are
// evaluated per step into even/odd partial sums; per-chunk partial sums are
// added in a fixed order.
//
// The exponential here is table driven (1024 entries of 2^(i/1024) in LDS and
// a cubic in the remainder).  Its relative error (a few 1e-16) is far inside
// the 1e-12 the weights are held to; the trajectories never use it.
// ---------------------------------------------------------------------------
using wterm::kTile;
using wterm::coord_key32;
using wterm::lower_index;
using wterm::sigma_half_octave;
using wterm::wave_max;
using wterm::wave_min;
using wterm::wave_sum_u64;

// ---- windowed evaluation -------------------------------------------------
// Row j only needs the columns whose coordinate d* lies within its
// half-width R_j = W_j sigma_j of u_jd*: every other column has a term at
// most q_k e^{-W_j^2/2}, and W_j is chosen from the row's own parent term so
// that all of them together stay below 2^-53 of the row sum (at most 37.7,
// where every omitted exponential is below e^-710).  Per stage: pick the
// coordinate d* with the largest spread among the columns (the windows then
// exclude the most columns: sigma is the same in every coordinate), sort the
// columns by it, sort the rows by (half-octave of sigma, descending; u_d*), and let every
// workgroup (128 consecutive sorted rows) visit only the union of its rows'
// windows; a wave also skips tiles outside its own lanes' union.

constexpr int kDimBlocks = 256;

__global__ __launch_bounds__(kBlock) void wdim_partial_kernel(WeightArgs a)
{
    __shared__ double sh[kBlock];
    const int M = (int)*a.M;
    double s1[kNP], s2[kNP];
#pragma unroll
    for (int d = 0; d < kNP; ++d) s1[d] = s2[d] = 0.0;
    for (int k = blockIdx.x * kBlock + threadIdx.x; k < M; k += gridDim.x * kBlock) {
#pragma unroll
        for (int d = 0; d < kNP; ++d) {
            const double v = a.cols[(size_t)k * 9 + d];
            s1[d] += v;
            s2[d] += v * v;
        }
    }
    for (int d = 0; d < kNP; ++d) {
        const double t1 = block_sum_f64(s1[d], sh);
        const double t2 = block_sum_f64(s2[d], sh);
        if (threadIdx.x == 0) {
            a.dimpart[blockIdx.x * 16 + d] = t1;
            a.dimpart[blockIdx.x * 16 + 8 + d] = t2;
        }
    }
}

__global__ __launch_bounds__(kBlock) void wdim_pick_kernel(WeightArgs a)
{
    __shared__ double sh[kBlock];
    const int M = (int)*a.M;
    double best = -1.0;
    int bd = 0;
    for (int d = 0; d < kNP; ++d) {
        const double t1 = block_sum_f64(threadIdx.x < kDimBlocks ? a.dimpart[threadIdx.x * 16 + d] : 0.0, sh);
        const double t2 = block_sum_f64(threadIdx.x < kDimBlocks ? a.dimpart[threadIdx.x * 16 + 8 + d] : 0.0, sh);
        const double mean = t1 / (double)M;
        const double var = t2 / (double)M - mean * mean;
        if (var > best) {
            best = var;
            bd = d;
        }
    }
    if (threadIdx.x == 0) *a.dstar = bd;
}

__global__ __launch_bounds__(kBlock) void wcolkeys_kernel(WeightArgs a)
{
    const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= a.npad) return;
    const int M = (int)*a.M;
    const int ds = *a.dstar;
    a.colkeys[i] = i < (size_t)M ? (coord_key32(a.cols[i * 9 + ds]) << 32) | (unsigned long long)i : ~0ull;
}

__global__ __launch_bounds__(kBlock) void wcolgather_kernel(WeightArgs a)
{
    const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    const int M = (int)*a.M;
    if (i >= (size_t)M) return;
    const int ds = *a.dstar;
    const size_t src = (size_t)(a.colkeys[i] & 0xFFFFFFFFull);
    const double* c = a.cols + src * 9;
    double* o = a.scols + i * 9;
#pragma unroll
    for (int d = 0; d < 9; ++d) o[d] = c[d];
    a.skey[i] = c[ds];
}

__global__ __launch_bounds__(kBlock) void wrowkeys_kernel(WeightArgs a)
{
    const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= a.npad) return;
    if (i >= (size_t)a.N) {
        a.rowkeys[i] = ~0ull;
        return;
    }
    const int ds = *a.dstar;
    // half-octaves in descending order: the widest windows are dispatched first
    const unsigned long long hi =
        ((127ull - sigma_half_octave(a.sigma[i])) << 25) | (coord_key32(a.u[i * kNP + ds]) >> 7);
    a.rowkeys[i] = (hi << 32) | (unsigned long long)i;
    double uj[kNP];
#pragma unroll
    for (int d = 0; d < kNP; ++d) uj[d] = a.u[i * kNP + d];
    const int32_t par = a.parent[i];
    const bool ok = par >= 0 && par < a.n_prev;
    a.rwin[i] = wterm::window_halfwidth(uj, a.sigma[i], ok ? a.u_prev + (size_t)par * kNP : uj,
                                        ok ? (double)a.q_prev[par] : 0.0, (double)a.cdf[a.n_prev - 1]);
}

// Window of each row block (kWeightRows consecutive sorted rows): the sorted
// column range that can hold a nonzero term for any of its rows.
__global__ __launch_bounds__(kWeightRows) void wwindow_kernel(WeightArgs a)
{
    __shared__ double slo[kWeightRows / kWave], shi[kWeightRows / kWave];
    const int r = blockIdx.x * kWeightRows + threadIdx.x;
    const int ds = *a.dstar;
    const int M = (int)*a.M;
    double lo = __builtin_inf(), hi = -__builtin_inf();
    unsigned long long own = 0;  // columns of this row's own window
    if (r < a.N) {
        const size_t j = (size_t)(a.rowkeys[r] & 0xFFFFFFFFull);
        const double R = a.rwin[j];
        const double x = a.u[j * kNP + ds];
        lo = x - R;
        hi = x + R;
        own = (unsigned long long)(lower_index(a.skey, M, hi, true) - lower_index(a.skey, M, lo, false));
    }
    own = wave_sum_u64(own);
    if ((threadIdx.x & (kWave - 1)) == 0 && own) atomicAdd(a.window_terms, own);
    lo = wave_min(lo);
    hi = wave_max(hi);
    if ((threadIdx.x & (kWave - 1)) == 0) {
        slo[threadIdx.x / kWave] = lo;
        shi[threadIdx.x / kWave] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < kWeightRows / kWave; ++q) {
            lo = slo[q] < lo ? slo[q] : lo;
            hi = shi[q] > hi ? shi[q] : hi;
        }
        lo = slo[0] < lo ? slo[0] : lo;
        hi = shi[0] > hi ? shi[0] : hi;
        a.win[blockIdx.x] = make_int2(lower_index(a.skey, M, lo, false), lower_index(a.skey, M, hi, true));
    }
}

// grid (row blocks, chunks): block (b, c) sums columns
// [first_b + c CH, min(end_b, first_b + (c+1) CH)) for its kWeightRows rows
// (two waves: 128-row blocks keep the windows tighter than 256-row ones, 3.5%
// faster at N = 131072); chunks past the window leave at once.
__global__ __launch_bounds__(kWeightRows) void weights_kernel(WeightArgs a)
{
    __shared__ double T[wterm::kTab];
    const int r = blockIdx.x * kWeightRows + threadIdx.x;   // sorted row position
    const bool active = r < a.N;
    const int2 wnd = a.win[blockIdx.x];
    const int k0 = wnd.x + (int)blockIdx.y * a.cols_per_chunk;
    const int k1 = min(wnd.y, k0 + a.cols_per_chunk);
    if (k0 >= k1) return;  // past the window: the finalize pass does not read this chunk
    wterm::load_table(T, a.tab);
    __syncthreads();
    const int ds = *a.dstar;
    double uj[kNP];
    double cj = 0.0, lo = __builtin_inf(), hi = -__builtin_inf();
    if (active) {
        const size_t j = (size_t)(a.rowkeys[r] & 0xFFFFFFFFull);
#pragma unroll
        for (int d = 0; d < kNP; ++d) uj[d] = a.u[j * kNP + d];
        const double sj = a.sigma[j];
        cj = wterm::row_scale(sj, a.ex);
        const double R = a.rwin[j];
        lo = uj[ds] - R;
        hi = uj[ds] + R;
    } else {
#pragma unroll
        for (int d = 0; d < kNP; ++d) uj[d] = 0.0;
    }
    const double wlo = wave_min(lo), whi = wave_max(hi);
    const unsigned long long lanes = (unsigned long long)__popcll(__ballot(active));
    unsigned long long evaluated = 0;
    // read-only for the whole launch: constant address space, so the
    // wave-uniform column reads become scalar loads
    const double total = wterm::row_sum(uj, cj, (wterm::const_col_ptr)a.scols, (wterm::const_col_ptr)a.skey, k0,
                                        k1, wlo, whi, T, a.ex, lanes, evaluated);
    if (active) a.partial[(size_t)blockIdx.y * a.N + r] = total;
    if ((threadIdx.x & (kWave - 1)) == 0 && evaluated) atomicAdd(a.terms, evaluated);
}

__global__ __launch_bounds__(kBlock) void wtable_kernel(double* tab)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < wterm::kTab) tab[i] = wterm::table_entry(i);
}

// Test hook: one importance-weight term per record {u_j[8], sigma_j, u_k[8],
// q_k}, by the weight kernels' own term code (table exponential from LDS,
// scaled by the row's c_j), accumulated as the first term of a row sum.
__global__ __launch_bounds__(kBlock) void wterm_debug_kernel(int64_t n, const double* in, double* out, WeightArgs a)
{
    __shared__ double T[wterm::kTab];
    for (int i = threadIdx.x; i < wterm::kTab; i += kBlock) T[i] = wterm::table_entry(i);
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const double* r = in + (size_t)i * 18;
    double uj[kNP];
    wterm::Col c;
#pragma unroll
    for (int d = 0; d < kNP; ++d) {
        uj[d] = r[d];
        c.u[d] = r[9 + d];
    }
    c.q = r[17];
    const double cj = wterm::row_scale(r[8], a.ex);
    out[i] = __builtin_fma(c.q, wterm::term_exp(uj, cj, c, T, a.ex), 0.0);
}

__global__ __launch_bounds__(kBlock) void weights_finalize_kernel(WeightArgs a)
{
    const int r = blockIdx.x * kBlock + threadIdx.x;
    if (r >= a.N) return;
    // the chunks that overlap the row block's window, in order
    const int2 wnd = a.win[r / kWeightRows];
    const int len = wnd.y > wnd.x ? wnd.y - wnd.x : 0;
    const int nch = min(a.chunks, (len + a.cols_per_chunk - 1) / a.cols_per_chunk);
    double L = 0.0;
    for (int c = 0; c < nch; ++c) L += a.partial[(size_t)c * a.N + r];
    const size_t j = (size_t)(a.rowkeys[r] & 0xFFFFFFFFull);
    a.logw[j] = 8.0 * dm::log(a.sigma[j]) - dm::log(L);
}

// ---------------------------------------------------------------------------
// W_j = exp(l_j - max l) / sum; ESS = 1 / sum W^2.  Per-block partials
// combined in block order.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void norm_max_kernel(NormArgs a)
{
    __shared__ double sh[kBlock];
    double mx = -__builtin_inf();
    for (int i = 0; i < kPer; ++i) {
        const int j = blockIdx.x * kChunk + i * kBlock + threadIdx.x;
        if (j < a.N) mx = a.logw[j] > mx ? a.logw[j] : mx;
    }
    mx = block_max_f64(mx, sh);
    if (threadIdx.x == 0) a.sc.d0[blockIdx.x] = mx;
}

__global__ __launch_bounds__(kBlock) void norm_exp_kernel(NormArgs a)
{
    __shared__ double sh[kBlock];
    double mx = -__builtin_inf();
    for (int b = threadIdx.x; b < (int)gridDim.x; b += kBlock) mx = a.sc.d0[b] > mx ? a.sc.d0[b] : mx;
    mx = block_max_f64(mx, sh);
    double s = 0.0;
    for (int i = 0; i < kPer; ++i) {
        const int j = blockIdx.x * kChunk + i * kBlock + threadIdx.x;
        if (j < a.N) {
            const double e = dm::exp(a.logw[j] - mx);
            a.W[j] = e;
            s += e;
        }
    }
    s = block_sum_f64(s, sh);
    if (threadIdx.x == 0) a.sc.d1[blockIdx.x] = s;
}

__device__ __forceinline__ double ordered_total(const double* part, int G, double* sh)
{
    // each thread sums a contiguous run of block partials, then a fixed tree
    const int per = (G + kBlock - 1) / kBlock;
    double s = 0.0;
    const int b0 = threadIdx.x * per, b1 = min(G, b0 + per);
    for (int b = b0; b < b1; ++b) s += part[b];
    return block_sum_f64(s, sh);
}

__global__ __launch_bounds__(kBlock) void norm_scale_kernel(NormArgs a)
{
    __shared__ double sh[kBlock];
    const double total = ordered_total(a.sc.d1, gridDim.x, sh);
    double s2 = 0.0;
    for (int i = 0; i < kPer; ++i) {
        const int j = blockIdx.x * kChunk + i * kBlock + threadIdx.x;
        if (j < a.N) {
            const double w = a.W[j] / total;
            a.W[j] = w;
            s2 += w * w;
        }
    }
    s2 = block_sum_f64(s2, sh);
    if (threadIdx.x == 0) a.sc.d0[blockIdx.x] = s2;
}

__global__ __launch_bounds__(kBlock) void norm_ess_kernel(NormArgs a, int G)
{
    __shared__ double sh[kBlock];
    const double s2 = ordered_total(a.sc.d0, G, sh);
    if (threadIdx.x == 0) *a.ess = 1.0 / s2;
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
// unsigned integers; digits of 11, 11, 11, 11, 11, 9 bits from the top), then
// a + (b-a) g, or b - (b-a)(1-g) when g >= 1/2.  Per pass: every block
// histograms its slice in LDS and adds it to the global bins; one block then
// picks the digit of both ranks.
// ---------------------------------------------------------------------------
constexpr int kBins = 2048;
enum { kPref0 = 0, kPref1, kMask0, kMask1, kRank0, kRank1, kR0, kR1 };

__device__ __forceinline__ int pass_shift(int pass) { return pass < 5 ? 53 - 11 * pass : 0; }
__device__ __forceinline__ unsigned long long pass_mask(int pass) { return (1ull << (pass < 5 ? 11 : 9)) - 1ull; }

__global__ __launch_bounds__(kBlock) void select_init_kernel(SelectArgs a)
{
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
    for (int b = threadIdx.x; b < 2 * kBins; b += kBlock) a.sc.hist[b] = 0u;
    if (threadIdx.x == 0) {
        unsigned long long* st = a.sc.sel;
        st[kPref0] = st[kPref1] = st[kMask0] = st[kMask1] = 0ull;
        st[kRank0] = (unsigned long long)r0;
        st[kRank1] = (unsigned long long)r1;
        st[kR0] = (unsigned long long)r0;
        st[kR1] = (unsigned long long)r1;
    }
}

__global__ __launch_bounds__(kBlock) void select_hist_kernel(SelectArgs a, int pass)
{
    __shared__ unsigned int h[2][kBins];
    for (int b = threadIdx.x; b < 2 * kBins; b += kBlock) (&h[0][0])[b] = 0u;
    __syncthreads();
    const unsigned long long* st = a.sc.sel;
    const unsigned long long p0 = st[kPref0], p1 = st[kPref1], m0 = st[kMask0], m1 = st[kMask1];
    const int sh = pass_shift(pass);
    const unsigned long long dmk = pass_mask(pass);
    for (int k = blockIdx.x * kBlock + threadIdx.x; k < a.N; k += gridDim.x * kBlock) {
        const unsigned long long bits = (unsigned long long)__double_as_longlong(a.x[k]);
        const unsigned int dig = (unsigned int)((bits >> sh) & dmk);
        if ((bits & m0) == p0) atomicAdd(&h[0][dig], 1u);
        if ((bits & m1) == p1) atomicAdd(&h[1][dig], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < 2 * kBins; b += kBlock) {
        const unsigned int v = (&h[0][0])[b];
        if (v) atomicAdd(&a.sc.hist[b], v);
    }
}

// One block: for each rank find the bin whose cumulative count passes it.
__global__ __launch_bounds__(kBlock) void select_pick_kernel(SelectArgs a, int pass)
{
    __shared__ unsigned long long part[kBlock];
    __shared__ unsigned long long s_bin[2], s_below[2];
    unsigned long long* st = a.sc.sel;
    const int sh = pass_shift(pass);
    const int nb = (int)pass_mask(pass) + 1;
    const int per = (nb + kBlock - 1) / kBlock;  // contiguous bins per thread
    for (int which = 0; which < 2; ++which) {
        const unsigned int* h = a.sc.hist + which * kBins;
        const unsigned long long rank = st[kRank0 + which];
        const int b0 = threadIdx.x * per, b1 = min(nb, b0 + per);
        unsigned long long s = 0;
        for (int b = b0; b < b1; ++b) s += h[b];
        unsigned long long tot;
        unsigned long long run = block_excl_scan_u64(s, part, &tot);
        // the thread whose run contains the rank locates the bin
        for (int b = b0; b < b1; ++b) {
            if (run <= rank && rank < run + h[b]) {
                s_bin[which] = (unsigned long long)b;
                s_below[which] = run;
            }
            run += h[b];
        }
        __syncthreads();
    }
    for (int b = threadIdx.x; b < 2 * kBins; b += kBlock) a.sc.hist[b] = 0u;
    if (threadIdx.x == 0) {
        for (int which = 0; which < 2; ++which) {
            st[kRank0 + which] -= s_below[which];
            st[kPref0 + which] |= s_bin[which] << sh;
            st[kMask0 + which] |= pass_mask(pass) << sh;
        }
        if (pass == 5) {
            const double xa = __longlong_as_double((long long)st[kPref0]);
            const double xb = __longlong_as_double((long long)st[kPref1]);
            double res;
            if (st[kR0] == st[kR1]) {
                res = xa;
            } else {
                const double v = ((double)a.N - 1.0) * a.alpha;
                const double g = v - __builtin_floor(v);
                const double diff = xb - xa;
                res = g >= 0.5 ? xb - diff * (1.0 - g) : xa + diff * g;
            }
            *a.out = res;
        }
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

inline unsigned blocks_of(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

void weight_exp_constants(double ex[7])
{
    const double L = 0.6931471805599453 / 1024.0;  // ln2 / 1024 (exact scaling of the double ln 2)
    ex[0] = L;
    ex[1] = (L * L) / 2.0;
    ex[2] = (L * L * L) / 6.0;
    ex[3] = 1477.3197218702985;           // 1024 / ln 2
    ex[4] = ex[5] = ex[6] = 0.0;
}

int weight_chunks(int64_t N)
{
    const int64_t row_blocks = (N + kBlock - 1) / kBlock;
    int64_t S = (2048 + row_blocks - 1) / row_blocks;
    const int64_t cap = ((int64_t)1 << 23) / N;
    if (S > cap) S = cap;
    if (S > 64) S = 64;
    if (S < 1) S = 1;
    return (int)S;
}

void launch_to_theta(const double* u, const Model& m, double* theta, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(to_theta_kernel, dim3(blocks_of(n * kNP, kBlock)), dim3(kBlock), 0, s, u, m, theta, n);
}

void launch_resample(const ResampleArgs& a, hipStream_t s)
{
    const dim3 g(blocks_of(a.N, kChunk)), b(kBlock);
    hipLaunchKernelGGL(resample_stats_kernel, g, b, 0, s, a);
    hipLaunchKernelGGL(resample_count_kernel, g, b, 0, s, a);
    hipLaunchKernelGGL(resample_write_kernel, g, b, 0, s, a);
}

void launch_weights_window(const WeightArgs& a, hipStream_t s)
{
    const dim3 b(kBlock);
    const unsigned gp = blocks_of((int64_t)a.npad, kBlock);
    hipLaunchKernelGGL(wdim_partial_kernel, dim3(kDimBlocks), b, 0, s, a);
    hipLaunchKernelGGL(wdim_pick_kernel, dim3(1), b, 0, s, a);
    hipLaunchKernelGGL(wcolkeys_kernel, dim3(gp), b, 0, s, a);
    hipLaunchKernelGGL(wrowkeys_kernel, dim3(gp), b, 0, s, a);
    launch_sort_u64_pair(a.colkeys, a.rowkeys, a.npad, s);
    hipLaunchKernelGGL(wcolgather_kernel, dim3(blocks_of(a.N, kBlock)), b, 0, s, a);
    hipLaunchKernelGGL(wwindow_kernel, dim3(blocks_of(a.N, kWeightRows)), dim3(kWeightRows), 0, s, a);
}

void launch_wterm_debug(int64_t n, const double* in, double* out, hipStream_t s)
{
    WeightArgs a{};
    weight_exp_constants(a.ex);
    hipLaunchKernelGGL(wterm_debug_kernel, dim3(blocks_of(n, kBlock)), dim3(kBlock), 0, s, n, in, out, a);
}

void launch_weight_table(double* tab, hipStream_t s)
{
    hipLaunchKernelGGL(wtable_kernel, dim3((wterm::kTab + kBlock - 1) / kBlock), dim3(kBlock), 0, s, tab);
}

void launch_weights_sum(const WeightArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(weights_kernel, dim3(blocks_of(a.N, kWeightRows), a.chunks), dim3(kWeightRows), 0, s, a);
}

void launch_weights_finalize(const WeightArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(weights_finalize_kernel, dim3(blocks_of(a.N, kBlock)), dim3(kBlock), 0, s, a);
}

// Columns per chunk (grid y) of a row block's window: at most 128 chunks of at
// least 1024 columns.  Finer chunks balance the uneven windows across the
// chip (1024-column chunks: 7% faster than 4096 at N = 131072).
int weight_cols_per_chunk(int64_t N)
{
    int64_t ch = 1024;
    while ((N + ch - 1) / ch > 128) ch <<= 1;
    return (int)ch;
}

int weight_window_chunks(int64_t N)
{
    const int64_t ch = weight_cols_per_chunk(N);
    return (int)((N + ch - 1) / ch);
}

void launch_normalise(const NormArgs& a, hipStream_t s)
{
    const unsigned G = blocks_of(a.N, kChunk);
    hipLaunchKernelGGL(norm_max_kernel, dim3(G), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(norm_exp_kernel, dim3(G), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(norm_scale_kernel, dim3(G), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(norm_ess_kernel, dim3(1), dim3(kBlock), 0, s, a, (int)G);
}

void launch_uniform_weights(double* W, double* logw, int32_t N, hipStream_t s)
{
    hipLaunchKernelGGL(uniform_weights_kernel, dim3(blocks_of(N, kBlock)), dim3(kBlock), 0, s, W, logw, N);
}

void launch_select(const SelectArgs& a, hipStream_t s)
{
    unsigned G = blocks_of(a.N, 4 * kBlock);
    if (G > 1024) G = 1024;
    hipLaunchKernelGGL(select_init_kernel, dim3(1), dim3(kBlock), 0, s, a);
    for (int pass = 0; pass < 6; ++pass) {
        hipLaunchKernelGGL(select_hist_kernel, dim3(G), dim3(kBlock), 0, s, a, pass);
        hipLaunchKernelGGL(select_pick_kernel, dim3(1), dim3(kBlock), 0, s, a, pass);
    }
}

}  // namespace abcsmc
