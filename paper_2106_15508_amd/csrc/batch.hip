// batch.hip -- kernels of the batched mode.  One stage of every run is the
// fixed sequence
//   begin -> [resample x3] -> propose (persistent) -> compact scan -> scatter
//         -> [weights -> finalize -> normalise | uniform] -> select -> end
// reading the stage index and per-run state from device memory, so the host
// captures it once in a graph and replays it per stage.  Per run the
// arithmetic is exactly the single-run path's (same per-lane proposal code,
// same first-N-in-index-order cut, same integer CDF and percentile), so a run
// gives the same bits batched or alone; only the weights' summation order
// differs (1e-12).
#include "batch.h"
#include "blockselect.h"
#include "dmath.h"
#include "propose.h"
#include "wterm.h"

namespace abcsmc {

namespace {

__device__ __forceinline__ unsigned long long ld_relaxed(const unsigned long long* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int ld_relaxed_i(const int* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
__device__ __forceinline__ T bsum(T v, T* sh)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (t < off) sh[t] += sh[t + off];
        __syncthreads();
    }
    const T r = sh[0];
    __syncthreads();
    return r;
}

__device__ __forceinline__ double bmax(double v, double* sh)
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

using bsel::bscan_excl;

// ------------------------------------------------------------------ begin/end

// Stage set-up of every run: tolerance (eps^0 = +inf; eps^i = eq. 8 result of
// stage i-1), eq. 16 Beta shape, counters, and the chunk budget the
// persistent kernel aims for (N / (rate C) x margin).
__global__ __launch_bounds__(kBlock) void begin_kernel(BatchArgs a)
{
    const int stage = a.g->stage;
    for (int r = threadIdx.x; r < a.n_runs; r += kBlock) {
        const BRun& R = a.runs[r];
        BState& S = a.st[r];
        if (S.failed) continue;
        S.eps = stage == 0 ? __builtin_inf() : S.eps_next;
        if (stage == 1) S.eps1 = S.eps;
        if (stage == 0) {
            S.beta_a = 0.0;
            S.beta_b = 0;
        } else if (R.step_schedule == 1) {
            S.beta_a = R.beta_a_fixed;
            S.beta_b = R.beta_b_fixed;
        } else {
            S.beta_a = S.eps / S.eps1;
            S.beta_b = 2 * stage;
        }
        S.nxt = stage == 0 ? 0 : 1 - S.cur;
        S.issued = S.completed = S.done_acc = S.accepted = S.proposals = 0;
        S.invalid = S.attempts = S.days = S.survivors = S.fallback = S.terms = S.window_terms = 0;
        const double rate = S.rate > 0.01 ? S.rate : 0.01;
        unsigned long long lim = stage == 0
                                     ? (unsigned long long)((R.N + kChunkP - 1) / kChunkP)
                                     : (unsigned long long)__builtin_ceil((double)R.N / (rate * kChunkP) * a.g->margin);
        if (lim < 1) lim = 1;
        S.limit = lim;
    }
}

__global__ __launch_bounds__(kBlock) void end_kernel(BatchArgs a)
{
    const int stage = a.g->stage;
    for (int r = threadIdx.x; r < a.n_runs; r += kBlock) {
        const BRun& R = a.runs[r];
        BState& S = a.st[r];
        if (S.failed) continue;
        S.cur = S.nxt;
        if (stage > 0) S.rate = (double)R.N / (double)S.proposals;
        S.stages_done = (unsigned long long)stage + 1;
    }
    __syncthreads();
    if (threadIdx.x == 0) a.g->stage = stage + 1;
}

// ------------------------------------------------------------------ resample

// Same three passes as the single-run resample, over each run's block range.
__device__ __forceinline__ void res_mode(const BRun& R, bool& strict, double& wmax, unsigned long long* shu,
                                         double* shd)
{
    unsigned long long ns = 0;
    double wmx = 0.0;
    for (int b = threadIdx.x; b < R.res_nblk; b += kBlock) {
        ns += R.red_u[b];
        wmx = R.red_d[b] > wmx ? R.red_d[b] : wmx;
    }
    ns = bsum(ns, shu);
    wmx = bmax(wmx, shd);
    strict = ns > 0;
    wmax = strict ? wmx : 0.0;
}

__device__ __forceinline__ unsigned long long quantise(double d, double eps, bool strict, double wmax)
{
    const bool in = strict ? (d < eps) : (d <= eps);
    if (!in) return 0ull;
    return wmax > 0.0 ? (unsigned long long)__builtin_floor(((eps - d) / wmax) * 0x1p40) : 1ull;
}

constexpr int kRChunk = 1024, kRPer = kRChunk / kBlock;

__global__ __launch_bounds__(kBlock) void res_stats_kernel(BatchArgs a)
{
    __shared__ unsigned long long shu[kBlock];
    __shared__ double shd[kBlock];
    const int2 rb = a.res_tab[blockIdx.x];
    const BRun& R = a.runs[rb.x];
    const BState& S = a.st[rb.x];
    if (S.failed) return;
    const double* d = R.d[S.cur];
    unsigned long long ns = 0;
    double wmx = 0.0;
    for (int i = 0; i < kRPer; ++i) {
        const int k = rb.y * kRChunk + i * kBlock + threadIdx.x;
        if (k < R.N && d[k] < S.eps) {
            ++ns;
            const double w = S.eps - d[k];
            wmx = w > wmx ? w : wmx;
        }
    }
    ns = bsum(ns, shu);
    wmx = bmax(wmx, shd);
    if (threadIdx.x == 0) {
        R.red_u[rb.y] = ns;
        R.red_d[rb.y] = wmx;
    }
}

__global__ __launch_bounds__(kBlock) void res_count_kernel(BatchArgs a)
{
    __shared__ unsigned long long shu[kBlock];
    __shared__ double shd[kBlock];
    const int2 rb = a.res_tab[blockIdx.x];
    const BRun& R = a.runs[rb.x];
    const BState& S = a.st[rb.x];
    if (S.failed) return;
    bool strict;
    double wmax;
    res_mode(R, strict, wmax, shu, shd);
    const double* d = R.d[S.cur];
    const int k0 = rb.y * kRChunk + threadIdx.x * kRPer;
    unsigned long long sq = 0, sc = 0;
    for (int i = 0; i < kRPer; ++i) {
        const int k = k0 + i;
        if (k < R.N) {
            const unsigned long long q = quantise(d[k], S.eps, strict, wmax);
            sq += q;
            sc += q > 0;
        }
    }
    sq = bsum(sq, shu);
    sc = bsum(sc, shu);
    if (threadIdx.x == 0) {
        R.red_u[R.res_nblk + rb.y] = sq;
        R.red_u[2 * R.res_nblk + rb.y] = sc;
    }
}

__global__ __launch_bounds__(kBlock) void res_write_kernel(BatchArgs a)
{
    __shared__ unsigned long long shu[kBlock];
    __shared__ double shd[kBlock];
    const int2 rb = a.res_tab[blockIdx.x];
    const BRun& R = a.runs[rb.x];
    BState& S = a.st[rb.x];
    if (S.failed) return;
    bool strict;
    double wmax;
    res_mode(R, strict, wmax, shu, shd);
    const int G = R.res_nblk;
    const unsigned long long* bq = R.red_u + G;
    const unsigned long long* bc = R.red_u + 2 * G;
    unsigned long long oq = 0, oc = 0, tc = 0;
    for (int b = threadIdx.x; b < G; b += kBlock) {
        if (b < rb.y) {
            oq += bq[b];
            oc += bc[b];
        }
        tc += bc[b];
    }
    oq = bsum(oq, shu);
    oc = bsum(oc, shu);
    tc = bsum(tc, shu);
    const double* d = R.d[S.cur];
    const double* up = R.u[S.cur];
    const int k0 = rb.y * kRChunk + threadIdx.x * kRPer;
    unsigned long long q[kRPer];
    unsigned long long sq = 0, sc = 0;
    for (int i = 0; i < kRPer; ++i) {
        const int k = k0 + i;
        q[i] = k < R.N ? quantise(d[k], S.eps, strict, wmax) : 0ull;
        sq += q[i];
        sc += q[i] > 0;
    }
    unsigned long long run = oq + bscan_excl(sq, shu);
    unsigned long long col = oc + bscan_excl(sc, shu);
    for (int i = 0; i < kRPer; ++i) {
        const int k = k0 + i;
        if (k >= R.N) break;
        run += q[i];
        R.q[k] = q[i];
        R.cdf[k] = run;
        if (q[i] > 0) {
            double* c = R.cols + (size_t)col * 9;
#pragma unroll
            for (int dd = 0; dd < kNP; ++dd) c[dd] = up[(size_t)k * kNP + dd];
            c[8] = (double)q[i];
            ++col;
        }
    }
    if (rb.y == G - 1 && threadIdx.x == 0) {
        S.survivors = tc;
        S.fallback = strict ? 0ull : 1ull;
    }
}

// ------------------------------------------------------------------ propose

// Work-item scheduler of the persistent kernel (thread 0 of a workgroup).
// Pass 0 issues chunks of runs below their budget; pass 1 over-issues for
// runs still short of N acceptances, with a bound on chunks in flight (stage 0,
// where every proposal is accepted, issues exactly ceil(N / chunk) chunks).
// Every call either returns a chunk index below the run's capacity or -1, and
// a workgroup that completes a chunk always calls again, so a run short of N
// is re-examined after its last chunk in flight and every workgroup reaches
// its exit.
__device__ int pick(const BatchArgs& a, int start, bool exact, int* chunk)
{
    const int R = a.n_runs;
    for (int pass = 0; pass < (exact ? 1 : 2); ++pass) {
        for (int i = 0; i < R; ++i) {
            const int r = a.order[(start + i) % R];
            const BRun& Rr = a.runs[r];
            BState& S = a.st[r];
            if (ld_relaxed_i(&S.failed)) continue;
            const unsigned long long done = ld_relaxed(&S.done_acc);
            if (done >= (unsigned long long)Rr.N) continue;
            const unsigned long long cap = (unsigned long long)Rr.cap_chunks;
            const unsigned long long issued = ld_relaxed(&S.issued);
            if (issued >= cap) continue;
            if (pass == 0) {
                if (issued >= S.limit) continue;
            } else {
                const unsigned long long inflight = issued - ld_relaxed(&S.completed);
                const double rate = S.rate > 0.01 ? S.rate : 0.01;
                const double need = __builtin_ceil((double)(Rr.N - done) / (rate * kChunkP)) * a.g->margin;
                const unsigned long long bound = need > 1.0 ? (unsigned long long)need : 1ull;
                if (inflight >= bound) continue;
            }
            const unsigned long long k = atomicAdd(&S.issued, 1ull);
            if (k < cap) {
                *chunk = (int)k;
                return r;
            }
        }
    }
    return -1;
}

template <bool kRound0>
__global__ __launch_bounds__(kBlock) void propose_persistent_kernel(BatchArgs a)
{
    __shared__ int s_run, s_chunk;
    __shared__ unsigned long long s_cnt[kBlock / kWave][4];
    const int stage = a.g->stage;
    int iter = 0;
    for (;;) {
        if (threadIdx.x == 0) {
            int ch = 0;
            const int r = pick(a, (int)((blockIdx.x + (unsigned)iter * gridDim.x) % (unsigned)a.n_runs), kRound0, &ch);
            s_run = r;
            s_chunk = ch;
        }
        __syncthreads();
        const int r = s_run, k = s_chunk;
        __syncthreads();
        if (r < 0) break;
        ++iter;
        const BRun& R = a.runs[r];
        const BState& S = a.st[r];
        const uint32_t p = (uint32_t)k * kChunkP + threadIdx.x;  // proposal index within the stage
        const int cur = S.cur;
        const lane::ProposalIn in{R.obs,
                                  (uint32_t)stage,
                                  R.max_attempts,
                                  S.eps,
                                  (R.early_exit && !kRound0) ? (S.eps * S.eps) * (1.0 + 0x1p-48) : __builtin_inf(),
                                  R.u[cur],
                                  R.cdf,
                                  R.N,
                                  S.beta_a,
                                  S.beta_b,
                                  R.step_is_variance,
                                  -1.0,
                                  0.0};
        lane::ProposalOut o;
        if (R.m.sampler == 0) lane::propose_one<kRound0, 0>(R.m, in, p, o);
        else lane::propose_one<kRound0, 1>(R.m, in, p, o);
        double* su = R.st_u + (size_t)p * kNP;
#pragma unroll
        for (int q = 0; q < kNP; ++q) su[q] = o.u[q];
        R.st_d[p] = o.d;
        R.st_sigma[p] = o.sigma;
        R.st_parent[p] = o.parent;
        R.st_att[p] = o.att;
        const unsigned long long mask = __ballot(o.acc);
        const unsigned long long inv = lane::wave_sum_u64(o.valid ? 0ull : 1ull);
        const unsigned long long natt = lane::wave_sum_u64((unsigned long long)(o.att < 0 ? -o.att : o.att));
        const unsigned long long ndays = lane::wave_sum_u64((unsigned long long)o.days);
        const int w = threadIdx.x / kWave;
        if ((threadIdx.x & (kWave - 1)) == 0) {
            R.wave_mask[p / kWave] = mask;
            s_cnt[w][0] = (unsigned long long)__popcll(mask);
            s_cnt[w][1] = inv;
            s_cnt[w][2] = natt;
            s_cnt[w][3] = ndays;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long c[4] = {0, 0, 0, 0};
            for (int ww = 0; ww < kBlock / kWave; ++ww)
                for (int f = 0; f < 4; ++f) c[f] += s_cnt[ww][f];
            BState& Sw = a.st[r];
            if (c[1]) atomicAdd(&Sw.invalid, c[1]);
            atomicAdd(&Sw.attempts, c[2]);
            atomicAdd(&Sw.days, c[3]);
            __threadfence();
            atomicAdd(&Sw.done_acc, c[0]);
            atomicAdd(&Sw.completed, 1ull);
        }
    }
}

// ------------------------------------------------------------------ compaction

// One block per run: exclusive prefix of per-wave acceptance counts over the
// issued chunks (index order) and the stage's acceptance total.
__global__ __launch_bounds__(kBlock) void bcompact_scan_kernel(BatchArgs a)
{
    __shared__ unsigned long long sh[kBlock];
    const int r = blockIdx.x;
    const BRun& R = a.runs[r];
    BState& S = a.st[r];
    if (S.failed) return;
    const unsigned long long issued = S.issued < (unsigned long long)R.cap_chunks ? S.issued : (unsigned long long)R.cap_chunks;
    const int nW = (int)issued * (kChunkP / kWave);
    const int per = (nW + kBlock - 1) / kBlock;
    const int w0 = threadIdx.x * per, w1 = min(nW, w0 + per);
    unsigned long long s = 0;
    for (int w = w0; w < w1; ++w) s += __popcll(R.wave_mask[w]);
    unsigned long long run = bscan_excl(s, sh);
    for (int w = w0; w < w1; ++w) {
        R.wave_off[w] = (uint32_t)run;
        run += __popcll(R.wave_mask[w]);
    }
    const unsigned long long tot = bsum(s, sh);
    if (threadIdx.x == 0) {
        S.accepted = tot;
        if (tot < (unsigned long long)R.N) S.failed = 1;  // out of proposals: the run keeps its last stage
    }
}

__global__ __launch_bounds__(kBlock) void bcompact_scatter_kernel(BatchArgs a)
{
    const int r = blockIdx.y, k = blockIdx.x;
    const BRun& R = a.runs[r];
    BState& S = a.st[r];
    if (S.failed) return;
    const unsigned long long issued = S.issued < (unsigned long long)R.cap_chunks ? S.issued : (unsigned long long)R.cap_chunks;
    if ((unsigned long long)k >= issued) return;
    const uint32_t p = (uint32_t)k * kChunkP + threadIdx.x;
    const unsigned long long mask = R.wave_mask[p / kWave];
    const uint32_t lane = p % kWave;
    if (!((mask >> lane) & 1ull)) return;
    const unsigned long long below = lane ? (mask & ((1ull << lane) - 1ull)) : 0ull;
    const unsigned long long gr = R.wave_off[p / kWave] + (unsigned long long)__popcll(below);
    if (gr >= (unsigned long long)R.N) return;
    const int nx = S.nxt;
    const double* su = R.st_u + (size_t)p * kNP;
    double* du = R.u[nx] + (size_t)gr * kNP;
#pragma unroll
    for (int q = 0; q < kNP; ++q) du[q] = su[q];
    R.d[nx][gr] = R.st_d[p];
    R.sigma[nx][gr] = R.st_sigma[p];
    R.parent[nx][gr] = R.st_parent[p];
    R.index[nx][gr] = p;
    R.att[nx][gr] = R.st_att[p];
    if (gr == (unsigned long long)(R.N - 1)) S.proposals = (unsigned long long)p + 1ull;
}

// ------------------------------------------------------------------ weights

// Weight window, per run (as the single-run pass): the sort coordinate d* of
// largest column variance; columns sorted by (run, u_{k,d*}); rows sorted by
// (run, sigma half-octave descending, u_{j,d*}); each row's half-width comes from its parent's
// term (wterm::window_halfwidth) and each 128-row block gets the union of its
// rows' column ranges.  One batch-wide bitonic
// sort per key set: the run index in the top 12 bits keeps every run's keys in
// its own slot range [off_r, off_r + N_r).
using wterm::coord_key32;
using wterm::lower_index;
using wterm::sigma_half_octave;
using wterm::wave_max;
using wterm::wave_min;
using wterm::wave_sum_u64;

// One block per run: variance of each coordinate over the run's columns.
__global__ __launch_bounds__(kBlock) void bwdim_kernel(BatchArgs a)
{
    __shared__ double sh[kBlock];
    const BRun& R = a.runs[blockIdx.x];
    BState& S = a.st[blockIdx.x];
    if (S.failed) return;
    const int M = (int)S.survivors;
    double best = -1.0;
    int bd = 0;
    for (int d = 0; d < kNP; ++d) {
        double s1 = 0.0, s2 = 0.0;
        for (int k = threadIdx.x; k < M; k += kBlock) {
            const double v = R.cols[(size_t)k * 9 + d];
            s1 += v;
            s2 += v * v;
        }
        s1 = bsum(s1, sh);
        s2 = bsum(s2, sh);
        const double mean = s1 / (double)M;
        const double var = s2 / (double)M - mean * mean;
        if (var > best) {
            best = var;
            bd = d;
        }
    }
    if (threadIdx.x == 0) S.dstar = bd;
}

// run owning batch-wide slot i (i < n_total)
__device__ __forceinline__ int slot_run(const BatchArgs& a, int i)
{
    int lo = 0, hi = a.n_runs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.runs[mid].off <= i) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(kBlock) void bkeys_kernel(BatchArgs a)
{
    const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= a.npad) return;
    if (i >= (size_t)a.n_total) {
        a.colkeys[i] = ~0ull;
        a.rowkeys[i] = ~0ull;
        return;
    }
    const int r = slot_run(a, (int)i);
    const BRun& R = a.runs[r];
    const BState& S = a.st[r];
    const unsigned long long k = (unsigned long long)((int)i - R.off);
    const unsigned long long run = (unsigned long long)r << 52;
    if (S.failed) {
        a.colkeys[i] = run | (0xFFFFFFFFull << 20) | k;
        a.rowkeys[i] = run | k;
        return;
    }
    const int ds = S.dstar;
    a.colkeys[i] = (k < (unsigned long long)S.survivors)
                       ? run | (coord_key32(R.cols[k * 9 + ds]) << 20) | k
                       : run | (0xFFFFFFFFull << 20) | k;
    const int nx = S.nxt;
    // half-octaves in descending order: the widest windows are dispatched first
    const unsigned long long oct = 127ull - sigma_half_octave(R.sigma[nx][k]);
    a.rowkeys[i] = run | (oct << 45) | ((coord_key32(R.u[nx][k * kNP + ds]) >> 7) << 20) | k;
    const double* uj = R.u[nx] + k * kNP;
    const int32_t par = R.parent[nx][k];
    const bool ok = par >= 0 && par < R.N;
    a.rwin[i] = wterm::window_halfwidth(uj, R.sigma[nx][k], ok ? R.u[1 - nx] + (size_t)par * kNP : uj,
                                        ok ? (double)R.q[par] : 0.0, (double)R.cdf[R.N - 1]);
}

__global__ __launch_bounds__(kBlock) void bcolgather_kernel(BatchArgs a)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= a.n_total) return;
    const int r = slot_run(a, i);
    const BRun& R = a.runs[r];
    const BState& S = a.st[r];
    if (S.failed || i - R.off >= (int)S.survivors) return;
    const size_t src = (size_t)(a.colkeys[i] & 0xFFFFFull);
    const double* c = R.cols + src * 9;
    double* o = a.scols + (size_t)i * 9;
#pragma unroll
    for (int d = 0; d < 9; ++d) o[d] = c[d];
    a.skey[i] = c[S.dstar];
}

// One block per (run, 256 sorted rows): the block's column window.
__global__ __launch_bounds__(kWeightRows) void bwindow_kernel(BatchArgs a)
{
    __shared__ double slo[kWeightRows / kWave], shi[kWeightRows / kWave];
    const int2 fb = a.fin_tab[blockIdx.x];
    const BRun& R = a.runs[fb.x];
    const BState& S = a.st[fb.x];
    if (S.failed) return;
    const int nx = S.nxt;
    const int rr = fb.y * kWeightRows + threadIdx.x;
    const int M = (int)S.survivors;
    const double* sk = a.skey + R.off;
    double lo = __builtin_inf(), hi = -__builtin_inf();
    unsigned long long own = 0;  // columns of this row's own window
    if (rr < R.N) {
        const size_t j = (size_t)(a.rowkeys[R.off + rr] & 0xFFFFFull);
        const double W = a.rwin[R.off + j];
        const double x = R.u[nx][j * kNP + S.dstar];
        lo = x - W;
        hi = x + W;
        own = (unsigned long long)(lower_index(sk, M, hi, true) - lower_index(sk, M, lo, false));
    }
    own = wave_sum_u64(own);
    if ((threadIdx.x & (kWave - 1)) == 0 && own) atomicAdd(&a.st[fb.x].window_terms, own);
    lo = wave_min(lo);
    hi = wave_max(hi);
    if ((threadIdx.x & (kWave - 1)) == 0) {
        slo[threadIdx.x / kWave] = lo;
        shi[threadIdx.x / kWave] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 0; q < kWeightRows / kWave; ++q) {
            lo = slo[q] < lo ? slo[q] : lo;
            hi = shi[q] > hi ? shi[q] : hi;
        }
        a.win[R.rb0 + fb.y] = make_int2(lower_index(sk, M, lo, false), lower_index(sk, M, hi, true));
    }
}

// grid = weight table (run, row block, chunk): chunk c of the block's window,
// sorted rows; partial sums go to the rows' own indices (finalize unchanged).
__global__ __launch_bounds__(kWeightRows) void bweights_kernel(BatchArgs a)
{
    __shared__ double T[wterm::kTab];
    const int4 wb = a.w_tab[blockIdx.x];
    const BRun& R = a.runs[wb.x];
    const BState& S = a.st[wb.x];
    if (S.failed) return;  // uniform across the block
    const int nx = S.nxt;
    const int rr = wb.y * kWeightRows + threadIdx.x;
    const bool active = rr < R.N;
    const size_t j = active ? (size_t)(a.rowkeys[R.off + rr] & 0xFFFFFull) : 0;
    const int2 wnd = a.win[R.rb0 + wb.y];
    const int len = wnd.y - wnd.x > 0 ? wnd.y - wnd.x : 0;
    const int Sc = R.wchunks, c = wb.z;
    const int k0 = wnd.x + (int)(((long long)len * c) / Sc);
    const int k1 = wnd.x + (int)(((long long)len * (c + 1)) / Sc);
    if (k0 >= k1) {
        if (active) R.wpart[(size_t)c * R.N + j] = 0.0;
        return;
    }
    wterm::load_table(T, a.wtab);
    __syncthreads();
    const int ds = S.dstar;
    double uj[kNP];
    double cj = 0.0, lo = __builtin_inf(), hi = -__builtin_inf();
    if (active) {
#pragma unroll
        for (int d = 0; d < kNP; ++d) uj[d] = R.u[nx][j * kNP + d];
        const double sj = R.sigma[nx][j];
        cj = wterm::row_scale(sj, a.ex);
        lo = uj[ds] - a.rwin[R.off + j];
        hi = uj[ds] + a.rwin[R.off + j];
    } else {
#pragma unroll
        for (int d = 0; d < kNP; ++d) uj[d] = 0.0;
    }
    const double wlo = wave_min(lo), whi = wave_max(hi);
    const unsigned long long lanes = (unsigned long long)__popcll(__ballot(active));
    unsigned long long evaluated = 0;
    const double total = wterm::row_sum(uj, cj, (wterm::const_col_ptr)(a.scols + (size_t)R.off * 9),
                                        (wterm::const_col_ptr)(a.skey + R.off), k0, k1, wlo, whi, T, a.ex, lanes,
                                        evaluated);
    if (active) R.wpart[(size_t)c * R.N + j] = total;
    if ((threadIdx.x & (kWave - 1)) == 0 && evaluated) atomicAdd(&a.st[wb.x].terms, evaluated);
}

__global__ __launch_bounds__(kWeightRows) void bfinalize_kernel(BatchArgs a)
{
    const int2 fb = a.fin_tab[blockIdx.x];
    const BRun& R = a.runs[fb.x];
    const BState& S = a.st[fb.x];
    if (S.failed) return;
    const int j = fb.y * kWeightRows + threadIdx.x;
    if (j >= R.N) return;
    double L = 0.0;
    for (int c = 0; c < R.wchunks; ++c) L += R.wpart[(size_t)c * R.N + j];
    R.logw[S.nxt][j] = 8.0 * dm::log(R.sigma[S.nxt][j]) - dm::log(L);
}

// One block per run: W = softmax(l), ESS.
__global__ __launch_bounds__(kBlock) void bnormalise_kernel(BatchArgs a, int uniform)
{
    __shared__ double sh[kBlock];
    const BRun& R = a.runs[blockIdx.x];
    BState& S = a.st[blockIdx.x];
    if (S.failed) return;
    const int nx = S.nxt;
    const double* l = R.logw[nx];
    double* W = R.W[nx];
    if (uniform) {
        for (int j = threadIdx.x; j < R.N; j += kBlock) {
            W[j] = 1.0 / (double)R.N;
            R.logw[nx][j] = 0.0;
        }
        if (threadIdx.x == 0) S.ess = (double)R.N;
        return;
    }
    double mx = -__builtin_inf();
    for (int j = threadIdx.x; j < R.N; j += kBlock) mx = l[j] > mx ? l[j] : mx;
    mx = bmax(mx, sh);
    double s = 0.0;
    for (int j = threadIdx.x; j < R.N; j += kBlock) {
        const double e = dm::exp(l[j] - mx);
        W[j] = e;
        s += e;
    }
    s = bsum(s, sh);
    double s2 = 0.0;
    for (int j = threadIdx.x; j < R.N; j += kBlock) {
        const double w = W[j] / s;
        W[j] = w;
        s2 += w * w;
    }
    s2 = bsum(s2, sh);
    if (threadIdx.x == 0) S.ess = 1.0 / s2;
}

// ------------------------------------------------------------------ select

// One block per run: eq. 8 type-7 percentile by radix select in LDS (same
// digits and interpolation as the single-run kernels).
__global__ __launch_bounds__(kBlock) void bselect_kernel(BatchArgs a)
{
    __shared__ bsel::Shared sh;
    const BRun& R = a.runs[blockIdx.x];
    BState& S = a.st[blockIdx.x];
    if (S.failed) return;  // uniform across the block
    const double res = bsel::quantile7(R.d[S.nxt], R.N, 1, R.surv_ratio, sh);
    if (threadIdx.x == 0) S.eps_next = res;
}

}  // namespace

void batch_launch_stage(const BatchArgs& a, bool stage0, hipStream_t s)
{
    const dim3 b(kBlock);
    hipLaunchKernelGGL(begin_kernel, dim3(1), b, 0, s, a);
    if (!stage0) {
        hipLaunchKernelGGL(res_stats_kernel, dim3(a.n_res_blocks), b, 0, s, a);
        hipLaunchKernelGGL(res_count_kernel, dim3(a.n_res_blocks), b, 0, s, a);
        hipLaunchKernelGGL(res_write_kernel, dim3(a.n_res_blocks), b, 0, s, a);
        hipLaunchKernelGGL(propose_persistent_kernel<false>, dim3(a.propose_blocks), b, 0, s, a);
    } else {
        hipLaunchKernelGGL(propose_persistent_kernel<true>, dim3(a.propose_blocks), b, 0, s, a);
    }
    hipLaunchKernelGGL(bcompact_scan_kernel, dim3(a.n_runs), b, 0, s, a);
    hipLaunchKernelGGL(bcompact_scatter_kernel, dim3(a.max_cap_chunks, a.n_runs), b, 0, s, a);
    if (!stage0) {
        hipLaunchKernelGGL(bwdim_kernel, dim3(a.n_runs), b, 0, s, a);
        hipLaunchKernelGGL(bkeys_kernel, dim3(a.n_key_blocks), b, 0, s, a);
        launch_sort_u64_pair(a.colkeys, a.rowkeys, a.npad, s);
        hipLaunchKernelGGL(bcolgather_kernel, dim3((a.n_total + kBlock - 1) / kBlock), b, 0, s, a);
        const dim3 bw(kWeightRows);
        hipLaunchKernelGGL(bwindow_kernel, dim3(a.n_fin_blocks), bw, 0, s, a);
        hipLaunchKernelGGL(bweights_kernel, dim3(a.n_w_blocks), bw, 0, s, a);
        hipLaunchKernelGGL(bfinalize_kernel, dim3(a.n_fin_blocks), bw, 0, s, a);
    }
    hipLaunchKernelGGL(bnormalise_kernel, dim3(a.n_runs), b, 0, s, a, stage0 ? 1 : 0);
    hipLaunchKernelGGL(bselect_kernel, dim3(a.n_runs), b, 0, s, a);
    hipLaunchKernelGGL(end_kernel, dim3(1), b, 0, s, a);
}

}  // namespace abcsmc
