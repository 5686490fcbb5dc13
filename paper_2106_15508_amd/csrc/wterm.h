// wterm.h -- one importance-weight term q_k exp(-|u_j - u_k|^2 / (2 sigma_j^2))
// with a table-driven exponential, the per-row column loop and the window
// helpers (device code shared by the single-run and batched weight kernels).
#pragma once

#include "dmath.h"
#include "kernels.h"

namespace abcsmc {
namespace wterm {

constexpr int kTile = 256;  // columns per skip-test tile

// Scalar-column form used by the weight kernels.  Columns (u_k[8], q_k) are
// the same for every lane of a wave, so they are read through a wave-uniform
// pointer in the constant address space (scalar loads into SGPRs, no LDS
// staging).  The exponential uses a 1024-entry table of 2^(i/1024):
//   t = D c_j with c_j = -1024 / (2 sigma_j^2 ln 2)  (the exponent in units
//   of ln2/1024), k = rint(t), r = (t - k) ln2/1024, |r| <= 3.4e-4,
//   exp = 2^(k >> 10) 2^((k & 1023)/1024) (1 + r + r^2/2 + r^3/6)
// (truncation r^4/24 < 6e-16 relative); the weight q_k enters by one fma
// into the running sum.  There is no cut-off: a term with
// exponent below -708 comes out as 0 or a subnormal-size value, which cannot
// change a row sum (every row holds its own parent's term, >= e^-185) -- the
// sums are those of the exact-zero convention.  For t below -2^31 (every far
// column of a row whose sigma is near the 1e-8 floor) the integer conversion
// saturates (cvt_i32_sat) and 2^(k >> 10) underflows to 0.
constexpr int kTabBits = 10;
constexpr int kTab = 1 << kTabBits;

typedef const __attribute__((address_space(4))) double* const_col_ptr;  // constant address space

struct Col {
    double u[kNP];
    double q;
};

__device__ __forceinline__ Col load_col(const_col_ptr cols, int k)
{
    Col c;
    const_col_ptr p = cols + (size_t)k * 9;
#pragma unroll
    for (int d = 0; d < kNP; ++d) c.u[d] = p[d];
    c.q = p[8];
    return c;
}

// k = rint(t) as an int32, saturating: v_cvt_i32_f64 clamps an input outside
// the int32 range to INT32_MIN / INT32_MAX by its definition, where a C++
// conversion of such a value would be undefined.  One instruction, as the
// plain conversion compiles to.
__device__ __forceinline__ int cvt_i32_sat(double x)
{
    int r;
    asm("v_cvt_i32_f64 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

// exp of the term (without q): with f = t - k in [-1/2, 1/2] and L = ln2/1024,
// e^(f L) = 1 + f (L + f (L^2/2 + f L^3/6)); ex[0..2] = L, L^2/2, L^3/6
// (kernel arguments: SGPRs).
__device__ __forceinline__ double term_exp(const double* uj, double cj, const Col& c, const double* T,
                                           const double* ex)
{
    double D = 0.0;
#pragma unroll
    for (int d = 0; d < kNP; ++d) {
        const double df = uj[d] - c.u[d];
        D = __builtin_fma(df, df, D);
    }
    const double t = D * cj;
    const double kk = __builtin_rint(t);
    const double f = t - kk;
    const int ik = cvt_i32_sat(kk);
    double p = __builtin_fma(f, ex[2], ex[1]);
    p = __builtin_fma(p, f, ex[0]);
    p = __builtin_fma(p, f, 1.0);
    return __builtin_ldexp(T[ik & (kTab - 1)] * p, ik >> kTabBits);
}

// Per-lane scale c_j of the row's exponent (ex[3] = 1024 / ln 2).
__device__ __forceinline__ double row_scale(double sigma, const double* ex)
{
    return -ex[3] / (2.0 * (sigma * sigma));
}

static_assert(kTab == kWeightTab, "table length");

// Table entry i: 2^(i/1024).
__device__ __forceinline__ double table_entry(int i)
{
    return dm::exp((double)i * (0.6931471805599453 / kTab));
}

// Copy of the table (written once per context by launch_weight_table) into
// LDS; all threads of the block take part.
__device__ __forceinline__ void load_table(double* T, const double* g)
{
    for (int i = threadIdx.x; i < kTab; i += blockDim.x) T[i] = g[i];
}

// Sum over the sorted columns [k0, k1) for this lane's row, in 256-column
// tiles; a tile that no row of the wave can reach (sort coordinate outside
// [wlo, whi]) is skipped.  Two interleaved partial sums (even and odd
// columns), four columns' scalar loads issued together per step.
__device__ __forceinline__ double row_sum(const double* uj, double cj, const_col_ptr cols, const_col_ptr skey,
                                          int k0, int k1, double wlo, double whi, const double* T,
                                          const double* ex, unsigned long long lanes,
                                          unsigned long long& evaluated)
{
    double total = 0.0;
    for (int c0 = k0; c0 < k1; c0 += kTile) {
        const int n = min(kTile, k1 - c0);
        if (skey[c0 + n - 1] < wlo || skey[c0] > whi) continue;
        evaluated += lanes * (unsigned long long)n;
        double p0 = 0.0, p1 = 0.0;
        int cc = 0;
        for (; cc + 3 < n; cc += 4) {
            const int k = __builtin_amdgcn_readfirstlane(c0 + cc);
            const Col a0 = load_col(cols, k), a1 = load_col(cols, k + 1), a2 = load_col(cols, k + 2), a3 = load_col(cols, k + 3);
            p0 = __builtin_fma(a0.q, term_exp(uj, cj, a0, T, ex), p0);
            p1 = __builtin_fma(a1.q, term_exp(uj, cj, a1, T, ex), p1);
            p0 = __builtin_fma(a2.q, term_exp(uj, cj, a2, T, ex), p0);
            p1 = __builtin_fma(a3.q, term_exp(uj, cj, a3, T, ex), p1);
        }
        for (; cc < n; cc += 2) {
            const int k = __builtin_amdgcn_readfirstlane(c0 + cc);
            const Col a0 = load_col(cols, k);
            p0 = __builtin_fma(a0.q, term_exp(uj, cj, a0, T, ex), p0);
            if (cc + 1 < n) {
                const Col a1 = load_col(cols, k + 1);
                p1 = __builtin_fma(a1.q, term_exp(uj, cj, a1, T, ex), p1);
            }
        }
        total += p0 + p1;
    }
    return total;
}

// Widest window of a row (the cap of window_halfwidth): a column whose sort
// coordinate differs by more than kWindow sigma_j gives an exponent below
// -710, where both exponentials are exactly 0.
constexpr double kWindow = 37.7;

// Narrower per-row window with a bound on what it leaves out.  Every column
// outside |u_kd - u_jd| <= W sigma_j (any one coordinate d) has a term at most
// q_k e^{-W^2/2}, so all of them together are at most Q e^{-W^2/2}
// (Q = sum_k q_k).  The row sum holds the parent's own term
// L_par = q_par e^{-|u_j - u_par|^2 / (2 sigma_j^2)}, so with
//   W^2 = 2 (ln Q - ln L_par + 53 ln 2)
// the omitted mass is at most 2^-53 of the row sum: one unit roundoff of the
// sum itself.  The parent always lies inside (W^2 >= |u_j - u_par|^2 /
// sigma_j^2 because Q >= q_par).  The result is capped at kWindow; a missing
// or zero parent weight leaves kWindow.  Returns the half-width W sigma_j.
__device__ __forceinline__ double window_halfwidth(const double* uj, double sj, const double* up, double qpar,
                                                   double Q)
{
    double W = kWindow;
    if (qpar > 0.0 && Q >= qpar && sj > 0.0) {
        double d2 = 0.0;
#pragma unroll
        for (int d = 0; d < kNP; ++d) {
            const double e = uj[d] - up[d];
            d2 = d2 + e * e;
        }
        const double x = d2 / (2.0 * sj * sj);
        const double w2 = 2.0 * ((dm::log(Q) - dm::log(qpar)) + x + 53.0 * 0.6931471805599453);
        const double w = __builtin_sqrt(w2);
        if (w < W) W = w;
    }
    return W * sj;
}

// 32-bit monotone key of a unit-cube coordinate (truncation: keys tie within
// 2.4e-10, far below the window margin 0.07 sigma >= 7e-10).
__device__ __forceinline__ unsigned long long coord_key32(double u)
{
    const double c = u < 0.0 ? 0.0 : (u > 1.0 ? 1.0 : u);
    return (unsigned long long)(unsigned int)(c * 4294967295.0);
}

// 7-bit half-octave of a step size: rows of similar sigma share windows well
// (half-octaves give 2.5% fewer evaluated terms than octaves at N = 131072
// and 6% at N = 2^20).
__device__ __forceinline__ unsigned long long sigma_half_octave(double s)
{
    int e;
    const double m = __builtin_frexp(s, &e);
    int h = 2 * (e + 40) + (m >= 0.7071067811865476 ? 1 : 0);
    h = h < 0 ? 0 : (h > 127 ? 127 : h);
    return (unsigned long long)h;
}

// first index in sorted v[0..n) with v >= x (or > x when strict)
__device__ __forceinline__ int lower_index(const double* v, int n, double x, bool strict)
{
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (strict ? (v[mid] <= x) : (v[mid] < x)) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__device__ __forceinline__ double wave_min(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(v, off, kWave);
        v = o < v ? o : v;
    }
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(v, off, kWave);
        v = o > v ? o : v;
    }
    return v;
}

}  // namespace wterm
}  // namespace abcsmc
