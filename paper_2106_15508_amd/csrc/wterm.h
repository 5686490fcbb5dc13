// wterm.h -- one importance-weight term q_k exp(-|u_j - u_k|^2 / (2 sigma_j^2))
// with a table-driven exponential (device code shared by the single-run and
// batched weight kernels).
//
// exp: x = (64 k + i) ln2/64 + r with |r| <= ln2/128,
// exp(x) = 2^k 2^(i/64) (1 + r + r^2/2 + ... + r^5/5!); relative error a few
// 1e-16.  The constants come in through kernel arguments (scalar registers).
#pragma once

#include "dmath.h"
#include "kernels.h"

namespace abcsmc {
namespace wterm {

constexpr int kTile = 256;  // columns per LDS tile

__device__ __forceinline__ double exp_tab(double x, const double* T, const double* ex)
{
    const double kk = __builtin_rint(x * ex[0]);
    double r = __builtin_fma(-kk, ex[1], x);
    r = __builtin_fma(-kk, ex[2], r);
    const int ik = (int)kk;
    double p = __builtin_fma(ex[6], r, ex[5]);
    p = __builtin_fma(p, r, ex[4]);
    p = __builtin_fma(p, r, ex[3]);
    p = __builtin_fma(p, r, 1.0);
    p = __builtin_fma(p, r, 1.0);
    return __builtin_ldexp(T[ik & 63] * p, ik >> 6);
}

__device__ __forceinline__ double pair_term(const double* uj, double ninv, const double (*tu)[kTile],
                                            const double* tq, int c, const double* T, const double* ex)
{
    double D = 0.0;
#pragma unroll
    for (int d = 0; d < kNP; ++d) {
        const double df = uj[d] - tu[d][c];
        D = __builtin_fma(df, df, D);
    }
    const double arg = D * ninv;
    return arg >= dm::kExpLo ? tq[c] * exp_tab(arg, T, ex) : 0.0;
}


// Window of a row: a column whose sort coordinate differs by more than
// kWindow sigma_j gives an exponent below -710, where both exponentials are
// exactly 0, so it can be skipped without changing the sum.
constexpr double kWindow = 37.7;

// 32-bit monotone key of a unit-cube coordinate (truncation: keys tie within
// 2.4e-10, far below the window margin 0.07 sigma >= 7e-10).
__device__ __forceinline__ unsigned long long coord_key32(double u)
{
    const double c = u < 0.0 ? 0.0 : (u > 1.0 ? 1.0 : u);
    return (unsigned long long)(unsigned int)(c * 4294967295.0);
}

// 6-bit octave of a step size (rows of similar sigma share windows well).
__device__ __forceinline__ unsigned long long sigma_octave(double s)
{
    int e;
    (void)__builtin_frexp(s, &e);
    int oct = e + 40;
    oct = oct < 0 ? 0 : (oct > 63 ? 63 : oct);
    return (unsigned long long)oct;
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

// 2^(i/64), i = 0..63, into LDS (call from the first 64 threads).
__device__ __forceinline__ double table_entry(int i) { return dm::exp((double)i * 0.010830424696249145); }

}  // namespace wterm
}  // namespace abcsmc
