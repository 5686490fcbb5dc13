// blockselect.h -- one workgroup's exact type-7 quantile of n non-negative
// doubles (eq. 8's percentile; numpy "linear" interpolation), by radix
// select on the IEEE bit patterns in LDS: 11/11/11/11/11/9-bit digits,
// both order statistics of the interpolation tracked at once.  Shared by the
// batched mode's per-run percentile and the predictive bands.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.h"

namespace abcsmc {
namespace bsel {

constexpr int kBins = 2048;

struct Shared {
    unsigned int h[2][kBins];
    unsigned long long part[kBlock];
    unsigned long long st[8];
    double res;
};

__device__ __forceinline__ unsigned long long bscan_excl(unsigned long long v, unsigned long long* sh)
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
    const unsigned long long r = sh[t] - v;
    __syncthreads();
    return r;
}

// x[k * stride], k < n (n >= 1); every thread of the block calls it and gets
// the result.
__device__ __forceinline__ double quantile7(const double* x, int64_t n, int64_t stride, double alpha, Shared& S)
{
    const double v = ((double)n - 1.0) * alpha;
    long long r0, r1;
    if (v >= (double)n - 1.0) {
        r0 = r1 = n - 1;
    } else if (v < 0.0) {
        r0 = r1 = 0;
    } else {
        r0 = (long long)__builtin_floor(v);
        r1 = r0 + 1;
    }
    if (threadIdx.x == 0) {
        S.st[0] = S.st[1] = S.st[2] = S.st[3] = 0ull;  // prefixes, masks
        S.st[4] = (unsigned long long)r0;
        S.st[5] = (unsigned long long)r1;
    }
    __syncthreads();
    for (int pass = 0; pass < 6; ++pass) {
        for (int b = threadIdx.x; b < 2 * kBins; b += kBlock) (&S.h[0][0])[b] = 0u;
        __syncthreads();
        const int sh = pass < 5 ? 53 - 11 * pass : 0;
        const unsigned long long dmk = (1ull << (pass < 5 ? 11 : 9)) - 1ull;
        const unsigned long long p0 = S.st[0], p1 = S.st[1], m0 = S.st[2], m1 = S.st[3];
        for (int64_t k = threadIdx.x; k < n; k += kBlock) {
            const unsigned long long bits = (unsigned long long)__double_as_longlong(x[k * stride]);
            const unsigned int dig = (unsigned int)((bits >> sh) & dmk);
            if ((bits & m0) == p0) atomicAdd(&S.h[0][dig], 1u);
            if ((bits & m1) == p1) atomicAdd(&S.h[1][dig], 1u);
        }
        __syncthreads();
        const int nb = (int)dmk + 1;
        const int per = (nb + kBlock - 1) / kBlock;
        for (int which = 0; which < 2; ++which) {
            const unsigned long long rank = S.st[4 + which];
            const int b0 = threadIdx.x * per, b1 = min(nb, b0 + per);
            unsigned long long s = 0;
            for (int b = b0; b < b1; ++b) s += S.h[which][b];
            unsigned long long run = bscan_excl(s, S.part);
            for (int b = b0; b < b1; ++b) {
                if (run <= rank && rank < run + S.h[which][b]) {
                    S.st[4 + which] = rank - run;
                    S.st[which] |= (unsigned long long)b << sh;
                    S.st[2 + which] |= dmk << sh;
                }
                run += S.h[which][b];
            }
            __syncthreads();
        }
    }
    if (threadIdx.x == 0) {
        const double xa = __longlong_as_double((long long)S.st[0]);
        const double xb = __longlong_as_double((long long)S.st[1]);
        double res;
        if (r0 == r1) {
            res = xa;
        } else {
            const double g = v - __builtin_floor(v);
            const double diff = xb - xa;
            res = g >= 0.5 ? xb - diff * (1.0 - g) : xa + diff * g;
        }
        S.res = res;
    }
    __syncthreads();
    const double out = S.res;
    __syncthreads();
    return out;
}

}  // namespace bsel
}  // namespace abcsmc
