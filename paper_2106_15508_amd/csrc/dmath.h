// dmath.h -- device-side numerics of the ABC-SMC hot path (gfx950, wave64).
//
// Every random quantity of the method is a transformed uniform (the
// reparameterisation of §III-A).  The transforms below are written so that
// each result is a fixed sequence of IEEE-754 binary64 operations
// (+ - * / sqrt fma floor rint ldexp frexp, all exact or correctly rounded on
// CDNA4 and built with -ffp-contract=off), which makes the draws, and hence
// the trajectories, reproducible bit for bit on any conforming machine:
//
//   u01(w)        ((w >> 12) + 1/2) * 2^-52                      in (0,1), exact
//   exp(x)        k = rint(x log2 e), r = (x - k ln2_hi) - k ln2_lo (fma),
//                 2^k * sum_{i<=13} r^i / i!   (Horner, fma); 0 below e^-708
//   log(x)        x = f 2^e, f in [1/sqrt2, sqrt2), s = (f-1)/(f+1),
//                 2 atanh(s) by its series to s^23, plus e ln2
//   log1p(x)      atanh series of x/(2+x) near 0, else log(1+x) + rounding error
//   expm1(x)      Taylor to x^14 for |x| <= ln2/2, else exp(x) - 1
//   cos/sin 2pi t quadrant and octant folding, Taylor to y^18 / y^17
//   normal pair   Box-Muller on the two 32-bit halves of one word
//   Bin(n,p)      sequential-search inversion when n min(p,1-p) < 10,
//                 else floor(m + 1/2 + sqrt(m(1-q)) z), clamped
//   Beta(a,b)     b integer: exp( sum_{m<b} log(U_m) / (a+m) )
//
// Counts are carried as doubles holding exact integers (< 2^53).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace abcsmc {
namespace dm {

// ---------------------------------------------------------------- Philox

struct u4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ u4 philox10(u4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t m0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t m1 = (uint64_t)0xCD9E8D57u * c.z;
        u4 n;
        n.x = (uint32_t)(m1 >> 32) ^ c.y ^ k0;
        n.y = (uint32_t)m1;
        n.z = (uint32_t)(m0 >> 32) ^ c.w ^ k1;
        n.w = (uint32_t)m0;
        c = n;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

enum : uint32_t { kPrior = 1, kPerturb = 2, kSim = 3 };

// The two 64-bit words of block `blk` of stream (index, round, purpose, sub).
struct w2 {
    uint64_t a, b;
};

__device__ __forceinline__ w2 block_words(uint64_t seed, uint32_t index, uint32_t round,
                                          uint32_t purpose, uint32_t sub, uint32_t blk)
{
    u4 c{index, round, (purpose << 24) | (sub & 0xFFFFFFu), blk};
    u4 o = philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    return w2{((uint64_t)o.y << 32) | o.x, ((uint64_t)o.w << 32) | o.z};
}

__device__ __forceinline__ double u01(uint64_t w)
{
    return ((double)(w >> 12) + 0.5) * 0x1p-52;
}

// ---------------------------------------------------------------- constants

constexpr double kLn2Hi = 0x1.62e42feep-1;           // ln 2 to 32 significant bits
constexpr double kLn2Lo = 0x1.a39ef35793c76p-33;     // ln 2 - kLn2Hi, rounded
constexpr double kLog2e = 1.4426950408889634;        // 1 / ln 2
constexpr double kSqrt1_2 = 0.70710678118654757;     // 1 / sqrt 2
constexpr double kHalfPi = 1.5707963267948966;       // pi / 2
constexpr double kExpHi = 709.782712893384;          // above: +inf
constexpr double kExpLo = -708.0;                    // below: 0

// 1/i! (i = 0..18), each the double nearest the exact value.
constexpr double kF0 = 1.0, kF1 = 1.0, kF2 = 1.0 / 2.0, kF3 = 1.0 / 6.0, kF4 = 1.0 / 24.0,
                 kF5 = 1.0 / 120.0, kF6 = 1.0 / 720.0, kF7 = 1.0 / 5040.0, kF8 = 1.0 / 40320.0,
                 kF9 = 1.0 / 362880.0, kF10 = 1.0 / 3628800.0, kF11 = 1.0 / 39916800.0,
                 kF12 = 1.0 / 479001600.0, kF13 = 1.0 / 6227020800.0,
                 kF14 = 1.0 / 87178291200.0, kF15 = 1.0 / 1307674368000.0,
                 kF16 = 1.0 / 20922789888000.0, kF17 = 1.0 / 355687428096000.0,
                 kF18 = 1.0 / 6402373705728000.0;

// ---------------------------------------------------------------- exp family

// e^r for |r| <= ln2/2 + tiny: degree-13 Taylor polynomial.
__device__ __forceinline__ double exp_poly(double r)
{
    double p = kF13;
    p = __builtin_fma(p, r, kF12);
    p = __builtin_fma(p, r, kF11);
    p = __builtin_fma(p, r, kF10);
    p = __builtin_fma(p, r, kF9);
    p = __builtin_fma(p, r, kF8);
    p = __builtin_fma(p, r, kF7);
    p = __builtin_fma(p, r, kF6);
    p = __builtin_fma(p, r, kF5);
    p = __builtin_fma(p, r, kF4);
    p = __builtin_fma(p, r, kF3);
    p = __builtin_fma(p, r, kF2);
    p = __builtin_fma(p, r, kF1);
    p = __builtin_fma(p, r, kF0);
    return p;
}

// exp(x) for x already known to lie in [kExpLo, kExpHi].
__device__ __forceinline__ double exp_core(double x)
{
    const double k = __builtin_rint(x * kLog2e);
    const double t = x - k * kLn2Hi;
    const double r = __builtin_fma(-k, kLn2Lo, t);
    return __builtin_ldexp(exp_poly(r), (int)k);
}

__device__ __forceinline__ double exp(double x)
{
    if (x != x) return x;
    if (x > kExpHi) return __builtin_inf();
    if (x < kExpLo) return 0.0;
    return exp_core(x);
}

__device__ __forceinline__ double expm1(double x)
{
    if (x != x) return x;
    if (__builtin_fabs(x) <= 0.34657359027997264) {
        double p = kF14;
        p = __builtin_fma(p, x, kF13);
        p = __builtin_fma(p, x, kF12);
        p = __builtin_fma(p, x, kF11);
        p = __builtin_fma(p, x, kF10);
        p = __builtin_fma(p, x, kF9);
        p = __builtin_fma(p, x, kF8);
        p = __builtin_fma(p, x, kF7);
        p = __builtin_fma(p, x, kF6);
        p = __builtin_fma(p, x, kF5);
        p = __builtin_fma(p, x, kF4);
        p = __builtin_fma(p, x, kF3);
        p = __builtin_fma(p, x, kF2);
        return __builtin_fma(x * x, p, x);
    }
    return exp(x) - 1.0;
}

// ---------------------------------------------------------------- log family

// s^2/3 + s^4/5 + ... + s^22/23 evaluated at z = s^2 (times z).
__device__ __forceinline__ double atanh_tail(double z)
{
    double q = 1.0 / 23.0;
    q = __builtin_fma(q, z, 1.0 / 21.0);
    q = __builtin_fma(q, z, 1.0 / 19.0);
    q = __builtin_fma(q, z, 1.0 / 17.0);
    q = __builtin_fma(q, z, 1.0 / 15.0);
    q = __builtin_fma(q, z, 1.0 / 13.0);
    q = __builtin_fma(q, z, 1.0 / 11.0);
    q = __builtin_fma(q, z, 1.0 / 9.0);
    q = __builtin_fma(q, z, 1.0 / 7.0);
    q = __builtin_fma(q, z, 1.0 / 5.0);
    q = __builtin_fma(q, z, 1.0 / 3.0);
    return z * q;
}

// log(x) for finite x > 0.
__device__ __forceinline__ double log_pos(double x)
{
    int e;
    double f = __builtin_frexp(x, &e);
    if (f < kSqrt1_2) {
        f = f * 2.0;
        e = e - 1;
    }
    const double a = f - 1.0;
    const double s = a / (2.0 + a);
    const double R = atanh_tail(s * s);
    const double lf = 2.0 * (s + s * R);
    const double de = (double)e;
    return de * kLn2Hi + (de * kLn2Lo + lf);
}

__device__ __forceinline__ double log(double x)
{
    if (x != x) return x;
    if (x < 0.0) return __builtin_nan("");
    if (x == 0.0) return -__builtin_inf();
    if (x == __builtin_inf()) return x;
    return log_pos(x);
}

__device__ __forceinline__ double log1p(double x)
{
    if (x != x) return x;
    if (x == -1.0) return -__builtin_inf();
    if (x < -1.0) return __builtin_nan("");
    if (x >= kSqrt1_2 - 1.0 && x <= 0.41421356237309515) {
        const double s = x / (2.0 + x);
        const double R = atanh_tail(s * s);
        return 2.0 * (s + s * R);
    }
    const double u = 1.0 + x;
    return log(u) + (x - (u - 1.0)) / u;
}

// ---------------------------------------------------------------- trig / normals

// (cos 2 pi t, sin 2 pi t) for t in [0, 1).
__device__ __forceinline__ void sincos2pi(double t, double& c, double& s)
{
    const double t4 = t * 4.0;
    const double q = __builtin_floor(t4);
    const double f = t4 - q;
    const bool fold = f > 0.5;
    const double g = fold ? 1.0 - f : f;
    const double y = g * kHalfPi;
    const double ny2 = -(y * y);
    double ps = kF17;
    ps = __builtin_fma(ps, ny2, kF15);
    ps = __builtin_fma(ps, ny2, kF13);
    ps = __builtin_fma(ps, ny2, kF11);
    ps = __builtin_fma(ps, ny2, kF9);
    ps = __builtin_fma(ps, ny2, kF7);
    ps = __builtin_fma(ps, ny2, kF5);
    ps = __builtin_fma(ps, ny2, kF3);
    ps = __builtin_fma(ps, ny2, kF1);
    const double sy = y * ps;
    double pc = kF18;
    pc = __builtin_fma(pc, ny2, kF16);
    pc = __builtin_fma(pc, ny2, kF14);
    pc = __builtin_fma(pc, ny2, kF12);
    pc = __builtin_fma(pc, ny2, kF10);
    pc = __builtin_fma(pc, ny2, kF8);
    pc = __builtin_fma(pc, ny2, kF6);
    pc = __builtin_fma(pc, ny2, kF4);
    pc = __builtin_fma(pc, ny2, kF2);
    pc = __builtin_fma(pc, ny2, kF0);
    const double cf = fold ? sy : pc;
    const double sf = fold ? pc : sy;
    const int iq = (int)q;
    if (iq == 0) {
        c = cf;
        s = sf;
    } else if (iq == 1) {
        c = -sf;
        s = cf;
    } else if (iq == 2) {
        c = -cf;
        s = -sf;
    } else {
        c = sf;
        s = -cf;
    }
}

// Box-Muller pair from one word: u1 = low half, u2 = high half.
__device__ __forceinline__ void normal_pair(uint64_t w, double& z0, double& z1)
{
    const double u1 = ((double)(uint32_t)w + 0.5) * 0x1p-32;
    const double u2 = ((double)(uint32_t)(w >> 32) + 0.5) * 0x1p-32;
    const double rho = __builtin_sqrt(-2.0 * log_pos(u1));
    double c, s;
    sincos2pi(u2, c, s);
    z0 = rho * c;
    z1 = rho * s;
}

// Cosine half of the pair only (the floor-normal and gamma samplers).
__device__ __forceinline__ double normal_one(uint64_t w)
{
    double z0, z1;
    normal_pair(w, z0, z1);
    return z0;
}

// ---------------------------------------------------------------- samplers

// Word w of stream (index, round, purpose, sub): half w % 2 of block w / 2.
__device__ __forceinline__ uint64_t word_at(uint64_t seed, uint32_t index, uint32_t round, uint32_t purpose,
                                            uint32_t sub, uint32_t w)
{
    const w2 b = block_words(seed, index, round, purpose, sub, w >> 1);
    return (w & 1u) ? b.b : b.a;
}

// Gamma(k) by Marsaglia & Tsang (ACM TOMS 2000): k' = k (k + 1 if k < 1),
// d = k' - 1/3, c = 1/sqrt(9 d); iteration m: z = first Box-Muller normal of
// word w0 + 2m, U from word w0 + 2m + 1, v = (1 + c z)^3, accept d v when
// v > 0 and log U < z^2/2 + d - d v + d log v; d after 32 rejections.  For
// k < 1 the result is scaled by U^(1/k), U from word w0 + 64.
__device__ __forceinline__ double gamma_mt(double k, uint64_t seed, uint32_t index, uint32_t round, uint32_t sub,
                                           uint32_t w0)
{
    const double kk = k < 1.0 ? k + 1.0 : k;
    const double d = kk - 1.0 / 3.0;
    const double c = 1.0 / __builtin_sqrt(9.0 * d);
    double g = d;
    for (uint32_t m = 0; m < 32; ++m) {
        const double z = normal_one(word_at(seed, index, round, kPerturb, sub, w0 + 2 * m));
        const double t = 1.0 + c * z;
        if (!(t > 0.0)) continue;
        const double v = t * t * t;
        const double U = u01(word_at(seed, index, round, kPerturb, sub, w0 + 2 * m + 1));
        if (log(U) < 0.5 * (z * z) + d - d * v + d * log(v)) {
            g = d * v;
            break;
        }
    }
    if (k < 1.0) g = g * exp(log(u01(word_at(seed, index, round, kPerturb, sub, w0 + 64))) / k);
    return g;
}

// Beta(a, b), real shapes: X / (X + Y), X ~ Gamma(a) from words 5.., Y ~
// Gamma(b) from words 70.. of the attempt's PERTURB stream; 0 if both vanish.
__device__ __forceinline__ double beta_general(double a, double b, uint64_t seed, uint32_t index, uint32_t round,
                                               uint32_t sub)
{
    const double X = gamma_mt(a, seed, index, round, sub, 5);
    const double Y = gamma_mt(b, seed, index, round, sub, 70);
    const double s = X + Y;
    return s > 0.0 ? X / s : 0.0;
}

constexpr double kTSwitch = 10.0;
constexpr int kBinvCap = 128;

// 1/j, j = 1..kBinvCap, rounded to nearest at compile time.  The inversion
// loop's step counter is the same in every lane still searching, so the
// entry is a wave-uniform (scalar) load.
struct RecipTab {
    double v[kBinvCap + 1];
    constexpr RecipTab() : v{}
    {
        for (int j = 1; j <= kBinvCap; ++j) v[j] = 1.0 / (double)j;
    }
};
__device__ constexpr RecipTab kRecip{};

// Bin(n, p) with the inversion uniform from word wu and, in the normal
// branch, the deviate of the Box-Muller pair of word wz (half 0: cosine,
// half 1: sine), formed on first use and kept in (have, z0, z1) for the
// draw that shares the pair; n is an exact integer held in a double.
__device__ __forceinline__ double binomial_pair(double n, double p, uint64_t wu, uint64_t wz, int half, bool& have,
                                                double& z0, double& z1)
{
    if (n <= 0.0 || p <= 0.0) return 0.0;
    if (p >= 1.0) return n;
    const bool flip = p > 0.5;
    const double q = flip ? 1.0 - p : p;
    const double m = n * q;
    double x;
    if (m < kTSwitch) {
        const double u = u01(wu);
        double f = exp(n * log1p(-q));
        double F = f;
        const double r = q / (1.0 - q);
        double k = 0.0;
        for (int it = 0; it < kBinvCap && u > F && k < n; ++it) {
            f = f * (((n - k) * r) * kRecip.v[it + 1]);  // (n - k) r / (k + 1), k = it
            k = k + 1.0;
            F = F + f;
        }
        x = k;
    } else {
        if (!have) {
            normal_pair(wz, z0, z1);
            have = true;
        }
        const double z = half ? z1 : z0;
        const double sd = __builtin_sqrt(m * (1.0 - q));
        const double y = (m + 0.5) + sd * z;
        x = __builtin_floor(y);
        if (x < 0.0) x = 0.0;
        if (x > n) x = n;
    }
    return flip ? n - x : x;
}

// Bin(n, p) from one word: its uniform and its cosine deviate.
__device__ __forceinline__ double binomial(double n, double p, uint64_t w)
{
    bool have = false;
    double z0, z1;
    return binomial_pair(n, p, w, w, 0, have, z0, z1);
}

// floor(N(h, sqrt h)) clamped to [0, n] (the paper's own transition sampler).
__device__ __forceinline__ double normal_floor(double n, double h, uint64_t w)
{
    if (n <= 0.0 || !(h > 0.0)) return 0.0;
    const double z = normal_one(w);
    double x = __builtin_floor(h + __builtin_sqrt(h) * z);
    if (x < 0.0) x = 0.0;
    if (x > n) x = n;
    return x;
}

}  // namespace dm
}  // namespace abcsmc
