// opcount.cpp -- op-counting build of the CPU oracle.
//
// MEASUREMENT INFRASTRUCTURE ONLY (like the oracle itself: only the tests and
// the op-count script load it).  The oracle's C source is compiled here as
// C++ with its `double` replaced by F64, a one-member wrapper (same size and
// layout as a double, so the oracle's ctypes interface is unchanged) whose
// operators perform the same IEEE operation and count it.  Every branch the
// oracle takes is therefore the one it takes in the plain build, and the
// counts are the FP64 operations the method performs on those branches.
//
// Categories: additions/subtractions, multiplications, divisions, square
// roots, fused multiply-adds, comparisons, int<->double conversions,
// roundings to integer (floor, rint), scalings (ldexp, frexp) and fabs.
// Flops = add + mul + div + sqrt + 2 fma.  Negation is a sign flip and is not
// counted.
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <cmath>

namespace opc {
enum Kind { ADD, MUL, DIV, SQRT, FMA, CMP, CVT, RND, SCALE, ABS, NKIND };
static uint64_t g_count[NKIND];
static inline void tick(Kind k) { ++g_count[k]; }
}  // namespace opc

struct F64 {
    double v;
    F64() = default;
    F64(double x) : v(x) {}  // a literal or a value already in FP64: no operation
    F64(float x) : v(x) {}
    F64(int x) : v((double)x) { opc::tick(opc::CVT); }
    F64(long x) : v((double)x) { opc::tick(opc::CVT); }
    F64(long long x) : v((double)x) { opc::tick(opc::CVT); }
    F64(unsigned x) : v((double)x) { opc::tick(opc::CVT); }
    F64(unsigned long x) : v((double)x) { opc::tick(opc::CVT); }
    F64(unsigned long long x) : v((double)x) { opc::tick(opc::CVT); }
    explicit operator double() const { return v; }
    explicit operator int() const { opc::tick(opc::CVT); return (int)v; }
    explicit operator long() const { opc::tick(opc::CVT); return (long)v; }
    explicit operator long long() const { opc::tick(opc::CVT); return (long long)v; }
    explicit operator unsigned long() const { opc::tick(opc::CVT); return (unsigned long)v; }
    explicit operator unsigned long long() const { opc::tick(opc::CVT); return (unsigned long long)v; }
    F64& operator+=(F64 o) { opc::tick(opc::ADD); v = v + o.v; return *this; }
    F64& operator-=(F64 o) { opc::tick(opc::ADD); v = v - o.v; return *this; }
    F64& operator*=(F64 o) { opc::tick(opc::MUL); v = v * o.v; return *this; }
    F64& operator/=(F64 o) { opc::tick(opc::DIV); v = v / o.v; return *this; }
};
static_assert(sizeof(F64) == sizeof(double), "F64 must have the layout of a double");

static inline F64 operator+(F64 a, F64 b) { opc::tick(opc::ADD); return F64(a.v + b.v); }
static inline F64 operator-(F64 a, F64 b) { opc::tick(opc::ADD); return F64(a.v - b.v); }
static inline F64 operator*(F64 a, F64 b) { opc::tick(opc::MUL); return F64(a.v * b.v); }
static inline F64 operator/(F64 a, F64 b) { opc::tick(opc::DIV); return F64(a.v / b.v); }
static inline F64 operator-(F64 a) { return F64(-a.v); }
static inline bool operator<(F64 a, F64 b) { opc::tick(opc::CMP); return a.v < b.v; }
static inline bool operator>(F64 a, F64 b) { opc::tick(opc::CMP); return a.v > b.v; }
static inline bool operator<=(F64 a, F64 b) { opc::tick(opc::CMP); return a.v <= b.v; }
static inline bool operator>=(F64 a, F64 b) { opc::tick(opc::CMP); return a.v >= b.v; }
static inline bool operator==(F64 a, F64 b) { opc::tick(opc::CMP); return a.v == b.v; }
static inline bool operator!=(F64 a, F64 b) { opc::tick(opc::CMP); return a.v != b.v; }

static inline F64 fma(F64 a, F64 b, F64 c) { opc::tick(opc::FMA); return F64(std::fma(a.v, b.v, c.v)); }
static inline F64 sqrt(F64 a) { opc::tick(opc::SQRT); return F64(std::sqrt(a.v)); }
static inline F64 floor(F64 a) { opc::tick(opc::RND); return F64(std::floor(a.v)); }
static inline F64 rint(F64 a) { opc::tick(opc::RND); return F64(std::rint(a.v)); }
static inline F64 fabs(F64 a) { opc::tick(opc::ABS); return F64(std::fabs(a.v)); }
static inline F64 ldexp(F64 a, int e) { opc::tick(opc::SCALE); return F64(std::ldexp(a.v, e)); }
static inline F64 frexp(F64 a, int* e) { opc::tick(opc::SCALE); return F64(std::frexp(a.v, e)); }

#define double F64
extern "C" {
#include "abcsmc_ref.c"
}
#undef double

extern "C" {

void opc_reset(void) { memset(opc::g_count, 0, sizeof opc::g_count); }

// out[0..9]: add, mul, div, sqrt, fma, cmp, cvt, rnd, scale, abs
void opc_read(uint64_t* out)
{
    for (int k = 0; k < opc::NKIND; ++k) out[k] = opc::g_count[k];
}

}  // extern "C"
