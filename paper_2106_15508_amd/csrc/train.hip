// train.hip -- one minibatch step of the surrogate network's training in
// three kernels (forward and backward data pass, weight gradients, gradient
// reduction and Adam), on the CDNA4 matrix cores with bfloat16 operands and
// FP32 accumulation.
//
// Rounding points are those of the per-layer products: every matrix product
// rounds both operands to bfloat16 (nearest even) and sums in FP32; GELU'(a)
// is kept between the passes as float16 (nearest even); bias, GELU and its
// derivative, the loss gradient 2 (out - y) / (3 n), the elementwise products
// with GELU' and the bias sums are FP32; weights, their gradients and the
// Adam moments are FP32.
//
//   kernel 1 (train_pass_kernel): 32 or 64 rows per workgroup through the four
//     layers, the loss gradient, and back through the data products
//     g_l = (g_{l+1} W_{l+1}) * GELU'(a_l), all row-local (activations and
//     GELU' in LDS).  Writes the
//     layers' inputs h_{l-1} and gradients g_l transposed (feature-major,
//     bfloat16) for the weight products, the per-row squared errors and the
//     block's bias-gradient sums.
//   kernel 2 (train_wgrad_kernel): dW_l = g_l^T h_{l-1} of W2 and W3 over
//     the minibatch rows, as 128 x 128 output tiles over row slices (partial
//     sums per slice); the thin W1 and W4 are summed per row block by kernel 1.
//   kernel 3 (train_update_kernel): per parameter, the slices' (weights) or
//     blocks' (biases) partial sums added in fixed orders -- the gradient,
//     deterministic -- then Adam and the bfloat16 copies of the new weights,
//     row-major for the forward products and transposed for the backward
//     ones.  A small kernel makes both copies where the parameters were set
//     elsewhere.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"
#include "mlp.h"

namespace abcsmc {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kPT = 512;       // its threads: 8 waves
constexpr int kCW = kH / (kPT / 64);  // columns of a 256-wide layer per wave (32)
constexpr int kNB = kCW / 16;  // 16-column blocks per wave
constexpr int kTP = kH + 8;    // LDS pitch (bf16) of 256-wide rows (16-byte skew)
constexpr int kXP = 40;        // LDS pitch (bf16) of rows padded to K = 32
constexpr int kOffB1 = kH * kIn, kOffW2 = kOffB1 + kH, kOffB2 = kOffW2 + kH * kH, kOffW3 = kOffB2 + kH,
              kOffB3 = kOffW3 + kH * kH, kOffW4 = kOffB3 + kH, kOffB4 = kOffW4 + kOut * kH;

__device__ __forceinline__ __bf16 to_bf16(float f) { return (__bf16)f; }  // round to nearest even

// GELU (tanh form) and its derivative at x.  With y = c (x + 0.044715 x^3)
// and s = 1 / (1 + e^{-2y}) (the logistic function at 2y), 0.5 (1 + tanh y)
// = s, so GELU(x) = x s and GELU'(x) = s + x s (1 - s) 2 y'(x), where
// 2 y'(x) = 2c (1 + 3 * 0.044715 x^2).  One exponential and one reciprocal.
__device__ __forceinline__ void gelu_both(float x, float& g, float& dg)
{
    const float k1 = 2.0f * 0.7978845608028654f;  // 2c
    const float k3 = k1 * 0.044715f;              // 2c * 0.044715
    const float l2e = 1.4426950408889634f;        // log2(e): e^{-2y} = 2^{-2y log2 e}
    const float x2 = x * x;
    const float e = __builtin_amdgcn_exp2f(-x * fmaf(k3 * l2e, x2, k1 * l2e));  // e^{-2y}; +inf for large negative x (then s = 0)
    const float s = __builtin_amdgcn_rcpf(1.0f + e);
    g = x * s;
    dg = fmaf(g * (1.0f - s), fmaf(3.0f * k3, x2, k1), s);
}

__device__ __forceinline__ bf16x8 ld8(const __bf16* p) { return *reinterpret_cast<const bf16x8*>(p); }

// eight bf16 at p, p + stride, ..., p + 7 stride (a column of a row-major
// LDS array as a K-contiguous operand fragment)
__device__ __forceinline__ bf16x8 gather8(const __bf16* p, int stride)
{
    bf16x8 v;
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = p[j * stride];
    return v;
}

// four consecutive bf16 (8 bytes)
__device__ __forceinline__ void st4(__bf16* p, float a, float b, float c, float d)
{
    const bf16x4 v = {to_bf16(a), to_bf16(b), to_bf16(c), to_bf16(d)};
    *reinterpret_cast<bf16x4*>(p) = v;
}

__device__ __forceinline__ f32x4 mfma(const bf16x8& a, const bf16x8& b, const f32x4& c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Bias-gradient sums of one row block: the wave's RB * 4 values per column
// (rows 16a + 4 lg + e) summed in (a, e) order, then the four lane groups in
// order 0, 1, 2, 3 (every lane ends with the block total of its column).
template <int RB>
__device__ __forceinline__ float block_colsum(const float (&v)[RB][4])
{
    float s = 0.f;
#pragma unroll
    for (int a = 0; a < RB; ++a)
#pragma unroll
        for (int e = 0; e < 4; ++e) s += v[a][e];
    const int lane = threadIdx.x & 63;
    const float s0 = __shfl(s, lane & 15, 64), s1 = __shfl(s, 16 + (lane & 15), 64);
    const float s2 = __shfl(s, 32 + (lane & 15), 64), s3 = __shfl(s, 48 + (lane & 15), 64);
    return ((s0 + s1) + s2) + s3;
}

// ---------------------------------------------------------------------------
// Kernel 1.  TR rows per workgroup: 64 where the minibatch has rows for 256
// such workgroups (every workgroup fetches all four weight matrices, so 64
// rows halve the fetches per row), else 32 (8192 rows fill 256 compute
// units).  8 waves (two per SIMD, to overlap one wave's latencies with the
// other's work).  Wave w owns columns [32w, 32w + 32) of each 256-wide layer
// for the TR rows: RB x 2 blocks of 16 x 16 (lane holds rows 16i + 4 lg + e,
// column 16b + lr of block (i, b); lr = lane % 16, lg = lane / 16).  A
// layer's weight fragments are all requested before the previous layer's
// epilogue, so their L2 latency overlaps that work.  GELU'(a) of the three
// hidden layers waits in LDS for the backward products, rounded to float16
// (nearest even; two per 32-bit word, each thread its own words).
// ---------------------------------------------------------------------------
template <int TR>
__global__ __launch_bounds__(kPT) void train_pass_kernel(TrainArgs a)
{
    constexpr int RB = TR / 16;  // 16-row blocks
    __shared__ __attribute__((aligned(16))) __bf16 Hs[TR][kTP];  // h_l (forward), then g_l (backward)
    __shared__ __attribute__((aligned(16))) __bf16 Xs[TR][kXP];  // x, then g4, K padded to 32
    __shared__ float G4[TR][4];
    __shared__ float Dl[TR][4];
    __shared__ __attribute__((aligned(16))) __bf16 Xf[16][TR + 8];  // x feature-major (rows 8..15 zero), for dW1
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63, lr = lane & 15, lg = lane >> 4;
    const int blk = blockIdx.x;
    const int r0 = blk * TR;
    const int c0 = kCW * wave;
    const int n = a.n;
    const int64_t kp = a.kpad;
    const int64_t nblk = kp / 32;  // block stride of a slot group in dbp (room for 32-row blocks)
    const bf16x8 zero8 = {};

    // B fragments of a 256 x kCW slice whose column c has its K values
    // contiguous at W + c * 256: all eight K steps, requested at once
    bf16x8 bw[8][kNB];
    // lane offset of its fragments in a 256 x 256 matrix: row c0 + 16 b + lr,
    // K offset 8 lg (the K steps are immediate offsets of 64 bytes)
    const int wofs = (c0 + lr) * kH + 8 * lg;
    auto load_w = [&](const __bf16* W) {
#pragma unroll
        for (int b = 0; b < kNB; ++b) {
            const bf16x8* p = reinterpret_cast<const bf16x8*>(W + wofs + 16 * b * kH);
#pragma unroll
            for (int ks = 0; ks < 8; ++ks) bw[ks][b] = p[4 * ks];
        }
    };
    load_w(a.wb + kOffW2);  // layer 2's fragments, in flight through layer 1

    for (int i = t; i < TR * 32; i += kPT) {
        const int r = i >> 5, k = i & 31;
        const float v = (k < kIn && r0 + r < n) ? a.x[(int64_t)(r0 + r) * kIn + k] : 0.f;
        Xs[r][k] = to_bf16(v);
    }
    __syncthreads();
    for (int i = t; i < 16 * TR; i += kPT) {
        const int k = i / TR, r = i % TR;
        Xf[k][r] = Xs[r][k];                                       // zero for k >= 8
        if (k < kIn) a.ht[(int64_t)k * kp + r0 + r] = Xs[r][k];  // h0^T
    }

    f32x4 acc[RB][kNB];
    __shared__ __attribute__((aligned(16))) unsigned int DPs[3][RB * kNB * 2][kPT];  // GELU'(a_l), float16 pairs
    float dp[RB][kNB][4];  // GELU'(a_l) of the layer at hand, this lane's elements
    auto zero_acc = [&]() {
#pragma unroll
        for (int i = 0; i < RB; ++i)
#pragma unroll
            for (int j = 0; j < kNB; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    };
    // GELU'(a_l) to and from LDS as float16 (round to nearest even), the
    // pairs (e, e + 1) of a lane packed in one word at [l][pair][thread]
    auto store_dp = [&](int L) {
#pragma unroll
        for (int i = 0; i < RB; ++i)
#pragma unroll
            for (int b = 0; b < kNB; ++b)
#pragma unroll
                for (int e = 0; e < 4; e += 2) {
                    const _Float16 lo = (_Float16)dp[i][b][e], hi = (_Float16)dp[i][b][e + 1];
                    DPs[L][(i * kNB + b) * 2 + e / 2][t] = (unsigned int)__builtin_bit_cast(unsigned short, lo) |
                                                           ((unsigned int)__builtin_bit_cast(unsigned short, hi) << 16);
                }
    };
    auto load_dp = [&](int L) {
#pragma unroll
        for (int i = 0; i < RB; ++i)
#pragma unroll
            for (int b = 0; b < kNB; ++b)
#pragma unroll
                for (int e = 0; e < 4; e += 2) {
                    const unsigned int w = DPs[L][(i * kNB + b) * 2 + e / 2][t];
                    dp[i][b][e] = (float)__builtin_bit_cast(_Float16, (unsigned short)(w & 0xffffu));
                    dp[i][b][e + 1] = (float)__builtin_bit_cast(_Float16, (unsigned short)(w >> 16));
                }
    };
    // forward layers start from the bias: a = bias + sum_k h_k W_ck, the sum
    // accumulated onto it by the matrix core
    auto bias_acc = [&](const float* bias) {
#pragma unroll
        for (int b = 0; b < kNB; ++b) {
            const float bc = bias[c0 + 16 * b + lr];
#pragma unroll
            for (int i = 0; i < RB; ++i) acc[i][b] = f32x4{bc, bc, bc, bc};
        }
    };
    // acc += Hs (TR x 256) times the slice held in bw; the A fragments of K
    // step ks + 1 are read while step ks's products run (two steps' worth of
    // registers at most: the scheduling barrier keeps later reads from being
    // hoisted)
    auto product256 = [&]() {
        bf16x8 af[2][RB];
#pragma unroll
        for (int i = 0; i < RB; ++i) af[0][i] = ld8(&Hs[16 * i + lr][8 * lg]);
#pragma unroll
        for (int ks = 0; ks < 8; ++ks) {
            if (ks < 7) {
#pragma unroll
                for (int i = 0; i < RB; ++i) af[(ks + 1) & 1][i] = ld8(&Hs[16 * i + lr][32 * (ks + 1) + 8 * lg]);
            }
#pragma unroll
            for (int i = 0; i < RB; ++i)
#pragma unroll
                for (int b = 0; b < kNB; ++b) acc[i][b] = mfma(af[ks & 1][i], bw[ks][b], acc[i][b]);
            __builtin_amdgcn_sched_barrier(0);
        }
    };
    // forward epilogue of a hidden layer: a = acc (bias included), h = GELU(a);
    // GELU'(a) to d, h^T to global and h to hp (bfloat16, for LDS).
    auto fwd_epilogue = [&](float (&d)[RB][kNB][4], bf16x4 (&hp)[RB][kNB], __bf16* ht) {
#pragma unroll
        for (int b = 0; b < kNB; ++b) {
            const int c = c0 + 16 * b + lr;
            bf16x4* hrow = reinterpret_cast<bf16x4*>(ht + (int64_t)c * kp + r0 + 4 * lg);  // + 4 i: row block i
#pragma unroll
            for (int i = 0; i < RB; ++i) {
                float h[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) gelu_both(acc[i][b][e], h[e], d[i][b][e]);
                hp[i][b] = bf16x4{to_bf16(h[0]), to_bf16(h[1]), to_bf16(h[2]), to_bf16(h[3])};
                hrow[4 * i] = hp[i][b];
            }
        }
    };
    auto store_lds = [&](const bf16x4 (&hp)[RB][kNB]) {
#pragma unroll
        for (int b = 0; b < kNB; ++b)
#pragma unroll
            for (int i = 0; i < RB; ++i)
#pragma unroll
                for (int e = 0; e < 4; ++e) Hs[16 * i + 4 * lg + e][c0 + 16 * b + lr] = hp[i][b][e];
    };

    // ---- layer 1 (8 -> 256): one K step, K padded to 32
    {
        bias_acc(a.params + kOffB1);
        bf16x8 bfr[kNB];
#pragma unroll
        for (int b = 0; b < kNB; ++b) bfr[b] = lg == 0 ? ld8(a.wb + (int64_t)(c0 + 16 * b + lr) * kIn) : zero8;
#pragma unroll
        for (int i = 0; i < RB; ++i) {
            const bf16x8 af = ld8(&Xs[16 * i + lr][8 * lg]);
#pragma unroll
            for (int b = 0; b < kNB; ++b) acc[i][b] = mfma(af, bfr[b], acc[i][b]);
        }
        bf16x4 hv[RB][kNB];
        fwd_epilogue(dp, hv, a.ht + (int64_t)kIn * kp);
        store_dp(0);
        store_lds(hv);
        __syncthreads();
    }
    // ---- layer 2 (256 -> 256)
    {
        bias_acc(a.params + kOffB2);
        product256();
        load_w(a.wb + kOffW3);  // next: layer 3
        bf16x4 hv[RB][kNB];
        fwd_epilogue(dp, hv, a.ht + (int64_t)(kIn + kH) * kp);
        store_dp(1);
        __syncthreads();  // every wave has read h1
        store_lds(hv);
        __syncthreads();
    }
    // ---- layer 3 (256 -> 256)
    {
        bias_acc(a.params + kOffB3);
        product256();
        load_w(a.wt + kWt3);  // next: the g2 product
        bf16x4 hv[RB][kNB];
        fwd_epilogue(dp, hv, a.ht + (int64_t)(kIn + 2 * kH) * kp);
        store_dp(2);
        __syncthreads();  // every wave has read h2
        store_lds(hv);
        __syncthreads();
    }
    // ---- layer 4 (256 -> 3, N padded to 16): waves 0 .. RB-1 take rows [16w, 16w + 16)
    if (wave < RB) {
        f32x4 o = {0.f, 0.f, 0.f, 0.f};
        for (int k0 = 0; k0 < kH; k0 += 32) {
            const bf16x8 bfr = lr < kOut ? ld8(a.wb + kOffW4 + (int64_t)lr * kH + k0 + 8 * lg) : zero8;
            const bf16x8 af = ld8(&Hs[16 * wave + lr][k0 + 8 * lg]);
            o = mfma(af, bfr, o);
        }
        // out = o + b4; residual d = out - y; g4 = 2 d / (3 n) (0 past n)
        if (lr < kOut) {
            const float bc = a.params[kOffB4 + lr];
            float g4v[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = 16 * wave + 4 * lg + e;
                float d = 0.f, g = 0.f;
                if (r0 + row < n) {
                    d = (o[e] + bc) - a.y[(int64_t)(r0 + row) * kOut + lr];
                    g = 2.f * d / (3.f * (float)n);
                }
                Dl[row][lr] = d;
                G4[row][lr] = g;
                g4v[e] = g;
            }
            st4(a.gt + (int64_t)(3 * kH + lr) * kp + r0 + 16 * wave + 4 * lg, g4v[0], g4v[1], g4v[2], g4v[3]);
        }
    }
    __syncthreads();
    if (t < TR && r0 + t < n) {
        float s = 0.f;
        for (int c = 0; c < kOut; ++c) s += Dl[t][c] * Dl[t][c];
        a.se[r0 + t] = s;
    }
    if (t < kOut) {
        float s = 0.f;
        for (int r = 0; r < TR; ++r) s += G4[r][t];
        a.dbp[part_index(3 * kH + t, blk, nblk)] = s;
    }
    // bf16(g4) as the K-padded operand of the first data product
    for (int i = t; i < TR * 32; i += kPT) {
        const int r = i >> 5, k = i & 31;
        Xs[r][k] = to_bf16(k < kOut ? G4[r][k] : 0.f);
    }
    __syncthreads();
    // this block's part of dW4 = g4^T h3 (3 x 256, K = the block's rows):
    // A = bf16(g4) columns of Xs, B = h3 columns of Hs (the wave's own
    // columns, which only it overwrites later), both gathered K-contiguous
    {
        f32x4 w4[kNB];
#pragma unroll
        for (int b = 0; b < kNB; ++b) w4[b] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k0 = 0; k0 < TR; k0 += 32) {
            const bf16x8 af = gather8(&Xs[k0 + 8 * lg][lr], kXP);
#pragma unroll
            for (int b = 0; b < kNB; ++b)
                w4[b] = mfma(af, gather8(&Hs[k0 + 8 * lg][c0 + 16 * b + lr], kTP), w4[b]);
        }
        if (lg == 0) {  // rows c = e < 3 of the product
#pragma unroll
            for (int b = 0; b < kNB; ++b)
#pragma unroll
                for (int e = 0; e < kOut; ++e)
                    a.dbp[part_index(kBiasGrads + kH * kIn + e * kH + c0 + 16 * b + lr, blk, nblk)] = w4[b][e];
        }
    }

    // backward epilogue of hidden layer L (2, 1, 0): g = acc * GELU'(a_L);
    // g^T to global and g to gp (bfloat16), the block's bias sums (FP32 g).
    auto bwd_epilogue = [&](int L, const float (&d)[RB][kNB][4], bf16x4 (&gp)[RB][kNB]) {
        __bf16* gt = a.gt + (int64_t)(L * kH) * kp;
#pragma unroll
        for (int b = 0; b < kNB; ++b) {
            const int c = c0 + 16 * b + lr;
            float cs[RB][4];
            bf16x4* grow = reinterpret_cast<bf16x4*>(gt + (int64_t)c * kp + r0 + 4 * lg);  // + 4 i: row block i
#pragma unroll
            for (int i = 0; i < RB; ++i) {
#pragma unroll
                for (int e = 0; e < 4; ++e) cs[i][e] = acc[i][b][e] * d[i][b][e];
                gp[i][b] = bf16x4{to_bf16(cs[i][0]), to_bf16(cs[i][1]), to_bf16(cs[i][2]), to_bf16(cs[i][3])};
                grow[4 * i] = gp[i][b];
            }
            const float s = block_colsum<RB>(cs);
            if (lg == 0) a.dbp[part_index(L * kH + c, blk, nblk)] = s;
        }
    };
    // ---- g3 = (g4 W4) * GELU'(a3): K = 3 padded to 32, B from W4^T [256][8]
    {
        zero_acc();
        bf16x8 bfr[kNB];
#pragma unroll
        for (int b = 0; b < kNB; ++b) bfr[b] = lg == 0 ? ld8(a.wt + kWt4 + (int64_t)(c0 + 16 * b + lr) * 8) : zero8;
#pragma unroll
        for (int i = 0; i < RB; ++i) {
            const bf16x8 af = ld8(&Xs[16 * i + lr][8 * lg]);
#pragma unroll
            for (int b = 0; b < kNB; ++b) acc[i][b] = mfma(af, bfr[b], acc[i][b]);
        }
        bf16x4 gv[RB][kNB];
        load_dp(2);
        bwd_epilogue(2, dp, gv);
        store_lds(gv);  // Hs (h3) was last read by layer 4, before the barrier above
        __syncthreads();
    }
    // ---- g2 = (g3 W3) * GELU'(a2): B from W3^T
    {
        zero_acc();
        product256();
        load_w(a.wt + kWt2);  // next: the g1 product
        bf16x4 gv[RB][kNB];
        load_dp(1);
        bwd_epilogue(1, dp, gv);
        __syncthreads();  // every wave has read g3
        store_lds(gv);
        __syncthreads();
    }
    // ---- g1 = (g2 W2) * GELU'(a1): B from W2^T
    {
        zero_acc();
        product256();

        bf16x4 gv[RB][kNB];
        load_dp(0);
        bwd_epilogue(0, dp, gv);
        // this block's part of dW1 = g1^T h0 (256 x 8, K = the block's rows),
        // as dW1^T = h0^T g1 with both operands feature-major in LDS: x in
        // Xf, g1 in the GELU' space (free now)
        __bf16(*Gf)[TR + 8] = reinterpret_cast<__bf16(*)[TR + 8]>(&DPs[0][0][0]);
        __syncthreads();  // every wave is done with GELU'
#pragma unroll
        for (int b = 0; b < kNB; ++b)
#pragma unroll
            for (int i = 0; i < RB; ++i) *reinterpret_cast<bf16x4*>(&Gf[c0 + 16 * b + lr][16 * i + 4 * lg]) = gv[i][b];
        __syncthreads();
        f32x4 w1[kNB];
#pragma unroll
        for (int b = 0; b < kNB; ++b) w1[b] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k0 = 0; k0 < TR; k0 += 32) {
            const bf16x8 af = ld8(&Xf[lr][k0 + 8 * lg]);
#pragma unroll
            for (int b = 0; b < kNB; ++b) w1[b] = mfma(af, ld8(&Gf[c0 + 16 * b + lr][k0 + 8 * lg]), w1[b]);
        }
        if (lg < 2) {  // rows i = 4 lg + e < 8 of dW1^T
#pragma unroll
            for (int b = 0; b < kNB; ++b)
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    a.dbp[part_index(kBiasGrads + (4 * lg + e) * kH + c0 + 16 * b + lr, blk, nblk)] = w1[b][e];
        }
    }
}

// ---------------------------------------------------------------------------
// Kernel 2.  dW = g^T h over row slice s: C[m][n] = sum_k Gt[m][k] Ht[n][k]
// (both feature-major, K = rows contiguous).  Workgroup: one 128 x 128 output
// tile of W2 or W3, 4 waves of 64 x 64
// (4 x 4 blocks of 16 x 16).  K advances 64 rows a step through two LDS
// buffers (one barrier a step); each thread's global loads run three steps
// ahead of their LDS stores, so the L2 / HBM latency is spread over three
// steps of products.
// ---------------------------------------------------------------------------
constexpr int kWK = 64;          // K rows per step
constexpr int kWP = kWK + 8;     // LDS pitch (bf16)
constexpr int kWDepth = 3;       // steps whose loads are in flight

// one step's staging: thread t holds row t / 2 of both operands, K offsets
// 32 (t % 2) + 8 q (q = 0..3)
struct WStage {
    bf16x8 g[4], h[4];
};

// Workgroup L of the (1-D) grid: quads of four tiles, quad p = (L % 8) +
// 8 ((L / 8) / 4), tile (L / 8) % 4 of it, so that a quad's workgroups share
// an XCD (workgroups go to the eight XCDs in turn) and its second read of
// each operand row is served by that XCD's L2.  Quad p: slice p / 2 of W2
// (p even) or W3 (p odd); the thin W1 and W4 are summed per row block by
// the pass kernel.
__global__ __launch_bounds__(256) void train_wgrad_kernel(TrainArgs a, int krows, int kslice, int slices)
{
    __shared__ __attribute__((aligned(16))) __bf16 As[2][128][kWP];
    __shared__ __attribute__((aligned(16))) __bf16 Bs[2][128][kWP];
    const int L = blockIdx.x, quad = (L & 7) + 8 * ((L >> 3) >> 2), u = (L >> 3) & 3;
    if (quad >= 2 * slices) return;  // whole workgroup
    const int s = quad >> 1;
    struct { int mat, m0, n0; } tl = {1 + (quad & 1), 128 * (u >> 1), 128 * (u & 1)};
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63, lr = lane & 15, lg = lane >> 4;
    const int64_t kp = a.kpad;
    // operand matrices: rows of Gt (the layer's gradients) and of Ht (its inputs), and the output
    const int gOff = tl.mat == 1 ? kH : 2 * kH, hOff = tl.mat == 1 ? kIn : kIn + kH;
    const int wOff = tl.mat == 1 ? kOffW2 : kOffW3;
    // krows and kslice are multiples of kWK: every step is whole
    const int kb = s * kslice, ke = min(krows, kb + kslice);  // this minibatch's rows only
    const int nsteps = kb < ke ? (ke - kb) / kWK : 0;
    const int sr = t >> 1, sk = 32 * (t & 1);
    const __bf16* G = a.gt + (int64_t)(gOff + tl.m0 + sr) * kp + kb + sk;
    const __bf16* H = a.ht + (int64_t)(hOff + tl.n0 + sr) * kp + kb + sk;
    auto load = [&](int j, WStage& r) {
        if (j < nsteps) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                r.g[q] = ld8(G + j * kWK + 8 * q);
                r.h[q] = ld8(H + j * kWK + 8 * q);
            }
        }
    };
    auto stage = [&](int j, const WStage& r) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            *reinterpret_cast<bf16x8*>(&As[j & 1][sr][sk + 8 * q]) = r.g[q];
            *reinterpret_cast<bf16x8*>(&Bs[j & 1][sr][sk + 8 * q]) = r.h[q];
        }
    };
    f32x4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int wm = 64 * (wave >> 1), wn = 64 * (wave & 1);
    auto compute = [&](int j) {
#pragma unroll
        for (int kk = 0; kk < kWK; kk += 32) {
            bf16x8 af[4], bfr[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) af[i] = ld8(&As[j & 1][wm + 16 * i + lr][kk + 8 * lg]);
#pragma unroll
            for (int q = 0; q < 4; ++q) bfr[q] = ld8(&Bs[j & 1][wn + 16 * q + lr][kk + 8 * lg]);
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[i][q] = mfma(af[i], bfr[q], acc[i][q]);
        }
    };
    WStage r[kWDepth];
#pragma unroll
    for (int d = 0; d < kWDepth; ++d) load(d, r[d]);
    // step j: stage j (loaded three steps ago), load j + 3 into the freed
    // registers, barrier, products of step j
    for (int j0 = 0; j0 < nsteps; j0 += kWDepth) {
#pragma unroll
        for (int d = 0; d < kWDepth; ++d) {
            const int j = j0 + d;
            if (j < nsteps) {
                stage(j, r[d]);
                load(j + kWDepth, r[d]);
                __syncthreads();
                compute(j);
            }
        }
    }
    float* out = a.wpart + (int64_t)s * kWpartStride + wOff;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int m = tl.m0 + wm + 16 * i + 4 * lg + e, nn = tl.n0 + wn + 16 * j + lr;
                out[(int64_t)m * kH + nn] = acc[i][j][e];
            }
}

// Transposed bfloat16 weights for the backward products, from wb: W2^T and
// W3^T through 64 x 64 LDS tiles (grid.y 0, 1; 16 tiles each), W4^T [256][8]
// (columns 3..7 zero) in 16-row pieces (grid.y 2).
__global__ __launch_bounds__(256) void train_transpose_kernel(TrainArgs a)
{
    __shared__ __bf16 T[64][66];
    const int tile = blockIdx.x, mat = blockIdx.y;
    const int t = threadIdx.x;
    if (mat == 2) {  // W4^T: tile x covers rows k in [16x, 16x + 16)
        if (t < 128) {
            const int k = 16 * tile + (t >> 3), c = t & 7;
            a.wt[kWt4 + k * 8 + c] = c < kOut ? a.wb[kOffW4 + c * kH + k] : to_bf16(0.f);
        }
        return;
    }
    const int o0 = 64 * (tile >> 2), k0 = 64 * (tile & 3);
    const __bf16* W = a.wb + (mat == 0 ? kOffW2 : kOffW3);
    __bf16* WT = a.wt + (mat == 0 ? kWt2 : kWt3);
    for (int i = t; i < 64 * 64; i += 256) {
        const int r = i >> 6, c = i & 63;
        T[r][c] = W[(o0 + r) * kH + k0 + c];  // row o0 + r of W, columns k0 + c
    }
    __syncthreads();
    for (int i = t; i < 64 * 64; i += 256) {
        const int r = i >> 6, c = i & 63;
        WT[(k0 + r) * kH + o0 + c] = T[c][r];  // W^T[k][o] = W[o][k]
    }
}

// One Adam step (beta1 0.9, beta2 0.999, eps 1e-8; c1, c2 the bias corrections)
__device__ __forceinline__ void adam_math(float w, float m, float v, float g, float lr, float c1, float c2, float& wn,
                                          float& mn, float& vn)
{
    const float b1 = 0.9f, b2 = 0.999f;
    mn = b1 * m + (1.f - b1) * g;
    vn = b2 * v + (1.f - b2) * g * g;
    wn = w - lr * (mn / c1) / (sqrtf(vn / c2) + 1e-8f);
}

__device__ __forceinline__ float adam_one(const TrainArgs& a, int i, float g, float lr, float c1, float c2)
{
    float w, m, v;
    adam_math(a.params[i], a.am[i], a.av[i], g, lr, c1, c2, w, m, v);
    a.am[i] = m;
    a.av[i] = v;
    a.params[i] = w;
    a.wb[i] = to_bf16(w);
    return w;
}

// Workgroups of the update: 128 tiles of 32 x 32 weights of W2 and W3
// (their transposed bfloat16 copies written through LDS), then one per group
// of 16 slots of the block sums (the 771 biases, the 2816 weights of W1 and
// W4).
constexpr int kUpdTiles = 2 * (kH / 32) * (kH / 32);
constexpr int kUpdBlocks = kUpdTiles + kPartGroups;

// Parameter i's gradient: W2 and W3, the slices' sums in slice order; the
// biases, W1 and W4 (block sums of the pass kernel), lane l sums blocks l,
// l + 64, ... in order and the lanes are added by a fixed butterfly.  Written to grad if given; with lr > 0 the Adam step
// (bias corrections c1, c2 from the host) and the bfloat16 copies.
__global__ __launch_bounds__(256) void train_update_kernel(TrainArgs a, int slices, int blocks, float lr, float c1,
                                                           float c2)
{
    __shared__ __bf16 T[32][34];
    const int bx = blockIdx.x, t = threadIdx.x;
    if (bx < kUpdTiles) {
        // rows o0 + r, columns k0 + 4 cq .. + 3 of W (mat 0: W2, 1: W3)
        const int mat = bx >> 6, tile = bx & 63;
        const int o0 = 32 * (tile >> 3), k0 = 32 * (tile & 7);
        const int r = t >> 3, cq = t & 7;
        const int off = mat == 0 ? kOffW2 : kOffW3;
        const int i0 = off + (o0 + r) * kH + k0 + 4 * cq;
        // the Adam state and every slice's partial sums requested at once
        // (the sum is taken in slice order)
        const f32x4 w0 = *reinterpret_cast<const f32x4*>(a.params + i0);
        const f32x4 m0 = *reinterpret_cast<const f32x4*>(a.am + i0);
        const f32x4 v0 = *reinterpret_cast<const f32x4*>(a.av + i0);
        f32x4 p[kTrainSlices];
#pragma unroll
        for (int s = 0; s < kTrainSlices; ++s)
            p[s] = s < slices ? *reinterpret_cast<const f32x4*>(a.wpart + (int64_t)s * kWpartStride + i0)
                              : f32x4{0.f, 0.f, 0.f, 0.f};
        f32x4 g = p[0];
#pragma unroll
        for (int s = 1; s < kTrainSlices; ++s)
            if (s < slices) g += p[s];
        if (a.grad) *reinterpret_cast<f32x4*>(a.grad + i0) = g;
        if (!(lr > 0.f)) return;
        f32x4 wn, mn, vn;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            float we, me, ve;
            adam_math(w0[e], m0[e], v0[e], g[e], lr, c1, c2, we, me, ve);
            wn[e] = we;
            mn[e] = me;
            vn[e] = ve;
            T[4 * cq + e][r] = to_bf16(we);
        }
        *reinterpret_cast<f32x4*>(a.params + i0) = wn;
        *reinterpret_cast<f32x4*>(a.am + i0) = mn;
        *reinterpret_cast<f32x4*>(a.av + i0) = vn;
        *reinterpret_cast<bf16x4*>(a.wb + i0) = bf16x4{to_bf16(wn[0]), to_bf16(wn[1]), to_bf16(wn[2]), to_bf16(wn[3])};
        __syncthreads();
        // W^T rows k0 + r, columns o0 + 4 cq .. + 3
        __bf16* WT = a.wt + (mat == 0 ? kWt2 : kWt3);
        const bf16x4 v = {T[r][4 * cq], T[r][4 * cq + 1], T[r][4 * cq + 2], T[r][4 * cq + 3]};
        *reinterpret_cast<bf16x4*>(WT + (k0 + r) * kH + o0 + 4 * cq) = v;
        return;
    }
    // group G of 16 slots: thread (wave v, lane l) sums slot 16 G + l % 16 over
    // blocks q, q + 16, ... (q = 4 v + l / 16; each 16-lane quarter reads
    // whole 64-byte lines), the quarters are added by a fixed butterfly, the
    // four waves in order through LDS
    __shared__ float red[4][16];
    const int G = bx - kUpdTiles, lane = t & 63, v = t >> 6, j = lane & 15, q = 4 * v + (lane >> 4);
    const int64_t nblk = a.kpad / 32;
    float g = 0.f;
    for (int b0 = q; b0 < blocks; b0 += 32 * 16) {  // 32 loads in flight, added in block order
        float p[32];
#pragma unroll
        for (int u = 0; u < 32; ++u) {
            const int b = b0 + 16 * u;
            p[u] = b < blocks ? a.dbp[part_index(16 * G + j, b, nblk)] : 0.f;
        }
#pragma unroll
        for (int u = 0; u < 32; ++u)
            if (b0 + 16 * u < blocks) g += p[u];
    }
    g += __shfl_xor(g, 16, 64);
    g += __shfl_xor(g, 32, 64);
    if (lane < 16) red[v][j] = g;
    __syncthreads();
    if (t >= 16) return;
    const int slot = 16 * G + t;
    if (slot >= kPartSlots) return;
    g = ((red[0][t] + red[1][t]) + red[2][t]) + red[3][t];
    // slot -> parameter: b1, b2, b3, b4, then W1 (i-major) and W4 (flat)
    const int w = slot - kBiasGrads;
    const int i = slot < 3 * kH      ? (slot < kH ? kOffB1 + slot : slot < 2 * kH ? kOffB2 + slot - kH : kOffB3 + slot - 2 * kH)
                  : slot < kBiasGrads ? kOffB4 + slot - 3 * kH
                  : w < kH * kIn      ? (w % kH) * kIn + w / kH
                                      : kOffW4 + (w - kH * kIn);
    if (a.grad) a.grad[i] = g;
    if (!(lr > 0.f)) return;
    const float wn = adam_one(a, i, g, lr, c1, c2);
    if (i >= kOffW4 && i < kOffB4) {  // W4^T [256][8]: element (k, c) = W4[c][k]
        const int c = (i - kOffW4) / kH, k = (i - kOffW4) % kH;
        a.wt[kWt4 + k * 8 + c] = to_bf16(wn);
    }
}

// bfloat16 copy of the current parameters (before a pass that follows an
// update made elsewhere)
__global__ __launch_bounds__(256) void train_copies_kernel(TrainArgs a)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < kMlpParams) a.wb[i] = to_bf16(a.params[i]);
}

// Sum of the per-row squared errors in double, in a fixed order: block b of
// kSeParts adds rows b, b + kSeParts * 256 ... per thread, then its threads
// by a fixed tree; one block then adds the block sums in order.
__global__ __launch_bounds__(256) void se_part_kernel(const float* se, int64_t n, double* part)
{
    __shared__ double sh[256];
    double v = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)kSeParts * 256) v += (double)se[i];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(64) void se_total_kernel(double* part)
{
    if (threadIdx.x != 0) return;
    double v = 0.0;
    for (int b = 0; b < kSeParts; ++b) v += part[b];
    part[kSeParts] = v;
}

}  // namespace

void launch_se_sum(const float* se, int64_t n, double* part, hipStream_t s)
{
    hipLaunchKernelGGL(se_part_kernel, dim3(kSeParts), dim3(256), 0, s, se, n, part);
    hipLaunchKernelGGL(se_total_kernel, dim3(1), dim3(64), 0, s, part);
}

int train_slices(int64_t rows)
{
    const int64_t kp = (rows + kWK - 1) / kWK * kWK;
    // about 256 rows per slice or more, at most kTrainSlices (8 output
    // tiles x 32 slices: one workgroup per compute unit)
    return (int)std::max<int64_t>(1, std::min<int64_t>(kTrainSlices, kp / 256));
}

void launch_train_copies(const TrainArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(train_copies_kernel, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, a);
    hipLaunchKernelGGL(train_transpose_kernel, dim3(16, 3), dim3(256), 0, s, a);
}

void launch_train_step(const TrainArgs& a, float lr, int step, hipStream_t s)
{
    // rows padded to a multiple of 64 (the weight products' K step); the
    // padding rows have zero loss gradient
    const int64_t kp = ((int64_t)a.n + kWK - 1) / kWK * kWK;
    // 64 rows per pass workgroup where that still gives every compute unit one
    const bool wide = kp >= 64 * 256;
    const int blocks = (int)(kp / (wide ? 64 : 32));
    if (wide) hipLaunchKernelGGL(train_pass_kernel<64>, dim3(blocks), dim3(kPT), 0, s, a);
    else hipLaunchKernelGGL(train_pass_kernel<32>, dim3(blocks), dim3(kPT), 0, s, a);
    const int slices = train_slices(a.n);
    const int kslice = (int)(((kp + slices - 1) / slices + kWK - 1) / kWK * kWK);
    const int quads = 2 * slices;
    hipLaunchKernelGGL(train_wgrad_kernel, dim3(32 * ((quads + 7) / 8)), dim3(256), 0, s, a, (int)kp, kslice, slices);
    float c1 = 1.f, c2 = 1.f;
    if (lr > 0.f) {
        c1 = 1.f - powf(0.9f, (float)step);
        c2 = 1.f - powf(0.999f, (float)step);
    }
    hipLaunchKernelGGL(train_update_kernel, dim3(kUpdBlocks), dim3(256), 0, s, a, slices, blocks, lr, c1, c2);
}

}  // namespace abcsmc
