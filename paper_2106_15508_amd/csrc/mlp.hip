// mlp.hip -- the learned surrogate's forward pass: an MLP 8 -> 256 -> 256 ->
// 256 -> 3 with tanh-GELU activations, used to screen proposals by predicted
// distance (its training step is in train.hip).  Matrix products run on the
// CDNA4 matrix cores: v_mfma_f32_16x16x32_bf16 with operands rounded to
// bfloat16 (round to nearest even) and FP32 accumulation.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"
#include "mlp.h"

namespace abcsmc {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kTK = 32;  // K step (one v_mfma_f32_16x16x32_bf16)
constexpr int kLdsK = kTK + 8;  // LDS row pitch (bf16) of the input tile (16-byte skew between rows)

__device__ __forceinline__ __bf16 to_bf16(float f) { return (__bf16)f; }  // round to nearest even

// tanh(y) = 1 - 2 / (1 + e^{2y}) with the hardware exp and divide (absolute
// error ~1e-7, saturates correctly at +-inf).
__device__ __forceinline__ float tanh_fast(float y) { return 1.0f - __fdividef(2.0f, 1.0f + __expf(2.0f * y)); }

// GELU, tanh form: 0.5 x (1 + tanh(c (x + 0.044715 x^3))), c = sqrt(2/pi)
__device__ __forceinline__ float gelu_f(float x)
{
    const float c = 0.7978845608028654f;
    const float t = tanh_fast(c * (x + 0.044715f * x * x * x));
    return 0.5f * x * (1.0f + t);
}

// ---------------------------------------------------------------------------
// Fused inference (scoring): one workgroup carries 128 rows through all four
// layers.  The activations stay in LDS as bf16 ([128][264], 16-byte row skew);
// the weights are read as bf16 from global memory (they stay in L2).  Wave w
// computes output columns [64w, 64w + 64) of each 256-wide layer for all 128
// rows (8 x 4 blocks of 16 x 16, v_mfma_f32_16x16x32_bf16); layer 1's K = 8 and
// layer 4's N = 3 are zero-padded to the instruction's 32 and 16.  Rounding
// points are those of the per-layer products: bf16 operands, fp32 sums, bias
// and GELU in fp32, the activation rounded to bf16 for the next layer.  The
// score is sum_c expm1(yhat_c)^2, the predicted squared distance (the targets
// are log1p of the three per-series distances); NaN and overflow rank last.
constexpr int kFR = 128;       // rows per workgroup
constexpr int kHP = kH + 8;    // LDS row pitch (bf16) of the activations
constexpr int kOffB1 = kH * kIn, kOffW2 = kOffB1 + kH, kOffB2 = kOffW2 + kH * kH, kOffW3 = kOffB2 + kH,
              kOffB3 = kOffW3 + kH * kH, kOffW4 = kOffB3 + kH, kOffB4 = kOffW4 + kOut * kH;

__global__ __launch_bounds__(256) void to_bf16_kernel(const float* __restrict__ p, __bf16* __restrict__ q, int n)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) q[i] = to_bf16(p[i]);
}

// acc + bias, GELU, bf16 into H (rows 16a + 4(lane/16) + e, column n0 + 16b + lane%16)
__device__ __forceinline__ void fused_epilogue(f32x4 (&acc)[8][4], const float* __restrict__ bias, int n0, int lane,
                                               __bf16 (*H)[kHP])
{
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int c = n0 + 16 * b + lane % 16;
        const float bc = bias[c];
#pragma unroll
        for (int a = 0; a < 8; ++a)
#pragma unroll
            for (int e = 0; e < 4; ++e) H[16 * a + 4 * (lane / 16) + e][c] = to_bf16(gelu_f(acc[a][b][e] + bc));
    }
}

__global__ __launch_bounds__(256) void mlp_fused_kernel(const float* __restrict__ params, const __bf16* __restrict__ wb,
                                                        const float* __restrict__ x, int64_t n, float* out,
                                                        double* score)
{
    __shared__ __attribute__((aligned(16))) __bf16 H[kFR][kHP];
    __shared__ __attribute__((aligned(16))) __bf16 X0[kFR][kLdsK];
    __shared__ float O[kFR][4];
    const int t = threadIdx.x, wave = t / 64, lane = t % 64;
    const int64_t r0 = (int64_t)blockIdx.x * kFR;
    const int n0 = 64 * wave;
    const bf16x8 zero8 = {};
    // inputs as bf16, K padded to 32
    for (int i = t; i < kFR * kTK; i += 256) {
        const int r = i / kTK, k = i % kTK;
        float v = 0.f;
        if (k < kIn && r0 + r < n) v = x[(r0 + r) * kIn + k];
        X0[r][k] = to_bf16(v);
    }
    __syncthreads();
    f32x4 acc[8][4];
    // layer 1 (8 -> 256): one K step
    {
#pragma unroll
        for (int a = 0; a < 8; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
        bf16x8 bfr[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int c = n0 + 16 * b + lane % 16;
            bfr[b] = lane / 16 == 0 ? *reinterpret_cast<const bf16x8*>(wb + (size_t)c * kIn) : zero8;
        }
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            const bf16x8 af = *reinterpret_cast<const bf16x8*>(&X0[16 * a + lane % 16][8 * (lane / 16)]);
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bfr[b], acc[a][b], 0, 0, 0);
        }
        fused_epilogue(acc, params + kOffB1, n0, lane, H);
    }
    __syncthreads();
    // layers 2 and 3 (256 -> 256)
    for (int L = 0; L < 2; ++L) {
        const __bf16* W = wb + (L == 0 ? kOffW2 : kOffW3);
        const float* bias = params + (L == 0 ? kOffB2 : kOffB3);
#pragma unroll
        for (int a = 0; a < 8; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
        for (int k0 = 0; k0 < kH; k0 += kTK) {
            bf16x8 bfr[4];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int c = n0 + 16 * b + lane % 16;
                bfr[b] = *reinterpret_cast<const bf16x8*>(W + (size_t)c * kH + k0 + 8 * (lane / 16));
            }
#pragma unroll
            for (int a = 0; a < 8; ++a) {
                const bf16x8 af = *reinterpret_cast<const bf16x8*>(&H[16 * a + lane % 16][k0 + 8 * (lane / 16)]);
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bfr[b], acc[a][b], 0, 0, 0);
            }
        }
        __syncthreads();  // every wave has read H
        fused_epilogue(acc, bias, n0, lane, H);
        __syncthreads();
    }
    // layer 4 (256 -> 3, N padded to 16): wave w takes rows [32w, 32w + 32)
    {
        f32x4 o[2] = {f32x4{0.f, 0.f, 0.f, 0.f}, f32x4{0.f, 0.f, 0.f, 0.f}};
        const int c = lane % 16;
        for (int k0 = 0; k0 < kH; k0 += kTK) {
            const bf16x8 bfr = c < kOut ? *reinterpret_cast<const bf16x8*>(wb + kOffW4 + (size_t)c * kH + k0 + 8 * (lane / 16))
                                        : zero8;
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                const bf16x8 af =
                    *reinterpret_cast<const bf16x8*>(&H[32 * wave + 16 * a + lane % 16][k0 + 8 * (lane / 16)]);
                o[a] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bfr, o[a], 0, 0, 0);
            }
        }
        if (c < kOut) {
            const float bc = params[kOffB4 + c];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int e = 0; e < 4; ++e) O[32 * wave + 16 * a + 4 * (lane / 16) + e][c] = o[a][e] + bc;
        }
    }
    __syncthreads();
    if (t < kFR && r0 + t < n) {
        const int64_t row = r0 + t;
        if (out)
            for (int c = 0; c < kOut; ++c) out[row * kOut + c] = O[t][c];
        if (score) {
            double sc = 0.0;
            for (int c = 0; c < kOut; ++c) {
                const double e = expm1((double)O[t][c]);
                sc += e * e;
            }
            score[row] = sc <= 1.0e300 ? sc : __builtin_inf();
        }
    }
}

}  // namespace

void mlp_infer(const float* params, __bf16* wb, const float* x, int64_t n, float* out, double* score, hipStream_t st)
{
    hipLaunchKernelGGL(to_bf16_kernel, dim3((kMlpParams + 255) / 256), dim3(256), 0, st, params, wb, kMlpParams);
    if (n > 0)
        hipLaunchKernelGGL(mlp_fused_kernel, dim3((unsigned)((n + kFR - 1) / kFR)), dim3(256), 0, st, params,
                           (const __bf16*)wb, x, n, out, score);
}

}  // namespace abcsmc
