// mlp.hip -- the learned surrogate: an MLP 8 -> 256 -> 256 -> 256 -> 3 with
// tanh-GELU activations, trained on the GPU on simulator outputs, used to
// screen proposals by predicted distance.  Matrix products run on the CDNA4
// matrix cores: v_mfma_f32_16x16x32_bf16 with operands rounded to bfloat16
// (round to nearest even) as they are staged into LDS and FP32 accumulation;
// master weights, activations, gradients and Adam state are FP32.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"
#include "mlp.h"

namespace abcsmc {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kTK = 32;           // K step (one v_mfma_f32_16x16x32_bf16)
constexpr int kLdsK = kTK + 8;    // LDS row pitch in bf16 (16-byte skew between rows)

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
__device__ __forceinline__ float gelu_grad_f(float x)
{
    const float c = 0.7978845608028654f;
    const float x2 = x * x;
    const float t = tanh_fast(c * (x + 0.044715f * x2 * x));
    return 0.5f * (1.0f + t) + 0.5f * x * (1.0f - t * t) * c * (1.0f + 3.0f * 0.044715f * x2);
}

// Stage rows [r0, r0 + kR) x k [k0, k0 + 32) of op(X) into S[row][k] as bf16,
// op(X)(r, k) = kcontig ? X[r*ld + k] : X[k*ld + r]; entries outside R x K are 0.
// vec: ld % 4 == 0 and X 16-byte aligned (float4 loads along the contiguous axis).
template <int kR>
__device__ __forceinline__ void stage_tile(const float* __restrict__ X, int ld, bool kcontig, int R, int K, int r0,
                                           int k0, __bf16 (*S)[kLdsK], int t, bool vec)
{
    constexpr int kIters = kR * kTK / 4 / 256;  // float4 per thread
    if (kcontig) {
#pragma unroll
        for (int i = 0; i < kIters; ++i) {
            const int idx = t + 256 * i;
            const int r = idx >> 3, kk = (idx & 7) * 4;
            const int gr = r0 + r, gk = k0 + kk;
            float v[4] = {0.f, 0.f, 0.f, 0.f};
            if (gr < R) {
                const float* src = X + (size_t)gr * ld + gk;
                if (vec && gk + 3 < K) {
                    const float4 f = *reinterpret_cast<const float4*>(src);
                    v[0] = f.x; v[1] = f.y; v[2] = f.z; v[3] = f.w;
                } else {
                    for (int e = 0; e < 4; ++e)
                        if (gk + e < K) v[e] = src[e];
                }
            }
            typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
            const bf16x4 pk = {to_bf16(v[0]), to_bf16(v[1]), to_bf16(v[2]), to_bf16(v[3])};
            *reinterpret_cast<bf16x4*>(&S[r][kk]) = pk;  // 8-byte aligned: kk % 4 == 0, pitch 80 bytes
        }
    } else {
        constexpr int kRow4 = kR / 4;  // float4 per k row
#pragma unroll
        for (int i = 0; i < kIters; ++i) {
            const int idx = t + 256 * i;
            const int kk = idx / kRow4, r = (idx % kRow4) * 4;
            const int gk = k0 + kk, gr = r0 + r;
            float v[4] = {0.f, 0.f, 0.f, 0.f};
            if (gk < K) {
                const float* src = X + (size_t)gk * ld + gr;
                if (vec && gr + 3 < R) {
                    const float4 f = *reinterpret_cast<const float4*>(src);
                    v[0] = f.x; v[1] = f.y; v[2] = f.z; v[3] = f.w;
                } else {
                    for (int e = 0; e < 4; ++e)
                        if (gr + e < R) v[e] = src[e];
                }
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) S[r + e][kk] = to_bf16(v[e]);
        }
    }
}

// C[M x N] = epi( op(A)[M x K] op(B)[K x N] ), row-major FP32 storage:
//   op(A)(m,k) = transA ? A[k*lda + m] : A[m*lda + k]
//   op(B)(k,n) = transB ? B[n*ldb + k] : B[k*ldb + n]
// epilogue (GemmArgs::epi): v = acc (+ C if accumulate) (+ bias[n]);
//   kStore: C = v; kGelu: P = v (if P), C = gelu(v); kGeluGrad: C = v * gelu'(P).
// Workgroup: 256 threads = 4 waves, tile kBM x kBN; wave w owns the
// (kBM/2) x (kBN/2) quadrant (w/2, w%2) as 16 x 16 MFMA blocks.  LDS keeps A
// as [kBM][32] and B transposed as [kBN][32] (both K-contiguous) so each
// lane's operand is one 16-byte read.  With gridDim.z > 1 (split K) slice z
// covers k in [z*kchunk, (z+1)*kchunk) and writes its raw sum to
// part + z*M*N (the reduction applies the epilogue).
template <int kBM, int kBN>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(GemmArgs g, int kchunk, float* part)
{
    __shared__ __attribute__((aligned(16))) __bf16 As[kBM][kLdsK];
    __shared__ __attribute__((aligned(16))) __bf16 Bs[kBN][kLdsK];
    constexpr int kFM = kBM / 32, kFN = kBN / 32;  // 16 x 16 blocks per wave
    const int t = threadIdx.x;
    const int wave = t / 64, lane = t % 64;
    const int m0 = blockIdx.y * kBM, n0 = blockIdx.x * kBN;
    const int wm = (wave / 2) * (kBM / 2), wn = (wave % 2) * (kBN / 2);
    const int kb = blockIdx.z * kchunk, ke = min(g.K, kb + kchunk);
    const bool vecA = (g.lda % 4 == 0) && ((reinterpret_cast<uintptr_t>(g.A) & 15) == 0);
    const bool vecB = (g.ldb % 4 == 0) && ((reinterpret_cast<uintptr_t>(g.B) & 15) == 0);
    f32x4 acc[kFM][kFN];
#pragma unroll
    for (int a = 0; a < kFM; ++a)
#pragma unroll
        for (int b = 0; b < kFN; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = kb; k0 < ke; k0 += kTK) {
        stage_tile<kBM>(g.A, g.lda, !g.transA, g.M, ke, m0, k0, As, t, vecA);
        stage_tile<kBN>(g.B, g.ldb, g.transB, g.N, ke, n0, k0, Bs, t, vecB);
        __syncthreads();
        bf16x8 af[kFM], bfr[kFN];
#pragma unroll
        for (int a = 0; a < kFM; ++a)
            af[a] = *reinterpret_cast<const bf16x8*>(&As[wm + 16 * a + lane % 16][8 * (lane / 16)]);
#pragma unroll
        for (int b = 0; b < kFN; ++b)
            bfr[b] = *reinterpret_cast<const bf16x8*>(&Bs[wn + 16 * b + lane % 16][8 * (lane / 16)]);
#pragma unroll
        for (int a = 0; a < kFM; ++a)
#pragma unroll
            for (int b = 0; b < kFN; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[a], bfr[b], acc[a][b], 0, 0, 0);
        __syncthreads();
    }
    // lane holds D[4*(lane/16)+e][lane%16] of each 16 x 16 block
    float* slice = part ? part + (size_t)blockIdx.z * g.M * g.N : nullptr;
#pragma unroll
    for (int a = 0; a < kFM; ++a)
#pragma unroll
        for (int b = 0; b < kFN; ++b)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int m = m0 + wm + 16 * a + 4 * (lane / 16) + e;
                const int n = n0 + wn + 16 * b + lane % 16;
                if (m >= g.M || n >= g.N) continue;
                float v = acc[a][b][e];
                if (slice) {
                    slice[(size_t)m * g.N + n] = v;
                    continue;
                }
                const size_t o = (size_t)m * g.ldc + n;
                if (g.accumulate) v += g.C[o];
                if (g.bias) v += g.bias[n];
                if (g.epi == kGelu) {
                    if (g.P) g.P[o] = v;
                    g.C[o] = gelu_f(v);
                } else if (g.epi == kGeluGrad) {
                    g.C[o] = v * gelu_grad_f(g.P[o]);
                } else {
                    g.C[o] = v;
                }
            }
}

// C = sum over slices z (in order) of part[z] (split-K reduction, kStore).
__global__ __launch_bounds__(256) void splitk_reduce_kernel(const float* part, int splits, int M, int N, float* C,
                                                            int ldc)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= M * N) return;
    float v = 0.f;
    for (int z = 0; z < splits; ++z) v += part[(size_t)z * M * N + i];
    C[(size_t)(i / N) * ldc + i % N] = v;
}

// Bias gradients out[n] = sum over m of X[m*ld + n]: chunk c of 256 rows
// sums its rows in order into part[c][n], then the chunks are added in order.
constexpr int kColRows = 64;
__global__ __launch_bounds__(256) void colsum_part_kernel(const float* X, int M, int N, int ld, float* part)
{
    const int n = blockIdx.x * 256 + threadIdx.x;
    if (n >= N) return;
    const int m0 = blockIdx.y * kColRows, m1 = min(M, m0 + kColRows);
    float s = 0.f;
#pragma unroll 16
    for (int m = m0; m < m1; ++m) s += X[(size_t)m * ld + n];
    part[(size_t)blockIdx.y * N + n] = s;
}

__global__ __launch_bounds__(256) void colsum_reduce_kernel(const float* part, int chunks, int N, float* out)
{
    const int n = blockIdx.x * 256 + threadIdx.x;
    if (n >= N) return;
    float s = 0.f;
#pragma unroll 16
    for (int c = 0; c < chunks; ++c) s += part[(size_t)c * N + n];
    out[n] = s;
}

// dOut = 2 (out - y) / (3 n); per-sample squared error for the loss.
__global__ __launch_bounds__(256) void mse_grad_kernel(const float* out, const float* y, int n, float* dout, float* se)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    float s = 0.f;
    for (int c = 0; c < 3; ++c) {
        const float d = out[i * 3 + c] - y[i * 3 + c];
        dout[i * 3 + c] = 2.f * d / (3.f * (float)n);
        s += d * d;
    }
    se[i] = s;
}

__global__ __launch_bounds__(256) void adam_kernel(float* w, const float* gr, float* m, float* v, int n, float lr,
                                                   float b1, float b2, float eps, float c1, float c2)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float g = gr[i];
    const float mi = b1 * m[i] + (1.f - b1) * g;
    const float vi = b2 * v[i] + (1.f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
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

void launch_gemm(const GemmArgs& g, float* part, hipStream_t s)
{
    if (g.M <= 0 || g.N <= 0) return;
    const int64_t big = ((int64_t)(g.M + 127) / 128) * ((g.N + 127) / 128);
    if (big >= 256) {
        const dim3 grid((g.N + 127) / 128, (g.M + 127) / 128, 1);
        hipLaunchKernelGGL((gemm_bf16_kernel<128, 128>), grid, dim3(256), 0, s, g, g.K, (float*)nullptr);
        return;
    }
    const dim3 grid((g.N + 63) / 64, (g.M + 63) / 64, 1);
    const int tiles = (int)(grid.x * grid.y);
    // split K for the few-tile, long-K products (weight gradients)
    int splits = 1;
    if (part && g.epi == kStore && !g.bias && !g.accumulate && g.ldc >= g.N) {
        splits = std::min(std::min(kSplitMax, std::max(1, 512 / tiles)), std::max(1, g.K / 256));
        if ((int64_t)splits * g.M * g.N > kSplitFloats) splits = (int)std::max<int64_t>(1, kSplitFloats / ((int64_t)g.M * g.N));
    }
    if (splits <= 1) {
        hipLaunchKernelGGL((gemm_bf16_kernel<64, 64>), grid, dim3(256), 0, s, g, g.K, (float*)nullptr);
        return;
    }
    const int kchunk = ((g.K + splits - 1) / splits + kTK - 1) / kTK * kTK;
    splits = (g.K + kchunk - 1) / kchunk;
    hipLaunchKernelGGL((gemm_bf16_kernel<64, 64>), dim3(grid.x, grid.y, splits), dim3(256), 0, s, g, kchunk, part);
    hipLaunchKernelGGL(splitk_reduce_kernel, dim3((g.M * g.N + 255) / 256), dim3(256), 0, s, part, splits, g.M, g.N,
                       g.C, g.ldc);
}

void launch_colsum(const float* X, int M, int N, int ld, float* out, float* part, hipStream_t s)
{
    const int chunks = (M + kColRows - 1) / kColRows;
    hipLaunchKernelGGL(colsum_part_kernel, dim3((N + 255) / 256, chunks), dim3(256), 0, s, X, M, N, ld, part);
    hipLaunchKernelGGL(colsum_reduce_kernel, dim3((N + 255) / 256), dim3(256), 0, s, part, chunks, N, out);
}

void launch_mse_grad(const float* out, const float* y, int n, float* dout, float* se, hipStream_t s)
{
    hipLaunchKernelGGL(mse_grad_kernel, dim3((n + 255) / 256), dim3(256), 0, s, out, y, n, dout, se);
}

void launch_adam(float* w, const float* g, float* m, float* v, int n, float lr, int step, hipStream_t s)
{
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(adam_kernel, dim3((n + 255) / 256), dim3(256), 0, s, w, g, m, v, n, lr, b1, b2, 1e-8f, c1, c2);
}


// ---------------------------------------------------------------------------
// Network passes built from the GEMM.  Parameters, flat FP32:
//   W1[256][8] b1[256] W2[256][256] b2[256] W3[256][256] b3[256] W4[3][256] b4[3]
// ---------------------------------------------------------------------------
MlpView mlp_view(float* p)
{
    MlpView v;
    v.W1 = p;
    v.b1 = v.W1 + kH * kIn;
    v.W2 = v.b1 + kH;
    v.b2 = v.W2 + kH * kH;
    v.W3 = v.b2 + kH;
    v.b3 = v.W3 + kH * kH;
    v.W4 = v.b3 + kH;
    v.b4 = v.W4 + kOut * kH;
    return v;
}

static GemmArgs gemm(const float* A, int lda, bool ta, const float* B, int ldb, bool tb, float* C, int ldc, int M,
                     int N, int K)
{
    GemmArgs g{};
    g.A = A;
    g.lda = lda;
    g.transA = ta;
    g.B = B;
    g.ldb = ldb;
    g.transB = tb;
    g.C = C;
    g.ldc = ldc;
    g.M = M;
    g.N = N;
    g.K = K;
    g.epi = kStore;
    return g;
}

// Forward over n rows of x (n x 8): a_l pre-activations, h_l activations, out n x 3.
void mlp_forward(const float* params, const float* x, int n, MlpActs& s, hipStream_t st)
{
    MlpView w = mlp_view(const_cast<float*>(params));
    GemmArgs g = gemm(x, kIn, false, w.W1, kIn, true, s.h1, kH, n, kH, kIn);
    g.bias = w.b1;
    g.epi = kGelu;
    g.P = s.a1;
    launch_gemm(g, nullptr, st);
    g = gemm(s.h1, kH, false, w.W2, kH, true, s.h2, kH, n, kH, kH);
    g.bias = w.b2;
    g.epi = kGelu;
    g.P = s.a2;
    launch_gemm(g, nullptr, st);
    g = gemm(s.h2, kH, false, w.W3, kH, true, s.h3, kH, n, kH, kH);
    g.bias = w.b3;
    g.epi = kGelu;
    g.P = s.a3;
    launch_gemm(g, nullptr, st);
    g = gemm(s.h3, kH, false, w.W4, kH, true, s.out, kOut, n, kOut, kH);
    g.bias = w.b4;
    launch_gemm(g, nullptr, st);
}

void mlp_infer(const float* params, __bf16* wb, const float* x, int64_t n, float* out, double* score, hipStream_t st)
{
    hipLaunchKernelGGL(to_bf16_kernel, dim3((kMlpParams + 255) / 256), dim3(256), 0, st, params, wb, kMlpParams);
    if (n > 0)
        hipLaunchKernelGGL(mlp_fused_kernel, dim3((unsigned)((n + kFR - 1) / kFR)), dim3(256), 0, st, params,
                           (const __bf16*)wb, x, n, out, score);
}

// Backward from dout (n x 3) to the flat gradient (same layout as params).
void mlp_backward(const float* params, const float* x, int n, MlpActs& s, const float* dout, float* grad,
                  hipStream_t st)
{
    MlpView w = mlp_view(const_cast<float*>(params));
    MlpView gw = mlp_view(grad);
    // layer 4
    launch_gemm(gemm(dout, kOut, true, s.h3, kH, false, gw.W4, kH, kOut, kH, n), s.part, st);
    launch_colsum(dout, n, kOut, kOut, gw.b4, s.part, st);
    GemmArgs g = gemm(dout, kOut, false, w.W4, kH, false, s.d3, kH, n, kH, kOut);
    g.epi = kGeluGrad;
    g.P = s.a3;
    launch_gemm(g, s.part, st);
    // layer 3
    launch_gemm(gemm(s.d3, kH, true, s.h2, kH, false, gw.W3, kH, kH, kH, n), s.part, st);
    launch_colsum(s.d3, n, kH, kH, gw.b3, s.part, st);
    g = gemm(s.d3, kH, false, w.W3, kH, false, s.d2, kH, n, kH, kH);
    g.epi = kGeluGrad;
    g.P = s.a2;
    launch_gemm(g, s.part, st);
    // layer 2
    launch_gemm(gemm(s.d2, kH, true, s.h1, kH, false, gw.W2, kH, kH, kH, n), s.part, st);
    launch_colsum(s.d2, n, kH, kH, gw.b2, s.part, st);
    g = gemm(s.d2, kH, false, w.W2, kH, false, s.d1, kH, n, kH, kH);
    g.epi = kGeluGrad;
    g.P = s.a1;
    launch_gemm(g, s.part, st);
    // layer 1
    launch_gemm(gemm(s.d1, kH, true, x, kIn, false, gw.W1, kIn, kH, kIn, n), s.part, st);
    launch_colsum(s.d1, n, kH, kH, gw.b1, s.part, st);
}

}  // namespace abcsmc
