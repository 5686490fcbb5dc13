// mlp.hip -- the learned surrogate: an MLP 8 -> 256 -> 256 -> 256 -> 3 with
// tanh-GELU activations, trained on the GPU on simulator outputs, used to
// screen proposals by predicted distance.  Matrix products run on the CDNA4
// matrix cores: v_mfma_f32_16x16x32_bf16 with operands rounded to bfloat16
// (round to nearest even) as they are staged into LDS and FP32 accumulation;
// master weights, activations, gradients and Adam state are FP32.
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "mlp.h"

namespace abcsmc {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kTM = 64, kTN = 64, kTK = 32;  // workgroup tile (M, N) and K step

__device__ __forceinline__ __bf16 to_bf16(float f) { return (__bf16)f; }  // round to nearest even

// GELU, tanh form: 0.5 x (1 + tanh(c (x + 0.044715 x^3))), c = sqrt(2/pi)
__device__ __forceinline__ float gelu_f(float x)
{
    const float c = 0.7978845608028654f;
    const float t = tanhf(c * (x + 0.044715f * x * x * x));
    return 0.5f * x * (1.0f + t);
}
__device__ __forceinline__ float gelu_grad_f(float x)
{
    const float c = 0.7978845608028654f;
    const float x2 = x * x;
    const float t = tanhf(c * (x + 0.044715f * x2 * x));
    return 0.5f * (1.0f + t) + 0.5f * x * (1.0f - t * t) * c * (1.0f + 3.0f * 0.044715f * x2);
}

// C[M x N] = epi( op(A)[M x K] op(B)[K x N] ), row-major FP32 storage:
//   op(A)(m,k) = transA ? A[k*lda + m] : A[m*lda + k]
//   op(B)(k,n) = transB ? B[n*ldb + k] : B[k*ldb + n]
// epilogue (GemmArgs::epi): v = acc (+ C if accumulate) (+ bias[n]);
//   kStore: C = v; kGelu: P = v, C = gelu(v); kGeluGrad: C = v * gelu'(P).
// Workgroup: 256 threads = 4 waves, tile 64 x 64; wave w owns the 32 x 32
// quadrant (w/2, w%2) as 2 x 2 MFMA blocks of 16 x 16.  LDS keeps A as
// [64][32] and B transposed as [64][32] (both K-contiguous) so each lane's
// operand is one 16-byte read.  Out-of-range rows/columns/k are zero-filled.
__global__ __launch_bounds__(256) void gemm_bf16_kernel(GemmArgs g)
{
    __shared__ __attribute__((aligned(16))) __bf16 As[kTM][kTK];
    __shared__ __attribute__((aligned(16))) __bf16 Bs[kTN][kTK];
    const int t = threadIdx.x;
    const int wave = t / 64, lane = t % 64;
    const int m0 = blockIdx.y * kTM, n0 = blockIdx.x * kTN;
    const int wm = (wave / 2) * 32, wn = (wave % 2) * 32;
    f32x4 acc[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < g.K; k0 += kTK) {
        // stage: each thread 8 elements of A and 8 of B
        for (int e = 0; e < 8; ++e) {
            const int idx = t * 8 + e;          // 0..2047 over a 64 x 32 tile
            const int r = idx / kTK, kk = idx % kTK;
            const int m = m0 + r, n = n0 + r, k = k0 + kk;
            float av = 0.f, bv = 0.f;
            if (m < g.M && k < g.K) av = g.transA ? g.A[(size_t)k * g.lda + m] : g.A[(size_t)m * g.lda + k];
            if (n < g.N && k < g.K) bv = g.transB ? g.B[(size_t)n * g.ldb + k] : g.B[(size_t)k * g.ldb + n];
            As[r][kk] = to_bf16(av);
            Bs[r][kk] = to_bf16(bv);
        }
        __syncthreads();
        bf16x8 af[2], bfr[2];
        for (int a = 0; a < 2; ++a) af[a] = *reinterpret_cast<const bf16x8*>(&As[wm + 16 * a + lane % 16][8 * (lane / 16)]);
        for (int b = 0; b < 2; ++b) bfr[b] = *reinterpret_cast<const bf16x8*>(&Bs[wn + 16 * b + lane % 16][8 * (lane / 16)]);
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[a], bfr[b], acc[a][b], 0, 0, 0);
        __syncthreads();
    }
    // lane holds D[4*(lane/16)+e][lane%16] of each 16 x 16 block
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int e = 0; e < 4; ++e) {
                const int m = m0 + wm + 16 * a + 4 * (lane / 16) + e;
                const int n = n0 + wn + 16 * b + lane % 16;
                if (m >= g.M || n >= g.N) continue;
                const size_t o = (size_t)m * g.ldc + n;
                float v = acc[a][b][e];
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

// out[n] = sum over m of X[m*ld + n] (bias gradients), fixed order per column.
__global__ __launch_bounds__(256) void colsum_kernel(const float* X, int M, int N, int ld, float* out)
{
    const int n = blockIdx.x * 256 + threadIdx.x;
    if (n >= N) return;
    float s = 0.f;
    for (int m = 0; m < M; ++m) s += X[(size_t)m * ld + n];
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

// score = sum_c expm1(yhat_c)^2: the predicted squared distance (targets are log1p of the
// three per-series distances).
__global__ __launch_bounds__(256) void score_kernel(const float* out, int n, double* score)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int c = 0; c < 3; ++c) {
        const double e = expm1((double)out[i * 3 + c]);
        s += e * e;
    }
    score[i] = s <= 1.0e300 ? s : __builtin_inf();  // NaN and overflow rank last
}

}  // namespace

void launch_gemm(const GemmArgs& g, hipStream_t s)
{
    const dim3 grid((g.N + kTN - 1) / kTN, (g.M + kTM - 1) / kTM);
    hipLaunchKernelGGL(gemm_bf16_kernel, grid, dim3(256), 0, s, g);
}

void launch_colsum(const float* X, int M, int N, int ld, float* out, hipStream_t s)
{
    hipLaunchKernelGGL(colsum_kernel, dim3((N + 255) / 256), dim3(256), 0, s, X, M, N, ld, out);
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

void launch_score(const float* out, int n, double* score, hipStream_t s)
{
    hipLaunchKernelGGL(score_kernel, dim3((n + 255) / 256), dim3(256), 0, s, out, n, score);
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
    launch_gemm(g, st);
    g = gemm(s.h1, kH, false, w.W2, kH, true, s.h2, kH, n, kH, kH);
    g.bias = w.b2;
    g.epi = kGelu;
    g.P = s.a2;
    launch_gemm(g, st);
    g = gemm(s.h2, kH, false, w.W3, kH, true, s.h3, kH, n, kH, kH);
    g.bias = w.b3;
    g.epi = kGelu;
    g.P = s.a3;
    launch_gemm(g, st);
    g = gemm(s.h3, kH, false, w.W4, kH, true, s.out, kOut, n, kOut, kH);
    g.bias = w.b4;
    launch_gemm(g, st);
}

void mlp_infer(const float* params, const float* x, int n, float* hA, float* hB, float* out, hipStream_t st)
{
    MlpView w = mlp_view(const_cast<float*>(params));
    GemmArgs g = gemm(x, kIn, false, w.W1, kIn, true, hA, kH, n, kH, kIn);
    g.bias = w.b1;
    g.epi = kGelu;
    launch_gemm(g, st);
    g = gemm(hA, kH, false, w.W2, kH, true, hB, kH, n, kH, kH);
    g.bias = w.b2;
    g.epi = kGelu;
    launch_gemm(g, st);
    g = gemm(hB, kH, false, w.W3, kH, true, hA, kH, n, kH, kH);
    g.bias = w.b3;
    g.epi = kGelu;
    launch_gemm(g, st);
    g = gemm(hA, kH, false, w.W4, kH, true, out, kOut, n, kOut, kH);
    g.bias = w.b4;
    launch_gemm(g, st);
}

// Backward from dout (n x 3) to the flat gradient (same layout as params).
void mlp_backward(const float* params, const float* x, int n, MlpActs& s, const float* dout, float* grad,
                  hipStream_t st)
{
    MlpView w = mlp_view(const_cast<float*>(params));
    MlpView gw = mlp_view(grad);
    // layer 4
    launch_gemm(gemm(dout, kOut, true, s.h3, kH, false, gw.W4, kH, kOut, kH, n), st);
    launch_colsum(dout, n, kOut, kOut, gw.b4, st);
    GemmArgs g = gemm(dout, kOut, false, w.W4, kH, false, s.d3, kH, n, kH, kOut);
    g.epi = kGeluGrad;
    g.P = s.a3;
    launch_gemm(g, st);
    // layer 3
    launch_gemm(gemm(s.d3, kH, true, s.h2, kH, false, gw.W3, kH, kH, kH, n), st);
    launch_colsum(s.d3, n, kH, kH, gw.b3, st);
    g = gemm(s.d3, kH, false, w.W3, kH, false, s.d2, kH, n, kH, kH);
    g.epi = kGeluGrad;
    g.P = s.a2;
    launch_gemm(g, st);
    // layer 2
    launch_gemm(gemm(s.d2, kH, true, s.h1, kH, false, gw.W2, kH, kH, kH, n), st);
    launch_colsum(s.d2, n, kH, kH, gw.b2, st);
    g = gemm(s.d2, kH, false, w.W2, kH, false, s.d1, kH, n, kH, kH);
    g.epi = kGeluGrad;
    g.P = s.a1;
    launch_gemm(g, st);
    // layer 1
    launch_gemm(gemm(s.d1, kH, true, x, kIn, false, gw.W1, kIn, kH, kIn, n), st);
    launch_colsum(s.d1, n, kH, kH, gw.b1, st);
}

}  // namespace abcsmc
