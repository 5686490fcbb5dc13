// mlp.h -- surrogate network: sizes, GEMM arguments, activation buffers and
// the screening-stage kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace abcsmc {

constexpr int kIn = 8, kH = 256, kOut = 3;
constexpr int kMlpParams = kH * kIn + kH + kH * kH + kH + kH * kH + kH + kOut * kH + kOut;  // 134659

enum : int32_t { kStore = 0, kGelu = 1, kGeluGrad = 2 };

struct GemmArgs {
    const float* A;
    const float* B;
    float* C;
    float* P;            // pre-activations (written by kGelu if not null, read by kGeluGrad)
    const float* bias;   // length N or null
    int32_t M, N, K, lda, ldb, ldc;
    int32_t transA, transB;
    int32_t accumulate;  // C += result
    int32_t epi;
};

struct MlpView {
    float *W1, *b1, *W2, *b2, *W3, *b3, *W4, *b4;
};

// Split-K slices of the weight-gradient products (and the bias-gradient
// partial sums): at most kSplitMax slices of up to 256 x 256.
constexpr int kSplitMax = 32;
constexpr int64_t kSplitFloats = (int64_t)kSplitMax * kH * kH;

// Activation scratch for up to `rows` samples, plus kSplitFloats of `part`.
struct MlpActs {
    float *a1, *a2, *a3, *h1, *h2, *h3, *out, *d1, *d2, *d3, *part;
};

MlpView mlp_view(float* params);
// part: split-K scratch (kSplitFloats) or null (no split).
void launch_gemm(const GemmArgs& g, float* part, hipStream_t s);
void launch_colsum(const float* X, int M, int N, int ld, float* out, float* part, hipStream_t s);
void launch_mse_grad(const float* out, const float* y, int n, float* dout, float* se, hipStream_t s);
void launch_adam(float* w, const float* g, float* m, float* v, int n, float lr, int step, hipStream_t s);
void mlp_forward(const float* params, const float* x, int n, MlpActs& s, hipStream_t st);
// Forward only, one fused kernel (activations in LDS): wb receives the bf16
// copy of the parameters (kMlpParams); out n x 3 and/or score n (predicted
// squared distance sum_c expm1(y_c)^2), either may be null.
void mlp_infer(const float* params, __bf16* wb, const float* x, int64_t n, float* out, double* score, hipStream_t st);
void mlp_backward(const float* params, const float* x, int n, MlpActs& s, const float* dout, float* grad,
                  hipStream_t st);

// ----------------------------------------------------------- screened stage

// Device counters of the screen over whole pool batches.
struct ScreenCounters {
    unsigned long long kept_screen;  // kept with score <= tau
    unsigned long long kept_audit;   // kept only through the audit
    unsigned long long acc_screen;   // accepted among kept_screen
    unsigned long long acc_audit;    // accepted among kept_audit
};

struct PerturbArgs {
    Model m;
    uint32_t round;
    uint32_t base, count;     // pool indices [base, base + count)
    int32_t max_attempts;
    const double* u_prev;
    const uint64_t* cdf;
    int32_t n_prev;
    double beta_a;
    int32_t beta_b;
    int32_t step_is_variance;
    double beta_b_real;       // > 0: real Beta shape b
    double* pu;               // count x 8 proposals
    double* psigma;
    int32_t* pparent;
    int32_t* patt;            // attempts; -max_attempts for a void proposal
    float* x;                 // count x 8 network inputs 2u - 1 (void proposals: 0)
    StageCounters* ctr;       // attempts, invalid
};

struct KeepArgs {
    uint32_t base, count;
    uint32_t round;
    uint64_t seed;
    const int32_t* patt;
    const double* score;      // predicted squared distance
    const double* tau;        // device scalar: keep score <= tau
    double rho;               // audit probability
    unsigned long long* wave_mask;  // ceil(count/64) ballots of kept proposals
    unsigned char* audit;     // 1 if kept only by the audit
    ScreenCounters* sc;
};

// Exact simulation of kept proposals kept[first .. first + n).  With
// tune_x != null the launch runs without early exit and also writes the
// network's training rows (x = 2u - 1, y = log1p of the per-series distances).
struct SimKeptArgs {
    Model m;
    const double* obs;
    uint32_t round;
    uint32_t base;
    uint32_t first, n;        // first is a multiple of 64
    const uint32_t* kept;     // pool positions of kept proposals, in index order
    const double* pu;
    const unsigned char* paudit;
    double eps;
    double exit_thr;
    double* kd;               // distances, indexed like kept
    unsigned long long* wave_mask;  // acceptance ballots, indexed like kept / 64
    float* tune_x;            // n x 8 or null
    float* tune_y;            // n x 3
    StageCounters* ctr;
    ScreenCounters* sc;
};

// Training data: stage-0 proposals j in [0, n) (the same prior streams as
// stage 0), simulated; x = 2u - 1, y = log1p of the per-series distances.
struct TrainDataArgs {
    Model m;
    const double* obs;
    int64_t n;
    float* x;                 // n x 8
    float* y;                 // n x 3
};

// Positions of the set ballot bits of `count` items in index order:
// wave_off = exclusive prefix of the per-wave popcounts, *total = their sum,
// list (if not null) = the positions.
struct MaskArgs {
    uint32_t count;
    const unsigned long long* wave_mask;
    uint32_t* wave_off;
    unsigned long long* total;
    uint32_t* list;
};

// Acceptances of one batch into population slots base_rank + rank (the
// first N acceptances of the stage in index order).
struct ScreenScatterArgs {
    uint32_t base;            // first pool index of the batch
    uint32_t nkept;
    int32_t N;
    unsigned long long base_rank;
    const uint32_t* kept;
    const unsigned long long* wave_mask;  // acceptance ballots over the kept list
    const uint32_t* wave_off;
    const double* pu;
    const double* kd;
    const double* psigma;
    const int32_t* pparent;
    const int32_t* patt;
    const unsigned char* paudit;
    Population pop;
    unsigned char* pop_audit;
    StageCounters* ctr;
};

void launch_mask_list(const MaskArgs& a, hipStream_t s);
void launch_screen_scatter(const ScreenScatterArgs& a, hipStream_t s);
void launch_mlp_init(float* p, uint64_t seed, hipStream_t s);
void launch_audit_weight(double* logw, const unsigned char* audit, int32_t N, double add, hipStream_t s);
void launch_perturb_only(const PerturbArgs& a, hipStream_t s);
void launch_keep(const KeepArgs& a, hipStream_t s);
void launch_sim_kept(const SimKeptArgs& a, hipStream_t s);
void launch_train_data(const TrainDataArgs& a, hipStream_t s);
void launch_fill_u8(unsigned char* p, uint8_t v, int64_t n, hipStream_t s);

}  // namespace abcsmc
