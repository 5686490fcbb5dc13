// mlp.h -- surrogate network: sizes, the training step's buffers and the
// screening-stage kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace abcsmc {

constexpr int kIn = 8, kH = 256, kOut = 3;
constexpr int kMlpParams = kH * kIn + kH + kH * kH + kH + kH * kH + kH + kOut * kH + kOut;  // 134659

// ----------------------------------------------------------- training step
// One minibatch step in three kernels (train.hip).  Buffers for up to kpad
// rows (a multiple of 64); all device memory:
//   wb  bfloat16 copy of the parameters (same flat layout; biases unused)
//   wt  bfloat16 transposed weights for the backward products: W2^T [256][256]
//       at kWt2, W3^T at kWt3, W4^T [256][8] (columns 3..7 zero) at kWt4
//   ht  layer inputs, feature-major bf16: h0 [8][kpad], h1, h2, h3 [256][kpad]
//   gt  layer gradients, feature-major bf16: g1, g2, g3 [256][kpad], g4 [3][kpad]
//   dbp gradient sums per row block of the pass kernel (kPartSlots slots:
//       the 771 biases, W1, W4), at part_index(slot, block, kpad / 32); a
//       row block is 32 rows, or 64 for minibatches of 16384 rows or more
//       (then only the first half of each group's blocks is written)
//   wpart W2 / W3 gradient sums per row slice, kWpartStride floats per slice
constexpr int kWt2 = 0, kWt3 = kH * kH, kWt4 = 2 * kH * kH, kWtElems = 2 * kH * kH + kH * 8;
constexpr int kBiasGrads = 3 * kH + kOut;
// per-block partial sums: the biases, then W1 (i-major: slot i * 256 + o for
// W1[o][i]) and W4 (flat: c * 256 + k), stored in groups of 16 slots, one
// 64-byte line per (group, block): slot s of block b at
// ((s / 16) * nblk + b) * 16 + s % 16, nblk = kpad / 32 (room for 32-row blocks)
constexpr int kPartSlots = kBiasGrads + kH * kIn + kOut * kH;
constexpr int kPartGroups = (kPartSlots + 15) / 16;
__host__ __device__ constexpr int64_t part_index(int slot, int64_t blk, int64_t nblk)
{
    return ((int64_t)(slot >> 4) * nblk + blk) * 16 + (slot & 15);
}
constexpr int kTrainSlices = 32;
constexpr int kWpartStride = (kMlpParams + 63) / 64 * 64;  // floats per slice of wpart (16-byte aligned slices)

struct TrainArgs {
    const float* x;     // n x 8 inputs
    const float* y;     // n x 3 targets
    int32_t n;          // rows of this minibatch (<= kpad)
    int64_t kpad;       // rows the ht / gt buffers hold
    float* params;
    float* grad;        // gradient out (may be null)
    float* am;
    float* av;
    __bf16* wb;
    __bf16* wt;
    __bf16* ht;
    __bf16* gt;
    float* dbp;
    float* wpart;
    float* se;          // per-row squared error sum over the 3 outputs
};

// part[kSeParts] = sum of se[0..n) in double (fixed order); part holds
// kSeParts + 1 doubles of device memory.
constexpr int kSeParts = 256;
void launch_se_sum(const float* se, int64_t n, double* part, hipStream_t s);
// Row slices of the weight-gradient products for a minibatch of `rows`.
int train_slices(int64_t rows);
// Refresh wb and wt from params (after params changed outside a step).
void launch_train_copies(const TrainArgs& a, hipStream_t s);
// Loss gradient of the minibatch (to a.grad if set); with lr > 0 also the
// Adam step number `step` and the bfloat16 copies of the updated weights.
void launch_train_step(const TrainArgs& a, float lr, int step, hipStream_t s);

// Forward only, one fused kernel (activations in LDS): wb receives the bf16
// copy of the parameters (kMlpParams); out n x 3 and/or score n (predicted
// squared distance sum_c expm1(y_c)^2), either may be null.
void mlp_infer(const float* params, __bf16* wb, const float* x, int64_t n, float* out, double* score, hipStream_t st);

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
