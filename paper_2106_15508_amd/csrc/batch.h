// batch.h -- device descriptors of the batched mode: many independent
// ABC-SMC runs (own population, horizon, particle count, seed and
// observations) advanced one stage at a time by one fixed kernel sequence that
// reads everything it needs from device memory, so a captured graph replays
// every stage.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace abcsmc {

constexpr int kChunkP = kBlock;  // proposals per work item of the persistent kernel
constexpr int kMaxWChunks = 32;  // column chunks per run in the weight kernel

// Read-only description of one run.
struct BRun {
    Model m;
    const double* obs;
    int32_t N;
    int32_t cap_chunks;        // staging capacity in work items
    int32_t step_schedule;
    int32_t beta_b_fixed;
    int32_t step_is_variance;
    int32_t max_attempts;
    int32_t early_exit;
    int32_t wchunks;           // column chunks of the weight kernel
    double beta_a_fixed;
    double surv_ratio;
    double* u[2];
    double* d[2];
    double* sigma[2];
    double* logw[2];
    double* W[2];
    int32_t* parent[2];
    uint32_t* index[2];
    int32_t* att[2];
    uint64_t* q;
    uint64_t* cdf;
    double* cols;
    double* wpart;             // wchunks x N
    double* st_u;
    double* st_d;
    double* st_sigma;
    int32_t* st_parent;
    int32_t* st_att;
    unsigned long long* wave_mask;
    uint32_t* wave_off;
    unsigned long long* red_u; // 3 x res_nblk
    double* red_d;             // 1 x res_nblk
    int32_t res_blk0;          // first block of this run in the segmented resample grid
    int32_t res_nblk;
    int32_t off;               // first slot of this run in the batch-wide sort arrays (sum of earlier N)
    int32_t rb0;               // first 128-row block of this run in the finalize / window tables
};

// Mutable state of one run (device).
struct BState {
    double eps;        // tolerance of the current stage
    double eps1;       // tolerance of stage 1
    double eps_next;   // eq. 8 result of the last completed stage
    double beta_a;
    double ess;
    double rate;       // acceptance rate of the last completed stage
    int32_t beta_b;
    int32_t failed;    // 1 once a stage ran out of proposals (run frozen)
    int32_t cur;       // population buffer of the last completed stage
    int32_t nxt;       // buffer the current stage writes
    int32_t dstar;     // sort coordinate of the weight window (largest column variance)
    int32_t pad_;
    unsigned long long issued, completed, done_acc, accepted, proposals, invalid, attempts, days,
        survivors, fallback, limit, stages_done, terms, window_terms;
};

struct BGlobal {
    int32_t stage;       // stage the next replay runs
    int32_t n_runs;
    double margin;       // over-issue factor of the chunk limiter
};

struct BatchArgs {
    const BRun* runs;
    BState* st;
    BGlobal* g;
    const int32_t* order;      // run visiting order of the persistent kernel
    const int2* res_tab;       // segmented resample grid: (run, local block)
    const int4* w_tab;         // weight grid: (run, row block, chunk, -)
    const int2* fin_tab;       // weight finalize grid: (run, row block)
    int32_t n_runs;
    int32_t max_cap_chunks;
    int32_t n_res_blocks, n_w_blocks, n_fin_blocks;
    int32_t propose_blocks;
    double ex[7];              // table-exp constants (as WeightArgs::ex)
    // weight window (batch-wide arrays; run r owns slots [off_r, off_r + N_r))
    unsigned long long* colkeys;  // npad: (run, column key, column) sorted
    unsigned long long* rowkeys;  // npad: (run, sigma half-octave, row key, row) sorted
    double* scols;             // n_total x 9 sorted columns (u_k, q_k)
    double* skey;              // n_total sorted sort-coordinate values
    double* rwin;              // n_total per-row window half-widths (slot off_r + j)
    int2* win;                 // per 128-row block: column window [x, y) within the run
    const double* wtab;        // kWeightTab entries 2^(i/1024) of the table exponential
    size_t npad;               // power-of-two sort length >= n_total
    int32_t n_total;           // sum of N_r
    int32_t n_key_blocks;      // ceil(npad / 256)
};

void batch_launch_stage(const BatchArgs& a, bool stage0, hipStream_t s);

}  // namespace abcsmc
