// kernels.h -- kernel argument blocks and launch wrappers of the HIP path.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace abcsmc {

constexpr int kNP = 8;        // parameters per particle (eq. 1)
constexpr int kBlock = 256;   // threads per workgroup of the per-lane kernels
constexpr int kWave = 64;
constexpr int kWeightRows = 128;  // sorted rows per workgroup (and per window) of the weight kernel

// Model constants shared by every simulation (§II-B).
struct Model {
    double lo[kNP];     // prior box lower corner
    double width[kNP];  // hi - lo
    double P;           // population (exact integer)
    double invP;        // 1 / P
    double A0, R0, D0;  // day-0 observed state
    int32_t T;          // days
    int32_t sampler;    // 0 binomial, 1 floor-normal
    uint64_t seed;
};

// Device counters of one stage (8-byte words).
struct StageCounters {
    unsigned long long accepted;   // acceptances over the batches run so far
    unsigned long long proposals;  // index of the N-th acceptance + 1 (0 until reached)
    unsigned long long invalid;    // void proposals over the batches run so far
    unsigned long long attempts;   // perturbation attempts over the batches run so far
    unsigned long long base_rank;  // acceptances before the current batch
    unsigned long long survivors;  // previous particles with q > 0
    unsigned long long fallback;   // 1 if the prior set used d <= eps (no d < eps)
    unsigned long long days;       // proposal-days simulated over the batches run so far
    unsigned long long terms;      // importance-weight terms evaluated (inside the windows)
    unsigned long long window_terms;  // sum over rows of the row's own window (terms the rows need)
};

// Population of one stage, array-of-structures for the per-particle gathers.
struct Population {
    double* u;        // N x 8
    double* d;        // N
    double* sigma;    // N
    int32_t* parent;  // N
    uint32_t* index;  // N
    int32_t* att;     // N
    double* logw;     // N
    double* W;        // N
};

struct ProposeArgs {
    Model m;
    const double* obs;  // (T+1) x 3, exact integers
    uint32_t round;
    uint32_t base;      // first proposal index of the batch
    uint32_t count;     // proposals in the batch
    int32_t max_attempts;
    double eps;         // accept iff d <= eps
    double exit_thr;    // early exit once the partial sum of squares exceeds this (+inf: off)
    // perturbation (stage >= 1)
    const double* u_prev;    // n_prev x 8
    const uint64_t* cdf;     // n_prev inclusive prefix sums of q
    int32_t n_prev;
    double beta_a;
    int32_t beta_b;
    int32_t step_is_variance;
    double s_fixed;          // >= 0: every proposal uses step size s_fixed (MCMC variant), no Beta draw
    double beta_b_real;      // > 0: real Beta shape b, general sampler (alternative parameterisations)
    // staging, indexed by p = j - base
    double* st_u;            // count x 8
    double* st_d;
    double* st_sigma;
    int32_t* st_parent;
    int32_t* st_att;
    unsigned long long* wave_mask;  // ceil(count/64) acceptance ballots
    StageCounters* ctr;
};

struct CompactArgs {
    uint32_t base;
    uint32_t count;
    int32_t N;
    const unsigned long long* wave_mask;
    uint32_t* wave_off;   // exclusive prefix of popcounts
    const double* st_u;
    const double* st_d;
    const double* st_sigma;
    const int32_t* st_parent;
    const int32_t* st_att;
    Population pop;
    StageCounters* ctr;
};

// Per-block partial results of the multi-block reductions and scans.
constexpr int kRedMax = 4096;  // max blocks of a reduction (N <= 2^22 at 1024 per block)
struct Scratch {
    unsigned long long* u0;  // kRedMax
    unsigned long long* u1;  // kRedMax
    unsigned long long* u2;  // kRedMax
    double* d0;              // kRedMax
    double* d1;              // kRedMax
    unsigned int* hist;      // 2 x 2048 radix-select bins
    unsigned long long* sel; // radix-select state: prefix[2], mask[2], rank[2], r0, r1
};

struct ResampleArgs {
    const double* d_prev;   // N
    const double* u_prev;   // N x 8
    int32_t N;
    double eps;
    uint64_t* q;            // N
    uint64_t* cdf;          // N
    double* cols;           // M x 9: u_k[8], q_k  (q_k > 0 only, index order)
    Scratch sc;
    StageCounters* ctr;
};

// Entries of the weight kernels' exponential table (2^(i/1024)).
constexpr int kWeightTab = 1024;

struct WeightArgs {
    const double* u;        // N x 8 rows
    const double* sigma;    // N
    const double* cols;     // M x 9
    int32_t N;
    int32_t chunks;         // column chunks (second grid dimension)
    const unsigned long long* M;  // device scalar: survivors
    double* partial;        // chunks x N row sums per column chunk
    double* logw;           // N
    // windowed evaluation: columns sorted by one coordinate, rows by
    // (step-size half-octave, same coordinate); each workgroup visits only the
    // columns that can give a nonzero term
    unsigned long long* rowkeys;  // Npad sort keys (row index in the low 32 bits)
    unsigned long long* colkeys;  // Npad sort keys (column index in the low 32 bits)
    double* scols;          // M x 9 columns in sorted order
    double* skey;           // M sorted coordinate values
    double* dimpart;        // per-block partial sums for the coordinate choice (kRedMax x 16)
    int32_t* dstar;         // device scalar: the coordinate
    size_t npad;            // padded sort length (power of two >= N)
    int2* win;              // per row block: sorted column range [first, end) of its window
    int32_t cols_per_chunk; // columns per grid-y chunk of a window
    unsigned long long* terms;  // device counter of evaluated terms
    unsigned long long* window_terms;  // device counter: sum over rows of the row's own window
    // per-row window half-widths from each row's parent term
    const int32_t* parent;  // N parent indices into the previous population
    const double* u_prev;   // previous population, n_prev x 8
    const uint64_t* q_prev; // its resampling weights q_k (0 for non-survivors)
    const uint64_t* cdf;    // its integer CDF (cdf[n_prev - 1] = Q)
    int32_t n_prev;
    double* rwin;           // N half-widths W_j sigma_j
    // table exponential: ln2/1024, its square / 2, its cube / 6, 1024/ln2
    // (kernel arguments so they sit in scalar registers)
    double ex[7];
    const double* tab;      // kWeightTab entries 2^(i/1024), written once per context
};

// Fill WeightArgs::ex.
void weight_exp_constants(double ex[7]);
// Write the kWeightTab table entries 2^(i/1024) to tab (device memory).
void launch_weight_table(double* tab, hipStream_t s);
// Test hook: n importance-weight terms, records {u_j[8], sigma_j, u_k[8], q_k}.
void launch_wterm_debug(int64_t n, const double* in, double* out, hipStream_t s);

// Bitonic sort of 64-bit keys (length a power of two >= 2048).
size_t sort_padded_size(size_t n);
void launch_sort_u64(unsigned long long* keys, size_t n_pow2, hipStream_t s);
// both arrays (each n_pow2 keys; keys1 may be null) by the same launches
void launch_sort_u64_pair(unsigned long long* keys0, unsigned long long* keys1, size_t n_pow2, hipStream_t s);

struct NormArgs {
    const double* logw;
    double* W;
    int32_t N;
    Scratch sc;
    double* ess;            // device scalar
};

struct SelectArgs {
    const double* x;        // N non-negative (or +inf) values
    int32_t N;
    double alpha;
    Scratch sc;
    double* out;            // device scalar: type-7 quantile
};

// Column chunks of the weight kernel for N rows: enough workgroups to give
// every SIMD about eight waves, with the partial sums bounded by 2^23 doubles.
int weight_chunks(int64_t N);
// Windowed weight kernel: columns per chunk and chunks per row block.
int weight_cols_per_chunk(int64_t N);
int weight_window_chunks(int64_t N);

struct TrajArgs {
    Model m;
    const double* theta;    // n x 8 (prior units)
    int64_t n;
    uint32_t round;
    uint32_t index0;
    int64_t* traj;          // n x (T+1) x 6
};

void launch_propose(const ProposeArgs& a, bool round0, hipStream_t s);
// Largest first batch of a stage without a measured acceptance rate: one
// round of the proposal kernel's resident waves on the current device (its
// occupancy in workgroups per compute unit x the compute units), so a first
// batch never leaves lanes of a second round to run on a mostly idle chip.
int64_t propose_first_batch_lanes();
void launch_compact(const CompactArgs& a, hipStream_t s);
void launch_resample(const ResampleArgs& a, hipStream_t s);
// The weight pass in three parts, so that the caller can time the sum kernel
// alone: the window pass (coordinate pick, column and row sorts, windows),
// the windowed sums, and the per-row merge of the chunk partial sums.
void launch_weights_window(const WeightArgs& a, hipStream_t s);
void launch_weights_sum(const WeightArgs& a, hipStream_t s);
void launch_weights_finalize(const WeightArgs& a, hipStream_t s);
void launch_normalise(const NormArgs& a, hipStream_t s);
void launch_select(const SelectArgs& a, hipStream_t s);
void launch_uniform_weights(double* W, double* logw, int32_t N, hipStream_t s);
void launch_simulate_traj(const TrajArgs& a, hipStream_t s);
void launch_to_theta(const double* u, const Model& m, double* theta, int64_t n, hipStream_t s);
void launch_debug_eval(int32_t fn, int64_t n, const void* in, void* out, double pa, int32_t pb,
                       hipStream_t s);

}  // namespace abcsmc
