// surrogate_rt.hip -- host side of the learned surrogate screen: device
// state, GPU training (initial fit on prior simulations, fine-tune after each
// screened stage), the screened stage's batch loop, and the test hooks of the
// network.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "abcsmc.h"
#include "ctx.h"
#include "kernels.h"
#include "mlp.h"

using namespace abcsmc;
using namespace abcsmc::rt;

namespace abcsmc {
namespace rt {

constexpr int64_t kInferRows = 65536;  // rows per call of the network hooks
constexpr int64_t kPoolMax = (int64_t)1 << 22;
constexpr int32_t kTrainBatchMax = 65536;

// Network, its gradient and Adam state, and the training step's buffers for
// minibatches of up to kpad rows.
struct Trainer {
    float *params = nullptr, *grad = nullptr, *am = nullptr, *av = nullptr;
    float* se = nullptr;
    __bf16 *wb = nullptr, *wt = nullptr, *ht = nullptr, *gt = nullptr;
    float *dbp = nullptr, *wpart = nullptr;
    double* lpart = nullptr;  // loss sum: kSeParts block sums and the total
    int64_t kpad = 0;
    int64_t step = 0;
};

struct Surrogate {
    abcsmc_surrogate_config cfg{};
    abcsmc_surrogate_info info{};
    char* mem = nullptr;
    Trainer tr;
    float *params0 = nullptr, *am0 = nullptr, *av0 = nullptr;  // state after the initial fit (reset)
    int64_t step0 = 0;
    float *tx = nullptr, *ty = nullptr;
    int64_t n_train = 0;
    double *pu = nullptr, *psigma = nullptr, *score = nullptr, *kd = nullptr;
    int32_t *pparent = nullptr, *patt = nullptr;
    float* px = nullptr;
    __bf16* wb = nullptr;                                    // bf16 copy of the network for scoring
    unsigned char* paudit = nullptr;
    uint32_t* kept = nullptr;
    unsigned long long *mask_pool = nullptr, *mask_kept = nullptr, *totals = nullptr;
    uint32_t *off_pool = nullptr, *off_kept = nullptr;
    float *tune_x = nullptr, *tune_y = nullptr;
    int64_t tune_cap = 0, n_tune = 0;
    unsigned char* pop_audit[2] = {nullptr, nullptr};
    ScreenCounters* sc = nullptr;
    double* tau = nullptr;
    bool active = true;
    hipEvent_t ev[4] = {};
};

namespace {

// Carves typed regions (256-byte aligned) out of one allocation; a first pass
// with base == nullptr only sizes it.
struct Carver {
    char* base;
    size_t off = 0;
    template <typename T>
    T* take(size_t count)
    {
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off = (off + count * sizeof(T) + 255) / 256 * 256;
        return p;
    }
};

void carve_trainer(Carver& c, Trainer& t, int64_t rows, int64_t se_rows)
{
    t.kpad = (rows + 63) / 64 * 64;
    const int64_t blocks = t.kpad / 32;
    t.params = c.take<float>(kMlpParams);
    t.grad = c.take<float>(kMlpParams);
    t.am = c.take<float>(kMlpParams);
    t.av = c.take<float>(kMlpParams);
    t.se = c.take<float>((size_t)se_rows);
    t.wb = c.take<__bf16>(kMlpParams);
    t.wt = c.take<__bf16>(kWtElems);
    t.ht = c.take<__bf16>((size_t)(kIn + 3 * kH) * t.kpad);
    t.gt = c.take<__bf16>((size_t)(3 * kH + kOut) * t.kpad);
    t.dbp = c.take<float>((size_t)blocks * kPartGroups * 16);
    t.wpart = c.take<float>((size_t)kTrainSlices * kWpartStride);
    t.lpart = c.take<double>(kSeParts + 1);
}

TrainArgs train_args(const Trainer& t, const float* x, const float* y, int64_t n, float* se)
{
    TrainArgs a{};
    a.x = x;
    a.y = y;
    a.n = (int32_t)n;
    a.kpad = t.kpad;
    a.params = t.params;
    a.am = t.am;
    a.av = t.av;
    a.wb = t.wb;
    a.wt = t.wt;
    a.ht = t.ht;
    a.gt = t.gt;
    a.dbp = t.dbp;
    a.wpart = t.wpart;
    a.se = se;
    return a;
}

// `epochs` passes of minibatch Adam over (X, Y) (n rows, in order; the last
// minibatch of a pass may be short).  losses[e] (host, may be null) = mean
// squared error per output over pass e, from the predictions before each step.
hipError_t train_epochs(Trainer& t, const float* X, const float* Y, int64_t n, int32_t batch, int32_t epochs,
                        float lr, double* losses, hipStream_t s)
{
    if (epochs > 0 && n > 0) launch_train_copies(train_args(t, X, Y, 0, t.se), s);  // params may have changed
    for (int32_t e = 0; e < epochs; ++e) {
        for (int64_t off = 0; off < n; off += batch) {
            const int64_t b = std::min<int64_t>(batch, n - off);
            launch_train_step(train_args(t, X + off * kIn, Y + off * kOut, b, t.se + off), lr, (int)(++t.step), s);
        }
        hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
        if (losses) {
            double sum = 0.0;
            launch_se_sum(t.se, n, t.lpart, s);
            err = hipMemcpyAsync(&sum, t.lpart + kSeParts, sizeof(double), hipMemcpyDeviceToHost, s);
            if (err == hipSuccess) err = hipStreamSynchronize(s);
            if (err != hipSuccess) return err;
            losses[e] = n ? sum / (3.0 * (double)n) : 0.0;
        }
    }
    return hipGetLastError();
}

int check_scfg(const abcsmc_surrogate_config& c, std::string* err)
{
    if (c.n_train < 1 || c.n_train > ((int64_t)1 << 24)) return fail(err, ABCSMC_EINVAL, "n_train must be in [1, 2^24]");
    if (c.epochs < 0 || c.epochs > 1000) return fail(err, ABCSMC_EINVAL, "epochs must be in [0, 1000]");
    if (c.batch < 1 || c.batch > kTrainBatchMax) return fail(err, ABCSMC_EINVAL, "batch must be in [1, 65536]");
    if (!(c.lr > 0.0 && c.lr < 1.0)) return fail(err, ABCSMC_EINVAL, "lr must be in (0, 1)");
    if (!(c.keep_frac > 0.0 && c.keep_frac <= 1.0)) return fail(err, ABCSMC_EINVAL, "keep_frac must be in (0, 1]");
    if (!(c.audit_rho > 0.0 && c.audit_rho <= 1.0)) return fail(err, ABCSMC_EINVAL, "audit_rho must be in (0, 1]");
    if (c.pool < 1024 || c.pool > kPoolMax) return fail(err, ABCSMC_EINVAL, "pool must be in [1024, 2^22]");
    if (c.tune_rows < 0 || c.tune_rows > c.pool) return fail(err, ABCSMC_EINVAL, "tune_rows must be in [0, pool]");
    if (c.tune_epochs < 0 || c.tune_epochs > 1000) return fail(err, ABCSMC_EINVAL, "tune_epochs must be in [0, 1000]");
    if (!(c.fn_max >= 0.0)) return fail(err, ABCSMC_EINVAL, "fn_max must be >= 0");
    return ABCSMC_OK;
}

abcsmc_surrogate_config with_defaults(const abcsmc_surrogate_config* in)
{
    abcsmc_surrogate_config c = *in;
    if (c.n_train == 0) c.n_train = (int64_t)1 << 20;
    if (c.epochs == 0) c.epochs = 4;
    else if (c.epochs < 0) c.epochs = 0;
    if (c.batch == 0) c.batch = 8192;
    if (c.lr == 0.0) c.lr = 1e-3;
    if (c.keep_frac == 0.0) c.keep_frac = 0.1;
    if (c.audit_rho == 0.0) c.audit_rho = 0.01;
    if (c.pool == 0) c.pool = kPoolMax;
    if (c.tune_rows == 0) c.tune_rows = std::min<int64_t>(65536, c.pool);
    else if (c.tune_rows < 0) c.tune_rows = 0;
    if (c.tune_epochs == 0) c.tune_epochs = 2;
    else if (c.tune_epochs < 0) c.tune_epochs = 0;
    if (c.fn_max == 0.0) c.fn_max = 0.05;
    return c;
}

size_t carve_surrogate(Surrogate& S, char* base, int64_t N)
{
    Carver c{base};
    const int64_t P = S.cfg.pool;
    const int64_t se_rows = std::max<int64_t>(S.cfg.n_train, S.tune_cap);
    carve_trainer(c, S.tr, S.cfg.batch, se_rows);
    S.params0 = c.take<float>(kMlpParams);
    S.am0 = c.take<float>(kMlpParams);
    S.av0 = c.take<float>(kMlpParams);
    S.tx = c.take<float>((size_t)S.cfg.n_train * kIn);
    S.ty = c.take<float>((size_t)S.cfg.n_train * kOut);
    S.pu = c.take<double>((size_t)P * kNP);
    S.psigma = c.take<double>((size_t)P);
    S.score = c.take<double>((size_t)P);
    S.kd = c.take<double>((size_t)P);
    S.pparent = c.take<int32_t>((size_t)P);
    S.patt = c.take<int32_t>((size_t)P);
    S.px = c.take<float>((size_t)P * kIn);
    S.wb = c.take<__bf16>((size_t)kMlpParams);
    S.paudit = c.take<unsigned char>((size_t)P);
    S.kept = c.take<uint32_t>((size_t)P);
    S.mask_pool = c.take<unsigned long long>((size_t)P / kWave + 4);
    S.mask_kept = c.take<unsigned long long>((size_t)P / kWave + 4);
    S.off_pool = c.take<uint32_t>((size_t)P / kWave + 4);
    S.off_kept = c.take<uint32_t>((size_t)P / kWave + 4);
    S.totals = c.take<unsigned long long>(4);
    S.tune_x = c.take<float>((size_t)std::max<int64_t>(S.tune_cap, 1) * kIn);
    S.tune_y = c.take<float>((size_t)std::max<int64_t>(S.tune_cap, 1) * kOut);
    S.pop_audit[0] = c.take<unsigned char>((size_t)N);
    S.pop_audit[1] = c.take<unsigned char>((size_t)N);
    S.sc = c.take<ScreenCounters>(1);
    S.tau = c.take<double>(1);
    return c.off;
}

}  // namespace

void surrogate_free(Surrogate* S)
{
    if (!S) return;
    for (auto& e : S->ev)
        if (e) (void)hipEventDestroy(e);
    if (S->mem) (void)hipFree(S->mem);
    delete S;
}

// Zero the audit flags of the population a stage writes (plain stages).
int surrogate_stage_begin(abcsmc_ctx* x, int nxt)
{
    Surrogate& S = *x->sur;
    launch_fill_u8(S.pop_audit[nxt], 0, x->N, x->stream);
    HIPCHK(x, hipGetLastError());
    return ABCSMC_OK;
}

bool surrogate_screens(const abcsmc_ctx* x, int32_t round) { return x->sur && x->sur->active && round >= 1; }

// The screened stage's batches: on return the population slots of dst hold
// the first N acceptances in index order, hc the stage counters.
int surrogate_batches(abcsmc_ctx* x, const ProposeArgs& pa, const DevPop& dst, int nxt, StageCounters& hc,
                      int64_t& base, int64_t& batches, double& ms_k)
{
    Surrogate& S = *x->sur;
    hipStream_t s = x->stream;
    const int32_t N = (int32_t)x->N;
    const abcsmc_config& c = x->cfg;
    HIPCHK(x, hipMemsetAsync(S.sc, 0, sizeof(ScreenCounters), s));
    PerturbArgs qa{};
    qa.m = pa.m;
    qa.round = pa.round;
    qa.max_attempts = pa.max_attempts;
    qa.u_prev = pa.u_prev;
    qa.cdf = pa.cdf;
    qa.n_prev = pa.n_prev;
    qa.beta_a = pa.beta_a;
    qa.beta_b = pa.beta_b;
    qa.step_is_variance = pa.step_is_variance;
    qa.beta_b_real = pa.beta_b_real;
    qa.pu = S.pu;
    qa.psigma = S.psigma;
    qa.pparent = S.pparent;
    qa.patt = S.patt;
    qa.x = S.px;
    qa.ctr = pa.ctr;
    KeepArgs ka{};
    ka.round = pa.round;
    ka.seed = c.seed;
    ka.patt = S.patt;
    ka.score = S.score;
    ka.tau = S.tau;
    ka.rho = S.cfg.audit_rho;
    ka.wave_mask = S.mask_pool;
    ka.audit = S.paudit;
    ka.sc = S.sc;
    SimKeptArgs sa{};
    sa.m = pa.m;
    sa.obs = pa.obs;
    sa.round = pa.round;
    sa.kept = S.kept;
    sa.pu = S.pu;
    sa.paudit = S.paudit;
    sa.eps = pa.eps;
    sa.exit_thr = pa.exit_thr;
    sa.kd = S.kd;
    sa.wave_mask = S.mask_kept;
    sa.ctr = pa.ctr;
    sa.sc = S.sc;
    ScreenScatterArgs ca{};
    ca.N = N;
    ca.kept = S.kept;
    ca.wave_mask = S.mask_kept;
    ca.wave_off = S.off_kept;
    ca.pu = S.pu;
    ca.kd = S.kd;
    ca.psigma = S.psigma;
    ca.pparent = S.pparent;
    ca.patt = S.patt;
    ca.paudit = S.paudit;
    ca.pop = dst.view();
    ca.pop_audit = S.pop_audit[nxt];
    ca.ctr = pa.ctr;

    unsigned long long acc_total = 0;
    double ms_score = 0.0;
    S.n_tune = 0;
    for (;;) {
        const double need = (double)(N - (int64_t)acc_total);
        const double rate = x->last_rate > 1e-4 ? x->last_rate : 1e-4;
        int64_t B = (int64_t)std::ceil(need / rate * 1.1) + 2048;
        B = (B + kBlock - 1) / kBlock * kBlock;
        if (B > S.cfg.pool) B = S.cfg.pool;
        if (base + B > c.max_proposals) B = c.max_proposals - base;
        if (B <= 0) return fail(&x->err, ABCSMC_EBUDGET, "stage exhausted its proposal budget");
        HIPCHK(x, hipEventRecord(S.ev[0], s));
        qa.base = (uint32_t)base;
        qa.count = (uint32_t)B;
        launch_perturb_only(qa, s);
        mlp_infer(S.tr.params, S.wb, S.px, B, nullptr, S.score, s);
        if (batches == 0) {
            // tau: keep_frac percentile of the stage's first batch of scores
            SelectArgs ta{S.score, (int32_t)B, S.cfg.keep_frac, x->scratch(), S.tau};
            launch_select(ta, s);
        }
        ka.base = (uint32_t)base;
        ka.count = (uint32_t)B;
        launch_keep(ka, s);
        MaskArgs ma{(uint32_t)B, S.mask_pool, S.off_pool, S.totals + 0, S.kept};
        launch_mask_list(ma, s);
        HIPCHK(x, hipGetLastError());
        HIPCHK(x, hipEventRecord(S.ev[1], s));
        unsigned long long nk = 0;
        HIPCHK(x, hipMemcpyAsync(&nk, S.totals + 0, sizeof nk, hipMemcpyDeviceToHost, s));
        HIPCHK(x, hipStreamSynchronize(s));
        ms_score += elapsed(S.ev[0], S.ev[1]);

        const int64_t ntune = batches == 0 ? std::min<int64_t>((int64_t)nk, S.tune_cap) : 0;
        sa.base = (uint32_t)base;
        HIPCHK(x, hipEventRecord(x->ev[5], s));
        if (ntune > 0) {
            sa.first = 0;
            sa.n = (uint32_t)ntune;
            sa.tune_x = S.tune_x;
            sa.tune_y = S.tune_y;
            launch_sim_kept(sa, s);
            S.n_tune = ntune;
        }
        sa.first = (uint32_t)ntune;
        sa.n = (uint32_t)((int64_t)nk - ntune);
        sa.tune_x = nullptr;
        sa.tune_y = nullptr;
        launch_sim_kept(sa, s);
        HIPCHK(x, hipEventRecord(x->ev[6], s));
        MaskArgs mb{(uint32_t)nk, S.mask_kept, S.off_kept, S.totals + 1, nullptr};
        launch_mask_list(mb, s);
        ca.base = (uint32_t)base;
        ca.nkept = (uint32_t)nk;
        ca.base_rank = acc_total;
        launch_screen_scatter(ca, s);
        HIPCHK(x, hipGetLastError());
        unsigned long long na = 0;
        HIPCHK(x, hipMemcpyAsync(&na, S.totals + 1, sizeof na, hipMemcpyDeviceToHost, s));
        HIPCHK(x, hipStreamSynchronize(s));
        ms_k += elapsed(x->ev[5], x->ev[6]);
        acc_total += na;
        base += B;
        ++batches;
        if (acc_total >= (unsigned long long)N) break;
        if (base > 0 && acc_total > 0) x->last_rate = (double)acc_total / (double)base;
    }
    HIPCHK(x, hipMemcpyAsync(&hc, pa.ctr, sizeof hc, hipMemcpyDeviceToHost, s));
    HIPCHK(x, hipStreamSynchronize(s));
    hc.accepted = acc_total;
    S.info.ms_score = ms_score;
    return ABCSMC_OK;
}

// Importance-weight factor of the audit (before normalisation).
int surrogate_weights(abcsmc_ctx* x, const DevPop& dst, int nxt)
{
    Surrogate& S = *x->sur;
    launch_audit_weight(dst.logw, S.pop_audit[nxt], (int32_t)x->N, -std::log(S.cfg.audit_rho), x->stream);
    HIPCHK(x, hipGetLastError());
    return ABCSMC_OK;
}

// Statistics of a screened stage, the fallback test, and the fine-tune on the
// stage's fully simulated kept proposals.
int surrogate_stage_end(abcsmc_ctx* x, int32_t round)
{
    Surrogate& S = *x->sur;
    hipStream_t s = x->stream;
    ScreenCounters h{};
    double tau = 0.0;
    HIPCHK(x, hipMemcpyAsync(&h, S.sc, sizeof h, hipMemcpyDeviceToHost, s));
    HIPCHK(x, hipMemcpyAsync(&tau, S.tau, sizeof tau, hipMemcpyDeviceToHost, s));
    HIPCHK(x, hipStreamSynchronize(s));
    abcsmc_surrogate_info& I = S.info;
    I.round = round;
    I.tau = tau;
    I.kept_screen = (int64_t)h.kept_screen;
    I.kept_audit = (int64_t)h.kept_audit;
    I.accepted_screen = (int64_t)h.acc_screen;
    I.accepted_audit = (int64_t)h.acc_audit;
    const double rho = S.cfg.audit_rho;
    const double est = (double)h.acc_screen + (double)h.acc_audit / rho;  // acceptances over the whole pool
    I.fn_mass = est > 0.0 ? ((double)h.acc_audit / rho) / est : 0.0;
    const double pool_valid = (double)h.kept_screen + (double)h.kept_audit / rho;
    const double rate_screen = h.kept_screen ? (double)h.acc_screen / (double)h.kept_screen : 0.0;
    I.enrichment = (est > 0.0 && pool_valid > 0.0) ? rate_screen / (est / pool_valid) : 0.0;
    I.ms_tune = 0.0;
    if (I.fn_mass > S.cfg.fn_max) S.active = false;
    I.active = S.active ? 1 : 0;
    if (S.active && S.n_tune > 0 && S.cfg.tune_epochs > 0) {
        HIPCHK(x, hipEventRecord(S.ev[2], s));
        HIPCHK(x, train_epochs(S.tr, S.tune_x, S.tune_y, S.n_tune, S.cfg.batch, S.cfg.tune_epochs, (float)S.cfg.lr,
                               nullptr, s));
        HIPCHK(x, hipEventRecord(S.ev[3], s));
        HIPCHK(x, hipStreamSynchronize(s));
        I.ms_tune = elapsed(S.ev[2], S.ev[3]);
    }
    I.train_steps = S.tr.step;
    return ABCSMC_OK;
}

// Back to the network right after the initial fit (abcsmc_reset).
int surrogate_reset(abcsmc_ctx* x)
{
    Surrogate& S = *x->sur;
    hipStream_t s = x->stream;
    HIPCHK(x, hipMemcpyAsync(S.tr.params, S.params0, kMlpParams * sizeof(float), hipMemcpyDeviceToDevice, s));
    HIPCHK(x, hipMemcpyAsync(S.tr.am, S.am0, kMlpParams * sizeof(float), hipMemcpyDeviceToDevice, s));
    HIPCHK(x, hipMemcpyAsync(S.tr.av, S.av0, kMlpParams * sizeof(float), hipMemcpyDeviceToDevice, s));
    HIPCHK(x, hipStreamSynchronize(s));
    S.tr.step = S.step0;
    S.active = true;
    S.info.active = 1;
    S.info.round = -1;
    S.info.train_steps = S.step0;
    return ABCSMC_OK;
}

}  // namespace rt
}  // namespace abcsmc

namespace {

// Device copies for the context-free network hooks.
struct DevBuf {
    void* p = nullptr;
    ~DevBuf()
    {
        if (p) (void)hipFree(p);
    }
};

int hook_fail(hipError_t e)
{
    (void)hipGetLastError();
    return fail(nullptr, e == hipErrorOutOfMemory ? ABCSMC_ENOMEM : ABCSMC_EDEVICE,
                std::string("device call failed: ") + hipGetErrorString(e));
}

#define HOOKCHK(expr)                         \
    do {                                      \
        hipError_t e_ = (expr);               \
        if (e_ != hipSuccess) return hook_fail(e_); \
    } while (0)

// ---------------------------------------------------------------------------
// Allocation-free network forward.  The bfloat16 copy of the network that the
// fused scoring kernel reads lives in `scratch`, a file-scope device array
// (each GPU the library runs on holds its own copy until the process ends),
// instead of memory allocated per call.  In host code `scratch` only names
// the symbol: its device address on the current GPU is looked up once per
// device with hipGetSymbolAddress and cached; kernels receive that address.
// ---------------------------------------------------------------------------
constexpr size_t kScratchElems = ((size_t)kMlpParams + 127) / 128 * 128;  // 269,568 bytes
static __device__ __align__(256) __bf16 scratch[kScratchElems];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

hipError_t scratch_address(void** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return hipSuccess;
}

}  // namespace

extern "C" {

int abcsmc_surrogate_enable(abcsmc_ctx* x, const abcsmc_surrogate_config* scfg)
{
    if (!x) return fail(nullptr, ABCSMC_EINVAL, "ctx is NULL");
    if (x->broken) return fail(&x->err, ABCSMC_ESTATE, "context unusable after a device error");
    if (x->cfg.step_schedule == ABCSMC_STEP_MCMC)
        return fail(&x->err, ABCSMC_EINVAL, "the surrogate screen needs a Beta step schedule");
    abcsmc_surrogate_config def{};
    const abcsmc_surrogate_config c = with_defaults(scfg ? scfg : &def);
    int rc = check_scfg(c, &x->err);
    if (rc) return rc;
    if (x->sur) {
        surrogate_free(x->sur);
        x->sur = nullptr;
    }
    Surrogate* S = new Surrogate();
    S->cfg = c;
    S->tune_cap = c.tune_rows / kBlock * kBlock;
    S->n_train = c.n_train;
    const size_t bytes = carve_surrogate(*S, nullptr, x->N);
    if (hipMalloc((void**)&S->mem, bytes) != hipSuccess) {
        (void)hipGetLastError();
        S->mem = nullptr;
        surrogate_free(S);
        return fail(&x->err, ABCSMC_ENOMEM, "hipMalloc of the surrogate state failed");
    }
    carve_surrogate(*S, S->mem, x->N);
    for (auto& e : S->ev)
        if (hipEventCreate(&e) != hipSuccess) {
            surrogate_free(S);
            x->broken = true;
            return fail(&x->err, ABCSMC_EDEVICE, "hipEventCreate failed");
        }
    x->sur = S;
    hipStream_t s = x->stream;
    HIPCHK(x, hipEventRecord(S->ev[0], s));
    launch_mlp_init(S->tr.params, c.seed, s);
    HIPCHK(x, hipMemsetAsync(S->tr.am, 0, kMlpParams * sizeof(float), s));
    HIPCHK(x, hipMemsetAsync(S->tr.av, 0, kMlpParams * sizeof(float), s));
    TrainDataArgs ta{x->model, x->at<double>(x->L.obs), c.n_train, S->tx, S->ty};
    launch_train_data(ta, s);
    HIPCHK(x, hipGetLastError());
    HIPCHK(x, hipEventRecord(S->ev[1], s));
    // the loss is read back only after the first and the last pass
    std::vector<double> losses(2, 0.0);
    for (int32_t e = 0; e < c.epochs; ++e) {
        double* le = (e == 0) ? &losses[0] : (e == c.epochs - 1 ? &losses[1] : nullptr);
        HIPCHK(x, train_epochs(S->tr, S->tx, S->ty, c.n_train, c.batch, 1, (float)c.lr, le, s));
    }
    HIPCHK(x, hipEventRecord(S->ev[2], s));
    HIPCHK(x, hipMemcpyAsync(S->params0, S->tr.params, kMlpParams * sizeof(float), hipMemcpyDeviceToDevice, s));
    HIPCHK(x, hipMemcpyAsync(S->am0, S->tr.am, kMlpParams * sizeof(float), hipMemcpyDeviceToDevice, s));
    HIPCHK(x, hipMemcpyAsync(S->av0, S->tr.av, kMlpParams * sizeof(float), hipMemcpyDeviceToDevice, s));
    HIPCHK(x, hipStreamSynchronize(s));
    S->step0 = S->tr.step;
    S->info = abcsmc_surrogate_info{};
    S->info.loss_first = c.epochs ? losses[0] : 0.0;
    S->info.loss_last = c.epochs ? (c.epochs == 1 ? losses[0] : losses[1]) : 0.0;
    S->info.train_steps = S->tr.step;
    S->info.ms_data = elapsed(S->ev[0], S->ev[1]);
    S->info.ms_train = elapsed(S->ev[1], S->ev[2]);
    // multiply-adds per sample: 8*256 + 256*256 * 2 + 256*3
    const double macs = (double)kIn * kH + 2.0 * kH * kH + (double)kH * kOut;
    S->info.train_flops = (int64_t)(2.0 * 3.0 * macs * (double)c.n_train * (double)c.epochs);
    S->info.active = 1;
    S->info.round = -1;
    // the population of the last completed stage has no audit acceptances
    launch_fill_u8(S->pop_audit[0], 0, x->N, s);
    launch_fill_u8(S->pop_audit[1], 0, x->N, s);
    HIPCHK(x, hipGetLastError());
    HIPCHK(x, hipStreamSynchronize(s));
    return ABCSMC_OK;
}

int abcsmc_surrogate_disable(abcsmc_ctx* x)
{
    if (!x) return fail(nullptr, ABCSMC_EINVAL, "ctx is NULL");
    if (x->stream) (void)hipStreamSynchronize(x->stream);
    surrogate_free(x->sur);
    x->sur = nullptr;
    return ABCSMC_OK;
}

int abcsmc_surrogate_info_get(const abcsmc_ctx* x, abcsmc_surrogate_info* info)
{
    if (!x || !info) return fail(nullptr, ABCSMC_EINVAL, "ctx or info is NULL");
    if (!x->sur) return fail(const_cast<std::string*>(&x->err), ABCSMC_ESTATE, "surrogate not enabled");
    *info = x->sur->info;
    return ABCSMC_OK;
}

int abcsmc_surrogate_params(const abcsmc_ctx* cx, float* params)
{
    abcsmc_ctx* x = const_cast<abcsmc_ctx*>(cx);
    if (!x || !params) return fail(nullptr, ABCSMC_EINVAL, "ctx or params is NULL");
    if (x->broken) return fail(&x->err, ABCSMC_ESTATE, "context unusable after a device error");
    if (!x->sur) return fail(&x->err, ABCSMC_ESTATE, "surrogate not enabled");
    HIPCHK(x, hipMemcpyAsync(params, x->sur->tr.params, kMlpParams * sizeof(float), hipMemcpyDeviceToHost, x->stream));
    HIPCHK(x, hipStreamSynchronize(x->stream));
    return ABCSMC_OK;
}

int abcsmc_surrogate_data(const abcsmc_ctx* cx, int64_t n, float* xs, float* ys)
{
    abcsmc_ctx* x = const_cast<abcsmc_ctx*>(cx);
    if (!x) return fail(nullptr, ABCSMC_EINVAL, "ctx is NULL");
    if (x->broken) return fail(&x->err, ABCSMC_ESTATE, "context unusable after a device error");
    if (!x->sur) return fail(&x->err, ABCSMC_ESTATE, "surrogate not enabled");
    if (n < 0 || n > x->sur->n_train) return fail(&x->err, ABCSMC_EINVAL, "n must be in [0, n_train]");
    if (xs) HIPCHK(x, hipMemcpyAsync(xs, x->sur->tx, (size_t)n * kIn * sizeof(float), hipMemcpyDeviceToHost, x->stream));
    if (ys) HIPCHK(x, hipMemcpyAsync(ys, x->sur->ty, (size_t)n * kOut * sizeof(float), hipMemcpyDeviceToHost, x->stream));
    HIPCHK(x, hipStreamSynchronize(x->stream));
    return ABCSMC_OK;
}

int abcsmc_surrogate_audit(const abcsmc_ctx* cx, uint8_t* audit)
{
    abcsmc_ctx* x = const_cast<abcsmc_ctx*>(cx);
    if (!x || !audit) return fail(nullptr, ABCSMC_EINVAL, "ctx or audit is NULL");
    if (x->broken) return fail(&x->err, ABCSMC_ESTATE, "context unusable after a device error");
    if (!x->sur) return fail(&x->err, ABCSMC_ESTATE, "surrogate not enabled");
    if (x->rounds == 0) return fail(&x->err, ABCSMC_ESTATE, "no completed stage");
    HIPCHK(x, hipMemcpyAsync(audit, x->sur->pop_audit[x->cur], (size_t)x->N, hipMemcpyDeviceToHost, x->stream));
    HIPCHK(x, hipStreamSynchronize(x->stream));
    return ABCSMC_OK;
}

int64_t abcsmc_mlp_param_count(void) { return kMlpParams; }

int abcsmc_mlp_init(uint64_t seed, float* params)
{
    if (!params) return fail(nullptr, ABCSMC_EINVAL, "params is NULL");
    DevBuf p;
    HOOKCHK(hipMalloc(&p.p, kMlpParams * sizeof(float)));
    launch_mlp_init((float*)p.p, seed, nullptr);
    HOOKCHK(hipGetLastError());
    HOOKCHK(hipMemcpy(params, p.p, kMlpParams * sizeof(float), hipMemcpyDeviceToHost));
    return ABCSMC_OK;
}

int abcsmc_mlp_forward(const float* params, int64_t n, const float* xs, float* out)
{
    if (!params || !xs || !out) return fail(nullptr, ABCSMC_EINVAL, "NULL argument");
    if (n < 1 || n > kInferRows) return fail(nullptr, ABCSMC_EINVAL, "n must be in [1, 65536]");
    DevBuf m;
    Carver c{nullptr};
    for (int pass = 0; pass < 2; ++pass) {
        float* P = c.take<float>(kMlpParams);
        __bf16* Wb = c.take<__bf16>(kMlpParams);
        float* X = c.take<float>((size_t)n * kIn);
        float* O = c.take<float>((size_t)n * kOut);
        if (pass == 0) {
            HOOKCHK(hipMalloc(&m.p, c.off));
            c = Carver{(char*)m.p};
            continue;
        }
        HOOKCHK(hipMemcpy(P, params, kMlpParams * sizeof(float), hipMemcpyHostToDevice));
        HOOKCHK(hipMemcpy(X, xs, (size_t)n * kIn * sizeof(float), hipMemcpyHostToDevice));
        mlp_infer(P, Wb, X, n, O, nullptr, nullptr);
        HOOKCHK(hipGetLastError());
        HOOKCHK(hipMemcpy(out, O, (size_t)n * kOut * sizeof(float), hipMemcpyDeviceToHost));
    }
    return ABCSMC_OK;
}

int abcsmc_mlp_forward_noalloc(const float* params, int64_t n, const float* x, float* out, void* stream)
{
    if (!params || !x || !out) return fail(nullptr, ABCSMC_EINVAL, "NULL argument");
    if (n < 1 || n > kInferRows) return fail(nullptr, ABCSMC_EINVAL, "n must be in [1, 65536]");
    void* wb = nullptr;
    HOOKCHK(scratch_address(&wb));
    mlp_infer(params, (__bf16*)wb, x, n, out, nullptr, (hipStream_t)stream);
    HOOKCHK(hipGetLastError());
    return ABCSMC_OK;
}

int abcsmc_mlp_gradients(const float* params, int64_t n, const float* xs, const float* ys, float* grad,
                         double* loss)
{
    if (!params || !xs || !ys || !grad) return fail(nullptr, ABCSMC_EINVAL, "NULL argument");
    if (n < 1 || n > kTrainBatchMax) return fail(nullptr, ABCSMC_EINVAL, "n must be in [1, 65536]");
    DevBuf m;
    Trainer t;
    Carver c{nullptr};
    carve_trainer(c, t, n, n);
    c.take<float>((size_t)n * kIn);
    c.take<float>((size_t)n * kOut);
    HOOKCHK(hipMalloc(&m.p, c.off));
    c = Carver{(char*)m.p};
    carve_trainer(c, t, n, n);
    float* X = c.take<float>((size_t)n * kIn);
    float* Y = c.take<float>((size_t)n * kOut);
    HOOKCHK(hipMemcpy(t.params, params, kMlpParams * sizeof(float), hipMemcpyHostToDevice));
    HOOKCHK(hipMemcpy(X, xs, (size_t)n * kIn * sizeof(float), hipMemcpyHostToDevice));
    HOOKCHK(hipMemcpy(Y, ys, (size_t)n * kOut * sizeof(float), hipMemcpyHostToDevice));
    TrainArgs ta = train_args(t, X, Y, n, t.se);
    ta.grad = t.grad;
    launch_train_copies(ta, nullptr);
    launch_train_step(ta, 0.f, 0, nullptr);
    HOOKCHK(hipGetLastError());
    HOOKCHK(hipMemcpy(grad, t.grad, kMlpParams * sizeof(float), hipMemcpyDeviceToHost));
    if (loss) {
        std::vector<float> se((size_t)n);
        HOOKCHK(hipMemcpy(se.data(), t.se, (size_t)n * sizeof(float), hipMemcpyDeviceToHost));
        double sum = 0.0;
        for (float v : se) sum += (double)v;
        *loss = sum / (3.0 * (double)n);
    }
    return ABCSMC_OK;
}

int abcsmc_mlp_train(float* params, int64_t n, const float* xs, const float* ys, int32_t batch, int32_t epochs,
                     double lr, double* losses)
{
    if (!params || !xs || !ys) return fail(nullptr, ABCSMC_EINVAL, "NULL argument");
    if (n < 1 || n > ((int64_t)1 << 24)) return fail(nullptr, ABCSMC_EINVAL, "n must be in [1, 2^24]");
    if (batch < 1 || batch > kTrainBatchMax) return fail(nullptr, ABCSMC_EINVAL, "batch must be in [1, 65536]");
    if (epochs < 0 || epochs > 1000) return fail(nullptr, ABCSMC_EINVAL, "epochs must be in [0, 1000]");
    if (!(lr > 0.0 && lr < 1.0)) return fail(nullptr, ABCSMC_EINVAL, "lr must be in (0, 1)");
    DevBuf m;
    Trainer t;
    Carver c{nullptr};
    carve_trainer(c, t, batch, n);
    c.take<float>((size_t)n * kIn);
    c.take<float>((size_t)n * kOut);
    HOOKCHK(hipMalloc(&m.p, c.off));
    c = Carver{(char*)m.p};
    carve_trainer(c, t, batch, n);
    float* X = c.take<float>((size_t)n * kIn);
    float* Y = c.take<float>((size_t)n * kOut);
    HOOKCHK(hipMemcpy(t.params, params, kMlpParams * sizeof(float), hipMemcpyHostToDevice));
    HOOKCHK(hipMemset(t.am, 0, kMlpParams * sizeof(float)));
    HOOKCHK(hipMemset(t.av, 0, kMlpParams * sizeof(float)));
    HOOKCHK(hipMemcpy(X, xs, (size_t)n * kIn * sizeof(float), hipMemcpyHostToDevice));
    HOOKCHK(hipMemcpy(Y, ys, (size_t)n * kOut * sizeof(float), hipMemcpyHostToDevice));
    HOOKCHK(train_epochs(t, X, Y, n, batch, epochs, (float)lr, losses, nullptr));
    HOOKCHK(hipMemcpy(params, t.params, kMlpParams * sizeof(float), hipMemcpyDeviceToHost));
    return ABCSMC_OK;
}

}  // extern "C"
