// runtime.hip -- host runtime behind the C ABI of include/abcsmc.h: config
// validation, device workspace, the stage loop (resample -> batches of
// proposals -> ordered compaction -> importance weights -> next tolerance)
// and the copy-out calls.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "abcsmc.h"
#include "kernels.h"
#include "ctx.h"
#include "predict.h"

using namespace abcsmc;
using namespace abcsmc::rt;

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int64_t default_batch_cap(int64_t N)
{
    int64_t b = 4 * N;
    if (b < 65536) b = 65536;
    if (b > (int64_t)1 << 22) b = (int64_t)1 << 22;
    return b;
}

int64_t batch_cap(const abcsmc_config& c)
{
    const int64_t b = c.batch > 0 ? c.batch : default_batch_cap(c.n_particles);
    return (b + kBlock - 1) / kBlock * kBlock;
}

Layout make_layout(const abcsmc_config& c)
{
    Layout L{};
    const size_t N = (size_t)c.n_particles, T = (size_t)c.n_days;
    const size_t B = (size_t)batch_cap(c);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    L.obs = take((T + 1) * 3 * sizeof(double));
    for (int p = 0; p < 2; ++p) {
        L.pop[p][0] = take(N * kNP * sizeof(double));
        L.pop[p][1] = take(N * sizeof(double));
        L.pop[p][2] = take(N * sizeof(double));
        L.pop[p][3] = take(N * sizeof(int32_t));
        L.pop[p][4] = take(N * sizeof(uint32_t));
        L.pop[p][5] = take(N * sizeof(int32_t));
        L.pop[p][6] = take(N * sizeof(double));
        L.pop[p][7] = take(N * sizeof(double));
    }
    L.q = take(N * sizeof(uint64_t));
    L.cdf = take(N * sizeof(uint64_t));
    L.cols = take(N * 9 * sizeof(double));
    L.st_u = take(B * kNP * sizeof(double));
    L.st_d = take(B * sizeof(double));
    L.st_sigma = take(B * sizeof(double));
    L.st_parent = take(B * sizeof(int32_t));
    L.st_att = take(B * sizeof(int32_t));
    L.wave_mask = take((B / kWave + 4) * sizeof(unsigned long long));
    L.wave_off = take((B / kWave + 4) * sizeof(uint32_t));
    L.ctr = take(sizeof(StageCounters));
    L.scal = take(8 * sizeof(double));
    L.theta = take(N * kNP * sizeof(double));
    for (int r = 0; r < 5; ++r) L.red[r] = take(kRedMax * 8);
    L.hist = take(2 * 2048 * sizeof(unsigned int));
    L.sel = take(8 * sizeof(unsigned long long));
    L.wpart = take((size_t)std::max(weight_chunks((int64_t)N), weight_window_chunks((int64_t)N)) * N * sizeof(double));
    const size_t npad = sort_padded_size(N);
    L.rowkeys = take(npad * 8);
    L.colkeys = take(npad * 8);
    L.scols = take(N * 9 * sizeof(double));
    L.skey = take(N * sizeof(double));
    L.dimpart = take(256 * 16 * sizeof(double));
    L.dstar = take(sizeof(int32_t));
    L.win = take(((N + kWeightRows - 1) / kWeightRows) * sizeof(int2));
    L.rwin = take(N * sizeof(double));
    L.wtab = take(kWeightTab * sizeof(double));
    L.total = o;
    return L;
}

int validate(const abcsmc_config* c, const int64_t* obs, std::string* err)
{
    if (!c) return fail(err, ABCSMC_EINVAL, "config is NULL");
    if (c->abi_version != ABCSMC_ABI_VERSION) return fail(err, ABCSMC_EINVAL, "abi_version mismatch");
    if (c->n_params != ABCSMC_NPAR) return fail(err, ABCSMC_EINVAL, "n_params must be 8");
    for (int d = 0; d < ABCSMC_NPAR; ++d)
        if (!(c->prior_lo[d] <= c->prior_hi[d]) || !std::isfinite(c->prior_lo[d]) || !std::isfinite(c->prior_hi[d]))
            return fail(err, ABCSMC_EINVAL, "prior box needs finite lo <= hi");
    if (c->population < 1 || c->population >= ((int64_t)1 << 53)) return fail(err, ABCSMC_EINVAL, "population out of range");
    if (c->n_days < 1 || c->n_days > 4096) return fail(err, ABCSMC_EINVAL, "n_days must be in [1, 4096]");
    if (c->n_particles < 2 || c->n_particles > ((int64_t)1 << 22)) return fail(err, ABCSMC_EINVAL, "n_particles must be in [2, 2^22]");
    if (c->batch < 0 || c->batch > ((int64_t)1 << 24)) return fail(err, ABCSMC_EINVAL, "batch must be in [0, 2^24]");
    if (!(c->surv_ratio > 0.0 && c->surv_ratio < 1.0)) return fail(err, ABCSMC_EINVAL, "surv_ratio must be in (0,1)");
    if (c->step_schedule < ABCSMC_STEP_PAPER || c->step_schedule > ABCSMC_STEP_MODECONC)
        return fail(err, ABCSMC_EINVAL, "unknown step_schedule");
    if (c->step_schedule == ABCSMC_STEP_MCMC &&
        (c->batch <= 0 || !(c->mcmc_s0 > 0.0) || !std::isfinite(c->mcmc_s0) || c->mcmc_tune < 0))
        return fail(err, ABCSMC_EINVAL, "MCMC step schedule needs batch > 0, mcmc_s0 > 0 and mcmc_tune >= 0");
    if (c->step_schedule == ABCSMC_STEP_FIXED && (!(c->beta_a > 0.0) || !std::isfinite(c->beta_a) || c->beta_b < 1 || c->beta_b > 64))
        return fail(err, ABCSMC_EINVAL, "fixed Beta needs a > 0 and integer 1 <= b <= 64");
    if (c->sampler != ABCSMC_SAMPLER_BINOMIAL && c->sampler != ABCSMC_SAMPLER_NORMAL_FLOOR)
        return fail(err, ABCSMC_EINVAL, "unknown sampler");
    if (c->flags & ~(ABCSMC_F_EARLY_EXIT | ABCSMC_F_STEP_IS_VARIANCE | ABCSMC_F_SKIP_WEIGHTS))
        return fail(err, ABCSMC_EINVAL, "unknown flags");
    if (c->n_eps_schedule < 0 || c->n_eps_schedule > 4096)
        return fail(err, ABCSMC_EINVAL, "n_eps_schedule must be in [0, 4096]");
    if (c->n_eps_schedule > 0) {
        if (!c->eps_schedule) return fail(err, ABCSMC_EINVAL, "eps_schedule is NULL");
        for (int32_t i = 0; i < c->n_eps_schedule; ++i)
            if (!(c->eps_schedule[i] >= 0.0) || !std::isfinite(c->eps_schedule[i]))
                return fail(err, ABCSMC_EINVAL, "eps_schedule values must be finite and >= 0");
    }
    if (c->max_attempts < 0 || c->max_attempts > 4096) return fail(err, ABCSMC_EINVAL, "max_attempts must be in [0, 4096]");
    if (c->max_proposals < 0) return fail(err, ABCSMC_EINVAL, "max_proposals must be >= 0");
    if (obs) {
        for (int64_t t = 0; t <= c->n_days; ++t)
            for (int k = 0; k < 3; ++k)
                if (obs[t * 3 + k] < 0 || obs[t * 3 + k] > c->population)
                    return fail(err, ABCSMC_EINVAL, "observations must be counts in [0, P]");
        if (obs[0] + obs[1] + obs[2] > c->population) return fail(err, ABCSMC_EINVAL, "A0 + R0 + D0 exceeds P");
    }
    return ABCSMC_OK;
}

Model make_model(const abcsmc_config& c, const int64_t* obs0)
{
    Model m{};
    for (int d = 0; d < kNP; ++d) {
        m.lo[d] = c.prior_lo[d];
        m.width[d] = c.prior_hi[d] - c.prior_lo[d];
    }
    m.P = (double)c.population;
    m.invP = 1.0 / m.P;
    m.A0 = (double)obs0[0];
    m.R0 = (double)obs0[1];
    m.D0 = (double)obs0[2];
    m.T = c.n_days;
    m.sampler = c.sampler;
    m.seed = c.seed;
    return m;
}

}  // namespace

namespace {

void bind_pops(abcsmc_ctx* x)
{
    for (int p = 0; p < 2; ++p) {
        x->pop[p].u = x->at<double>(x->L.pop[p][0]);
        x->pop[p].d = x->at<double>(x->L.pop[p][1]);
        x->pop[p].sigma = x->at<double>(x->L.pop[p][2]);
        x->pop[p].parent = x->at<int32_t>(x->L.pop[p][3]);
        x->pop[p].index = x->at<uint32_t>(x->L.pop[p][4]);
        x->pop[p].att = x->at<int32_t>(x->L.pop[p][5]);
        x->pop[p].logw = x->at<double>(x->L.pop[p][6]);
        x->pop[p].W = x->at<double>(x->L.pop[p][7]);
    }
}

}  // namespace

extern "C" {

int abcsmc_abi_version(void) { return ABCSMC_ABI_VERSION; }

const char* abcsmc_strerror(int code)
{
    switch (code) {
    case ABCSMC_OK: return "ok";
    case ABCSMC_EINVAL: return "invalid argument";
    case ABCSMC_ENOMEM: return "out of device memory";
    case ABCSMC_EDEVICE: return "device error";
    case ABCSMC_EBUDGET: return "proposal budget exhausted";
    case ABCSMC_ESTATE: return "invalid state";
    case ABCSMC_EDEGENERATE: return "degenerate population";
    default: return "unknown error";
    }
}

const char* abcsmc_last_error(const abcsmc_ctx* ctx)
{
    return ctx ? ctx->err.c_str() : g_last_error.c_str();
}

int abcsmc_workspace_size(const abcsmc_config* cfg, size_t* bytes)
{
    std::string e;
    int rc = validate(cfg, nullptr, &e);
    if (rc) return rc;
    if (!bytes) return fail(nullptr, ABCSMC_EINVAL, "bytes is NULL");
    *bytes = make_layout(*cfg).total;
    return ABCSMC_OK;
}

void abcsmc_free(abcsmc_ctx* ctx)
{
    if (!ctx) return;
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    surrogate_free(ctx->sur);
    for (auto& e : ctx->ev)
        if (e) (void)hipEventDestroy(e);
    if (ctx->stage_host) (void)hipHostFree(ctx->stage_host);
    if (ctx->own_ws && ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

int abcsmc_init(const abcsmc_config* cfg, const int64_t* obs, abcsmc_ctx** out)
{
    if (!out) return fail(nullptr, ABCSMC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!obs) return fail(nullptr, ABCSMC_EINVAL, "obs is NULL");
    std::string e;
    int rc = validate(cfg, obs, &e);
    if (rc) return rc;
    abcsmc_ctx* x = new abcsmc_ctx();
    x->cfg = *cfg;
    if (x->cfg.max_attempts == 0) x->cfg.max_attempts = 256;
    x->N = cfg->n_particles;
    const int64_t cap = ((int64_t)1 << 32) - 1 - batch_cap(*cfg);
    if (x->cfg.max_proposals == 0 || x->cfg.max_proposals > cap)
        x->cfg.max_proposals = std::min<int64_t>(cap, x->cfg.max_proposals ? x->cfg.max_proposals : 4096 * x->N);
    x->obs.assign(obs, obs + (size_t)(cfg->n_days + 1) * 3);
    x->eps_sched.assign(cfg->eps_schedule, cfg->eps_schedule + cfg->n_eps_schedule);
    x->cfg.eps_schedule = x->eps_sched.empty() ? nullptr : x->eps_sched.data();
    x->mcmc_s = cfg->mcmc_s0;
    x->model = make_model(x->cfg, obs);
    x->L = make_layout(x->cfg);
    auto bail = [&](int code) {
        std::string msg = x->err;
        abcsmc_free(x);
        g_last_error = msg;
        return code;
    };
    if (cfg->stream) {
        x->stream = (hipStream_t)cfg->stream;
    } else {
        if (hipStreamCreateWithFlags(&x->stream, hipStreamNonBlocking) != hipSuccess) {
            x->err = "hipStreamCreate failed";
            return bail(ABCSMC_EDEVICE);
        }
        x->own_stream = true;
    }
    if (cfg->workspace) {
        if (cfg->workspace_bytes < x->L.total) {
            x->err = "workspace too small";
            return bail(ABCSMC_ENOMEM);
        }
        if (((uintptr_t)cfg->workspace) % kAlign) {
            x->err = "workspace must be 256-byte aligned";
            return bail(ABCSMC_EINVAL);
        }
        x->ws = (char*)cfg->workspace;
    } else {
        if (hipMalloc((void**)&x->ws, x->L.total) != hipSuccess) {
            x->err = "hipMalloc of the workspace failed";
            (void)hipGetLastError();
            x->ws = nullptr;
            return bail(ABCSMC_ENOMEM);
        }
        x->own_ws = true;
    }
    bind_pops(x);
    x->first_batch = propose_first_batch_lanes();
    for (auto& ev : x->ev)
        if (hipEventCreate(&ev) != hipSuccess) {
            x->err = "hipEventCreate failed";
            return bail(ABCSMC_EDEVICE);
        }
    std::vector<double> od(x->obs.begin(), x->obs.end());
    launch_weight_table(x->at<double>(x->L.wtab), x->stream);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(x->at<double>(x->L.obs), od.data(), od.size() * sizeof(double), hipMemcpyHostToDevice,
                       x->stream) != hipSuccess ||
        hipStreamSynchronize(x->stream) != hipSuccess) {
        x->err = "set-up of the exponential table or copy of the observations failed";
        return bail(ABCSMC_EDEVICE);
    }
    *out = x;
    return ABCSMC_OK;
}

int abcsmc_rounds_done(const abcsmc_ctx* ctx) { return ctx ? ctx->rounds : ABCSMC_EINVAL; }

int abcsmc_reset(abcsmc_ctx* x)
{
    if (!x) return fail(nullptr, ABCSMC_EINVAL, "ctx is NULL");
    if (x->broken) return fail(&x->err, ABCSMC_ESTATE, "context unusable after a device error");
    x->rounds = 0;
    x->cur = 0;
    x->eps_next = INFINITY;
    x->eps1 = INFINITY;
    x->last_rate = 0.5;
    x->mcmc_s = x->cfg.mcmc_s0;
    x->mcmc_tunes = 0;
    x->mcmc_nacc = 0;
    if (x->sur) return surrogate_reset(x);
    return ABCSMC_OK;
}

int abcsmc_round(abcsmc_ctx* x, abcsmc_round_info* info)
{
    if (!x) return fail(nullptr, ABCSMC_EINVAL, "ctx is NULL");
    if (x->broken) return fail(&x->err, ABCSMC_ESTATE, "context unusable after a device error");
    const abcsmc_config& c = x->cfg;
    const int32_t r = x->rounds;
    const int N = (int)x->N;
    const int nxt = x->rounds == 0 ? 0 : 1 - x->cur;  // buffer the new stage is written to
    const DevPop& prev = x->pop[x->cur];
    const DevPop& dst = x->pop[nxt];
    StageCounters* ctr = x->at<StageCounters>(x->L.ctr);
    double* scal = x->at<double>(x->L.scal);
    hipStream_t s = x->stream;

    // eq. 8's percentile of the last stage, or the replayed schedule
    const double eps = r == 0 ? INFINITY : (r <= c.n_eps_schedule ? x->eps_sched[(size_t)r - 1] : x->eps_next);
    double ba = 0.0, bb_real = 0.0;
    int32_t bb = 0;
    const bool general = c.step_schedule == ABCSMC_STEP_MEANVAR || c.step_schedule == ABCSMC_STEP_MODECONC;
    if (r > 0 && general) {
        // alternative parameterisations of the step-size Beta from the two
        // quantities eq. 16 tunes: the tolerance ratio and the stage index
        const double e1 = r == 1 ? eps : x->eps1;
        const double ratio = eps / e1;
        if (c.step_schedule == ABCSMC_STEP_MEANVAR) {
            double mu = ratio / 3.0;                                           // mean
            if (mu < 1e-12) mu = 1e-12;                                        // eps_i = 0
            const double var = mu * (1.0 - mu) / (3.0 * (double)r + 1.0);       // variance
            const double k = mu * (1.0 - mu) / var - 1.0;
            ba = mu * k;
            bb_real = (1.0 - mu) * k;
        } else {
            const double w = ratio / 4.0;                                       // mode
            const double k = 2.0 * (double)r + 2.0;                             // concentration
            ba = w * (k - 2.0) + 1.0;
            bb_real = (1.0 - w) * (k - 2.0) + 1.0;
        }
    } else if (r > 0 && c.step_schedule != ABCSMC_STEP_MCMC) {
        if (c.step_schedule == ABCSMC_STEP_FIXED) {
            ba = c.beta_a;
            bb = c.beta_b;
        } else {
            const double e1 = r == 1 ? eps : x->eps1;
            ba = eps / e1;  // eq. 16: alpha_i = eps_i / eps_1, beta_i = 2 i
            bb = 2 * r;
            if (bb > 128) return fail(&x->err, ABCSMC_EINVAL, "eq. 16 schedule limited to 64 stages");
        }
    }
    const double exit_thr = ((c.flags & ABCSMC_F_EARLY_EXIT) && std::isfinite(eps))
                                ? (eps * eps) * (1.0 + 0x1p-48)
                                : INFINITY;

    const bool screened = surrogate_screens(x, r);
    HIPCHK(x, hipMemsetAsync(ctr, 0, sizeof(StageCounters), s));
    if (x->sur) {
        const int rc = surrogate_stage_begin(x, nxt);
        if (rc) return rc;
    }
    HIPCHK(x, hipEventRecord(x->ev[0], s));
    if (r > 0) {
        ResampleArgs ra{prev.d, prev.u, N, eps, x->at<uint64_t>(x->L.q), x->at<uint64_t>(x->L.cdf),
                        x->at<double>(x->L.cols), x->scratch(), ctr};
        launch_resample(ra, s);
        HIPCHK(x, hipGetLastError());
    }
    HIPCHK(x, hipEventRecord(x->ev[1], s));

    ProposeArgs pa{};
    pa.m = x->model;
    pa.obs = x->at<double>(x->L.obs);
    pa.round = (uint32_t)r;
    pa.max_attempts = c.max_attempts;
    pa.eps = eps;
    pa.exit_thr = exit_thr;
    pa.u_prev = prev.u;
    pa.cdf = x->at<uint64_t>(x->L.cdf);
    pa.n_prev = N;
    pa.beta_a = ba;
    pa.beta_b = bb;
    pa.step_is_variance = (c.flags & ABCSMC_F_STEP_IS_VARIANCE) ? 1 : 0;
    const bool mcmc = c.step_schedule == ABCSMC_STEP_MCMC;
    pa.s_fixed = (mcmc && r > 0) ? x->mcmc_s : -1.0;
    pa.beta_b_real = (general && r > 0) ? bb_real : 0.0;
    pa.st_u = x->at<double>(x->L.st_u);
    pa.st_d = x->at<double>(x->L.st_d);
    pa.st_sigma = x->at<double>(x->L.st_sigma);
    pa.st_parent = x->at<int32_t>(x->L.st_parent);
    pa.st_att = x->at<int32_t>(x->L.st_att);
    pa.wave_mask = x->at<unsigned long long>(x->L.wave_mask);
    pa.ctr = ctr;
    CompactArgs ca{};
    ca.N = N;
    ca.wave_mask = pa.wave_mask;
    ca.wave_off = x->at<uint32_t>(x->L.wave_off);
    ca.st_u = pa.st_u;
    ca.st_d = pa.st_d;
    ca.st_sigma = pa.st_sigma;
    ca.st_parent = pa.st_parent;
    ca.st_att = pa.st_att;
    ca.pop = dst.view();
    ca.ctr = ctr;

    const int64_t cap = batch_cap(c);
    int64_t base = 0, batches = 0;
    double ms_k_propose = 0.0;
    StageCounters hc{};
    unsigned long long prev_acc = 0, prev_inv = 0;
    if (screened) {
        const int rc = surrogate_batches(x, pa, dst, nxt, hc, base, batches, ms_k_propose);
        if (rc) return rc;
    }
    // A first batch that will all but surely reach N acceptances (stage 0,
    // where every valid proposal is accepted, and stages >= 2, sized from the
    // measured rate with a margin) is not read back on its own: the stage
    // goes straight on to its weights and tolerance, and the batch counters
    // come back with them in one host wait.  A batch that falls short after
    // all is completed by further batches, and the weights and tolerance are
    // formed again (every result is that of the batch-by-batch loop).
    bool spec_ok = !screened && !mcmc && !x->sur && r != 1;
    int64_t pending = 0;  // size of a batch whose counters are not yet read
    const bool weighted = r > 0 && !(c.flags & ABCSMC_F_SKIP_WEIGHTS);
    double hs[2] = {0, 0};
    unsigned long long hterms[2] = {0, 0};  // terms, window_terms (adjacent counters)
    for (;;) {
        while (!screened) {
            int64_t B;
            bool sure = false;  // the batch is sized to reach N acceptances
            if (r == 0) {
                B = std::min<int64_t>(cap, (int64_t)N - (int64_t)hc.accepted);
                sure = B == (int64_t)N - (int64_t)hc.accepted;
            } else if (c.batch > 0) {
                B = c.batch;
            } else {
                const double need = (double)(N - (int64_t)hc.accepted);
                const double rate = x->last_rate > 1e-4 ? x->last_rate : 1e-4;
                B = (int64_t)std::ceil(need / rate * 1.1) + 2048;
                B = (B + kBlock - 1) / kBlock * kBlock;
                sure = B <= cap;
                // stage 1 has no measured acceptance rate yet: its first batch is
                // capped (a batch sized by the 0.5 guess simulated twice the
                // proposals needed at C2); later batches use the rate measured
                if (r == 1 && base == 0 && x->first_batch > 0 && B > x->first_batch) B = x->first_batch;
                if (B > cap) B = cap;
            }
            if (base + B > c.max_proposals) {
                B = c.max_proposals - base;
                sure = false;
            }
            if (B <= 0) return fail(&x->err, ABCSMC_EBUDGET, "stage exhausted its proposal budget");
            pa.base = (uint32_t)base;
            pa.count = (uint32_t)B;
            HIPCHK(x, hipEventRecord(x->ev[5], s));
            launch_propose(pa, r == 0, s);
            HIPCHK(x, hipGetLastError());
            HIPCHK(x, hipEventRecord(x->ev[6], s));
            ca.base = pa.base;
            ca.count = pa.count;
            launch_compact(ca, s);
            HIPCHK(x, hipGetLastError());
            if (spec_ok && sure && batches == 0) {
                pending = B;  // read back with the tolerance at the end of the stage
                break;
            }
            HIPCHK(x, hipMemcpyAsync(&hc, ctr, sizeof hc, hipMemcpyDeviceToHost, s));
            HIPCHK(x, hipStreamSynchronize(s));
            ms_k_propose += elapsed(x->ev[5], x->ev[6]);
            base += B;
            ++batches;
            if (mcmc && r > 0 && x->mcmc_tunes < c.mcmc_tune) {
                // eqs. 14-15 over this batch: A = accepted / valid proposals
                const int64_t acc_b = (int64_t)(hc.accepted - prev_acc);
                const int64_t valid_b = B - (int64_t)(hc.invalid - prev_inv);
                x->mcmc_nacc += acc_b;
                const double A = valid_b > 0 ? (double)acc_b / (double)valid_b : 0.0;
                x->mcmc_s = x->mcmc_s * (1.0 + (A - 0.234) / ((1.0 - 0.234) * ((double)x->mcmc_nacc + 1.0)));
                x->mcmc_tunes += 1;
                pa.s_fixed = x->mcmc_s;
            }
            prev_acc = hc.accepted;
            prev_inv = hc.invalid;
            if (hc.accepted >= (unsigned long long)N) break;
            if (r > 0 && base > 0) x->last_rate = (double)hc.accepted / (double)base;
        }
        HIPCHK(x, hipEventRecord(x->ev[2], s));
        if (!weighted) {
            launch_uniform_weights(dst.W, dst.logw, N, s);
        } else {
            WeightArgs wa{};
            wa.u = dst.u;
            wa.sigma = dst.sigma;
            wa.cols = x->at<double>(x->L.cols);
            wa.N = N;
            wa.chunks = weight_window_chunks(N);
            wa.cols_per_chunk = weight_cols_per_chunk(N);
            wa.win = x->at<int2>(x->L.win);
            wa.terms = &ctr->terms;
            wa.window_terms = &ctr->window_terms;
            wa.M = &ctr->survivors;
            wa.partial = x->at<double>(x->L.wpart);
            wa.logw = dst.logw;
            wa.rowkeys = x->at<unsigned long long>(x->L.rowkeys);
            wa.colkeys = x->at<unsigned long long>(x->L.colkeys);
            wa.scols = x->at<double>(x->L.scols);
            wa.skey = x->at<double>(x->L.skey);
            wa.dimpart = x->at<double>(x->L.dimpart);
            wa.dstar = x->at<int32_t>(x->L.dstar);
            wa.npad = sort_padded_size((size_t)N);
            wa.parent = dst.parent;
            wa.u_prev = prev.u;
            wa.q_prev = x->at<uint64_t>(x->L.q);
            wa.cdf = x->at<uint64_t>(x->L.cdf);
            wa.n_prev = N;
            wa.rwin = x->at<double>(x->L.rwin);
            wa.tab = x->at<double>(x->L.wtab);
            weight_exp_constants(wa.ex);
            launch_weights_window(wa, s);
            HIPCHK(x, hipGetLastError());
            HIPCHK(x, hipEventRecord(x->ev[7], s));
            launch_weights_sum(wa, s);
            HIPCHK(x, hipGetLastError());
            HIPCHK(x, hipEventRecord(x->ev[8], s));
            launch_weights_finalize(wa, s);
            HIPCHK(x, hipGetLastError());
            if (screened) {
                const int rc = surrogate_weights(x, dst, nxt);
                if (rc) return rc;
            }
            NormArgs na{dst.logw, dst.W, N, x->scratch(), scal + 1};
            launch_normalise(na, s);
        }
        HIPCHK(x, hipGetLastError());
        HIPCHK(x, hipEventRecord(x->ev[3], s));
        SelectArgs sa{dst.d, N, c.surv_ratio, x->scratch(), scal + 0};
        launch_select(sa, s);
        HIPCHK(x, hipGetLastError());
        HIPCHK(x, hipEventRecord(x->ev[4], s));
        HIPCHK(x, hipMemcpyAsync(hs, scal, sizeof hs, hipMemcpyDeviceToHost, s));
        HIPCHK(x, hipMemcpyAsync(hterms, &ctr->terms, sizeof hterms, hipMemcpyDeviceToHost, s));
        if (pending) HIPCHK(x, hipMemcpyAsync(&hc, ctr, sizeof hc, hipMemcpyDeviceToHost, s));
        HIPCHK(x, hipStreamSynchronize(s));
        if (pending) {
            ms_k_propose += elapsed(x->ev[5], x->ev[6]);
            base += pending;
            ++batches;
            pending = 0;
            prev_acc = hc.accepted;
            prev_inv = hc.invalid;
            if (hc.accepted < (unsigned long long)N) {
                // short of N after all: the remaining batches, then the weights again
                if (r > 0) x->last_rate = (double)hc.accepted / (double)base;
                spec_ok = false;
                HIPCHK(x, hipMemsetAsync(&ctr->terms, 0, 2 * sizeof(unsigned long long), s));
                continue;
            }
        }
        break;
    }  // stage passes
    if (r > 0) x->last_rate = (double)N / (double)hc.proposals;

    // commit the stage
    x->cur = nxt;
    x->rounds = r + 1;
    if (r == 1) x->eps1 = eps;
    x->eps_next = hs[0];
    if (screened) {
        const int rc = surrogate_stage_end(x, r);
        if (rc) return rc;
    }
    if (info) {
        abcsmc_round_info& I = *info;
        std::memset(&I, 0, sizeof I);
        I.round = r;
        I.eps = eps;
        I.eps_next = hs[0];
        I.beta_a = ba;
        I.beta_b = bb;
        I.ess = weighted ? hs[1] : (double)N;
        I.proposals = (int64_t)hc.proposals;
        I.simulated = base;
        I.invalid = (int64_t)hc.invalid;
        I.attempts = (int64_t)hc.attempts;
        I.survivors = r == 0 ? 0 : (int64_t)hc.survivors;
        I.batches = batches;
        I.ms_resample = elapsed(x->ev[0], x->ev[1]);
        I.ms_simulate = elapsed(x->ev[1], x->ev[2]);
        I.ms_weights = elapsed(x->ev[2], x->ev[3]);
        I.ms_select = elapsed(x->ev[3], x->ev[4]);
        I.ms_total = elapsed(x->ev[0], x->ev[4]);
        I.ms_k_propose = ms_k_propose;
        I.ms_k_weights = weighted ? elapsed(x->ev[7], x->ev[8]) : 0.0;
        I.n_k_propose = batches;
        I.sim_days = (int64_t)hc.days;
        I.weight_pairs = weighted ? (int64_t)N * (int64_t)hc.survivors : 0;
        I.weight_terms = (int64_t)hterms[0];
        I.weight_window_terms = (int64_t)hterms[1];
        I.mcmc_s = mcmc ? x->mcmc_s : 0.0;
        I.beta_b_real = general ? bb_real : (double)bb;
    }
    return ABCSMC_OK;
}

}  // extern "C"

extern "C" {

namespace {

// Device-to-host copies of up to kCopies arrays through the context's pinned
// staging buffer (pinned transfers run at link speed; pageable ones are
// staged by the runtime in small pieces), then one host copy per array.
struct CopyOut {
    void* dst;
    const void* src;
    size_t bytes;
};

int copy_out(abcsmc_ctx* x, const CopyOut* c, int n)
{
    size_t total = 0;
    for (int k = 0; k < n; ++k)
        if (c[k].dst) total += (c[k].bytes + 255) / 256 * 256;
    if (total > x->stage_bytes) {
        if (x->stage_host) (void)hipHostFree(x->stage_host);
        x->stage_host = nullptr;
        x->stage_bytes = 0;
        if (hipHostMalloc((void**)&x->stage_host, total, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            x->stage_host = nullptr;
            return fail(&x->err, ABCSMC_ENOMEM, "hipHostMalloc of the copy-out staging failed");
        }
        x->stage_bytes = total;
    }
    size_t off = 0;
    for (int k = 0; k < n; ++k) {
        if (!c[k].dst) continue;
        HIPCHK(x, hipMemcpyAsync(x->stage_host + off, c[k].src, c[k].bytes, hipMemcpyDeviceToHost, x->stream));
        off += (c[k].bytes + 255) / 256 * 256;
    }
    HIPCHK(x, hipStreamSynchronize(x->stream));
    off = 0;
    for (int k = 0; k < n; ++k) {
        if (!c[k].dst) continue;
        std::memcpy(c[k].dst, x->stage_host + off, c[k].bytes);
        off += (c[k].bytes + 255) / 256 * 256;
    }
    return ABCSMC_OK;
}

}  // namespace

int abcsmc_weights(const abcsmc_ctx* cx, double* theta, double* dist, double* weight)
{
    abcsmc_ctx* x = const_cast<abcsmc_ctx*>(cx);
    if (!x) return fail(nullptr, ABCSMC_EINVAL, "ctx is NULL");
    if (x->broken) return fail(&x->err, ABCSMC_ESTATE, "context unusable after a device error");
    if (x->rounds == 0) return fail(&x->err, ABCSMC_ESTATE, "no completed stage");
    const DevPop& p = x->pop[x->cur];
    const size_t N = (size_t)x->N;
    hipStream_t s = x->stream;
    double* th = x->at<double>(x->L.theta);
    if (theta) {
        launch_to_theta(p.u, x->model, th, (int64_t)N, s);
        HIPCHK(x, hipGetLastError());
    }
    const CopyOut c[3] = {{theta, th, N * kNP * sizeof(double)},
                          {dist, p.d, N * sizeof(double)},
                          {weight, p.W, N * sizeof(double)}};
    return copy_out(x, c, 3);
}

int abcsmc_population(const abcsmc_ctx* cx, double* u, double* sigma, int64_t* parent, int64_t* index,
                      int32_t* attempts, double* logw)
{
    abcsmc_ctx* x = const_cast<abcsmc_ctx*>(cx);
    if (!x) return fail(nullptr, ABCSMC_EINVAL, "ctx is NULL");
    if (x->broken) return fail(&x->err, ABCSMC_ESTATE, "context unusable after a device error");
    if (x->rounds == 0) return fail(&x->err, ABCSMC_ESTATE, "no completed stage");
    const DevPop& p = x->pop[x->cur];
    const size_t N = (size_t)x->N;
    std::vector<int32_t> pi(parent ? N : 0);
    std::vector<uint32_t> ii(index ? N : 0);
    const CopyOut c[6] = {{u, p.u, N * kNP * sizeof(double)},
                          {sigma, p.sigma, N * sizeof(double)},
                          {parent ? pi.data() : nullptr, p.parent, N * sizeof(int32_t)},
                          {index ? ii.data() : nullptr, p.index, N * sizeof(uint32_t)},
                          {attempts, p.att, N * sizeof(int32_t)},
                          {logw, p.logw, N * sizeof(double)}};
    if (const int rc = copy_out(x, c, 6)) return rc;
    for (size_t k = 0; k < pi.size(); ++k) parent[k] = pi[k];
    for (size_t k = 0; k < ii.size(); ++k) index[k] = ii[k];
    return ABCSMC_OK;
}

int abcsmc_predict(const abcsmc_ctx* cx, int32_t n_days, uint64_t seed, int32_t n_quant, const double* quant,
                   double* bands)
{
    abcsmc_ctx* x = const_cast<abcsmc_ctx*>(cx);
    if (!x) return fail(nullptr, ABCSMC_EINVAL, "ctx is NULL");
    if (x->broken) return fail(&x->err, ABCSMC_ESTATE, "context unusable after a device error");
    if (x->rounds == 0) return fail(&x->err, ABCSMC_ESTATE, "no completed stage");
    if (n_days < 1 || n_days > 4096) return fail(&x->err, ABCSMC_EINVAL, "n_days must be in [1, 4096]");
    if (n_quant < 1 || n_quant > 64 || !quant || !bands) return fail(&x->err, ABCSMC_EINVAL, "need 1..64 quantiles");
    for (int k = 0; k < n_quant; ++k)
        if (!(quant[k] >= 0.0 && quant[k] <= 1.0)) return fail(&x->err, ABCSMC_EINVAL, "quantiles must be in [0, 1]");
    const size_t N = (size_t)x->N;
    const size_t rows = (size_t)3 * (n_days + 1);
    const size_t bytes = rows * N * 8 + 64 * 8 + rows * 64 * 8;
    char* mem = nullptr;
    if (hipMalloc((void**)&mem, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(&x->err, ABCSMC_ENOMEM, "hipMalloc of the predictive series failed");
    }
    PredictArgs a{};
    a.m = x->model;
    a.m.T = n_days;
    a.u = x->pop[x->cur].u;
    a.n = (int64_t)N;
    a.round = kPredictRound;
    a.m.seed = seed;
    a.series = (double*)mem;
    a.quant = (const double*)(mem + rows * N * 8);
    a.n_quant = n_quant;
    a.bands = (double*)(mem + rows * N * 8 + 64 * 8);
    hipStream_t s = x->stream;
    hipError_t e = hipMemcpyAsync((void*)a.quant, quant, (size_t)n_quant * 8, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        launch_predict(a, s);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(bands, a.bands, rows * (size_t)n_quant * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(mem);
    if (e != hipSuccess) {
        x->broken = true;
        return fail(&x->err, ABCSMC_EDEVICE, std::string("predictive simulation: ") + hipGetErrorString(e));
    }
    return ABCSMC_OK;
}

int abcsmc_resampling(const abcsmc_ctx* cx, uint64_t* q, uint64_t* cdf)
{
    abcsmc_ctx* x = const_cast<abcsmc_ctx*>(cx);
    if (!x) return fail(nullptr, ABCSMC_EINVAL, "ctx is NULL");
    if (x->broken) return fail(&x->err, ABCSMC_ESTATE, "context unusable after a device error");
    if (x->rounds < 2) return fail(&x->err, ABCSMC_ESTATE, "no resampling before stage 1");
    const size_t N = (size_t)x->N;
    hipStream_t s = x->stream;
    if (q) HIPCHK(x, hipMemcpyAsync(q, x->at<uint64_t>(x->L.q), N * 8, hipMemcpyDeviceToHost, s));
    if (cdf) HIPCHK(x, hipMemcpyAsync(cdf, x->at<uint64_t>(x->L.cdf), N * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(x, hipStreamSynchronize(s));
    return ABCSMC_OK;
}

int abcsmc_run(const abcsmc_config* cfg, const int64_t* obs, int32_t n_rounds, double* theta, double* dist,
               double* weight, abcsmc_round_info* infos)
{
    if (n_rounds < 1) return fail(nullptr, ABCSMC_EINVAL, "n_rounds must be >= 1");
    abcsmc_ctx* x = nullptr;
    int rc = abcsmc_init(cfg, obs, &x);
    if (rc) return rc;
    for (int32_t i = 0; i < n_rounds && rc == ABCSMC_OK; ++i) rc = abcsmc_round(x, infos ? infos + i : nullptr);
    if (rc == ABCSMC_OK) rc = abcsmc_weights(x, theta, dist, weight);
    if (rc) g_last_error = x->err;
    abcsmc_free(x);
    return rc;
}

int abcsmc_simulate(const abcsmc_config* cfg, int64_t n, const double* theta, const int64_t* obs0, uint64_t seed,
                    uint32_t round, uint32_t index0, int64_t* traj)
{
    std::string e;
    int rc = validate(cfg, nullptr, &e);
    if (rc) return rc;
    if (n < 1 || !theta || !obs0 || !traj) return fail(nullptr, ABCSMC_EINVAL, "bad simulate arguments");
    if (obs0[0] < 0 || obs0[1] < 0 || obs0[2] < 0 || obs0[0] + obs0[1] + obs0[2] > cfg->population)
        return fail(nullptr, ABCSMC_EINVAL, "obs0 must be counts with A0+R0+D0 <= P");
    if ((uint64_t)index0 + (uint64_t)n > ((uint64_t)1 << 32)) return fail(nullptr, ABCSMC_EINVAL, "index range exceeds 2^32");
    TrajArgs ta{};
    ta.m = make_model(*cfg, obs0);
    ta.m.seed = seed;
    ta.n = n;
    ta.round = round;
    ta.index0 = index0;
    const size_t tb = (size_t)n * (size_t)(cfg->n_days + 1) * 6 * sizeof(int64_t);
    double* dth = nullptr;
    int64_t* dtr = nullptr;
    hipStream_t s = (hipStream_t)cfg->stream;
    auto cleanup = [&]() {
        if (dth) (void)hipFree(dth);
        if (dtr) (void)hipFree(dtr);
    };
    if (hipMalloc((void**)&dth, (size_t)n * kNP * sizeof(double)) != hipSuccess ||
        hipMalloc((void**)&dtr, tb) != hipSuccess) {
        (void)hipGetLastError();
        cleanup();
        return fail(nullptr, ABCSMC_ENOMEM, "hipMalloc failed in simulate");
    }
    ta.theta = dth;
    ta.traj = dtr;
    hipError_t err = hipMemcpyAsync(dth, theta, (size_t)n * kNP * sizeof(double), hipMemcpyHostToDevice, s);
    if (err == hipSuccess) {
        launch_simulate_traj(ta, s);
        err = hipGetLastError();
    }
    if (err == hipSuccess) err = hipMemcpyAsync(traj, dtr, tb, hipMemcpyDeviceToHost, s);
    if (err == hipSuccess) err = hipStreamSynchronize(s);
    cleanup();
    if (err != hipSuccess) return fail(nullptr, ABCSMC_EDEVICE, std::string("simulate: ") + hipGetErrorString(err));
    return ABCSMC_OK;
}

int abcsmc_debug_eval(int32_t fn, int64_t n, const void* in, void* out, double param_a, int32_t param_b)
{
    if (n < 1 || !in || !out || fn < 0 || fn > 14) return fail(nullptr, ABCSMC_EINVAL, "bad debug_eval arguments");
    if (fn == 13 && (!(param_a >= 0.0) || param_a > 9007199254740992.0))
        return fail(nullptr, ABCSMC_EINVAL, "seed must be an integer-valued double in [0, 2^53]");
    if (fn == 11 && (param_b < 1 || param_b > 128)) return fail(nullptr, ABCSMC_EINVAL, "beta b out of range");
    size_t in_b = 0, out_b = 0;
    switch (fn) {
    case 7: in_b = 16 * n; out_b = 8 * n; break;
    case 8: in_b = 24 * n; out_b = 16 * n; break;
    case 9: in_b = 8 * n; out_b = 16 * n; break;
    case 10: case 12: in_b = 24 * n; out_b = 8 * n; break;
    case 11: in_b = 8 * (size_t)n * param_b; out_b = 8 * n; break;
    case 13: in_b = 16; out_b = 8 * n; break;
    case 14: in_b = 18 * 8 * (size_t)n; out_b = 8 * n; break;
    default: in_b = 8 * n; out_b = 8 * n; break;
    }
    void *din = nullptr, *dout = nullptr;
    if (hipMalloc(&din, in_b) != hipSuccess || hipMalloc(&dout, out_b) != hipSuccess) {
        (void)hipGetLastError();
        if (din) (void)hipFree(din);
        if (dout) (void)hipFree(dout);
        return fail(nullptr, ABCSMC_ENOMEM, "hipMalloc failed in debug_eval");
    }
    hipError_t err = hipMemcpy(din, in, in_b, hipMemcpyHostToDevice);
    if (err == hipSuccess) {
        launch_debug_eval(fn, n, din, dout, param_a, param_b, nullptr);
        err = hipGetLastError();
    }
    if (err == hipSuccess) err = hipMemcpy(out, dout, out_b, hipMemcpyDeviceToHost);
    (void)hipFree(din);
    (void)hipFree(dout);
    if (err != hipSuccess) return fail(nullptr, ABCSMC_EDEVICE, std::string("debug_eval: ") + hipGetErrorString(err));
    return ABCSMC_OK;
}

}  // extern "C"
