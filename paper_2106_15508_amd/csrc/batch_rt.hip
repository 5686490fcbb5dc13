// batch_rt.hip -- host side of the batched mode: layout of many runs in one
// device workspace, work tables, graph capture of the per-stage kernel
// sequence (one graph for stage 0, one replayed for every later stage), and
// the schedule autotuner with its on-disk cache.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "abcsmc.h"
#include "batch.h"
#include "kernels.h"

using namespace abcsmc;

namespace {

thread_local std::string g_batch_err;

constexpr size_t kAl = 256;
inline size_t al(size_t x) { return (x + kAl - 1) / kAl * kAl; }

int bfail(std::string* e, int code, const std::string& m)
{
    if (e) *e = m;
    g_batch_err = m;
    return code;
}

int run_cap_chunks(const abcsmc_config& c)
{
    int64_t cap = c.max_proposals > 0 ? c.max_proposals : std::max<int64_t>(4 * c.n_particles, 16384);
    if (cap > ((int64_t)1 << 24)) cap = (int64_t)1 << 24;
    return (int)((cap + kChunkP - 1) / kChunkP);
}

int wchunks_max(int64_t N) { return (int)std::min<int64_t>(kMaxWChunks, std::max<int64_t>(1, (N / 2 + 2047) / 2048)); }

int wchunks_for(int64_t N, int weight_cols)
{
    const int64_t c = std::max<int64_t>(1, (N / 2 + weight_cols - 1) / weight_cols);
    return (int)std::min<int64_t>(c, wchunks_max(N));
}

struct RunLayout {
    size_t obs, u[2], d[2], sigma[2], logw[2], W[2], parent[2], index[2], att[2], q, cdf, cols, wpart, st_u, st_d,
        st_sigma, st_parent, st_att, wmask, woff, red_u, red_d, end;
};

RunLayout run_layout(const abcsmc_config& c, size_t o)
{
    RunLayout L{};
    const size_t N = (size_t)c.n_particles, T = (size_t)c.n_days;
    const size_t B = (size_t)run_cap_chunks(c) * kChunkP;
    const size_t nres = (N + 1023) / 1024;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = al(o + bytes);
        return at;
    };
    L.obs = take((T + 1) * 3 * 8);
    for (int p = 0; p < 2; ++p) {
        L.u[p] = take(N * kNP * 8);
        L.d[p] = take(N * 8);
        L.sigma[p] = take(N * 8);
        L.logw[p] = take(N * 8);
        L.W[p] = take(N * 8);
        L.parent[p] = take(N * 4);
        L.index[p] = take(N * 4);
        L.att[p] = take(N * 4);
    }
    L.q = take(N * 8);
    L.cdf = take(N * 8);
    L.cols = take(N * 9 * 8);
    L.wpart = take((size_t)wchunks_max((int64_t)N) * N * 8);
    L.st_u = take(B * kNP * 8);
    L.st_d = take(B * 8);
    L.st_sigma = take(B * 8);
    L.st_parent = take(B * 4);
    L.st_att = take(B * 4);
    L.wmask = take(B / kWave * 8);
    L.woff = take(B / kWave * 4);
    L.red_u = take(3 * nres * 8);
    L.red_d = take(nres * 8);
    L.end = o;
    return L;
}

// Batch-wide weight-window arrays after the tables: column and row sort keys
// (power-of-two length), sorted columns, their sort-coordinate values, one
// window per kWeightRows-row block, and the exponential table.
struct WinLayout {
    size_t colkeys, rowkeys, scols, skey, rwin, win, wtab, end, npad;
};

WinLayout win_layout(size_t o, size_t n_total, size_t n_fin)
{
    WinLayout L{};
    L.npad = sort_padded_size(n_total);
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = al(o + bytes);
        return at;
    };
    L.colkeys = take(L.npad * 8);
    L.rowkeys = take(L.npad * 8);
    L.scols = take(n_total * 9 * 8);
    L.skey = take(n_total * 8);
    L.rwin = take(n_total * 8);
    L.win = take(n_fin * sizeof(int2));
    L.wtab = take(kWeightTab * 8);
    L.end = o;
    return L;
}

// what batched runs do not support, on top of the single-run rules
int bunsupported(const abcsmc_config& c, std::string* e)
{
    if (c.step_schedule != ABCSMC_STEP_PAPER && c.step_schedule != ABCSMC_STEP_FIXED)
        return bfail(e, ABCSMC_EINVAL, "batched runs: eq. 16 or fixed Beta step schedules only");
    if (c.n_eps_schedule != 0) return bfail(e, ABCSMC_EINVAL, "batched runs: no tolerance schedule");
    if (c.flags & ABCSMC_F_SKIP_WEIGHTS) return bfail(e, ABCSMC_EINVAL, "batched runs: weights are always computed");
    return ABCSMC_OK;
}

// validation shared with the single-run path's rules (subset relevant here)
int bvalidate(const abcsmc_config& c, const int64_t* obs, std::string* e)
{
    size_t dummy;
    if (const int u = bunsupported(c, e)) return u;
    abcsmc_config cc = c;
    cc.batch = 0;
    const int rc = abcsmc_workspace_size(&cc, &dummy);
    if (rc) return bfail(e, rc, std::string("run config: ") + abcsmc_last_error(nullptr));
    if (!obs) return bfail(e, ABCSMC_EINVAL, "obs is NULL");
    for (int64_t t = 0; t <= c.n_days; ++t)
        for (int k = 0; k < 3; ++k)
            if (obs[t * 3 + k] < 0 || obs[t * 3 + k] > c.population)
                return bfail(e, ABCSMC_EINVAL, "observations must be counts in [0, P]");
    if (obs[0] + obs[1] + obs[2] > c.population) return bfail(e, ABCSMC_EINVAL, "A0 + R0 + D0 exceeds P");
    if (c.n_particles > ((int64_t)1 << 20)) return bfail(e, ABCSMC_EINVAL, "batched runs: N <= 2^20");
    return ABCSMC_OK;
}

}  // namespace

struct abcsmc_batch {
    int R = 0;
    std::vector<abcsmc_config> cfgs;
    std::vector<std::vector<int64_t>> obs;
    std::vector<RunLayout> lay;
    std::vector<BRun> runs;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    bool own_ws = false;
    size_t off_runs = 0, off_st = 0, off_g = 0, off_order = 0, off_res = 0, off_w = 0, off_fin = 0;
    int n_res = 0, max_w_blocks = 0, n_fin = 0, max_cap_chunks = 0;
    abcsmc_schedule sched{};
    BatchArgs args{};
    hipGraphExec_t exec[2] = {nullptr, nullptr};  // stage 0, later stages
    int stage = 0;
    bool broken = false;
    std::string err;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    std::vector<BState> hst;
};

namespace {

#define BCHK(b, expr)                                                                                  \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess) {                                                                        \
            (b)->broken = true;                                                                        \
            return bfail(&(b)->err, ABCSMC_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
        }                                                                                              \
    } while (0)

void default_schedule(abcsmc_schedule& s)
{
    s.propose_blocks = 0;
    s.run_order = 1;
    s.weight_cols = 4096;
    s.issue_margin = 1.1;
}

void drop_graphs(abcsmc_batch* b)
{
    for (auto& e : b->exec)
        if (e) {
            (void)hipGraphExecDestroy(e);
            e = nullptr;
        }
}

std::vector<int32_t> run_order(const abcsmc_batch* b, int mode)
{
    std::vector<int32_t> o(b->R);
    for (int r = 0; r < b->R; ++r) o[r] = r;
    auto work = [&](int r) { return (double)b->cfgs[r].n_particles * (double)b->cfgs[r].n_days; };
    if (mode >= 1) std::stable_sort(o.begin(), o.end(), [&](int x, int y) { return work(x) > work(y); });
    if (mode == 2) {  // largest, smallest, second largest, ...
        std::vector<int32_t> z;
        int lo = 0, hi = b->R - 1;
        while (lo <= hi) {
            z.push_back(o[lo++]);
            if (lo <= hi) z.push_back(o[hi--]);
        }
        o = z;
    }
    return o;
}

// (Re)build the schedule-dependent tables and descriptors and drop old graphs.
int apply_schedule(abcsmc_batch* b)
{
    drop_graphs(b);
    const abcsmc_schedule& s = b->sched;
    std::vector<int32_t> order = run_order(b, s.run_order);
    std::vector<int4> wt;
    for (int i = 0; i < b->R; ++i) {
        const int r = order[i];
        b->runs[r].wchunks = wchunks_for(b->cfgs[r].n_particles, s.weight_cols);
        const int rb = (int)((b->cfgs[r].n_particles + kWeightRows - 1) / kWeightRows);
        for (int y = 0; y < rb; ++y)
            for (int c = 0; c < b->runs[r].wchunks; ++c) wt.push_back(make_int4(r, y, c, 0));
    }
    if ((int)wt.size() > b->max_w_blocks) return bfail(&b->err, ABCSMC_EINVAL, "weight table overflow");
    BCHK(b, hipMemcpyAsync(b->ws + b->off_runs, b->runs.data(), b->runs.size() * sizeof(BRun), hipMemcpyHostToDevice,
                           b->stream));
    BCHK(b, hipMemcpyAsync(b->ws + b->off_order, order.data(), order.size() * 4, hipMemcpyHostToDevice, b->stream));
    BCHK(b, hipMemcpyAsync(b->ws + b->off_w, wt.data(), wt.size() * sizeof(int4), hipMemcpyHostToDevice, b->stream));
    BGlobal g{b->stage, b->R, s.issue_margin > 1.0 ? s.issue_margin : 1.0};
    BCHK(b, hipMemcpyAsync(b->ws + b->off_g, &g, sizeof g, hipMemcpyHostToDevice, b->stream));
    BCHK(b, hipStreamSynchronize(b->stream));
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    b->args.n_w_blocks = (int)wt.size();
    b->args.propose_blocks = s.propose_blocks > 0 ? s.propose_blocks : 2 * cus;
    b->args.g = reinterpret_cast<BGlobal*>(b->ws + b->off_g);
    return ABCSMC_OK;
}

int initial_states(abcsmc_batch* b)
{
    b->hst.assign(b->R, BState{});
    for (auto& st : b->hst) {
        st.eps = st.eps1 = st.eps_next = INFINITY;
        // acceptance-rate guess for stage 1 (no rate measured yet): its first
        // perturbations accept 0.8-0.9 of the proposals on the uneven batch;
        // 0.8 issued 2% fewer simulations and ran 1% faster than 0.5 (the
        // persistent kernel tops up a run that falls short)
        st.rate = 0.8;
    }
    BCHK(b, hipMemcpyAsync(b->ws + b->off_st, b->hst.data(), b->hst.size() * sizeof(BState), hipMemcpyHostToDevice,
                           b->stream));
    b->stage = 0;
    BGlobal g{0, b->R, b->sched.issue_margin > 1.0 ? b->sched.issue_margin : 1.0};
    BCHK(b, hipMemcpyAsync(b->ws + b->off_g, &g, sizeof g, hipMemcpyHostToDevice, b->stream));
    BCHK(b, hipStreamSynchronize(b->stream));
    return ABCSMC_OK;
}

int capture(abcsmc_batch* b, int which)
{
    hipGraph_t graph = nullptr;
    BCHK(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    batch_launch_stage(b->args, which == 0, b->stream);
    const hipError_t le = hipGetLastError();
    const hipError_t ce = hipStreamEndCapture(b->stream, &graph);
    BCHK(b, le);
    BCHK(b, ce);
    const hipError_t ie = hipGraphInstantiate(&b->exec[which], graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    BCHK(b, ie);
    return ABCSMC_OK;
}

std::string signature(const abcsmc_batch* b)
{
    uint64_t h = 1469598103934665603ull;  // FNV-1a over the run shapes
    auto mix = [&](uint64_t v) {
        for (int i = 0; i < 8; ++i) {
            h ^= (v >> (8 * i)) & 0xFF;
            h *= 1099511628211ull;
        }
    };
    for (const auto& c : b->cfgs) {
        mix((uint64_t)c.n_particles);
        mix((uint64_t)c.n_days);
        mix((uint64_t)c.population);
        mix((uint64_t)c.step_schedule);
    }
    char buf[32];
    snprintf(buf, sizeof buf, "%016llx", (unsigned long long)h);
    return std::string(buf) + "_" + std::to_string(b->R);
}

}  // namespace

extern "C" {

const char* abcsmc_batch_last_error(const abcsmc_batch* b) { return b ? b->err.c_str() : g_batch_err.c_str(); }

void abcsmc_batch_free(abcsmc_batch* b)
{
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    drop_graphs(b);
    if (b->ev0) (void)hipEventDestroy(b->ev0);
    if (b->ev1) (void)hipEventDestroy(b->ev1);
    if (b->own_ws && b->ws) (void)hipFree(b->ws);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

int abcsmc_batch_workspace_size(const abcsmc_config* cfgs, int32_t n_runs, size_t* bytes)
{
    if (!cfgs || n_runs < 1 || n_runs > 4096 || !bytes) return bfail(nullptr, ABCSMC_EINVAL, "bad batch arguments");
    size_t o = 0;
    int n_res = 0, n_w = 0, n_fin = 0;
    for (int r = 0; r < n_runs; ++r) {
        size_t dummy;
        abcsmc_config cc = cfgs[r];
        cc.batch = 0;
        const int rc = abcsmc_workspace_size(&cc, &dummy);
        if (rc) return rc;
        if (const int u = bunsupported(cfgs[r], nullptr)) return u;
        const RunLayout L = run_layout(cfgs[r], o);
        o = L.end;
        n_res += (int)((cfgs[r].n_particles + 1023) / 1024);
        n_fin += (int)((cfgs[r].n_particles + kWeightRows - 1) / kWeightRows);
        n_w += (int)((cfgs[r].n_particles + kWeightRows - 1) / kWeightRows) * wchunks_max(cfgs[r].n_particles);
    }
    o = al(o + (size_t)n_runs * sizeof(BRun));
    o = al(o + (size_t)n_runs * sizeof(BState));
    o = al(o + sizeof(BGlobal));
    o = al(o + (size_t)n_runs * 4);
    o = al(o + (size_t)n_res * sizeof(int2));
    o = al(o + (size_t)n_w * sizeof(int4));
    o = al(o + (size_t)n_fin * sizeof(int2));
    size_t n_total = 0;
    for (int r = 0; r < n_runs; ++r) n_total += (size_t)cfgs[r].n_particles;
    if (n_total > ((size_t)1 << 26)) return bfail(nullptr, ABCSMC_EINVAL, "batched runs: sum of N <= 2^26");
    o = win_layout(o, n_total, (size_t)n_fin).end;
    *bytes = o;
    return ABCSMC_OK;
}

int abcsmc_batch_init(const abcsmc_config* cfgs, int32_t n_runs, const int64_t* const* obs, abcsmc_batch** out)
{
    if (!out) return bfail(nullptr, ABCSMC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!cfgs || !obs || n_runs < 1 || n_runs > 4096) return bfail(nullptr, ABCSMC_EINVAL, "bad batch arguments");
    for (int r = 0; r < n_runs; ++r) {
        std::string e;
        const int rc = bvalidate(cfgs[r], obs[r], &e);
        if (rc) return bfail(nullptr, rc, "run " + std::to_string(r) + ": " + e);
    }
    size_t bytes = 0;
    int rc = abcsmc_batch_workspace_size(cfgs, n_runs, &bytes);
    if (rc) return rc;
    abcsmc_batch* b = new abcsmc_batch();
    b->R = n_runs;
    b->cfgs.assign(cfgs, cfgs + n_runs);
    for (auto& c : b->cfgs)
        if (c.max_attempts == 0) c.max_attempts = 256;
    auto bail = [&](int code, const std::string& m) {
        abcsmc_batch_free(b);
        return bfail(nullptr, code, m);
    };
    if (cfgs[0].stream) {
        b->stream = (hipStream_t)cfgs[0].stream;
    } else {
        if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess)
            return bail(ABCSMC_EDEVICE, "hipStreamCreate failed");
        b->own_stream = true;
    }
    if (cfgs[0].workspace) {
        if (cfgs[0].workspace_bytes < bytes) return bail(ABCSMC_ENOMEM, "workspace too small");
        if ((uintptr_t)cfgs[0].workspace % kAl) return bail(ABCSMC_EINVAL, "workspace must be 256-byte aligned");
        b->ws = (char*)cfgs[0].workspace;
    } else {
        if (hipMalloc((void**)&b->ws, bytes) != hipSuccess) {
            (void)hipGetLastError();
            b->ws = nullptr;
            return bail(ABCSMC_ENOMEM, "hipMalloc of the batch workspace failed");
        }
        b->own_ws = true;
    }
    b->ws_bytes = bytes;
    if (hipEventCreate(&b->ev0) != hipSuccess || hipEventCreate(&b->ev1) != hipSuccess)
        return bail(ABCSMC_EDEVICE, "hipEventCreate failed");
    // per-run regions and descriptors
    size_t o = 0, n_total = 0;
    std::vector<int2> res_tab, fin_tab;
    b->runs.resize(n_runs);
    for (int r = 0; r < n_runs; ++r) {
        const abcsmc_config& c = b->cfgs[r];
        const RunLayout L = run_layout(c, o);
        o = L.end;
        b->lay.push_back(L);
        BRun& R = b->runs[r];
        std::memset(&R, 0, sizeof R);
        for (int d = 0; d < kNP; ++d) {
            R.m.lo[d] = c.prior_lo[d];
            R.m.width[d] = c.prior_hi[d] - c.prior_lo[d];
        }
        R.m.P = (double)c.population;
        R.m.invP = 1.0 / R.m.P;
        R.m.A0 = (double)obs[r][0];
        R.m.R0 = (double)obs[r][1];
        R.m.D0 = (double)obs[r][2];
        R.m.T = c.n_days;
        R.m.sampler = c.sampler;
        R.m.seed = c.seed;
        char* w = b->ws;
        R.obs = (const double*)(w + L.obs);
        R.N = (int32_t)c.n_particles;
        R.cap_chunks = run_cap_chunks(c);
        R.step_schedule = c.step_schedule;
        R.beta_b_fixed = c.beta_b;
        R.beta_a_fixed = c.beta_a;
        R.step_is_variance = (c.flags & ABCSMC_F_STEP_IS_VARIANCE) ? 1 : 0;
        R.max_attempts = c.max_attempts;
        R.early_exit = (c.flags & ABCSMC_F_EARLY_EXIT) ? 1 : 0;
        R.surv_ratio = c.surv_ratio;
        for (int p = 0; p < 2; ++p) {
            R.u[p] = (double*)(w + L.u[p]);
            R.d[p] = (double*)(w + L.d[p]);
            R.sigma[p] = (double*)(w + L.sigma[p]);
            R.logw[p] = (double*)(w + L.logw[p]);
            R.W[p] = (double*)(w + L.W[p]);
            R.parent[p] = (int32_t*)(w + L.parent[p]);
            R.index[p] = (uint32_t*)(w + L.index[p]);
            R.att[p] = (int32_t*)(w + L.att[p]);
        }
        R.q = (uint64_t*)(w + L.q);
        R.cdf = (uint64_t*)(w + L.cdf);
        R.cols = (double*)(w + L.cols);
        R.wpart = (double*)(w + L.wpart);
        R.st_u = (double*)(w + L.st_u);
        R.st_d = (double*)(w + L.st_d);
        R.st_sigma = (double*)(w + L.st_sigma);
        R.st_parent = (int32_t*)(w + L.st_parent);
        R.st_att = (int32_t*)(w + L.st_att);
        R.wave_mask = (unsigned long long*)(w + L.wmask);
        R.wave_off = (uint32_t*)(w + L.woff);
        R.red_u = (unsigned long long*)(w + L.red_u);
        R.red_d = (double*)(w + L.red_d);
        R.off = (int32_t)n_total;
        R.rb0 = (int32_t)fin_tab.size();
        n_total += (size_t)c.n_particles;
        R.res_blk0 = (int32_t)res_tab.size();
        R.res_nblk = (int32_t)((c.n_particles + 1023) / 1024);
        for (int k = 0; k < R.res_nblk; ++k) res_tab.push_back(make_int2(r, k));
        const int rb = (int)((c.n_particles + kWeightRows - 1) / kWeightRows);
        for (int y = 0; y < rb; ++y) fin_tab.push_back(make_int2(r, y));
        b->max_w_blocks += rb * wchunks_max(c.n_particles);
        b->max_cap_chunks = std::max(b->max_cap_chunks, R.cap_chunks);
        std::vector<double> od(obs[r], obs[r] + (size_t)(c.n_days + 1) * 3);
        b->obs.emplace_back(obs[r], obs[r] + (size_t)(c.n_days + 1) * 3);
        if (hipMemcpy(w + L.obs, od.data(), od.size() * 8, hipMemcpyHostToDevice) != hipSuccess)
            return bail(ABCSMC_EDEVICE, "copy of observations failed");
    }
    b->off_runs = o;
    o = al(o + (size_t)n_runs * sizeof(BRun));
    b->off_st = o;
    o = al(o + (size_t)n_runs * sizeof(BState));
    b->off_g = o;
    o = al(o + sizeof(BGlobal));
    b->off_order = o;
    o = al(o + (size_t)n_runs * 4);
    b->off_res = o;
    o = al(o + res_tab.size() * sizeof(int2));
    b->off_w = o;
    o = al(o + (size_t)b->max_w_blocks * sizeof(int4));
    b->off_fin = o;
    o = al(o + fin_tab.size() * sizeof(int2));
    const WinLayout WL = win_layout(o, n_total, fin_tab.size());
    o = WL.end;
    if (o > bytes) return bail(ABCSMC_EINVAL, "internal layout mismatch");
    if (hipMemcpy(b->ws + b->off_res, res_tab.data(), res_tab.size() * sizeof(int2), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->ws + b->off_fin, fin_tab.data(), fin_tab.size() * sizeof(int2), hipMemcpyHostToDevice) != hipSuccess)
        return bail(ABCSMC_EDEVICE, "copy of work tables failed");
    b->n_res = (int)res_tab.size();
    b->n_fin = (int)fin_tab.size();
    BatchArgs& A = b->args;
    A.runs = (const BRun*)(b->ws + b->off_runs);
    A.st = (BState*)(b->ws + b->off_st);
    A.g = (BGlobal*)(b->ws + b->off_g);
    A.order = (const int32_t*)(b->ws + b->off_order);
    A.res_tab = (const int2*)(b->ws + b->off_res);
    A.w_tab = (const int4*)(b->ws + b->off_w);
    A.fin_tab = (const int2*)(b->ws + b->off_fin);
    A.n_runs = n_runs;
    A.max_cap_chunks = b->max_cap_chunks;
    A.n_res_blocks = b->n_res;
    A.n_fin_blocks = b->n_fin;
    A.colkeys = (unsigned long long*)(b->ws + WL.colkeys);
    A.rowkeys = (unsigned long long*)(b->ws + WL.rowkeys);
    A.scols = (double*)(b->ws + WL.scols);
    A.skey = (double*)(b->ws + WL.skey);
    A.rwin = (double*)(b->ws + WL.rwin);
    A.win = (int2*)(b->ws + WL.win);
    A.wtab = (const double*)(b->ws + WL.wtab);
    launch_weight_table((double*)(b->ws + WL.wtab), b->stream);
    if (hipGetLastError() != hipSuccess) return bail(ABCSMC_EDEVICE, "launch of the exponential table failed");
    A.npad = WL.npad;
    A.n_total = (int32_t)n_total;
    A.n_key_blocks = (int32_t)((WL.npad + kBlock - 1) / kBlock);
    weight_exp_constants(A.ex);
    default_schedule(b->sched);
    if ((rc = apply_schedule(b)) || (rc = initial_states(b))) {
        const std::string m = b->err;
        return bail(rc, m);
    }
    *out = b;
    return ABCSMC_OK;
}

int abcsmc_batch_set_schedule(abcsmc_batch* b, const abcsmc_schedule* s)
{
    if (!b || !s) return bfail(nullptr, ABCSMC_EINVAL, "NULL argument");
    if (b->broken) return bfail(&b->err, ABCSMC_ESTATE, "batch unusable after a device error");
    if (s->propose_blocks < 0 || s->propose_blocks > 65536 || s->run_order < 0 || s->run_order > 2 ||
        (s->weight_cols != 0 && (s->weight_cols < 256 || s->weight_cols > (1 << 20))) ||
        (s->issue_margin != 0.0 && !(s->issue_margin >= 1.0 && s->issue_margin <= 8.0)))
        return bfail(&b->err, ABCSMC_EINVAL, "schedule out of range");
    b->sched = *s;
    if (b->sched.weight_cols == 0) b->sched.weight_cols = 4096;
    if (b->sched.issue_margin == 0.0) b->sched.issue_margin = 1.1;
    return apply_schedule(b);
}

int abcsmc_batch_get_schedule(const abcsmc_batch* b, abcsmc_schedule* s)
{
    if (!b || !s) return bfail(nullptr, ABCSMC_EINVAL, "NULL argument");
    *s = b->sched;
    return ABCSMC_OK;
}

int abcsmc_batch_reset(abcsmc_batch* b)
{
    if (!b) return bfail(nullptr, ABCSMC_EINVAL, "batch is NULL");
    if (b->broken) return bfail(&b->err, ABCSMC_ESTATE, "batch unusable after a device error");
    return initial_states(b);
}

int abcsmc_batch_round(abcsmc_batch* b, abcsmc_round_info* infos)
{
    if (!b) return bfail(nullptr, ABCSMC_EINVAL, "batch is NULL");
    if (b->broken) return bfail(&b->err, ABCSMC_ESTATE, "batch unusable after a device error");
    const int which = b->stage == 0 ? 0 : 1;
    for (int r = 0; r < b->R; ++r)
        if (b->cfgs[r].step_schedule == ABCSMC_STEP_PAPER && 2 * b->stage > 128)
            return bfail(&b->err, ABCSMC_EINVAL, "eq. 16 schedule limited to 64 stages");
    if (!b->exec[which]) {
        const int rc = capture(b, which);
        if (rc) return rc;
    }
    BCHK(b, hipEventRecord(b->ev0, b->stream));
    BCHK(b, hipGraphLaunch(b->exec[which], b->stream));
    BCHK(b, hipEventRecord(b->ev1, b->stream));
    BCHK(b, hipMemcpyAsync(b->hst.data(), b->ws + b->off_st, b->hst.size() * sizeof(BState), hipMemcpyDeviceToHost,
                           b->stream));
    BCHK(b, hipStreamSynchronize(b->stream));
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, b->ev0, b->ev1);
    const int stage = b->stage;
    b->stage += 1;
    if (infos) {
        for (int r = 0; r < b->R; ++r) {
            const BState& S = b->hst[r];
            abcsmc_round_info& I = infos[r];
            std::memset(&I, 0, sizeof I);
            I.round = stage;
            I.eps = S.eps;
            I.eps_next = S.eps_next;
            I.beta_a = S.beta_a;
            I.beta_b = S.beta_b;
            I.ess = S.ess;
            I.proposals = (int64_t)S.proposals;
            const unsigned long long cap = (unsigned long long)b->runs[r].cap_chunks;
            I.simulated = (int64_t)std::min<unsigned long long>(S.issued, cap) * kChunkP;
            I.invalid = (int64_t)S.invalid;
            I.attempts = (int64_t)S.attempts;
            I.survivors = (int64_t)S.survivors;
            I.batches = 1;
            I.ms_total = ms;
            I.sim_days = (int64_t)S.days;
            I.weight_pairs = stage == 0 ? 0 : (int64_t)b->cfgs[r].n_particles * (int64_t)S.survivors;
            I.weight_terms = (int64_t)S.terms;
            I.weight_window_terms = (int64_t)S.window_terms;
        }
    }
    return ABCSMC_OK;
}

int abcsmc_batch_status(const abcsmc_batch* b, int32_t run)
{
    if (!b || run < 0 || run >= b->R) return ABCSMC_EINVAL;
    return b->hst[run].failed ? ABCSMC_EBUDGET : ABCSMC_OK;
}

int abcsmc_batch_rounds_done(const abcsmc_batch* b, int32_t run)
{
    if (!b || run < 0 || run >= b->R) return ABCSMC_EINVAL;
    return (int)b->hst[run].stages_done;
}

int abcsmc_batch_run(abcsmc_batch* b, int32_t n_rounds, abcsmc_round_info* infos)
{
    if (!b || n_rounds < 1) return bfail(nullptr, ABCSMC_EINVAL, "bad arguments");
    for (int i = 0; i < n_rounds; ++i) {
        const int rc = abcsmc_batch_round(b, infos ? infos + (size_t)i * b->R : nullptr);
        if (rc) return rc;
    }
    return ABCSMC_OK;
}

int abcsmc_batch_population(const abcsmc_batch* b, int32_t run, double* u, double* sigma, int64_t* parent,
                            int64_t* index, int32_t* attempts, double* logw, double* dist, double* weight)
{
    if (!b || run < 0 || run >= b->R) return bfail(nullptr, ABCSMC_EINVAL, "bad arguments");
    abcsmc_batch* x = const_cast<abcsmc_batch*>(b);
    if (x->broken) return bfail(&x->err, ABCSMC_ESTATE, "batch unusable after a device error");
    if (x->hst[run].stages_done == 0) return bfail(&x->err, ABCSMC_ESTATE, "run has no completed stage");
    const BRun& R = x->runs[run];
    const int c = x->hst[run].cur;
    const size_t N = (size_t)R.N;
    hipStream_t s = x->stream;
    std::vector<int32_t> pi(parent ? N : 0);
    std::vector<uint32_t> ii(index ? N : 0);
    if (u) BCHK(x, hipMemcpyAsync(u, R.u[c], N * kNP * 8, hipMemcpyDeviceToHost, s));
    if (sigma) BCHK(x, hipMemcpyAsync(sigma, R.sigma[c], N * 8, hipMemcpyDeviceToHost, s));
    if (parent) BCHK(x, hipMemcpyAsync(pi.data(), R.parent[c], N * 4, hipMemcpyDeviceToHost, s));
    if (index) BCHK(x, hipMemcpyAsync(ii.data(), R.index[c], N * 4, hipMemcpyDeviceToHost, s));
    if (attempts) BCHK(x, hipMemcpyAsync(attempts, R.att[c], N * 4, hipMemcpyDeviceToHost, s));
    if (logw) BCHK(x, hipMemcpyAsync(logw, R.logw[c], N * 8, hipMemcpyDeviceToHost, s));
    if (dist) BCHK(x, hipMemcpyAsync(dist, R.d[c], N * 8, hipMemcpyDeviceToHost, s));
    if (weight) BCHK(x, hipMemcpyAsync(weight, R.W[c], N * 8, hipMemcpyDeviceToHost, s));
    BCHK(x, hipStreamSynchronize(s));
    for (size_t k = 0; k < pi.size(); ++k) parent[k] = pi[k];
    for (size_t k = 0; k < ii.size(); ++k) index[k] = ii[k];
    return ABCSMC_OK;
}

int abcsmc_batch_autotune(abcsmc_batch* b, int32_t stages, const char* cache_path, abcsmc_schedule* chosen)
{
    if (!b || stages < 0 || stages > 16) return bfail(nullptr, ABCSMC_EINVAL, "bad arguments");
    if (b->broken) return bfail(&b->err, ABCSMC_ESTATE, "batch unusable after a device error");
    const std::string key = signature(b);
    if (cache_path) {
        std::ifstream in(cache_path);
        std::string line;
        while (std::getline(in, line)) {
            std::istringstream ss(line);
            std::string k;
            abcsmc_schedule s{};
            double ms;
            if (ss >> k >> s.propose_blocks >> s.run_order >> s.weight_cols >> s.issue_margin >> ms && k == key) {
                int rc = abcsmc_batch_set_schedule(b, &s);
                if (!rc) rc = abcsmc_batch_reset(b);
                if (!rc && chosen) *chosen = b->sched;
                return rc;
            }
        }
    }
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    auto measure = [&](const abcsmc_schedule& s, double* ms) -> int {
        int rc = abcsmc_batch_set_schedule(b, &s);
        if (!rc) rc = abcsmc_batch_reset(b);
        if (rc) return rc;
        hipEvent_t e0, e1;
        BCHK(b, hipEventCreate(&e0));
        BCHK(b, hipEventCreate(&e1));
        BCHK(b, hipEventRecord(e0, b->stream));
        rc = abcsmc_batch_run(b, 1 + stages, nullptr);
        if (!rc) {
            BCHK(b, hipEventRecord(e1, b->stream));
            BCHK(b, hipEventSynchronize(e1));
            float f = 0.f;
            (void)hipEventElapsedTime(&f, e0, e1);
            *ms = f;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return rc;
    };
    // coordinate descent, one knob at a time
    abcsmc_schedule best = b->sched;
    double best_ms = 0.0;
    int rc = measure(best, &best_ms);
    if (rc) return rc;
    const int pb[] = {cus, 2 * cus, 4 * cus, 8 * cus};
    const int ro[] = {0, 1, 2};
    const int wc[] = {2048, 4096, 8192};
    const double mg[] = {1.05, 1.1, 1.3};
    for (int knob = 0; knob < 4; ++knob) {
        const int n = knob == 0 ? 4 : 3;
        for (int i = 0; i < n; ++i) {
            abcsmc_schedule s = best;
            if (knob == 0) s.propose_blocks = pb[i];
            if (knob == 1) s.run_order = ro[i];
            if (knob == 2) s.weight_cols = wc[i];
            if (knob == 3) s.issue_margin = mg[i];
            double ms = 0.0;
            if ((rc = measure(s, &ms))) return rc;
            if (ms < best_ms) {
                best_ms = ms;
                best = s;
            }
        }
    }
    rc = abcsmc_batch_set_schedule(b, &best);
    if (!rc) rc = abcsmc_batch_reset(b);
    if (rc) return rc;
    if (cache_path) {
        std::ofstream outf(cache_path, std::ios::app);
        outf << key << ' ' << best.propose_blocks << ' ' << best.run_order << ' ' << best.weight_cols << ' '
             << best.issue_margin << ' ' << best_ms << '\n';
    }
    if (chosen) *chosen = best;
    return ABCSMC_OK;
}

}  // extern "C"
