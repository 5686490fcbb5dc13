// checkpoint.hip -- abcsmc_snapshot / abcsmc_restore: the host-side copy of
// what the next stage reads from the last completed one, so that a run can
// stop after any stage and continue later, bit for bit.
#include <hip/hip_runtime.h>

#include <cstring>
#include <string>
#include <vector>

#include "abcsmc.h"
#include "ctx.h"

using namespace abcsmc;
using namespace abcsmc::rt;

namespace {

constexpr char kMagic[8] = {'A', 'B', 'C', 'S', 'M', 'C', 'K', '1'};

struct SnapHeader {
    char magic[8];
    uint32_t abi;
    int32_t rounds;         // stages completed (>= 1)
    uint64_t fingerprint;   // configuration and observations
    int64_t N;
    double eps_next;        // eq. 8 percentile of the last stage
    double eps1;            // eps of stage 1 (eq. 16)
    double last_rate;       // acceptance rate of the last stage (batch sizing only)
    double mcmc_s;          // MCMC variant state
    int64_t mcmc_nacc;
    int32_t mcmc_tunes;
    int32_t reserved;
};

// Population arrays in snapshot order: f64 u (N x 8), d, sigma, logw, W;
// then i32 parent, u32 index, i32 attempts.
size_t snapshot_bytes(int64_t N)
{
    return sizeof(SnapHeader) + (size_t)N * (kNP + 4) * sizeof(double) + (size_t)N * 3 * sizeof(int32_t);
}

struct Fnv {
    uint64_t h = 1469598103934665603ull;
    void bytes(const void* p, size_t n)
    {
        const unsigned char* c = (const unsigned char*)p;
        for (size_t i = 0; i < n; ++i) {
            h ^= c[i];
            h *= 1099511628211ull;
        }
    }
    template <typename T>
    void val(const T& v) { bytes(&v, sizeof v); }
};

// Everything the trajectories of later stages depend on: the model, the
// priors, the samplers and schedules, the seed, the budget and the
// observations (field by field: struct padding is not hashed).  The batch
// size enters only where results depend on it (the MCMC variant).
uint64_t fingerprint(const abcsmc_ctx* x)
{
    const abcsmc_config& c = x->cfg;
    Fnv f;
    f.val(c.n_params);
    for (int d = 0; d < ABCSMC_NPAR; ++d) {
        f.val(c.prior_lo[d]);
        f.val(c.prior_hi[d]);
    }
    f.val(c.population);
    f.val(c.n_days);
    f.val(c.n_particles);
    f.val(c.surv_ratio);
    f.val(c.step_schedule);
    f.val(c.beta_a);
    f.val(c.beta_b);
    f.val(c.sampler);
    f.val(c.flags);
    f.val(c.max_attempts);
    f.val(c.seed);
    f.val(c.max_proposals);
    f.val(c.mcmc_s0);
    f.val(c.mcmc_tune);
    if (c.step_schedule == ABCSMC_STEP_MCMC) f.val(c.batch);
    f.val(c.n_eps_schedule);
    for (double e : x->eps_sched) f.val(e);
    for (int64_t o : x->obs) f.val(o);
    return f.h;
}

}  // namespace

extern "C" {

int abcsmc_snapshot(const abcsmc_ctx* cx, void* buf, size_t* bytes)
{
    abcsmc_ctx* x = const_cast<abcsmc_ctx*>(cx);
    if (!x) return fail(nullptr, ABCSMC_EINVAL, "ctx is NULL");
    if (!bytes) return fail(&x->err, ABCSMC_EINVAL, "bytes is NULL");
    if (x->broken) return fail(&x->err, ABCSMC_ESTATE, "context unusable after a device error");
    if (x->rounds == 0) return fail(&x->err, ABCSMC_ESTATE, "no completed stage");
    if (x->sur) return fail(&x->err, ABCSMC_ESTATE, "snapshots of a context with the learned screen are not supported");
    const size_t need = snapshot_bytes(x->N);
    if (!buf) {
        *bytes = need;
        return ABCSMC_OK;
    }
    if (*bytes < need) return fail(&x->err, ABCSMC_EINVAL, "snapshot buffer too small");
    SnapHeader h{};
    std::memcpy(h.magic, kMagic, sizeof kMagic);
    h.abi = ABCSMC_ABI_VERSION;
    h.rounds = x->rounds;
    h.fingerprint = fingerprint(x);
    h.N = x->N;
    h.eps_next = x->eps_next;
    h.eps1 = x->eps1;
    h.last_rate = x->last_rate;
    h.mcmc_s = x->mcmc_s;
    h.mcmc_nacc = x->mcmc_nacc;
    h.mcmc_tunes = x->mcmc_tunes;
    char* o = (char*)buf;
    std::memcpy(o, &h, sizeof h);
    o += sizeof h;
    const size_t N = (size_t)x->N;
    const DevPop& p = x->pop[x->cur];
    hipStream_t s = x->stream;
    const void* src[8] = {p.u, p.d, p.sigma, p.logw, p.W, p.parent, p.index, p.att};
    const size_t len[8] = {N * kNP * 8, N * 8, N * 8, N * 8, N * 8, N * 4, N * 4, N * 4};
    for (int k = 0; k < 8; ++k) {
        HIPCHK(x, hipMemcpyAsync(o, src[k], len[k], hipMemcpyDeviceToHost, s));
        o += len[k];
    }
    HIPCHK(x, hipStreamSynchronize(s));
    *bytes = need;
    return ABCSMC_OK;
}

int abcsmc_restore(const abcsmc_config* cfg, const int64_t* obs, const void* buf, size_t bytes, abcsmc_ctx** out)
{
    if (!out) return fail(nullptr, ABCSMC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!buf || bytes < sizeof(SnapHeader)) return fail(nullptr, ABCSMC_EINVAL, "snapshot buffer too short");
    SnapHeader h;
    std::memcpy(&h, buf, sizeof h);
    if (std::memcmp(h.magic, kMagic, sizeof kMagic) != 0 || h.abi != ABCSMC_ABI_VERSION)
        return fail(nullptr, ABCSMC_EINVAL, "not a snapshot of this library version");
    if (h.rounds < 1 || h.N < 2 || h.N > ((int64_t)1 << 22) || bytes != snapshot_bytes(h.N))
        return fail(nullptr, ABCSMC_EINVAL, "malformed snapshot");
    abcsmc_ctx* x = nullptr;
    int rc = abcsmc_init(cfg, obs, &x);
    if (rc) return rc;
    auto bail = [&](int code, const std::string& msg) {
        abcsmc_free(x);
        return fail(nullptr, code, msg);
    };
    if (h.N != x->N || h.fingerprint != fingerprint(x))
        return bail(ABCSMC_EINVAL, "snapshot was taken under another configuration or other observations");
    const char* in = (const char*)buf + sizeof h;
    const size_t N = (size_t)x->N;
    const DevPop& p = x->pop[0];
    void* dst[8] = {p.u, p.d, p.sigma, p.logw, p.W, p.parent, p.index, p.att};
    const size_t len[8] = {N * kNP * 8, N * 8, N * 8, N * 8, N * 8, N * 4, N * 4, N * 4};
    for (int k = 0; k < 8; ++k) {
        if (hipMemcpyAsync(dst[k], in, len[k], hipMemcpyHostToDevice, x->stream) != hipSuccess)
            return bail(ABCSMC_EDEVICE, "copy of the snapshot to the device failed");
        in += len[k];
    }
    if (hipStreamSynchronize(x->stream) != hipSuccess) return bail(ABCSMC_EDEVICE, "copy of the snapshot failed");
    x->cur = 0;
    x->rounds = h.rounds;
    x->eps_next = h.eps_next;
    x->eps1 = h.eps1;
    x->last_rate = h.last_rate;
    x->mcmc_s = h.mcmc_s;
    x->mcmc_nacc = h.mcmc_nacc;
    x->mcmc_tunes = h.mcmc_tunes;
    *out = x;
    return ABCSMC_OK;
}

}  // extern "C"
