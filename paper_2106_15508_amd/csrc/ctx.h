// ctx.h -- host-side state of a single-run context (shared by the stage
// loop and the surrogate-screened stage).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "abcsmc.h"
#include "kernels.h"

namespace abcsmc {
namespace rt {

inline thread_local std::string g_last_error;

struct DevPop {
    double* u;
    double* d;
    double* sigma;
    int32_t* parent;
    uint32_t* index;
    int32_t* att;
    double* logw;
    double* W;
    Population view() const { return Population{u, d, sigma, parent, index, att, logw, W}; }
};

// Byte layout of the device workspace (every region 256-byte aligned).
struct Layout {
    size_t obs, pop[2][8], q, cdf, cols, st_u, st_d, st_sigma, st_parent, st_att, wave_mask, wave_off,
        ctr, scal, theta, red[5], hist, sel, wpart, rowkeys, colkeys, scols, skey, dimpart, dstar, win, rwin, wtab, total;
};

inline int fail(std::string* where, int code, const std::string& msg)
{
    if (where) *where = msg;
    g_last_error = msg;
    return code;
}

inline float elapsed(hipEvent_t a, hipEvent_t b)
{
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.f;
    return ms;
}

struct Surrogate;

}  // namespace rt
}  // namespace abcsmc

struct abcsmc_ctx;

namespace abcsmc {
namespace rt {

// Surrogate-screened stages (surrogate_rt.hip).
void surrogate_free(Surrogate* S);
bool surrogate_screens(const abcsmc_ctx* x, int32_t round);
int surrogate_stage_begin(abcsmc_ctx* x, int nxt);
int surrogate_batches(abcsmc_ctx* x, const ProposeArgs& pa, const DevPop& dst, int nxt, StageCounters& hc,
                      int64_t& base, int64_t& batches, double& ms_k);
int surrogate_weights(abcsmc_ctx* x, const DevPop& dst, int nxt);
int surrogate_stage_end(abcsmc_ctx* x, int32_t round);
int surrogate_reset(abcsmc_ctx* x);

}  // namespace rt
}  // namespace abcsmc

#define HIPCHK(ctx, expr)                                                                  \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess) {                                                            \
            (ctx)->broken = true;                                                          \
            return fail(&(ctx)->err, ABCSMC_EDEVICE,                                       \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                \
        }                                                                                  \
    } while (0)

struct abcsmc_ctx {
    abcsmc::rt::Surrogate* sur = nullptr;  // learned screen, or null
    abcsmc_config cfg{};
    abcsmc::Model model{};
    abcsmc::rt::Layout L{};
    std::vector<int64_t> obs;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    char* ws = nullptr;
    bool own_ws = false;
    bool broken = false;
    std::string err;
    hipEvent_t ev[9] = {};
    abcsmc::rt::DevPop pop[2]{};
    int cur = 0;                 // pop[cur] holds the last completed stage
    int32_t rounds = 0;          // stages completed
    double eps_next = INFINITY;  // eps of the next stage
    double eps1 = INFINITY;      // eps of stage 1 (eq. 16 normaliser)
    std::vector<double> eps_sched;  // replayed tolerances of stages 1.. (cfg.eps_schedule points here)
    char* stage_host = nullptr;  // pinned staging for the copy-out calls (allocated on first use)
    size_t stage_bytes = 0;
    double last_rate = 0.5;      // acceptance rate of the last stage (batch sizing)
    int64_t first_batch = 0;     // largest first batch of stage 1 (no measured rate yet)
    double mcmc_s = 0.0;         // MCMC variant: current step size
    int32_t mcmc_tunes = 0;      // MCMC variant: tuned batches so far
    int64_t mcmc_nacc = 0;       // MCMC variant: acceptances of the tuned batches
    int64_t N = 0;
    template <typename T>
    T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
    abcsmc::Scratch scratch() const
    {
        return abcsmc::Scratch{at<unsigned long long>(L.red[0]), at<unsigned long long>(L.red[1]),
                       at<unsigned long long>(L.red[2]), at<double>(L.red[3]), at<double>(L.red[4]),
                       at<unsigned int>(L.hist), at<unsigned long long>(L.sel)};
    }
};

