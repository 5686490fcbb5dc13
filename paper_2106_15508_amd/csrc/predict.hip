// predict.hip -- posterior predictive simulation (§IV-B, Fig. 7): the
// particles of a completed stage simulated over a longer horizon, and per
// day the type-7 quantiles of A, R and D over the particles.
#include "blockselect.h"
#include "kernels.h"
#include "predict.h"
#include "propose.h"

namespace abcsmc {

namespace {

// Lane per particle j: theta = lo + u width, trajectory of the stream
// (seed, j, round) written as series[(3 t + c) N + j].
template <int kSampler>
__global__ __launch_bounds__(kBlock) void predict_series_kernel(PredictArgs a)
{
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= a.n) return;
    double th[kNP];
#pragma unroll
    for (int q = 0; q < kNP; ++q) th[q] = a.m.lo[q] + a.u[j * kNP + q] * a.m.width[q];
    int32_t days = 0;
    lane::simulate_distance<kSampler, true>(a.m, th, nullptr, a.round, (uint32_t)j, __builtin_inf(), nullptr, days,
                                            nullptr, a.series + j, a.n);
}

// One block per (day, series) row: its n_quant quantiles.
__global__ __launch_bounds__(kBlock) void predict_band_kernel(PredictArgs a)
{
    __shared__ bsel::Shared sh;
    const int64_t row = blockIdx.x;  // 3 t + c
    const double* x = a.series + (size_t)row * a.n;
    for (int k = 0; k < a.n_quant; ++k) {
        const double v = bsel::quantile7(x, a.n, 1, a.quant[k], sh);
        if (threadIdx.x == 0) a.bands[row * a.n_quant + k] = v;
    }
}

}  // namespace

void launch_predict(const PredictArgs& a, hipStream_t s)
{
    const dim3 grid((unsigned)((a.n + kBlock - 1) / kBlock));
    if (a.m.sampler == 0)
        hipLaunchKernelGGL((predict_series_kernel<0>), grid, dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL((predict_series_kernel<1>), grid, dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(predict_band_kernel, dim3((unsigned)(3 * (a.m.T + 1))), dim3(kBlock), 0, s, a);
}

}  // namespace abcsmc
