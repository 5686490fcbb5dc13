// peak.hip -- what the device sustains, as context for the roofline
// fractions (the fractions themselves are taken against the published
// peaks): FP64 vector FMA throughput with the shader clock it ran at, and
// device-to-device copy bandwidth.  Not part of the method.
#include <hip/hip_runtime.h>

#include <string>

#include "abcsmc.h"
#include "ctx.h"

namespace abcsmc {

namespace {

constexpr int kPeakBlock = 256;
constexpr int kChains = 8;    // independent FMA chains per lane
constexpr int kUnroll = 16;   // FMAs per chain per loop step

// kChains independent chains a <- a b + c per lane (b < 1: each chain
// approaches c / (1 - b), so values stay finite); lane 0 of block 0 also
// reads the shader-clock counter and the constant 100 MHz counter at both
// ends, which gives the clock the FMAs ran at.
__global__ __launch_bounds__(kPeakBlock) void peak_fp64_kernel(double* out, unsigned long long* clk, int iters,
                                                               double b, double c)
{
    const int64_t g = (int64_t)blockIdx.x * kPeakBlock + threadIdx.x;
    const bool timer = g == 0;
    unsigned long long c0 = 0, r0 = 0;
    if (timer) {
        c0 = __builtin_readcyclecounter();
        r0 = __builtin_amdgcn_s_memrealtime();
    }
    double a[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) a[k] = 1e-3 * (double)(threadIdx.x + k);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
#pragma unroll
            for (int k = 0; k < kChains; ++k) a[k] = __builtin_fma(a[k], b, c);
        }
    }
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kChains; ++k) s += a[k];
    out[g] = s;
    if (timer) {
        const unsigned long long c1 = __builtin_readcyclecounter();
        const unsigned long long r1 = __builtin_amdgcn_s_memrealtime();
        clk[0] = c1 - c0;
        clk[1] = r1 - r0;
    }
}

// Grid-stride copy in 16-byte elements.  Launched with about two elements
// per lane: on gfx950 a large grid of short-lived waves copied 6.1 TB/s,
// against 4.3-4.8 TB/s for 8-32 workgroups per compute unit looping over
// the buffer (with or without four loads in flight per lane).
__global__ __launch_bounds__(kPeakBlock) void peak_copy_kernel(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                               int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * kPeakBlock;
    for (int64_t i = (int64_t)blockIdx.x * kPeakBlock + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

}  // namespace

}  // namespace abcsmc

extern "C" {

int abcsmc_measure_peaks(int32_t repeats, double* fp64_tflops, double* clock_mhz, double* copy_gbs)
{
    using namespace abcsmc;
    using rt::fail;
    if (repeats < 1 || repeats > 100 || !fp64_tflops || !clock_mhz || !copy_gbs)
        return fail(nullptr, ABCSMC_EINVAL, "measure_peaks: repeats in [1, 100] and three outputs");
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        return fail(nullptr, ABCSMC_EDEVICE, "measure_peaks: no device");
    }
    // eight waves per SIMD on every compute unit
    const int blocks = cus * 4 * 8 * 64 / kPeakBlock;
    const int iters = 4096;
    const int64_t threads = (int64_t)blocks * kPeakBlock;
    const size_t copy_bytes = (size_t)1 << 30;  // 1 GiB each way: beyond the last-level cache
    double* out = nullptr;
    unsigned long long* clk = nullptr;
    void *src = nullptr, *dst = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto release = [&]() {
        if (out) (void)hipFree(out);
        if (clk) (void)hipFree(clk);
        if (src) (void)hipFree(src);
        if (dst) (void)hipFree(dst);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
    if (hipMalloc((void**)&out, threads * sizeof(double)) != hipSuccess ||
        hipMalloc((void**)&clk, 2 * sizeof(unsigned long long)) != hipSuccess ||
        hipMalloc(&src, copy_bytes) != hipSuccess || hipMalloc(&dst, copy_bytes) != hipSuccess) {
        (void)hipGetLastError();
        release();
        return fail(nullptr, ABCSMC_ENOMEM, "measure_peaks: hipMalloc failed");
    }
    hipError_t err = hipEventCreate(&e0);
    if (err == hipSuccess) err = hipEventCreate(&e1);
    if (err == hipSuccess) err = hipMemset(src, 0, copy_bytes);
    double best_fp64 = 0.0, mhz = 0.0, best_copy = 0.0;
    const double flops = (double)threads * iters * kUnroll * kChains * 2.0;
    for (int r = 0; r <= repeats && err == hipSuccess; ++r) {  // launch 0 is a warm-up
        err = hipEventRecord(e0, nullptr);
        if (err == hipSuccess) {
            hipLaunchKernelGGL(peak_fp64_kernel, dim3(blocks), dim3(kPeakBlock), 0, nullptr, out, clk, iters,
                               1.0 - 0x1p-20, 0x1p-20);
            err = hipGetLastError();
        }
        if (err == hipSuccess) err = hipEventRecord(e1, nullptr);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float ms = 0.f;
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        unsigned long long hc[2] = {0, 0};
        if (err == hipSuccess) err = hipMemcpy(hc, clk, sizeof hc, hipMemcpyDeviceToHost);
        if (err == hipSuccess && r > 0 && ms > 0.f) {
            const double tf = flops / (ms * 1e-3) / 1e12;
            if (tf > best_fp64) {
                best_fp64 = tf;
                mhz = hc[1] ? 100.0 * (double)hc[0] / (double)hc[1] : 0.0;
            }
        }
    }
    const int64_t n16 = (int64_t)(copy_bytes / 16);
    const int cblocks = cus * 512;
    for (int r = 0; r <= repeats && err == hipSuccess; ++r) {  // launch 0 is a warm-up
        err = hipEventRecord(e0, nullptr);
        if (err == hipSuccess) {
            hipLaunchKernelGGL(peak_copy_kernel, dim3(cblocks), dim3(kPeakBlock), 0, nullptr, (const uint4*)src,
                               (uint4*)dst, n16);
            err = hipGetLastError();
        }
        if (err == hipSuccess) err = hipEventRecord(e1, nullptr);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float ms = 0.f;
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        if (err == hipSuccess && r > 0 && ms > 0.f) {
            const double gbs = 2.0 * (double)copy_bytes / (ms * 1e-3) / 1e9;
            if (gbs > best_copy) best_copy = gbs;
        }
    }
    release();
    if (err != hipSuccess) return fail(nullptr, ABCSMC_EDEVICE, std::string("measure_peaks: ") + hipGetErrorString(err));
    *fp64_tflops = best_fp64;
    *clock_mhz = mhz;
    *copy_gbs = best_copy;
    return ABCSMC_OK;
}

}  // extern "C"
