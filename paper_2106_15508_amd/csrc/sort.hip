// sort.hip -- ascending bitonic sort of 64-bit keys in place (power-of-two
// length, pad with UINT64_MAX).  Callers make keys unique (payload index in
// the low bits), so the order is fully determined.  Strides below 2048 run
// inside LDS; larger strides are one compare-exchange per thread per launch.
#include "kernels.h"

namespace abcsmc {

namespace {

constexpr int kSortThreads = 1024;
constexpr int kSortTile = 2 * kSortThreads;  // keys per LDS tile

__device__ __forceinline__ void cmpx(unsigned long long& a, unsigned long long& b, bool up)
{
    if ((a > b) == up) {
        const unsigned long long t = a;
        a = b;
        b = t;
    }
}

// Every bitonic stage up to the tile size (k = 2 .. 2048), directions taken
// from the global index so tiles combine into the global network.
__global__ __launch_bounds__(kSortThreads) void bitonic_tile_kernel(unsigned long long* keys)
{
    __shared__ unsigned long long s[kSortTile];
    const size_t base = (size_t)blockIdx.x * kSortTile;
    s[threadIdx.x] = keys[base + threadIdx.x];
    s[threadIdx.x + kSortThreads] = keys[base + threadIdx.x + kSortThreads];
    __syncthreads();
    for (int k = 2; k <= kSortTile; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            const int t = threadIdx.x;
            const int i = (t / j) * 2 * j + (t % j);
            const bool up = (((base + (size_t)i) & (size_t)k) == 0);
            cmpx(s[i], s[i + j], up);
            __syncthreads();
        }
    }
    keys[base + threadIdx.x] = s[threadIdx.x];
    keys[base + threadIdx.x + kSortThreads] = s[threadIdx.x + kSortThreads];
}

// Strides j < 2048 of stage k (k > 2048) inside LDS.
__global__ __launch_bounds__(kSortThreads) void bitonic_merge_tile_kernel(unsigned long long* keys, size_t k)
{
    __shared__ unsigned long long s[kSortTile];
    const size_t base = (size_t)blockIdx.x * kSortTile;
    s[threadIdx.x] = keys[base + threadIdx.x];
    s[threadIdx.x + kSortThreads] = keys[base + threadIdx.x + kSortThreads];
    __syncthreads();
    const bool up = ((base & k) == 0);  // the whole tile lies in one k-block
    for (int j = kSortTile >> 1; j > 0; j >>= 1) {
        const int t = threadIdx.x;
        const int i = (t / j) * 2 * j + (t % j);
        cmpx(s[i], s[i + j], up);
        __syncthreads();
    }
    keys[base + threadIdx.x] = s[threadIdx.x];
    keys[base + threadIdx.x + kSortThreads] = s[threadIdx.x + kSortThreads];
}

// One global compare-exchange step (stage k, stride j >= 2048).
__global__ __launch_bounds__(kBlock) void bitonic_step_kernel(unsigned long long* keys, size_t n, size_t k, size_t j)
{
    const size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= n / 2) return;
    const size_t i = (t / j) * 2 * j + (t % j);
    unsigned long long a = keys[i], b = keys[i + j];
    cmpx(a, b, (i & k) == 0);
    keys[i] = a;
    keys[i + j] = b;
}

}  // namespace

size_t sort_padded_size(size_t n)
{
    size_t p = kSortTile;
    while (p < n) p <<= 1;
    return p;
}

void launch_sort_u64(unsigned long long* keys, size_t n_pow2, hipStream_t s)
{
    const unsigned tiles = (unsigned)(n_pow2 / kSortTile);
    hipLaunchKernelGGL(bitonic_tile_kernel, dim3(tiles), dim3(kSortThreads), 0, s, keys);
    for (size_t k = (size_t)kSortTile << 1; k <= n_pow2; k <<= 1) {
        for (size_t j = k >> 1; j >= (size_t)kSortTile; j >>= 1)
            hipLaunchKernelGGL(bitonic_step_kernel, dim3((unsigned)((n_pow2 / 2 + kBlock - 1) / kBlock)), dim3(kBlock),
                               0, s, keys, n_pow2, k, j);
        hipLaunchKernelGGL(bitonic_merge_tile_kernel, dim3(tiles), dim3(kSortThreads), 0, s, keys, k);
    }
}

}  // namespace abcsmc
