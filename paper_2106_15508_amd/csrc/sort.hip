// sort.hip -- ascending bitonic sort of 64-bit keys in place (power-of-two
// length, pad with UINT64_MAX).  Callers make keys unique (payload index in
// the low bits), so the order is fully determined.  Strides below 2048 run
// inside LDS; larger strides run two per launch where they can (four keys per
// thread).  Two arrays of the same length can be sorted by the same launches
// (grid.y selects the array), which halves the launches of the weight pass.
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
__global__ __launch_bounds__(kSortThreads) void bitonic_tile_kernel(unsigned long long* keys0, unsigned long long* keys1)
{
    __shared__ unsigned long long s[kSortTile];
    unsigned long long* keys = blockIdx.y ? keys1 : keys0;
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
__global__ __launch_bounds__(kSortThreads) void bitonic_merge_tile_kernel(unsigned long long* keys0,
                                                                         unsigned long long* keys1, size_t k)
{
    __shared__ unsigned long long s[kSortTile];
    unsigned long long* keys = blockIdx.y ? keys1 : keys0;
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
__global__ __launch_bounds__(kBlock) void bitonic_step_kernel(unsigned long long* keys0, unsigned long long* keys1,
                                                              size_t n, size_t k, size_t j)
{
    unsigned long long* keys = blockIdx.y ? keys1 : keys0;
    const size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= n / 2) return;
    const size_t i = (t / j) * 2 * j + (t % j);
    unsigned long long a = keys[i], b = keys[i + j];
    cmpx(a, b, (i & k) == 0);
    keys[i] = a;
    keys[i + j] = b;
}

// Two consecutive global steps of stage k, strides j and h = j/2 (h >= 2048):
// thread t owns the keys i, i + h, i + j, i + j + h with i = (t / h) 2j + t % h,
// all in one 2j-block and so in one k-block (2j <= k): the stride-j pairs
// (i, i + j), (i + h, i + j + h), then the stride-h pairs (i, i + h),
// (i + j, i + j + h).  Every key belongs to exactly one thread.
__global__ __launch_bounds__(kBlock) void bitonic_step2_kernel(unsigned long long* keys0, unsigned long long* keys1,
                                                               size_t n, size_t k, size_t j)
{
    unsigned long long* keys = blockIdx.y ? keys1 : keys0;
    const size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= n / 4) return;
    const size_t h = j >> 1;
    const size_t i = (t / h) * 2 * j + (t % h);
    unsigned long long a = keys[i], b = keys[i + h], c = keys[i + j], d = keys[i + j + h];
    const bool up = (i & k) == 0;
    cmpx(a, c, up);
    cmpx(b, d, up);
    cmpx(a, b, up);
    cmpx(c, d, up);
    keys[i] = a;
    keys[i + h] = b;
    keys[i + j] = c;
    keys[i + j + h] = d;
}

}  // namespace

size_t sort_padded_size(size_t n)
{
    size_t p = kSortTile;
    while (p < n) p <<= 1;
    return p;
}

void launch_sort_u64_pair(unsigned long long* keys0, unsigned long long* keys1, size_t n_pow2, hipStream_t s)
{
    const unsigned tiles = (unsigned)(n_pow2 / kSortTile);
    const unsigned arrays = keys1 ? 2u : 1u;
    const dim3 bt(kSortThreads), bs(kBlock);
    const dim3 g1((unsigned)((n_pow2 / 2 + kBlock - 1) / kBlock), arrays);
    const dim3 g2((unsigned)((n_pow2 / 4 + kBlock - 1) / kBlock), arrays);
    hipLaunchKernelGGL(bitonic_tile_kernel, dim3(tiles, arrays), bt, 0, s, keys0, keys1);
    for (size_t k = (size_t)kSortTile << 1; k <= n_pow2; k <<= 1) {
        size_t j = k >> 1;
        for (; j >= 2 * (size_t)kSortTile; j >>= 2)
            hipLaunchKernelGGL(bitonic_step2_kernel, g2, bs, 0, s, keys0, keys1, n_pow2, k, j);
        if (j >= (size_t)kSortTile) hipLaunchKernelGGL(bitonic_step_kernel, g1, bs, 0, s, keys0, keys1, n_pow2, k, j);
        hipLaunchKernelGGL(bitonic_merge_tile_kernel, dim3(tiles, arrays), bt, 0, s, keys0, keys1, k);
    }
}

void launch_sort_u64(unsigned long long* keys, size_t n_pow2, hipStream_t s)
{
    launch_sort_u64_pair(keys, nullptr, n_pow2, s);
}

}  // namespace abcsmc
