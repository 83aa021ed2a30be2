// Preprocessing (Section 2.1; Section 3.1 host step 3): per client row, order
// the facilities by (distance, index) and emit the first K = m - p + 1
// entries of the ordering Pi', the gap terms Delta' and the sorted distances
// D'.
//
// One workgroup sorts one row in LDS.  A facility becomes the 64-bit key
// (d_ij << 16) | j; keys are distinct, so an ascending sort of keys is the
// order by distance with ties broken by the lower index, the order the
// paper's Example 1 prints.  The row is padded to a power of two with
// all-ones keys and sorted by a bitonic network (Batcher, 1968).  The
// epilogue splits the first K keys back into index and distance and takes
// the first difference of the distances.
#include "common.hpp"

namespace pmp {

namespace {

constexpr int kSortThreads = 512;

__global__ __launch_bounds__(kSortThreads) void k_sort_rows(
    const int32_t *__restrict__ d, int64_t ld, int32_t m, int32_t m2,
    int32_t K, int32_t pitch, uint16_t *__restrict__ pi,
    int32_t *__restrict__ delta, int32_t *__restrict__ ds,
    uint32_t *__restrict__ err)
{
    extern __shared__ uint64_t key[];
    const int32_t i = blockIdx.x;
    const int32_t *row = d + (int64_t)i * ld;
    int negative = 0;
    for (int j = threadIdx.x; j < m2; j += kSortThreads) {
        uint64_t k = ~0ull;
        if (j < m) {
            const int32_t v = row[j];
            negative |= v < 0;
            k = ((uint64_t)(uint32_t)v << 16) | (uint64_t)j;
        }
        key[j] = k;
    }
    if (__syncthreads_or(negative) && threadIdx.x == 0)
        atomicOr(err, ERR_NEGATIVE_DISTANCE);

    const int half = m2 >> 1;
    for (int size = 2; size <= m2; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = threadIdx.x; t < half; t += kSortThreads) {
                const int lo = 2 * t - (t & (stride - 1));
                const int hi = lo + stride;
                const bool ascending = (lo & size) == 0;
                const uint64_t a = key[lo], b = key[hi];
                if ((a > b) == ascending) {
                    key[lo] = b;
                    key[hi] = a;
                }
            }
            __syncthreads();
        }
    }

    const int64_t base = (int64_t)i * pitch;
    for (int k = threadIdx.x; k < pitch; k += kSortThreads) {
        uint16_t f = 0;
        int32_t dist = 0, gap = 0;
        if (k < K) {
            const uint64_t x = key[k];
            f = (uint16_t)(x & 0xFFFFu);
            dist = (int32_t)(x >> 16);
            gap = k == 0 ? dist : dist - (int32_t)(key[k - 1] >> 16);
        }
        pi[base + k] = f;
        ds[base + k] = dist;
        delta[base + k] = gap;
    }
}

__global__ void k_zero(uint32_t *p, size_t words)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < words;
         k += stride)
        p[k] = 0;
}

}  // namespace

hipError_t launch_sort_rows(const int32_t *d, int64_t ld, int32_t n, int32_t m,
                            int32_t K, int32_t pitch, uint16_t *pi,
                            int32_t *delta, int32_t *ds, uint32_t *err,
                            hipStream_t s)
{
    int32_t m2 = 2;
    while (m2 < m)
        m2 <<= 1;
    const size_t lds = sizeof(uint64_t) * (size_t)m2;
    hipLaunchKernelGGL(k_sort_rows, dim3(n), dim3(kSortThreads), lds, s, d, ld,
                       m, m2, K, pitch, pi, delta, ds, err);
    return hipGetLastError();
}

// Zero a device buffer with a kernel (safe inside stream capture).
hipError_t launch_zero(void *p, size_t bytes, hipStream_t s)
{
    if (bytes == 0)
        return hipSuccess;
    if (bytes % 4 != 0)
        return hipErrorInvalidValue;
    const size_t words = bytes / 4;
    size_t blocks = (words + 255) / 256;
    if (blocks > 1024)
        blocks = 1024;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, s,
                       (uint32_t *)p, words);
    return hipGetLastError();
}

}  // namespace pmp
