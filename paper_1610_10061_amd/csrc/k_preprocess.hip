// Preprocessing (Section 2.1; Section 3.1 host step 3): per client row, order
// the facilities by (distance, index) and emit the first K = m - p + 1
// entries of the ordering Pi', the gap terms Delta' and the sorted distances
// D'.
//
// One workgroup sorts one row in LDS.  A facility becomes the key
// (d_ij << 16) | j; keys are distinct, so an ascending sort of keys is the
// order by distance with ties broken by the lower index, the order the
// paper's Example 1 prints.  When every distance of the row is below 2^16
// the key fits 32 bits, so the sort moves half the LDS bytes and twice as
// many rows are sorted at once; otherwise it takes 64 bits.  The row is padded to a power of two with all-ones keys
// and sorted by a bitonic network (Batcher, 1968).  The epilogue splits the
// first K keys back into index and distance and takes the first difference
// of the distances.
#include <algorithm>

#include "common.hpp"

namespace pmp {

namespace {

constexpr int kSortThreads = 512;
constexpr int kSortPerThread = PMP_MAX_FACILITIES / kSortThreads;  // 16

// Compare-exchange t of a stage joins keys lo = 2t - (t mod stride) and
// lo + stride.  With stride <= 32 the 64 threads of a wave (t in an aligned
// block of 64) touch only their own aligned block of 128 keys, the same
// block in every such stage, so consecutive stages of that kind need only
// the wave's own ordering; a workgroup barrier is needed around the others.
template <class Key>
__device__ __forceinline__ void bitonic_sort(Key *key, int m2)
{
    const int half = m2 >> 1;
    for (int size = 2; size <= m2; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = threadIdx.x; t < half; t += kSortThreads) {
                const int lo = 2 * t - (t & (stride - 1));
                const int hi = lo + stride;
                const bool ascending = (lo & size) == 0;
                const Key a = key[lo], b = key[hi];
                if ((a > b) == ascending) {
                    key[lo] = b;
                    key[hi] = a;
                }
            }
            const int next = stride > 1 ? stride >> 1 : size;  // the next stage's stride
            if (stride > 32 || next > 32) {
                __syncthreads();
            } else {
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                __builtin_amdgcn_wave_barrier();
            }
        }
    }
    __syncthreads();
}

template <class Key>
__device__ __forceinline__ void emit_row(const Key *key, int K, int pitch, int64_t base,
                                         uint16_t *pi, int32_t *delta, int32_t *ds)
{
    for (int k = threadIdx.x; k < pitch; k += kSortThreads) {
        uint16_t f = 0;
        int32_t dist = 0, gap = 0;
        if (k < K) {
            const Key x = key[k];
            f = (uint16_t)(x & 0xFFFFu);
            dist = (int32_t)(x >> 16);
            gap = k == 0 ? dist : dist - (int32_t)(key[k - 1] >> 16);
        }
        pi[base + k] = f;
        ds[base + k] = dist;
        delta[base + k] = gap;
    }
}

// Two launches, one per key width: the 32-bit one (m2 x 4 bytes of LDS, so
// twice as many workgroups stay resident) sorts the rows whose distances are
// all below 2^16 and checks every row for negative distances; the 64-bit one
// sorts the others.  Each reads the row and skips it when it belongs to the
// other.  m2 <= PMP_MAX_FACILITIES; dynamic LDS holds m2 keys.
template <class Key>
__global__ __launch_bounds__(kSortThreads) void k_sort_rows(
    const int32_t *__restrict__ d, int64_t ld, int32_t m, int32_t m2,
    int32_t K, int32_t pitch, uint16_t *__restrict__ pi,
    int32_t *__restrict__ delta, int32_t *__restrict__ ds,
    uint32_t *__restrict__ err)
{
    constexpr bool k32 = sizeof(Key) == 4;
    extern __shared__ uint64_t lds_keys[];
    Key *key = reinterpret_cast<Key *>(lds_keys);
    const int32_t i = blockIdx.x;
    const int32_t *row = d + (int64_t)i * ld;
    int32_t v[kSortPerThread];
    int negative = 0, wide = 0;
#pragma unroll
    for (int r = 0; r < kSortPerThread; ++r) {
        const int j = threadIdx.x + r * kSortThreads;
        v[r] = row[j < m ? j : m - 1];  // every load at a valid address
        if (j < m) {
            negative |= v[r] < 0;
            wide |= v[r] >= 65536;
        }
    }
    if (k32 && __syncthreads_or(negative) && threadIdx.x == 0)
        atomicOr(err, ERR_NEGATIVE_DISTANCE);
    if ((__syncthreads_or(wide) != 0) == k32)
        return;  // the other launch's row
#pragma unroll
    for (int r = 0; r < kSortPerThread; ++r) {
        const int j = threadIdx.x + r * kSortThreads;
        if (j < m2)
            key[j] = j < m ? ((Key)(uint32_t)v[r] << 16) | (Key)j : ~(Key)0;
    }
    __syncthreads();
    bitonic_sort(key, m2);
    emit_row(key, K, pitch, (int64_t)i * pitch, pi, delta, ds);
}

// ---------------------------------------------------------------------------
// Rows wider than PMP_MAX_FACILITIES (m up to 65535): the same bitonic
// network on the padded row (m2 keys, a power of two), 64-bit keys, run in
// device memory.  Each row's keys live in a scratch array; chunks of
// kWideChunk keys are sorted in LDS by every stage of size <= kWideChunk
// (compare directions from the keys' global indices, as in the whole
// network); each larger size runs its strides >= kWideChunk as passes over
// the scratch (a thread per compare-exchange) and its smaller strides in LDS
// again, chunk by chunk.
// ---------------------------------------------------------------------------
constexpr int kWideChunk = PMP_MAX_FACILITIES;  // keys per LDS chunk (64 KB)

// Stages (size, stride) with size in [size_lo, size_hi] and stride < kWideChunk
// on the chunk at global index base (keys in LDS).
__device__ __forceinline__ void bitonic_chunk(uint64_t *key, int base, int size_lo, int size_hi)
{
    const int half = kWideChunk >> 1;
    for (int size = size_lo; size <= size_hi; size <<= 1) {
        for (int stride = min(size, kWideChunk) >> 1; stride > 0; stride >>= 1) {
            for (int t = threadIdx.x; t < half; t += kSortThreads) {
                const int lo = 2 * t - (t & (stride - 1));
                const int hi = lo + stride;
                const bool ascending = ((base + lo) & size) == 0;
                const uint64_t a = key[lo], b = key[hi];
                if ((a > b) == ascending) {
                    key[lo] = b;
                    key[hi] = a;
                }
            }
            __syncthreads();
        }
    }
}

// Load the keys of row blockIdx.y, chunk blockIdx.x (padding past m with
// all-ones keys; negative distances flagged), sort the chunk by every stage
// of size <= kWideChunk, store it to the row's scratch.
__global__ __launch_bounds__(kSortThreads) void k_wide_chunks(
    const int32_t *__restrict__ d, int64_t ld, int32_t row0, int32_t m, int32_t m2,
    uint64_t *__restrict__ scratch, uint32_t *__restrict__ err)
{
    extern __shared__ uint64_t lds_keys[];
    const int32_t i = row0 + (int32_t)blockIdx.y;
    const int base = (int)blockIdx.x * kWideChunk;
    const int32_t *row = d + (int64_t)i * ld;
    uint64_t *out = scratch + (int64_t)blockIdx.y * m2 + base;
    int negative = 0;
    for (int k = threadIdx.x; k < kWideChunk; k += kSortThreads) {
        const int j = base + k;
        uint64_t key = ~0ull;
        if (j < m) {
            const int32_t v = row[j];
            negative |= v < 0;
            key = ((uint64_t)(uint32_t)v << 16) | (uint64_t)j;
        }
        lds_keys[k] = key;
    }
    if (__syncthreads_or(negative) && threadIdx.x == 0)
        atomicOr(err, ERR_NEGATIVE_DISTANCE);
    bitonic_chunk(lds_keys, base, 2, kWideChunk);
    for (int k = threadIdx.x; k < kWideChunk; k += kSortThreads)
        out[k] = lds_keys[k];
}

// One stage (size, stride >= kWideChunk) of every row of the batch: a
// thread per compare-exchange.
__global__ void k_wide_step(uint64_t *__restrict__ scratch, int32_t m2, int32_t size,
                            int32_t stride)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int half = m2 >> 1;
    if (t >= half)
        return;
    uint64_t *key = scratch + (int64_t)blockIdx.y * m2;
    const int lo = 2 * (int)t - ((int)t & (stride - 1));
    const int hi = lo + stride;
    const bool ascending = (lo & size) == 0;
    const uint64_t a = key[lo], b = key[hi];
    if ((a > b) == ascending) {
        key[lo] = b;
        key[hi] = a;
    }
}

// The strides below kWideChunk of stage `size`, chunk by chunk in LDS.
__global__ __launch_bounds__(kSortThreads) void k_wide_local(uint64_t *__restrict__ scratch,
                                                            int32_t m2, int32_t size)
{
    extern __shared__ uint64_t lds_keys[];
    const int base = (int)blockIdx.x * kWideChunk;
    uint64_t *key = scratch + (int64_t)blockIdx.y * m2 + base;
    for (int k = threadIdx.x; k < kWideChunk; k += kSortThreads)
        lds_keys[k] = key[k];
    __syncthreads();
    const int half = kWideChunk >> 1;
    for (int stride = kWideChunk >> 1; stride > 0; stride >>= 1) {
        for (int t = threadIdx.x; t < half; t += kSortThreads) {
            const int lo = 2 * t - (t & (stride - 1));
            const int hi = lo + stride;
            const bool ascending = ((base + lo) & size) == 0;
            const uint64_t a = lds_keys[lo], b = lds_keys[hi];
            if ((a > b) == ascending) {
                lds_keys[lo] = b;
                lds_keys[hi] = a;
            }
        }
        __syncthreads();
    }
    for (int k = threadIdx.x; k < kWideChunk; k += kSortThreads)
        key[k] = lds_keys[k];
}

// Pi', Delta', D' of the batch's rows from their sorted keys.
__global__ __launch_bounds__(kSortThreads) void k_wide_emit(const uint64_t *__restrict__ scratch,
                                                           int32_t row0, int32_t m2, int32_t K,
                                                           int32_t pitch, uint16_t *pi,
                                                           int32_t *delta, int32_t *ds)
{
    const uint64_t *key = scratch + (int64_t)blockIdx.y * m2;
    const int64_t base = (int64_t)(row0 + (int32_t)blockIdx.y) * pitch;
    for (int k = (int)blockIdx.x * kSortThreads + threadIdx.x; k < pitch;
         k += (int)gridDim.x * kSortThreads) {
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

int wide_sort_rows_per_batch(int32_t m)
{
    int32_t m2 = 2;
    while (m2 < m)
        m2 <<= 1;
    // about 256 MB of scratch keys per batch
    const int64_t rows = (256ll << 20) / ((int64_t)m2 * 8);
    return (int)std::max<int64_t>(1, std::min<int64_t>(rows, 65535));
}

hipError_t launch_sort_rows_wide(const int32_t *d, int64_t ld, int32_t n, int32_t m,
                                 int32_t K, int32_t pitch, uint16_t *pi, int32_t *delta,
                                 int32_t *ds, uint32_t *err, uint64_t *scratch, int32_t batch,
                                 hipStream_t s)
{
    int32_t m2 = 2;
    while (m2 < m)
        m2 <<= 1;
    const int chunks = m2 / kWideChunk;
    const size_t lds = sizeof(uint64_t) * kWideChunk;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_wide_chunks),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_wide_local),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess)
        return e;
    for (int32_t row0 = 0; row0 < n; row0 += batch) {
        const int32_t rows = std::min(batch, n - row0);
        hipLaunchKernelGGL(k_wide_chunks, dim3(chunks, rows), dim3(kSortThreads), lds, s, d, ld,
                           row0, m, m2, scratch, err);
        for (int size = 2 * kWideChunk; size <= m2; size <<= 1) {
            for (int stride = size >> 1; stride >= kWideChunk; stride >>= 1)
                hipLaunchKernelGGL(k_wide_step, dim3((m2 / 2 + 255) / 256, rows), dim3(256), 0,
                                   s, scratch, m2, size, stride);
            hipLaunchKernelGGL(k_wide_local, dim3(chunks, rows), dim3(kSortThreads), lds, s,
                               scratch, m2, size);
        }
        hipLaunchKernelGGL(k_wide_emit, dim3((pitch + kSortThreads - 1) / kSortThreads, rows),
                           dim3(kSortThreads), 0, s, scratch, row0, m2, K, pitch, pi, delta, ds);
        e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

hipError_t launch_sort_rows(const int32_t *d, int64_t ld, int32_t n, int32_t m,
                            int32_t K, int32_t pitch, uint16_t *pi,
                            int32_t *delta, int32_t *ds, uint32_t *err,
                            hipStream_t s)
{
    int32_t m2 = 2;
    while (m2 < m)
        m2 <<= 1;
    hipLaunchKernelGGL(k_sort_rows<uint32_t>, dim3(n), dim3(kSortThreads),
                       sizeof(uint32_t) * (size_t)m2, s, d, ld, m, m2, K, pitch, pi, delta, ds,
                       err);
    hipLaunchKernelGGL(k_sort_rows<uint64_t>, dim3(n), dim3(kSortThreads),
                       sizeof(uint64_t) * (size_t)m2, s, d, ld, m, m2, K, pitch, pi, delta, ds,
                       err);
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
