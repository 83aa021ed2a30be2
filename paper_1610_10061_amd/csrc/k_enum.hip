// Exhaustive enumeration of the open sets (Eq. (1)-(3) minimised over all
// C(m, p) subsets), a second workload of the evaluation kernel: batches of
// consecutive lexicographic ranks are unranked into chromosome masks, the
// evaluation kernel scores them, and each batch's least (cost, rank) is kept.
//
// Unranking (the combinatorial number system in lexicographic order): for
// the i-th smallest element, skip candidates x while the subsets that begin
// with x (C(m - x - 1, p - i - 1) of them) all come before the rank.
#include "common.hpp"

namespace pmp {

namespace {

// masks[r - r0] = the subset of lexicographic rank r, r0 <= r < r0 + count.
// binom[a * (p + 1) + b] = C(a, b) for a < m, b <= p (saturating).
__global__ void k_unrank(const unsigned long long *binom, int m, int p, int W,
                         unsigned long long r0, int count, uint64_t *masks)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count)
        return;
    unsigned long long r = r0 + (unsigned long long)t;
    uint64_t *out = masks + (int64_t)t * W;
    for (int w = 0; w < W; ++w)
        out[w] = 0ull;
    int x = 0;
    for (int i = 0; i < p; ++i) {
        // subsets whose i-th element is x: choose the remaining p - i - 1
        // from the m - x - 1 elements above x
        for (;;) {
            const unsigned long long c = binom[(int64_t)(m - x - 1) * (p + 1) + (p - i - 1)];
            if (r < c)
                break;
            r -= c;
            ++x;
        }
        out[x >> 6] |= 1ull << (x & 63);
        ++x;
    }
}

// Least (cost, index) of each block's range of fitness values; ties go to
// the lower index.
__global__ __launch_bounds__(256) void k_argmin(const unsigned long long *fit, int count,
                                                unsigned long long *best_cost, int *best_idx)
{
    __shared__ unsigned long long sc[256];
    __shared__ int si[256];
    const int t = blockIdx.x * 256 + threadIdx.x;
    unsigned long long f = ~0ull;
    int idx = 0x7FFFFFFF;
    if (t < count) {
        f = fit[t];
        idx = t;
    }
    sc[threadIdx.x] = f;
    si[threadIdx.x] = idx;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            const unsigned long long of = sc[threadIdx.x + s];
            const int oi = si[threadIdx.x + s];
            if (of < sc[threadIdx.x] || (of == sc[threadIdx.x] && oi < si[threadIdx.x])) {
                sc[threadIdx.x] = of;
                si[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        best_cost[blockIdx.x] = sc[0];
        best_idx[blockIdx.x] = si[0];
    }
}

// Fold the block results of one batch (ranks r0 + index) into the running
// best run[0] = cost, run[1] = rank.  Batches come in rank order, so a tie
// keeps the earlier rank.
__global__ __launch_bounds__(256) void k_fold(const unsigned long long *bc, const int *bi,
                                              int nblk, unsigned long long r0,
                                              unsigned long long *run)
{
    __shared__ unsigned long long sc[256];
    __shared__ int si[256];
    unsigned long long f = ~0ull;
    int idx = 0x7FFFFFFF;
    for (int b = threadIdx.x; b < nblk; b += 256) {
        const unsigned long long v = bc[b];
        const int i = bi[b];
        if (v < f || (v == f && i < idx)) {
            f = v;
            idx = i;
        }
    }
    sc[threadIdx.x] = f;
    si[threadIdx.x] = idx;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            const unsigned long long of = sc[threadIdx.x + s];
            const int oi = si[threadIdx.x + s];
            if (of < sc[threadIdx.x] || (of == sc[threadIdx.x] && oi < si[threadIdx.x])) {
                sc[threadIdx.x] = of;
                si[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0 && sc[0] < run[0]) {
        run[0] = sc[0];
        run[1] = r0 + (unsigned long long)si[0];
    }
}

}  // namespace

hipError_t launch_fold(const unsigned long long *bc, const int *bi, int nblk,
                       unsigned long long r0, unsigned long long *run, hipStream_t s)
{
    hipLaunchKernelGGL(k_fold, dim3(1), dim3(256), 0, s, bc, bi, nblk, r0, run);
    return hipGetLastError();
}

hipError_t launch_unrank(const unsigned long long *binom, int m, int p, int W,
                         unsigned long long r0, int count, uint64_t *masks, hipStream_t s)
{
    if (count <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_unrank, dim3((count + 255) / 256), dim3(256), 0, s, binom, m, p, W, r0,
                       count, masks);
    return hipGetLastError();
}

hipError_t launch_argmin(const unsigned long long *fit, int count, unsigned long long *best_cost,
                         int *best_idx, hipStream_t s)
{
    if (count <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_argmin, dim3((count + 255) / 256), dim3(256), 0, s, fit, count,
                       best_cost, best_idx);
    return hipGetLastError();
}

}  // namespace pmp
