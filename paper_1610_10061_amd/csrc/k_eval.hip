// Population evaluation kernels: one launch evaluates a population
// (eval_device.hpp), a second adds the client-tile partial sums up.
#include <hip/hip_ext.h>

#include <atomic>

#include "eval_device.hpp"

namespace pmp {

namespace {

template <int WD, bool R, bool H, int NV, bool GT = false>
__global__ __launch_bounds__(kEvalTile *NV) void k_eval(EvalArgs a)
{
    __shared__ __align__(16) uint32_t smask[eval_stage_words<WD>()];
    __shared__ unsigned long long sred[2 * NV * kEvalTile];
    // (A stopped GA run enqueues no-op generations: eval_tile checks the
    // stop flag once its loads are on their way.)
    // All chromosome tiles of one client tile on one XCD (workgroups are
    // dealt to the 8 XCDs round-robin).
    const int ntiles = a.tiles_c * a.tiles_i;
    const int per_xcd = (int)gridDim.x >> 3;
    const int logical = ((int)blockIdx.x & 7) * per_xcd + ((int)blockIdx.x >> 3);
    const bool live = logical < ntiles;  // (tested inside, once the loads are out)
    const int lt = live ? logical : 0;
    const int ti = lt / a.tiles_c;
    eval_tile<WD, R, H, NV, false, GT>(a, ti, lt - ti * a.tiles_c, smask, sred, nullptr, nullptr,
                                       live);
}

// Facility-major copy of chromosome tile tc's word w by one wave: lane c
// holds chromosome c's word, the transpose gives lane f the bits of
// facility 64 w + f in all 64 chromosomes.  Wave (tc, 0) also writes the
// all-zero and all-ones words after the tile's 64 W words.
__global__ __launch_bounds__(256) void k_tile_major(const uint64_t *__restrict__ masks, int P,
                                                    int W, int tiles_c, uint64_t *__restrict__ tg,
                                                    int64_t stride)
{
    const int gw = (int)blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (gw >= tiles_c * W)
        return;
    const int tc = gw / W, w = gw - tc * W;
    const int c = tc * kEvalTile + lane;
    const uint64_t v = masks[(int64_t)min(c, P - 1) * W + w];
    uint32_t lo = c < P ? (uint32_t)v : 0u, hi = c < P ? (uint32_t)(v >> 32) : 0u;
    const TransposeLanes tl(lane);
    transpose64(lo, hi, lane, tl);
    uint64_t *t = tg + (int64_t)tc * stride;
    t[(int64_t)w * 64 + lane] = ((uint64_t)hi << 32) | lo;
    if (w == 0 && lane < 2)
        t[(int64_t)W * 64 + lane] = lane ? ~0ull : 0ull;
}

// Feasibility of every chromosome (a wave each): exactly p open facilities
// and no bits at positions >= m.
__global__ __launch_bounds__(256) void k_check_masks(const uint64_t *__restrict__ masks, int P,
                                                     int W, int m, int p, uint32_t *err)
{
    const int c = (int)blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (c >= P)
        return;
    const uint64_t past = (m & 63) ? ~((1ull << (m & 63)) - 1ull) : 0ull;
    uint32_t ones = 0, stray = 0;
    for (int w = lane; w < W; w += 64) {
        const uint64_t v = masks[(int64_t)c * W + w];
        ones += (uint32_t)__builtin_popcountll(v);
        if (w == W - 1 && (v & past))
            stray = 1;
    }
    for (int o = 32; o > 0; o >>= 1) {
        ones += (uint32_t)__shfl_xor((int)ones, o);
        stray |= (uint32_t)__shfl_xor((int)stray, o);
    }
    if (lane == 0) {
        if (ones != (uint32_t)p)
            atomicOr(err, ERR_POPCOUNT);
        if (stray)
            atomicOr(err, ERR_STRAY_BITS);
    }
}

// fitness[c] (and scan[c]) = sum over client tiles of the partial sums.
__global__ __launch_bounds__(256) void k_reduce(
    const unsigned long long *__restrict__ part, const uint32_t *__restrict__ spart,
    int tiles_i, int P, unsigned long long *__restrict__ fitness,
    unsigned long long *__restrict__ scan, long long c0)
{
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= P)
        return;
    unsigned long long f = 0, s = 0;
    for (int t = 0; t < tiles_i; ++t) {
        f += part[(int64_t)t * P + c];
        if (spart)
            s += spart[(int64_t)t * P + c];
    }
    fitness[c] = f + (unsigned long long)c0;
    if (scan)
        scan[c] = s;
}

template <int WD, bool R, bool H, int NV>
hipError_t launch_nv(const EvalArgs &a, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    const int tiles = a.tiles_c * a.tiles_i;
    const int grid = ((tiles + 7) / 8) * 8;
    auto kernel = k_eval<WD, R, H, NV>;
    if (e0 && e1) {
        // events stamped by the dispatch itself: their interval is the
        // kernel's execution, without the gaps around it
        hipExtLaunchKernelGGL(kernel, dim3(grid), dim3(kEvalTile * NV), 0, s, e0, e1, 0, a);
    } else {
        hipLaunchKernelGGL(kernel, dim3(grid), dim3(kEvalTile * NV), 0, s, a);
    }
    return hipGetLastError();
}

// Waves per workgroup: 4 (the default), 8 or 16; the reduced walk runs
// with 4.
template <int WD, bool R, bool H>
hipError_t launch_wd(const EvalArgs &a, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    if constexpr (!R) {
        if (a.waves == 8)
            return launch_nv<WD, R, H, 8>(a, s, e0, e1);
        if (a.waves == 16)
            return launch_nv<WD, R, H, 16>(a, s, e0, e1);
    }
    return launch_nv<WD, R, H, kEvalWaves>(a, s, e0, e1);
}

}  // namespace

hipError_t launch_tile_major(const EvalArgs &a, uint64_t *tg, hipStream_t s)
{
    const int W = a.t.W;
    hipLaunchKernelGGL(k_check_masks, dim3((a.P + 3) / 4), dim3(256), 0, s, a.masks, a.P, W,
                       a.t.m, a.t.p, a.err);
    hipLaunchKernelGGL(k_tile_major, dim3((a.tiles_c * W + 3) / 4), dim3(256), 0, s, a.masks,
                       a.P, W, a.tiles_c, tg, a.tg_stride);
    return hipGetLastError();
}

hipError_t launch_reduce(const EvalArgs &a, unsigned long long *fitness,
                         unsigned long long *scan, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce, dim3((a.P + 255) / 256), dim3(256), 0, s, a.part,
                       a.spart, a.tiles_i, a.P, fitness, scan, a.c0);
    return hipGetLastError();
}

namespace {

template <int WD, bool R, bool H, int NV, bool GT = false>
int resident_nv()
{
    static std::atomic<int> cached{0};  // the same for every call: computed once
    int per_cu = cached.load(std::memory_order_relaxed);
    if (per_cu == 0) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &per_cu, reinterpret_cast<const void *>(k_eval<WD, R, H, NV, GT>),
                kEvalTile * NV, 0) != hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        cached.store(per_cu, std::memory_order_relaxed);
    }
    return per_cu;
}

template <int WD, bool R, bool H>
int resident_wd(int waves)
{
    if constexpr (!R) {
        if (waves == 8)
            return resident_nv<WD, R, H, 8>();
        if (waves == 16)
            return resident_nv<WD, R, H, 16>();
    }
    return resident_nv<WD, R, H, kEvalWaves>();
}

}  // namespace

int eval_workgroups_per_cu(int W, bool reduced, bool paired, int waves)
{
    const int w2 = 2 * W;
#define PMP_EVAL_WD(N)                                                           \
    if (w2 <= N)                                                                 \
        return reduced ? resident_wd<N, true, false>(waves)                       \
                       : (paired ? resident_wd<N, false, true>(waves)             \
                                 : resident_wd<N, false, false>(waves));
    PMP_EVAL_WD(2)
    PMP_EVAL_WD(4)
    PMP_EVAL_WD(8)
    PMP_EVAL_WD(16)
    PMP_EVAL_WD(32)
    PMP_EVAL_WD(48)
    PMP_EVAL_WD(64)
    PMP_EVAL_WD(96)
    PMP_EVAL_WD(128)
    PMP_EVAL_WD(160)
    PMP_EVAL_WD(192)
    PMP_EVAL_WD(256)
#undef PMP_EVAL_WD
    return resident_nv<2, false, false, 16, true>();  // wide: the device-memory tile walk
}

hipError_t launch_eval(const EvalArgs &a, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    if (a.P <= 0 || a.tiles_c <= 0 || a.tiles_i <= 0)
        return hipSuccess;
    const bool red = a.rlen != nullptr;
    const int w2 = 2 * a.t.W;
    if (a.tg) {  // wide chromosomes: the single walk on the device-memory tiles, 16 waves
        if (red || a.paired)
            return hipErrorInvalidValue;
        const int tiles = a.tiles_c * a.tiles_i;
        const int grid = ((tiles + 7) / 8) * 8;
        auto kernel = k_eval<2, false, false, 16, true>;
        if (e0 && e1)
            hipExtLaunchKernelGGL(kernel, dim3(grid), dim3(kEvalTile * 16), 0, s, e0, e1, 0, a);
        else
            hipLaunchKernelGGL(kernel, dim3(grid), dim3(kEvalTile * 16), 0, s, a);
        return hipGetLastError();
    }
#define PMP_EVAL_WD(N)                                                         \
    if (w2 <= N)                                                               \
        return red ? launch_wd<N, true, false>(a, s, e0, e1)                     \
                   : (a.paired ? launch_wd<N, false, true>(a, s, e0, e1)         \
                               : launch_wd<N, false, false>(a, s, e0, e1));
    PMP_EVAL_WD(2)
    PMP_EVAL_WD(4)
    PMP_EVAL_WD(8)
    PMP_EVAL_WD(16)
    PMP_EVAL_WD(32)
    PMP_EVAL_WD(48)
    PMP_EVAL_WD(64)
    PMP_EVAL_WD(96)
    PMP_EVAL_WD(128)
    PMP_EVAL_WD(160)
    PMP_EVAL_WD(192)
    PMP_EVAL_WD(256)
#undef PMP_EVAL_WD
    return hipErrorInvalidValue;
}

}  // namespace pmp
