// Genetic-algorithm kernels.  Two launch schemes run the same device code
// (ga_device.hpp, eval_device.hpp):
//
//  - one kernel per step: k_init, the evaluation kernel, k_stage for each
//    stage, k_best; ordered by the stream.
//  - k_ga_persistent: one cooperative launch runs whole generations; its
//    phases are separated by grid barriers, which removes the per-launch
//    gaps and prologues that dominate at a few microseconds of work per
//    stage.
#include "eval_device.hpp"
#include "ga_device.hpp"

namespace pmp {

namespace {

__global__ __launch_bounds__(64 * kGaWaves) void k_init(GaArgs g)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int c = blockIdx.x * kGaWaves + wave;
    if (c >= g.P || ga_stopped(g))
        return;
    ga_init_one(g, c, lane);
}

__global__ __launch_bounds__(64 * kGaWaves) void k_stage(GaArgs g, int in,
                                                         int prev, int op,
                                                         int index)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int c = blockIdx.x * kGaWaves + wave;
    if (c >= g.P || ga_stopped(g))
        return;
    ga_stage_one(g, c, lane, in, prev, op, index);
}

// Group best per workgroup; the last workgroup to finish does the global
// update (release fence before the arrival count, acquire fence after).
__global__ __launch_bounds__(1024) void k_best(GaArgs g, int fb)
{
    __shared__ unsigned long long sc[16];
    __shared__ int si[16];
    __shared__ int last;
    if (ga_stopped(g))
        return;
    ga_group_best(g, fb, blockIdx.x, sc, si);
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0)
        last = atomicAdd(g.arrive, 1u) == (uint32_t)(g.NB - 1);
    __syncthreads();
    if (!last)
        return;
    __threadfence();
    ga_global(g, sc, si);
    if (threadIdx.x == 0)
        *g.arrive = 0;
}

// ---------------------------------------------------------------------------
// Grid barrier of the persistent kernel, without a contended counter: each
// workgroup publishes its writes (agent-scope release) and then stores the
// barrier's epoch number into its own flag (its own 128-byte line);
// workgroup 0's threads wait until every flag shows the epoch and then store
// it into the shared epoch word, which the other workgroups wait on.  Every
// workgroup passes the same sequence of barriers, so each knows the epoch
// number it is waiting for.  Waits are bounded by the 100 MHz real-time
// clock: past the bound (only if some workgroup never arrives) the error
// word records it and every later barrier and loop of the kernel returns at
// once, so the grid always drains.
// ---------------------------------------------------------------------------
constexpr uint64_t kBarrierTicks = 200000000ull;  // 2 s at 100 MHz
constexpr int kFlagStride = 32;                   // words between flags

__device__ __forceinline__ uint32_t load_agent(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait until *p == want; false on timeout (and the error is recorded).
__device__ __forceinline__ bool wait_for(const uint32_t *p, uint32_t want,
                                         uint32_t *err)
{
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    while (load_agent(p) != want) {
        __builtin_amdgcn_s_sleep(1);
        if (__builtin_amdgcn_s_memrealtime() - t0 > kBarrierTicks) {
            atomicOr(err, ERR_BARRIER_TIMEOUT);
            return false;
        }
    }
    return true;
}

struct GridBarrier {
    uint32_t *epoch;  // bar[0]
    uint32_t *flags;  // bar + kFlagStride, one per workgroup
    uint32_t next;    // epoch number of the next barrier

    __device__ __forceinline__ explicit GridBarrier(uint32_t *bar)
        : epoch(bar), flags(bar + kFlagStride), next(load_agent(bar) + 1u)
    {
    }

    __device__ __forceinline__ bool sync(const GaArgs &g, int *flag)
    {
        __syncthreads();
        const uint32_t want = next++;
        if (threadIdx.x == 0) {
            int ok = (load_agent(g.err) & ERR_BARRIER_TIMEOUT) == 0;
            if (ok) {
                // publish this workgroup's writes (L2 write-back), then arrive
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                __hip_atomic_store(flags + (size_t)blockIdx.x * kFlagStride, want,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            *flag = ok;
        }
        __syncthreads();
        if (!*flag)
            return false;
        if (blockIdx.x == 0) {
            int ok = 1;
            for (int b = threadIdx.x; b < (int)gridDim.x && ok; b += blockDim.x)
                ok = wait_for(flags + (size_t)b * kFlagStride, want, g.err);
            if (!ok)
                *flag = 0;
            __syncthreads();
            if (threadIdx.x == 0 && *flag)
                __hip_atomic_store(epoch, want, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else if (threadIdx.x == 0) {
            if (!wait_for(epoch, want, g.err))
                *flag = 0;
        }
        if (threadIdx.x == 0)  // see the other workgroups' writes (L2 invalidate)
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        __syncthreads();
        return *flag != 0;
    }
};

// Evaluation phase: the (client tile, chromosome tile) items, client-tile
// major, are cut into 8 contiguous ranges; the workgroups of XCD x (block
// index = x mod 8) take range x, so chromosome tiles sharing Pi' rows share
// an L2.
template <int WD>
__device__ __forceinline__ void eval_phase(const EvalArgs &e, uint32_t *smask,
                                           unsigned long long *sred)
{
    const int ntiles = e.tiles_c * e.tiles_i;
    const int chunk = (ntiles + 7) / 8;
    const int x = blockIdx.x & 7, per = (int)gridDim.x >> 3;
    const int end = min(ntiles, (x + 1) * chunk);
    for (int item = x * chunk + ((int)blockIdx.x >> 3); item < end; item += per) {
        const int ti = item / e.tiles_c;
        eval_tile<WD>(e, ti, item - ti * e.tiles_c, smask, sred);
    }
}

template <int WD>
__global__ __launch_bounds__(64 * kGaWaves) void k_ga_persistent(GaArgs g,
                                                                 EvalArgs e,
                                                                 int generations)
{
    extern __shared__ uint64_t lds[];
    uint32_t *smask = reinterpret_cast<uint32_t *>(lds);
    unsigned long long *sred =
        reinterpret_cast<unsigned long long *>(lds + (kEvalTile * WD) / 2);
    __shared__ unsigned long long sc[16];
    __shared__ int si[16];
    __shared__ int flag;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int gw = blockIdx.x * kGaWaves + wave, nw = gridDim.x * kGaWaves;
    const int X = ga_xstages(g), S = X + g.Y;
    const int fb = (S % 2) ^ 1;
    GridBarrier bar(g.bar);

    for (int gen = 0; gen < generations; ++gen) {
        if (ga_stopped(g))
            return;
        for (int c = gw; c < g.P; c += nw)
            ga_init_one(g, c, lane);
        if (!bar.sync(g, &flag))
            return;
        e.masks = g.off[0];
        e.active = g.ok[0];
        eval_phase<WD>(e, smask, sred);
        if (!bar.sync(g, &flag))
            return;
        for (int k = 0; k <= S; ++k) {
            int prev, op, index;
            ga_stage_ops(k, X, S, &prev, &op, &index);
            for (int c = gw; c < g.P; c += nw)
                ga_stage_one(g, c, lane, k & 1, prev, op, index);
            if (!bar.sync(g, &flag))
                return;
            if (op != OP_NONE) {
                e.masks = buf(g.off, (k & 1) ^ 1);
                e.active = buf(g.ok, (k & 1) ^ 1);
                eval_phase<WD>(e, smask, sred);
                if (!bar.sync(g, &flag))
                    return;
            }
        }
        for (int b = blockIdx.x; b < g.NB; b += gridDim.x)
            ga_group_best(g, fb, b, sc, si);
        if (!bar.sync(g, &flag))
            return;
        if (blockIdx.x == 0)
            ga_global(g, sc, si);
        if (!bar.sync(g, &flag))
            return;
    }
}

inline dim3 per_wave(int P)
{
    return dim3((unsigned)((P + kGaWaves - 1) / kGaWaves));
}

template <int WD>
size_t persistent_lds()
{
    const size_t eval = sizeof(uint32_t) * kEvalTile * WD +
                        sizeof(unsigned long long) * 2 * kEvalWaves * kEvalTile;
    return eval;
}

template <int WD>
hipError_t persistent_wd(const GaArgs &g, const EvalArgs &e, int generations,
                         int max_blocks, hipStream_t s, int *grid_out)
{
    auto fn = k_ga_persistent<WD>;
    const size_t lds = persistent_lds<WD>();
    hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                                         hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)lds);
    if (err != hipSuccess)
        return err;
    int per_cu = 0, dev = 0, cus = 0;
    err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64 * kGaWaves, lds);
    if (err == hipSuccess)
        err = hipGetDevice(&dev);
    if (err == hipSuccess)
        err = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (err != hipSuccess)
        return err;
    if (per_cu < 1)
        return hipErrorInvalidConfiguration;
    // enough workgroups for the widest phase, no more than fit at once
    const int want = max(e.tiles_c * e.tiles_i, max((g.P + kGaWaves - 1) / kGaWaves, g.NB));
    int grid = min(want, min(per_cu, 4) * cus);
    if (max_blocks > 0)
        grid = min(grid, max_blocks);
    grid = max(8, (grid / 8) * 8);
    if (grid > per_cu * cus || grid > kMaxPersistentBlocks)
        return hipErrorInvalidConfiguration;
    *grid_out = grid;
    GaArgs ga = g;
    EvalArgs ea = e;
    int gens = generations;
    void *args[] = {&ga, &ea, &gens};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(fn), dim3(grid),
                                      dim3(64 * kGaWaves), args, (unsigned)lds, s);
}

}  // namespace

hipError_t launch_ga_init(const GaArgs &g, hipStream_t s)
{
    hipLaunchKernelGGL(k_init, per_wave(g.P), dim3(64 * kGaWaves), 0, s, g);
    return hipGetLastError();
}

hipError_t launch_ga_stage(const GaArgs &g, int in, int prev, int op, int index,
                           hipStream_t s)
{
    hipLaunchKernelGGL(k_stage, per_wave(g.P), dim3(64 * kGaWaves), 0, s, g, in,
                       prev, op, index);
    return hipGetLastError();
}

hipError_t launch_ga_best(const GaArgs &g, int fb, hipStream_t s)
{
    const int threads = ((g.NT + 63) / 64) * 64;
    hipLaunchKernelGGL(k_best, dim3(g.NB), dim3(threads < 64 ? 64 : threads), 0, s,
                       g, fb);
    return hipGetLastError();
}

hipError_t launch_ga_persistent(const GaArgs &g, const EvalArgs &e,
                                int generations, int max_blocks, hipStream_t s,
                                int *grid)
{
    const int w2 = 2 * g.t.W;
    if (w2 <= 2) return persistent_wd<2>(g, e, generations, max_blocks, s, grid);
    if (w2 <= 4) return persistent_wd<4>(g, e, generations, max_blocks, s, grid);
    if (w2 <= 8) return persistent_wd<8>(g, e, generations, max_blocks, s, grid);
    if (w2 <= 16) return persistent_wd<16>(g, e, generations, max_blocks, s, grid);
    if (w2 <= 32) return persistent_wd<32>(g, e, generations, max_blocks, s, grid);
    if (w2 <= 48) return persistent_wd<48>(g, e, generations, max_blocks, s, grid);
    if (w2 <= 64) return persistent_wd<64>(g, e, generations, max_blocks, s, grid);
    if (w2 <= 96) return persistent_wd<96>(g, e, generations, max_blocks, s, grid);
    if (w2 <= 128) return persistent_wd<128>(g, e, generations, max_blocks, s, grid);
    if (w2 <= 160) return persistent_wd<160>(g, e, generations, max_blocks, s, grid);
    if (w2 <= 192) return persistent_wd<192>(g, e, generations, max_blocks, s, grid);
    if (w2 <= 256) return persistent_wd<256>(g, e, generations, max_blocks, s, grid);
    return hipErrorInvalidValue;
}

}  // namespace pmp
