// The two thread mappings the paper weighs for the Fitness function (its
// observations on the fitness bottleneck, Section 5), kept as explicit
// alternatives to the tiled evaluation kernel so the load-balance argument
// can be measured:
//  - one thread per chromosome (the paper's choice): a lane walks Pi' for
//    every client in turn and sums D' at the first open facility;
//  - one thread per client (the "n threads" scenario): a lane walks one
//    client's row for one chromosome; a wave is done only when its slowest
//    lane is, and the per-wave sums are added up afterwards.
// Both compute Eq. (6) exactly, as the tiled kernel does.
#include "common.hpp"

namespace pmp {

namespace {

// Popcount and stray-bit check of one chromosome (W words at mk).
__device__ __forceinline__ void check_mask(const uint64_t *mk, const Tables &t, uint32_t *err)
{
    int ones = 0;
    uint64_t stray = 0;
    for (int w = 0; w < t.W; ++w) {
        const uint64_t v = mk[w];
        ones += __builtin_popcountll(v);
        if (w == t.W - 1 && (t.m & 63))
            stray = v & ~((1ull << (t.m & 63)) - 1ull);
    }
    if (ones != t.p)
        atomicOr(err, ERR_POPCOUNT);
    if (stray)
        atomicOr(err, ERR_STRAY_BITS);
}

// Position of the first open facility in client i's row (0-based), or K
// when the truncated row has none (an infeasible chromosome).
__device__ __forceinline__ int first_open(const Tables &t, int i, const uint64_t *mk)
{
    const uint16_t *prow = t.pi + (int64_t)i * t.pitch;
    int k = 0;
    for (; k < t.K; ++k) {
        const uint32_t j = prow[k];
        if ((mk[j >> 6] >> (j & 63)) & 1ull)
            break;
    }
    return k;
}

__global__ __launch_bounds__(256) void k_eval_per_chromosome(EvalArgs a,
                                                             unsigned long long *fitness,
                                                             unsigned long long *scan)
{
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= a.P)
        return;
    const uint64_t *mk = a.masks + (int64_t)c * a.t.W;
    check_mask(mk, a.t, a.err);
    unsigned long long acc = 0, sc = 0;
    bool overrun = false;
    for (int i = 0; i < a.t.n; ++i) {
        const int k = first_open(a.t, i, mk);
        if (k >= a.t.K) {
            overrun = true;
            continue;
        }
        acc += (unsigned long long)a.t.ds[(int64_t)i * a.t.pitch + k];
        sc += (unsigned long long)(k + 1);
    }
    if (overrun)
        atomicOr(a.err, ERR_SCAN_OVERRUN);
    fitness[c] = acc;
    if (scan)
        scan[c] = sc;
}

// Workgroup (c, q): clients 256 q .. 256 q + 255 of chromosome c; wave v's
// sum goes to part[(4 q + v) * P + c].
__global__ __launch_bounds__(256) void k_eval_per_client(EvalArgs a, int groups)
{
    __shared__ uint64_t smk[PMP_MAX_FACILITIES / 64];
    const int c = blockIdx.x / groups, q = blockIdx.x - c * groups;
    const uint64_t *mk = a.masks + (int64_t)c * a.t.W;
    for (int w = threadIdx.x; w < a.t.W; w += 256)
        smk[w] = mk[w];
    __syncthreads();
    if (q == 0 && threadIdx.x == 0)
        check_mask(smk, a.t, a.err);
    const int i = q * 256 + (int)threadIdx.x;
    unsigned long long cost = 0, sc = 0;
    bool overrun = false;
    if (i < a.t.n) {
        const int k = first_open(a.t, i, smk);
        if (k >= a.t.K) {
            overrun = true;
        } else {
            cost = (unsigned long long)a.t.ds[(int64_t)i * a.t.pitch + k];
            sc = (unsigned long long)(k + 1);
        }
    }
    if (__builtin_amdgcn_ballot_w64(overrun) != 0ull && (threadIdx.x & 63) == 0)
        atomicOr(a.err, ERR_SCAN_OVERRUN);
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        cost += __shfl_xor(cost, d);
        sc += __shfl_xor(sc, d);
    }
    if ((threadIdx.x & 63) == 0) {
        const int64_t row = (int64_t)(4 * q + (int)(threadIdx.x >> 6)) * a.P + c;
        a.part[row] = cost;
        if (a.spart)
            a.spart[row] = (uint32_t)sc;
    }
}

}  // namespace

hipError_t launch_eval_per_chromosome(const EvalArgs &a, unsigned long long *fitness,
                                      unsigned long long *scan, hipStream_t s)
{
    hipLaunchKernelGGL(k_eval_per_chromosome, dim3((a.P + 255) / 256), dim3(256), 0, s, a,
                       fitness, scan);
    return hipGetLastError();
}

// a.tiles_i must be 4 * ceil(n / 256) and a.part / a.spart that many rows.
hipError_t launch_eval_per_client(const EvalArgs &a, hipStream_t s)
{
    const int groups = (a.t.n + 255) / 256;
    hipLaunchKernelGGL(k_eval_per_client, dim3((unsigned)((int64_t)a.P * groups)), dim3(256), 0,
                       s, a, groups);
    return hipGetLastError();
}

}  // namespace pmp
