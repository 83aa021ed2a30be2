// Learned swap proposal (not in the paper): feature gathering, candidate
// scoring on the MFMA units, ranking, and the first scored swap of every
// chromosome; plus the per-instance static feature sums.
//
// k_propose runs once per generation, after the crossover stages, with one
// workgroup per chromosome:
//  1. C swap candidates (j open, k closed): candidate t draws r_j uniform in
//     [0, p) and r_k uniform in [0, m - p) from its own Philox stream
//     (tag TAG_PROPOSE, stage t) and takes the r_j-th open and the r_k-th
//     closed facility in index order;
//  2. one walk over all clients gathers the slot sums of the (at most 2C)
//     candidate facilities (learn_device.hpp);
//  3. input row t = [16 features of j_t | 16 features of k_t] in BF16, and
//     the network's score (the predicted normalised change of the cost);
//  4. candidates are ranked by score (ties: lower t); mutation attempt a < L
//     takes rank a, or with probability explore/1000 (draws of stream
//     TAG_EXPLORE, stage a) a candidate drawn uniformly;
//  5. the attempts' swaps and input rows go to the GA (swap list, replay
//     ring), and attempt 0's offspring is written for evaluation.
#include "learn_device.hpp"
#include "ga_device.hpp"
#include "mlp.hpp"

namespace pmp {

namespace {

constexpr int kLearnWaves = 8;   // walk the clients
constexpr int kMlpWaves = 4;     // score the 64 candidate rows (16 rows each)
constexpr int kLearnThreads = 64 * kLearnWaves;
constexpr int kPrefetch = 8;     // clients in flight per wave

// Position of the set bit of x that has exactly r set bits below it.
__device__ __forceinline__ int select_bit(uint64_t x, int r)
{
    int b = 0;
#pragma unroll
    for (int step = 32; step > 0; step >>= 1) {
        const int t = b + step;
        if (t <= 63 && __builtin_popcountll(x & ((1ull << t) - 1ull)) <= r)
            b = t;
    }
    return b;
}

// Walk every client of the instance.  Wave w takes the clients w + kLearnWaves
// * (kPrefetch * r + d), d < kPrefetch, in batches of kPrefetch: the first
// chunk of every client of the next batch is loaded while the current batch
// is walked (the walk is bound by the latency of these loads).  The loads are
// unconditional, at a clamped row and column that are always in bounds, so
// none of them has to complete before its value is used.  Returns the wave's
// summed c1 (wave-uniform); *bad if some row has no open facility.
template <class SlotFn>
__device__ __forceinline__ long long scan_all(const Tables &t, const uint32_t *smask,
                                              const SlotFn &slot, SlotBins &B, int wave,
                                              int lane, bool *bad)
{
    constexpr int step = kLearnWaves * kPrefetch;
    long long f = 0;
    const int col = lane < t.K ? lane : t.K - 1;
    const int last = t.n - 1;
    // Row offsets are computed in vector registers (the row index is copied
    // into one): per client a multiply-add there instead of several 64-bit
    // scalar instructions, which the walk is short of.
    auto entry = [&](int i) -> int64_t {
        int iv;
        asm volatile("v_mov_b32 %0, %1" : "=v"(iv) : "s"(i));
        return (int64_t)min(iv, last) * t.pitch + col;
    };
    int fac[kPrefetch];
    int32_t dist[kPrefetch];
#pragma unroll
    for (int d = 0; d < kPrefetch; ++d) {
        const int64_t e = entry(wave + kLearnWaves * d);
        fac[d] = t.pi[e];
        dist[d] = t.ds[e];
    }
    for (int i0 = wave; i0 < t.n; i0 += step) {
        int nfac[kPrefetch];
        int32_t ndist[kPrefetch];
#pragma unroll
        for (int d = 0; d < kPrefetch; ++d) {
            const int64_t e = entry(i0 + step + kLearnWaves * d);
            nfac[d] = t.pi[e];
            ndist[d] = t.ds[e];
        }
#pragma unroll
        for (int d = 0; d < kPrefetch; ++d) {
            const int i = i0 + kLearnWaves * d;
            if (i < t.n) {
                const int32_t c1 = scan_client(t, i, fac[d], dist[d], smask, slot, B, lane);
                if (c1 < 0)
                    *bad = true;
                else
                    f += c1;
            }
        }
#pragma unroll
        for (int d = 0; d < kPrefetch; ++d) {
            fac[d] = nfac[d];
            dist[d] = ndist[d];
        }
    }
    return f;
}

struct FacSlot {  // features of facilities base .. base + kSlots - 1
    int base;
    __device__ __forceinline__ int operator()(int f) const
    {
        const int s = f - base;
        return (s >= 0 && s < kSlots) ? s : -1;
    }
};

struct MapSlot {  // slot table in LDS (0xFF: none)
    const uint8_t *map;
    __device__ __forceinline__ int operator()(int f) const
    {
        const int s = map[f];
        return s == 0xFF ? -1 : s;
    }
};

// Block-wide sum of the waves' costs.
__device__ __forceinline__ long long block_cost(long long f, long long *sf, int wave,
                                                int lane)
{
    if (lane == 0)
        sf[wave] = f;
    __syncthreads();
    long long tot = 0;
    for (int w = 0; w < kLearnWaves; ++w)
        tot += sf[w];
    return tot;
}

// Features of every facility: block (c, q) takes chromosome c and
// facilities 128q .. 128q + 127.
__global__ __launch_bounds__(kLearnThreads) void k_features(Tables t, const uint64_t *masks,
                                                            FeatCtx ctx, float *out,
                                                            uint32_t *err)
{
    __shared__ uint64_t smask[kMaxWords];
    __shared__ SlotBins B;
    __shared__ long long sf[kLearnWaves];
    __shared__ int scount, sbad;
    const int c = blockIdx.x, q = blockIdx.y;
    const int wave = wave_id(), lane = threadIdx.x & 63;
    bins_clear(B);
    if (threadIdx.x == 0)
        sbad = 0;
    if (!load_mask(masks + (int64_t)c * t.W, t.W, t.m, t.p, smask, &scount)) {
        if (threadIdx.x == 0)
            atomicOr(err, ERR_POPCOUNT);
        return;
    }
    bool bad = false;
    const long long f = scan_all(t, reinterpret_cast<const uint32_t *>(smask),
                                 FacSlot{q * kSlots}, B, wave, lane, &bad);
    if (bad)
        sbad = 1;
    ctx.f = block_cost(f, sf, wave, lane);
    if (sbad) {
        if (threadIdx.x == 0)
            atomicOr(err, ERR_SCAN_OVERRUN);
        return;
    }
    const int j = q * kSlots + (int)threadIdx.x;
    if (threadIdx.x < kSlots && j < t.m) {
        float v[kFeatures];
        const bool open = (smask[j >> 6] >> (j & 63)) & 1ull;
        features16(ctx, B, (int)threadIdx.x, j, open, v);
        float *o = out + ((int64_t)c * t.m + j) * kFeatures;
#pragma unroll
        for (int k = 0; k < kFeatures; ++k)
            o[k] = v[k];
    }
}

struct ProposeLds {
    uint64_t smask[kMaxWords / 2];  // m <= PMP_MAX_LEARNED_FACILITIES
    uint8_t slotmap[PMP_MAX_LEARNED_FACILITIES];
    SlotBins B;
    int32_t pre[kMaxWords / 2];     // inclusive prefix of open counts per word
    int32_t cj[PMP_MAX_CANDIDATES], ck[PMP_MAX_CANDIDATES];
    int32_t order[PMP_MAX_CANDIDATES];
    float score[PMP_MAX_CANDIDATES];
    __align__(16) uint16_t x[PMP_MAX_CANDIDATES * kXStride];
    __align__(16) uint16_t h[kMlpWaves][16 * kHStride];
    long long sf[kLearnWaves];
    int scount, sbad;
};

__global__ __launch_bounds__(kLearnThreads) void k_propose(LearnArgs A, int in)
{
    __shared__ ProposeLds L;
    const GaArgs &g = A.g;
    const int c = blockIdx.x;
    if (c >= g.P || ga_stopped(g))
        return;
    const int out = in ^ 1;
    const int wave = wave_id(), lane = threadIdx.x & 63;
    const Tables &t = g.t;
    const int W = t.W, m = t.m, p = t.p, C = A.C;
    const uint64_t gen = g.gs[GS_GEN];

    bins_clear(L.B);
    for (int f = threadIdx.x; f < m; f += blockDim.x)
        L.slotmap[f] = 0xFF;
    if (threadIdx.x == 0)
        L.sbad = 0;
    const uint64_t *mask = buf(g.cur, out) + (int64_t)c * W;
    if (!load_mask(mask, W, m, p, L.smask, &L.scount)) {
        if (threadIdx.x == 0)
            atomicOr(g.err, ERR_POPCOUNT);
        return;
    }
    // 1. candidates (wave 0; lane t draws candidate t)
    if (wave == 0) {
        const uint32_t pc = lane < W ? (uint32_t)__builtin_popcountll(L.smask[lane]) : 0u;
        const uint32_t inc = wave_scan_incl(pc, lane);
        if (lane < W)
            L.pre[lane] = (int32_t)inc;
        wave_lds_sync();
        if (lane < C) {
            PhiloxStream st(g.seed, ROLE_EVOLVE, gen, (uint64_t)c, TAG_PROPOSE,
                            (uint64_t)lane);
            const int rj = (int)st.below((uint64_t)p);
            const int rk = (int)st.below((uint64_t)(m - p));
            // r_j-th open facility: first word whose inclusive count exceeds r_j
            int lo = 0, hi = W - 1;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (L.pre[mid] > rj)
                    hi = mid;
                else
                    lo = mid + 1;
            }
            const int j = lo * 64 + select_bit(L.smask[lo], rj - (lo ? L.pre[lo - 1] : 0));
            // r_k-th closed facility
            lo = 0;
            hi = W - 1;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (min(64 * (mid + 1), m) - L.pre[mid] > rk)
                    hi = mid;
                else
                    lo = mid + 1;
            }
            const int before = lo ? 64 * lo - L.pre[lo - 1] : 0;
            const int nbits = min(64, m - 64 * lo);
            const uint64_t valid = nbits == 64 ? ~0ull : ((1ull << nbits) - 1ull);
            const int k = lo * 64 + select_bit(~L.smask[lo] & valid, rk - before);
            L.cj[lane] = j;
            L.ck[lane] = k;
            L.slotmap[j] = (uint8_t)(2 * lane);
            L.slotmap[k] = (uint8_t)(2 * lane + 1);
        }
    }
    __syncthreads();
    // 2. gather
    bool bad = false;
    const long long f = scan_all(t, reinterpret_cast<const uint32_t *>(L.smask),
                                 MapSlot{L.slotmap}, L.B, wave, lane, &bad);
    if (bad)
        L.sbad = 1;
    FeatCtx ctx;
    ctx.n = t.n;
    ctx.m = m;
    ctx.p = p;
    ctx.near_len = A.near_len;
    ctx.total = A.total;
    ctx.colsum = A.colsum;
    ctx.nearc = A.nearc;
    ctx.gen_frac = (float)((double)gen / (double)g.generations);
    ctx.f = block_cost(f, L.sf, wave, lane);
    if (L.sbad) {
        if (threadIdx.x == 0)
            atomicOr(g.err, ERR_SCAN_OVERRUN);
        return;
    }
    // 3. input rows: thread (row, quarter) writes 8 inputs
    if (threadIdx.x < 4 * PMP_MAX_CANDIDATES) {
        const int row = threadIdx.x >> 2, qtr = threadIdx.x & 3;
        uint16_t v8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        if (row < C) {
            const int fac = qtr < 2 ? L.cj[row] : L.ck[row];
            const int sl = L.slotmap[fac];
            float v[kFeatures];
            features16(ctx, L.B, sl == 0xFF ? -1 : sl, fac, qtr < 2, v);
#pragma unroll
            for (int e = 0; e < 8; ++e)
                v8[e] = f32_to_bf16(v[(qtr & 1) * 8 + e]);
        }
        uint2 *d = reinterpret_cast<uint2 *>(L.x + row * kXStride + qtr * 8);
        d[0] = uint2{v8[0] | ((uint32_t)v8[1] << 16), v8[2] | ((uint32_t)v8[3] << 16)};
        d[1] = uint2{v8[4] | ((uint32_t)v8[5] << 16), v8[6] | ((uint32_t)v8[7] << 16)};
    }
    __syncthreads();
    // scores (16 rows per wave)
    if (wave < kMlpWaves) {
        f32x4 z1[8], z2[8];
        float y[4];
        mlp_forward16(A.net, L.x + wave * 16 * kXStride, L.h[wave], lane, z1, z2, y);
        if ((lane & 15) == 0)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                L.score[wave * 16 + 4 * (lane >> 4) + i] = y[i];
    }
    __syncthreads();
    // 4. rank (wave 0): rank of t = #{u : (y_u, u) < (y_t, t)}, NaN as +inf
    if (wave == 0) {
        float y = lane < C ? L.score[lane] : __builtin_inff();
        if (lane < C)
            A.scores[(int64_t)c * C + lane] = y;
        if (y != y)
            y = __builtin_inff();
        int rank = 0;
        for (int u = 0; u < 64; ++u) {
            const float yu = __shfl(y, u);
            rank += (yu < y || (yu == y && u < lane)) ? 1 : 0;
        }
        if (lane < C)
            L.order[rank] = lane;
        wave_lds_sync();
        // 5. the attempts' picks, swaps and replay rows
        if (lane < A.L) {
            PhiloxStream st(g.seed, ROLE_EVOLVE, gen, (uint64_t)c, TAG_EXPLORE,
                            (uint64_t)lane);
            const int e = (int)st.below(1000);
            const int u = (int)st.below((uint64_t)C);
            const int pick = e < A.explore ? u : L.order[lane];
            const int j = L.cj[pick], k = L.ck[pick];
            int32_t *sw = A.swaps + ((int64_t)c * A.L + lane) * 2;
            sw[0] = j;
            sw[1] = k;
            const int64_t slot =
                ((int64_t)(gen % (uint64_t)A.H) * A.L + lane) * g.P + c;
            const uint2 *src = reinterpret_cast<const uint2 *>(L.x + pick * kXStride);
            uint2 *dst = reinterpret_cast<uint2 *>(A.rep_x + slot * kIn);
#pragma unroll
            for (int w = 0; w < kIn / 4; ++w)
                dst[w] = src[w];
            A.rep_jk[slot * 2] = j;
            A.rep_jk[slot * 2 + 1] = k;
            A.rep_d[slot * 2] = 0;
            A.rep_d[slot * 2 + 1] = ctx.f;
            A.rep_t[slot] = 0.f;
            A.rep_w[slot] = 0.f;
        }
    }
    __syncthreads();
    // attempt 0's offspring
    const int32_t *sw0 = A.swaps + (int64_t)c * A.L * 2;
    const int j0 = sw0[0], k0 = sw0[1];
    uint64_t *F = buf(g.off, out) + (int64_t)c * W;
    for (int w = threadIdx.x; w < W; w += blockDim.x) {
        uint64_t v = L.smask[w];
        if ((j0 >> 6) == w)
            v ^= 1ull << (j0 & 63);
        if ((k0 >> 6) == w)
            v ^= 1ull << (k0 & 63);
        F[w] = v;
    }
    if (threadIdx.x == 0)
        buf(g.ok, out)[c] = 1;
}

// Column sums of d (int64), rows split over gridDim.y slices.
__global__ void k_colsum(const int32_t *d, int64_t ld, int n, int m,
                         unsigned long long *colsum)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m)
        return;
    const int per = (n + gridDim.y - 1) / gridDim.y;
    const int i0 = blockIdx.y * per, i1 = min(n, i0 + per);
    unsigned long long s = 0;
    for (int i = i0; i < i1; ++i)
        s += (unsigned long long)(uint32_t)d[(int64_t)i * ld + j];
    if (i1 > i0)
        atomicAdd(colsum + j, s);
}

// near_j = #{i : j among the first L entries of Pi'_i}.
__global__ void k_near(const uint16_t *pi, int pitch, int n, int L, uint32_t *nearc)
{
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= (int64_t)n * L)
        return;
    const int64_t i = x / L, s = x - i * L;
    atomicAdd(nearc + pi[i * pitch + s], 1u);
}

}  // namespace

hipError_t launch_features(const Tables &t, const uint64_t *masks, int P, const FeatCtx &ctx,
                           float *out, uint32_t *err, hipStream_t s)
{
    if (P <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_features, dim3(P, (t.m + kSlots - 1) / kSlots), dim3(kLearnThreads),
                       0, s, t, masks, ctx, out, err);
    return hipGetLastError();
}

hipError_t launch_propose(const LearnArgs &a, int in, hipStream_t s)
{
    hipLaunchKernelGGL(k_propose, dim3(a.g.P), dim3(kLearnThreads), 0, s, a, in);
    return hipGetLastError();
}

hipError_t launch_static_sums(const int32_t *d, int64_t ld, int n, int m, const uint16_t *pi,
                              int pitch, int L, unsigned long long *colsum, uint32_t *nearc,
                              hipStream_t s)
{
    const int slices = n < 64 ? n : 64;
    hipLaunchKernelGGL(k_colsum, dim3((m + 255) / 256, slices), dim3(256), 0, s, d, ld, n, m,
                       colsum);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    const int64_t cells = (int64_t)n * L;
    hipLaunchKernelGGL(k_near, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0, s, pi,
                       pitch, n, L, nearc);
    return hipGetLastError();
}

}  // namespace pmp
