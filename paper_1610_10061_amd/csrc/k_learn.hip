// Learned swap proposal (not in the paper), once per generation after the
// crossover stages, in three launches:
//  1. k_prop_cand: C swap candidates per chromosome (j open, k closed):
//     candidate t draws r_j uniform in [0, p) and r_k uniform in [0, m - p)
//     from its own Philox stream (tag TAG_PROPOSE, stage t) and takes the
//     r_j-th open and the r_k-th closed facility in index order;
//  2. k_prop_walk: one walk over all clients gathers the slot sums of the
//     (at most 2C) candidate facilities of every chromosome
//     (learn_device.hpp);
//  3. k_prop_score: input row t = [16 features of j_t | 16 features of k_t]
//     in BF16 and the network's score (the predicted normalised change of
//     the cost); candidates ranked by score (ties: lower t); mutation
//     attempt a < L takes rank a or, with probability explore/1000 (draws of
//     stream TAG_EXPLORE, stage a), a candidate drawn uniformly; the swaps
//     and input rows go to the GA (swap list, training ring), and attempt
//     0's offspring is written for evaluation.
// Also here: the full feature table of pmp_features and the per-instance
// static sums.
#include "eval_device.hpp"
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

// ---------------------------------------------------------------------------
// Proposal, step 1 (one wave per chromosome): the C candidates and the bitmap
// of candidate facilities with the number of candidate facilities before
// each of its words (a facility's slot is that count plus the candidate bits
// below it in its word).
// ---------------------------------------------------------------------------
constexpr int kCandWaves = 4;

__global__ __launch_bounds__(64 * kCandWaves) void k_prop_cand(LearnArgs A, int out)
{
    __shared__ unsigned long long sb[kCandWaves][64];
    const GaArgs &g = A.g;
    const int wave = wave_id(), lane = threadIdx.x & 63;
    const int c = blockIdx.x * kCandWaves + wave;
    if (c >= g.P)
        return;
    const Tables &t = g.t;
    const int W = t.W, m = t.m, p = t.p, C = A.C;
    const uint64_t gen = g.gs[GS_GEN];
    const uint64_t w0 = buf(g.cur, out)[(int64_t)c * W + min(lane, W - 1)];
    if (ga_stopped(g))
        return;
    const uint64_t word = lane < W ? w0 : 0ull;
    const uint32_t inc = wave_scan_incl((uint32_t)__builtin_popcountll(word), lane);
    // closed facilities up to and including word w
    const int nbits = lane < W ? min(64, m - 64 * lane) : 0;
    const uint32_t cinc = (uint32_t)min(64 * (lane + 1), m) - inc;
    const uint64_t valid = nbits >= 64 ? ~0ull : ((1ull << nbits) - 1ull);
    const uint64_t cword = ~word & valid;

    PhiloxStream st(g.seed, ROLE_EVOLVE, gen, (uint64_t)c, TAG_PROPOSE, (uint64_t)lane);
    const uint32_t rj = (uint32_t)st.below((uint64_t)p);
    const uint32_t rk = (uint32_t)st.below((uint64_t)(m - p));
    // first word whose inclusive count exceeds the rank (every lane takes part
    // in every shuffle)
    int wj = 0, wk = 0;
#pragma unroll
    for (int b = 32; b > 0; b >>= 1) {
        const int qj = min(wj + b - 1, 63), qk = min(wk + b - 1, 63);
        const uint32_t vj = (uint32_t)__shfl((int)inc, qj);
        const uint32_t vk = (uint32_t)__shfl((int)cinc, qk);
        if (wj + b - 1 < W && vj <= rj)
            wj += b;
        if (wk + b - 1 < W && vk <= rk)
            wk += b;
    }
    wj = min(wj, W - 1);
    wk = min(wk, W - 1);
    // unconditional shuffles (a lane outside the active set reads as 0)
    const uint32_t pj = (uint32_t)__shfl((int)inc, max(wj - 1, 0));
    const uint32_t pk = (uint32_t)__shfl((int)cinc, max(wk - 1, 0));
    const uint32_t bj = wj > 0 ? pj : 0u;
    const uint32_t bk = wk > 0 ? pk : 0u;
    const uint64_t xj = (uint64_t)(uint32_t)__shfl((int)(uint32_t)word, wj) |
                        ((uint64_t)(uint32_t)__shfl((int)(uint32_t)(word >> 32), wj) << 32);
    const uint64_t xk = (uint64_t)(uint32_t)__shfl((int)(uint32_t)cword, wk) |
                        ((uint64_t)(uint32_t)__shfl((int)(uint32_t)(cword >> 32), wk) << 32);
    const int j = wj * 64 + select_bit(xj, (int)(rj - bj));
    const int k = wk * 64 + select_bit(xk, (int)(rk - bk));

    // candidate-facility bitmap
    sb[wave][lane] = 0ull;
    wave_lds_sync();
    if (lane < C) {
        atomicOr(&sb[wave][j >> 6], 1ull << (j & 63));
        atomicOr(&sb[wave][k >> 6], 1ull << (k & 63));
        int32_t *cd = A.cand + ((int64_t)c * C + lane) * 2;
        cd[0] = j;
        cd[1] = k;
    }
    wave_lds_sync();
    const uint64_t cb = sb[wave][lane];
    const uint32_t cpc = (uint32_t)__builtin_popcountll(cb);
    const uint32_t cex = wave_scan_incl(cpc, lane) - cpc;
    if (lane < W) {
        A.cbits[(int64_t)c * W + lane] = cb;
        A.cpre[(int64_t)c * W + lane] = (uint8_t)cex;
    }
}

// ---------------------------------------------------------------------------
// Proposal, step 2: the walk.  A workgroup takes CH chromosomes
// (masks, candidate bitmaps, slot bases and slot sums in LDS) and every
// client; each of its NW waves takes clients wave, wave + NW, ...,
// the first 64-entry chunk of kWalkAhead clients in flight.  Lane l holds
// entry l of the chunk; for each chromosome one LDS read per lane and a
// ballot give the open positions in the chunk; with two or more, s1 and s2
// are the two lowest, and the lanes up to s2 whose facility is a candidate
// of that chromosome add their terms to its slot sums (LDS integer atomics:
// deterministic).  Rows with fewer than two open facilities in the first
// chunk take the general path.  The sums are stored once at the end.
// ---------------------------------------------------------------------------
constexpr int kWalkAhead = 4;

template <int CH>
struct WalkLds {
    uint64_t mask[CH][kMaxWords / 2];
    uint64_t cb[CH][kMaxWords / 2];
    uint8_t cp[CH][kMaxWords / 2];
    SlotBins bins[CH];
};

template <int CH>
__device__ __forceinline__ int walk_slot(const WalkLds<CH> &L, int g, int fac)
{
    const uint64_t w = L.cb[g][fac >> 6];
    const int fb = fac & 63;
    return ((w >> fb) & 1ull) ? L.cp[g][fac >> 6] + __builtin_popcountll(w & ((1ull << fb) - 1ull))
                              : -1;
}

template <int CH>
struct SlotFnLds {  // slot of a facility for chromosome g of the walk's LDS
    const WalkLds<CH> *L;
    int g;
    __device__ __forceinline__ int operator()(int f) const { return walk_slot(*L, g, f); }
};

// CH chromosomes per workgroup, NW waves.
template <int CH, int NW>
__global__ __launch_bounds__(64 * NW) void k_prop_walk(LearnArgs A, int out)
{
    __shared__ WalkLds<CH> L;
    const GaArgs &g = A.g;
    const Tables &t = g.t;
    const int c0 = blockIdx.x * CH, rows = min(CH, g.P - c0);
    const int lane = threadIdx.x & 63, wave = wave_id();
    const int W = t.W, K = t.K;
    // loads first: masks, bitmaps, slot bases (clamped, unconditional) and
    // the first clients' chunks
    const uint64_t *cur = buf(g.cur, out);
    for (int e = threadIdx.x; e < CH * (kMaxWords / 2); e += (64 * NW)) {
        const int cc = e / (kMaxWords / 2), w = e - cc * (kMaxWords / 2);
        const int64_t src = (int64_t)(c0 + min(cc, rows - 1)) * W + min(w, W - 1);
        const uint64_t mv = cur[src], cv = A.cbits[src];
        const uint8_t pv = A.cpre[src];
        const bool in = cc < rows && w < W;
        L.mask[cc][w] = in ? mv : 0ull;
        L.cb[cc][w] = in ? cv : 0ull;
        L.cp[cc][w] = in ? pv : (uint8_t)0;
    }
    for (int e = threadIdx.x; e < CH * kSlots; e += (64 * NW)) {
        SlotBins &B = L.bins[e / kSlots];
        const int sl = e % kSlots;
        B.a[sl] = 0;
        B.dd[sl] = 0;
        B.b[sl] = 0;
        B.cc[sl] = 0;
        B.e[sl] = 0;
    }
    const int col = lane < K ? lane : K - 1;
    const int last = t.n - 1;
    constexpr int step = NW * kWalkAhead;
    int fac[kWalkAhead];
    int32_t dist[kWalkAhead];
#pragma unroll
    for (int d = 0; d < kWalkAhead; ++d) {
        const int64_t e = (int64_t)min(wave + NW * d, last) * t.pitch + col;
        fac[d] = t.pi[e];
        dist[d] = t.ds[e];
    }
    if (ga_stopped(g))
        return;
    __syncthreads();
    const bool valid = lane < K;
    for (int i0 = wave; i0 < t.n; i0 += step) {
        // this batch's operands (loaded one batch ago), taken before the next
        // batch's loads are issued so that no wait falls inside the work
        int fw[kWalkAhead], fb[kWalkAhead];
        int32_t dv[kWalkAhead];
#pragma unroll
        for (int d = 0; d < kWalkAhead; ++d) {
            fw[d] = fac[d] >> 6;
            fb[d] = fac[d] & 63;
            dv[d] = dist[d];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int d = 0; d < kWalkAhead; ++d) {
            const int64_t e = (int64_t)min(i0 + step + NW * d, last) * t.pitch + col;
            fac[d] = t.pi[e];
            dist[d] = t.ds[e];
        }
        uint32_t slow = 0;  // (client d, chromosome cc) pairs for the general path
#pragma unroll
        for (int d = 0; d < kWalkAhead; ++d) {
            if (i0 + NW * d >= t.n)
                break;
            const uint64_t below = (1ull << fb[d]) - 1ull;
            for (int cc = 0; cc < rows; ++cc) {
                const uint64_t mw = L.mask[cc][fw[d]];
                const uint64_t cw = L.cb[cc][fw[d]];
                const int cpv = L.cp[cc][fw[d]];
                const bool open = (((mw >> fb[d]) & 1ull) != 0ull) & valid;
                const uint64_t bits = __builtin_amdgcn_ballot_w64(open);
                const uint64_t rest = bits & (bits - 1ull);
                if (rest == 0ull) {
                    slow |= 1u << (d * CH + cc);
                    continue;
                }
                const int s1 = (int)__builtin_ctzll(bits);
                const int s2 = (int)__builtin_ctzll(rest);
                const int32_t c1 = __builtin_amdgcn_readlane(dv[d], s1);
                const int32_t c2 = __builtin_amdgcn_readlane(dv[d], s2);
                const bool hit = (((cw >> fb[d]) & 1ull) != 0ull) & (lane <= s2);
                if (hit) {
                    const int sl = cpv + __builtin_popcountll(cw & below);
                    SlotBins &B = L.bins[cc];
                    const bool upto1 = lane <= s1, first = lane == s1, second = lane == s2;
                    int32_t v = c2 - dv[d];           // between
                    v = second ? c2 - c1 : v;
                    v = first ? c1 : v;
                    v = lane < s1 ? c1 - dv[d] : v;   // ahead
                    atomicAdd(upto1 ? &B.a[sl] : &B.dd[sl], 1u);
                    atomicAdd(upto1 ? &B.b[sl] : (second ? &B.e[sl] : &B.cc[sl]),
                              (unsigned long long)v);
                    atomicAdd(&B.cc[sl], first ? (unsigned long long)(c2 - c1) : 0ull);
                }
            }
        }
        // rows whose second open facility lies past the first chunk (rare)
        while (slow) {
            const int bit = (int)__builtin_ctz(slow);
            slow &= slow - 1u;
            const int d = bit / CH, cc = bit - d * CH;
            int32_t dcur = dv[0];
            int fcur = fw[0] * 64 + fb[0];
#pragma unroll
            for (int q = 1; q < kWalkAhead; ++q)
                if (q == d) {
                    dcur = dv[q];
                    fcur = fw[q] * 64 + fb[q];
                }
            const SlotFnLds<CH> fn{&L, cc};
            if (scan_client(t, i0 + NW * d, fcur, dcur,
                            reinterpret_cast<const uint32_t *>(L.mask[cc]), fn, L.bins[cc],
                            lane) < 0 &&
                lane == 0)
                atomicOr(g.err, ERR_SCAN_OVERRUN);
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < rows * kSlots; e += (64 * NW)) {
        const SlotBins &B = L.bins[e / kSlots];
        const int sl = e % kSlots;
        const int64_t o = (int64_t)(c0 + e / kSlots) * kSlots + sl;
        A.sums.a[o] = B.a[sl];
        A.sums.dd[o] = B.dd[sl];
        A.sums.b[o] = B.b[sl];
        A.sums.cc[o] = B.cc[sl];
        A.sums.e[o] = B.e[sl];
    }
}

// ---------------------------------------------------------------------------
// Proposal, step 3 (one workgroup per chromosome): input rows from the slot
// sums, scores, ranking, the attempts' picks, ring rows and attempt 0's
// offspring.
// ---------------------------------------------------------------------------
struct ScoreLds {
    uint64_t cb[kMaxWords / 2];
    uint8_t cp[kMaxWords / 2];
    int32_t cj[PMP_MAX_CANDIDATES], ck[PMP_MAX_CANDIDATES];
    int32_t order[PMP_MAX_CANDIDATES];
    float score[PMP_MAX_CANDIDATES];
    __align__(16) uint16_t x[PMP_MAX_CANDIDATES * kXStride];
    __align__(16) uint16_t h[PMP_MAX_CANDIDATES * kHStride];
    float ys[PMP_MAX_CANDIDATES * 4];  // per row, the four tile pairs' output sums
    int32_t prank[kMlpWaves][PMP_MAX_CANDIDATES];  // partial ranks by quarter
    int32_t pe[PMP_MAX_CANDIDATES], pu[PMP_MAX_CANDIDATES];  // exploration draws
    int32_t swap0[2];                                     // attempt 0's (j, k)
};

__global__ __launch_bounds__(64 * kMlpWaves) void k_prop_score(LearnArgs A, int out)
{
    __shared__ ScoreLds L;
    const GaArgs &g = A.g;
    const int c = blockIdx.x;
    const Tables &t = g.t;
    const int W = t.W, C = A.C;
    const int wave = wave_id(), lane = threadIdx.x & 63;
    const uint64_t gen = g.gs[GS_GEN];
    const unsigned long long f = buf(g.fit, out)[c];
    if (threadIdx.x < W) {
        L.cb[threadIdx.x] = A.cbits[(int64_t)c * W + threadIdx.x];
        L.cp[threadIdx.x] = A.cpre[(int64_t)c * W + threadIdx.x];
    }
    if (threadIdx.x < C) {
        L.cj[threadIdx.x] = A.cand[((int64_t)c * C + threadIdx.x) * 2];
        L.ck[threadIdx.x] = A.cand[((int64_t)c * C + threadIdx.x) * 2 + 1];
    }
    if (ga_stopped(g))
        return;
    __syncthreads();
    FeatCtx ctx;
    ctx.n = t.n;
    ctx.m = t.m;
    ctx.p = t.p;
    ctx.near_len = A.near_len;
    ctx.total = A.total;
    ctx.colsum = A.colsum;
    ctx.nearc = A.nearc;
    ctx.gen_frac = (float)((double)gen / (double)g.generations);
    ctx.f = (int64_t)f;
    // input rows: thread (row, quarter) writes 8 inputs; j is open, k closed
    {
        const int row = threadIdx.x >> 2, qtr = threadIdx.x & 3;
        uint16_t v8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        if (row < C) {
            const int fac = qtr < 2 ? L.cj[row] : L.ck[row];
            const uint64_t w = L.cb[fac >> 6];
            const int sl = L.cp[fac >> 6] + __builtin_popcountll(w & ((1ull << (fac & 63)) - 1ull));
            const int64_t o = (int64_t)c * kSlots + sl;
            float v[8];
            features8_sums(ctx, (double)A.sums.a[o], (double)A.sums.dd[o], (double)A.sums.b[o],
                           (double)A.sums.cc[o], (double)A.sums.e[o], fac, qtr < 2, qtr & 1, v);
#pragma unroll
            for (int e = 0; e < 8; ++e)
                v8[e] = f32_to_bf16(v[e]);
        }
        uint2 *d = reinterpret_cast<uint2 *>(L.x + row * kXStride + qtr * 8);
        d[0] = uint2{v8[0] | ((uint32_t)v8[1] << 16), v8[2] | ((uint32_t)v8[3] << 16)};
        d[1] = uint2{v8[4] | ((uint32_t)v8[5] << 16), v8[6] | ((uint32_t)v8[7] << 16)};
    }
    __syncthreads();
    mlp_forward64(A.net, L.x, L.h, L.ys, wave, lane);
    __syncthreads();
    if (threadIdx.x < PMP_MAX_CANDIDATES)
        L.score[threadIdx.x] = out_sum(L.ys + threadIdx.x * 4, A.net.b3[0]);
    __syncthreads();
    static_assert(kMlpWaves * 16 == PMP_MAX_CANDIDATES, "a quarter of the candidates per wave");
    // rank of t = #{u : (y_u, u) < (y_t, t)}, NaN as +inf: wave v counts
    // the u of the quarter 16 v .. 16 v + 15 for every t; wave 1 also makes
    // the attempts' exploration draws
    {
        float y = lane < C ? L.score[lane] : __builtin_inff();
        if (y != y)
            y = __builtin_inff();
        int cnt = 0;
#pragma unroll
        for (int uu = 0; uu < 16; ++uu) {
            const int u = wave * 16 + uu;
            float yu = u < C ? L.score[u] : __builtin_inff();
            if (yu != yu)
                yu = __builtin_inff();
            cnt += (yu < y || (yu == y && u < lane)) ? 1 : 0;
        }
        L.prank[wave][lane] = cnt;
        if (wave == 1 && lane < A.L) {
            PhiloxStream st(g.seed, ROLE_EVOLVE, gen, (uint64_t)c, TAG_EXPLORE, (uint64_t)lane);
            L.pe[lane] = (int)st.below(1000);
            L.pu[lane] = (int)st.below((uint64_t)C);
        }
    }
    __syncthreads();
    if (wave == 0) {
        if (lane < C)
            A.scores[(int64_t)c * C + lane] = L.score[lane];
        const int rank = L.prank[0][lane] + L.prank[1][lane] + L.prank[2][lane] + L.prank[3][lane];
        if (lane < C)
            L.order[rank] = lane;
        wave_lds_sync();
        // the attempts' picks, swaps and ring rows
        if (lane < A.L) {
            const int pick = L.pe[lane] < A.explore ? L.pu[lane] : L.order[lane];
            const int j = L.cj[pick], k = L.ck[pick];
            int32_t *sw = A.swaps + ((int64_t)c * A.L + lane) * 2;
            sw[0] = j;
            sw[1] = k;
            if (lane == 0) {
                L.swap0[0] = j;
                L.swap0[1] = k;
            }
            const int64_t slot = ((int64_t)(gen % (uint64_t)A.H) * A.L + lane) * g.P + c;
            const uint2 *src = reinterpret_cast<const uint2 *>(L.x + pick * kXStride);
            uint2 *dst = reinterpret_cast<uint2 *>(A.rep_x + slot * kIn);
#pragma unroll
            for (int w = 0; w < kIn / 4; ++w)
                dst[w] = src[w];
            A.rep_jk[slot * 2] = j;
            A.rep_jk[slot * 2 + 1] = k;
            A.rep_d[slot * 2] = 0;
            A.rep_d[slot * 2 + 1] = (long long)f;
            A.rep_t[slot] = 0.f;
            A.rep_w[slot] = 0.f;
        }
    }
    __syncthreads();
    // attempt 0's offspring
    const int j0 = L.swap0[0], k0 = L.swap0[1];
    const uint64_t *mask = buf(g.cur, out) + (int64_t)c * W;
    uint64_t *F = buf(g.off, out) + (int64_t)c * W;
    for (int w = threadIdx.x; w < W; w += blockDim.x) {
        uint64_t v = mask[w];
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

// report[0] = sum of the column sums, report[1] = the error word (one
// workgroup).
__global__ __launch_bounds__(256) void k_total(const unsigned long long *colsum, int m,
                                               const uint32_t *err, unsigned long long *report)
{
    __shared__ unsigned long long part[256];
    unsigned long long t = 0;
    for (int j = threadIdx.x; j < m; j += 256)
        t += colsum[j];
    part[threadIdx.x] = t;
    __syncthreads();
    for (int half = 128; half > 0; half >>= 1) {
        if (threadIdx.x < half)
            part[threadIdx.x] += part[threadIdx.x + half];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        report[0] = part[0];
        report[1] = *err;
    }
}


// ---------------------------------------------------------------------------
// Two-pass walk (the default).  Pass 1 (k_prop_s12) uses the evaluation's
// tiling: the workgroup of a chromosome tile (64 chromosomes) and a client
// tile stages the tile's masks facility-major in LDS; a wave takes a client,
// its lanes hold the row's positions, one transpose gives lane c the open
// positions of chromosome c in the chunk, and two lowest-bit steps give s1
// and s2 (chunk after chunk until every chromosome has both or the row ends),
// their costs from the lanes holding them.  Pass 2 (k_prop_slots), a
// workgroup per chromosome: a candidate facility f's slot sums come from the
// index entries (i, k) with Pi'_i[k] = f, k < kNearL, tested against (s1, s2)
// of the chromosome and client i; positions at or past kNearL (rows whose
// second open facility lies further) are walked directly.  The sums are the
// one-pass walk's (the same integer terms, added in another order).
// ---------------------------------------------------------------------------
constexpr int kS12Waves = 16;
constexpr int kS12Clients = 64;  // clients per workgroup
constexpr int kMaxLearnWords = PMP_MAX_LEARNED_FACILITIES / 64;
constexpr int kSlotWaves = 8;
constexpr int kSlotRows = 4 * kSlotWaves;  // 16-lane rows per workgroup
constexpr int kFarCap = 256;               // listed far clients per chromosome
constexpr int kStageClients = 4096;        // (12 bytes of LDS each)

// Lowest set bit of the 64-bit (hi:lo), -1 if none.
__device__ __forceinline__ int lowest64(uint32_t lo, uint32_t hi)
{
    const uint32_t a = (uint32_t)lowest_bit(lo);
    const uint32_t b = __builtin_elementwise_add_sat((uint32_t)lowest_bit(hi), 32u);
    return (int)(a < b ? a : b);
}

__global__ __launch_bounds__(64 * kS12Waves) void k_prop_s12(LearnArgs A, int out, int tiles_c)
{
    // the rows staged at a padded stride (32-bit words), then in place the
    // facility-major words T[64 w + lane] and T[64 W] = 0: 64 (2W + 1) words
    // of dynamic LDS (s12_lds_bytes)
    extern __shared__ __align__(16) uint32_t sm[];
    // results by chromosome and client (padded rows), written out row by row
    __shared__ uint32_t o_s[kEvalTile][kS12Clients + 1];
    __shared__ int32_t o_c1[kEvalTile][kS12Clients + 1], o_c2[kEvalTile][kS12Clients + 1];
    const GaArgs &g = A.g;
    const Tables &t = g.t;
    const int W = t.W, SD = 2 * W + 1;
    const int ntiles = tiles_c * ((t.n + kS12Clients - 1) / kS12Clients);
    const int per_xcd = (int)gridDim.x >> 3;
    const int logical = ((int)blockIdx.x & 7) * per_xcd + ((int)blockIdx.x >> 3);
    if (logical >= ntiles)  // (the whole workgroup, before any barrier)
        return;
    const int ti = logical / tiles_c, tc = logical - ti * tiles_c;
    const int c0 = tc * kEvalTile, rows = min(kEvalTile, g.P - c0);
    const int i0 = ti * kS12Clients, ni = min(kS12Clients, t.n - i0);
    const int lane = threadIdx.x & 63, wave = wave_id();
    const uint32_t *g32 = reinterpret_cast<const uint32_t *>(buf(g.cur, out));
    for (int e = threadIdx.x; e < kEvalTile * 2 * W; e += 64 * kS12Waves) {
        const int c = e / (2 * W), w = e - c * (2 * W);
        const uint32_t v = g32[(int64_t)(c0 + min(c, rows - 1)) * 2 * W + w];
        sm[c * SD + w] = c < rows ? v : 0u;
    }
    // each wave's clients: their first chunks in flight with the staging
    constexpr int R = kS12Clients / kS12Waves;
    const uint32_t jz = (uint32_t)(64 * W);
    uint32_t j0[R];
    int32_t d0[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int il = wave + r * kS12Waves;
        const int i = i0 + min(il, ni - 1);
        const int kc = min(lane, t.K - 1);
        j0[r] = lane < t.K ? (uint32_t)t.pi[(int64_t)i * t.pitch + kc] : jz;
        d0[r] = t.ds[(int64_t)i * t.pitch + kc];
    }
    if (ga_stopped(g))
        return;
    __syncthreads();
    constexpr int NW = (kMaxLearnWords + kS12Waves - 1) / kS12Waves;
    uint32_t rlo[NW], rhi[NW];
#pragma unroll
    for (int r = 0; r < NW; ++r) {
        const int w = min(wave + r * kS12Waves, W - 1);
        rlo[r] = sm[lane * SD + 2 * w];
        rhi[r] = sm[lane * SD + 2 * w + 1];
    }
    __syncthreads();
    uint64_t *sT = reinterpret_cast<uint64_t *>(sm);
    const TransposeLanes tl(lane);
#pragma unroll
    for (int r = 0; r < NW; ++r) {
        const int w = wave + r * kS12Waves;
        if (w < W) {
            transpose64(rlo[r], rhi[r], lane, tl);
            sT[w * 64 + lane] = ((uint64_t)rhi[r] << 32) | rlo[r];
        }
    }
    if (threadIdx.x == 0)
        sT[64 * W] = 0ull;
    __syncthreads();
    const bool mine = lane < rows;  // lane c: chromosome c0 + c
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int il = wave + r * kS12Waves;
        if (il >= ni)  // (uniform)
            break;
        const int i = i0 + il;
        const uint16_t *prow = t.pi + (int64_t)i * t.pitch;
        const int32_t *drow = t.ds + (int64_t)i * t.pitch;
        int s1 = -1, s2 = -1;
        int32_t c1 = 0, c2 = 0;
        uint32_t j = j0[r];
        int32_t d = d0[r];
        for (int base = 0;;) {
            const uint64_t row = sT[j];
            uint32_t lo = (uint32_t)row, hi = (uint32_t)(row >> 32);
            transpose64(lo, hi, lane, tl);
            const int a = lowest64(lo, hi);
            const int32_t da = __builtin_amdgcn_ds_bpermute(a << 2, d);
            if (s1 < 0 && a >= 0) {  // the chunk's first open position is s1
                s1 = base + a;
                c1 = da;
                if (a < 32)
                    lo &= lo - 1u;
                else
                    hi &= hi - 1u;
            }
            const int b = lowest64(lo, hi);
            const int32_t db = __builtin_amdgcn_ds_bpermute(b << 2, d);
            if (s1 >= 0 && s2 < 0 && b >= 0) {
                s2 = base + b;
                c2 = db;
            }
            base += 64;
            if (base >= t.K || __builtin_amdgcn_ballot_w64(mine && s2 < 0) == 0ull)
                break;
            const int k = base + lane;
            const int kc = min(k, t.K - 1);
            j = k < t.K ? (uint32_t)prow[kc] : jz;
            d = drow[kc];
        }
        if (__builtin_amdgcn_ballot_w64(mine && s1 < 0) != 0ull && lane == 0)
            atomicOr(g.err, ERR_SCAN_OVERRUN);  // a row without an open facility
        const bool none2 = s2 < 0;
        if (mine && none2)
            c2 = drow[t.K - 1];
        o_s[lane][il] = (uint32_t)max(s1, 0) | ((uint32_t)(none2 ? 0xFFFF : s2) << 16);
        o_c1[lane][il] = c1;
        o_c2[lane][il] = c2;
    }
    __syncthreads();
    uint2 *c12 = reinterpret_cast<uint2 *>(A.c12);
    for (int e = threadIdx.x; e < kEvalTile * kS12Clients; e += 64 * kS12Waves) {
        const int c = e / kS12Clients, il = e - c * kS12Clients;
        if (c < rows && il < ni) {
            const int64_t o = (int64_t)(c0 + c) * t.n + i0 + il;
            A.s12[o] = o_s[c][il];
            c12[o] = uint2{(uint32_t)o_c1[c][il], (uint32_t)o_c2[c][il]};
        }
    }
}

// Slot of facility f among the chromosome's candidates (bitmap cb, prefix
// counts cp), -1 if f is not one.
__device__ __forceinline__ int cand_slot(const uint64_t *cb, const uint8_t *cp, int f)
{
    const uint64_t w = cb[f >> 6];
    const uint64_t bit = 1ull << (f & 63);
    return (w & bit) ? (int)cp[f >> 6] + __builtin_popcountll(w & (bit - 1ull)) : -1;
}

// Sum over each 16-lane row; lane 15 of the row ends with the total.
__device__ __forceinline__ unsigned long long row_sum64(unsigned long long v)
{
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
    dpp_add64<0x111, 0xF>(lo, hi);  // row_shr:1
    dpp_add64<0x112, 0xF>(lo, hi);  // row_shr:2
    dpp_add64<0x114, 0xF>(lo, hi);  // row_shr:4
    dpp_add64<0x118, 0xF>(lo, hi);  // row_shr:8
    return ((unsigned long long)hi << 32) | lo;
}

// Client i's (s1 | s2 << 16) and (c1, c2): from LDS when staged, else from
// device memory.
template <bool Stage>
struct RowState {
    const uint32_t *S;  // LDS when staged
    const uint2 *C;
    const uint32_t *gs;
    const uint2 *gc;
    __device__ __forceinline__ uint32_t s(int i) const
    {
        if constexpr (Stage)
            return S[i];
        else
            return gs[i];
    }
    __device__ __forceinline__ uint2 c(int i) const
    {
        if constexpr (Stage)
            return C[i];
        else
            return gc[i];
    }
};

// Positions nearL .. e2 - 1 of client ii's row (those beyond the index)
// walked by a group of `width` lanes (a 16-lane row or the whole wave; this
// lane is number `sub` of it), four steps of loads in flight per round.
__device__ __forceinline__ void walk_far(const Tables &t, SlotBins &B, const uint64_t *cb,
                                         const uint8_t *cp, int ii, uint32_t v, uint2 cc,
                                         int nearL, int sub, int width)
{
    const int s1 = (int)(v & 0xFFFFu), s2x = (int)(v >> 16);
    const int s2 = s2x == 0xFFFF ? -1 : s2x;
    const int e2 = s2 < 0 ? t.K : s2 + 1;
    const uint16_t *prow = t.pi + (int64_t)ii * t.pitch;
    const int32_t *drow = t.ds + (int64_t)ii * t.pitch;
    // four steps' loads in flight per round (clamped into the row)
    for (int p0 = nearL; p0 < e2; p0 += 4 * width) {
        int f[4];
        int32_t d[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int pos = min(p0 + u * width + sub, e2 - 1);
            f[u] = prow[pos];
            d[u] = drow[pos];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int pos = p0 + u * width + sub;
            if (pos < e2) {
                const int sl = cand_slot(cb, cp, f[u]);
                if (sl >= 0)
                    add_terms(B, sl, pos, s1, s2, (int32_t)cc.x, (int32_t)cc.y, d[u]);
            }
        }
    }
}

// One 16-lane row's sums of a slot's index entries: an entry (client i,
// position k, D'_{i,k}) adds the terms of position k of client i's walk (the
// one-pass walk's terms) when k lies up to the client's second open
// position.
struct SlotAcc {
    unsigned long long ad = 0, sb = 0, scc = 0, se = 0;  // ad: a | dd << 32
    template <bool Stage>
    __device__ __forceinline__ void add(uint2 en, const RowState<Stage> &rs)
    {
        if (en.x == 0xFFFFFFFFu)
            return;
        const int i = (int)(en.x >> 6), k = (int)(en.x & 63u);
        const int32_t dist = (int32_t)en.y;
        const uint32_t sv = rs.s(i);
        const int s1 = (int)(sv & 0xFFFFu), s2x = (int)(sv >> 16);
        if (k <= s2x) {  // (s2x = 0xFFFF, no second: every k < nearL)
            const uint2 cc = rs.c(i);
            const int32_t c1 = (int32_t)cc.x, c2 = (int32_t)cc.y;
            const bool upto1 = k <= s1, first = k == s1, second = k == s2x;
            ad += upto1 ? 1ull : (1ull << 32);
            const int32_t v = k < s1 ? c1 - dist : (first ? c1 : (second ? c2 - c1 : c2 - dist));
            const unsigned long long uv = (unsigned long long)v;
            sb += upto1 ? uv : 0ull;
            se += !upto1 && second ? uv : 0ull;
            scc += !upto1 && !second ? uv : 0ull;
            scc += first ? (unsigned long long)(c2 - c1) : 0ull;
        }
    }
    // the row's totals into slot `slot` (lane 15 of the row adds them; rows
    // walking listed clients add to the same bins)
    __device__ __forceinline__ void flush(SlotBins &B, int slot, int sub)
    {
        const unsigned long long a = row_sum64(ad), b = row_sum64(sb), c = row_sum64(scc),
                                 e = row_sum64(se);
        if (sub == 15) {
            atomicAdd(&B.a[slot], (uint32_t)a);
            atomicAdd(&B.dd[slot], (uint32_t)(a >> 32));
            atomicAdd(&B.b[slot], b);
            atomicAdd(&B.cc[slot], c);
            atomicAdd(&B.e[slot], e);
        }
    }
};

// Pass 2, a workgroup per chromosome (eight waves per SIMD: four workgroups
// per CU, so that a population of 1024 is resident at once).  Its clients' (s1, s2, c1, c2) are
// staged in LDS (n <= kStageClients) with one coalesced sweep that also lists
// the clients whose walk reaches past the index.  Then each 16-lane row takes
// tasks: a candidate slot (its facility's index entries, 16 at a time, four
// loads in flight, summed over the row) or a listed client (its positions
// from kNearL on).  Clients past the list's capacity are walked by the wave
// that finds them.
template <bool Stage>
__global__ __launch_bounds__(64 * kSlotWaves) __attribute__((amdgpu_waves_per_eu(8)))
void k_prop_slots(LearnArgs A)
{
    extern __shared__ __align__(16) uint32_t dyn[];  // staged: (c1, c2) x n, then s12 x n
    __shared__ SlotBins B;
    __shared__ uint64_t cb[kMaxLearnWords];
    __shared__ uint8_t cp[kMaxLearnWords];
    __shared__ int32_t fac[kSlots], soff[kSlots], scnt[kSlots];
    __shared__ int32_t farl[kFarCap];
    __shared__ int32_t nslots, nfar;
    const GaArgs &g = A.g;
    const Tables &t = g.t;
    const int c = blockIdx.x;
    if (c >= g.P || ga_stopped(g))  // (the whole workgroup)
        return;
    const int lane = threadIdx.x & 63, W = t.W, n = t.n;
    const int nearL = min(kNearL, t.K);
    const uint64_t *gcb = A.cbits + (int64_t)c * W;
    const uint8_t *gcp = A.cpre + (int64_t)c * W;
    // slot -> facility (slots in facility order)
    for (int w = threadIdx.x; w < W; w += blockDim.x) {
        uint64_t bits = gcb[w];
        int sl = gcp[w];
        cb[w] = bits;
        cp[w] = (uint8_t)sl;
        while (bits) {
            fac[sl++] = w * 64 + __builtin_ctzll(bits);
            bits &= bits - 1ull;
        }
        if (w == W - 1)
            nslots = sl;
    }
    bins_clear(B);
    if (threadIdx.x == 0)
        nfar = 0;
    __syncthreads();
    RowState<Stage> rs;
    rs.C = reinterpret_cast<const uint2 *>(dyn);
    rs.S = dyn + 2 * n;
    rs.gs = A.s12 + (int64_t)c * n;
    rs.gc = reinterpret_cast<const uint2 *>(A.c12) + (int64_t)c * n;
    const int ns = nslots;
    if ((int)threadIdx.x < ns) {
        const int f = fac[threadIdx.x];
        const int e0 = A.near_off[f];
        soff[threadIdx.x] = e0;
        scnt[threadIdx.x] = A.near_off[f + 1] - e0;
    }
    // the sweep: U clients per thread in flight
    constexpr int U = 4;
    constexpr int NT = 64 * kSlotWaves;
    for (int x0 = 0; x0 < n; x0 += U * NT) {
        uint32_t sv[U];
        uint2 cv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int x = x0 + u * NT + (int)threadIdx.x;
            sv[u] = x < n ? rs.gs[x] : 0u;
            cv[u] = x < n ? rs.gc[x] : uint2{0u, 0u};
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int x = x0 + u * NT + (int)threadIdx.x;
            if (x0 + u * NT >= n)  // (uniform)
                break;
            if constexpr (Stage) {
                if (x < n) {
                    uint2 *C = reinterpret_cast<uint2 *>(dyn);
                    C[x] = cv[u];
                    dyn[2 * n + x] = sv[u];
                }
            }
            const int s2x = (int)(sv[u] >> 16);
            const int end = s2x == 0xFFFF ? t.K : s2x + 1;
            const bool far = x < n && end > nearL;
            const uint64_t fb = __builtin_amdgcn_ballot_w64(far);
            if (fb == 0ull)
                continue;
            int base = 0;
            if (lane == 0)
                base = atomicAdd(&nfar, __builtin_popcountll(fb));
            base = __shfl(base, 0);
            const int idx = base + (int)__builtin_amdgcn_mbcnt_hi(
                                       (uint32_t)(fb >> 32),
                                       __builtin_amdgcn_mbcnt_lo((uint32_t)fb, 0u));
            if (far && idx < kFarCap)
                farl[idx] = x;
            uint64_t over = __builtin_amdgcn_ballot_w64(far && idx >= kFarCap);
            while (over) {  // the list is full: this wave walks the row itself
                const int l = (int)__builtin_ctzll(over);
                over &= over - 1ull;
                const int ii = x0 + u * NT + (int)(threadIdx.x & ~63u) + l;
                const uint32_t v = (uint32_t)__builtin_amdgcn_readlane((int)sv[u], l);
                const uint2 cc = {(uint32_t)__builtin_amdgcn_readlane((int)cv[u].x, l),
                                  (uint32_t)__builtin_amdgcn_readlane((int)cv[u].y, l)};
                walk_far(t, B, cb, cp, ii, v, cc, nearL, lane, 64);
            }
        }
    }
    __syncthreads();
    const int nf = min(nfar, kFarCap);
    const int row = (int)threadIdx.x >> 4, sub = lane & 15;
    // slot tasks two at a time per row: both slots' first 64 entries are
    // loaded in one round (further entries, rare, one chunk at a time)
    for (int t0 = row; t0 < ns; t0 += 2 * kSlotRows) {  // (uniform in the row)
        const int t1 = t0 + kSlotRows;
        const bool two = t1 < ns;
        const uint2 *ent[2] = {A.near_q + soff[t0], A.near_q + soff[two ? t1 : t0]};
        const int cnt[2] = {scnt[t0], two ? scnt[t1] : 0};
        uint2 en[2][4];
#pragma unroll
        for (int v = 0; v < 2; ++v)
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int q = 16 * u + sub;
                en[v][u] = q < cnt[v] ? ent[v][q] : uint2{0xFFFFFFFFu, 0u};
            }
#pragma unroll
        for (int v = 0; v < 2; ++v) {
            SlotAcc acc;
            for (int q0 = 0;;) {
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    acc.add(en[v][u], rs);
                q0 += 64;
                if (q0 >= cnt[v])
                    break;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int q = q0 + 16 * u + sub;
                    en[v][u] = q < cnt[v] ? ent[v][q] : uint2{0xFFFFFFFFu, 0u};
                }
            }
            if (v == 0 || two)
                acc.flush(B, v == 0 ? t0 : t1, sub);
        }
    }
    // listed clients whose walk reaches past the index
    for (int f = row; f < nf; f += kSlotRows) {
        const int ii = farl[f];
        walk_far(t, B, cb, cp, ii, rs.s(ii), rs.c(ii), nearL, sub, 16);
    }
    __syncthreads();
    for (int sl = threadIdx.x; sl < kSlots; sl += blockDim.x) {
        const int64_t o = (int64_t)c * kSlots + sl;
        A.sums.a[o] = B.a[sl];
        A.sums.dd[o] = B.dd[sl];
        A.sums.b[o] = B.b[sl];
        A.sums.cc[o] = B.cc[sl];
        A.sums.e[o] = B.e[sl];
    }
}

__global__ void k_near_count(Tables t, int L, int32_t *count)
{
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= (int64_t)t.n * L)
        return;
    const int64_t i = x / L, k = x - i * L;
    atomicAdd(count + t.pi[i * t.pitch + k], 1);
}

__global__ void k_near_fill(Tables t, int L, int32_t *cursor, uint2 *q)
{
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= (int64_t)t.n * L)
        return;
    const int64_t i = x / L, k = x - i * L;
    const int e = atomicAdd(cursor + t.pi[i * t.pitch + k], 1);
    q[e] = uint2{((uint32_t)i << 6) | (uint32_t)k, (uint32_t)t.ds[i * t.pitch + k]};
}

}  // namespace

hipError_t launch_near_count(const Tables &t, int32_t *count, hipStream_t s)
{
    const int L = min(kNearL, t.K);
    const int64_t cells = (int64_t)t.n * L;
    hipLaunchKernelGGL(k_near_count, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0, s, t,
                       L, count);
    return hipGetLastError();
}

hipError_t launch_near_fill(const Tables &t, int32_t *cursor, uint2 *q, hipStream_t s)
{
    const int L = min(kNearL, t.K);
    const int64_t cells = (int64_t)t.n * L;
    hipLaunchKernelGGL(k_near_fill, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0, s, t, L,
                       cursor, q);
    return hipGetLastError();
}

hipError_t launch_features(const Tables &t, const uint64_t *masks, int P, const FeatCtx &ctx,
                           float *out, uint32_t *err, hipStream_t s)
{
    if (P <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_features, dim3(P, (t.m + kSlots - 1) / kSlots), dim3(kLearnThreads),
                       0, s, t, masks, ctx, out, err);
    return hipGetLastError();
}

template <int CH, int NW>
hipError_t launch_walk_t(const LearnArgs &a, int out, hipStream_t s)
{
    hipLaunchKernelGGL((k_prop_walk<CH, NW>), dim3((a.g.P + CH - 1) / CH), dim3(64 * NW), 0, s,
                       a, out);
    return hipGetLastError();
}

// Walk shape: chromosomes per workgroup x waves (the default keeps eight
// waves per SIMD resident at P = 1024).
hipError_t launch_walk(const LearnArgs &a, int out, hipStream_t s)
{
    if (a.walk == 0) {  // the two-pass walk
        const int tiles_c = (a.g.P + kEvalTile - 1) / kEvalTile;
        const int tiles = tiles_c * ((a.g.t.n + kS12Clients - 1) / kS12Clients);
        const size_t lds = sizeof(uint32_t) * kEvalTile * (2 * (size_t)a.g.t.W + 1);
        hipLaunchKernelGGL(k_prop_s12, dim3(((tiles + 7) / 8) * 8), dim3(64 * kS12Waves), lds, s,
                           a, out, tiles_c);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
        if (a.g.t.n <= kStageClients)
            hipLaunchKernelGGL(k_prop_slots<true>, dim3(a.g.P), dim3(64 * kSlotWaves),
                               (size_t)a.g.t.n * 12, s, a);
        else
            hipLaunchKernelGGL(k_prop_slots<false>, dim3(a.g.P), dim3(64 * kSlotWaves), 0, s, a);
        return hipGetLastError();
    }
    switch (a.walk) {
    case 1: return launch_walk_t<1, 8>(a, out, s);
    case 4: return launch_walk_t<4, 16>(a, out, s);
    default: return launch_walk_t<2, 16>(a, out, s);
    }
}

hipError_t launch_propose(const LearnArgs &a, int in, hipStream_t s)
{
    const int out = in ^ 1;
    hipLaunchKernelGGL(k_prop_cand, dim3((a.g.P + kCandWaves - 1) / kCandWaves),
                       dim3(64 * kCandWaves), 0, s, a, out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    e = launch_walk(a, out, s);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_prop_score, dim3(a.g.P), dim3(64 * kMlpWaves), 0, s, a, out);
    return hipGetLastError();
}

hipError_t launch_static_sums(const int32_t *d, int64_t ld, int n, int m, const uint16_t *pi,
                              int pitch, int L, unsigned long long *colsum, uint32_t *nearc,
                              const uint32_t *err, unsigned long long *report, hipStream_t s)
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
    hipLaunchKernelGGL(k_total, dim3(1), dim3(256), 0, s, colsum, m, err, report);
    return hipGetLastError();
}

}  // namespace pmp
