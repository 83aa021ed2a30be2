// Genetic-algorithm kernels (Section 3.2 Evolve steps, Section 4 operators).
//
// One thread owns one chromosome (W 64-bit words in global memory).  The
// operators work on whole words: population sampling sets p bits, crossover
// selects bits with popcounts and lowest-set-bit extraction, mutation moves
// runs of up to 64 bits at a time.  Fitness is computed by the population
// evaluation kernel between these steps.  Every kernel first reads the
// run's stop flag, so generations enqueued after the stop do nothing.
#include "common.hpp"
#include "philox.hpp"

namespace pmp {

namespace {

constexpr int kGaThreads = 64;

__device__ __forceinline__ bool stopped(const GaArgs &g)
{
    return g.gs[GS_DONE] != 0ull;
}

__device__ __forceinline__ void count(unsigned long long *slot, bool pred)
{
    const uint64_t b = __builtin_amdgcn_ballot_w64(pred);
    if ((threadIdx.x & 63) == 0 && b)
        atomicAdd(slot, (unsigned long long)__builtin_popcountll(b));
}

// ---------------------------------------------------------------------------
// Population of one Evolve call (Section 3.1 steps 7/11 and 16; Section 4.1
// and 4.5).  Fresh slots get a uniform p-subset by Floyd's method
// (Bentley & Floyd, CACM 1987): for j = m-p .. m-1 draw t uniform in [0, j];
// take t, or j if t is already taken.  From the second generation on, slot
// b*NT of group b receives that group's best of the previous generation.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kGaThreads) void k_init(GaArgs g)
{
    const int c = blockIdx.x * kGaThreads + threadIdx.x;
    if (c >= g.P || stopped(g))
        return;
    const uint64_t gen = g.gs[GS_GEN];
    const int W = g.t.W;
    uint64_t *row = g.cur + (int64_t)c * W;
    if (gen > 0 && (c % g.NT) == 0) {
        const uint64_t *src = g.gmask + (int64_t)(c / g.NT) * W;
        for (int w = 0; w < W; ++w)
            row[w] = src[w];
    } else {
        for (int w = 0; w < W; ++w)
            row[w] = 0;
        PhiloxStream st(g.seed, ROLE_POPULATION, gen, (uint64_t)c, TAG_SAMPLE, 0);
        for (int j = g.t.m - g.t.p; j < g.t.m; ++j) {
            const int t = (int)st.below((uint64_t)j + 1);
            const bool taken = (row[t >> 6] >> (t & 63)) & 1ull;
            const int pick = taken ? j : t;
            row[pick >> 6] |= 1ull << (pick & 63);
        }
    }
    g.fit[c] = 0;
    g.ok[c] = 1;
    g.improved[c] = 0;
}

// Turn off (own=1, other=0) or on (own=0, other=1) the first `quota`
// positions of that kind met when walking from r1 and wrapping past the
// end.  Words are visited in that cyclic order; inside a word the lowest
// qualifying bits come first.
__device__ __forceinline__ void exchange_first(const uint64_t *A,
                                               const uint64_t *B, uint64_t *F,
                                               int W, int r1, int quota,
                                               bool turn_off)
{
    const int w0 = r1 >> 6, b0 = r1 & 63;
    int left = quota;
    for (int t = 0; t <= W && left > 0; ++t) {
        const int w = (w0 + t) % W;
        uint64_t seg;
        if (t == 0)
            seg = ~0ull << b0;
        else if (t == W)
            seg = b0 ? ((1ull << b0) - 1ull) : 0ull;
        else
            seg = ~0ull;
        uint64_t cand = (turn_off ? (A[w] & ~B[w]) : (~A[w] & B[w])) & seg;
        const int cnt = __builtin_popcountll(cand);
        uint64_t take;
        if (cnt <= left) {
            take = cand;
            left -= cnt;
        } else {
            take = 0;
            for (int r = 0; r < left; ++r) {
                const uint64_t low = cand & (0ull - cand);
                take |= low;
                cand ^= low;
            }
            left = 0;
        }
        if (turn_off)
            F[w] &= ~take;
        else
            F[w] |= take;
    }
}

// ---------------------------------------------------------------------------
// Crossover stage (Evolve step 3; Section 4.3).  Slot t pairs with
// t XOR stride inside its group; the pair's lower slot owns the draws
// r1 in [0, m) and i in [1, floor(p/2)].  Offspring = own parent with the
// first i "own 1, partner 0" genes turned off and the first i "own 0,
// partner 1" genes turned on, walking from r1.  Too few differing genes:
// no offspring.  The current population is only read here, so both
// partners see each other as the stage began.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kGaThreads) void k_crossover(GaArgs g, int stage)
{
    const int c = blockIdx.x * kGaThreads + threadIdx.x;
    if (c >= g.P || stopped(g))
        return;
    const uint64_t gen = g.gs[GS_GEN];
    const int W = g.t.W;
    const int stride = g.NT >> (1 + stage % g.lg);
    const int partner = c ^ stride;
    const int leader = c < partner ? c : partner;
    PhiloxStream st(g.seed, ROLE_EVOLVE, gen, (uint64_t)leader, TAG_CROSSOVER,
                    (uint64_t)stage);
    const int r1 = (int)st.below((uint64_t)g.t.m);
    const int quota = 1 + (int)st.below((uint64_t)(g.t.p / 2));

    const uint64_t *A = g.cur + (int64_t)c * W;
    const uint64_t *B = g.cur + (int64_t)partner * W;
    uint64_t *F = g.off + (int64_t)c * W;
    int differ = 0;
    for (int w = 0; w < W; ++w)
        differ += __builtin_popcountll(A[w] & ~B[w]);
    const bool ok = differ >= quota;
    if (ok) {
        for (int w = 0; w < W; ++w)
            F[w] = A[w];
        exchange_first(A, B, F, W, r1, quota, true);
        exchange_first(A, B, F, W, r1, quota, false);
    }
    g.ok[c] = ok ? 1 : 0;
    g.ofit[c] = 0;
    count(g.gs + GS_XO_FAIL, !ok);
}

// len (1..64) bits of A starting at bit pos, pos + len <= 64 * W.
__device__ __forceinline__ uint64_t bits_at(const uint64_t *A, int W, int pos,
                                            int len)
{
    const int w = pos >> 6, o = pos & 63;
    uint64_t v = A[w] >> o;
    if (o != 0 && w + 1 < W)
        v |= A[w + 1] << (64 - o);
    return len == 64 ? v : (v & ((1ull << len) - 1ull));
}

// `len` bits of the cyclic sequence A[lo..hi] starting at position s0
// (lo <= s0 <= hi, len <= hi - lo + 1).
__device__ __forceinline__ uint64_t cyclic_bits(const uint64_t *A, int W,
                                                int lo, int hi, int s0,
                                                int len)
{
    const int r = hi + 1 - s0;
    if (len <= r)
        return bits_at(A, W, s0, len);
    return bits_at(A, W, s0, r) | (bits_at(A, W, lo, len - r) << r);
}

// ---------------------------------------------------------------------------
// Mutation attempt (Evolve step 5; Section 4.4).  Draws, in order: type
// (circular or block shift), direction (right = toward higher index), then
// the amount s in [1, m-1] for a circular shift, or the block ends (a
// uniform pair of distinct positions a < b) and s in [1, b-a].  The offspring
// is built word by word: destination bit q takes source bit
// lo + ((q - lo - move) mod L) inside the rotated range [lo, hi] of length
// L, and source bit q outside it.  Chromosomes already improved in this
// cycle, and offspring equal to their parent, are not evaluated.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kGaThreads) void k_mutate(GaArgs g, int attempt)
{
    const int c = blockIdx.x * kGaThreads + threadIdx.x;
    if (c >= g.P || stopped(g))
        return;
    if (g.improved[c]) {
        g.ok[c] = 0;
        return;
    }
    const uint64_t gen = g.gs[GS_GEN];
    const int W = g.t.W, m = g.t.m;
    PhiloxStream st(g.seed, ROLE_EVOLVE, gen, (uint64_t)c, TAG_MUTATION,
                    (uint64_t)attempt);
    const int type = (int)st.below(2);
    const int dir = (int)st.below(2);
    int lo, hi;
    if (type == 0) {
        lo = 0;
        hi = m - 1;
    } else {
        const int x = (int)st.below((uint64_t)m);
        int y = (int)st.below((uint64_t)(m - 1));
        if (y >= x)
            ++y;
        lo = x < y ? x : y;
        hi = x < y ? y : x;
    }
    const int L = hi - lo + 1;
    const int s = 1 + (int)st.below((uint64_t)(L - 1));
    const int move = dir == 0 ? s : L - s;

    const uint64_t *A = g.cur + (int64_t)c * W;
    uint64_t *F = g.off + (int64_t)c * W;
    bool changed = false;
    for (int w = 0; w < W; ++w) {
        const int q0 = w * 64;
        const int q1 = min(m, q0 + 64);
        uint64_t v = A[w];
        const int qa = max(q0, lo), qb = min(q1, hi + 1);
        if (qa < qb) {
            const int nin = qb - qa;
            const int s0 = lo + (((qa - lo - move) % L) + L) % L;
            const uint64_t part = cyclic_bits(A, W, lo, hi, s0, nin);
            const uint64_t mask =
                (nin == 64 ? ~0ull : ((1ull << nin) - 1ull)) << (qa - q0);
            v = (v & ~mask) | (part << (qa - q0));
        }
        F[w] = v;
        changed |= v != A[w];
    }
    g.ok[c] = changed ? 1 : 0;
    g.ofit[c] = 0;
}

// Replace a parent by its offspring when strictly fitter (Evolve steps 3e
// and 5c).
__global__ __launch_bounds__(kGaThreads) void k_accept(GaArgs g, int mutation)
{
    const int c = blockIdx.x * kGaThreads + threadIdx.x;
    const bool live = c < g.P && !stopped(g);
    bool take = false;
    if (live && g.ok[c] && g.ofit[c] < g.fit[c]) {
        take = true;
        const int W = g.t.W;
        const uint64_t *F = g.off + (int64_t)c * W;
        uint64_t *A = g.cur + (int64_t)c * W;
        for (int w = 0; w < W; ++w)
            A[w] = F[w];
        g.fit[c] = g.ofit[c];
        if (mutation)
            g.improved[c] = 1;
    }
    count(g.gs + (mutation ? GS_MUT_TAKEN : GS_XO_TAKEN), take);
}

// Group best (Evolve steps 7-8): least fitness, lowest slot on ties.
__global__ __launch_bounds__(256) void k_group_best(GaArgs g)
{
    if (stopped(g))
        return;
    __shared__ unsigned long long sc[256];
    __shared__ int si[256];
    const int b = blockIdx.x;
    const int base = b * g.NT;
    unsigned long long bc = ~0ull;
    int bi = 0x7FFFFFFF;
    for (int t = threadIdx.x; t < g.NT; t += 256) {
        const unsigned long long f = g.fit[base + t];
        if (f < bc) {  // t ascends per thread: keeps the lowest slot
            bc = f;
            bi = t;
        }
    }
    sc[threadIdx.x] = bc;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            const unsigned long long oc = sc[threadIdx.x + h];
            const int oi = si[threadIdx.x + h];
            if (oc < sc[threadIdx.x] || (oc == sc[threadIdx.x] && oi < si[threadIdx.x])) {
                sc[threadIdx.x] = oc;
                si[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    const int W = g.t.W;
    const uint64_t *src = g.cur + (int64_t)(base + si[0]) * W;
    for (int w = threadIdx.x; w < W; w += 256)
        g.gmask[(int64_t)b * W + w] = src[w];
    if (threadIdx.x == 0)
        g.gcost[b] = sc[0];
}

// Global best, saturation and stop (Section 3.1 host steps 13-15).
__global__ __launch_bounds__(256) void k_global(GaArgs g)
{
    if (stopped(g))
        return;
    __shared__ unsigned long long sc[256];
    __shared__ int si[256];
    __shared__ int improved;
    unsigned long long bc = ~0ull;
    int bi = 0x7FFFFFFF;
    for (int b = threadIdx.x; b < g.NB; b += 256) {
        const unsigned long long f = g.gcost[b];
        if (f < bc) {
            bc = f;
            bi = b;
        }
    }
    sc[threadIdx.x] = bc;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            const unsigned long long oc = sc[threadIdx.x + h];
            const int oi = si[threadIdx.x + h];
            if (oc < sc[threadIdx.x] || (oc == sc[threadIdx.x] && oi < si[threadIdx.x])) {
                sc[threadIdx.x] = oc;
                si[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        improved = sc[0] < g.gs[GS_BEST];
    __syncthreads();
    const int W = g.t.W;
    if (improved)
        for (int w = threadIdx.x; w < W; w += 256)
            g.best_mask[w] = g.gmask[(int64_t)si[0] * W + w];
    if (threadIdx.x == 0) {
        if (improved) {
            g.gs[GS_BEST] = sc[0];
            g.gs[GS_SAT] = 0;
        } else {
            g.gs[GS_SAT] += 1;
        }
        const unsigned long long gen = g.gs[GS_GEN] + 1;
        g.gs[GS_GEN] = gen;
        if ((g.saturation > 0 && g.gs[GS_SAT] >= (unsigned long long)g.saturation) ||
            gen >= (unsigned long long)g.generations)
            g.gs[GS_DONE] = 1;
    }
}

inline dim3 per_chromosome(int P)
{
    return dim3((unsigned)((P + kGaThreads - 1) / kGaThreads));
}

}  // namespace

hipError_t launch_ga_init(const GaArgs &g, hipStream_t s)
{
    hipLaunchKernelGGL(k_init, per_chromosome(g.P), dim3(kGaThreads), 0, s, g);
    return hipGetLastError();
}

hipError_t launch_ga_crossover(const GaArgs &g, int stage, hipStream_t s)
{
    hipLaunchKernelGGL(k_crossover, per_chromosome(g.P), dim3(kGaThreads), 0, s,
                       g, stage);
    return hipGetLastError();
}

hipError_t launch_ga_mutate(const GaArgs &g, int attempt, hipStream_t s)
{
    hipLaunchKernelGGL(k_mutate, per_chromosome(g.P), dim3(kGaThreads), 0, s, g,
                       attempt);
    return hipGetLastError();
}

hipError_t launch_ga_accept(const GaArgs &g, int mutation, hipStream_t s)
{
    hipLaunchKernelGGL(k_accept, per_chromosome(g.P), dim3(kGaThreads), 0, s, g,
                       mutation);
    return hipGetLastError();
}

hipError_t launch_ga_best(const GaArgs &g, hipStream_t s)
{
    hipLaunchKernelGGL(k_group_best, dim3(g.NB), dim3(256), 0, s, g);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_global, dim3(1), dim3(256), 0, s, g);
    return hipGetLastError();
}

}  // namespace pmp
