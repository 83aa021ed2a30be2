// Genetic-algorithm device code (Section 3.2 Evolve steps, Section 4
// operators), shared by the one-kernel-per-step launch sequence and the
// persistent kernel.
//
// One wavefront owns one chromosome; its lanes own the chromosome's 64-bit
// words (two per lane above m = 4096).  Every random choice is drawn by all
// lanes from the same Philox stream, so control flow stays uniform.
//
// A generation is: population (with migrants), evaluation, then for each
// operator stage a stage step followed by an evaluation, then a last stage
// step with no operator, then the group and global bests.  A stage step first
// finishes the previous stage for its chromosome (sum the evaluation's
// partial costs, take the offspring if strictly fitter) and then starts the
// next operator.  State is double-buffered between stages, so a crossover
// partner is always read as the previous stage left it, whatever order waves
// run in.
#pragma once

#include "common.hpp"
#include "philox.hpp"

namespace pmp {

constexpr int kMaxWords = PMP_MAX_FACILITIES / 64;  // 128
constexpr int kGaWaves = 4;                         // waves per workgroup

// Buffer k of a double-buffered pair, by select (indexing the kernel
// argument array with a run-time value would copy it to scratch).
template <class T>
__device__ __forceinline__ T *buf(T *const (&pair)[2], int k)
{
    return k ? pair[1] : pair[0];
}

__device__ __forceinline__ bool ga_stopped(const GaArgs &g)
{
    return g.gs[GS_DONE] != 0ull;
}

// Crossover stages a generation runs (none when p < 2 or NT = 1).
__device__ __forceinline__ int ga_xstages(const GaArgs &g)
{
    return (g.t.p >= 2 && g.lg > 0) ? g.X : 0;
}

// Wave-wide inclusive prefix sums with DPP lane moves instead of LDS
// permutes: shifts by 1, 2, 4 and 8 within each 16-lane row (lanes without
// a source add 0), then the last lane of row 0 and of row 2 is broadcast into
// rows 1 and 3, and the last lane of row 1 into rows 2 and 3.
template <int Ctrl, int RowMask>
__device__ __forceinline__ uint32_t dpp_from(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, Ctrl, RowMask, 0xF, false);
}

__device__ __forceinline__ uint32_t wave_scan_incl(uint32_t v, int /*lane*/)
{
    v += dpp_from<0x111, 0xF>(v);  // row_shr:1
    v += dpp_from<0x112, 0xF>(v);  // row_shr:2
    v += dpp_from<0x114, 0xF>(v);  // row_shr:4
    v += dpp_from<0x118, 0xF>(v);  // row_shr:8
    v += dpp_from<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_from<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
    return v;
}

// The same on 64-bit values (low and high words, carry by compare).
template <int Ctrl, int RowMask>
__device__ __forceinline__ void dpp_add64(uint32_t &lo, uint32_t &hi)
{
    const uint32_t l2 = dpp_from<Ctrl, RowMask>(lo), h2 = dpp_from<Ctrl, RowMask>(hi);
    const uint32_t nl = lo + l2;
    hi = hi + h2 + (nl < lo ? 1u : 0u);
    lo = nl;
}

// Sum over the wave, the same value in every lane.
__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v)
{
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
    dpp_add64<0x111, 0xF>(lo, hi);
    dpp_add64<0x112, 0xF>(lo, hi);
    dpp_add64<0x114, 0xF>(lo, hi);
    dpp_add64<0x118, 0xF>(lo, hi);
    dpp_add64<0x142, 0xA>(lo, hi);
    dpp_add64<0x143, 0xC>(lo, hi);
    const uint32_t tl = (uint32_t)__builtin_amdgcn_readlane((int)lo, 63);
    const uint32_t th = (uint32_t)__builtin_amdgcn_readlane((int)hi, 63);
    return ((unsigned long long)th << 32) | tl;
}

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int lane)
{
    const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)v, lane);
    const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}

// v of lane src (src may differ between lanes; every lane must take part)
__device__ __forceinline__ uint64_t readpair(uint64_t v, int src)
{
    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, src);
    const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}

// Orders a wave's LDS accesses before and after it (one wave owns the data).
__device__ __forceinline__ void wave_lds_fence()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// The k lowest set bits of x (all of x when it has no more than k, none
// when k <= 0).  No branches: lanes of a wave seldom agree on the cases.
// The half holding the k-th set bit is found from the low half's count,
// then the bit within that half by a 5-step search on 32-bit popcounts.
__device__ __forceinline__ uint64_t lowest_bits(uint64_t x, int k)
{
    const uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
    const int nlo = __builtin_popcount(lo);
    const bool in_lo = k <= nlo;
    const uint32_t v = in_lo ? lo : hi;
    const int kk = in_lo ? k : k - nlo;
    // largest q with popcount(v below bit q) < kk; the kk-th set bit of v
    // is at q
    int q = 0;
#pragma unroll
    for (int step = 16; step > 0; step >>= 1) {
        const int t = q + step;
        if (__builtin_popcount(v & ((1u << t) - 1u)) < kk)
            q = t;
    }
    const uint32_t keep = q >= 31 ? ~0u : ((2u << q) - 1u);  // bits 0..q
    const uint64_t cut = in_lo ? (uint64_t)(lo & keep) : (((uint64_t)(hi & keep) << 32) | lo);
    return k <= 0 ? 0ull : (__builtin_popcountll(x) <= k ? x : cut);
}

// Philox4x64-10 block (philox.hpp) for counter (c0, c1, c2, c3).
__device__ __forceinline__ void philox_block(uint64_t k0, uint64_t k1,
                                             uint64_t c0, uint64_t c1,
                                             uint64_t c2, uint64_t c3,
                                             uint64_t out[4])
{
    PhiloxStream st(k0, k1, c0, c1, 0, 0);
    st.c2 = c2;
    st.block = c3;
    st.refill();
    out[0] = st.buf[0];
    out[1] = st.buf[1];
    out[2] = st.buf[2];
    out[3] = st.buf[3];
}

// ---------------------------------------------------------------------------
// Floyd's method (Bentley & Floyd, CACM 1987) draws a uniform p-subset of
// [0, m): for j = m-p .. m-1 draw t uniform in [0, j]; take t, or j if t is
// already taken.  The loop is sequential, but its result has a closed form
// that lanes can evaluate together.  Write e = j - (m-p) and t_e for the
// draw of step e.  Since every earlier pick is below j, t_e is already taken
// exactly when it equals an earlier draw, or equals an earlier j whose own
// draw was already taken.  So with
//   col(e) = [t_e = t_e' for some e' < e]
//            or [m-p <= t_e < j_e and col(t_e - (m-p))]
// the subset is {t_e : all e} together with {j_e : col(e)}.  The lanes
// evaluate the draws 64 at a time in step order: a draw repeated from an
// earlier batch shows in the bitmap T of all earlier draws; one repeated
// within the batch shows in a match of the draws' bits by ballots; col of an
// earlier batch is read from the bitmap Cb; col of a lower lane of the same
// batch is taken once that lane has settled (the lowest unsettled lane
// always can, so the loop ends).  Returns false, before writing anything,
// when a draw would need Lemire's rejection step: the caller then runs the
// loop one step at a time, which consumes the stream in the same order.
// sw: 2 * W words of LDS owned by the wave.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool floyd_wave(const GaArgs &g, uint64_t gen, int c,
                                           int lane, uint64_t *sw,
                                           uint64_t &word0, uint64_t &word1)
{
    const int W = g.t.W, m = g.t.m, p = g.t.p;
    const int off = m - p, nC = (p + 63) >> 6;
    uint64_t *T = sw, *Cb = sw + W;
    for (int w = lane; w < 2 * W; w += 64)
        sw[w] = 0ull;
    wave_lds_fence();
    const int nbits = m > 1 ? 32 - __builtin_clz((unsigned)(m - 1)) : 1;
    const uint64_t below = (1ull << lane) - 1ull;
    uint64_t q[4];
    for (int ch = 0; ch < nC; ++ch) {
        // draw e = 64 ch + lane is word (lane & 3) of block 16 ch + lane / 4;
        // lane l computes block 64 r + l for r = ch / 4
        if ((ch & 3) == 0)
            philox_block(g.seed, ROLE_POPULATION, gen, (uint64_t)c,
                         (TAG_SAMPLE << 32), (uint64_t)(64 * (ch >> 2) + lane), q);
        const int src = 16 * (ch & 3) + (lane >> 2), sel = lane & 3;
        const uint64_t x0 = readpair(q[0], src), x1 = readpair(q[1], src);
        const uint64_t x2 = readpair(q[2], src), x3 = readpair(q[3], src);
        const uint64_t x = sel == 0 ? x0 : sel == 1 ? x1 : sel == 2 ? x2 : x3;
        const int e = 64 * ch + lane;
        const bool valid = e < p;
        const uint64_t r = (uint64_t)(off + e) + 1ull;
        if (__builtin_amdgcn_ballot_w64(valid && x * r < r) != 0ull)
            return false;
        const int t = valid ? (int)__umul64hi(x, r) : 0;
        // repeated from an earlier batch
        bool col = valid && ((T[t >> 6] >> (t & 63)) & 1ull) != 0ull;
        // repeated from a lower lane of this batch
        uint64_t same = __builtin_amdgcn_ballot_w64(valid);
        for (int b = 0; b < nbits; ++b) {
            const bool set = ((t >> b) & 1) != 0;
            const uint64_t v = __builtin_amdgcn_ballot_w64(set);
            same &= set ? v : ~v;
        }
        col = col || (valid && (same & below) != 0ull);
        // equal to an earlier j: that step's col decides
        const bool ref = valid && !col && t >= off && t < off + e;
        const int tgt = ref ? t - off : 0;
        const bool ref_prev = ref && tgt < 64 * ch;
        const uint64_t cw = Cb[tgt >> 6];
        if (ref_prev)
            col = ((cw >> (tgt & 63)) & 1ull) != 0ull;
        bool pending = ref && !ref_prev;
        const int tl = pending ? tgt - 64 * ch : lane;
        while (__builtin_amdgcn_ballot_w64(pending) != 0ull) {
            const int tp = __shfl((int)pending, tl);
            const int tc = __shfl((int)col, tl);
            if (pending && tp == 0) {
                col = tc != 0;
                pending = false;
            }
        }
        const uint64_t cmask = __builtin_amdgcn_ballot_w64(col);
        wave_lds_fence();  // every lane has read T and Cb for this batch
        if (lane == 0)
            Cb[ch] = cmask;
        if (valid)
            atomicOr((unsigned long long *)&T[t >> 6], 1ull << (t & 63));
        wave_lds_fence();
    }
    // the subset: every draw, and j = m-p+e for each e with col(e)
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int w = lane + 64 * k;
        const int wl = min(w, W - 1);
        const int base = 64 * wl - off;  // bit of Cb for facility 64 w
        const int i = base >> 6, o = base & 63;
        const uint64_t lo = (i >= 0 && i < nC) ? Cb[i] : 0ull;
        const uint64_t hi = (i + 1 >= 0 && i + 1 < nC) ? Cb[i + 1] : 0ull;
        const uint64_t jb = o == 0 ? lo : ((lo >> o) | (hi << (64 - o)));
        const uint64_t v = w < W ? (T[wl] | jb) : 0ull;
        if (k == 0)
            word0 = v;
        else
            word1 = v;
    }
    return true;
}

// Blocks 0 and 1 of the Philox4x64-10 stream with key (k0, k1) and counter
// words (c0, c1, c2): two independent round chains side by side, so their
// latencies overlap (the same rounds as PhiloxStream::refill).
__device__ __forceinline__ void philox_two_blocks(uint64_t k0, uint64_t k1, uint64_t c0,
                                                  uint64_t c1, uint64_t c2,
                                                  uint64_t out[8])
{
    const uint64_t kM0 = 0xD2E7470EE14C6C93ull, kM1 = 0xCA5A826395121157ull;
    const uint64_t kW0 = 0x9E3779B97F4A7C15ull, kW1 = 0xBB67AE8584CAA73Bull;
    uint64_t x0 = c0, x1 = c1, x2 = c2, x3 = 0;
    uint64_t y0 = c0, y1 = c1, y2 = c2, y3 = 1;
    uint64_t a = k0, b = k1;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t hx0 = __umul64hi(kM0, x0), lx0 = kM0 * x0;
        const uint64_t hy0 = __umul64hi(kM0, y0), ly0 = kM0 * y0;
        const uint64_t hx1 = __umul64hi(kM1, x2), lx1 = kM1 * x2;
        const uint64_t hy1 = __umul64hi(kM1, y2), ly1 = kM1 * y2;
        x0 = hx1 ^ x1 ^ a;
        y0 = hy1 ^ y1 ^ a;
        x1 = lx1;
        y1 = ly1;
        x2 = hx0 ^ x3 ^ b;
        y2 = hy0 ^ y3 ^ b;
        x3 = lx0;
        y3 = ly0;
        a += kW0;
        b += kW1;
    }
    out[0] = x0;
    out[1] = x1;
    out[2] = x2;
    out[3] = x3;
    out[4] = y0;
    out[5] = y1;
    out[6] = y2;
    out[7] = y3;
}

// The high word of x * r, uniform in [0, r) when the draw needs no
// rejection step; flags `rej` when it might (then the caller redraws the
// whole stream one word at a time with PhiloxStream::below).
__device__ __forceinline__ uint64_t lemire_fast(uint64_t x, uint64_t r, bool &rej)
{
    rej = rej || x * r < r;
    return __umul64hi(x, r);
}

// Mutation operands from the draws type, direction, block ends x and y
// (y skips x) and the amount: the rotated range [lo, hi] and the move.
__device__ __forceinline__ void mutation_draws(uint64_t type, uint64_t dir, uint64_t x,
                                               uint64_t y, uint64_t sh, int m, OpDraw &d)
{
    int lo = 0, hi = m - 1;
    if (type != 0) {
        int yy = (int)y;
        if (yy >= (int)x)
            ++yy;
        lo = (int)x < yy ? (int)x : yy;
        hi = (int)x < yy ? yy : (int)x;
    }
    const int L = hi - lo + 1;
    d.a = lo;
    d.b = hi;
    d.c = dir == 0 ? 1 + (int)sh : L - 1 - (int)sh;
}

// ---------------------------------------------------------------------------
// The operator draws of chromosome c for one generation, one stream per lane
// (the streams are independent): crossover stage k draws r1 in [0, m) and
// the quota i in [1, floor(p/2)] from c's stream for stage k (used when c is
// the lower slot of its pair, Section 4.3); mutation attempt a draws the
// type, the direction, the block ends if any and the amount from c's stream
// for attempt a (Section 4.4).  The stage kernels load them with their other
// inputs instead of running the generator on their critical path.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void ga_draws_one(const GaArgs &g, uint64_t gen, int c,
                                             int lane)
{
    const int m = g.t.m, p = g.t.p, S = g.X + g.Y;
    const uint64_t rq = (uint64_t)max(p / 2, 1);
    for (int s0 = 0; s0 < S; s0 += 64) {
        const int s = s0 + lane;
        const bool isx = s < g.X;
        const uint64_t tag = isx ? TAG_CROSSOVER : TAG_MUTATION;
        const uint64_t idx = (uint64_t)(isx ? s : s - g.X);
        uint64_t w[8];
        philox_two_blocks(g.seed, ROLE_EVOLVE, gen, (uint64_t)c,
                          (tag << 32) | (idx & 0xFFFFFFFFull), w);
        // without rejections the draws are words 0, 1, ... of the stream
        bool rej = false;
        OpDraw d{0, 0, 0, 0};
        if (isx) {
            d.a = (int)lemire_fast(w[0], (uint64_t)m, rej);
            d.b = 1 + (int)lemire_fast(w[1], rq, rej);
        } else {
            const uint64_t type = lemire_fast(w[0], 2, rej);
            const uint64_t dir = lemire_fast(w[1], 2, rej);
            uint64_t x = 0, y = 0, sh;
            if (type != 0) {
                x = lemire_fast(w[2], (uint64_t)m, rej);
                y = lemire_fast(w[3], (uint64_t)(m - 1), rej);
                const int yy = (int)y >= (int)x ? (int)y + 1 : (int)y;
                const int L = ((int)x < yy ? yy - (int)x : (int)x - yy) + 1;
                sh = lemire_fast(w[4], (uint64_t)(L - 1), rej);
            } else {
                sh = lemire_fast(w[2], (uint64_t)(m - 1), rej);
            }
            mutation_draws(type, dir, x, y, sh, m, d);
        }
        if (rej) {
            PhiloxStream st(g.seed, ROLE_EVOLVE, gen, (uint64_t)c, tag, idx);
            if (isx) {
                d.a = (int)st.below((uint64_t)m);
                d.b = 1 + (int)st.below(rq);
            } else {
                const uint64_t type = st.below(2), dir = st.below(2);
                uint64_t x = 0, y = 0;
                int L = m;
                if (type != 0) {
                    x = st.below((uint64_t)m);
                    y = st.below((uint64_t)(m - 1));
                    const int yy = (int)y >= (int)x ? (int)y + 1 : (int)y;
                    L = ((int)x < yy ? yy - (int)x : (int)x - yy) + 1;
                }
                const uint64_t sh = st.below((uint64_t)(L - 1));
                mutation_draws(type, dir, x, y, sh, m, d);
            }
        }
        if (isx && p < 2)
            d = OpDraw{0, 0, 0, 0};
        if (s < S)
            g.draws[(int64_t)c * S + s] = d;
    }
}

// The sample stream of chromosome c read one draw at a time by the whole
// wave: lane l holds block base + l, and the k-th draw is word k & 3 of block
// k >> 2, read from its lane.
struct SerialDraws {
    uint64_t q[4];
    int64_t base = 0, k = 0;

    __device__ __forceinline__ SerialDraws(const GaArgs &g, uint64_t gen, int c, int lane)
    {
        philox_block(g.seed, ROLE_POPULATION, gen, (uint64_t)c, (TAG_SAMPLE << 32),
                     (uint64_t)lane, q);
    }

    __device__ __forceinline__ uint64_t next(const GaArgs &g, uint64_t gen, int c, int lane)
    {
        if ((k >> 2) - base >= 64) {
            base += 64;
            philox_block(g.seed, ROLE_POPULATION, gen, (uint64_t)c, (TAG_SAMPLE << 32),
                         (uint64_t)(base + lane), q);
        }
        const int src = (int)((k >> 2) - base), sel = (int)(k & 3);
        const uint64_t mine = sel == 0 ? q[0] : sel == 1 ? q[1] : sel == 2 ? q[2] : q[3];
        ++k;
        return readlane64(mine, src);
    }

    // uniform in [0, r), r >= 1, by Lemire's multiply-and-reject method
    __device__ __forceinline__ uint64_t below(const GaArgs &g, uint64_t gen, int c, int lane,
                                              uint64_t r)
    {
        uint64_t x = next(g, gen, c, lane);
        uint64_t lo = x * r;
        if (lo < r) {
            const uint64_t thresh = (0ull - r) % r;
            while (lo < thresh) {
                x = next(g, gen, c, lane);
                lo = x * r;
            }
        }
        return __umul64hi(x, r);
    }
};

// Chromosome generation by rank (Section 4.1): the p-subset of lexicographic
// rank r, r uniform below C(m, p).  Element i is the least candidate x >= x0
// (x0 one past element i - 1) such that the subsets whose element i lies in
// [x0, x] reach past r.  By the hockey-stick identity there are
// C(m - x0, p - i) - C(m - x - 1, p - i) of them, so x is the least candidate
// with C(m - x - 1, p - i) < C(m - x0, p - i) - r; the lanes test 64
// candidates at a time and a ballot picks the least.  The subsets skipped,
// C(m - x0, p - i) - C(m - x, p - i), come off r.  Every binomial read has
// top index below m except C(m, p) itself.
__device__ __forceinline__ void unrank_wave(const GaArgs &g, uint64_t r, int lane,
                                            uint64_t &word0, uint64_t &word1)
{
    const int m = g.t.m, p = g.t.p;
    const unsigned long long *bn = g.binom;  // C(a, b) at a (p + 1) + b, a < m
    auto C = [&](int a, int b) -> uint64_t {
        if (a < b || a < 0)
            return 0ull;
        return a == m ? g.nsets : (uint64_t)bn[(int64_t)a * (p + 1) + b];
    };
    int x0 = 0;
    for (int i = 0; i < p; ++i) {
        const int b = p - i;
        const uint64_t top = C(m - x0, b);
        const uint64_t need = top - r;  // >= 1
        int x = -1;
        for (int base = x0; x < 0; base += 64) {
            const int xc = base + lane;
            const bool hit = C(m - xc - 1, b) < need;
            const uint64_t bal = __builtin_amdgcn_ballot_w64(hit);
            if (bal)
                x = base + (int)__builtin_ctzll(bal);
        }
        r -= top - C(m - x, b);
        const uint64_t bit = 1ull << (x & 63);
        if (lane == (x >> 6))
            word0 |= bit;
        if (lane + 64 == (x >> 6))
            word1 |= bit;
        x0 = x + 1;
    }
}

// ---------------------------------------------------------------------------
// Population of one Evolve call (Section 3.1 steps 7/11 and 16; Sections 4.1
// and 4.5), chromosome c, by its wave.  Fresh slots get a uniform p-subset by
// Floyd's method: floyd_wave above, or, when a draw needs Lemire's rejection
// step, one step at a time; either way the draws are consumed in stream
// order, so the result is the same as drawing one at a time.  With init by rank
// a fresh slot takes the subset of a uniform lexicographic rank instead, the
// rank being the first bounded draw of the same stream.  From the
// second generation on the group bests migrate: group b's best to slot b*NT
// (the same block) or to slot b (one block).  The population goes to off[0]
// with fitness "infinite", so the first stage takes it as the current one.
// The generation's operator draws are made here too (ga_draws_one): with
// part -1 by the same wave, else part 0 makes the population slot and part 1
// the draws, so that two waves share the work.
// sw: 2 * W words of LDS owned by the wave.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void ga_init_one(const GaArgs &g, int c, int lane,
                                            uint64_t *sw, int part = -1, bool ahead = false)
{
    // ahead: the next generation's population, made while this one's last
    // steps run (its migrants are placed by the group-best step)
    const uint64_t gen = g.gs[GS_GEN] + (ahead ? 1u : 0u);
    if (part == 1) {  // only the operator draws
        ga_draws_one(g, gen, c, lane);
        return;
    }
    const int W = g.t.W, m = g.t.m, p = g.t.p;
    uint64_t *dst = g.off[0] + (int64_t)c * W;
    // migrant slots: b*NT for group b (same block) or b (one block)
    const bool one = g.migration == PMP_MIG_ONE_BLOCK;
    const bool migrant = gen > 0 && (one ? c < g.NB : (c % g.NT) == 0);
    if (migrant) {
        if (!ahead) {
            const uint64_t *src = g.gmask + (int64_t)(one ? c : c / g.NT) * W;
            for (int w = lane; w < W; w += 64)
                dst[w] = src[w];
        }
    } else {
        // the subset's words live in the lanes: word w in lane w (w < 64)
        // or in the second register of lane w - 64
        uint64_t word0 = 0, word1 = 0;
        if (g.init_rank) {
            SerialDraws sd(g, gen, c, lane);
            unrank_wave(g, sd.below(g, gen, c, lane, g.nsets), lane, word0, word1);
        } else if (!floyd_wave(g, gen, c, lane, sw, word0, word1)) {
            word0 = word1 = 0ull;
            SerialDraws sd(g, gen, c, lane);
            for (int j = m - p; j < m; ++j) {
                const int t = (int)sd.below(g, gen, c, lane, (uint64_t)j + 1);
                const int tw = t >> 6;
                const uint64_t held = lane == tw ? word0 : (lane + 64 == tw ? word1 : 0ull);
                const bool taken =
                    __builtin_amdgcn_ballot_w64(((held >> (t & 63)) & 1ull) != 0ull) != 0ull;
                const int pick = taken ? j : t;
                const uint64_t bit = 1ull << (pick & 63);
                if (lane == (pick >> 6))
                    word0 |= bit;
                if (lane + 64 == (pick >> 6))
                    word1 |= bit;
            }
        }
        if (lane < W)
            dst[lane] = word0;
        if (lane + 64 < W)
            dst[lane + 64] = word1;
    }
    if (part < 0)
        ga_draws_one(g, gen, c, lane);
    if (lane == 0) {
        g.ok[0][c] = 1;
        g.fit[0][c] = ~0ull;
        g.improved[c] = 0;
    }
}

// A chromosome held by a wave: word w in register w >> 6 of lane w & 63.
struct WaveWords {
    uint64_t v[2];

    // word w, for a lane-varying w (two ds_bpermute per register)
    __device__ __forceinline__ uint64_t at(int w) const
    {
        const uint64_t lo = __shfl(v[0], w & 63), hi = __shfl(v[1], w & 63);
        return (w >> 6) ? hi : lo;
    }
    // word w, for a wave-uniform w
    __device__ __forceinline__ uint64_t at_uniform(int w) const
    {
        return readlane64((w >> 6) ? v[1] : v[0], w & 63);
    }
};

// len (1..64) bits of A starting at bit pos, pos + len <= 64 * W (lanes may
// ask for different positions).
__device__ __forceinline__ uint64_t bits_at(const WaveWords &A, int W, int pos,
                                            int len)
{
    const int w = pos >> 6, o = pos & 63;
    uint64_t v = A.at(w) >> o;
    const uint64_t next = A.at(w + 1 < W ? w + 1 : w);
    if (o != 0 && w + 1 < W)
        v |= next << (64 - o);
    return len == 64 ? v : (v & ((1ull << len) - 1ull));
}

// `len` bits of the cyclic sequence A[lo..hi] starting at position s0
// (lo <= s0 <= hi, len <= hi - lo + 1).  Branch-free, so every lane takes
// part in the shuffles of both runs.
__device__ __forceinline__ uint64_t cyclic_bits(const WaveWords &A, int W,
                                                int lo, int hi, int s0,
                                                int len)
{
    const int first = min(len, hi + 1 - s0);  // bits before the wrap
    const int second = len - first;           // bits after it (0: none)
    const uint64_t v1 = bits_at(A, W, s0, first);
    const uint64_t v2 = bits_at(A, W, lo, second > 0 ? second : 1);
    return second > 0 ? (v1 | (v2 << first)) : v1;
}

// Where an operator's result words go: a row of device memory, or (in the
// stage steps fused with the evaluation) a chromosome's row of the
// evaluation's LDS staging area as two 32-bit halves, plus the device row
// when the workgroup keeps the run's state (null otherwise).
__device__ __forceinline__ void store_word(uint64_t *F, int w, uint64_t v)
{
    F[w] = v;
}

struct StagedRow {
    uint64_t *global;  // may be null
    uint32_t *lds;     // 2 W words
};

__device__ __forceinline__ void store_word(const StagedRow &F, int w, uint64_t v)
{
    if (F.global)
        F.global[w] = v;
    F.lds[2 * w] = (uint32_t)v;
    F.lds[2 * w + 1] = (uint32_t)(v >> 32);
}

// ---------------------------------------------------------------------------
// Crossover (Section 4.3) of own parent A with partner B, both as the
// previous stage left them.  Walking from r1 and wrapping past the end,
// turn off the first `quota` genes with A = 1, B = 0 and turn on the first
// `quota` with A = 0, B = 1.  The walk is split into segments: the part of
// word r1/64 from bit r1%64 up, the following words in cyclic order, and the
// part of word r1/64 below bit r1%64.  A wave prefix sum of the per-segment
// counts tells each lane how many qualifying genes come before its segment,
// hence how many of its own to take (its lowest ones).  Returns false when
// the parents differ in fewer than 2*quota genes (no offspring).
// ---------------------------------------------------------------------------
template <class Out>
__device__ __forceinline__ bool crossover_wave(const WaveWords &A,
                                               const WaveWords &B, const Out &F,
                                               int W, int r1, int quota,
                                               int lane)
{
    const int w0 = r1 >> 6, b0 = r1 & 63;
    const uint64_t low_mask = b0 ? ((1ull << b0) - 1ull) : 0ull;
    const uint64_t a0 = A.at_uniform(w0), bb0 = B.at_uniform(w0);
    const uint64_t xl = a0 & ~bb0 & low_mask, yl = ~a0 & bb0 & low_mask;

    uint64_t x[2] = {0, 0}, y[2] = {0, 0}, av[2] = {0, 0};
    int wd[2] = {-1, -1};
    uint32_t v[2] = {0, 0};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        if (h == 1 && W <= 64)  // uniform: no second register
            break;
        const int r = lane + 64 * h;
        int w = w0 + r;
        if (w >= W)
            w -= W;
        const uint64_t a = A.at(w < W ? w : 0), b = B.at(w < W ? w : 0);
        if (r < W) {
            const uint64_t seg = r == 0 ? (~0ull << b0) : ~0ull;
            x[h] = a & ~b & seg;
            y[h] = ~a & b & seg;
            av[h] = a;
            wd[h] = w;
            v[h] = (uint32_t)__builtin_popcountll(x[h]) |
                   ((uint32_t)__builtin_popcountll(y[h]) << 16);
        }
    }
    const uint32_t inc0 = wave_scan_incl(v[0], lane);
    const uint32_t tot0 = (uint32_t)__builtin_amdgcn_readlane((int)inc0, 63);
    const uint32_t inc1 = W > 64 ? wave_scan_incl(v[1], lane) + tot0 : tot0;
    const uint32_t tot = W > 64 ? (uint32_t)__builtin_amdgcn_readlane((int)inc1, 63) : tot0;
    const int main_x = (int)(tot & 0xFFFFu), main_y = (int)(tot >> 16);
    const int differ = main_x + __builtin_popcountll(xl);
    if (differ < quota)
        return false;
    const uint32_t inc[2] = {inc0, inc1};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        if (wd[h] < 0)
            continue;
        const uint32_t ex = inc[h] - v[h];
        // Word r1/64 (lane 0, h = 0) also holds the last segment, below bit
        // r1 mod 64, which the walk reaches only once every other gene of
        // the kind is taken (its first segment included): one lowest_bits
        // per kind on every lane, no divergent extra calls.
        const bool first = lane + 64 * h == 0;
        const int kx = quota - (int)(ex & 0xFFFFu), ky = quota - (int)(ex >> 16);
        const bool x_in = !first || kx <= __builtin_popcountll(x[h]);
        const bool y_in = !first || ky <= __builtin_popcountll(y[h]);
        const uint64_t take_x = lowest_bits(x_in ? x[h] : xl, x_in ? kx : quota - main_x) |
                                (x_in ? 0ull : x[h]);
        const uint64_t take_y = lowest_bits(y_in ? y[h] : yl, y_in ? ky : quota - main_y) |
                                (y_in ? 0ull : y[h]);
        store_word(F, wd[h], (av[h] & ~take_x) | take_y);
    }
    return true;
}

// ---------------------------------------------------------------------------
// Mutation (Section 4.4) of A into F: destination bit q takes source bit
// lo + ((q - lo - move) mod L) inside the rotated range [lo, hi] of length
// L, and source bit q outside it.  Each lane builds its destination words
// from at most two runs of source bits.  Returns whether F differs from A.
// ---------------------------------------------------------------------------
template <class Out>
__device__ __forceinline__ bool mutate_wave(const WaveWords &A, const Out &F,
                                            int W, int m, int lo, int hi,
                                            int move, int lane)
{
    const int L = hi - lo + 1;
    bool changed = false;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        if (h == 1 && W <= 64)  // uniform: no second register
            break;
        const int w = lane + 64 * h;
        const int q0 = w * 64;
        const int q1 = min(m, q0 + 64);
        const int qa = max(q0, lo), qb = min(q1, hi + 1);
        // every lane takes part in the shuffles; only words < W are kept
        const bool inside = w < W && qa < qb;
        const int nin = inside ? qb - qa : 1;
        // source of bit qa: lo + (qa - lo - move) mod L; with qa - lo in
        // [0, L) and the drawn move in [1, L) one conditional add reduces it
        int t = qa - lo - move;
        t += t < 0 ? L : 0;
        const int s0 = inside ? lo + t : lo;
        const uint64_t part = cyclic_bits(A, W, lo, hi, s0, nin);
        if (w < W) {
            uint64_t val = A.v[h];
            if (inside) {
                const uint64_t mask =
                    (nin == 64 ? ~0ull : ((1ull << nin) - 1ull)) << (qa - q0);
                val = (val & ~mask) | (part << (qa - q0));
            }
            changed |= val != A.v[h];
            store_word(F, w, val);
        }
    }
    return __builtin_amdgcn_ballot_w64(changed) != 0ull;
}

// ---------------------------------------------------------------------------
// One stage (Evolve steps 3 and 5) for chromosome c, by its wave.  Finish
// the previous operator (take the evaluated offspring if strictly fitter:
// Evolve steps 3e and 5c), then start operator `op`:
//  - crossover stage `index`: stride NT >> (1 + index mod lg NT), partner
//    c XOR stride; the pair's lower slot owns the draws r1 in [0, m) and
//    i in [1, floor(p/2)] (Section 4.3);
//  - mutation attempt `index`: skipped once the cycle has improved c;
//    draws type, direction, then the amount s in [1, m-1] or the block ends
//    (a uniform pair of distinct positions) and s in [1, b - a]; an
//    offspring equal to its parent is not evaluated (Section 4.4).
// The draws were made with the population (ga_draws_one).  All of the step's
// loads are issued together; the operators then work on the words held by
// the lanes.
// ---------------------------------------------------------------------------
//
// With op = OP_MUT_ALL the stage runs on ceil(Y / mpw) waves per chromosome:
// wave `sub` makes mutants sub mpw ... of the parent, and only wave 0 writes
// the chromosome's own state (every wave computes the same parent from the
// same loads).
// Everything one stage step of chromosome c reads, loaded in one round:
// every load is unconditional at an address that is always valid (clamped
// index; the partner is c itself when no crossover runs) and values outside
// the range are masked afterwards.
struct StageLoad {
    uint64_t gen;
    int32_t sj, sk;
    uint8_t okc_b, okp_b, imp_b;
    unsigned long long fin, fpin, cs_old;
    unsigned long long pf0, ph0, pf1, ph1;  // partial sums of client tiles 0-127
    uint32_t ps0, ps1;
    WaveWords cc, oc, cp, opw;  // own and partner's chromosome and offspring
    OpDraw dr;
};

__device__ __forceinline__ int stage_partner(const GaArgs &g, int c, int op, int index)
{
    return op == OP_XOVER ? (c ^ (g.NT >> (1 + index % g.lg))) : c;
}

__device__ __forceinline__ void stage_load(const GaArgs &g, int c, int lane, int in, int op,
                                           int index, StageLoad &L)
{
    const int W = g.t.W;
    const bool xo = op == OP_XOVER;
    const int pc = stage_partner(g, c, op, index);
    L.gen = g.gs[GS_GEN];
    L.sj = 0;
    L.sk = 0;
    if (op == OP_SWAP) {
        const int32_t *sw = g.swaps + ((int64_t)c * g.L + index) * 2;
        L.sj = sw[0];
        L.sk = sw[1];
    }
    L.okc_b = buf(g.ok, in)[c];
    L.okp_b = buf(g.ok, in)[pc];
    L.fin = buf(g.fit, in)[c];
    L.fpin = buf(g.fit, in)[pc];
    L.imp_b = g.improved[c];
    // lane k < CS_COUNT holds counter k of chromosome c
    L.cs_old = g.cstat[(int64_t)c * CS_COUNT + (lane < CS_COUNT ? lane : 0)];
    // partial sums of the first 128 client tiles (straight-line; more tiles
    // are added when the step finishes); tile t of chromosome x at
    // t * ts + x * xs
    const int64_t ts = g.pcm ? 1 : g.P, xs = g.pcm ? g.TI : 1;
    const int64_t row0 = (int64_t)min(lane, g.TI - 1) * ts;
    L.pf0 = g.part[row0 + c * xs];
    L.ph0 = g.part[row0 + pc * xs];
    L.ps0 = g.spart[row0 + c * xs];
    // tiles 64..127 in the same round (the branch is uniform)
    L.pf1 = 0;
    L.ph1 = 0;
    L.ps1 = 0;
    if (g.TI > 64) {
        const int64_t row1 = (int64_t)min(lane + 64, g.TI - 1) * ts;
        L.pf1 = g.part[row1 + c * xs];
        L.ph1 = g.part[row1 + pc * xs];
        L.ps1 = g.spart[row1 + c * xs];
    }
    L.cc = WaveWords{};
    L.oc = WaveWords{};
    L.cp = WaveWords{};
    L.opw = WaveWords{};
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        if (k == 1 && W <= 64)
            break;
        const int w = lane + 64 * k;
        const int wl = min(w, W - 1);
        const uint64_t a0 = buf(g.cur, in)[(int64_t)c * W + wl];
        const uint64_t a1 = buf(g.off, in)[(int64_t)c * W + wl];
        const uint64_t a2 = buf(g.cur, in)[(int64_t)pc * W + wl];
        const uint64_t a3 = buf(g.off, in)[(int64_t)pc * W + wl];
        L.cc.v[k] = w < W ? a0 : 0ull;
        L.oc.v[k] = w < W ? a1 : 0ull;
        L.cp.v[k] = w < W ? a2 : 0ull;
        L.opw.v[k] = w < W ? a3 : 0ull;
    }
    // the operator's draws (the branch is uniform); for the whole mutation
    // cycle, lane a loads attempt a's
    L.dr = OpDraw{0, 0, 0, 0};
    if (xo || op == OP_MUT) {
        const int leader = c < pc ? c : pc;
        L.dr = g.draws[(int64_t)(xo ? leader : c) * (g.X + g.Y) + (xo ? index : g.X + index)];
    } else if (op == OP_MUT_ALL) {
        L.dr = g.draws[(int64_t)c * (g.X + g.Y) + g.X + min(lane, g.Y - 1)];
    }
}

// The rest of the stage step from its loads.  `primary`: this wave writes
// the chromosome's state (population, fitness, flags, counters); F receives
// the new offspring's words.  Returns whether an offspring was made.
template <class Out>
__device__ __forceinline__ bool stage_finish(const GaArgs &g, int c, int lane, int in,
                                             int prev, int op, int index, int sub,
                                             bool primary, const StageLoad &L, const Out &F)
{
    const int out = in ^ 1;
    const int W = g.t.W, m = g.t.m;
    const bool xo = op == OP_XOVER;
    const int pc = stage_partner(g, c, op, index);
    const uint64_t gen = L.gen;
    const OpDraw dr = L.dr;
    const bool use0 = lane < g.TI, use1 = lane + 64 < g.TI;
    unsigned long long f = (use0 ? L.pf0 : 0ull) + (use1 ? L.pf1 : 0ull);
    unsigned long long h = (use0 ? L.ph0 : 0ull) + (use1 ? L.ph1 : 0ull);
    unsigned long long s = (unsigned long long)(use0 ? L.ps0 : 0u) + (use1 ? L.ps1 : 0u);
    const int64_t ts = g.pcm ? 1 : g.P, xs = g.pcm ? g.TI : 1;
    for (int t0 = 128; t0 < g.TI; t0 += 64) {
        const bool use = t0 + lane < g.TI;
        const int64_t row = (int64_t)min(t0 + lane, g.TI - 1) * ts;
        const unsigned long long pf = g.part[row + c * xs], ph = g.part[row + pc * xs];
        const uint32_t ps = g.spart[row + c * xs];
        f += use ? pf : 0ull;
        s += use ? ps : 0u;
        h += use ? ph : 0ull;
    }
    // prev == OP_NONE: the previous operator was already finished (the
    // learned proposal ran in between), so there is nothing to take
    const bool okc = L.okc_b != 0 && prev != OP_NONE;
    const bool okp = xo && L.okp_b != 0;
    const bool was_improved = L.imp_b != 0;
    const unsigned long long fin = L.fin, fpin = L.fpin;

    const int r1 = dr.a, quota = dr.b;
    const int lo = op == OP_MUT ? dr.a : 0, hi = op == OP_MUT ? dr.b : m - 1;
    const int move = dr.c;

    // finish the previous operator: c, and for a crossover the partner
    const unsigned long long fo = wave_sum(f), scan = wave_sum(s), fop = wave_sum(h);
    const bool take = okc && fo < fin;
    const bool ptake = okp && fop < fpin;
    const WaveWords A = take ? L.oc : L.cc;
    uint64_t *cur = buf(g.cur, out) + (int64_t)c * W;
#pragma unroll
    for (int k = 0; k < 2; ++k)
        if (primary && lane + 64 * k < W)
            cur[lane + 64 * k] = A.v[k];
    const bool mut_prev = prev == OP_MUT || prev == OP_SWAP;
    const bool improved = was_improved || (mut_prev && take);
    // this stage's counter increments, lane k for counter k
    unsigned long long cs_inc = 0;
    if (okc) {
        cs_inc += lane == CS_EVALS ? 1ull : 0ull;
        cs_inc += lane == CS_SCAN ? scan : 0ull;
    }
    if (take && prev == OP_XOVER)
        cs_inc += lane == CS_XO_TAKEN ? 1ull : 0ull;
    if (take && mut_prev)
        cs_inc += lane == (prev == OP_MUT ? CS_MUT_TAKEN : CS_SWAP_TAKEN) ? 1ull : 0ull;
    if (prev == OP_SWAP && okc)
        cs_inc += lane == CS_SWAP_TRIED ? 1ull : 0ull;
    if (primary && lane == 0) {
        buf(g.fit, out)[c] = take ? fo : fin;
        if (take && mut_prev)
            g.improved[c] = 1;
        if (prev == OP_SWAP && okc) {
            // training tuple of attempt index - 1: exact change of cost,
            // normalised by the parent's cost per open facility, clamped
            const int64_t slot =
                ((int64_t)(gen % (uint64_t)g.H) * g.L + (index - 1)) * g.P + c;
            const long long delta = (long long)fo - (long long)fin;
            double tv = (double)delta * (double)g.t.p / (fin > 0 ? (double)fin : 1.0);
            tv = tv < -4.0 ? -4.0 : (tv > 4.0 ? 4.0 : tv);
            g.rep_d[2 * slot] = delta;
            g.rep_t[slot] = (float)tv;
            g.rep_w[slot] = 1.f;
        }
    }

    // start the next operator
    bool ok = false;
    if (xo) {
        const WaveWords B = ptake ? L.opw : L.cp;
        ok = crossover_wave(A, B, F, W, r1, quota, lane);
        if (!ok)
            cs_inc += lane == CS_XO_FAIL ? 1ull : 0ull;
    } else if (op == OP_MUT && !improved) {
        ok = mutate_wave(A, F, W, m, lo, hi, move, lane);
    } else if (op == OP_MUT_ALL) {
        // every attempt mutates the same parent A (the cycle has not improved
        // it yet); ga_resolve_one takes the first strictly fitter mutant
        const int a1 = min(g.Y, (sub + 1) * g.mpw);
        for (int a = sub * g.mpw; a < a1; ++a) {
            const int64_t row = (int64_t)c * g.Y + a;
            bool ch = true;
            if (a < g.L) {  // scored swap: close its j, open its k
                const int32_t *swp = g.swaps + ((int64_t)c * g.L + a) * 2;
                const int aj = swp[0], ak = swp[1];
                uint64_t *Fm = g.mut + row * W;
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    const int w = lane + 64 * k;
                    if (w < W) {
                        uint64_t v = A.v[k];
                        if ((aj >> 6) == w)
                            v ^= 1ull << (aj & 63);
                        if ((ak >> 6) == w)
                            v ^= 1ull << (ak & 63);
                        Fm[w] = v;
                    }
                }
            } else {
                const int lo_a = __builtin_amdgcn_readlane(dr.a, a);
                const int hi_a = __builtin_amdgcn_readlane(dr.b, a);
                const int mv_a = __builtin_amdgcn_readlane(dr.c, a);
                ch = mutate_wave(A, g.mut + row * W, W, m, lo_a, hi_a, mv_a, lane);
            }
            if (lane == 0)
                g.mut_ok[row] = ch ? 1 : 0;
        }
    } else if (op == OP_SWAP && !improved) {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int w = lane + 64 * k;
            if (w < W) {
                uint64_t v = A.v[k];
                if ((L.sj >> 6) == w)
                    v ^= 1ull << (L.sj & 63);
                if ((L.sk >> 6) == w)
                    v ^= 1ull << (L.sk & 63);
                store_word(F, w, v);
            }
        }
        ok = true;
    }
    if (primary && lane == 0)
        buf(g.ok, out)[c] = ok ? 1 : 0;
    if (primary && lane < CS_COUNT && cs_inc != 0ull)
        g.cstat[(int64_t)c * CS_COUNT + lane] = L.cs_old + cs_inc;
    return ok;
}

__device__ __forceinline__ void ga_stage_one(const GaArgs &g, int c, int lane,
                                             int in, int prev, int op,
                                             int index, int sub = 0)
{
    StageLoad L;
    stage_load(g, c, lane, in, op, index, L);
    if (ga_stopped(g))  // checked once the loads are on their way
        return;
    stage_finish(g, c, lane, in, prev, op, index, sub, sub == 0, L,
                 buf(g.off, in ^ 1) + (int64_t)c * g.t.W);
}

// ---------------------------------------------------------------------------
// The mutation cycle resolved at once (Evolve step 5).  All Y attempts mutate
// the same parent - the chromosome as the crossover cycle left it - until one
// is strictly fitter, after which the cycle stops; so having evaluated every
// mutant together, taking the first strictly fitter one in attempt order
// gives exactly the sequential cycle's result.  The counters count what the
// sequential cycle evaluates (mutants that differ from the parent, up to and
// including the first improvement); the others go to the speculative
// counters.
//
// A wave takes 64 / YP chromosomes (YP = Y rounded up to a power of two),
// lane (c, a) for mutant a of chromosome c: it adds up its mutant's client
// tile partial sums (consecutive lanes read consecutive entries), and a
// ballot over the chromosome's lanes finds the first improvement.  Reads
// buffer `in`, writes buffer `out` (possibly the same: a lane reads the words
// it then writes).  Y <= 64.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void ga_resolve_wave(const GaArgs &g, int gw, int lane, int YP,
                                                int in, int out, bool mark_improved = true)
{
    const int W = g.t.W, Y = g.Y;
    const int64_t PY = (int64_t)g.P * Y;
    const int per = 64 / YP, grp = lane / YP, a = lane - grp * YP;
    const int c = gw * per + grp;
    const bool valid_c = c < g.P, valid = valid_c && a < Y;
    const int cc = min(c, g.P - 1);
    const int64_t row = (int64_t)cc * Y + min(a, Y - 1);
    const uint8_t okm = g.mut_ok[row];
    const unsigned long long fin = buf(g.fit, in)[cc];
    unsigned long long *cs = g.cstat + (int64_t)cc * CS_COUNT;
    // the group leader's counters (the other lanes load them too, unused)
    const unsigned long long c_ev = cs[CS_EVALS], c_sc = cs[CS_SCAN], c_mt = cs[CS_MUT_TAKEN];
    const unsigned long long c_se = cs[CS_SPEC_EVALS], c_ss = cs[CS_SPEC_SCAN];
    const unsigned long long c_st = cs[CS_SWAP_TRIED], c_sk = cs[CS_SWAP_TAKEN];
    unsigned long long f = 0, sc = 0;
#pragma unroll 16
    for (int t = 0; t < g.TIm; ++t) {  // up to 16 tiles' loads in one round
        f += g.mpart[(int64_t)t * PY + row];
        sc += g.mspart[(int64_t)t * PY + row];
    }
    if (ga_stopped(g))  // checked once the loads are on their way (uniform)
        return;
    const bool ok_l = valid && okm != 0;
    const uint64_t gmask = (YP == 64 ? ~0ull : ((1ull << YP) - 1ull)) << (grp * YP);
    const uint64_t imp = __builtin_amdgcn_ballot_w64(ok_l && f < fin) & gmask;
    const int first = imp ? __builtin_ctzll(imp) : -1;  // lane of the taken mutant
    const uint64_t upto = first < 0 ? ~0ull : (first == 63 ? ~0ull : ((2ull << first) - 1ull));
    const bool counted = ok_l && ((upto >> lane) & 1ull);
    const bool spec = ok_l && !counted;
    unsigned long long s_cnt = counted ? sc : 0ull, s_spec = spec ? sc : 0ull;
    for (int d = 1; d < YP; d <<= 1) {  // sums within the chromosome's lanes
        s_cnt += __shfl_xor(s_cnt, d);
        s_spec += __shfl_xor(s_spec, d);
    }
    const int n_cnt = __builtin_popcountll(__builtin_amdgcn_ballot_w64(counted) & gmask);
    const int n_spec = __builtin_popcountll(__builtin_amdgcn_ballot_w64(spec) & gmask);
    const unsigned long long f_taken = __shfl(f, first < 0 ? lane : first);
    const int taken = first < 0 ? -1 : first - grp * YP;
    // learned proposal: the first L attempts are scored swaps; each one the
    // attempt-by-attempt cycle evaluates leaves its training tuple
    const bool swap_l = counted && a < g.L;
    const int n_swap = __builtin_popcountll(__builtin_amdgcn_ballot_w64(swap_l) & gmask);
    if (swap_l) {
        const uint64_t gen = g.gs[GS_GEN];
        const int64_t slot = ((int64_t)(gen % (uint64_t)g.H) * g.L + a) * g.P + cc;
        const long long delta = (long long)f - (long long)fin;
        double tv = (double)delta * (double)g.t.p / (fin > 0 ? (double)fin : 1.0);
        tv = tv < -4.0 ? -4.0 : (tv > 4.0 ? 4.0 : tv);
        g.rep_d[2 * slot] = delta;
        g.rep_t[slot] = (float)tv;
        g.rep_w[slot] = 1.f;
    }
    // the chromosome: the taken mutant or the parent, word w by lane w mod YP
    if (valid_c) {
        uint64_t *dst = buf(g.cur, out) + (int64_t)cc * W;
        const uint64_t *src = taken >= 0 ? g.mut + ((int64_t)cc * Y + taken) * W
                                         : buf(g.cur, in) + (int64_t)cc * W;
        for (int w = a; w < W; w += YP)
            dst[w] = src[w];
    }
    if (valid_c && a == 0) {
        buf(g.fit, out)[cc] = taken >= 0 ? f_taken : fin;
        buf(g.ok, out)[cc] = 0;
        if (taken >= 0 && mark_improved)
            g.improved[cc] = 1;
        if (n_cnt) {
            cs[CS_EVALS] = c_ev + (unsigned long long)n_cnt;
            cs[CS_SCAN] = c_sc + s_cnt;
        }
        if (taken >= 0 && taken < g.L)
            cs[CS_SWAP_TAKEN] = c_sk + 1ull;
        else if (taken >= 0)
            cs[CS_MUT_TAKEN] = c_mt + 1ull;
        if (n_swap)
            cs[CS_SWAP_TRIED] = c_st + (unsigned long long)n_swap;
        if (n_spec) {
            cs[CS_SPEC_EVALS] = c_se + (unsigned long long)n_spec;
            cs[CS_SPEC_SCAN] = c_ss + s_spec;
        }
    }
}

// Reduce (cost, index) pairs of a workgroup to the least cost, lowest index
// on ties.  All threads call it; the result is in sc[0], si[0].
__device__ __forceinline__ void block_argmin(unsigned long long f, int idx,
                                             unsigned long long *sc, int *si)
{
    const int lane = threadIdx.x & 63, wave = wave_id();
    const int nwaves = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        const unsigned long long of = __shfl_xor(f, d);
        const int oi = __shfl_xor(idx, d);
        if (of < f || (of == f && oi < idx)) {
            f = of;
            idx = oi;
        }
    }
    __syncthreads();
    if (lane == 0) {
        sc[wave] = f;
        si[wave] = idx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < nwaves; ++w)
            if (sc[w] < sc[0] || (sc[w] == sc[0] && si[w] < si[0])) {
                sc[0] = sc[w];
                si[0] = si[w];
            }
    }
    __syncthreads();
}

// Group best of group b (Evolve steps 7-8: least fitness, lowest slot on
// ties) from population buffer fb, by a whole workgroup.
__device__ __forceinline__ void ga_group_best(const GaArgs &g, int fb, int b,
                                              unsigned long long *sc, int *si,
                                              uint64_t *next_pop = nullptr)
{
    unsigned long long f = ~0ull;
    int idx = 0x7FFFFFFF;
    for (int t = threadIdx.x; t < g.NT; t += blockDim.x) {
        const unsigned long long v = buf(g.fit, fb)[(int64_t)b * g.NT + t];
        if (v < f) {  // t ascends per thread: keeps the lowest slot
            f = v;
            idx = t;
        }
    }
    block_argmin(f, idx, sc, si);
    const int W = g.t.W;
    const uint64_t *src = buf(g.cur, fb) + ((int64_t)b * g.NT + si[0]) * W;
    // next_pop: the next generation's population, made ahead; the group
    // best is its migrant (slot b * NT, or b with the one-block variant)
    const int64_t slot = g.migration == PMP_MIG_ONE_BLOCK ? b : (int64_t)b * g.NT;
    for (int w = threadIdx.x; w < W; w += blockDim.x) {
        const uint64_t v = src[w];
        g.gmask[(int64_t)b * W + w] = v;
        if (next_pop)
            next_pop[slot * W + w] = v;
    }
    if (threadIdx.x == 0)
        g.gcost[b] = sc[0];
}

// The run state after a generation: global best, saturation count, stop
// test (Section 3.1 host steps 13-15), by one workgroup; the caller supplies
// the least cost found and how to load word w of its mask.
template <class LoadWord>
__device__ __forceinline__ void ga_update_state(const GaArgs &g, unsigned long long cost,
                                                LoadWord load, unsigned long long prev_best)
{
    const bool better = cost < prev_best;
    const int W = g.t.W;
    if (better)
        for (int w = threadIdx.x; w < W; w += blockDim.x)
            g.best_mask[w] = load(w);
    __syncthreads();
    if (threadIdx.x == 0) {
        if (better) {
            g.gs[GS_BEST] = cost;
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

// Global best straight from the population: the least fitness over all P
// slots, lowest slot on ties.  Groups are contiguous slot ranges, so this is
// the least group best with the lowest group on ties, without waiting for
// the other groups' results.
__device__ __forceinline__ void ga_global_direct(const GaArgs &g, int fb,
                                                 unsigned long long *sc, int *si)
{
    const unsigned long long prev_best = g.gs[GS_BEST];  // loaded with the fitness
    unsigned long long f = ~0ull;
    int idx = 0x7FFFFFFF;
    for (int t = threadIdx.x; t < g.P; t += blockDim.x) {
        const unsigned long long v = buf(g.fit, fb)[t];
        if (v < f) {  // t ascends per thread: keeps the lowest slot
            f = v;
            idx = t;
        }
    }
    block_argmin(f, idx, sc, si);
    const uint64_t *src = buf(g.cur, fb) + (int64_t)si[0] * g.t.W;
    ga_update_state(g, sc[0], [src](int w) { return src[w]; }, prev_best);
}

// Global best, saturation count and stop test (Section 3.1 host steps
// 13-15), by one workgroup once every group best is written and visible.
__device__ __forceinline__ void ga_global(const GaArgs &g,
                                          unsigned long long *sc, int *si)
{
    const unsigned long long prev_best = g.gs[GS_BEST];
    unsigned long long f = ~0ull;
    int idx = 0x7FFFFFFF;
    for (int k = threadIdx.x; k < g.NB; k += blockDim.x) {
        const unsigned long long v =
            __hip_atomic_load(g.gcost + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (v < f) {
            f = v;
            idx = k;
        }
    }
    block_argmin(f, idx, sc, si);
    const uint64_t *src = g.gmask + (int64_t)si[0] * g.t.W;
    ga_update_state(g, sc[0], [src](int w) {
        return __hip_atomic_load(src + w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }, prev_best);
}

}  // namespace pmp
