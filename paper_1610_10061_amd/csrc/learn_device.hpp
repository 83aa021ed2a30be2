// Features of the learned swap proposal (not in the paper): per facility
// and chromosome, integer sums gathered while walking each client's Pi' row
// (the walk of Section 4.2, continued to the second open facility), then
// normalised into 16 FP32 features.
//
// For chromosome x and client i, with positions counted in the truncated
// row Pi'_i (K = m - p + 1 entries, ordered by (d_ij, j)):
//   s1, a_i, c1_i   first open position, its facility and cost (Eq. (6)'s
//                   term for client i);
//   s2, b_i, c2_i   second open position, facility and cost; when the row
//                   holds no second open facility, c2_i = D'_{i,K} (the
//                   least cost the second open facility can have) and b_i
//                   is none.
// Integer sums per facility j:
//   open j:   count   = #{i : a_i = j}            served = sum c1_i over them
//             loss    = sum (c2_i - c1_i) over them (cost of closing j)
//             cnt2    = #{i : b_i = j}            c2share = sum (c2_i - c1_i)
//   closed j: ahead   = #{i : j before s1}        gain = sum (c1_i - d_ij)
//             bcount  = #{i : j between s1, s2}   bgain = sum (c2_i - d_ij)
//             ("between": after s1 and before s2, or up to K without s2)
// The features (f = cost of x, F = max(f, 1), T = max(sum of d, 1)):
//    0 open flag           1 count p/n       2 served p/F     3 loss p/F
//    4 cnt2 p/n            5 c2share p/F     6 ahead p/n      7 gain p/F
//    8 bcount p/n          9 bgain p/F      10 colsum_j m/T
//   11 near_j m/(n L)      (near_j = #{i : j among the first L = ceil(m/p)
//                           entries of Pi'_i})
//   12 p/m                13 f m/T          14 generation fraction   15 one
// Each is computed as (float)(a * b / c) in double from integers, so any
// implementation that follows the definition gets the same bits.
#pragma once

#include "common.hpp"
#include "mlp.hpp"

namespace pmp {

constexpr int kSlots = 128;      // facilities gathered per workgroup
constexpr int kFeatures = 16;

// Per-slot sums in LDS; a slot holds one facility, open or closed, so the
// open and closed sums share storage.
struct SlotBins {
    uint32_t a[kSlots];             // count | ahead
    uint32_t dd[kSlots];            // cnt2 | bcount
    unsigned long long b[kSlots];   // served | gain
    unsigned long long cc[kSlots];  // loss | bgain
    unsigned long long e[kSlots];   // c2share
};

__device__ __forceinline__ void bins_clear(SlotBins &B)
{
    for (int s = threadIdx.x; s < kSlots; s += blockDim.x) {
        B.a[s] = 0;
        B.dd[s] = 0;
        B.b[s] = 0;
        B.cc[s] = 0;
        B.e[s] = 0;
    }
}

__device__ __forceinline__ bool mask_bit(const uint32_t *smask, int f)
{
    return (smask[f >> 5] >> (f & 31)) & 1u;
}

// Add one Pi' entry's terms to its slot: position pos of client i's row
// (facility's slot sl >= 0, distance dist), first / second open positions
// s1 / s2 (s2 = -1: none inside the row), costs c1 / c2.  Branch-free: the
// counter and sum are chosen by selects, and the first open facility's loss
// term is a third add (of zero for the other positions).
__device__ __forceinline__ void add_terms(SlotBins &B, int sl, int pos, int s1, int s2,
                                          int32_t c1, int32_t c2, int32_t dist)
{
    const bool upto1 = pos <= s1, first = pos == s1, second = pos == s2;
    // counts: ahead and first open -> a; between and second open -> dd
    atomicAdd(upto1 ? &B.a[sl] : &B.dd[sl], 1u);
    // sums: ahead -> gain, first -> served, second -> c2share, between -> bgain
    unsigned long long *sum = upto1 ? &B.b[sl] : (second ? &B.e[sl] : &B.cc[sl]);
    const int32_t v = pos < s1 ? c1 - dist : (first ? c1 : (second ? c2 - c1 : c2 - dist));
    atomicAdd(sum, (unsigned long long)v);
    atomicAdd(&B.cc[sl], first ? (unsigned long long)(c2 - c1) : 0ull);  // loss
}

// Walk client i's row (its first chunk already loaded: fac0/dist0 = entry
// `lane`, meaningful below K) and add its terms to the slots `slot(facility)`
// names (-1: not gathered).  Returns c1_i (wave-uniform), or -1 if the row
// holds no open facility (infeasible chromosome).
template <class SlotFn>
__device__ __forceinline__ int32_t scan_client(const Tables &t, int i, int fac0,
                                               int32_t dist0, const uint32_t *smask,
                                               const SlotFn &slot, SlotBins &B, int lane)
{
    const int K = t.K;
    const bool valid0 = lane < K;
    const uint64_t bits0 = __builtin_amdgcn_ballot_w64(valid0 && mask_bit(smask, fac0));
    if (__builtin_popcountll(bits0) >= 2) {
        // common case: both open positions inside the first chunk
        const int s1 = (int)__builtin_ctzll(bits0);
        const int s2 = (int)__builtin_ctzll(bits0 & (bits0 - 1));
        const int32_t c1 = __builtin_amdgcn_readlane(dist0, s1);
        const int32_t c2 = __builtin_amdgcn_readlane(dist0, s2);
        const int sl = lane <= s2 ? slot(fac0) : -1;
        if (sl >= 0)
            add_terms(B, sl, lane, s1, s2, c1, c2, dist0);
        return c1;
    }
    // general case: positions beyond the first chunk
    const uint16_t *prow = t.pi + (int64_t)i * t.pitch;
    const int32_t *drow = t.ds + (int64_t)i * t.pitch;
    int s1 = -1, s2 = -1;
    int32_t c1 = 0, c2 = 0;
    for (int base = 0; base < K && s2 < 0; base += 64) {
        const bool valid = base + lane < K;
        int fac = fac0;
        int32_t dist = dist0;
        if (base > 0) {
            fac = valid ? (int)prow[base + lane] : 0;
            dist = valid ? drow[base + lane] : 0;
        }
        uint64_t bits = __builtin_amdgcn_ballot_w64(valid && mask_bit(smask, fac));
        if (s1 < 0 && bits) {
            const int l = (int)__builtin_ctzll(bits);
            s1 = base + l;
            c1 = __builtin_amdgcn_readlane(dist, l);
            bits &= bits - 1;
        }
        if (s1 >= 0 && bits) {
            const int l = (int)__builtin_ctzll(bits);
            s2 = base + l;
            c2 = __builtin_amdgcn_readlane(dist, l);
        }
    }
    if (s1 < 0)
        return -1;
    if (s2 < 0)
        c2 = drow[K - 1];
    const int end = s2 >= 0 ? s2 + 1 : K;
    for (int base = 0; base < end; base += 64) {
        const int pos = base + lane;
        int fac = fac0;
        int32_t dist = dist0;
        if (base > 0 && pos < end) {
            fac = prow[pos];
            dist = drow[pos];
        }
        const int sl = pos < end ? slot(fac) : -1;
        if (sl >= 0)
            add_terms(B, sl, pos, s1, s2, c1, c2, dist);
    }
    return c1;
}

// Everything the normalisation needs besides the slot sums.
struct FeatCtx {
    int32_t n, m, p, near_len;
    int64_t f, total;
    float gen_frac;
    const unsigned long long *colsum;  // m
    const uint32_t *nearc;             // m
};

__device__ __forceinline__ float fdiv3(double a, double b, double c)
{
    return (float)(a * b / c);
}

// The 16 features of facility j from its five sums (A = count | ahead,
// D = cnt2 | bcount, Bv = served | gain, Cv = loss | bgain, E = c2share).
__device__ __forceinline__ void features16_sums(const FeatCtx &x, double A, double D,
                                                double Bv, double Cv, double E, int j,
                                                bool open, float out[kFeatures])
{
    const double n = x.n, m = x.m, p = x.p;
    const double F = x.f > 0 ? (double)x.f : 1.0;
    const double T = x.total > 0 ? (double)x.total : 1.0;
    out[0] = open ? 1.f : 0.f;
    out[1] = open ? fdiv3(A, p, n) : 0.f;
    out[2] = open ? fdiv3(Bv, p, F) : 0.f;
    out[3] = open ? fdiv3(Cv, p, F) : 0.f;
    out[4] = open ? fdiv3(D, p, n) : 0.f;
    out[5] = open ? fdiv3(E, p, F) : 0.f;
    out[6] = open ? 0.f : fdiv3(A, p, n);
    out[7] = open ? 0.f : fdiv3(Bv, p, F);
    out[8] = open ? 0.f : fdiv3(D, p, n);
    out[9] = open ? 0.f : fdiv3(Cv, p, F);
    out[10] = fdiv3((double)x.colsum[j], m, T);
    out[11] = fdiv3((double)x.nearc[j], m, n * (double)x.near_len);
    out[12] = (float)(p / m);
    out[13] = fdiv3((double)x.f, m, T);
    out[14] = x.gen_frac;
    out[15] = 1.f;
}

// Half `half` (features 8 half .. 8 half + 7) of features16_sums, with six
// divisions whatever the half and the open flag (the operands are selected,
// the results the same bit for bit): the lanes of a wave that split a row's
// features this way all run the same instructions.
__device__ __forceinline__ void features8_sums(const FeatCtx &x, double A, double D, double Bv,
                                               double Cv, double E, int j, bool open, int half,
                                               float out[8])
{
    const double n = x.n, m = x.m, p = x.p;
    const double F = x.f > 0 ? (double)x.f : 1.0;
    const double T = x.total > 0 ? (double)x.total : 1.0;
    const bool h = half != 0;
    const float s0 = fdiv3(h ? D : A, p, n);
    const float s1 = fdiv3(h ? Cv : Bv, p, F);
    const double cs = (double)x.colsum[j], nc = (double)x.nearc[j];
    const float s2 = fdiv3(h ? cs : Cv, h ? m : p, h ? T : F);
    const float s3 = fdiv3(h ? nc : D, h ? m : p, h ? n * (double)x.near_len : n);
    const float s4 = fdiv3(h ? p : E, h ? 1.0 : p, h ? m : F);  // (p * 1 / m = p / m)
    const float s5 = fdiv3(h ? (double)x.f : 0.0, h ? m : 1.0, h ? T : 1.0);
    if (!h) {
        out[0] = open ? 1.f : 0.f;
        out[1] = open ? s0 : 0.f;
        out[2] = open ? s1 : 0.f;
        out[3] = open ? s2 : 0.f;
        out[4] = open ? s3 : 0.f;
        out[5] = open ? s4 : 0.f;
        out[6] = open ? 0.f : s0;
        out[7] = open ? 0.f : s1;
    } else {
        out[0] = open ? 0.f : s0;
        out[1] = open ? 0.f : s1;
        out[2] = s2;
        out[3] = s3;
        out[4] = s4;
        out[5] = s5;
        out[6] = x.gen_frac;
        out[7] = 1.f;
    }
}

// The 16 features of facility j (slot s of B, or -1 for none gathered).
__device__ __forceinline__ void features16(const FeatCtx &x, const SlotBins &B, int s,
                                           int j, bool open, float out[kFeatures])
{
    features16_sums(x, s >= 0 ? (double)B.a[s] : 0.0, s >= 0 ? (double)B.dd[s] : 0.0,
                    s >= 0 ? (double)B.b[s] : 0.0, s >= 0 ? (double)B.cc[s] : 0.0,
                    s >= 0 ? (double)B.e[s] : 0.0, j, open, out);
}

// Slot sums of every chromosome in device memory: kSlots slots each.
struct SlotSums {
    uint32_t *a, *dd;             // P x kSlots
    unsigned long long *b, *cc, *e;
};

// Arguments of the proposal kernel.
struct LearnArgs {
    GaArgs g;
    MlpDev net;
    const unsigned long long *colsum;  // per-instance static sums
    const uint32_t *nearc;
    int64_t total;
    int32_t near_len;
    int32_t C, L, explore, H;          // candidates, attempts, per mille, ring
    int32_t *swaps;                    // P x L x 2
    uint16_t *rep_x;                   // ring rows x 32 BF16 inputs
    int32_t *rep_jk;                   // ring rows x 2
    long long *rep_d;                  // ring rows x 2
    float *rep_t, *rep_w;              // ring rows
    float *scores;                     // P x C scores of the last proposal
    int32_t *cand;                     // P x C x 2 candidate swaps (j, k)
    uint64_t *cbits;                   // P x W candidate-facility bitmaps
    uint8_t *cpre;                     // P x W slots before each bitmap word
    SlotSums sums;                     // per chromosome and slot
    int32_t clients_per_block, tiles_i;  // client tiling of the walk
    int32_t walk;                      // walk: 0 two passes, else chromosomes per workgroup
    // two-pass walk: per (chromosome, client) the row's first two open
    // positions and their costs, then the index of every row's first kNearL
    // positions by facility
    uint32_t *s12;            // P x n: s1 | s2 << 16 (s2 = 0xFFFF: no second in the row)
    int32_t *c12;             // P x n x 2: c1, c2 (c2 = D'_{i,K-1} without a second)
    const int32_t *near_off;  // m + 1: facility f's entries at [near_off[f], near_off[f + 1])
    const uint2 *near_q;      // entries: (client i << 6 | position k, D'_{i,k})
};

// Positions per row in the facility index of the two-pass walk.
constexpr int kNearL = 64;
// Index of the first min(kNearL, K) positions of every Pi' row by facility:
// per-facility counts, then (offsets from the host's prefix sums) the
// entries, in any order within a facility.
hipError_t launch_near_count(const Tables &t, int32_t *count, hipStream_t s);
hipError_t launch_near_fill(const Tables &t, int32_t *cursor, uint2 *q, hipStream_t s);

hipError_t launch_features(const Tables &t, const uint64_t *masks, int P, const FeatCtx &ctx,
                           float *out, uint32_t *err, hipStream_t s);
// The proposal of one generation (candidates, walk, scoring and picks);
// `in` is the buffer the finished crossover stages read.
hipError_t launch_propose(const LearnArgs &a, int in, hipStream_t s);
// Column sums of d and near counts (first L entries of the Pi' rows); then
// report[0] = the sum of d, report[1] = the error word err (one read-back).
hipError_t launch_static_sums(const int32_t *d, int64_t ld, int n, int m, const uint16_t *pi,
                              int pitch, int L, unsigned long long *colsum, uint32_t *nearc,
                              const uint32_t *err, unsigned long long *report, hipStream_t s);

// Load a chromosome into LDS (as 32-bit words) and check it: exactly p
// open facilities, no bits at positions >= m.  Block-wide; returns the
// check's result to every thread.
__device__ __forceinline__ bool load_mask(const uint64_t *mask, int W, int m, int p,
                                          uint64_t *smask64, int *scount)
{
    if (threadIdx.x == 0)
        *scount = 0;
    __syncthreads();
    int cnt = 0;
    bool stray = false;
    for (int w = threadIdx.x; w < W; w += blockDim.x) {
        uint64_t v = mask[w];
        if (w == W - 1 && (m & 63)) {
            const uint64_t keep = (1ull << (m & 63)) - 1ull;
            stray = (v & ~keep) != 0ull;
        }
        smask64[w] = v;
        cnt += __builtin_popcountll(v);
    }
    if (cnt || stray)
        atomicAdd(scount, stray ? (1 << 20) + cnt : cnt);
    __syncthreads();
    return *scount == p;
}

}  // namespace pmp
