// Population evaluation, device side: Eq. (6), computed as the Fitness function of
// Section 4.2 does it, for a whole population at once.
//
// For chromosome c and client i the walk reads Pi'_i from the front until it
// meets an open facility, at 1-based position s*; the client then costs
// D'_{i,s*} (the sum of the first s* gap terms).  fitness[c] is the sum over
// clients, exact in 64-bit integers.
//
// Mapping (gfx950, wave64).  A workgroup owns a tile of 64 chromosomes and
// a tile of clients; each of its four waves takes every fourth client of the
// tile.  The tile's masks are staged in LDS and turned facility-major once:
// T[j] is a 64-bit word whose bit c says whether facility j is open in
// chromosome c (a 64 x 64 bit transpose per 64 facilities).  For one client
// the wave loads 64 consecutive entries of Pi'_i and D'_i, one per lane
// (coalesced), and every lane reads T of the facility at its position: lane
// k then holds row k of the 64 x 64 bit matrix "position k is open in
// chromosome c".  One more transpose in registers (lane exchanges and bit
// selects, about 35 instructions) gives lane c its column, and the column's
// lowest set bit is chromosome c's first open position in this chunk.  One
// ds_bpermute then fetches each chromosome's D' entry from the lane that
// holds it (the lane is bits 7:2 of its address, so position -1 needs no
// mask: lanes without a hit discard the value), so a chunk costs the same for
// all 64 chromosomes whatever their
// scan lengths up to 64.  Chromosomes still unmatched go on to the next 64
// entries.  This replaces the paper's one-thread-per-chromosome loop: lanes
// never diverge and Pi' rows are read once per 64 chromosomes.
//
// Partial sums of the four waves are combined in LDS and stored, one int64
// per (client tile, chromosome), with plain stores; the consumer (the
// reduction below or the GA's next stage) adds the client tiles up.  Integer
// addition makes the result exact and independent of tiling.  Workgroups
// are numbered so that all chromosome tiles of one client tile run on the
// same XCD and share its L2, and each wave loads the next client's chunk of
// Pi' and D' before it works on the current one.
#pragma once

#include "common.hpp"

namespace pmp {


// Lowest set bit of x, -1 when x is 0 (v_ffbl_b32 returns -1 for zero).
__device__ __forceinline__ int lowest_bit(uint32_t x)
{
    int r;
    asm("v_ffbl_b32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

// The value of v in lane (this lane) ^ J: ds_swizzle's xor mode (within 32
// lanes) for J = 16, 8, 4, DPP quad permutations for J = 2, 1.
template <int J>
__device__ __forceinline__ uint32_t from_lane_xor(uint32_t v)
{
    if constexpr (J >= 4)
        return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x1F | (J << 10));
    else  // every lane has a source, so no old value is needed
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, J == 2 ? 0x4E : 0xB1, 0xF, 0xF, true);
}

// Per-lane operands of the transpose steps J = 16, 8, 4, 2, 1 (index 0-4).
// J = 16 and 8 move whole bytes: a v_perm_b32 byte selector per lane takes
// the kept bytes from the lane's own word and the others from its
// partner's.  J = 4, 2, 1: the bits a lane keeps, and the rotation that
// brings its partner's bits into the others.
struct TransposeLanes {
    uint32_t sel[2], keep[3], rot[3];  // sel: steps 16, 8; keep, rot: steps 4, 2, 1

    __device__ __forceinline__ explicit TransposeLanes(int lane)
    {
        // v_perm_b32(own, partner, sel): selector byte 4-7 = own byte 0-3,
        // 0-3 = partner byte 0-3
        sel[0] = (lane & 16) ? 0x07060302u : 0x01000504u;  // [p2 p3 o2 o3] / [o0 o1 p0 p1]
        sel[1] = (lane & 8) ? 0x07030501u : 0x02060004u;   // [p1 o1 p3 o3] / [o0 p0 o2 p2]
        constexpr uint32_t M[3] = {0x0F0F0F0Fu, 0x33333333u, 0x55555555u};
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            const int J = 4 >> s;
            const bool up = (lane & J) != 0;
            keep[s] = up ? ~M[s] : M[s];
            rot[s] = up ? (uint32_t)J : (uint32_t)(32 - J);
        }
    }
};

// Step J of a 32 x 32 bit transpose (rows in the lanes of each half-wave,
// one 32-bit word per row): exchange bit J of the row and the column index.
// A lane whose row has that bit clear keeps its bits at positions with bit J
// clear and takes its partner's bits moved up by J; the partner keeps the
// others and takes this lane's moved down by J.  Rotations stand in for the
// shifts: the bits they wrap around land in positions that are not taken.
// (a & mask) | (b & ~mask) in one instruction (written out, so that the
// compiler does not split it into ands and ors shared with the next step)
__device__ __forceinline__ uint32_t bit_select(uint32_t mask, uint32_t a, uint32_t b)
{
    uint32_t r;
    asm("v_bfi_b32 %0, %1, %2, %3" : "=v"(r) : "v"(mask), "v"(a), "v"(b));
    return r;
}

template <int S>
__device__ __forceinline__ void transpose_step(uint32_t &lo, uint32_t &hi,
                                               const TransposeLanes &tl)
{
    constexpr int J = 16 >> S;
    const uint32_t ylo = from_lane_xor<J>(lo), yhi = from_lane_xor<J>(hi);
    if constexpr (S < 2) {
        lo = __builtin_amdgcn_perm(lo, ylo, tl.sel[S]);
        hi = __builtin_amdgcn_perm(hi, yhi, tl.sel[S]);
    } else {
        const uint32_t k = tl.keep[S - 2], r = tl.rot[S - 2];
        lo = bit_select(k, lo, __builtin_amdgcn_alignbit(ylo, ylo, r));
        hi = bit_select(k, hi, __builtin_amdgcn_alignbit(yhi, yhi, r));
    }
}

// Transpose of the 64 x 64 bit matrix whose row l is lane l's (hi:lo): on
// return lane c holds column c, bit l = bit c of row l.  Bit 5 of the row and
// column index is exchanged first: v_permlane32_swap of the low and high
// words swaps the low words of lanes 32-63 with the high words of lanes
// 0-31.  Then bits 4 to 0 within each half-wave.
__device__ __forceinline__ void transpose64(uint32_t &lo, uint32_t &hi, int lane,
                                            const TransposeLanes &tl)
{
    (void)lane;
    const auto sw = __builtin_amdgcn_permlane32_swap(lo, hi, false, false);
    lo = (uint32_t)sw[0];
    hi = (uint32_t)sw[1];
    transpose_step<0>(lo, hi, tl);
    transpose_step<1>(lo, hi, tl);
    transpose_step<2>(lo, hi, tl);
    transpose_step<3>(lo, hi, tl);
    transpose_step<4>(lo, hi, tl);
}

// All 64 chromosomes of the tile against one 64-entry chunk: lane k's row is
// T of the facility at its position (0 for positions that do not count).
// Returns, in lane c, chromosome c's first open position in the chunk (-1 if
// none).  first_open2: lanes 0-31 and 32-63 hold the first 32 positions of
// two clients A and B, and lane c gets both clients' first open positions.
__device__ __forceinline__ int first_open(uint64_t row, int lane, const TransposeLanes &tl)
{
    uint32_t lo = (uint32_t)row, hi = (uint32_t)(row >> 32);
    transpose64(lo, hi, lane, tl);
    // v_ffbl gives 0xFFFFFFFF for a zero word: the unsigned minimum of the
    // low word's position and 32 plus the high word's (saturating, so that
    // "none" stays 0xFFFFFFFF) is the first open position, or -1
    const uint32_t a = (uint32_t)lowest_bit(lo);
    const uint32_t b = __builtin_elementwise_add_sat((uint32_t)lowest_bit(hi), 32u);
    return (int)(a < b ? a : b);
}

__device__ __forceinline__ void first_open2(uint64_t row, int lane, const TransposeLanes &tl,
                                            int &hit_a, int &hit_b)
{
    uint32_t lo = (uint32_t)row, hi = (uint32_t)(row >> 32);
    transpose64(lo, hi, lane, tl);
    hit_a = lowest_bit(lo);
    hit_b = lowest_bit(hi);
}

// The rest of one client's walk from position `base` for the chromosomes in
// `pend` (64-entry chunks, loaded here).  sT: the tile's facility-major masks,
// with an all-zero word at index jz for positions past the row.
__device__ __forceinline__ void walk_tail(const EvalArgs &a, const uint16_t *prow,
                                          const int32_t *drow, int base, uint64_t pend,
                                          int lane, const uint64_t *sT, uint32_t jz,
                                          const TransposeLanes &tl, unsigned long long &acc,
                                          uint32_t &scn)
{
    for (; pend != 0ull; base += 64) {
        if (base >= a.t.K) {  // fewer than p open facilities
            if (lane == 0)
                atomicOr(a.err, ERR_SCAN_OVERRUN);
            break;
        }
        const int k = base + lane;
        const bool in = k < a.t.K;
        const int kc = in ? k : a.t.K - 1;
        const uint32_t j = prow[kc];
        const int32_t dist = drow[kc];
        const int hit = first_open(sT[in ? j : jz], lane, tl);
        const bool found = ((pend >> lane) & 1ull) && hit >= 0;
        const int32_t cost = __builtin_amdgcn_ds_bpermute(hit << 2, dist);
        if (found) {
            acc += (uint32_t)cost;
            scn += (uint32_t)(base + hit + 1);
        }
        // (= pend & ~ballot(found): found is hit >= 0 on pend's lanes)
        pend &= ~__builtin_amdgcn_ballot_w64(hit >= 0);
    }
}

// LDS words (32-bit) eval_tile needs for its staged masks: rows of WD words
// at an odd stride WD + 1, so that reading one word of every row (a lane per
// row) hits 64 different banks.  The facility-major copy, 64 W 64-bit words
// and two more (all zeros, all ones), reuses the same space.
template <int WD>
constexpr int eval_stage_words()
{
    static_assert(WD % 2 == 0, "WD is even");
    return kEvalTile * (WD + 1);
}

// Evaluate chromosome tile tc (64 chromosomes) on client tile ti and store
// the tile's partial sums.  Called by a whole workgroup of NV waves (each
// walks every NV-th client of the tile; more waves share one staged tile,
// so more of them are resident per CU and each walks fewer clients);
// smask holds eval_stage_words<WD>() words (8-byte aligned), sred
// 2 * NV * 64 words.
//
// R: the walk tables of the reduced polynomial (k_hbp.hip) instead of the
// instance's: row i stops at position K_i - 1 at the latest (a.rlen) and
// the value read there is the int64 running sum a.e64.  The stop is made
// with no extra work in the walk: the last position's lane takes a row of
// all ones, as if its facility were open in every chromosome.
//
// H (short scans, not with R): a wave walks its clients two at a time, the
// first 32 entries of each row in one chunk (first_open2); the few rows
// whose first open facility lies past entry 31 finish in walk_tail.
//
// PRE: the caller has already staged the tile's masks in smask (rows at
// stride WD + 1, zero past 2W words) and the chromosomes' active flags in
// sact, and synchronised the workgroup (the stage steps fused with the
// evaluation make the offspring right there).
// Clients whose first 64-entry chunk a wave of the single-client walk has
// in flight (loaded up to this many clients ahead, so that the wait for a
// client's chunk falls several clients' work after its load).
constexpr int kPrefetch = 4;

// The first chunks (Pi' entry and D' value of this lane's position) of the
// first clients a lane's wave walks in client tile ti: kPrefetch clients for
// the single-client walk, one pair for the paired walk (H: lanes 32-63 hold
// the pair's second client).  Always in bounds: rows clamped into the tile,
// columns below K.
struct FirstChunks {
    uint32_t j[kPrefetch];
    int32_t d[kPrefetch];
};

template <bool H, int NV>
__device__ __forceinline__ void eval_first_chunks(const EvalArgs &a, int ti, int lane, int wave,
                                                  FirstChunks &fc)
{
    const int i0 = ti * a.clients_per_block;
    const int i1 = min(a.t.n, i0 + a.clients_per_block);
    const int i = i0 + wave, last = i1 - 1;
    const int pos = H ? (lane & 31) : lane;
    const int col = pos < a.t.K ? pos : a.t.K - 1;
    constexpr int Q = H ? 1 : kPrefetch;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int row = (H && lane >= 32) ? min(i + NV, last) : min(i + NV * q, last);
        fc.j[q] = a.t.pi[(int64_t)row * a.t.pitch + col];
        fc.d[q] = a.t.ds[(int64_t)row * a.t.pitch + col];
    }
}

//
// GT: the tile's facility-major copy is in device memory (a.tg; chromosomes
// wider than the LDS staging allows), made and checked by launch_tile_major;
// nothing is staged in LDS.
// live = false: a workgroup past the last tile (called with tile 0), which
// issues the loads and leaves with the stop test, so that no branch comes
// before the loads (the compiler then issues them, and the kernel arguments
// they need, in one round each).
static __device__ const unsigned long long kNoStopFlag = 0ull;

template <int WD, bool R = false, bool H = false, int NV = kEvalWaves, bool PRE = false,
          bool GT = false>
__device__ __forceinline__ void eval_tile(const EvalArgs &a, int ti, int tc,
                                          uint32_t *smask,
                                          unsigned long long *sred,
                                          const uint8_t *sact = nullptr,
                                          const FirstChunks *pre = nullptr,
                                          bool live = true)
{
    constexpr int SD = WD + 1;  // staged row stride
    const int c0 = tc * kEvalTile;
    const int i0 = ti * a.clients_per_block;
    const int i1 = min(a.t.n, i0 + a.clients_per_block);
    const int lane = threadIdx.x & 63;
    const int wave = wave_id();
    const int W = a.t.W, W2 = 2 * W;

    // The tile's independent loads go out together (one memory round trip):
    // this lane's active flag, chunk 0 of the wave's first client, and the
    // tile's masks, staged to LDS whether active or not (an inactive
    // chromosome is never pending, so its stale mask is never consulted).
    const int my_c = c0 + lane;
    int i = i0 + wave;
    // Chunk 0 of the current client is loaded one client ahead.  The loads
    // are unconditional, at a row clamped into the tile and a column clamped
    // below K (always in bounds; lanes at or past K are masked when used), so
    // the compiler never has to wait for a prefetch before using the
    // previous one.
    // (H: lanes 32-63 hold the wave's second client of the pair)
    const int pos = H ? (lane & 31) : lane;
    const int col = pos < a.t.K ? pos : a.t.K - 1;
    const bool in_row = pos < a.t.K;
    const int last = i1 - 1;
    const int row_first = (H && lane >= 32) ? min(i + NV, last) : min(i, last);
    // queue of the next clients' first chunks (the single-client walk keeps
    // kPrefetch in flight; the reduced and paired walks one)
    constexpr int PF = (!H && !R) ? kPrefetch : 1;
    uint32_t jq[PF];
    int32_t dq[PF];
    long long e_cur = 0;
    int k_cur = 0;  // R: the row's length K_i
    if constexpr (PRE) {  // loaded by the caller (eval_first_chunks)
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            jq[q] = pre->j[q];
            dq[q] = pre->d[q];
        }
    } else if constexpr (R) {
        jq[0] = a.t.pi[(int64_t)row_first * a.t.pitch + col];
        dq[0] = 0;
        e_cur = a.e64[(int64_t)min(i, last) * a.t.pitch + col];
        k_cur = a.rlen[min(i, last)];
    } else {
        FirstChunks fc;
        eval_first_chunks<H, NV>(a, ti, lane, wave, fc);
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            jq[q] = fc.j[q];
            dq[q] = fc.d[q];
        }
    }
    uint32_t j_cur = jq[0];
    int32_t d_cur = dq[0];
    // Masks: every load unconditional at a clamped (always valid) address,
    // in batches, so that a batch costs one round trip; out-of-range words
    // are replaced by 0 when stored.
    const uint32_t *g32 = reinterpret_cast<const uint32_t *>(a.masks);
    const int rows = min(kEvalTile, a.P - c0);
    constexpr int kTot = kEvalTile * WD, kThreads = kEvalTile * NV;
    constexpr int kIt = (kTot + kThreads - 1) / kThreads;
    constexpr int kBatch = kIt < 16 ? kIt : 16;
    // active flag: also an unconditional load (of any valid byte when every
    // chromosome is active)
    uint8_t actv = 0;
    // the stop flag of a GA run (a no-op generation), loaded in the same
    // round (PRE: the caller has tested it)
    unsigned long long stop = 0ull;
    if constexpr (!PRE)
        stop = *(a.done ? a.done : &kNoStopFlag);
    if constexpr (PRE) {
        actv = sact[lane];
    } else {
        const uint8_t *ap = a.active ? a.active + min(my_c, a.P - 1) : (const uint8_t *)a.masks;
        actv = *ap;
    }
#pragma unroll
    for (int r0 = 0; !PRE && !GT && r0 < kIt; r0 += kBatch) {
        uint32_t v[kBatch];
#pragma unroll
        for (int r = 0; r < kBatch; ++r) {
            const int k = min((int)threadIdx.x + (r0 + r) * kThreads, kTot - 1);
            const int c = k / WD, w = k - (k / WD) * WD;
            v[r] = g32[(int64_t)(c0 + min(c, rows - 1)) * W2 + min(w, W2 - 1)];
        }
#pragma unroll
        for (int r = 0; r < kBatch; ++r) {
            const int k = (int)threadIdx.x + (r0 + r) * kThreads;
            const int c = k / WD, w = k - (k / WD) * WD;
            if (k < kTot)
                smask[c * SD + w] = (w < W2 && c < rows) ? v[r] : 0u;
        }
    }
    const bool my_act = my_c < a.P && ((!PRE && a.active == nullptr) || actv != 0);
    const uint64_t act = __builtin_amdgcn_ballot_w64(my_act);
    // nothing to do (same in every wave: the whole workgroup leaves), or a
    // stopped GA run, whose later generations are no-ops
    if (!live || act == 0ull || stop != 0ull)
        return;
    if constexpr (!GT)
        __syncthreads();

    // Facility-major copy: wave v turns the tile's 64-bit words v, v + 4, ...
    // (one row per lane) into T[64 w + f], f = 0..63, by one transpose each,
    // in place once every wave has read its rows.
    const uint64_t *sT = nullptr;
    const uint32_t jz = (uint32_t)(64 * W), jone = jz + 1u;
    const TransposeLanes tl(lane);
    if constexpr (GT) {
        sT = a.tg + (int64_t)tc * a.tg_stride;
    } else {
        constexpr int NW = (WD / 2 + NV - 1) / NV;
        uint32_t rlo[NW], rhi[NW];
#pragma unroll
        for (int r = 0; r < NW; ++r) {
            const int w = min(wave + r * NV, W - 1);
            rlo[r] = smask[lane * SD + 2 * w];
            rhi[r] = smask[lane * SD + 2 * w + 1];
        }
        // Feasibility of each chromosome (lane), checked once (first client
        // tile) from the rows just read: each wave counts the open facilities in
        // its words and looks for bits past m in the last word; wave 0 adds the
        // waves' counts up once the copy's barrier has passed.
        __shared__ uint32_t s_ones[NV][kEvalTile];
        __shared__ uint32_t s_stray[NV][kEvalTile];
        if (ti == 0) {
            uint32_t ones = 0, stray = 0;
            const uint64_t past = (a.t.m & 63) ? ~((1ull << (a.t.m & 63)) - 1ull) : 0ull;
#pragma unroll
            for (int r = 0; r < NW; ++r) {
                const int w = wave + r * NV;
                if (w < W) {
                    ones += __builtin_popcount(rlo[r]) + __builtin_popcount(rhi[r]);
                    if (w == W - 1)
                        stray |= (((uint64_t)rhi[r] << 32 | rlo[r]) & past) != 0ull ? 1u : 0u;
                }
            }
            s_ones[wave][lane] = ones;
            s_stray[wave][lane] = stray;
        }
        __syncthreads();
        uint64_t *sTw = reinterpret_cast<uint64_t *>(smask);
        sT = sTw;
#pragma unroll
        for (int r = 0; r < NW; ++r) {
            const int w = wave + r * NV;
            if (w < W) {
                transpose64(rlo[r], rhi[r], lane, tl);
                sTw[w * 64 + lane] = ((uint64_t)rhi[r] << 32) | rlo[r];
            }
        }
        // T[64 W]: no chromosome open (positions that do not count); T[64 W + 1]:
        // every chromosome open (the reduced walk's stop)
        if (wave == 0 && lane < 2)
            sTw[jz + lane] = lane ? ~0ull : 0ull;
        __syncthreads();
        if (ti == 0 && wave == 0 && my_act) {
            uint32_t ones = 0, stray = 0;
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                ones += s_ones[v][lane];
                stray |= s_stray[v][lane];
            }
            if (ones != (uint32_t)a.t.p)
                atomicOr(a.err, ERR_POPCOUNT);
            if (stray)
                atomicOr(a.err, ERR_STRAY_BITS);
        }
    }
    unsigned long long acc = 0;
    uint32_t scn = 0;
    if constexpr (H) {
        for (; i < i1; i += 2 * NV) {
            const int ib = i + NV;
            const bool has_b = ib < i1;
            const int na = min(i + 2 * NV, last), nb = min(i + 3 * NV, last);
            const int rown = lane >= 32 ? nb : na;
            const uint32_t j_nxt = a.t.pi[(int64_t)rown * a.t.pitch + col];
            const int32_t d_nxt = a.t.ds[(int64_t)rown * a.t.pitch + col];
            const bool use = in_row && !(lane >= 32 && !has_b);
            int ha, hb;
            first_open2(sT[use ? j_cur : jz], lane, tl, ha, hb);
            const uint64_t pa = act, pb = has_b ? act : 0ull;
            const bool fa = ((pa >> lane) & 1ull) && ha >= 0;
            const bool fb = ((pb >> lane) & 1ull) && hb >= 0;
            const int32_t ca = __builtin_amdgcn_ds_bpermute(ha << 2, d_cur);
            const int32_t cb = __builtin_amdgcn_ds_bpermute((hb << 2) + 128, d_cur);
            if (fa) {
                acc += (uint32_t)ca;
                scn += (uint32_t)(ha + 1);
            }
            if (fb) {
                acc += (uint32_t)cb;
                scn += (uint32_t)(hb + 1);
            }
            const uint64_t ra = pa & ~__builtin_amdgcn_ballot_w64(ha >= 0);
            const uint64_t rb = pb & ~__builtin_amdgcn_ballot_w64(hb >= 0);
            if (ra)
                walk_tail(a, a.t.pi + (int64_t)i * a.t.pitch, a.t.ds + (int64_t)i * a.t.pitch,
                          32, ra, lane, sT, jz, tl, acc, scn);
            if (rb)
                walk_tail(a, a.t.pi + (int64_t)ib * a.t.pitch, a.t.ds + (int64_t)ib * a.t.pitch,
                          32, rb, lane, sT, jz, tl, acc, scn);
            j_cur = j_nxt;
            d_cur = d_nxt;
        }
    }
    for (; !H && i < i1; i += NV) {
        j_cur = jq[0];
        d_cur = dq[0];
        // refill the queue: the client PF places ahead
#pragma unroll
        for (int q = 0; q + 1 < PF; ++q) {
            jq[q] = jq[q + 1];
            dq[q] = dq[q + 1];
        }
        const int inext = min(i + NV * PF, last);
        jq[PF - 1] = a.t.pi[(int64_t)inext * a.t.pitch + col];
        long long e_nxt = 0;
        int k_nxt = 0;
        if (R) {
            e_nxt = a.e64[(int64_t)inext * a.t.pitch + col];
            k_nxt = a.rlen[inext];
        } else {
            dq[PF - 1] = a.t.ds[(int64_t)inext * a.t.pitch + col];
        }
        const uint16_t *prow = a.t.pi + (int64_t)i * a.t.pitch;
        const int32_t *drow = a.t.ds + (int64_t)i * a.t.pitch;
        const long long *erow = R ? a.e64 + (int64_t)i * a.t.pitch : nullptr;
        uint64_t pend = act;
        for (int base = 0; pend != 0ull; base += 64) {
            if (base >= a.t.K) {  // fewer than p open facilities
                if (lane == 0)
                    atomicOr(a.err, ERR_SCAN_OVERRUN);
                break;
            }
            const int k = base + lane;
            uint32_t j = 0;
            bool use = false;
            int32_t dist = 0;
            long long ev = 0;
            if (base == 0) {
                j = j_cur;
                use = in_row;
                if (R)
                    ev = e_cur;
                else
                    dist = d_cur;
            } else if (k < a.t.K) {
                j = prow[k];
                use = true;
                if (R)
                    ev = erow[k];
                else
                    dist = drow[k];
            }
            uint32_t jt = use ? j : jz;
            if (R && k == k_cur - 1)  // the row's last kept position
                jt = jone;
            const int hit = first_open(sT[jt], lane, tl);
            const bool found = ((pend >> lane) & 1ull) && hit >= 0;
            if (R) {
                const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_bpermute(
                    hit << 2, (int)(uint32_t)(unsigned long long)ev);
                const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_bpermute(
                    hit << 2, (int)(uint32_t)((unsigned long long)ev >> 32));
                if (found) {
                    acc += ((unsigned long long)hi << 32) | lo;
                    scn += (uint32_t)(base + hit + 1);
                }
            } else {
                const int32_t cost = __builtin_amdgcn_ds_bpermute(hit << 2, dist);
                if (found) {
                    acc += (uint32_t)cost;
                    scn += (uint32_t)(base + hit + 1);
                }
            }
            pend &= ~__builtin_amdgcn_ballot_w64(hit >= 0);  // as in walk_tail
        }
        e_cur = e_nxt;
        k_cur = k_nxt;
    }

    sred[wave * kEvalTile + lane] = acc;
    sred[NV * kEvalTile + wave * kEvalTile + lane] = scn;
    __syncthreads();
    if (wave == 0 && my_act) {
        unsigned long long f = 0, s = 0;
#pragma unroll
        for (int w = 0; w < NV; ++w) {
            f += sred[w * kEvalTile + lane];
            s += sred[NV * kEvalTile + w * kEvalTile + lane];
        }
        const int64_t o = a.pcm ? (int64_t)my_c * a.tiles_i + ti : (int64_t)ti * a.P + my_c;
        a.part[o] = f;
        if (a.spart)
            a.spart[o] = (uint32_t)s;
    }
}

}  // namespace pmp
