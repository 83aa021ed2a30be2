// Population evaluation, device side: Eq. (6), computed as the Fitness function of
// Section 4.2 does it, for a whole population at once.
//
// For chromosome c and client i the walk reads Pi'_i from the front until it
// meets an open facility, at 1-based position s*; the client then costs
// D'_{i,s*} (the sum of the first s* gap terms).  fitness[c] is the sum over
// clients, exact in 64-bit integers.
//
// Mapping (gfx950, wave64).  A workgroup owns a tile of 64 chromosomes (one
// per lane, their masks staged in LDS) and a tile of clients; each of its
// four waves takes every fourth client of the tile.  For one client the wave
// loads 64 consecutive entries of Pi'_i and D'_i, one per lane (coalesced),
// and then, for each chromosome of the tile, every lane tests "is the
// facility at my position open in chromosome c" with one LDS read of the
// word holding that facility's bit.  A ballot gives the 64 answers; its
// lowest set bit is the chromosome's first open position in this chunk.
// That position is written into lane c of a register, and one ds_bpermute
// then fetches each chromosome's D' entry from the lane that holds it, so a
// (chromosome, client) pair costs one LDS read and three VALU operations
// whatever its scan length up to 64.  Chromosomes still unmatched go on to
// the next 64 entries.  This replaces the paper's one-thread-per-chromosome
// loop: lanes never diverge and Pi' rows are read once per 64 chromosomes.
//
// Partial sums of the four waves are combined in LDS and stored, one int64
// per (client tile, chromosome), with plain stores; the consumer (the
// reduction below or the GA's next stage) adds the client tiles up.  Integer
// addition makes the result exact and independent of tiling.  Workgroups
// are numbered so that all chromosome tiles of one client tile run on the
// same XCD and share its L2, and each wave loads the next client's chunk of
// Pi' and D' before it works on the current one.
#pragma once

#include <utility>

#include "common.hpp"

namespace pmp {

using kLanes = std::make_integer_sequence<int, kEvalTile>;
using kQuads = std::make_integer_sequence<int, kEvalTile / 4>;

// Lowest set lane of a ballot, -1 when none (s_ff1_i32_b64 returns -1 for
// zero, so no compare and select are needed around it).
__device__ __forceinline__ int first_lane(uint64_t b)
{
    int r;
    asm("s_ff1_i32_b64 %0, %1" : "=s"(r) : "s"(b));
    return r;
}

// Lane C of `hit` takes the wave-uniform value `v` (v_writelane_b32 with the
// lane as an inline constant).
template <int C>
__device__ __forceinline__ void write_lane(int &hit, int v)
{
    asm("v_writelane_b32 %0, %1, %2" : "+v"(hit) : "s"(v), "n"(C));
}

// All 64 chromosomes of the tile against one 64-entry chunk of a Pi' row.
template <int WD, int C>
__device__ __forceinline__ void match_one(const uint32_t *sm, uint32_t bit,
                                          int &hit)
{
    const uint32_t w = sm[C * WD];
    const uint64_t b = __builtin_amdgcn_ballot_w64((w & bit) != 0u);
    write_lane<C>(hit, first_lane(b));
}

// Chromosomes 4Q .. 4Q+3 together: four ballots live in four SGPR pairs and
// one asm block takes their four lowest lanes, so the compare, find-first
// and write-lane steps of neighbouring chromosomes overlap instead of
// waiting on one shared scalar register.  Chromosome C goes to register
// C mod 4.
template <int WD, int Q>
__device__ __forceinline__ void match_quad(const uint32_t *sm, uint32_t bit, int &h0,
                                           int &h1, int &h2, int &h3)
{
    constexpr int C = 4 * Q;
    const uint32_t w0 = sm[C * WD], w1 = sm[(C + 1) * WD];
    const uint32_t w2 = sm[(C + 2) * WD], w3 = sm[(C + 3) * WD];
    const uint64_t b0 = __builtin_amdgcn_ballot_w64((w0 & bit) != 0u);
    const uint64_t b1 = __builtin_amdgcn_ballot_w64((w1 & bit) != 0u);
    const uint64_t b2 = __builtin_amdgcn_ballot_w64((w2 & bit) != 0u);
    const uint64_t b3 = __builtin_amdgcn_ballot_w64((w3 & bit) != 0u);
    int f0, f1, f2, f3;
    asm("s_ff1_i32_b64 %0, %4\n\t"
        "s_ff1_i32_b64 %1, %5\n\t"
        "s_ff1_i32_b64 %2, %6\n\t"
        "s_ff1_i32_b64 %3, %7"
        : "=&s"(f0), "=&s"(f1), "=&s"(f2), "=&s"(f3)
        : "s"(b0), "s"(b1), "s"(b2), "s"(b3));
    write_lane<C>(h0, f0);
    write_lane<C + 1>(h1, f1);
    write_lane<C + 2>(h2, f2);
    write_lane<C + 3>(h3, f3);
}

// Every chromosome of the tile (kEvalTile = 64) against one chunk.
template <int WD, int... Q>
__device__ __forceinline__ int match_dense(const uint32_t *sm, uint32_t bit,
                                           int lane,
                                           std::integer_sequence<int, Q...>)
{
    int h0 = -1, h1 = -1, h2 = -1, h3 = -1;
    (match_quad<WD, Q>(sm, bit, h0, h1, h2, h3), ...);
    const int q = lane & 3;
    return q == 0 ? h0 : q == 1 ? h1 : q == 2 ? h2 : h3;
}

// Two clients per chunk (short scans): lanes 0-31 hold the first 32 entries
// of client A's row, lanes 32-63 those of client B.  One compare per
// chromosome serves both rows; the ballot's low and high halves give each
// client's first open position.
template <int WD, int Q>
__device__ __forceinline__ void match_quad2(const uint32_t *sm, uint32_t bit, int (&ha)[4],
                                            int (&hb)[4])
{
    constexpr int C = 4 * Q;
    const uint32_t w0 = sm[C * WD], w1 = sm[(C + 1) * WD];
    const uint32_t w2 = sm[(C + 2) * WD], w3 = sm[(C + 3) * WD];
    const uint64_t b0 = __builtin_amdgcn_ballot_w64((w0 & bit) != 0u);
    const uint64_t b1 = __builtin_amdgcn_ballot_w64((w1 & bit) != 0u);
    const uint64_t b2 = __builtin_amdgcn_ballot_w64((w2 & bit) != 0u);
    const uint64_t b3 = __builtin_amdgcn_ballot_w64((w3 & bit) != 0u);
    int a0, a1, a2, a3, e0, e1, e2, e3;
    asm("s_ff1_i32_b32 %0, %8\n\t"
        "s_ff1_i32_b32 %1, %9\n\t"
        "s_ff1_i32_b32 %2, %10\n\t"
        "s_ff1_i32_b32 %3, %11\n\t"
        "s_ff1_i32_b32 %4, %12\n\t"
        "s_ff1_i32_b32 %5, %13\n\t"
        "s_ff1_i32_b32 %6, %14\n\t"
        "s_ff1_i32_b32 %7, %15"
        : "=&s"(a0), "=&s"(a1), "=&s"(a2), "=&s"(a3), "=&s"(e0), "=&s"(e1), "=&s"(e2),
          "=&s"(e3)
        : "s"((uint32_t)b0), "s"((uint32_t)b1), "s"((uint32_t)b2), "s"((uint32_t)b3),
          "s"((uint32_t)(b0 >> 32)), "s"((uint32_t)(b1 >> 32)), "s"((uint32_t)(b2 >> 32)),
          "s"((uint32_t)(b3 >> 32)));
    write_lane<C>(ha[0], a0);
    write_lane<C + 1>(ha[1], a1);
    write_lane<C + 2>(ha[2], a2);
    write_lane<C + 3>(ha[3], a3);
    write_lane<C>(hb[0], e0);
    write_lane<C + 1>(hb[1], e1);
    write_lane<C + 2>(hb[2], e2);
    write_lane<C + 3>(hb[3], e3);
}

template <int WD, int... Q>
__device__ __forceinline__ void match_dense2(const uint32_t *sm, uint32_t bit, int lane,
                                             int &hit_a, int &hit_b,
                                             std::integer_sequence<int, Q...>)
{
    int ha[4] = {-1, -1, -1, -1}, hb[4] = {-1, -1, -1, -1};
    (match_quad2<WD, Q>(sm, bit, ha, hb), ...);
    const int q = lane & 3;
    hit_a = q == 0 ? ha[0] : q == 1 ? ha[1] : q == 2 ? ha[2] : ha[3];
    hit_b = q == 0 ? hb[0] : q == 1 ? hb[1] : q == 2 ? hb[2] : hb[3];
}

// Only the chromosomes in q (few left after the first chunk).
template <int WD>
__device__ __forceinline__ int match_sparse(const uint32_t *sm, uint32_t bit,
                                            uint64_t q, int lane)
{
    int hit = -1;
    while (q) {
        const int c = __builtin_ctzll(q);
        q &= q - 1;
        const uint32_t w = sm[c * WD];
        const uint64_t b = __builtin_amdgcn_ballot_w64((w & bit) != 0u);
        const int v = first_lane(b);
        hit = lane == c ? v : hit;
    }
    return hit;
}

// The rest of one client's walk from position `base` for the chromosomes in
// `pend` (64-entry chunks, loaded here).
template <int WD>
__device__ __forceinline__ void walk_tail(const EvalArgs &a, const uint16_t *prow,
                                          const int32_t *drow, int base, uint64_t pend,
                                          int lane, const uint32_t *smask,
                                          unsigned long long &acc, uint32_t &scn)
{
    for (; pend != 0ull; base += 64) {
        if (base >= a.t.K) {  // fewer than p open facilities
            if (lane == 0)
                atomicOr(a.err, ERR_SCAN_OVERRUN);
            break;
        }
        const int k = base + lane;
        uint32_t off = 0, bit = 0;
        int32_t dist = 0;
        if (k < a.t.K) {
            const uint32_t j = prow[k];
            off = j >> 5;
            bit = 1u << (j & 31u);
            dist = drow[k];
        }
        const uint32_t *sm = smask + off;
        const int hit = __builtin_popcountll(pend) >= 16
                            ? match_dense<WD>(sm, bit, lane, kQuads{})
                            : match_sparse<WD>(sm, bit, pend, lane);
        const bool found = ((pend >> lane) & 1ull) && hit >= 0;
        const int32_t cost = __builtin_amdgcn_ds_bpermute((hit & 63) << 2, dist);
        if (found) {
            acc += (uint32_t)cost;
            scn += (uint32_t)(base + hit + 1);
        }
        pend &= ~__builtin_amdgcn_ballot_w64(found);
    }
}

// Evaluate chromosome tile tc (64 chromosomes) on client tile ti and store
// the tile's partial sums.  Called by a whole 256-thread workgroup;
// smask holds 64 * WD words, sred 2 * kEvalWaves * 64 words.
//
// R: the walk tables of the reduced polynomial (k_hbp.hip) instead of the
// instance's: row i stops at position K_i - 1 at the latest (a.rlen) and
// the value read there is the int64 running sum a.e64.  The stop is made
// with no extra work in the walk: the last position's lane tests a mask
// word that is all ones for every chromosome (word 2W of each staged row,
// so WD > 2W).
//
// H (short scans, not with R): a wave walks its clients two at a time, the
// first 32 entries of each row in one chunk (match_dense2); the few rows
// whose first open facility lies past entry 31 finish in walk_tail.
template <int WD, bool R = false, bool H = false>
__device__ __forceinline__ void eval_tile(const EvalArgs &a, int ti, int tc,
                                          uint32_t *smask,
                                          unsigned long long *sred)
{
    const int c0 = tc * kEvalTile;
    const int i0 = ti * a.clients_per_block;
    const int i1 = min(a.t.n, i0 + a.clients_per_block);
    const int lane = threadIdx.x & 63;
    const int wave = wave_id();
    const int W2 = 2 * a.t.W;

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
    const int row_first = (H && lane >= 32) ? min(i + kEvalWaves, last) : min(i, last);
    const uint32_t j_first = a.t.pi[(int64_t)row_first * a.t.pitch + col];
    int32_t d_cur = 0;
    long long e_cur = 0;
    int k_cur = 0;  // R: the row's length K_i
    if (R) {
        e_cur = a.e64[(int64_t)min(i, last) * a.t.pitch + col];
        k_cur = a.rlen[min(i, last)];
    } else {
        d_cur = a.t.ds[(int64_t)row_first * a.t.pitch + col];
    }
    // Masks: every load unconditional at a clamped (always valid) address,
    // in batches, so that a batch costs one round trip; out-of-range words
    // are replaced by 0 when stored.
    const uint32_t *g32 = reinterpret_cast<const uint32_t *>(a.masks);
    const int rows = min(kEvalTile, a.P - c0);
    constexpr int kTot = kEvalTile * WD, kThreads = kEvalTile * kEvalWaves;
    constexpr int kIt = (kTot + kThreads - 1) / kThreads;
    constexpr int kBatch = kIt < 16 ? kIt : 16;
    // active flag: also an unconditional load (of any valid byte when every
    // chromosome is active)
    const uint8_t *ap = a.active ? a.active + min(my_c, a.P - 1) : (const uint8_t *)a.masks;
    const uint8_t actv = *ap;
#pragma unroll
    for (int r0 = 0; r0 < kIt; r0 += kBatch) {
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
                smask[k] = (w < W2 && c < rows) ? v[r] : ((R && w == W2) ? ~0u : 0u);
        }
    }
    const bool my_act = my_c < a.P && (a.active == nullptr || actv != 0);
    const uint64_t act = __builtin_amdgcn_ballot_w64(my_act);
    // nothing to do (same in every wave: the whole workgroup leaves), or a
    // stopped GA run, whose later generations are no-ops
    if (act == 0ull || (a.done && *a.done))
        return;
    __syncthreads();

    // Feasibility of each chromosome, checked once (first client tile).
    // Lanes start at different words so the reads hit different banks.
    if (ti == 0 && wave == 0 && my_act) {
        int ones = 0;
        uint32_t stray = 0;
        const int full = a.t.m >> 5, rem = a.t.m & 31;
        for (int k = 0; k < W2; ++k) {
            int w = lane + k;
            w = w >= W2 ? w - W2 * (w / W2) : w;
            const uint32_t v = smask[lane * WD + w];
            ones += __builtin_popcount(v);
            if (w > full || (w == full && rem == 0))
                stray |= v;
            else if (w == full)
                stray |= v & ~((1u << rem) - 1u);
        }
        if (ones != a.t.p)
            atomicOr(a.err, ERR_POPCOUNT);
        if (stray)
            atomicOr(a.err, ERR_STRAY_BITS);
    }

    unsigned long long acc = 0;
    uint32_t scn = 0;
    // chunk-0 operands of the current client: mask word, bit (0 past K)
    uint32_t off_cur = j_first >> 5;
    uint32_t bit_cur = in_row ? 1u << (j_first & 31u) : 0u;
    if constexpr (H) {
        for (; i < i1; i += 2 * kEvalWaves) {
            const int ib = i + kEvalWaves;
            const bool has_b = ib < i1;
            const int na = min(i + 2 * kEvalWaves, last), nb = min(i + 3 * kEvalWaves, last);
            const int rown = lane >= 32 ? nb : na;
            const uint32_t j_nxt = a.t.pi[(int64_t)rown * a.t.pitch + col];
            const int32_t d_nxt = a.t.ds[(int64_t)rown * a.t.pitch + col];
            const uint32_t bit = (lane >= 32 && !has_b) ? 0u : bit_cur;
            int ha, hb;
            match_dense2<WD>(smask + off_cur, bit, lane, ha, hb, kQuads{});
            const uint64_t pa = act, pb = has_b ? act : 0ull;
            const bool fa = ((pa >> lane) & 1ull) && ha >= 0;
            const bool fb = ((pb >> lane) & 1ull) && hb >= 0;
            const int32_t ca = __builtin_amdgcn_ds_bpermute((ha & 31) << 2, d_cur);
            const int32_t cb = __builtin_amdgcn_ds_bpermute((32 + (hb & 31)) << 2, d_cur);
            if (fa) {
                acc += (uint32_t)ca;
                scn += (uint32_t)(ha + 1);
            }
            if (fb) {
                acc += (uint32_t)cb;
                scn += (uint32_t)(hb + 1);
            }
            const uint64_t ra = pa & ~__builtin_amdgcn_ballot_w64(fa);
            const uint64_t rb = pb & ~__builtin_amdgcn_ballot_w64(fb);
            if (ra)
                walk_tail<WD>(a, a.t.pi + (int64_t)i * a.t.pitch, a.t.ds + (int64_t)i * a.t.pitch,
                              32, ra, lane, smask, acc, scn);
            if (rb)
                walk_tail<WD>(a, a.t.pi + (int64_t)ib * a.t.pitch,
                              a.t.ds + (int64_t)ib * a.t.pitch, 32, rb, lane, smask, acc, scn);
            off_cur = j_nxt >> 5;
            bit_cur = in_row ? 1u << (j_nxt & 31u) : 0u;
            d_cur = d_nxt;
        }
    }
    for (; !H && i < i1; i += kEvalWaves) {
        const int inext = min(i + kEvalWaves, last);
        const uint32_t j_nxt = a.t.pi[(int64_t)inext * a.t.pitch + col];
        int32_t d_nxt = 0;
        long long e_nxt = 0;
        int k_nxt = 0;
        if (R) {
            e_nxt = a.e64[(int64_t)inext * a.t.pitch + col];
            k_nxt = a.rlen[inext];
        } else {
            d_nxt = a.t.ds[(int64_t)inext * a.t.pitch + col];
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
            uint32_t off = 0, bit = 0;
            int32_t dist = 0;
            long long ev = 0;
            if (base == 0) {
                off = off_cur;
                bit = bit_cur;
                if (R)
                    ev = e_cur;
                else
                    dist = d_cur;
            } else if (k < a.t.K) {
                const uint32_t j = prow[k];
                off = j >> 5;
                bit = 1u << (j & 31u);
                if (R)
                    ev = erow[k];
                else
                    dist = drow[k];
            }
            if (R && k == k_cur - 1) {  // the row's last kept position
                off = (uint32_t)W2;
                bit = 1u;
            }
            const uint32_t *sm = smask + off;
            const int hit = (base == 0 || __builtin_popcountll(pend) >= 16)
                                ? match_dense<WD>(sm, bit, lane, kQuads{})
                                : match_sparse<WD>(sm, bit, pend, lane);
            const bool found = ((pend >> lane) & 1ull) && hit >= 0;
            if (R) {
                const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_bpermute(
                    (hit & 63) << 2, (int)(uint32_t)(unsigned long long)ev);
                const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_bpermute(
                    (hit & 63) << 2, (int)(uint32_t)((unsigned long long)ev >> 32));
                if (found) {
                    acc += ((unsigned long long)hi << 32) | lo;
                    scn += (uint32_t)(base + hit + 1);
                }
            } else {
                const int32_t cost = __builtin_amdgcn_ds_bpermute((hit & 63) << 2, dist);
                if (found) {
                    acc += (uint32_t)cost;
                    scn += (uint32_t)(base + hit + 1);
                }
            }
            pend &= ~__builtin_amdgcn_ballot_w64(found);
        }
        // the next client's operands, computed here so that the wait for
        // its loads falls after this client's work
        off_cur = j_nxt >> 5;
        bit_cur = in_row ? 1u << (j_nxt & 31u) : 0u;
        d_cur = d_nxt;
        e_cur = e_nxt;
        k_cur = k_nxt;
    }

    sred[wave * kEvalTile + lane] = acc;
    sred[kEvalWaves * kEvalTile + wave * kEvalTile + lane] = scn;
    __syncthreads();
    if (wave == 0 && my_act) {
        unsigned long long f = 0, s = 0;
#pragma unroll
        for (int w = 0; w < kEvalWaves; ++w) {
            f += sred[w * kEvalTile + lane];
            s += sred[kEvalWaves * kEvalTile + w * kEvalTile + lane];
        }
        const int64_t o = (int64_t)ti * a.P + my_c;
        a.part[o] = f;
        if (a.spart)
            a.spart[o] = (uint32_t)s;
    }
}

}  // namespace pmp
