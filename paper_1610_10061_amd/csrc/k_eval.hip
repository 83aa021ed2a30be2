// Population evaluation: Eq. (6), computed as the Fitness function of
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
// Partial sums of the four waves are combined in LDS and added to the
// output with 64-bit atomics (integer addition, so the order is irrelevant
// and the result exact).  Workgroups are numbered so that all chromosome
// tiles of one client tile run on the same XCD and share its L2.
#include <utility>

#include "common.hpp"

namespace pmp {

namespace {

using kLanes = std::make_integer_sequence<int, kEvalTile>;

__device__ __forceinline__ int first_lane(uint64_t b)
{
    return __builtin_ffsll((long long)b) - 1;  // -1 when b == 0
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

template <int WD, int... C>
__device__ __forceinline__ int match_dense(const uint32_t *sm, uint32_t bit,
                                           std::integer_sequence<int, C...>)
{
    int hit = -1;
    (match_one<WD, C>(sm, bit, hit), ...);
    return hit;
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

template <int WD>
__global__ __launch_bounds__(kEvalTile *kEvalWaves) void k_eval(EvalArgs a)
{
    __shared__ uint32_t smask[kEvalTile * WD];
    __shared__ unsigned long long sred[2][kEvalWaves][kEvalTile];

    const int ntiles = a.tiles_c * a.tiles_i;
    const int per_xcd = (int)gridDim.x >> 3;
    const int logical = ((int)blockIdx.x & 7) * per_xcd + ((int)blockIdx.x >> 3);
    if (logical >= ntiles)
        return;
    const int ti = logical / a.tiles_c;
    const int tc = logical - ti * a.tiles_c;
    const int c0 = tc * kEvalTile;
    const int i0 = ti * a.clients_per_block;
    const int i1 = min(a.t.n, i0 + a.clients_per_block);
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int W2 = 2 * a.t.W;

    const int my_c = c0 + lane;
    const bool my_act = my_c < a.P && (a.active == nullptr || a.active[my_c]);
    const uint64_t act = __builtin_amdgcn_ballot_w64(my_act);

    // Stage the tile's masks (inactive chromosomes as zeros: they never match).
    const uint32_t *g32 = reinterpret_cast<const uint32_t *>(a.masks);
    for (int k = threadIdx.x; k < kEvalTile * WD; k += kEvalTile * kEvalWaves) {
        const int c = k / WD, w = k - (k / WD) * WD;
        uint32_t v = 0;
        if (w < W2 && ((act >> c) & 1ull))
            v = g32[(int64_t)(c0 + c) * W2 + w];
        smask[k] = v;
    }
    __syncthreads();

    // Feasibility of each chromosome, checked once (first client tile).
    if (ti == 0 && wave == 0 && my_act) {
        int ones = 0;
        uint32_t stray = 0;
        const int full = a.t.m >> 5, rem = a.t.m & 31;
        for (int w = 0; w < W2; ++w) {
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

    unsigned long long acc = 0, scn = 0;
    for (int i = i0 + wave; i < i1; i += kEvalWaves) {
        const uint16_t *prow = a.t.pi + (int64_t)i * a.t.pitch;
        const int32_t *drow = a.t.ds + (int64_t)i * a.t.pitch;
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
            if (k < a.t.K) {
                const uint32_t j = prow[k];
                off = j >> 5;
                bit = 1u << (j & 31u);
                dist = drow[k];
            }
            const uint32_t *sm = smask + off;
            const int hit = (base == 0 || __builtin_popcountll(pend) >= 16)
                                ? match_dense<WD>(sm, bit, kLanes{})
                                : match_sparse<WD>(sm, bit, pend, lane);
            const bool found = ((pend >> lane) & 1ull) && hit >= 0;
            const int32_t cost = __builtin_amdgcn_ds_bpermute((hit & 63) << 2, dist);
            if (found) {
                acc += (uint32_t)cost;
                scn += (unsigned long long)(base + hit + 1);
            }
            pend &= ~__builtin_amdgcn_ballot_w64(found);
        }
    }

    sred[0][wave][lane] = acc;
    sred[1][wave][lane] = scn;
    __syncthreads();
    if (wave == 0) {
        unsigned long long f = 0, s = 0;
#pragma unroll
        for (int w = 0; w < kEvalWaves; ++w) {
            f += sred[0][w][lane];
            s += sred[1][w][lane];
        }
        if (my_act) {
            atomicAdd(a.fitness + my_c, f);
            if (a.scan)
                atomicAdd(a.scan + my_c, s);
        }
        if (a.gstate) {
            unsigned long long t = s;
#pragma unroll
            for (int d = 32; d > 0; d >>= 1)
                t += __shfl_xor(t, d);
            if (lane == 0) {
                atomicAdd(a.gstate + GS_SCAN_TOTAL, t);
                if (ti == 0)
                    atomicAdd(a.gstate + GS_CHROM_EVALS,
                              (unsigned long long)__builtin_popcountll(act));
            }
        }
    }
}

template <int WD>
hipError_t launch_wd(const EvalArgs &a, hipStream_t s)
{
    const int tiles = a.tiles_c * a.tiles_i;
    const int grid = ((tiles + 7) / 8) * 8;
    hipLaunchKernelGGL(k_eval<WD>, dim3(grid), dim3(kEvalTile * kEvalWaves), 0,
                       s, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_eval(const EvalArgs &a, hipStream_t s)
{
    if (a.P <= 0 || a.tiles_c <= 0 || a.tiles_i <= 0)
        return hipSuccess;
    const int w2 = 2 * a.t.W;
    if (w2 <= 2) return launch_wd<2>(a, s);
    if (w2 <= 4) return launch_wd<4>(a, s);
    if (w2 <= 8) return launch_wd<8>(a, s);
    if (w2 <= 16) return launch_wd<16>(a, s);
    if (w2 <= 32) return launch_wd<32>(a, s);
    if (w2 <= 48) return launch_wd<48>(a, s);
    if (w2 <= 64) return launch_wd<64>(a, s);
    if (w2 <= 96) return launch_wd<96>(a, s);
    if (w2 <= 128) return launch_wd<128>(a, s);
    if (w2 <= 160) return launch_wd<160>(a, s);
    if (w2 <= 192) return launch_wd<192>(a, s);
    if (w2 <= 256) return launch_wd<256>(a, s);
    return hipErrorInvalidValue;
}

}  // namespace pmp
