// The reduced Hammer-Beresnev polynomial on the device (Section 2.1, after
// Eq. (6), and Example 1).  Term t >= 1 of client i has coefficient
// Delta'_{i,t} and the monomial "the first t facilities of row i are all
// closed"; rows whose first t facilities form the same set give the same
// monomial, and the reduced polynomial adds their coefficients (zero terms
// add nothing and a set with only zero terms disappears).  The constant is
// the sum of the rows' first terms.
//
// Construction:
//  1. every positive term (i, t) gets a 64-bit key, a hash of the set (a sum
//     of per-facility hashes, so the order inside the prefix does not
//     matter) mixed with t;
//  2. an open-addressing table merges equal keys: coefficient sum, lowest
//     row (the set's owner) and lowest/highest degree;
//  3. every non-owner term checks, exactly, that its set equals its owner's
//     (each of its t facilities sits within the owner row's first t
//     positions), so a hash collision is reported, never merged;
//  4. row i keeps positions 0 .. K_i - 1, K_i - 1 being the highest degree
//     it owns, with E_i[f] = the sum of its owned coefficients of degree
//     <= f; a client then costs E_i[min(first open, K_i - 1)];
//  5. kept rows are compacted (padded to a common pitch for the evaluation
//     kernel) and the owned terms are listed row by row.
#include "common.hpp"

namespace pmp {

namespace {

__device__ __forceinline__ uint64_t mix64(uint64_t x)
{
    // SplitMix64 finaliser (Steele, Lea & Flood, OOPSLA 2014)
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

__device__ __forceinline__ uint64_t term_key(uint64_t set_hash, int t)
{
    const uint64_t k = mix64(set_hash ^ ((uint64_t)t << 48) ^ (uint64_t)t);
    return k ? k : 1ull;  // 0 marks an empty slot
}

__device__ __forceinline__ uint64_t wave_scan_u64(uint64_t v, int lane)
{
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint64_t u = __shfl_up(v, d);
        if (lane >= d)
            v += u;
    }
    return v;
}

// One wave per row: prefix-set keys of the positive terms (key[i][t], 0 for
// zero terms and t = 0) and the count of positive terms into *npos.
__global__ __launch_bounds__(256) void k_hbp_keys(HbpArgs h)
{
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + wave_id();
    if (i >= h.t.n)
        return;
    const uint16_t *prow = h.t.pi + (int64_t)i * h.t.pitch;
    const int32_t *drow = h.t.ds + (int64_t)i * h.t.pitch;
    uint64_t carry = 0;
    unsigned cnt = 0;
    for (int base = 0; base < h.t.K; base += 64) {
        const int t = base + lane;  // term t covers positions 0 .. t-1
        const bool in = t < h.t.K;
        // hash of the facility at position t - 1 (none for t = 0)
        uint64_t x = 0;
        if (in && t >= 1)
            x = mix64((uint64_t)prow[t - 1] * 0x2545F4914F6CDD1Dull + 0x6A09E667F3BCC909ull);
        const uint64_t pre = carry + wave_scan_u64(x, lane);
        carry = __shfl(pre, 63);
        int32_t gap = 0;
        if (in && t >= 1)
            gap = drow[t] - drow[t - 1];
        const bool pos = in && t >= 1 && gap > 0;
        if (in)
            h.key[(int64_t)i * h.t.pitch + t] = pos ? term_key(pre, t) : 0ull;
        cnt += pos ? 1u : 0u;
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1)
        cnt += __shfl_xor(cnt, d);
    if (lane == 0 && cnt)
        atomicAdd(h.npos, (unsigned long long)cnt);
}

// Position of each facility within each row's first K (0xFFFF past K).
__global__ __launch_bounds__(256) void k_hbp_posinv(HbpArgs h)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)h.t.n * h.t.K)
        return;
    const int i = (int)(e / h.t.K), k = (int)(e - (int64_t)i * h.t.K);
    h.posinv[(int64_t)i * h.t.m + h.t.pi[(int64_t)i * h.t.pitch + k]] = (uint16_t)k;
}

// Thread per term: merge into the table (linear probing; the table holds at
// least twice the positive terms, so a free slot is always found).
__global__ __launch_bounds__(256) void k_hbp_insert(HbpArgs h)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)h.t.n * h.t.K)
        return;
    const int i = (int)(e / h.t.K), t = (int)(e - (int64_t)i * h.t.K);
    const int64_t o = (int64_t)i * h.t.pitch + t;
    const uint64_t k = h.key[o];
    if (k == 0ull)
        return;
    const int32_t gap = h.t.ds[o] - h.t.ds[o - 1];
    uint64_t s = k & h.mask;
    for (uint64_t probe = 0; probe <= h.mask; ++probe) {
        const unsigned long long prev =
            atomicCAS((unsigned long long *)&h.slot_key[s], 0ull, (unsigned long long)k);
        if (prev == 0ull || prev == k) {
            atomicMin(&h.slot_row[s], i);
            atomicMin(&h.slot_tmin[s], t);
            atomicMax(&h.slot_tmax[s], t);
            atomicAdd(&h.slot_sum[s], (unsigned long long)gap);
            h.slot_of[o] = (int32_t)s;
            return;
        }
        s = (s + 1) & h.mask;
    }
    atomicOr(h.err, ERR_HASH_TABLE);
}

// Thread per term: ownership, and the exact check of merged sets.
__global__ __launch_bounds__(256) void k_hbp_own(HbpArgs h)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)h.t.n * h.t.K)
        return;
    const int i = (int)(e / h.t.K), t = (int)(e - (int64_t)i * h.t.K);
    const int64_t o = (int64_t)i * h.t.pitch + t;
    long long charged = 0;
    if (h.key[o] != 0ull) {
        const int s = h.slot_of[o];
        const int r = h.slot_row[s];
        if (h.slot_tmin[s] != h.slot_tmax[s])
            atomicOr(h.err, ERR_HASH_COLLISION);
        if (r == i) {
            charged = (long long)h.slot_sum[s];
        } else {
            const uint16_t *prow = h.t.pi + (int64_t)i * h.t.pitch;
            const uint16_t *inv = h.posinv + (int64_t)r * h.t.m;
            bool same = true;
            for (int x = 0; x < t; ++x)
                same = same && inv[prow[x]] < t;
            if (!same)
                atomicOr(h.err, ERR_HASH_COLLISION);
        }
    }
    h.charged[o] = charged;
}

// One wave per row: K_i, the running sums E_i, the owned-term count, the
// largest K_i.
__global__ __launch_bounds__(256) void k_hbp_rows(HbpArgs h)
{
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + wave_id();
    if (i >= h.t.n)
        return;
    const long long *crow = h.charged + (int64_t)i * h.t.pitch;
    long long carry = 0;
    int last = -1, owned = 0;
    for (int base = 0; base < h.t.K; base += 64) {
        const int t = base + lane;
        const long long c = t < h.t.K ? crow[t] : 0ll;
        const long long pre = carry + (long long)wave_scan_u64((uint64_t)c, lane);
        carry = __shfl(pre, 63);
        if (t < h.t.K)
            h.esum[(int64_t)i * h.t.pitch + t] = pre;
        if (c != 0) {
            last = t;
            ++owned;
        }
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        last = max(last, __shfl_xor(last, d));
        owned += __shfl_xor(owned, d);
    }
    if (lane == 0) {
        const int Ki = last + 1;
        h.rlen_full[i] = Ki;
        h.owned[i] = owned;
        if (Ki > 0)
            atomicMax(h.maxlen, Ki);
        atomicAdd(h.c0, (unsigned long long)h.t.ds[(int64_t)i * h.t.pitch]);
    }
}

// One workgroup: exclusive scans over rows of "kept" (K_i > 0) and of the
// owned-term counts; totals into tot[0], tot[1].
__global__ __launch_bounds__(1024) void k_hbp_scan(HbpArgs h)
{
    __shared__ int sk[1024], so[1024];
    const int n = h.t.n, per = (n + 1023) / 1024;
    const int r0 = min(n, (int)threadIdx.x * per), r1 = min(n, r0 + per);
    int kk = 0, oo = 0;
    for (int r = r0; r < r1; ++r) {
        kk += h.rlen_full[r] > 0 ? 1 : 0;
        oo += h.owned[r];
    }
    sk[threadIdx.x] = kk;
    so[threadIdx.x] = oo;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const int a = threadIdx.x >= (unsigned)d ? sk[threadIdx.x - d] : 0;
        const int b = threadIdx.x >= (unsigned)d ? so[threadIdx.x - d] : 0;
        __syncthreads();
        sk[threadIdx.x] += a;
        so[threadIdx.x] += b;
        __syncthreads();
    }
    int ek = sk[threadIdx.x] - kk, eo = so[threadIdx.x] - oo;
    for (int r = r0; r < r1; ++r) {
        h.kept_at[r] = h.rlen_full[r] > 0 ? ek : -1;
        h.term_at[r] = eo;
        ek += h.rlen_full[r] > 0 ? 1 : 0;
        eo += h.owned[r];
    }
    if (threadIdx.x == 1023) {
        h.tot[0] = sk[1023];
        h.tot[1] = so[1023];
    }
}

// One wave per row: the compacted walk tables (padded past K_i with the
// last kept entry) and the row's owned terms.
__global__ __launch_bounds__(256) void k_hbp_emit(HbpArgs h)
{
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + wave_id();
    if (i >= h.t.n)
        return;
    const int Ki = h.rlen_full[i], r = h.kept_at[i];
    const uint16_t *prow = h.t.pi + (int64_t)i * h.t.pitch;
    const long long *erow = h.esum + (int64_t)i * h.t.pitch;
    const long long *crow = h.charged + (int64_t)i * h.t.pitch;
    if (r >= 0) {
        for (int f = lane; f < h.rpitch; f += 64) {
            const int src = min(f, Ki - 1);
            h.rpi[(int64_t)r * h.rpitch + f] = prow[src];
            h.re[(int64_t)r * h.rpitch + f] = erow[src];
        }
        if (lane == 0)
            h.rlen[r] = Ki;
    }
    int at = h.term_at[i];
    for (int base = 0; base < Ki; base += 64) {
        const int t = base + lane;
        const long long c = t < Ki ? crow[t] : 0ll;
        const uint64_t b = __builtin_amdgcn_ballot_w64(c != 0);
        if (c != 0) {
            const int o = at + __builtin_popcountll(b & ((1ull << lane) - 1ull));
            h.term_row[o] = i;
            h.term_deg[o] = t;
            h.term_coef[o] = c;
        }
        at += __builtin_popcountll(b);
    }
}

inline dim3 grid_of(int64_t items, int per)
{
    return dim3((unsigned)((items + per - 1) / per));
}

}  // namespace

hipError_t launch_hbp_keys(const HbpArgs &h, hipStream_t s)
{
    hipLaunchKernelGGL(k_hbp_keys, grid_of(h.t.n, 4), dim3(256), 0, s, h);
    return hipGetLastError();
}

hipError_t launch_hbp_table(const HbpArgs &h, hipStream_t s)
{
    const int64_t cells = (int64_t)h.t.n * h.t.K;
    hipLaunchKernelGGL(k_hbp_posinv, grid_of(cells, 256), dim3(256), 0, s, h);
    hipLaunchKernelGGL(k_hbp_insert, grid_of(cells, 256), dim3(256), 0, s, h);
    hipLaunchKernelGGL(k_hbp_own, grid_of(cells, 256), dim3(256), 0, s, h);
    hipLaunchKernelGGL(k_hbp_rows, grid_of(h.t.n, 4), dim3(256), 0, s, h);
    hipLaunchKernelGGL(k_hbp_scan, dim3(1), dim3(1024), 0, s, h);
    return hipGetLastError();
}

hipError_t launch_hbp_emit(const HbpArgs &h, hipStream_t s)
{
    hipLaunchKernelGGL(k_hbp_emit, grid_of(h.t.n, 4), dim3(256), 0, s, h);
    return hipGetLastError();
}

}  // namespace pmp
