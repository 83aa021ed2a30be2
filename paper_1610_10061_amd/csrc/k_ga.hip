// Genetic-algorithm kernels.  Two launch schemes run the same device code
// (ga_device.hpp, eval_device.hpp):
//
//  - one kernel per step: k_init, the evaluation kernel, k_stage for each
//    stage, k_best; ordered by the stream.
//  - k_ga_batch: one persistent launch runs whole generations of one or
//    many instances; its phases are separated by grid barriers.  It pays
//    off when a phase holds much work (a batch of instances); for a single
//    small instance the per-step kernels are faster, because every barrier
//    costs each workgroup an L2 write-back and invalidate.
#include <hip/hip_ext.h>
#include "eval_device.hpp"
#include "ga_device.hpp"

namespace pmp {

namespace {

// Two waves per chromosome: the population slot, and the operator draws.
__global__ __launch_bounds__(64 * kGaWaves) void k_init(GaArgs g)
{
    __shared__ uint64_t sw[kGaWaves][2 * kMaxWords];
    const int wave = wave_id(), lane = threadIdx.x & 63;
    const int gw = blockIdx.x * kGaWaves + wave;
    const int c = gw >> 1;
    if (c >= g.P || ga_stopped(g))
        return;
    ga_init_one(g, c, lane, sw[wave], gw & 1);
}

__global__ __launch_bounds__(64 * kGaWaves) void k_stage(GaArgs g, int in,
                                                         int prev, int op,
                                                         int index)
{
    const int wave = wave_id(), lane = threadIdx.x & 63;
    const int gw = blockIdx.x * kGaWaves + wave;
    // the whole mutation cycle at once: ceil(Y / mpw) waves per chromosome
    const int per = op == OP_MUT_ALL ? (g.Y + g.mpw - 1) / g.mpw : 1;
    const int c = gw / per, sub = gw - c * per;
    if (c >= g.P)
        return;
    ga_stage_one(g, c, lane, in, prev, op, index, sub);  // checks the stop flag itself
}

// ---------------------------------------------------------------------------
// A crossover stage fused with the evaluation of its offspring (chromosomes
// of at most 16 words).  The workgroup of chromosome tile tc and client tile
// ti first runs the stage step for the tile's 64 chromosomes: each of its 16
// waves takes 4 chromosomes, a row of 16 lanes per chromosome and a word per
// lane.  A row adds up the previous evaluation's partial sums, takes the
// offspring if strictly fitter (for the chromosome and its partner), and
// runs the crossover of Section 4.3 on its words: row prefix sums of the
// qualifying genes per word (A = 1, B = 0 and A = 0, B = 1), rearranged into
// the cyclic walk order from r1, tell each lane how many genes of each kind
// come before its word, hence which of its own to take.  The new offspring
// goes straight into the evaluation's staging rows, and the tile is then
// evaluated on the workgroup's clients.  Every client tile's workgroup
// computes the same offspring from the same inputs (what the previous
// launch left); only client tile 0's writes the run's state (population,
// fitness, offspring, flags, counters).  The partial sums it reads and the
// ones it writes are different buffers (launches alternate them).
// ---------------------------------------------------------------------------
constexpr int kFusedWaves = 16;
constexpr int kFusedMaxW = 16;

// Inclusive prefix sums within each 16-lane row (DPP row shifts; lanes
// without a source add 0).
__device__ __forceinline__ uint32_t row_scan_incl(uint32_t v)
{
    v += dpp_from<0x111, 0xF>(v);  // row_shr:1
    v += dpp_from<0x112, 0xF>(v);  // row_shr:2
    v += dpp_from<0x114, 0xF>(v);  // row_shr:4
    v += dpp_from<0x118, 0xF>(v);  // row_shr:8
    return v;
}

// Sum over the 16 lanes of each row (xor butterflies stay inside a row).
__device__ __forceinline__ unsigned long long row_sum(unsigned long long v)
{
    v += __shfl_xor(v, 8);
    v += __shfl_xor(v, 4);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 1);
    return v;
}

template <int WD, bool H>
__global__ __launch_bounds__(kEvalTile *kFusedWaves) void k_stage_eval(GaArgs g, EvalArgs a,
                                                                      int in, int prev,
                                                                      int index)
{
    constexpr int SD = WD + 1;
    __shared__ __align__(16) uint32_t smask[eval_stage_words<WD>()];
    __shared__ unsigned long long sred[2 * kFusedWaves * kEvalTile];
    __shared__ uint8_t sact[kEvalTile];
    const int ntiles = a.tiles_c * a.tiles_i;
    const int per_xcd = (int)gridDim.x >> 3;
    const int logical = ((int)blockIdx.x & 7) * per_xcd + ((int)blockIdx.x >> 3);
    // Nothing branches before the loads below, so the arguments they need
    // and the loads themselves go out in one round each (a workgroup past
    // the last tile loads tile 0's inputs and leaves with the stop test).
    const bool live = logical < ntiles;
    const int lt = live ? logical : 0;
    const int ti = lt / a.tiles_c, tc = lt - ti * a.tiles_c;
    const int c0 = tc * kEvalTile, rows = min(kEvalTile, g.P - c0);
    const int lane = threadIdx.x & 63, wave = wave_id();
    const int W = g.t.W, out = in ^ 1;
    const int stride = g.NT >> (1 + index % g.lg);
    const int q = lane >> 4, w = lane & 15, rb = lane & ~15;  // row, word, row's first lane
    const int cl = 4 * wave + q;                               // chromosome of the tile
    const bool valid = cl < rows, inw = w < W;
    const int c = c0 + min(cl, rows - 1), pc = c ^ stride;
    const int wl = min(w, W - 1);
    // one round of loads
    const uint64_t *cin = buf(g.cur, in), *oin = buf(g.off, in);
    const uint64_t cc = cin[(int64_t)c * W + wl], oc = oin[(int64_t)c * W + wl];
    const uint64_t cp = cin[(int64_t)pc * W + wl], op = oin[(int64_t)pc * W + wl];
    const unsigned long long fin = buf(g.fit, in)[c], fpin = buf(g.fit, in)[pc];
    const uint8_t okc_b = buf(g.ok, in)[c], okp_b = buf(g.ok, in)[pc];
    const OpDraw dr = g.draws[(int64_t)min(c, pc) * (g.X + g.Y) + index];
    // lanes 0-3 of a row: the counters this stage may change
    const int cs_k = w == 0 ? CS_EVALS : (w == 1 ? CS_SCAN : (w == 2 ? CS_XO_TAKEN : CS_XO_FAIL));
    unsigned long long *cs = g.cstat + (int64_t)c * CS_COUNT;
    const unsigned long long cs_old = cs[cs_k];
    // partial sums of client tile w (a clamped load, always issued; tile t
    // of chromosome x at t * ts + x * xs: the previous fused stage leaves
    // them chromosome-major, one or two cache lines per chromosome), tile
    // w + 16 when there are more than 16, and the evaluation's first chunks,
    // in the same round
    const int64_t ts = g.pcm ? 1 : g.P, xs = g.pcm ? g.TI : 1;
    unsigned long long f = 0, h = 0, sc = 0;
    {
        const int64_t t = min(w, g.TI - 1) * ts;
        const unsigned long long pf = g.part[t + c * xs];
        const unsigned long long ph = g.part[t + pc * xs];
        const uint32_t ps = g.spart[t + c * xs];
        // masked, not branched: a branch would let the compiler move the
        // loads behind it
        const unsigned long long keep = w < g.TI ? ~0ull : 0ull;
        f = pf & keep;
        h = ph & keep;
        sc = ps & keep;
    }
    unsigned long long f2 = 0, h2 = 0, sc2 = 0;
    if (g.TI > 16) {  // uniform
        const int64_t t = min(w + 16, g.TI - 1) * ts;
        const unsigned long long pf = g.part[t + c * xs];
        const unsigned long long ph = g.part[t + pc * xs];
        const uint32_t ps = g.spart[t + c * xs];
        const unsigned long long keep = w + 16 < g.TI ? ~0ull : 0ull;
        f2 = pf & keep;
        h2 = ph & keep;
        sc2 = ps & keep;
    }
    FirstChunks fc;
    eval_first_chunks<H, kFusedWaves>(a, ti, lane, wave, fc);
    // client tiles past 32 (small populations of many clients)
    for (int t = w + 32; t < g.TI; t += 16) {
        f2 += g.part[t * ts + c * xs];
        h2 += g.part[t * ts + pc * xs];
        sc2 += g.spart[t * ts + c * xs];
    }
    if (!live || ga_stopped(g))  // the same for every wave of the workgroup
        return;
    f = row_sum(f + f2);
    h = row_sum(h + h2);
    sc = row_sum(sc + sc2);
    // finish the previous stage for the chromosome and its partner
    const bool okc = okc_b != 0 && prev != OP_NONE;
    const bool take = okc && f < fin;
    const bool ptake = okp_b != 0 && h < fpin;
    const uint64_t A = inw ? (take ? oc : cc) : 0ull;
    const uint64_t B = inw ? (ptake ? op : cp) : 0ull;
    // crossover: from r1 on, cyclically, turn off the first `quota` genes
    // with A = 1, B = 0 and turn on the first `quota` with A = 0, B = 1
    const int r1 = dr.a, quota = dr.b;
    const int w0 = r1 >> 6, b0 = r1 & 63;
    const uint64_t hi_m = ~0ull << b0, lo_m = b0 ? ((1ull << b0) - 1ull) : 0ull;
    const uint64_t x = A & ~B, y = ~A & B;
    // counts packed as (x | y << 16): at most 1024 genes of each kind
    const uint32_t v = (uint32_t)__builtin_popcountll(x) | ((uint32_t)__builtin_popcountll(y) << 16);
    const uint32_t vlo = (uint32_t)__builtin_popcountll(x & lo_m) |
                         ((uint32_t)__builtin_popcountll(y & lo_m) << 16);
    const uint32_t incl = row_scan_incl(v), excl = incl - v;
    const uint32_t total = (uint32_t)__shfl((int)incl, rb + 15);
    const uint32_t excl0 = (uint32_t)__shfl((int)excl, rb + w0);
    const uint32_t lo0 = (uint32_t)__shfl((int)vlo, rb + w0);
    // genes of each kind before this lane's word in the walk order: word w0
    // from bit b0 up, words w0 + 1 ... W - 1, 0 ... w0 - 1, word w0 below b0
    const uint32_t before = w > w0 ? excl - excl0 - lo0 : (w < w0 ? total - excl0 - lo0 + excl : 0u);
    const int tot_x = (int)(total & 0xFFFFu);
    const bool ok = valid && tot_x >= quota;
    // One lowest_bits per kind and lane, the same code for every lane: word
    // w0 is walked in two segments, from bit b0 up first and below b0 last;
    // the walk reaches the low segment only after every other gene of the
    // kind, the whole high segment included.
    const bool first = w == w0;
    const uint32_t main_ = total - lo0;  // genes before the low segment of word w0
    const uint32_t hi_n = v - vlo;       // (lane w0) genes in its high segment
    const int hx = (int)(hi_n & 0xFFFFu), hy = (int)(hi_n >> 16);
    const bool x_hi = quota <= hx, y_hi = quota <= hy;
    const uint64_t sx = first ? (x_hi ? x & hi_m : x & lo_m) : x;
    const uint64_t sy = first ? (y_hi ? y & hi_m : y & lo_m) : y;
    const int kx = first ? (x_hi ? quota : quota - (int)(main_ & 0xFFFFu))
                         : quota - (int)(before & 0xFFFFu);
    const int ky = first ? (y_hi ? quota : quota - (int)(main_ >> 16))
                         : quota - (int)(before >> 16);
    const uint64_t tx = lowest_bits(sx, kx) | (first && !x_hi ? x & hi_m : 0ull);
    const uint64_t ty = lowest_bits(sy, ky) | (first && !y_hi ? y & hi_m : 0ull);
    const uint64_t F = (A & ~tx) | ty;
    if (ok && inw) {
        smask[cl * SD + 2 * w] = (uint32_t)F;
        smask[cl * SD + 2 * w + 1] = (uint32_t)(F >> 32);
    }
    if (w == 0)
        sact[cl] = ok ? 1 : 0;
    if (ti == 0 && valid) {  // the run's state
        if (inw) {
            buf(g.cur, out)[(int64_t)c * W + w] = A;
            if (ok)
                buf(g.off, out)[(int64_t)c * W + w] = F;
        }
        if (w == 0) {
            buf(g.fit, out)[c] = take ? f : fin;
            buf(g.ok, out)[c] = ok ? 1 : 0;
        }
        unsigned long long inc = 0;
        if (w == 0 && okc)
            inc = 1;
        if (w == 1 && okc)
            inc = sc;
        if (w == 2 && take && prev == OP_XOVER)
            inc = 1;
        if (w == 3 && !ok)
            inc = 1;
        if (w < 4 && inc)
            cs[cs_k] = cs_old + inc;
    }
    __syncthreads();
    eval_tile<WD, false, H, kFusedWaves, true>(a, ti, tc, smask, sred, sact, &fc);
}

// The mutation cycle resolved at once (ga_resolve_wave): 64 / YP
// chromosomes per wave.
__global__ __launch_bounds__(64 * kGaWaves) void k_resolve(GaArgs g, int YP, int in, int out)
{
    const int gw = blockIdx.x * kGaWaves + wave_id();
    if (gw * (64 / YP) >= g.P)
        return;
    ga_resolve_wave(g, gw, threadIdx.x & 63, YP, in, out);
}

// The mutation cycle resolved (as k_resolve) by workgroups [0, nres), and the
// next generation's population and operator draws (as k_init) by the
// others.  The two share no data: the new population goes to off[0] with
// its flags, which this generation no longer reads, while the resolve reads
// and writes buffer 1 (the launch is used only when that holds); the
// `improved` flags the resolve would set are dead in this schedule and the
// sampling resets them.  So the sampling runs beside the latency-bound
// resolve instead of in a launch of its own; k_best places the migrants.
__global__ __launch_bounds__(64 * kGaWaves) void k_resolve_init(GaArgs g, int YP, int in,
                                                                int out, int nres)
{
    __shared__ uint64_t sw[kGaWaves][2 * kMaxWords];
    const int wave = wave_id(), lane = threadIdx.x & 63;
    if ((int)blockIdx.x < nres) {
        const int gw = blockIdx.x * kGaWaves + wave;
        if (gw * (64 / YP) >= g.P)
            return;
        ga_resolve_wave(g, gw, lane, YP, in, out, false);
        return;
    }
    const int gw = ((int)blockIdx.x - nres) * kGaWaves + wave;
    const int c = gw >> 1;
    if (c >= g.P || ga_stopped(g))
        return;
    ga_init_one(g, c, lane, sw[wave], gw & 1, true);
}

// Group best per workgroup b < NB; workgroup NB takes the global best
// straight from the population and updates the run state at the same time,
// so no workgroup waits for another.  The group-best workgroups do not test
// the stop flag: workgroup NB may set it in this launch, and once a run has
// stopped its population no longer changes, so rewriting a group best
// stores the same values.
__global__ __launch_bounds__(1024) void k_best(GaArgs g, int fb, int place)
{
    __shared__ unsigned long long sc[16];
    __shared__ int si[16];
    if ((int)blockIdx.x < g.NB)
        ga_group_best(g, fb, blockIdx.x, sc, si, place ? g.off[0] : nullptr);
    else if (!ga_stopped(g))
        ga_global_direct(g, fb, sc, si);
}

// ---------------------------------------------------------------------------
// Grid barrier of the persistent kernel, without a contended counter: each
// workgroup publishes its writes (agent-scope release) and then stores the
// barrier's epoch number into its own flag (its own 128-byte line);
// workgroup 0's threads wait until every flag shows the epoch and then store
// it into the shared epoch word, which the other workgroups wait on.  Every
// workgroup passes the same sequence of barriers, so each knows the epoch
// number it is waiting for.  Waits are bounded by the 100 MHz real-time
// clock: past the bound (only if some workgroup never arrives) the error
// word records it and every later barrier and loop of the kernel returns at
// once, so the grid always drains.
// ---------------------------------------------------------------------------
constexpr uint64_t kBarrierTicks = 200000000ull;  // 2 s at 100 MHz
constexpr int kFlagStride = 32;                   // words between flags

__device__ __forceinline__ uint32_t load_agent(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait until *p == want; false on timeout (and the error is recorded).
__device__ __forceinline__ bool wait_for(const uint32_t *p, uint32_t want,
                                         uint32_t *err)
{
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    while (load_agent(p) != want) {
        __builtin_amdgcn_s_sleep(1);
        if (__builtin_amdgcn_s_memrealtime() - t0 > kBarrierTicks) {
            atomicOr(err, ERR_BARRIER_TIMEOUT);
            return false;
        }
    }
    return true;
}

struct GridBarrier {
    uint32_t *epoch;  // bar[0]
    uint32_t *flags;  // bar + kFlagStride, one per workgroup
    uint32_t *err;
    uint32_t next;    // epoch number of the next barrier

    __device__ __forceinline__ GridBarrier(uint32_t *bar, uint32_t *e)
        : epoch(bar), flags(bar + kFlagStride), err(e), next(load_agent(bar) + 1u)
    {
    }

    __device__ __forceinline__ bool sync(int *flag)
    {
        __syncthreads();
        const uint32_t want = next++;
        if (threadIdx.x == 0) {
            int ok = (load_agent(err) & ERR_BARRIER_TIMEOUT) == 0;
            if (ok) {
                // publish this workgroup's writes (L2 write-back), then arrive
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                __hip_atomic_store(flags + (size_t)blockIdx.x * kFlagStride, want,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            *flag = ok;
        }
        __syncthreads();
        if (!*flag)
            return false;
        if (blockIdx.x == 0) {
            int ok = 1;
            for (int b = threadIdx.x; b < (int)gridDim.x && ok; b += blockDim.x)
                ok = wait_for(flags + (size_t)b * kFlagStride, want, err);
            if (!ok)
                *flag = 0;
            __syncthreads();
            if (threadIdx.x == 0 && *flag)
                __hip_atomic_store(epoch, want, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else if (threadIdx.x == 0) {
            if (!wait_for(epoch, want, err))
                *flag = 0;
        }
        if (threadIdx.x == 0)  // see the other workgroups' writes (L2 invalidate)
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        __syncthreads();
        return *flag != 0;
    }
};

// Evaluation phase: evaluation tiles of every instance whose generation has
// a stage k (k < 0: the population's first evaluation), evaluating offspring
// buffer `buf`.  The global tile range (instance-major, client-tile major
// inside an instance) is cut into 8 contiguous parts; the workgroups of XCD
// x (block index = x mod 8) take part x, so chromosome tiles sharing Pi'
// rows share an L2.
template <int WD>
__device__ __forceinline__ void eval_phase(const BatchArgs &B, int k, int buf,
                                           uint32_t *smask,
                                           unsigned long long *sred)
{
    const int ntiles = B.tile0[B.count];
    const int chunk = (ntiles + 7) / 8;
    const int x = blockIdx.x & 7, per = (int)gridDim.x >> 3;
    const int end = min(ntiles, (x + 1) * chunk);
    for (int item = x * chunk + ((int)blockIdx.x >> 3); item < end; item += per) {
        const int b = B.tile_run[item];
        const BatchItem &it = B.items[b];
        if (ga_stopped(it.g) || k >= it.S)
            continue;
        EvalArgs e = it.e;
        e.masks = buf ? it.g.off[1] : it.g.off[0];
        e.active = buf ? it.g.ok[1] : it.g.ok[0];
        const int local = item - B.tile0[b];
        const int ti = local / e.tiles_c;
        eval_tile<WD>(e, ti, local - ti * e.tiles_c, smask, sred);
    }
}

// All instances stopped?  (Every workgroup reads the same flags after the
// same barrier, so the answer is the same everywhere.)
__device__ __forceinline__ bool all_stopped(const BatchArgs &B)
{
    for (int b = 0; b < B.count; ++b)
        if (!ga_stopped(B.items[b].g))
            return false;
    return true;
}

// ---------------------------------------------------------------------------
// Persistent kernel: `generations` generations of every instance of the
// batch in one launch.  Each phase spreads the work items of all instances
// (chromosomes, evaluation tiles, groups) over the whole grid; grid barriers
// separate the phases.  Instances with fewer stages skip the later ones,
// stopped instances skip everything.  A single instance is a batch of one.
// ---------------------------------------------------------------------------
template <int WD>
__global__ __launch_bounds__(64 * kGaWaves) void k_ga_batch(BatchArgs B,
                                                            int generations)
{
    extern __shared__ uint64_t lds[];
    uint32_t *smask = reinterpret_cast<uint32_t *>(lds);
    unsigned long long *sred =
        reinterpret_cast<unsigned long long *>(lds + eval_stage_words<WD>() / 2);
    __shared__ unsigned long long sc[16];
    __shared__ int si[16];
    __shared__ int flag;
    const int wave = wave_id(), lane = threadIdx.x & 63;
    const int gw = blockIdx.x * kGaWaves + wave, nw = gridDim.x * kGaWaves;
    const int nchrom = B.chrom0[B.count], ngroups = B.group0[B.count];
    GridBarrier bar(B.bar, B.err);

    for (int gen = 0; gen < generations; ++gen) {
        if (all_stopped(B))
            return;
        for (int cg = gw; cg < nchrom; cg += nw) {
            const int b = B.chrom_run[cg];
            const BatchItem &it = B.items[b];
            // the sampler's 2 W words per wave fit in WD (>= 2 W) words of
            // the evaluation's LDS, which is idle in this phase
            if (!ga_stopped(it.g))
                ga_init_one(it.g, cg - B.chrom0[b], lane, lds + wave * WD);
        }
        if (!bar.sync(&flag))
            return;
        eval_phase<WD>(B, -1, 0, smask, sred);
        if (!bar.sync(&flag))
            return;
        for (int k = 0; k <= B.max_S; ++k) {
            for (int cg = gw; cg < nchrom; cg += nw) {
                const int b = B.chrom_run[cg];
                const BatchItem &it = B.items[b];
                if (ga_stopped(it.g) || k > it.S)
                    continue;
                int prev, op, index;
                ga_stage_ops(k, it.X, it.S, &prev, &op, &index);
                ga_stage_one(it.g, cg - B.chrom0[b], lane, k & 1, prev, op, index);
            }
            if (!bar.sync(&flag))
                return;
            if (k < B.max_S) {
                eval_phase<WD>(B, k, (k & 1) ^ 1, smask, sred);
                if (!bar.sync(&flag))
                    return;
            }
        }
        for (int xg = blockIdx.x; xg < ngroups; xg += gridDim.x) {
            const int b = B.group_run[xg];
            const BatchItem &it = B.items[b];
            if (!ga_stopped(it.g))
                ga_group_best(it.g, it.fb, xg - B.group0[b], sc, si);
        }
        if (!bar.sync(&flag))
            return;
        for (int b = blockIdx.x; b < B.count; b += gridDim.x)
            if (!ga_stopped(B.items[b].g))
                ga_global(B.items[b].g, sc, si);
        if (!bar.sync(&flag))
            return;
    }
}

// ---------------------------------------------------------------------------
// The same phases as separate kernels, each spanning every instance of the
// batch (the stream orders them; a hipGraph replays whole generations).
// With a batch, each phase holds milliseconds of work, so launch gaps are
// negligible and each kernel runs at its own register budget.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64 * kGaWaves) void k_batch_init(BatchArgs B)
{
    __shared__ uint64_t sw[kGaWaves][2 * kMaxWords];
    const int cg = blockIdx.x * kGaWaves + wave_id();
    if (cg >= B.chrom0[B.count])
        return;
    const int b = B.chrom_run[cg];
    const BatchItem &it = B.items[b];
    if (!ga_stopped(it.g))
        ga_init_one(it.g, cg - B.chrom0[b], threadIdx.x & 63, sw[wave_id()]);
}

// The batch evaluation runs 16 waves per workgroup (one staged chromosome
// tile shared by more resident waves, each walking fewer clients: the
// fastest shape of the single-run evaluation too).
constexpr int kBatchEvalWaves = 16;

template <int WD>
__global__ __launch_bounds__(kEvalTile *kBatchEvalWaves) void k_batch_eval(BatchArgs B, int k,
                                                                           int buf)
{
    __shared__ __align__(16) uint32_t smask[eval_stage_words<WD>()];
    __shared__ unsigned long long sred[2 * kBatchEvalWaves * kEvalTile];
    const int ntiles = B.tile0[B.count];
    // blocks are dealt to the 8 XCDs round-robin: give XCD x a contiguous
    // eighth of the tile range
    const int per_xcd = (int)gridDim.x >> 3;
    const int item = ((int)blockIdx.x & 7) * per_xcd + ((int)blockIdx.x >> 3);
    if (item >= ntiles)
        return;
    const int b = B.tile_run[item];
    const BatchItem &it = B.items[b];
    if (ga_stopped(it.g) || k >= it.S)
        return;
    EvalArgs e = it.e;
    e.masks = buf ? it.g.off[1] : it.g.off[0];
    e.active = buf ? it.g.ok[1] : it.g.ok[0];
    const int local = item - B.tile0[b];
    const int ti = local / e.tiles_c;
    // the walk each instance's scan lengths call for (uniform per workgroup)
    if (e.paired)
        eval_tile<WD, false, true, kBatchEvalWaves>(e, ti, local - ti * e.tiles_c, smask, sred);
    else
        eval_tile<WD, false, false, kBatchEvalWaves>(e, ti, local - ti * e.tiles_c, smask, sred);
}

__global__ __launch_bounds__(64 * kGaWaves) void k_batch_stage(BatchArgs B, int k)
{
    const int cg = blockIdx.x * kGaWaves + wave_id();
    if (cg >= B.chrom0[B.count])
        return;
    const int b = B.chrom_run[cg];
    const BatchItem &it = B.items[b];
    if (ga_stopped(it.g) || k > it.S)
        return;
    int prev, op, index;
    ga_stage_ops(k, it.X, it.S, &prev, &op, &index);
    ga_stage_one(it.g, cg - B.chrom0[b], threadIdx.x & 63, k & 1, prev, op, index);
}

// Group bests; the last group of an instance to finish does that
// instance's global update.
__global__ __launch_bounds__(256) void k_batch_best(BatchArgs B)
{
    __shared__ unsigned long long sc[16];
    __shared__ int si[16];
    __shared__ int last;
    const int xg = blockIdx.x;
    const int b = B.group_run[xg];
    const BatchItem &it = B.items[b];
    if (ga_stopped(it.g))
        return;
    ga_group_best(it.g, it.fb, xg - B.group0[b], sc, si);
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0)
        last = atomicAdd(it.g.arrive, 1u) == (uint32_t)(it.g.NB - 1);
    __syncthreads();
    if (!last)
        return;
    __threadfence();
    ga_global(it.g, sc, si);
    if (threadIdx.x == 0)
        *it.g.arrive = 0;
}

template <int WD>
hipError_t batch_kernels_wd(const BatchArgs &b, int nchrom, int ntiles, int ngroups,
                            int generations, hipStream_t s, const BatchEvents &ev)
{
    const dim3 waves((unsigned)((nchrom + kGaWaves - 1) / kGaWaves));
    const dim3 tiles((unsigned)(((ntiles + 7) / 8) * 8));
    // the evaluation launch, bracketed by the next pair of events if any
    auto eval = [&](int k, int buf) {
        if (ev.events && *ev.used + 2 <= ev.cap) {
            hipExtLaunchKernelGGL(k_batch_eval<WD>, tiles, dim3(kEvalTile * kBatchEvalWaves), 0,
                                  s, ev.events[*ev.used], ev.events[*ev.used + 1], 0, b, k,
                                  buf);
            *ev.used += 2;
        } else {
            hipLaunchKernelGGL(k_batch_eval<WD>, tiles, dim3(kEvalTile * kBatchEvalWaves), 0, s,
                               b, k, buf);
        }
    };
    for (int gen = 0; gen < generations; ++gen) {
        hipLaunchKernelGGL(k_batch_init, waves, dim3(64 * kGaWaves), 0, s, b);
        eval(-1, 0);
        for (int k = 0; k <= b.max_S; ++k) {
            hipLaunchKernelGGL(k_batch_stage, waves, dim3(64 * kGaWaves), 0, s, b, k);
            if (k < b.max_S)
                eval(k, (k & 1) ^ 1);
        }
        hipLaunchKernelGGL(k_batch_best, dim3((unsigned)ngroups), dim3(256), 0, s, b);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

inline dim3 per_wave(int P)
{
    return dim3((unsigned)((P + kGaWaves - 1) / kGaWaves));
}

template <int WD>
size_t batch_lds()
{
    return sizeof(uint32_t) * eval_stage_words<WD>() +
           sizeof(unsigned long long) * 2 * kEvalWaves * kEvalTile;
}

template <int WD>
hipError_t batch_wd(const BatchArgs &b, int generations, int max_blocks,
                    int want, hipStream_t s, int *grid_out, bool cooperative)
{
    auto fn = k_ga_batch<WD>;
    const size_t lds = batch_lds<WD>();
    hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                                         hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)lds);
    if (err != hipSuccess)
        return err;
    int per_cu = 0, dev = 0, cus = 0;
    err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64 * kGaWaves, lds);
    if (err == hipSuccess)
        err = hipGetDevice(&dev);
    if (err == hipSuccess)
        err = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (err != hipSuccess)
        return err;
    if (per_cu < 1)
        return hipErrorInvalidConfiguration;
    // enough workgroups for the widest phase, no more than fit at once
    int grid = min(want, min(per_cu, 4) * cus);
    if (max_blocks > 0)
        grid = min(grid, max_blocks);
    grid = max(8, (grid / 8) * 8);
    if (grid > per_cu * cus || grid > kMaxPersistentBlocks)
        return hipErrorInvalidConfiguration;
    *grid_out = grid;
    if (!cooperative) {
        // every workgroup fits at once (checked above); the barrier waits
        // are bounded in any case
        hipLaunchKernelGGL(fn, dim3(grid), dim3(64 * kGaWaves), lds, s, b, generations);
        return hipGetLastError();
    }
    BatchArgs ba = b;
    int gens = generations;
    void *args[] = {&ba, &gens};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(fn), dim3(grid),
                                      dim3(64 * kGaWaves), args, (unsigned)lds, s);
}

}  // namespace

hipError_t launch_ga_init(const GaArgs &g, hipStream_t s)
{
    hipLaunchKernelGGL(k_init, per_wave(2 * g.P), dim3(64 * kGaWaves), 0, s, g);
    return hipGetLastError();
}

hipError_t launch_ga_stage(const GaArgs &g, int in, int prev, int op, int index,
                           hipStream_t s)
{
    const int waves = op == OP_MUT_ALL ? g.P * ((g.Y + g.mpw - 1) / g.mpw) : g.P;
    hipLaunchKernelGGL(k_stage, per_wave(waves), dim3(64 * kGaWaves), 0, s, g, in,
                       prev, op, index);
    return hipGetLastError();
}

bool ga_stage_eval_fits(int W)
{
    return W <= kFusedMaxW;
}

hipError_t launch_ga_stage_eval(const GaArgs &g, const EvalArgs &a, int in, int prev,
                                int index, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    const int tiles = a.tiles_c * a.tiles_i;
    const dim3 grid((unsigned)(((tiles + 7) / 8) * 8)), block(kEvalTile * kFusedWaves);
    const int w2 = 2 * g.t.W;
#define PMP_FUSED_WD(N)                                                                 \
    if (w2 <= N) {                                                                      \
        auto fn = a.paired ? k_stage_eval<N, true> : k_stage_eval<N, false>;            \
        if (e0 && e1)                                                                   \
            hipExtLaunchKernelGGL(fn, grid, block, 0, s, e0, e1, 0, g, a, in, prev, index); \
        else                                                                            \
            hipLaunchKernelGGL(fn, grid, block, 0, s, g, a, in, prev, index);           \
        return hipGetLastError();                                                       \
    }
    PMP_FUSED_WD(2)
    PMP_FUSED_WD(4)
    PMP_FUSED_WD(8)
    PMP_FUSED_WD(16)
    PMP_FUSED_WD(32)
#undef PMP_FUSED_WD
    return hipErrorInvalidValue;
}

hipError_t launch_ga_resolve(const GaArgs &g, int in, int out, hipStream_t s)
{
    int YP = 1;
    while (YP < g.Y)
        YP <<= 1;
    const int per = 64 / YP;
    hipLaunchKernelGGL(k_resolve, per_wave((g.P + per - 1) / per), dim3(64 * kGaWaves), 0, s, g,
                       YP, in, out);
    return hipGetLastError();
}

hipError_t launch_ga_best(const GaArgs &g, int fb, hipStream_t s, bool place_migrants)
{
    const int threads = ((g.NT + 63) / 64) * 64;
    hipLaunchKernelGGL(k_best, dim3(g.NB + 1), dim3(threads < 64 ? 64 : threads), 0, s,
                       g, fb, place_migrants ? 1 : 0);
    return hipGetLastError();
}

namespace {

// One workgroup: counter totals by a strided sum and an LDS reduction per
// counter, then the run state, the error words and the best mask.
__global__ __launch_bounds__(256) void k_report(GaArgs g, const uint32_t *err0,
                                                const uint32_t *err1, unsigned long long *out)
{
    __shared__ unsigned long long sum[CS_COUNT][256];
    unsigned long long t[CS_COUNT];
#pragma unroll
    for (int k = 0; k < CS_COUNT; ++k)
        t[k] = 0;
    for (int c = threadIdx.x; c < g.P; c += 256) {
#pragma unroll
        for (int k = 0; k < CS_COUNT; ++k)
            t[k] += g.cstat[(int64_t)c * CS_COUNT + k];
    }
#pragma unroll
    for (int k = 0; k < CS_COUNT; ++k)
        sum[k][threadIdx.x] = t[k];
    __syncthreads();
    for (int half = 128; half > 0; half >>= 1) {
        if (threadIdx.x < half) {
#pragma unroll
            for (int k = 0; k < CS_COUNT; ++k)
                sum[k][threadIdx.x] += sum[k][threadIdx.x + half];
        }
        __syncthreads();
    }
    if (threadIdx.x < CS_COUNT)
        out[RP_TOT + threadIdx.x] = sum[threadIdx.x][0];
    if (threadIdx.x < GS_COUNT)
        out[RP_GS + threadIdx.x] = g.gs[threadIdx.x];
    if (threadIdx.x == 0)
        out[RP_ERR] = (unsigned long long)(*err0 | (err1 ? *err1 : 0u));
    for (int w = threadIdx.x; w < g.t.W; w += 256)
        out[RP_MASK + w] = g.best_mask[w];
}

}  // namespace

hipError_t launch_ga_report(const GaArgs &g, const uint32_t *err0, const uint32_t *err1,
                            unsigned long long *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_report, dim3(1), dim3(256), 0, s, g, err0, err1, out);
    return hipGetLastError();
}

hipError_t launch_ga_resolve_init(const GaArgs &g, int in, int out, hipStream_t s)
{
    int YP = 1;
    while (YP < g.Y)
        YP <<= 1;
    const int per = 64 / YP;
    const int nres = ((g.P + per - 1) / per + kGaWaves - 1) / kGaWaves;
    const int ninit = (2 * g.P + kGaWaves - 1) / kGaWaves;
    hipLaunchKernelGGL(k_resolve_init, dim3(nres + ninit), dim3(64 * kGaWaves), 0, s, g, YP, in,
                       out, nres);
    return hipGetLastError();
}

hipError_t launch_ga_batch_kernels(const BatchArgs &b, int nchrom, int ntiles,
                                   int ngroups, int generations, int max_w2,
                                   hipStream_t s, const BatchEvents &ev)
{
    const int w2 = max_w2;
#define PMP_BATCH_KWD(N)                                                       \
    if (w2 <= N)                                                               \
        return batch_kernels_wd<N>(b, nchrom, ntiles, ngroups, generations, s, ev);
    PMP_BATCH_KWD(2)
    PMP_BATCH_KWD(4)
    PMP_BATCH_KWD(8)
    PMP_BATCH_KWD(16)
    PMP_BATCH_KWD(32)
    PMP_BATCH_KWD(48)
    PMP_BATCH_KWD(64)
    PMP_BATCH_KWD(96)
    PMP_BATCH_KWD(128)
    PMP_BATCH_KWD(160)
    PMP_BATCH_KWD(192)
    PMP_BATCH_KWD(256)
#undef PMP_BATCH_KWD
    return hipErrorInvalidValue;
}

template <int WD>
hipError_t batch_eval_wd(const BatchArgs &b, int ntiles, hipStream_t s)
{
    const dim3 tiles((unsigned)(((ntiles + 7) / 8) * 8));
    hipLaunchKernelGGL(k_batch_eval<WD>, tiles, dim3(kEvalTile * kBatchEvalWaves), 0, s, b, -1,
                       0);
    return hipGetLastError();
}

hipError_t launch_ga_batch_eval(const BatchArgs &b, int ntiles, int max_w2, hipStream_t s)
{
#define PMP_BATCH_EWD(N)                                                       \
    if (max_w2 <= N)                                                           \
        return batch_eval_wd<N>(b, ntiles, s);
    PMP_BATCH_EWD(2)
    PMP_BATCH_EWD(4)
    PMP_BATCH_EWD(8)
    PMP_BATCH_EWD(16)
    PMP_BATCH_EWD(32)
    PMP_BATCH_EWD(48)
    PMP_BATCH_EWD(64)
    PMP_BATCH_EWD(96)
    PMP_BATCH_EWD(128)
    PMP_BATCH_EWD(160)
    PMP_BATCH_EWD(192)
    PMP_BATCH_EWD(256)
#undef PMP_BATCH_EWD
    return hipErrorInvalidValue;
}

hipError_t launch_ga_batch(const BatchArgs &b, int generations, int max_w2,
                           int max_blocks, int want_blocks, hipStream_t s,
                           int *grid, bool cooperative)
{
    const int w2 = max_w2;
#define PMP_BATCH_WD(N)                                                        \
    if (w2 <= N)                                                               \
        return batch_wd<N>(b, generations, max_blocks, want_blocks, s, grid,   \
                           cooperative);
    PMP_BATCH_WD(2)
    PMP_BATCH_WD(4)
    PMP_BATCH_WD(8)
    PMP_BATCH_WD(16)
    PMP_BATCH_WD(32)
    PMP_BATCH_WD(48)
    PMP_BATCH_WD(64)
    PMP_BATCH_WD(96)
    PMP_BATCH_WD(128)
    PMP_BATCH_WD(160)
    PMP_BATCH_WD(192)
    PMP_BATCH_WD(256)
#undef PMP_BATCH_WD
    return hipErrorInvalidValue;
}

}  // namespace pmp
