// Host runtime of the p-median library: argument checking, device memory
// owned by handles, launch sequencing and the extern "C" entry points
// declared in pmp.h.
#include "pmp.h"

#include <algorithm>
#include <atomic>
#include <climits>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "common.hpp"
#include "learn_device.hpp"

using namespace pmp;

namespace {

thread_local std::string g_last_error;

pmp_status fail(pmp_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

#define HIP_TRY(expr)                                                       \
    do {                                                                    \
        hipError_t e_ = (expr);                                             \
        if (e_ != hipSuccess)                                               \
            return fail(PMP_EDEVICE, "%s failed: %s", #expr,                \
                        hipGetErrorString(e_));                             \
    } while (0)

template <class T>
hipError_t dalloc(T **p, size_t count)
{
    *p = nullptr;
    if (count == 0)
        count = 1;
    return hipMalloc((void **)p, sizeof(T) * count);
}

template <class T>
void dfree(T *&p)
{
    if (p)
        (void)hipFree((void *)p);
    p = nullptr;
}

// Pinned host memory shared by the process for small read-backs (a few
// hundred bytes), used under its lock: one asynchronous copy on the
// caller's stream, then a wait for that stream.
struct Staging {
    std::mutex mu;
    unsigned long long *host = nullptr;
    size_t cap = 0;

    // (called with mu held)
    hipError_t reserve(size_t words)
    {
        if (cap >= words)
            return hipSuccess;
        if (host)
            (void)hipHostFree(host);
        host = nullptr;
        cap = 0;
        const hipError_t e =
            hipHostMalloc((void **)&host, sizeof(unsigned long long) * words, hipHostMallocDefault);
        if (e == hipSuccess)
            cap = words;
        return e;
    }
    // words device words after the work on s, into out
    hipError_t read(const unsigned long long *dev, size_t words, hipStream_t s,
                    std::vector<unsigned long long> &out)
    {
        std::lock_guard<std::mutex> lock(mu);
        hipError_t e = reserve(words);
        if (e == hipSuccess)
            e = hipMemcpyAsync(host, dev, sizeof(unsigned long long) * words,
                               hipMemcpyDeviceToHost, s);
        if (e == hipSuccess)
            e = hipStreamSynchronize(s);
        if (e == hipSuccess)
            out.assign(host, host + words);
        return e;
    }
};

Staging &staging()
{
    static Staging st;
    return st;
}

// Fixed-size buffers of one object carved out of a single device
// allocation (one hipMalloc and one hipFree instead of one per buffer).
// Members are listed with add(), then carve() allocates and assigns them;
// release() frees the block and clears the members.  Buffers that are
// reallocated later keep allocations of their own.
struct Arena {
    void *base = nullptr;
    std::vector<std::pair<void **, size_t>> members;

    template <class T>
    void add(T **p, size_t count)
    {
        members.emplace_back(reinterpret_cast<void **>(p),
                             sizeof(T) * (count == 0 ? 1 : count));
    }
    size_t bytes() const
    {
        size_t total = 0;
        for (const auto &m : members)
            total += (m.second + 255) & ~size_t(255);
        return total;
    }
    hipError_t carve()
    {
        const size_t total = bytes();
        hipError_t e = hipMalloc(&base, total);
        if (e != hipSuccess) {
            base = nullptr;
            return e;
        }
        char *q = static_cast<char *>(base);
        for (const auto &m : members) {
            *m.first = q;
            q += (m.second + 255) & ~size_t(255);
        }
        return hipSuccess;
    }
    // every member zeroed (one memset over the allocation)
    hipError_t zero() const { return hipMemset(base, 0, bytes()); }
    void release()
    {
        for (const auto &m : members)
            *m.first = nullptr;
        if (base)
            (void)hipFree(base);
        base = nullptr;
        members.clear();
    }
};

int env_int(const char *name, int dflt)
{
    const char *v = getenv(name);
    if (!v || !*v)
        return dflt;
    return atoi(v);
}

// Whether the evaluation walks two clients per chunk.  A pair's chunk holds
// 32 entries of each row, and a row goes on to a tail chunk as soon as one
// of the tile's 64 chromosomes has its first open facility past entry 31;
// a tail chunk costs as much as a full one.  With mean scan (m+1)/(p+1) = 10
// (G900, E5000 p = 500) most rows need the tail, and the single 64-entry
// walk is faster (G900 80 -> 87 G evaluations/s, E5000 p = 500 85 -> 63 us),
// so pairs are taken only for mean scans up to 4, where a row's 64
// chromosomes rarely reach past 32.  PMP_EVAL_PAIRED=0/1 forces it.
int paired_scans(int m, int p)
{
    const int forced = env_int("PMP_EVAL_PAIRED", -1);
    if (forced >= 0)
        return forced ? 1 : 0;
    return (int64_t)m + 1 <= 4LL * ((int64_t)p + 1) ? 1 : 0;
}

// Clients per workgroup of the evaluation kernel.  A workgroup first stages
// its chromosome tile (W words per chromosome loaded and turned
// facility-major), then walks its clients.  With long scans (mean
// (m+1)/(p+1) of 128 entries or more) the walks dominate: enough workgroups
// to fill 256 CUs four times over, at most 64 clients each, so that uneven
// scan lengths even out.  With short scans the staging counts: the fewest
// client tiles that still give every CU of the device about 2.75
// workgroups, or that fill every CU's resident slots once when it holds
// fewer than 3.5, so that no workgroup waits for a slot.
// Waves per workgroup of the evaluation kernel (4, 8 or 16 waves share one
// staged chromosome tile).  PMP_EVAL_WAVES forces it.
int eval_waves(int n, int P, int m, int p, int W)
{
    (void)n;
    (void)P;
    (void)m;
    (void)p;
    (void)W;
    const int forced = env_int("PMP_EVAL_WAVES", 0);
    if (forced == 4 || forced == 8 || forced == 16)
        return forced;
    // 16 waves were fastest on every measured shape: G900 88.7 -> 98.3 G
    // evaluations/s against 4; E5000 p = 10 / 100 / 500 1.63 / 0.224 /
    // 0.067 -> 0.95 / 0.154 / 0.050 ms (more waves resident per CU for the
    // same staged tile, and fewer clients in each wave's chain)
    return 16;
}

// Clients per workgroup of the fused stage-and-evaluation launches.  Each
// client tile's workgroup repeats the stage step of its 64 chromosomes, so
// these tiles are larger than the plain evaluation's: about 512 workgroups,
// 64 clients at least.  PMP_FUSED_CLIENTS forces it.
int fused_clients_per_block(int n, int P)
{
    const int forced = env_int("PMP_FUSED_CLIENTS", 0);
    if (forced > 0)
        return forced;
    const long tiles_c = (P + kEvalTile - 1) / kEvalTile;
    const long ti = std::max(1L, 512 / std::max(1L, tiles_c));
    long f = ((long)n + ti - 1) / ti;
    f = std::max(f, 64L);
    return (int)std::min<long>(f, n);
}

int clients_per_block(int n, int P, int m, int p, int W, bool reduced = false,
                      int waves = kEvalWaves)
{
    const int forced = env_int("PMP_CLIENTS_PER_BLOCK", 0);
    if (forced > 0)
        return forced;
    const long tiles_c = (P + kEvalTile - 1) / kEvalTile;
    const bool long_scans = (long)m + 1 >= 128L * ((long)p + 1);
    if (long_scans) {
        long cpb = (long)n * tiles_c / 1024;
        cpb = std::min(64L, std::max(4L, cpb));
        return (int)(((cpb + waves - 1) / waves) * waves);
    }
    const bool paired = paired_scans(m, p) != 0;
    static std::atomic<int> cus_of[64];  // per device, queried once
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess && dev >= 0 && dev < 64) {
        cus = cus_of[dev].load(std::memory_order_relaxed);
        if (cus == 0 &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess)
            cus_of[dev].store(cus, std::memory_order_relaxed);
    }
    if (cus < 1)
        cus = 256;
    const long slots = (long)cus * eval_workgroups_per_cu(W, reduced, paired, waves);
    // When the CUs hold fewer than 3.5 workgroups each, fill the slots once;
    // else aim at about 2.75 per CU (G900: 20 clients per workgroup measured
    // 2 % faster than 16, 12 and 32 slower)
    const long busy = slots < (long)cus * 7 / 2 ? slots : (long)cus * 11 / 4;
    const long want = std::min(slots, busy);
    long ti = want >= slots ? std::max(1L, slots / tiles_c) : (want + tiles_c - 1) / tiles_c;
    ti = std::min(ti, std::max(1L, ((long)n + 3) / 4));
    long cpb = std::max(1L, ((long)n + ti - 1) / ti);
    // Small tiles: the same number of clients (of client pairs, when paired)
    // for each of the 4 waves, or one wave's extra client sets the
    // workgroup's time.  (When the slots are the limit, rounding down would
    // add a client tile and a partial second round of workgroups.)
    const long unit = (paired ? 2 : 1) * waves;
    if (cpb < 64 && want < slots && cpb >= unit)
        cpb -= cpb % unit;
    return (int)cpb;
}

// binom[a (p + 1) + b] = C(a, b) for a < m, b <= p, by Pascal's rule,
// saturating at 2^63; returns C(m, p) (kBinomSat when it saturates).
constexpr unsigned long long kBinomSat = 1ull << 63;

unsigned long long binomial_table(int m, int p, std::vector<unsigned long long> &binom)
{
    binom.assign((size_t)m * (p + 1), 0ull);
    auto add = [](unsigned long long x, unsigned long long y) {
        return x >= kBinomSat - y ? kBinomSat : x + y;
    };
    for (int a = 0; a < m; ++a) {
        binom[(size_t)a * (p + 1)] = 1;
        for (int b = 1; b <= p && b <= a; ++b) {
            const unsigned long long x = binom[(size_t)(a - 1) * (p + 1) + b - 1];
            const unsigned long long y = b <= a - 1 ? binom[(size_t)(a - 1) * (p + 1) + b] : 0ull;
            binom[(size_t)a * (p + 1) + b] = add(x, y);
        }
    }
    // C(m, p) = C(m - 1, p - 1) + C(m - 1, p)
    return add(binom[(size_t)(m - 1) * (p + 1) + p - 1], binom[(size_t)(m - 1) * (p + 1) + p]);
}

pmp_status status_from_err(uint32_t e)
{
    if (e & ERR_BARRIER_TIMEOUT)
        return fail(PMP_EDEVICE, "a grid barrier of the GA kernel timed out");
    if (e & ERR_NEGATIVE_DISTANCE)
        return fail(PMP_EINVAL, "negative distance in d");
    if (e & (ERR_POPCOUNT | ERR_STRAY_BITS | ERR_SCAN_OVERRUN))
        return fail(PMP_EINFEASIBLE,
                    "chromosome without exactly p open facilities (error bits 0x%x)",
                    e);
    return PMP_OK;
}

}  // namespace

struct pmp_instance {
    int32_t n = 0, m = 0, p = 0, K = 0, W = 0, pitch = 0;
    uint16_t *pi = nullptr;
    int32_t *ds = nullptr;
    int32_t *delta = nullptr;
    uint32_t *err = nullptr;
    // staging for host-pointer evaluation
    uint64_t *h_masks = nullptr;
    unsigned long long *h_fit = nullptr;
    unsigned long long *h_scan = nullptr;
    int32_t h_cap = 0;
    // client-tile partial sums of the evaluation kernel
    unsigned long long *part = nullptr;
    uint32_t *spart = nullptr;
    size_t part_cap = 0;
    // facility-major tiles of chromosomes wider than the LDS staging
    uint64_t *tg = nullptr;
    size_t tg_cap = 0;
    // static sums of the learned proposal's features
    unsigned long long *colsum = nullptr;  // m column sums of d
    uint32_t *nearc = nullptr;             // m near counts
    mutable int64_t total = 0;             // sum of d
    mutable bool total_pending = false;    // not read back yet (asynchronous preprocessing)
    int32_t near_len = 1;                  // ceil(m / p)
    unsigned long long *dtotal = nullptr;  // the sum and the error word, read back together
    Arena arena;                           // pi, ds, delta, err, colsum, nearc, dtotal

    // the sum of d, read back on its first use after an asynchronous
    // preprocessing (which may still be running on its stream)
    hipError_t resolve_total() const
    {
        if (!total_pending)
            return hipSuccess;
        unsigned long long t = 0;
        hipError_t e = hipDeviceSynchronize();
        if (e == hipSuccess)
            e = hipMemcpy(&t, dtotal, sizeof t, hipMemcpyDeviceToHost);
        if (e == hipSuccess) {
            total = (int64_t)t;
            total_pending = false;
        }
        return e;
    }

    Tables tables() const
    {
        Tables t;
        t.pi = pi;
        t.ds = ds;
        t.n = n;
        t.m = m;
        t.p = p;
        t.K = K;
        t.W = W;
        t.pitch = pitch;
        return t;
    }
};

namespace {

// Device-side description of a set of GA runs advanced together by the
// persistent kernel (k_ga_batch).
struct BatchHost {
    std::vector<pmp_ga *> gas;
    BatchItem *d_items = nullptr;
    int32_t *d_prefix = nullptr;  // chrom0 | tile0 | group0, count + 1 each
    uint32_t *d_bar = nullptr;
    uint32_t *d_err = nullptr;
    BatchArgs args{};
    int max_w2 = 2, want = 8, last_grid = 0;
    int nchrom = 0, ntiles = 0, ngroups = 0;
    std::map<int, hipGraphExec_t> graphs;  // by generations per launch
    // host copies of the run table and prefix offsets; each run's clients
    // per workgroup from its own tuning (scaled to the batch kernel's
    // waves), or `clients` for every run (0: none)
    std::vector<BatchItem> items;
    std::vector<int32_t> prefix;
    std::vector<int32_t> base_cpb;
    int clients = 0;
    // run of every chromosome, group and evaluation tile (host copy and
    // device table; tiles sized for the most any tiling can give)
    std::vector<int32_t> runs;
    int32_t *d_runs = nullptr;
    int max_tiles = 0;

    void drop_graphs()
    {
        for (auto &kv : graphs)
            (void)hipGraphExecDestroy(kv.second);
        graphs.clear();
    }

    void release()
    {
        drop_graphs();
        dfree(d_items);
        dfree(d_prefix);
        dfree(d_runs);
        dfree(d_bar);
        dfree(d_err);
    }
};

}  // namespace

// A scoring network: device parameters, Adam state and staging buffers.
struct pmp_model {
    MlpModelDev d{};
    float *partials = nullptr;   // training partial sums (kPartFloats, by part_index)
    float *grad = nullptr;       // staging of a host gradient output
    float *loss = nullptr;       // one float
    float *xf = nullptr;         // staging of host inputs (rows x 32)
    uint16_t *xb = nullptr;      // BF16 inputs (rows x 32)
    float *tf = nullptr, *wf = nullptr, *yf = nullptr;  // rows each
    int64_t cap = 0;             // rows the staging holds
};

namespace {
constexpr int kTrainBlocks = kMaxTrainBlocks;  // workgroups of a training gradient launch
}

struct pmp_ga {
    pmp_instance *inst = nullptr;
    pmp_ga_params prm{};
    int NB = 0, lg = 0, X = 0, Y = 0, TI = 0, cpb = 0;
    bool fused = true;            // crossover stages fused with their evaluations
    int fcpb = 0, fTI = 0;        // client tiles of the fused launches
    int waves = kEvalWaves;       // waves per workgroup of the population's evaluation
    int spec_waves = kEvalWaves;  // and of the mutants' evaluation
    uint64_t *cur[2] = {nullptr, nullptr}, *off[2] = {nullptr, nullptr};
    unsigned long long *fit[2] = {nullptr, nullptr};
    uint8_t *ok[2] = {nullptr, nullptr};
    uint8_t *improved = nullptr;
    OpDraw *draws = nullptr;
    // the mutation cycle evaluated at once (allocated on first use)
    uint64_t *mut = nullptr;
    uint8_t *mut_ok = nullptr;
    unsigned long long *mpart = nullptr;
    uint32_t *mspart = nullptr;
    int spec_ti = 0;  // client tiles mpart was sized for (the mutants' evaluation)
    int spec_cpb = 0;  // its clients per workgroup
    bool spec_on = true;
    unsigned long long *part = nullptr;
    uint32_t *spart = nullptr;
    // second set of partial sums: fused stage launches alternate between the
    // two (one reads the previous stage's sums while it writes its own)
    unsigned long long *part2 = nullptr;
    uint32_t *spart2 = nullptr;
    uint64_t *gmask = nullptr, *best = nullptr;
    unsigned long long *binom = nullptr;  // PMP_INIT_RANK: binomial table
    uint64_t nsets = 0;                   // PMP_INIT_RANK: C(m, p)
    unsigned long long *gcost = nullptr, *gs = nullptr, *cstat = nullptr;
    uint32_t *arrive = nullptr;
    uint32_t *bar = nullptr;
    unsigned long long *report = nullptr;  // GaReport layout, RP_MASK + W words
    Arena arena;  // the fixed-size buffers above (not part/spart, mut, mpart)
    Arena parts;  // part, spart, part2, spart2 (sized by the client tiling)

    // the client-tile partial sums for `tiles` tiles (both sets)
    hipError_t carve_parts(int tiles)
    {
        parts.release();
        const size_t cells = (size_t)tiles * prm.population;
        parts.add(&part, cells);
        parts.add(&spart, cells);
        parts.add(&part2, cells);
        parts.add(&spart2, cells);
        return parts.carve();
    }
    bool persistent = false;  // one persistent launch per pmp_ga_step call
    BatchHost *self = nullptr;  // this run as a batch of one
    // graph of `graph_gens` generations of the per-step launch sequence
    int graph_gens = 0;
    hipGraphExec_t gexec = nullptr;
    int max_blocks = 0;
    int last_grid = 0;
    // profiling of the evaluation kernel
    bool prof = false;
    std::vector<hipEvent_t> ev;
    size_t ev_used = 0;
    unsigned long long base_scan = 0, base_evals = 0;
    // learned proposal (model == nullptr: plain GA)
    pmp_model *model = nullptr;
    int LC = 0, LL = 0, Lexp = 0, LH = 0, Levery = 0;
    float Llr = 0.f;
    int32_t *swaps = nullptr;
    uint16_t *rep_x = nullptr;
    float *rep_t = nullptr, *rep_w = nullptr;
    int32_t *rep_jk = nullptr;
    long long *rep_d = nullptr;
    float *scores = nullptr;
    int32_t *cand = nullptr;
    uint64_t *cbits = nullptr;
    uint8_t *cpre = nullptr;
    void *sums = nullptr;  // P x kSlots: a, dd (uint32), b, cc, e (uint64)
    unsigned long long *last_trained = nullptr;
    int walk_shape = 0;  // proposal walk: 0 two passes, else chromosomes per workgroup
    // two-pass walk: first two open positions and costs per (chromosome,
    // client), and the facility index of every row's first positions
    uint32_t *s12 = nullptr;
    int32_t *c12 = nullptr;
    int32_t *near_off = nullptr;
    uint2 *near_q = nullptr;

    int64_t ring_rows() const { return (int64_t)LH * LL * prm.population; }

    // crossover stages actually run (none when p < 2 or NT = 1)
    int xstages() const { return (inst->p >= 2 && lg > 0) ? X : 0; }
    // buffer holding the population after a generation's last stage
    int final_buf() const { return ((xstages() + Y) % 2) ^ 1; }
    // The next generation's population is made in the launch of this
    // generation's resolve step (launch_ga_resolve_init) when nothing of this
    // generation reads buffer 0 after the mutants are made: the whole cycle
    // at once, no learned proposal, the resolve reading and writing buffer 1.
    bool merge_init(const GaArgs &g) const
    {
        return spec() && g.L == 0 && xstages() % 2 == 0 && final_buf() == 1;
    }
    // the device already holds the population and draws of the generation
    // the run is at (made ahead by the previous one's resolve launch)
    bool init_ahead = false;
    // the per-step schedule evaluates the whole mutation cycle at once (one
    // evaluation of P x Y mutants instead of Y dependent ones; with the
    // learned proposal the scored swaps are among them); the batched and
    // persistent schedules run it attempt by attempt.  Both give the same
    // results.
    bool spec() const
    {
        return spec_on && Y >= 2 && Y <= kMaxSpec;
    }
    // The mutants' evaluation covers Y times the population, so it takes
    // larger client tiles than the population's (about 2048 workgroups):
    // fewer partial sums for the resolve step to add up.
    hipError_t ensure_spec()
    {
        const size_t PY = (size_t)prm.population * Y;
        if (!mut) {
            hipError_t e = dalloc(&mut, PY * inst->W);
            if (e == hipSuccess)
                e = dalloc(&mut_ok, PY);
            if (e != hipSuccess)
                return e;
        }
        const long tiles_c = (long)((PY + kEvalTile - 1) / kEvalTile);
        const int n = inst->n;
        const long target = std::max(1, env_int("PMP_MUTANT_WORKGROUPS", 1024));
        int ti = (int)std::max(1L, std::min((long)n, target / std::max(1L, tiles_c)));
        ti = std::max(ti, (n + 127) / 128);  // at most 128 clients per workgroup
        int cpb = (n + ti - 1) / ti;
        cpb = std::max(cpb, this->cpb);
        cpb = ((cpb + 3) / 4) * 4;
        ti = (n + cpb - 1) / cpb;
        if (spec_ti != ti || spec_cpb != cpb) {
            dfree(mpart);
            dfree(mspart);
            spec_ti = 0;
            hipError_t e = dalloc(&mpart, PY * ti);
            if (e == hipSuccess)
                e = dalloc(&mspart, PY * ti);
            if (e != hipSuccess)
                return e;
            spec_ti = ti;
            spec_cpb = cpb;
            if (gexec) {  // a captured graph holds the old buffers
                (void)hipGraphExecDestroy(gexec);
                gexec = nullptr;
            }
        }
        return hipSuccess;
    }

    GaArgs args() const
    {
        GaArgs g{};
        g.t = inst->tables();
        g.seed = prm.seed;
        g.P = prm.population;
        g.NT = prm.group_size;
        g.NB = NB;
        g.lg = lg;
        g.X = X;
        g.Y = Y;
        g.generations = prm.generations;
        g.saturation = prm.saturation;
        g.migration = prm.migration;
        g.init_rank = prm.init == PMP_INIT_RANK;
        g.binom = binom;
        g.nsets = nsets;
        for (int k = 0; k < 2; ++k) {
            g.cur[k] = cur[k];
            g.fit[k] = fit[k];
            g.off[k] = off[k];
            g.ok[k] = ok[k];
        }
        g.improved = improved;
        g.draws = draws;
        g.mut = mut;
        g.mut_ok = mut_ok;
        g.mpart = mpart;
        g.mspart = mspart;
        g.TIm = spec_ti;
        // two mutants per wave measured best at G900 (1, 2, 4, 8 tried)
        g.mpw = std::max(1, env_int("PMP_MUTANTS_PER_WAVE", 2));
        g.part = part;
        g.spart = spart;
        g.TI = TI;
        g.gmask = gmask;
        g.gcost = gcost;
        g.best_mask = best;
        g.gs = gs;
        g.cstat = cstat;
        g.arrive = arrive;
        g.bar = bar;
        g.err = inst->err;
        g.swaps = swaps;
        g.rep_t = rep_t;
        g.rep_w = rep_w;
        g.rep_d = rep_d;
        g.L = model ? LL : 0;
        g.H = model ? LH : 1;
        return g;
    }

    LearnArgs learn_args(const GaArgs &g) const
    {
        LearnArgs a{};
        a.g = g;
        a.net = model->d.view();
        a.colsum = inst->colsum;
        a.nearc = inst->nearc;
        a.total = inst->total;
        a.near_len = inst->near_len;
        a.C = LC;
        a.L = LL;
        a.explore = Lexp;
        a.H = LH;
        a.swaps = swaps;
        a.rep_x = rep_x;
        a.rep_jk = rep_jk;
        a.rep_d = rep_d;
        a.rep_t = rep_t;
        a.rep_w = rep_w;
        a.scores = scores;
        a.cand = cand;
        a.cbits = cbits;
        a.cpre = cpre;
        const size_t PS = (size_t)prm.population * kSlots;
        a.sums.a = (uint32_t *)sums;
        a.sums.dd = a.sums.a + PS;
        a.sums.b = (unsigned long long *)(a.sums.dd + PS);
        a.sums.cc = a.sums.b + PS;
        a.sums.e = a.sums.cc + PS;
        a.clients_per_block = cpb;
        a.tiles_i = TI;
        a.walk = walk_shape;
        a.s12 = s12;
        a.c12 = c12;
        a.near_off = near_off;
        a.near_q = near_q;
        return a;
    }

    void free_learned()
    {
        dfree(swaps);
        dfree(rep_x);
        dfree(rep_t);
        dfree(rep_w);
        dfree(rep_jk);
        dfree(rep_d);
        dfree(scores);
        dfree(cand);
        dfree(cbits);
        dfree(cpre);
        if (sums)
            (void)hipFree(sums);
        sums = nullptr;
        dfree(last_trained);
        dfree(s12);
        dfree(c12);
        dfree(near_off);
        dfree(near_q);
    }
};


namespace {

EvalArgs ga_eval_args(const pmp_ga *ga, const GaArgs &g, int buf);

// The batch's client tiling: with clients = 0 every run keeps its own
// tuning (base_cpb), else every run takes `clients` clients per evaluation
// workgroup, or more where its partial-sum buffers (sized for the larger of
// its own and its fused launches' tile counts) hold fewer tiles than that
// gives; the stage steps read the partial sums with the same tiling.
// Uploads the run table and prefix offsets; graphs captured for another
// tiling are dropped.
hipError_t batch_tiles(BatchHost &bh, int clients)
{
    const int count = (int)bh.gas.size();
    int32_t *c0 = bh.prefix.data(), *t0 = c0 + count + 1, *g0 = t0 + count + 1;
    for (int b = 0; b < count; ++b) {
        BatchItem &it = bh.items[b];
        const pmp_ga *ga = bh.gas[b];
        const int n = ga->inst->n, cap = std::max(ga->TI, ga->fTI);
        it.e.clients_per_block =
            clients > 0 ? std::max(clients, (n + cap - 1) / cap) : bh.base_cpb[b];
        it.e.tiles_i = (bh.gas[b]->inst->n + it.e.clients_per_block - 1) / it.e.clients_per_block;
        it.g.TI = it.e.tiles_i;
        t0[b + 1] = t0[b] + it.e.tiles_c * it.e.tiles_i;
    }
    int32_t *tile_run = bh.runs.data() + c0[count] + g0[count];
    for (int b = 0; b < count; ++b)
        for (int x = t0[b]; x < t0[b + 1]; ++x)
            tile_run[x] = b;
    bh.drop_graphs();
    hipError_t e = hipMemcpy(bh.d_items, bh.items.data(), sizeof(BatchItem) * count,
                             hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(bh.d_prefix, bh.prefix.data(), sizeof(int32_t) * bh.prefix.size(),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(bh.d_runs, bh.runs.data(), sizeof(int32_t) * bh.runs.size(),
                      hipMemcpyHostToDevice);
    bh.clients = clients;
    bh.nchrom = c0[count];
    bh.ntiles = t0[count];
    bh.ngroups = g0[count];
    const int waves = (c0[count] + 3) / 4;  // one wave per chromosome, 4 per workgroup
    bh.want = std::max(std::max(t0[count], waves), g0[count]);
    return e;
}

hipError_t batch_build(BatchHost &bh, pmp_ga *const *gas, int count)
{
    bh.gas.assign(gas, gas + count);
    bh.items.assign((size_t)count, BatchItem{});
    bh.prefix.assign(3 * ((size_t)count + 1), 0);
    bh.base_cpb.assign((size_t)count, 0);
    int32_t *c0 = bh.prefix.data(), *g0 = c0 + 2 * (count + 1);
    int max_S = 0, max_w2 = 2;
    for (int b = 0; b < count; ++b) {
        pmp_ga *ga = gas[b];
        BatchItem &it = bh.items[b];
        it.g = ga->args();
        it.e = ga_eval_args(ga, it.g, 0);
        it.e.done = nullptr;
        // The batch evaluation runs 16 waves per workgroup: a tile tuned for
        // fewer waves keeps its clients per wave with proportionally more
        // clients per workgroup (fewer client tiles, so the partial sums
        // still fit).
        const int scale = 16 / std::max(1, std::min(16, ga->waves));
        bh.base_cpb[b] = ga->cpb * scale;
        it.X = ga->xstages();
        it.S = it.X + ga->Y;
        it.fb = ga->final_buf();
        c0[b + 1] = c0[b] + ga->prm.population;
        g0[b + 1] = g0[b] + ga->NB;
        max_S = max_S > it.S ? max_S : it.S;
        max_w2 = max_w2 > 2 * ga->inst->W ? max_w2 : 2 * ga->inst->W;
    }
    // a run's tile count is at most its partial-sum capacity in any tiling
    bh.max_tiles = 0;
    for (int b = 0; b < count; ++b)
        bh.max_tiles += bh.items[b].e.tiles_c * std::max(gas[b]->TI, gas[b]->fTI);
    bh.runs.assign((size_t)c0[count] + g0[count] + bh.max_tiles, 0);
    for (int b = 0; b < count; ++b) {
        for (int x = c0[b]; x < c0[b + 1]; ++x)
            bh.runs[x] = b;
        for (int x = g0[b]; x < g0[b + 1]; ++x)
            bh.runs[c0[count] + x] = b;
    }
    if (dalloc(&bh.d_items, (size_t)count) || dalloc(&bh.d_prefix, bh.prefix.size()) ||
        dalloc(&bh.d_runs, bh.runs.size()) || dalloc(&bh.d_bar, kBarrierWords) ||
        dalloc(&bh.d_err, 1))
        return hipErrorOutOfMemory;
    hipError_t e = hipMemset(bh.d_bar, 0, sizeof(uint32_t) * kBarrierWords);
    if (e == hipSuccess)
        e = hipMemset(bh.d_err, 0, sizeof(uint32_t));
    bh.args.items = bh.d_items;
    bh.args.chrom0 = bh.d_prefix;
    bh.args.tile0 = bh.d_prefix + count + 1;
    bh.args.group0 = bh.d_prefix + 2 * (count + 1);
    bh.args.chrom_run = bh.d_runs;
    bh.args.group_run = bh.d_runs + c0[count];
    bh.args.tile_run = bh.d_runs + c0[count] + g0[count];
    bh.args.count = count;
    bh.args.max_S = max_S;
    bh.args.bar = bh.d_bar;
    bh.args.err = bh.d_err;
    bh.max_w2 = max_w2;
    if (e == hipSuccess)
        e = batch_tiles(bh, env_int("PMP_BATCH_CLIENTS", 0));
    return e;
}

hipError_t batch_launch(BatchHost &bh, int generations, int max_blocks,
                        hipStream_t s, bool cooperative)
{
    return launch_ga_batch(bh.args, generations, bh.max_w2, max_blocks, bh.want, s,
                           &bh.last_grid, cooperative);
}

}  // namespace

struct pmp_batch {
    BatchHost bh;
    bool graphs = true;
    bool persistent = false;  // one persistent kernel instead of per-phase kernels
    int max_blocks = 0;
    // profiling of the evaluation launches (pmp_batch_profile)
    bool prof = false;
    std::vector<hipEvent_t> ev;
    int ev_used = 0;
};

namespace {

// Enqueue `generations` generations of a batch: one persistent kernel, or
// one batch-wide kernel per phase.
hipError_t batch_enqueue(pmp_batch *bt, int generations, hipStream_t s, bool cooperative)
{
    BatchHost &bh = bt->bh;
    if (bt->persistent)
        return batch_launch(bh, generations, bt->max_blocks, s, cooperative);
    BatchEvents ev;
    if (bt->prof) {
        // one pair per evaluation launch: max_S + 1 per generation
        const size_t need = (size_t)bt->ev_used + 2 * (size_t)generations * (bh.args.max_S + 1);
        while (bt->ev.size() < need) {
            hipEvent_t e = nullptr;
            const hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess)
                return r;
            bt->ev.push_back(e);
        }
        ev.events = bt->ev.data();
        ev.cap = (int)bt->ev.size();
        ev.used = &bt->ev_used;
    }
    return launch_ga_batch_kernels(bh.args, bh.nchrom, bh.ntiles, bh.ngroups, generations,
                                   bh.max_w2, s, ev);
}

// Workspace of pmp_eval_population_noalloc: the client-tile partial sums
// (int64 costs, then uint32 scan lengths) of one evaluation, in memory the
// library never allocates at run time.  Each GPU holds its own copy from the
// moment the code object is loaded until the process ends.
constexpr size_t kNoAllocCells = (size_t)PMP_NOALLOC_CELLS;
static __device__ __align__(256) unsigned char scratch[kNoAllocCells * 12];

// Device address of this GPU's copy of `scratch`, taken once per device
// with that device current.  In host code the array's name is only a
// host-side stand-in, never a device address: every kernel argument is
// derived from the address returned here.
constexpr int kMaxDevices = 64;
std::atomic<void *> g_scratch_addr[kMaxDevices];
std::mutex g_scratch_mu;

hipError_t scratch_address(void **out)
{
    *out = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    if (dev < 0 || dev >= kMaxDevices)
        return hipErrorInvalidDevice;
    void *p = g_scratch_addr[dev].load(std::memory_order_acquire);
    if (!p) {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        p = g_scratch_addr[dev].load(std::memory_order_acquire);
        if (!p) {
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess)
                return e;
            if (!p)
                return hipErrorInvalidSymbol;
            g_scratch_addr[dev].store(p, std::memory_order_release);
        }
    }
    *out = p;
    return hipSuccess;
}

}  // namespace

extern "C" {

const char *pmp_status_str(pmp_status s)
{
    switch (s) {
    case PMP_OK: return "ok";
    case PMP_EINVAL: return "invalid argument";
    case PMP_ENOMEM: return "out of memory";
    case PMP_EDEVICE: return "device error";
    case PMP_EINFEASIBLE: return "infeasible chromosome";
    case PMP_EUNSUPPORTED: return "unsupported size";
    }
    return "unknown status";
}

const char *pmp_last_error(void) { return g_last_error.c_str(); }

void pmp_instance_destroy(pmp_instance *inst)
{
    if (!inst)
        return;
    inst->arena.release();
    dfree(inst->h_masks);
    dfree(inst->h_fit);
    dfree(inst->h_scan);
    dfree(inst->part);
    dfree(inst->spart);
    dfree(inst->tg);
    delete inst;
}

pmp_status pmp_preprocess(const int32_t *d, int64_t ld, int32_t n, int32_t m,
                          int32_t p, uint32_t flags, void *stream,
                          pmp_instance **out)
{
    if (!out)
        return fail(PMP_EINVAL, "out is NULL");
    *out = nullptr;
    if (!d)
        return fail(PMP_EINVAL, "d is NULL");
    if (n < 1 || m < 2 || p < 1 || p > m - 1)
        return fail(PMP_EINVAL, "need n >= 1, m >= 2, 1 <= p <= m-1 (n=%d m=%d p=%d)",
                    n, m, p);
    if (m > PMP_MAX_EVAL_FACILITIES)
        return fail(PMP_EINVAL, "m=%d above %d (facility indices are 16-bit)", m,
                    PMP_MAX_EVAL_FACILITIES);
    if (ld < m)
        return fail(PMP_EINVAL, "row stride %lld < m", (long long)ld);
    hipStream_t s = (hipStream_t)stream;
    const bool on_dev = flags & PMP_ON_DEVICE;
    const bool async = flags & PMP_ASYNC;
    if (async && !on_dev)
        return fail(PMP_EINVAL, "PMP_ASYNC needs device input (PMP_ON_DEVICE)");
    if (!on_dev) {
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = 0; j < m; ++j)
                if (d[i * ld + j] < 0)
                    return fail(PMP_EINVAL, "d[%lld][%lld] < 0", (long long)i,
                                (long long)j);
    }
    pmp_instance *inst = new pmp_instance;
    inst->n = n;
    inst->m = m;
    inst->p = p;
    inst->K = m - p + 1;
    inst->W = (m + 63) / 64;
    inst->pitch = ((inst->K + 63) / 64) * 64;
    const size_t cells = (size_t)n * inst->pitch;
    inst->near_len = (m + p - 1) / p;
    inst->arena.add(&inst->pi, cells);
    inst->arena.add(&inst->ds, cells);
    inst->arena.add(&inst->delta, cells);
    inst->arena.add(&inst->err, 1);
    inst->arena.add(&inst->colsum, (size_t)m);
    inst->arena.add(&inst->nearc, (size_t)m);
    inst->arena.add(&inst->dtotal, 2);
    if (inst->arena.carve() != hipSuccess) {
        pmp_instance_destroy(inst);
        return fail(PMP_ENOMEM, "device allocation of tables (%zu cells)", cells);
    }
    int32_t *dd = nullptr;
    uint64_t *wide = nullptr;  // sort scratch of rows wider than PMP_MAX_FACILITIES
    const int32_t *src = d;
    int64_t src_ld = ld;
    pmp_status st = PMP_OK;
    do {
        hipError_t e = hipMemsetAsync(inst->err, 0, sizeof(uint32_t), s);
        if (e != hipSuccess) {
            st = fail(PMP_EDEVICE, "hipMemsetAsync: %s", hipGetErrorString(e));
            break;
        }
        if (!on_dev) {
            if (dalloc(&dd, (size_t)n * m) != hipSuccess) {
                st = fail(PMP_ENOMEM, "device copy of d");
                break;
            }
            e = hipMemcpy2DAsync(dd, sizeof(int32_t) * m, d, sizeof(int32_t) * ld,
                                 sizeof(int32_t) * m, n, hipMemcpyHostToDevice, s);
            if (e != hipSuccess) {
                st = fail(PMP_EDEVICE, "copy of d: %s", hipGetErrorString(e));
                break;
            }
            src = dd;
            src_ld = m;
        }
        if (m <= PMP_MAX_FACILITIES) {
            e = launch_sort_rows(src, src_ld, n, m, inst->K, inst->pitch, inst->pi,
                                 inst->delta, inst->ds, inst->err, s);
        } else {  // rows wider than one workgroup's LDS: the sort in device memory
            int32_t m2 = 2;
            while (m2 < m)
                m2 <<= 1;
            const int batch = std::min(n, wide_sort_rows_per_batch(m));
            if (dalloc(&wide, (size_t)batch * m2) != hipSuccess) {
                st = fail(PMP_ENOMEM, "sort scratch (%d rows x %d keys)", batch, m2);
                break;
            }
            e = launch_sort_rows_wide(src, src_ld, n, m, inst->K, inst->pitch, inst->pi,
                                      inst->delta, inst->ds, inst->err, wide, batch, s);
        }
        if (e != hipSuccess) {
            st = fail(PMP_EDEVICE, "sort kernel launch: %s", hipGetErrorString(e));
            break;
        }
        // static sums of the learned proposal's features; the sum of d and
        // the error word come back in one copy
        e = hipMemsetAsync(inst->colsum, 0, sizeof(unsigned long long) * m, s);
        if (e == hipSuccess)
            e = hipMemsetAsync(inst->nearc, 0, sizeof(uint32_t) * m, s);
        if (e == hipSuccess)
            e = launch_static_sums(src, src_ld, n, m, inst->pi, inst->pitch, inst->near_len,
                                   inst->colsum, inst->nearc, inst->err, inst->dtotal, s);
        if (e == hipSuccess && async) {  // the error word stays for pmp_instance_check
            inst->total_pending = true;
            break;
        }
        std::vector<unsigned long long> rb;
        if (e == hipSuccess)
            e = staging().read(inst->dtotal, 2, s, rb);
        if (e != hipSuccess) {
            st = fail(PMP_EDEVICE, "preprocess: %s", hipGetErrorString(e));
            break;
        }
        inst->total = (int64_t)rb[0];
        st = status_from_err((uint32_t)rb[1]);
    } while (0);
    dfree(dd);
    dfree(wide);
    if (st != PMP_OK) {
        pmp_instance_destroy(inst);
        return st;
    }
    *out = inst;
    return PMP_OK;
}

pmp_status pmp_instance_info(const pmp_instance *inst, int32_t *n, int32_t *m,
                             int32_t *p, int32_t *K, int32_t *W)
{
    if (!inst)
        return fail(PMP_EINVAL, "instance is NULL");
    if (n) *n = inst->n;
    if (m) *m = inst->m;
    if (p) *p = inst->p;
    if (K) *K = inst->K;
    if (W) *W = inst->W;
    return PMP_OK;
}

pmp_status pmp_instance_tables(const pmp_instance *inst, uint16_t *pi,
                               int32_t *delta, int32_t *dsorted,
                               uint32_t flags, void *stream)
{
    if (!inst)
        return fail(PMP_EINVAL, "instance is NULL");
    hipStream_t s = (hipStream_t)stream;
    const hipMemcpyKind kind = (flags & PMP_ON_DEVICE) ? hipMemcpyDeviceToDevice
                                                        : hipMemcpyDeviceToHost;
    const size_t K = inst->K, pitch = inst->pitch, n = inst->n;
    if (pi)
        HIP_TRY(hipMemcpy2DAsync(pi, K * 2, inst->pi, pitch * 2, K * 2, n, kind, s));
    if (delta)
        HIP_TRY(hipMemcpy2DAsync(delta, K * 4, inst->delta, pitch * 4, K * 4, n, kind, s));
    if (dsorted)
        HIP_TRY(hipMemcpy2DAsync(dsorted, K * 4, inst->ds, pitch * 4, K * 4, n, kind, s));
    if (!(flags & PMP_ON_DEVICE) || !(flags & PMP_ASYNC))
        HIP_TRY(hipStreamSynchronize(s));
    return PMP_OK;
}

// ---------------------------------------------------------------------------
// The reduced polynomial (k_hbp.hip): construction and evaluation.
// ---------------------------------------------------------------------------
struct pmp_hbp {
    pmp_instance *inst = nullptr;
    long long c0 = 0;
    int32_t terms = 0, rows = 0, maxlen = 0, rpitch = 0, kept = 0;
    uint16_t *rpi = nullptr;
    long long *re = nullptr;
    int32_t *rlen = nullptr, *rlen_full = nullptr;
    int32_t *term_row = nullptr, *term_deg = nullptr;
    long long *term_coef = nullptr;
    unsigned long long *part = nullptr, *h_fit = nullptr, *h_scan = nullptr;
    uint32_t *spart = nullptr;
    uint64_t *h_masks = nullptr;
    size_t part_cap = 0;
    int32_t h_cap = 0;
    ~pmp_hbp()
    {
        dfree(rpi);
        dfree(re);
        dfree(rlen);
        dfree(rlen_full);
        dfree(term_row);
        dfree(term_deg);
        dfree(term_coef);
        dfree(part);
        dfree(spart);
        dfree(h_fit);
        dfree(h_scan);
        dfree(h_masks);
    }
};

// Temporaries of one construction, freed on every return.
struct HbpScratch {
    HbpArgs h{};
    ~HbpScratch()
    {
        dfree(h.key);
        dfree(h.slot_of);
        dfree(h.posinv);
        dfree(h.slot_key);
        dfree(h.slot_row);
        dfree(h.slot_tmin);
        dfree(h.slot_tmax);
        dfree(h.slot_sum);
        dfree(h.charged);
        dfree(h.esum);
        dfree(h.owned);
        dfree(h.maxlen);
        dfree(h.kept_at);
        dfree(h.term_at);
        dfree(h.tot);
        dfree(h.npos);
        dfree(h.c0);
        dfree(h.err);
    }
};

pmp_status pmp_hbp_reduce(pmp_instance *inst, void *stream, pmp_hbp **out)
{
    if (inst && inst->m > PMP_MAX_FACILITIES)
        return fail(PMP_EUNSUPPORTED, "the reduced polynomial takes m <= %d", PMP_MAX_FACILITIES);
    if (!inst || !out)
        return fail(PMP_EINVAL, "instance or out is NULL");
    *out = nullptr;
    hipStream_t s = (hipStream_t)stream;
    const int n = inst->n, m = inst->m;
    const size_t cells = (size_t)n * inst->pitch;
    HbpScratch sc;
    HbpArgs &h = sc.h;
    h.t = inst->tables();
    bool bad = dalloc(&h.key, cells) || dalloc(&h.npos, 1) || dalloc(&h.c0, 1) ||
               dalloc(&h.err, 1);
    if (bad)
        return fail(PMP_ENOMEM, "reduced polynomial keys (n=%d)", n);
    HIP_TRY(hipMemsetAsync(h.npos, 0, sizeof(unsigned long long), s));
    HIP_TRY(hipMemsetAsync(h.c0, 0, sizeof(unsigned long long), s));
    HIP_TRY(hipMemsetAsync(h.err, 0, sizeof(uint32_t), s));
    HIP_TRY(launch_hbp_keys(h, s));
    unsigned long long npos = 0;
    HIP_TRY(hipMemcpyAsync(&npos, h.npos, sizeof npos, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    // table of at least twice the positive terms (load factor <= 1/2)
    uint64_t cap = 64;
    while (cap < 2 * npos)
        cap <<= 1;
    h.mask = cap - 1;
    bad = dalloc(&h.slot_of, cells) || dalloc(&h.posinv, (size_t)n * m) ||
          dalloc(&h.slot_key, cap) || dalloc(&h.slot_row, cap) || dalloc(&h.slot_tmin, cap) ||
          dalloc(&h.slot_tmax, cap) || dalloc(&h.slot_sum, cap) || dalloc(&h.charged, cells) ||
          dalloc(&h.esum, cells) || dalloc(&h.owned, (size_t)n) || dalloc(&h.maxlen, 1) ||
          dalloc(&h.kept_at, (size_t)n) || dalloc(&h.term_at, (size_t)n) || dalloc(&h.tot, 2);
    if (bad)
        return fail(PMP_ENOMEM, "reduced polynomial table (%llu slots)", (unsigned long long)cap);
    pmp_hbp *r = new pmp_hbp;
    std::unique_ptr<pmp_hbp> guard(r);
    r->inst = inst;
    if (dalloc(&r->rlen_full, (size_t)n))
        return fail(PMP_ENOMEM, "reduced polynomial rows");
    h.rlen_full = r->rlen_full;
    HIP_TRY(hipMemsetAsync(h.posinv, 0xFF, sizeof(uint16_t) * (size_t)n * m, s));
    HIP_TRY(hipMemsetAsync(h.slot_of, 0, sizeof(int32_t) * cells, s));
    HIP_TRY(hipMemsetAsync(h.slot_key, 0, sizeof(uint64_t) * cap, s));
    HIP_TRY(hipMemsetAsync(h.slot_row, 0x7F, sizeof(int32_t) * cap, s));
    HIP_TRY(hipMemsetAsync(h.slot_tmin, 0x7F, sizeof(int32_t) * cap, s));
    HIP_TRY(hipMemsetAsync(h.slot_tmax, 0, sizeof(int32_t) * cap, s));
    HIP_TRY(hipMemsetAsync(h.slot_sum, 0, sizeof(unsigned long long) * cap, s));
    HIP_TRY(hipMemsetAsync(h.maxlen, 0, sizeof(int32_t), s));
    HIP_TRY(launch_hbp_table(h, s));
    int32_t tot[2] = {0, 0}, maxlen = 0;
    uint32_t err = 0;
    unsigned long long c0 = 0;
    HIP_TRY(hipMemcpyAsync(tot, h.tot, sizeof tot, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&maxlen, h.maxlen, sizeof maxlen, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&err, h.err, sizeof err, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&c0, h.c0, sizeof c0, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (err & (ERR_HASH_TABLE | ERR_HASH_COLLISION))
        return fail(PMP_EUNSUPPORTED, "reduced polynomial: set keys collided (error bits 0x%x)",
                    err);
    r->c0 = (long long)c0;
    r->kept = tot[0];
    r->terms = tot[1];
    // an instance whose rows all reduce to constants keeps one dummy row
    // (length 1, value 0) so that the evaluation still checks feasibility
    r->rows = std::max(1, tot[0]);
    r->maxlen = std::max(1, maxlen);
    r->rpitch = ((r->maxlen + 63) / 64) * 64;
    const size_t rcells = (size_t)r->rows * r->rpitch;
    bad = dalloc(&r->rpi, rcells) || dalloc(&r->re, rcells) || dalloc(&r->rlen, (size_t)r->rows) ||
          dalloc(&r->term_row, (size_t)r->terms) || dalloc(&r->term_deg, (size_t)r->terms) ||
          dalloc(&r->term_coef, (size_t)r->terms);
    if (bad)
        return fail(PMP_ENOMEM, "reduced polynomial walk tables (%d rows)", r->rows);
    if (tot[0] == 0) {
        const int32_t one = 1;
        HIP_TRY(hipMemsetAsync(r->rpi, 0, sizeof(uint16_t) * rcells, s));
        HIP_TRY(hipMemsetAsync(r->re, 0, sizeof(long long) * rcells, s));
        HIP_TRY(hipMemcpyAsync(r->rlen, &one, sizeof one, hipMemcpyHostToDevice, s));
    }
    h.rpi = r->rpi;
    h.re = r->re;
    h.rlen = r->rlen;
    h.rpitch = r->rpitch;
    h.term_row = r->term_row;
    h.term_deg = r->term_deg;
    h.term_coef = r->term_coef;
    HIP_TRY(launch_hbp_emit(h, s));
    HIP_TRY(hipStreamSynchronize(s));
    *out = guard.release();
    return PMP_OK;
}

pmp_status pmp_hbp_info(const pmp_hbp *hp, int64_t *constant, int64_t *monomials,
                        int32_t *rows, int32_t *max_len)
{
    if (!hp)
        return fail(PMP_EINVAL, "handle is NULL");
    if (constant)
        *constant = hp->c0;
    if (monomials)
        *monomials = hp->terms;
    if (rows)
        *rows = hp->kept;
    if (max_len)
        *max_len = hp->kept ? hp->maxlen : 0;
    return PMP_OK;
}

pmp_status pmp_hbp_terms(const pmp_hbp *hp, int32_t *row, int32_t *degree, int64_t *coef,
                         int32_t *row_len, uint32_t flags, void *stream)
{
    if (!hp)
        return fail(PMP_EINVAL, "handle is NULL");
    hipStream_t s = (hipStream_t)stream;
    const hipMemcpyKind kind =
        (flags & PMP_ON_DEVICE) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    const size_t T = (size_t)hp->terms;
    if (row && T)
        HIP_TRY(hipMemcpyAsync(row, hp->term_row, sizeof(int32_t) * T, kind, s));
    if (degree && T)
        HIP_TRY(hipMemcpyAsync(degree, hp->term_deg, sizeof(int32_t) * T, kind, s));
    if (coef && T)
        HIP_TRY(hipMemcpyAsync(coef, hp->term_coef, sizeof(int64_t) * T, kind, s));
    if (row_len)
        HIP_TRY(hipMemcpyAsync(row_len, hp->rlen_full, sizeof(int32_t) * hp->inst->n, kind, s));
    HIP_TRY(hipStreamSynchronize(s));
    return PMP_OK;
}

pmp_status pmp_hbp_eval(pmp_hbp *hp, const uint64_t *masks, int32_t P, int64_t *fitness,
                        int64_t *scan_total, uint32_t flags, void *stream)
{
    if (!hp)
        return fail(PMP_EINVAL, "handle is NULL");
    if (P < 0)
        return fail(PMP_EINVAL, "P < 0");
    if (P == 0)
        return PMP_OK;
    if (!masks || !fitness)
        return fail(PMP_EINVAL, "masks or fitness is NULL");
    pmp_instance *inst = hp->inst;
    hipStream_t s = (hipStream_t)stream;
    const bool on_dev = flags & PMP_ON_DEVICE;
    const bool async = on_dev && (flags & PMP_ASYNC);
    const size_t W = inst->W;
    const uint64_t *dmask = masks;
    unsigned long long *dfit = (unsigned long long *)fitness;
    unsigned long long *dscan = (unsigned long long *)scan_total;
    if (!on_dev) {
        if (hp->h_cap < P) {
            dfree(hp->h_masks);
            dfree(hp->h_fit);
            dfree(hp->h_scan);
            hp->h_cap = 0;
            if (dalloc(&hp->h_masks, (size_t)P * W) || dalloc(&hp->h_fit, (size_t)P) ||
                dalloc(&hp->h_scan, (size_t)P))
                return fail(PMP_ENOMEM, "staging for P=%d", P);
            hp->h_cap = P;
        }
        HIP_TRY(hipMemcpyAsync(hp->h_masks, masks, sizeof(uint64_t) * P * W,
                               hipMemcpyHostToDevice, s));
        dmask = hp->h_masks;
        dfit = hp->h_fit;
        dscan = scan_total ? hp->h_scan : nullptr;
    }
    if (!async)
        HIP_TRY(launch_zero(inst->err, sizeof(uint32_t), s));
    EvalArgs a{};
    a.t = inst->tables();
    a.t.pi = hp->rpi;
    a.t.ds = nullptr;
    a.t.n = hp->rows;
    a.t.K = hp->maxlen;
    a.t.pitch = hp->rpitch;
    a.rlen = hp->rlen;
    a.e64 = hp->re;
    a.c0 = hp->c0;
    a.masks = dmask;
    a.P = P;
    a.err = inst->err;
    a.clients_per_block = clients_per_block(hp->rows, P, inst->m, inst->p, inst->W, true);
    a.tiles_c = (P + kEvalTile - 1) / kEvalTile;
    a.tiles_i = (hp->rows + a.clients_per_block - 1) / a.clients_per_block;
    const size_t cells = (size_t)a.tiles_i * P;
    if (hp->part_cap < cells) {
        dfree(hp->part);
        dfree(hp->spart);
        hp->part_cap = 0;
        if (dalloc(&hp->part, cells) || dalloc(&hp->spart, cells))
            return fail(PMP_ENOMEM, "evaluation workspace (%zu cells)", cells);
        hp->part_cap = cells;
    }
    a.part = hp->part;
    a.spart = dscan ? hp->spart : nullptr;
    HIP_TRY(launch_eval(a, s));
    HIP_TRY(launch_reduce(a, dfit, dscan, s));
    if (!on_dev) {
        HIP_TRY(hipMemcpyAsync(fitness, dfit, sizeof(int64_t) * P, hipMemcpyDeviceToHost, s));
        if (scan_total)
            HIP_TRY(hipMemcpyAsync(scan_total, dscan, sizeof(int64_t) * P,
                                   hipMemcpyDeviceToHost, s));
    }
    if (async)
        return PMP_OK;
    uint32_t herr = 0;
    HIP_TRY(hipMemcpyAsync(&herr, inst->err, sizeof herr, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return status_from_err(herr);
}

void pmp_hbp_destroy(pmp_hbp *hp)
{
    delete hp;
}

// Work buffers of pmp_apsp, kept per device and grown on demand (a call
// would otherwise pay for allocating and freeing an n x n matrix); calls are
// serialised by the mutex.  Held until the process ends.
struct ApspCache {
    std::mutex mu;
    struct Dev {
        uint32_t *work = nullptr, *wmax = nullptr;
        int32_t *w = nullptr, *d = nullptr;  // staging for host arguments
        size_t work_cap = 0, stage_cap = 0;
    };
    std::map<int, Dev> dev;
};

ApspCache &apsp_cache()
{
    static ApspCache *c = new ApspCache;  // never destroyed: outlives the runtime
    return *c;
}

pmp_status pmp_apsp(const int32_t *w, int64_t ldw, int32_t n, int32_t *d, int64_t ldd,
                    uint32_t flags, void *stream)
{
    if (!w || !d)
        return fail(PMP_EINVAL, "w or d is NULL");
    if (n < 1 || n > 32768 || ldw < n || ldd < n)
        return fail(PMP_EINVAL, "need 1 <= n <= 32768 and strides >= n (n=%d ldw=%lld ldd=%lld)",
                    n, (long long)ldw, (long long)ldd);
    hipStream_t s = (hipStream_t)stream;
    const bool on_dev = flags & PMP_ON_DEVICE;
    const int ld = apsp_padded(n);
    int device = 0;
    HIP_TRY(hipGetDevice(&device));
    ApspCache &cache = apsp_cache();
    std::lock_guard<std::mutex> lock(cache.mu);
    ApspCache::Dev &b = cache.dev[device];
    const size_t cells = (size_t)ld * ld;
    if (b.work_cap < cells) {
        dfree(b.work);
        b.work_cap = 0;
        if (dalloc(&b.work, cells) != hipSuccess)
            return fail(PMP_ENOMEM, "APSP work matrix (%d x %d)", ld, ld);
        b.work_cap = cells;
    }
    if (!b.wmax && dalloc(&b.wmax, 1) != hipSuccess)
        return fail(PMP_ENOMEM, "APSP word");
    const int32_t *dw = w;
    int32_t *dd = d;
    int64_t ldw_dev = ldw, ldd_dev = ldd;
    if (!on_dev) {
        const size_t nn = (size_t)n * n;
        if (b.stage_cap < nn) {
            dfree(b.w);
            dfree(b.d);
            b.stage_cap = 0;
            if (dalloc(&b.w, nn) != hipSuccess || dalloc(&b.d, nn) != hipSuccess)
                return fail(PMP_ENOMEM, "APSP staging (n=%d)", n);
            b.stage_cap = nn;
        }
        HIP_TRY(hipMemcpy2DAsync(b.w, (size_t)n * 4, w, (size_t)ldw * 4, (size_t)n * 4, n,
                                 hipMemcpyHostToDevice, s));
        dw = b.w;
        dd = b.d;
        ldw_dev = ldd_dev = n;
    }
    HIP_TRY(launch_zero(b.wmax, sizeof(uint32_t), s));
    HIP_TRY(launch_apsp_in(dw, ldw_dev, n, b.work, b.wmax, s));
    uint32_t wmax = 0;
    HIP_TRY(hipMemcpyAsync(&wmax, b.wmax, sizeof wmax, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if ((int64_t)(n - 1) * (int64_t)wmax >= 0x7FFFFFFFll)
        return fail(PMP_EUNSUPPORTED, "path lengths may exceed int32: (n-1) * max weight = %lld",
                    (long long)(n - 1) * (long long)wmax);
    HIP_TRY(launch_apsp_rounds(b.work, n, s));
    HIP_TRY(launch_apsp_out(b.work, n, dd, ldd_dev, s));
    if (!on_dev)
        HIP_TRY(hipMemcpy2DAsync(d, (size_t)ldd * 4, b.d, (size_t)n * 4, (size_t)n * 4, n,
                                 hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return PMP_OK;
}

pmp_status pmp_instance_check(pmp_instance *inst, void *stream)
{
    if (!inst)
        return fail(PMP_EINVAL, "instance is NULL");
    hipStream_t s = (hipStream_t)stream;
    uint32_t herr = 0;
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipMemcpy(&herr, inst->err, sizeof herr, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemset(inst->err, 0, sizeof herr));
    return status_from_err(herr);
}

pmp_status pmp_eval_population(pmp_instance *inst, const uint64_t *masks,
                               int32_t P, int64_t *fitness,
                               int64_t *scan_total, uint32_t flags,
                               void *stream)
{
    if (!inst)
        return fail(PMP_EINVAL, "instance is NULL");
    if (P < 0)
        return fail(PMP_EINVAL, "P < 0");
    if (P == 0)
        return PMP_OK;
    if (!masks || !fitness)
        return fail(PMP_EINVAL, "masks or fitness is NULL");
    const uint32_t scheme = flags & (PMP_EVAL_PER_CHROMOSOME | PMP_EVAL_PER_CLIENT);
    if (scheme == (PMP_EVAL_PER_CHROMOSOME | PMP_EVAL_PER_CLIENT))
        return fail(PMP_EINVAL, "at most one evaluation scheme flag");
    const bool wide = inst->W > kMaxStagedWords;
    if (scheme && wide)
        return fail(PMP_EUNSUPPORTED, "the per-chromosome and per-client schemes take m <= %d",
                    PMP_MAX_FACILITIES);
    hipStream_t s = (hipStream_t)stream;
    const bool on_dev = flags & PMP_ON_DEVICE;
    const bool async = on_dev && (flags & PMP_ASYNC);
    const size_t W = inst->W;

    const uint64_t *dmask = masks;
    unsigned long long *dfit = (unsigned long long *)fitness;
    unsigned long long *dscan = (unsigned long long *)scan_total;
    if (!on_dev) {
        if (inst->h_cap < P) {
            dfree(inst->h_masks);
            dfree(inst->h_fit);
            dfree(inst->h_scan);
            inst->h_cap = 0;
            if (dalloc(&inst->h_masks, (size_t)P * W) != hipSuccess ||
                dalloc(&inst->h_fit, (size_t)P) != hipSuccess ||
                dalloc(&inst->h_scan, (size_t)P) != hipSuccess)
                return fail(PMP_ENOMEM, "staging for P=%d", P);
            inst->h_cap = P;
        }
        HIP_TRY(hipMemcpyAsync(inst->h_masks, masks, sizeof(uint64_t) * P * W,
                               hipMemcpyHostToDevice, s));
        dmask = inst->h_masks;
        dfit = inst->h_fit;
        dscan = scan_total ? inst->h_scan : nullptr;
    }
    if (!async)
        HIP_TRY(launch_zero(inst->err, sizeof(uint32_t), s));

    EvalArgs a{};
    a.t = inst->tables();
    a.paired = paired_scans(inst->m, inst->p);
    a.masks = dmask;
    a.P = P;
    a.active = nullptr;
    a.done = nullptr;
    a.err = inst->err;
    // (wide chromosomes take the device-memory tile walk, 16 waves only)
    a.waves = wide ? 16 : eval_waves(inst->n, P, inst->m, inst->p, inst->W);
    a.clients_per_block = clients_per_block(inst->n, P, inst->m, inst->p, inst->W, false, a.waves);
    // a tile's summed scan lengths are kept in 32 bits
    const int64_t cpb_scan = ((1ll << 32) - 1) / inst->K;
    if (dscan && (int64_t)a.clients_per_block > cpb_scan)
        a.clients_per_block = (int32_t)cpb_scan;
    a.tiles_c = (P + kEvalTile - 1) / kEvalTile;
    a.tiles_i = (inst->n + a.clients_per_block - 1) / a.clients_per_block;
    if (scheme == PMP_EVAL_PER_CLIENT)
        a.tiles_i = 4 * ((inst->n + 255) / 256);  // one partial per wave of 64 clients
    const size_t cells = (size_t)a.tiles_i * P;
    if (inst->part_cap < cells) {
        dfree(inst->part);
        dfree(inst->spart);
        inst->part_cap = 0;
        if (dalloc(&inst->part, cells) != hipSuccess ||
            dalloc(&inst->spart, cells) != hipSuccess)
            return fail(PMP_ENOMEM, "evaluation workspace (%zu cells)", cells);
        inst->part_cap = cells;
    }
    a.part = inst->part;
    a.spart = dscan ? inst->spart : nullptr;
    if (wide) {
        // chromosomes too wide to stage in LDS: their tiles' facility-major
        // copies in device memory (made and checked first), the single walk
        a.paired = 0;
        a.tg_stride = 64 * (int64_t)inst->W + 2;
        const size_t tg_words = (size_t)a.tiles_c * (size_t)a.tg_stride;
        if (inst->tg_cap < tg_words) {
            dfree(inst->tg);
            inst->tg_cap = 0;
            if (dalloc(&inst->tg, tg_words) != hipSuccess)
                return fail(PMP_ENOMEM, "facility-major tiles (%zu words)", tg_words);
            inst->tg_cap = tg_words;
        }
        a.tg = inst->tg;
        HIP_TRY(launch_tile_major(a, inst->tg, s));
    }
    if (scheme == PMP_EVAL_PER_CHROMOSOME) {
        HIP_TRY(launch_eval_per_chromosome(a, dfit, dscan, s));
    } else {
        HIP_TRY(scheme == PMP_EVAL_PER_CLIENT ? launch_eval_per_client(a, s) : launch_eval(a, s));
        HIP_TRY(launch_reduce(a, dfit, dscan, s));
    }

    if (!on_dev) {
        HIP_TRY(hipMemcpyAsync(fitness, dfit, sizeof(int64_t) * P,
                               hipMemcpyDeviceToHost, s));
        if (scan_total)
            HIP_TRY(hipMemcpyAsync(scan_total, dscan, sizeof(int64_t) * P,
                                   hipMemcpyDeviceToHost, s));
    }
    if (async)
        return PMP_OK;
    uint32_t herr = 0;
    HIP_TRY(hipMemcpyAsync(&herr, inst->err, sizeof herr, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return status_from_err(herr);
}

pmp_status pmp_eval_population_noalloc(pmp_instance *inst, const uint64_t *masks,
                                       int32_t P, int64_t *fitness,
                                       int64_t *scan_total, uint32_t flags,
                                       void *stream)
{
    if (!inst)
        return fail(PMP_EINVAL, "instance is NULL");
    if (!(flags & PMP_ON_DEVICE))
        return fail(PMP_EINVAL, "pmp_eval_population_noalloc takes device pointers only "
                                "(PMP_ON_DEVICE): host buffers would need staging memory");
    if (flags & (PMP_EVAL_PER_CHROMOSOME | PMP_EVAL_PER_CLIENT))
        return fail(PMP_EINVAL, "pmp_eval_population_noalloc runs the tiled scheme only");
    if (inst->W > kMaxStagedWords)
        return fail(PMP_EUNSUPPORTED, "pmp_eval_population_noalloc takes m <= %d",
                    PMP_MAX_FACILITIES);
    if (P < 0)
        return fail(PMP_EINVAL, "P < 0");
    if ((size_t)P > kNoAllocCells)
        return fail(PMP_EINVAL, "P = %d exceeds the no-allocation workspace (%zu chromosomes)",
                    P, kNoAllocCells);
    if (P == 0)
        return PMP_OK;
    if (!masks || !fitness)
        return fail(PMP_EINVAL, "masks or fitness is NULL");
    hipStream_t s = (hipStream_t)stream;
    const bool async = flags & PMP_ASYNC;
    void *ws = nullptr;
    HIP_TRY(scratch_address(&ws));

    EvalArgs a{};
    a.t = inst->tables();
    a.paired = paired_scans(inst->m, inst->p);
    a.masks = masks;
    a.P = P;
    a.active = nullptr;
    a.done = nullptr;
    a.err = inst->err;
    a.tiles_c = (P + kEvalTile - 1) / kEvalTile;
    a.waves = eval_waves(inst->n, P, inst->m, inst->p, inst->W);
    int64_t cpb = clients_per_block(inst->n, P, inst->m, inst->p, inst->W, false, a.waves);
    int64_t ti = ((int64_t)inst->n + cpb - 1) / cpb;
    const int64_t ti_max = (int64_t)(kNoAllocCells / (size_t)P);  // >= 1
    if (ti > ti_max) {  // wider client tiles, so that ti x P cells fit
        cpb = ((int64_t)inst->n + ti_max - 1) / ti_max;
        ti = ((int64_t)inst->n + cpb - 1) / cpb;
    }
    // a tile's summed scan lengths are kept in 32 bits
    if (scan_total && cpb * (int64_t)inst->K >= (1ll << 32))
        return fail(PMP_EUNSUPPORTED, "scan sums of %lld-client tiles may pass 2^32",
                    (long long)cpb);
    a.clients_per_block = (int32_t)cpb;
    a.tiles_i = (int32_t)ti;
    a.part = (unsigned long long *)ws;
    a.spart = scan_total ? (uint32_t *)((unsigned char *)ws + kNoAllocCells * 8) : nullptr;
    if (!async)
        HIP_TRY(launch_zero(inst->err, sizeof(uint32_t), s));
    HIP_TRY(launch_eval(a, s));
    HIP_TRY(launch_reduce(a, (unsigned long long *)fitness, (unsigned long long *)scan_total,
                          s));
    if (async)
        return PMP_OK;
    uint32_t herr = 0;
    HIP_TRY(hipMemcpyAsync(&herr, inst->err, sizeof herr, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return status_from_err(herr);
}

void pmp_ga_destroy(pmp_ga *ga)
{
    if (!ga)
        return;
    ga->arena.release();  // (clears its members: the frees below skip them)
    ga->parts.release();
    for (int k = 0; k < 2; ++k) {
        dfree(ga->cur[k]);
        dfree(ga->off[k]);
        dfree(ga->fit[k]);
        dfree(ga->ok[k]);
    }
    dfree(ga->improved);
    dfree(ga->binom);
    dfree(ga->draws);
    dfree(ga->mut);
    dfree(ga->mut_ok);
    dfree(ga->mpart);
    dfree(ga->mspart);
    dfree(ga->gmask);
    dfree(ga->best);
    dfree(ga->gcost);
    dfree(ga->gs);
    dfree(ga->cstat);
    dfree(ga->arrive);
    dfree(ga->bar);
    dfree(ga->report);
    ga->free_learned();
    if (ga->self) {
        ga->self->release();
        delete ga->self;
    }
    if (ga->gexec)
        (void)hipGraphExecDestroy(ga->gexec);
    for (hipEvent_t e : ga->ev)
        (void)hipEventDestroy(e);
    delete ga;
}

pmp_status pmp_ga_create(pmp_instance *inst, const pmp_ga_params *prm,
                         pmp_ga **out)
{
    if (!out)
        return fail(PMP_EINVAL, "out is NULL");
    *out = nullptr;
    if (!inst || !prm)
        return fail(PMP_EINVAL, "instance or params is NULL");
    const int P = prm->population, NT = prm->group_size;
    if (P < 1 || NT < 1 || NT > 1024 || (NT & (NT - 1)) || P % NT)
        return fail(PMP_EINVAL,
                    "population %d must be a multiple of a power-of-two group size %d <= 1024",
                    P, NT);
    if (prm->generations < 1 || prm->saturation < 0 || prm->crossover_iters < 0 ||
        prm->mutation_iters < 0 ||
        (prm->migration != PMP_MIG_SAME_BLOCK && prm->migration != PMP_MIG_ONE_BLOCK) ||
        (prm->init != PMP_INIT_SUBSET && prm->init != PMP_INIT_RANK))
        return fail(PMP_EINVAL, "bad GA parameters");
    if (inst->m > PMP_MAX_FACILITIES)
        return fail(PMP_EUNSUPPORTED, "GA runs take m <= %d (the instance has m = %d)",
                    PMP_MAX_FACILITIES, inst->m);
    std::vector<unsigned long long> binom;
    const unsigned long long nsets =
        prm->init == PMP_INIT_RANK ? binomial_table(inst->m, inst->p, binom) : 0ull;
    if (prm->init == PMP_INIT_RANK && nsets >= kBinomSat)
        return fail(PMP_EUNSUPPORTED, "C(%d, %d) is too large to draw ranks from", inst->m,
                    inst->p);
    pmp_ga *ga = new pmp_ga;
    ga->inst = inst;
    ga->prm = *prm;
    ga->NB = P / NT;
    int lg = 0;
    while ((1 << (lg + 1)) <= NT)
        ++lg;
    ga->lg = lg;
    ga->X = prm->crossover_iters > 0 ? prm->crossover_iters : lg;
    ga->Y = prm->mutation_iters > 0 ? prm->mutation_iters : lg;
    ga->waves = eval_waves(inst->n, P, inst->m, inst->p, inst->W);
    ga->spec_waves = ga->waves;
    ga->fused = env_int("PMP_GA_FUSED", 1) != 0 && ga_stage_eval_fits(inst->W);
    ga->cpb = clients_per_block(inst->n, P, inst->m, inst->p, inst->W, false, ga->waves);
    ga->TI = (inst->n + ga->cpb - 1) / ga->cpb;
    ga->fcpb = fused_clients_per_block(inst->n, P);
    ga->fTI = (inst->n + ga->fcpb - 1) / ga->fcpb;
    const size_t W = inst->W, PW = (size_t)P * W;
    for (int k = 0; k < 2; ++k) {
        ga->arena.add(&ga->cur[k], PW);
        ga->arena.add(&ga->off[k], PW);
        ga->arena.add(&ga->fit[k], (size_t)P);
        ga->arena.add(&ga->ok[k], (size_t)P);
    }
    ga->arena.add(&ga->improved, (size_t)P);
    ga->arena.add(&ga->draws, (size_t)P * std::max(1, ga->X + ga->Y));
    ga->arena.add(&ga->gmask, (size_t)ga->NB * W);
    ga->arena.add(&ga->best, W);
    ga->arena.add(&ga->gcost, (size_t)ga->NB);
    ga->arena.add(&ga->gs, GS_COUNT);
    ga->arena.add(&ga->cstat, (size_t)P * CS_COUNT);
    ga->arena.add(&ga->arrive, 1);
    ga->arena.add(&ga->bar, kBarrierWords);
    ga->arena.add(&ga->report, (size_t)RP_MASK + W);
    if (!binom.empty())
        ga->arena.add(&ga->binom, binom.size());
    const bool bad = ga->arena.carve() != hipSuccess ||
                     ga->carve_parts(std::max(ga->TI, ga->fTI)) != hipSuccess;
    if (bad) {
        pmp_ga_destroy(ga);
        return fail(PMP_ENOMEM, "GA buffers for P=%d", P);
    }
    // every buffer of the arena starts at zero (populations, fitness, bests,
    // counters, barrier and arrival words), then the run state
    hipError_t e = ga->arena.zero();
    unsigned long long init[GS_COUNT] = {0};
    init[GS_BEST] = (unsigned long long)INT64_MAX;
    if (e == hipSuccess)
        e = hipMemcpy(ga->gs, init, sizeof init, hipMemcpyHostToDevice);
    if (e == hipSuccess && ga->binom)
        e = hipMemcpy(ga->binom, binom.data(), sizeof(unsigned long long) * binom.size(),
                      hipMemcpyHostToDevice);
    ga->nsets = nsets;
    {
        const char *mode = getenv("PMP_GA_MODE");
        ga->persistent = mode && strcmp(mode, "persistent") == 0;
        ga->max_blocks = env_int("PMP_GA_BLOCKS", 0);
        ga->graph_gens = (mode && strcmp(mode, "kernels") == 0) ? 0
                                                                : env_int("PMP_GA_GRAPH_GENS", 8);
        ga->spec_on = env_int("PMP_GA_SPEC", 1) != 0;
    }
    if (e == hipSuccess)
        e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        pmp_ga_destroy(ga);
        return fail(PMP_EDEVICE, "GA state init: %s", hipGetErrorString(e));
    }
    *out = ga;
    return PMP_OK;
}

namespace {

hipEvent_t next_event(pmp_ga *ga)
{
    if (ga->ev_used == ga->ev.size()) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess)
            return nullptr;
        ga->ev.push_back(e);
    }
    return ga->ev[ga->ev_used++];
}

EvalArgs ga_eval_args(const pmp_ga *ga, const GaArgs &g, int buf)
{
    EvalArgs a{};
    a.t = g.t;
    a.paired = paired_scans(g.t.m, g.t.p);
    a.masks = g.off[buf];
    a.P = g.P;
    a.active = g.ok[buf];
    a.part = ga->part;
    a.spart = ga->spart;
    a.done = g.gs + GS_DONE;
    a.err = g.err;
    a.clients_per_block = ga->cpb;
    a.tiles_c = (g.P + kEvalTile - 1) / kEvalTile;
    a.tiles_i = ga->TI;
    a.waves = ga->waves;
    return a;
}

// Record a profiling event on s (no-op when profiling is off).
hipError_t mark(pmp_ga *ga, hipStream_t s)
{
    if (!ga->prof)
        return hipSuccess;
    hipEvent_t e = next_event(ga);
    if (!e)
        return hipErrorOutOfMemory;
    return hipEventRecord(e, s);
}

// Evaluate the offspring buffer `buf` (only slots flagged in ok[buf]); when
// profiling, with a pair of events stamped by the launch itself.
hipError_t ga_eval(pmp_ga *ga, const GaArgs &g, int buf, hipStream_t s, bool mutants = false)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (ga->prof) {
        e0 = next_event(ga);
        e1 = next_event(ga);
        if (!e0 || !e1)
            return hipErrorOutOfMemory;
    }
    EvalArgs a = ga_eval_args(ga, g, buf);
    if (mutants) {
        // the P x Y mutants of the mutation cycle, evaluated at once
        a.masks = g.mut;
        a.P = g.P * g.Y;
        a.active = g.mut_ok;
        a.part = ga->mpart;
        a.spart = ga->mspart;
        a.tiles_c = (a.P + kEvalTile - 1) / kEvalTile;
        a.clients_per_block = ga->spec_cpb;
        a.tiles_i = ga->spec_ti;
        a.waves = ga->spec_waves;
    }
    return launch_eval(a, s, e0, e1);
}

// A crossover stage fused with the evaluation of its offspring (buffer
// in ^ 1); when profiling, with a pair of events stamped by the launch.
hipError_t ga_stage_eval(pmp_ga *ga, const GaArgs &g, int in, int prev, int index,
                         hipStream_t s)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (ga->prof) {
        e0 = next_event(ga);
        e1 = next_event(ga);
        if (!e0 || !e1)
            return hipErrorOutOfMemory;
    }
    // launch k reads the partial sums launch k - 1 wrote (the population's
    // evaluation wrote `part` before launch 0) and writes the other set
    GaArgs gk = g;
    EvalArgs a = ga_eval_args(ga, g, in ^ 1);
    const bool odd = (index & 1) != 0;
    gk.part = odd ? ga->part2 : ga->part;
    gk.spart = odd ? ga->spart2 : ga->spart;
    gk.TI = index == 0 ? ga->TI : ga->fTI;  // the tiling of the sums it reads
    gk.pcm = index != 0;  // fused launches write chromosome-major sums
    a.pcm = 1;
    a.part = odd ? ga->part : ga->part2;
    a.spart = odd ? ga->spart : ga->spart2;
    a.clients_per_block = ga->fcpb;
    a.tiles_i = ga->fTI;
    return launch_ga_stage_eval(gk, a, in, prev, index, s, e0, e1);
}

// The run's report (GaReport layout) read into `out` with one copy after the
// work on stream s: gathered by a kernel, copied through the pinned staging
// memory.
hipError_t ga_report(pmp_ga *ga, hipStream_t s, std::vector<unsigned long long> &out)
{
    const size_t words = (size_t)RP_MASK + ga->inst->W;
    hipError_t e = launch_ga_report(ga->args(), ga->inst->err,
                                    ga->self ? ga->self->d_err : nullptr, ga->report, s);
    if (e == hipSuccess)
        e = staging().read(ga->report, words, s, out);
    return e;
}

// Totals of the per-chromosome counters.
hipError_t ga_counters(pmp_ga *ga, unsigned long long tot[CS_COUNT], hipStream_t s = nullptr)
{
    std::vector<unsigned long long> r;
    const hipError_t e = ga_report(ga, s, r);
    for (int k = 0; k < CS_COUNT; ++k)
        tot[k] = e == hipSuccess ? r[RP_TOT + k] : 0ull;
    return e;
}

}  // namespace

namespace {

// One Adam step on the learned proposal's ring after every Levery-th
// generation (gated on the device, so a captured graph replays correctly).
hipError_t launch_train(pmp_ga *ga, const GaArgs &g, hipStream_t s)
{
    TrainGate gate{g.gs + GS_GEN, ga->last_trained, ga->Levery};
    int nb = 0;
    pmp_model *md = ga->model;
    hipError_t e = launch_mlp_grad(md->d.view(), ga->rep_x, ga->rep_t, ga->rep_w,
                                   (int)ga->ring_rows(), md->partials, kTrainBlocks, md->d, gate,
                                   &nb, s);
    if (e == hipSuccess)
        e = launch_mlp_update(md->d, md->partials, nb, ga->Llr, nullptr, nullptr, gate, s);
    return e;
}

// Enqueue `generations` generations of the per-step launch sequence.
// capture: the sequence goes into a graph, which assumes that the first
// generation's population has been made ahead whenever the schedule makes
// populations ahead (pmp_ga_step ensures it before each replay).
hipError_t enqueue_generations(pmp_ga *ga, const GaArgs &g, int generations,
                               hipStream_t s, bool capture = false)
{
    const int X = ga->xstages(), S = X + ga->Y, L = g.L;
    const bool train = L > 0 && ga->Levery > 0;
    if (ga->spec()) {
        // crossover stages as usual; stage X finishes the last crossover and
        // makes all Y mutants; one evaluation; the cycle is resolved (with
        // the next generation's sampling in the same launch when merge)
        const bool merge = ga->merge_init(g);
        bool ahead = capture ? merge : (merge && ga->init_ahead);
        for (int gen = 0; gen < generations; ++gen) {
            hipError_t e = ahead ? hipSuccess : launch_ga_init(g, s);
            if (e == hipSuccess)
                e = ga_eval(ga, g, 0, s);
            for (int k = 0; k < X && e == hipSuccess; ++k) {
                int prev, op, index;
                ga_stage_ops(k, X, S, &prev, &op, &index, 0);
                if (ga->fused) {
                    e = ga_stage_eval(ga, g, k & 1, prev, index, s);
                } else {
                    e = launch_ga_stage(g, k & 1, prev, op, index, s);
                    if (e == hipSuccess)
                        e = ga_eval(ga, g, (k & 1) ^ 1, s);
                }
            }
            int in = X & 1;  // the buffer holding the last crossover's results
            const int prev = X == 0 ? OP_INIT : OP_XOVER;
            // the partial sums of the last evaluation (fused launches
            // alternate the two sets: launch k writes set (k + 1) mod 2)
            GaArgs gl = g;
            if (ga->fused && X > 0) {
                gl.TI = ga->fTI;
                gl.pcm = 1;
                if (X & 1) {
                    gl.part = ga->part2;
                    gl.spart = ga->spart2;
                }
            }
            if (L > 0) {
                // finish the crossovers, score the swaps of the chromosomes as
                // they stand, then make every mutant (the swaps among them)
                if (e == hipSuccess)
                    e = launch_ga_stage(gl, in, prev, OP_NONE, 0, s);
                if (e == hipSuccess)
                    e = launch_propose(ga->learn_args(g), in, s);
                in ^= 1;
                if (e == hipSuccess)
                    e = launch_ga_stage(g, in, OP_NONE, OP_MUT_ALL, 0, s);
            } else if (e == hipSuccess) {
                e = launch_ga_stage(gl, in, prev, OP_MUT_ALL, 0, s);
            }
            if (e == hipSuccess)
                e = ga_eval(ga, g, 0, s, true);
            if (e == hipSuccess)
                e = merge ? launch_ga_resolve_init(g, in ^ 1, ga->final_buf(), s)
                          : launch_ga_resolve(g, in ^ 1, ga->final_buf(), s);
            if (e == hipSuccess)
                e = launch_ga_best(g, ga->final_buf(), s, merge);
            if (e == hipSuccess && train)
                e = launch_train(ga, g, s);
            if (!capture)
                ga->init_ahead = merge && e == hipSuccess;
            if (e != hipSuccess)
                return e;
            ahead = merge;
        }
        return hipSuccess;
    }
    if (!capture)
        ga->init_ahead = false;
    for (int gen = 0; gen < generations; ++gen) {
        hipError_t e = launch_ga_init(g, s);
        if (e == hipSuccess)
            e = ga_eval(ga, g, 0, s);
        for (int k = 0; k <= S && e == hipSuccess; ++k) {
            int prev, op, index;
            ga_stage_ops(k, X, S, &prev, &op, &index, L);
            if (L > 0 && k == X) {
                // first mutation stage: finish the crossovers, then the
                // proposal kernel starts attempt 0 (a scored swap)
                e = launch_ga_stage(g, k & 1, prev, OP_NONE, 0, s);
                if (e == hipSuccess)
                    e = launch_propose(ga->learn_args(g), k & 1, s);
            } else {
                e = launch_ga_stage(g, k & 1, prev, op, index, s);
            }
            if (e == hipSuccess && op != OP_NONE)
                e = ga_eval(ga, g, (k & 1) ^ 1, s);
        }
        if (e == hipSuccess)
            e = launch_ga_best(g, ga->final_buf(), s);
        if (e == hipSuccess && train)
            e = launch_train(ga, g, s);
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

// Capture graph_gens generations of the launch sequence into a graph (once).
hipError_t ensure_graph(pmp_ga *ga, const GaArgs &g)
{
    if (ga->gexec)
        return hipSuccess;
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess)
        return e;
    hipGraph_t graph = nullptr;
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        const bool prof = ga->prof;
        ga->prof = false;  // no events inside the graph
        hipError_t ee = enqueue_generations(ga, g, ga->graph_gens, cs, true);
        ga->prof = prof;
        e = hipStreamEndCapture(cs, &graph);
        if (ee != hipSuccess)
            e = ee;
    }
    if (e == hipSuccess)
        e = hipGraphInstantiate(&ga->gexec, graph, nullptr, nullptr, 0);
    if (graph)
        (void)hipGraphDestroy(graph);
    (void)hipStreamDestroy(cs);
    return e;
}

}  // namespace

pmp_status pmp_ga_step(pmp_ga *ga, int32_t generations, void *stream)
{
    if (!ga)
        return fail(PMP_EINVAL, "ga is NULL");
    if (generations < 0)
        return fail(PMP_EINVAL, "generations < 0");
    if (generations == 0)
        return PMP_OK;
    hipStream_t s = (hipStream_t)stream;
    if (!ga->persistent && ga->spec() && ga->ensure_spec() != hipSuccess)
        return fail(PMP_ENOMEM, "mutation-cycle buffers for P=%d, Y=%d", ga->prm.population,
                    ga->Y);
    const GaArgs g = ga->args();
    if (ga->persistent) {
        if (ga->model)
            return fail(PMP_EUNSUPPORTED, "learned proposal in persistent-kernel mode");
        if (!ga->self) {
            ga->self = new BatchHost;
            pmp_ga *one = ga;
            if (batch_build(*ga->self, &one, 1) != hipSuccess)
                return fail(PMP_ENOMEM, "persistent launch set-up");
        }
        ga->init_ahead = false;
        HIP_TRY(mark(ga, s));
        HIP_TRY(batch_launch(*ga->self, generations, ga->max_blocks, s, true));
        HIP_TRY(mark(ga, s));
        return PMP_OK;
    }
    int left = generations;
    if (ga->graph_gens > 0 && !ga->prof && left >= ga->graph_gens) {
        HIP_TRY(ensure_graph(ga, g));
        if (ga->spec() && ga->merge_init(g) && !ga->init_ahead) {
            // the graph starts from a population made ahead
            HIP_TRY(launch_ga_init(g, s));
            ga->init_ahead = true;
        }
        for (; left >= ga->graph_gens; left -= ga->graph_gens)
            HIP_TRY(hipGraphLaunch(ga->gexec, s));
    }
    HIP_TRY(enqueue_generations(ga, g, left, s));
    // Profiled generations are launched one by one; build the graph of the
    // later ones now, on the host, while these run on the device.
    if (ga->prof && ga->graph_gens > 0)
        HIP_TRY(ensure_graph(ga, g));
    return PMP_OK;
}

pmp_status pmp_ga_best(pmp_ga *ga, uint64_t *mask, int64_t *cost,
                       pmp_ga_stats *stats, void *stream)
{
    if (!ga)
        return fail(PMP_EINVAL, "ga is NULL");
    hipStream_t s = (hipStream_t)stream;
    std::vector<unsigned long long> r;
    HIP_TRY(ga_report(ga, s, r));
    const unsigned long long *gs = r.data() + RP_GS;
    if (mask)
        for (int w = 0; w < ga->inst->W; ++w)
            mask[w] = r[RP_MASK + w];
    if (cost)
        *cost = (int64_t)gs[GS_BEST];
    if (stats) {
        const unsigned long long *tot = r.data() + RP_TOT;
        stats->generations = (int64_t)gs[GS_GEN];
        stats->saturation_count = (int64_t)gs[GS_SAT];
        stats->done = (int64_t)gs[GS_DONE];
        stats->best_cost = (int64_t)gs[GS_BEST];
        stats->chromosome_evals = (int64_t)tot[CS_EVALS];
        stats->crossover_fail = (int64_t)tot[CS_XO_FAIL];
        stats->crossover_taken = (int64_t)tot[CS_XO_TAKEN];
        stats->mutation_taken = (int64_t)tot[CS_MUT_TAKEN];
        stats->scan_total = (int64_t)tot[CS_SCAN];
        stats->pair_evals = (int64_t)tot[CS_EVALS] * ga->inst->n;
        stats->swap_tried = (int64_t)tot[CS_SWAP_TRIED];
        stats->swap_taken = (int64_t)tot[CS_SWAP_TAKEN];
        stats->speculative_evals = (int64_t)tot[CS_SPEC_EVALS];
    }
    return status_from_err((uint32_t)r[RP_ERR]);
}

pmp_status pmp_ga_state(pmp_ga *ga, uint64_t *population, int64_t *fitness,
                        uint64_t *group_masks, int64_t *group_costs,
                        void *stream)
{
    if (!ga)
        return fail(PMP_EINVAL, "ga is NULL");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipStreamSynchronize(s));
    const size_t W = ga->inst->W, P = ga->prm.population, NB = ga->NB;
    const int f = ga->final_buf();
    if (population)
        HIP_TRY(hipMemcpy(population, ga->cur[f], sizeof(uint64_t) * P * W,
                          hipMemcpyDeviceToHost));
    if (fitness)
        HIP_TRY(hipMemcpy(fitness, ga->fit[f], sizeof(int64_t) * P, hipMemcpyDeviceToHost));
    if (group_masks)
        HIP_TRY(hipMemcpy(group_masks, ga->gmask, sizeof(uint64_t) * NB * W,
                          hipMemcpyDeviceToHost));
    if (group_costs)
        HIP_TRY(hipMemcpy(group_costs, ga->gcost, sizeof(int64_t) * NB,
                          hipMemcpyDeviceToHost));
    return PMP_OK;
}

pmp_status pmp_ga_profile(pmp_ga *ga, int32_t enable)
{
    if (!ga)
        return fail(PMP_EINVAL, "ga is NULL");
    HIP_TRY(hipDeviceSynchronize());
    unsigned long long tot[CS_COUNT];
    HIP_TRY(ga_counters(ga, tot));
    ga->prof = enable != 0;
    ga->ev_used = 0;
    ga->base_scan = tot[CS_SCAN] + tot[CS_SPEC_SCAN];
    ga->base_evals = tot[CS_EVALS] + tot[CS_SPEC_EVALS];
    return PMP_OK;
}

pmp_status pmp_ga_profile_read(pmp_ga *ga, pmp_profile *out, void *stream)
{
    if (!ga || !out)
        return fail(PMP_EINVAL, "ga or out is NULL");
    hipStream_t s = (hipStream_t)stream;
    unsigned long long tot[CS_COUNT];
    HIP_TRY(ga_counters(ga, tot, s));  // (waits for the stream)
    double ms = 0;
    for (size_t k = 0; k + 1 < ga->ev_used; k += 2) {
        float t = 0;
        HIP_TRY(hipEventElapsedTime(&t, ga->ev[k], ga->ev[k + 1]));
        ms += t;
    }
    // every evaluation the kernel ran, the mutation cycle's speculative ones
    // included
    const int64_t evals = (int64_t)(tot[CS_EVALS] + tot[CS_SPEC_EVALS] - ga->base_evals);
    const int64_t scan = (int64_t)(tot[CS_SCAN] + tot[CS_SPEC_SCAN] - ga->base_scan);
    const int64_t pairs = evals * ga->inst->n;
    out->eval_ms = ms;
    out->eval_launches = (int64_t)(ga->ev_used / 2);
    out->eval_pairs = pairs;
    out->eval_bytes = 2 * scan + 4 * pairs + evals * (8 * (int64_t)ga->inst->W + 8);
    ga->ev_used = 0;
    ga->base_scan = tot[CS_SCAN] + tot[CS_SPEC_SCAN];
    ga->base_evals = tot[CS_EVALS] + tot[CS_SPEC_EVALS];
    return PMP_OK;
}

pmp_status pmp_ga_autotune(pmp_ga *ga, int32_t *clients, int32_t *waves, void *stream)
{
    if (!ga)
        return fail(PMP_EINVAL, "ga is NULL");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipStreamSynchronize(s));
    unsigned long long gs[GS_COUNT];
    HIP_TRY(hipMemcpy(gs, ga->gs, sizeof gs, hipMemcpyDeviceToHost));
    if (gs[GS_GEN] != 0)
        return fail(PMP_EINVAL, "autotune a GA before its first generation");
    const pmp_instance *inst = ga->inst;
    const int P = ga->prm.population, n = inst->n;
    // the shape's default: the rule's waves and clients per workgroup
    int best = ga->cpb, best_w = ga->waves;
    const bool forced = env_int("PMP_CLIENTS_PER_BLOCK", 0) > 0 || env_int("PMP_EVAL_WAVES", 0) > 0;
    // measured choices are shared by runs of similar shape
    static std::mutex mu;
    static std::map<std::tuple<int, int, int, int>, std::pair<int, int>> cache;
    const auto key = std::make_tuple((int)std::lround(std::log((double)n) / std::log(1.15)),
                                     2 * inst->W,
                                     (int)std::lround(std::log((inst->m + 1.0) / (inst->p + 1.0)) /
                                                      std::log(1.3)),
                                     P);
    bool cached = false;
    if (!forced) {
        std::lock_guard<std::mutex> lock(mu);
        auto it = cache.find(key);
        if (it != cache.end()) {
            best = it->second.first;
            best_w = it->second.second;
            cached = true;
        }
    }
    if (!forced && !cached) {
        // a generation-0 population to time the evaluation on, and (when the
        // mutation cycle is evaluated at once) Y copies of it standing in for
        // the mutants, whose evaluation runs with the same waves
        GaArgs g = ga->args();
        HIP_TRY(launch_ga_init(g, s));
        const bool spec = ga->spec();
        const size_t PY = (size_t)P * ga->Y, W = inst->W;
        uint64_t *stand_in = nullptr;
        if (spec) {
            if (ga->ensure_spec() != hipSuccess || dalloc(&stand_in, PY * W) != hipSuccess)
                return fail(PMP_ENOMEM, "autotune mutant stand-ins");
            for (int y = 0; y < ga->Y; ++y)
                HIP_TRY(hipMemcpyAsync(stand_in + (size_t)y * P * W, g.off[0],
                                       sizeof(uint64_t) * P * W, hipMemcpyDeviceToDevice, s));
        }
        const int cands[] = {4, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512};
        const int wcands[] = {16, 8, 4};
        const int max_ti = (n + 3) / 4;
        unsigned long long *part = nullptr;
        uint32_t *spart = nullptr;
        if (dalloc(&part, (size_t)max_ti * P) || dalloc(&spart, (size_t)max_ti * P)) {
            dfree(part);
            dfree(stand_in);
            return fail(PMP_ENOMEM, "autotune workspace");
        }
        hipEvent_t e0 = nullptr, e1 = nullptr;
        hipError_t e = hipEventCreate(&e0);
        if (e == hipSuccess)
            e = hipEventCreate(&e1);
        // The shape's default is timed first and is only replaced by a
        // candidate at least 3 % faster.  A candidate's time is the least of
        // three trials of four back-to-back pairs (the population's
        // evaluation, then the mutants'), so that one disturbed trial does
        // not decide.
        const int dflt = best, dflt_w = best_w;
        float best_ms = 1e30f;
        auto time_it = [&](int cpb, int wv) -> float {
            EvalArgs a = ga_eval_args(ga, g, 0);
            a.done = nullptr;
            a.part = part;
            a.spart = spart;
            a.clients_per_block = cpb;
            a.tiles_i = (n + cpb - 1) / cpb;
            a.waves = wv;
            EvalArgs am = a;
            if (spec) {
                am.masks = stand_in;
                am.P = (int32_t)PY;
                am.active = nullptr;
                am.part = ga->mpart;
                am.spart = ga->mspart;
                am.clients_per_block = ga->spec_cpb;
                am.tiles_c = (int32_t)((PY + kEvalTile - 1) / kEvalTile);
                am.tiles_i = ga->spec_ti;
            }
            auto pair = [&]() {
                hipError_t r = launch_eval(a, s);
                if (r == hipSuccess && spec)
                    r = launch_eval(am, s);
                return r;
            };
            e = pair();  // warm-up
            float least = 1e30f;
            for (int trial = 0; trial < 3 && e == hipSuccess; ++trial) {
                e = hipEventRecord(e0, s);
                for (int rep = 0; rep < 4 && e == hipSuccess; ++rep)
                    e = pair();
                if (e == hipSuccess)
                    e = hipEventRecord(e1, s);
                if (e == hipSuccess)
                    e = hipEventSynchronize(e1);
                float ms = 0;
                if (e == hipSuccess)
                    e = hipEventElapsedTime(&ms, e0, e1);
                if (e == hipSuccess && ms < least)
                    least = ms;
            }
            return e == hipSuccess ? least : 1e30f;
        };
        best_ms = time_it(dflt, dflt_w);
        for (int wv : wcands) {
            int last_ti = -1;
            for (int cpb : cands) {
                if (e != hipSuccess)
                    break;
                const int ti = (n + cpb - 1) / cpb;
                if (ti == last_ti || cpb > max_ti * 4 || (wv == dflt_w && ti == (n + dflt - 1) / dflt))
                    continue;
                last_ti = ti;
                const float ms = time_it(cpb, wv);
                if (ms < 0.97f * best_ms) {
                    best_ms = ms;
                    best = cpb;
                    best_w = wv;
                }
                if (ti == 1)
                    break;
            }
        }
        if (e0)
            (void)hipEventDestroy(e0);
        if (e1)
            (void)hipEventDestroy(e1);
        dfree(part);
        dfree(spart);
        dfree(stand_in);
        if (e != hipSuccess)
            return fail(PMP_EDEVICE, "autotune: %s", hipGetErrorString(e));
        std::lock_guard<std::mutex> lock(mu);
        cache[key] = std::make_pair(best, best_w);
    }
    ga->waves = best_w;
    ga->spec_waves = best_w;
    if (best != ga->cpb) {
        const int ti = (n + best - 1) / best;
        if (ga->carve_parts(std::max(ti, ga->fTI)) != hipSuccess)
            return fail(PMP_ENOMEM, "GA partial sums for %d client tiles", ti);
        ga->cpb = best;
        ga->TI = ti;
        if (ga->self) {
            ga->self->release();
            delete ga->self;
            ga->self = nullptr;
        }
    }
    if (ga->gexec) {  // captured with the old tile
        (void)hipGraphExecDestroy(ga->gexec);
        ga->gexec = nullptr;
    }
    if (clients)
        *clients = best;
    if (waves)
        *waves = best_w;
    return PMP_OK;
}

pmp_status pmp_batch_create(pmp_ga *const *gas, int32_t count, pmp_batch **out)
{
    if (!out)
        return fail(PMP_EINVAL, "out is NULL");
    *out = nullptr;
    if (!gas || count < 1)
        return fail(PMP_EINVAL, "need at least one GA");
    for (int b = 0; b < count; ++b) {
        if (!gas[b])
            return fail(PMP_EINVAL, "GA %d is NULL", b);
        if (gas[b]->model)
            return fail(PMP_EUNSUPPORTED, "GA %d uses a learned proposal (not batched)", b);
        for (int c = 0; c < b; ++c)
            if (gas[c] == gas[b])
                return fail(PMP_EINVAL, "GA %d appears twice", b);
    }
    pmp_batch *bt = new pmp_batch;
    hipError_t e = batch_build(bt->bh, gas, count);
    if (e != hipSuccess) {
        bt->bh.release();
        delete bt;
        return fail(PMP_ENOMEM, "batch set-up: %s", hipGetErrorString(e));
    }
    const char *g = getenv("PMP_BATCH_GRAPH");
    bt->graphs = !(g && strcmp(g, "0") == 0);
    const char *mode = getenv("PMP_BATCH_MODE");
    bt->persistent = mode && strcmp(mode, "persistent") == 0;
    bt->max_blocks = env_int("PMP_GA_BLOCKS", 0);
    *out = bt;
    return PMP_OK;
}

pmp_status pmp_batch_autotune(pmp_batch *bt, int32_t *clients, void *stream)
{
    if (!bt)
        return fail(PMP_EINVAL, "batch is NULL");
    hipStream_t s = (hipStream_t)stream;
    BatchHost &bh = bt->bh;
    HIP_TRY(hipStreamSynchronize(s));
    if (env_int("PMP_BATCH_CLIENTS", 0) > 0) {  // set by hand: no timing
        if (clients)
            *clients = bh.clients;
        return PMP_OK;
    }
    // measured choices are shared by batches of the same run shapes
    static std::mutex mu;
    static std::map<std::vector<int32_t>, int> cache;
    std::vector<int32_t> key;
    key.reserve(5 * bh.gas.size());
    for (size_t b = 0; b < bh.gas.size(); ++b) {
        const pmp_ga *ga = bh.gas[b];
        key.insert(key.end(), {ga->inst->n, ga->inst->m, ga->inst->p, ga->prm.population,
                               bh.base_cpb[b]});
    }
    {
        std::lock_guard<std::mutex> lock(mu);
        auto it = cache.find(key);
        if (it != cache.end()) {
            if (batch_tiles(bh, it->second) != hipSuccess)
                return fail(PMP_EDEVICE, "batch tiling upload");
            if (clients)
                *clients = it->second;
            return PMP_OK;
        }
    }
    // the probe's inputs: every run's generation-0 population (buffer 0),
    // made again by the first step; a run past it would lose its population
    for (size_t b = 0; b < bh.gas.size(); ++b) {
        unsigned long long gen = 0;
        HIP_TRY(hipMemcpy(&gen, bh.gas[b]->gs + GS_GEN, sizeof gen, hipMemcpyDeviceToHost));
        if (gen != 0)
            return fail(PMP_EINVAL, "autotune a batch before its first step (run %zu)", b);
    }
    for (pmp_ga *ga : bh.gas)
        HIP_TRY(launch_ga_init(ga->args(), s));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess)
        e = hipEventCreate(&e1);
    // A tiling's time is the least of three trials of four back-to-back
    // evaluations; the runs' own tiling (0) is timed first and is only
    // replaced by a common one at least 3 % faster.
    auto time_it = [&](int common) -> float {
        if (e == hipSuccess)
            e = batch_tiles(bh, common);
        if (e == hipSuccess)
            e = launch_ga_batch_eval(bh.args, bh.ntiles, bh.max_w2, s);  // warm-up
        float least = 1e30f;
        for (int trial = 0; trial < 3 && e == hipSuccess; ++trial) {
            e = hipEventRecord(e0, s);
            for (int rep = 0; rep < 4 && e == hipSuccess; ++rep)
                e = launch_ga_batch_eval(bh.args, bh.ntiles, bh.max_w2, s);
            if (e == hipSuccess)
                e = hipEventRecord(e1, s);
            if (e == hipSuccess)
                e = hipEventSynchronize(e1);
            float ms = 0;
            if (e == hipSuccess)
                e = hipEventElapsedTime(&ms, e0, e1);
            if (e == hipSuccess && ms < least)
                least = ms;
        }
        return least;
    };
    int best = 0;
    float best_ms = time_it(0);
    const int commons[] = {64, 96, 128, 192, 256, 384, 512};
    for (int f : commons) {
        if (e != hipSuccess)
            break;
        const float ms = time_it(f);
        if (ms < 0.97f * best_ms) {
            best_ms = ms;
            best = f;
        }
    }
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    if (e == hipSuccess)
        e = batch_tiles(bh, best);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return fail(PMP_EDEVICE, "batch autotune: %s", hipGetErrorString(e));
    {
        std::lock_guard<std::mutex> lock(mu);
        cache[key] = best;
    }
    if (clients)
        *clients = best;
    return PMP_OK;
}

pmp_status pmp_batch_step(pmp_batch *bt, int32_t generations, void *stream)
{
    if (!bt)
        return fail(PMP_EINVAL, "batch is NULL");
    if (generations < 0)
        return fail(PMP_EINVAL, "generations < 0");
    if (generations == 0)
        return PMP_OK;
    hipStream_t s = (hipStream_t)stream;
    BatchHost &bh = bt->bh;
    for (pmp_ga *ga : bh.gas)  // the batch kernels make each generation's population
        ga->init_ahead = false;
    if (!bt->graphs || bt->prof) {
        HIP_TRY(batch_enqueue(bt, generations, s, true));
        return PMP_OK;
    }
    auto it = bh.graphs.find(generations);
    if (it == bh.graphs.end()) {
        // capture the single persistent launch once per generation count
        hipStream_t cs = nullptr;
        HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipError_t le = batch_enqueue(bt, generations, cs, false);
            e = hipStreamEndCapture(cs, &graph);
            if (le != hipSuccess)
                e = le;
        }
        if (e == hipSuccess)
            e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (graph)
            (void)hipGraphDestroy(graph);
        (void)hipStreamDestroy(cs);
        if (e != hipSuccess)
            return fail(PMP_EDEVICE, "capturing the batch launch: %s", hipGetErrorString(e));
        it = bh.graphs.emplace(generations, exec).first;
    }
    HIP_TRY(hipGraphLaunch(it->second, s));
    return PMP_OK;
}

pmp_status pmp_batch_check(pmp_batch *bt, int32_t *grid, void *stream)
{
    if (!bt)
        return fail(PMP_EINVAL, "batch is NULL");
    HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    uint32_t herr = 0;
    HIP_TRY(hipMemcpy(&herr, bt->bh.d_err, sizeof herr, hipMemcpyDeviceToHost));
    if (grid)
        *grid = bt->bh.last_grid;
    return status_from_err(herr);
}

void pmp_batch_destroy(pmp_batch *bt)
{
    if (!bt)
        return;
    bt->bh.release();
    for (hipEvent_t e : bt->ev)
        (void)hipEventDestroy(e);
    delete bt;
}

pmp_status pmp_batch_profile(pmp_batch *bt, int32_t enable)
{
    if (!bt)
        return fail(PMP_EINVAL, "batch is NULL");
    if (bt->persistent)
        return fail(PMP_EUNSUPPORTED, "profiling the persistent batch kernel");
    HIP_TRY(hipDeviceSynchronize());
    bt->prof = enable != 0;
    bt->ev_used = 0;
    return PMP_OK;
}

pmp_status pmp_batch_profile_read(pmp_batch *bt, double *eval_ms, int64_t *eval_launches,
                                  void *stream)
{
    if (!bt)
        return fail(PMP_EINVAL, "batch is NULL");
    HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    double ms = 0;
    for (int k = 0; k + 1 < bt->ev_used; k += 2) {
        float t = 0;
        HIP_TRY(hipEventElapsedTime(&t, bt->ev[k], bt->ev[k + 1]));
        ms += t;
    }
    if (eval_ms)
        *eval_ms = ms;
    if (eval_launches)
        *eval_launches = bt->ev_used / 2;
    bt->ev_used = 0;
    return PMP_OK;
}

pmp_status pmp_ga_step_batch(pmp_ga *const *gas, int32_t count, int32_t generations,
                             void *stream)
{
    pmp_batch *bt = nullptr;
    pmp_status st = pmp_batch_create(gas, count, &bt);
    if (st != PMP_OK)
        return st;
    const bool graphs = bt->graphs;
    bt->graphs = false;  // a one-off launch needs no graph
    st = pmp_batch_step(bt, generations, stream);
    bt->graphs = graphs;
    if (st == PMP_OK)
        st = pmp_batch_check(bt, nullptr, stream);
    pmp_batch_destroy(bt);
    return st;
}

pmp_status pmp_solve(const int32_t *d, int32_t n, int32_t m, int32_t p,
                     const pmp_ga_params *params, uint8_t *open, int64_t *cost,
                     pmp_ga_stats *stats)
{
    if (!params || !open || !cost)
        return fail(PMP_EINVAL, "params, open or cost is NULL");
    pmp_instance *inst = nullptr;
    pmp_status st = pmp_preprocess(d, m, n, m, p, 0, nullptr, &inst);
    if (st != PMP_OK)
        return st;
    pmp_ga *ga = nullptr;
    st = pmp_ga_create(inst, params, &ga);
    // Enqueue generations in chunks and stop enqueueing once the run has
    // stopped (saturation can end it long before EvolveLimit).
    for (int done_gens = 0; st == PMP_OK && done_gens < params->generations;) {
        const int chunk = params->generations - done_gens < 32
                              ? params->generations - done_gens : 32;
        st = pmp_ga_step(ga, chunk, nullptr);
        done_gens += chunk;
        unsigned long long flag = 0;
        if (st == PMP_OK &&
            hipMemcpy(&flag, ga->gs + GS_DONE, sizeof flag, hipMemcpyDeviceToHost) != hipSuccess)
            st = fail(PMP_EDEVICE, "reading the stop flag");
        if (flag)
            break;
    }
    std::vector<uint64_t> mask((size_t)inst->W);
    if (st == PMP_OK)
        st = pmp_ga_best(ga, mask.data(), cost, stats, nullptr);
    if (st == PMP_OK)
        for (int j = 0; j < m; ++j)
            open[j] = (uint8_t)((mask[j / 64] >> (j % 64)) & 1u);
    pmp_ga_destroy(ga);
    pmp_instance_destroy(inst);
    return st;
}


pmp_status pmp_features(pmp_instance *inst, const uint64_t *masks, int32_t P,
                        float gen_frac, float *out, uint32_t flags, void *stream)
{
    if (!inst)
        return fail(PMP_EINVAL, "instance is NULL");
    if (P < 0)
        return fail(PMP_EINVAL, "P < 0");
    if (inst->m > PMP_MAX_LEARNED_FACILITIES)
        return fail(PMP_EUNSUPPORTED, "m=%d above %d", inst->m, PMP_MAX_LEARNED_FACILITIES);
    if (P == 0)
        return PMP_OK;
    if (!masks || !out)
        return fail(PMP_EINVAL, "masks or out is NULL");
    if (inst->resolve_total() != hipSuccess)
        return fail(PMP_EDEVICE, "sum of d of the instance");
    hipStream_t s = (hipStream_t)stream;
    const bool on_dev = flags & PMP_ON_DEVICE;
    const size_t W = inst->W, cells = (size_t)P * inst->m * kFeatures;
    const uint64_t *dm = masks;
    float *dout = out;
    uint64_t *tm = nullptr;
    float *to = nullptr;
    pmp_status st = PMP_OK;
    do {
        if (!on_dev) {
            if (dalloc(&tm, (size_t)P * W) || dalloc(&to, cells)) {
                st = fail(PMP_ENOMEM, "feature staging for P=%d", P);
                break;
            }
            if (hipMemcpyAsync(tm, masks, sizeof(uint64_t) * P * W, hipMemcpyHostToDevice,
                               s) != hipSuccess) {
                st = fail(PMP_EDEVICE, "copy of masks");
                break;
            }
            dm = tm;
            dout = to;
        }
        FeatCtx ctx{};
        ctx.n = inst->n;
        ctx.m = inst->m;
        ctx.p = inst->p;
        ctx.near_len = inst->near_len;
        ctx.total = inst->total;
        ctx.gen_frac = gen_frac;
        ctx.colsum = inst->colsum;
        ctx.nearc = inst->nearc;
        hipError_t e = launch_zero(inst->err, sizeof(uint32_t), s);
        if (e == hipSuccess)
            e = launch_features(inst->tables(), dm, P, ctx, dout, inst->err, s);
        if (e == hipSuccess && !on_dev)
            e = hipMemcpyAsync(out, dout, sizeof(float) * cells, hipMemcpyDeviceToHost, s);
        uint32_t herr = 0;
        if (e == hipSuccess)
            e = hipMemcpyAsync(&herr, inst->err, sizeof herr, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess)
            e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            st = fail(PMP_EDEVICE, "features: %s", hipGetErrorString(e));
            break;
        }
        st = status_from_err(herr);
    } while (0);
    dfree(tm);
    dfree(to);
    return st;
}

void pmp_model_destroy(pmp_model *md)
{
    if (!md)
        return;
    dfree(md->d.master);
    dfree(md->d.m1);
    dfree(md->d.m2);
    dfree(md->d.W1);
    dfree(md->d.W2);
    dfree(md->d.W2T);
    dfree(md->d.w3);
    dfree(md->d.step);
    dfree(md->partials);
    dfree(md->grad);
    dfree(md->loss);
    dfree(md->xf);
    dfree(md->xb);
    dfree(md->tf);
    dfree(md->wf);
    dfree(md->yf);
    delete md;
}

pmp_status pmp_model_create(uint64_t seed, pmp_model **out)
{
    if (!out)
        return fail(PMP_EINVAL, "out is NULL");
    *out = nullptr;
    pmp_model *md = new pmp_model;
    MlpModelDev &d = md->d;
    if (dalloc(&d.master, kParams) || dalloc(&d.m1, kParams) || dalloc(&d.m2, kParams) ||
        dalloc(&d.W1, (size_t)kHidden * kIn) || dalloc(&d.W2, (size_t)kHidden * kHidden) ||
        dalloc(&d.W2T, (size_t)kHidden * kHidden) || dalloc(&d.w3, kHidden) ||
        dalloc(&d.step, 1) || dalloc(&md->partials, kPartFloats) ||
        dalloc(&md->grad, kParams) || dalloc(&md->loss, 1)) {
        pmp_model_destroy(md);
        return fail(PMP_ENOMEM, "model buffers");
    }
    hipError_t e = launch_mlp_init(d, seed, nullptr);
    if (e == hipSuccess)
        e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        pmp_model_destroy(md);
        return fail(PMP_EDEVICE, "model init: %s", hipGetErrorString(e));
    }
    *out = md;
    return PMP_OK;
}

pmp_status pmp_model_get(pmp_model *md, float *params, uint32_t flags, void *stream)
{
    if (!md || !params)
        return fail(PMP_EINVAL, "model or params is NULL");
    hipStream_t s = (hipStream_t)stream;
    const bool on_dev = flags & PMP_ON_DEVICE;
    HIP_TRY(hipMemcpyAsync(params, md->d.master, sizeof(float) * kParams,
                           on_dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
    if (!on_dev)
        HIP_TRY(hipStreamSynchronize(s));
    return PMP_OK;
}

pmp_status pmp_model_set(pmp_model *md, const float *params, uint32_t flags, void *stream)
{
    if (!md || !params)
        return fail(PMP_EINVAL, "model or params is NULL");
    hipStream_t s = (hipStream_t)stream;
    const bool on_dev = flags & PMP_ON_DEVICE;
    HIP_TRY(hipMemcpyAsync(md->d.master, params, sizeof(float) * kParams,
                           on_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
    HIP_TRY(launch_zero(md->d.m1, sizeof(float) * kParams, s));
    HIP_TRY(launch_zero(md->d.m2, sizeof(float) * kParams, s));
    HIP_TRY(launch_zero(md->d.step, sizeof(uint32_t), s));
    HIP_TRY(launch_mlp_publish(md->d, s));
    if (!on_dev)
        HIP_TRY(hipStreamSynchronize(s));
    return PMP_OK;
}

namespace {

// Device copies of a call's rows: BF16 inputs, and targets / weights.
pmp_status model_stage(pmp_model *md, const float *x, const float *t, const float *w,
                       int32_t rows, bool on_dev, hipStream_t s, const float **dt,
                       const float **dw)
{
    if (md->cap < rows) {
        dfree(md->xf);
        dfree(md->xb);
        dfree(md->tf);
        dfree(md->wf);
        dfree(md->yf);
        md->cap = 0;
        if (dalloc(&md->xf, (size_t)rows * kIn) || dalloc(&md->xb, (size_t)rows * kIn) ||
            dalloc(&md->tf, (size_t)rows) || dalloc(&md->wf, (size_t)rows) ||
            dalloc(&md->yf, (size_t)rows))
            return fail(PMP_ENOMEM, "model staging for %d rows", rows);
        md->cap = rows;
    }
    const float *dx = x;
    if (!on_dev) {
        HIP_TRY(hipMemcpyAsync(md->xf, x, sizeof(float) * rows * kIn, hipMemcpyHostToDevice, s));
        dx = md->xf;
    }
    HIP_TRY(launch_to_bf16(dx, md->xb, (int64_t)rows * kIn, s));
    if (dt) {
        *dt = t;
        if (t && !on_dev) {
            HIP_TRY(hipMemcpyAsync(md->tf, t, sizeof(float) * rows, hipMemcpyHostToDevice, s));
            *dt = md->tf;
        }
    }
    if (dw) {
        *dw = w;
        if (w && !on_dev) {
            HIP_TRY(hipMemcpyAsync(md->wf, w, sizeof(float) * rows, hipMemcpyHostToDevice, s));
            *dw = md->wf;
        }
    }
    return PMP_OK;
}

}  // namespace

pmp_status pmp_model_forward(pmp_model *md, const float *x, int32_t rows, float *y,
                             uint32_t flags, void *stream)
{
    if (!md)
        return fail(PMP_EINVAL, "model is NULL");
    if (rows < 0)
        return fail(PMP_EINVAL, "rows < 0");
    if (rows == 0)
        return PMP_OK;
    if (!x || !y)
        return fail(PMP_EINVAL, "x or y is NULL");
    hipStream_t s = (hipStream_t)stream;
    const bool on_dev = flags & PMP_ON_DEVICE;
    pmp_status st = model_stage(md, x, nullptr, nullptr, rows, on_dev, s, nullptr, nullptr);
    if (st != PMP_OK)
        return st;
    float *dy = on_dev ? y : md->yf;
    HIP_TRY(launch_mlp_forward(md->d.view(), md->xb, rows, dy, s));
    if (!on_dev) {
        HIP_TRY(hipMemcpyAsync(y, dy, sizeof(float) * rows, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    return PMP_OK;
}

namespace {

pmp_status model_steps(pmp_model *md, const float *x, const float *t, const float *w,
                       int32_t rows, float lr, int32_t steps, float *grad, float *loss,
                       uint32_t flags, hipStream_t s)
{
    if (!md)
        return fail(PMP_EINVAL, "model is NULL");
    if (rows < 1 || !x || !t)
        return fail(PMP_EINVAL, "need rows >= 1, x and t");
    const bool on_dev = flags & PMP_ON_DEVICE;
    const float *dt = nullptr, *dw = nullptr;
    pmp_status st = model_stage(md, x, t, w, rows, on_dev, s, &dt, &dw);
    if (st != PMP_OK)
        return st;
    float *dgrad = grad ? (on_dev ? grad : md->grad) : nullptr;
    if (dgrad)
        HIP_TRY(launch_zero(dgrad, sizeof(float) * kParams, s));
    if (loss)
        HIP_TRY(launch_zero(md->loss, sizeof(float), s));
    for (int k = 0; k < steps; ++k) {
        int nb = 0;
        HIP_TRY(launch_mlp_grad(md->d.view(), md->xb, dt, dw, rows, md->partials, kTrainBlocks,
                                md->d, TrainGate{nullptr, nullptr, 1}, &nb, s));
        const bool last = k == steps - 1;
        HIP_TRY(launch_mlp_update(md->d, md->partials, nb, lr, last ? dgrad : nullptr,
                                  last && loss ? md->loss : nullptr,
                                  TrainGate{nullptr, nullptr, 1}, s));
    }
    if (grad && !on_dev)
        HIP_TRY(hipMemcpyAsync(grad, dgrad, sizeof(float) * kParams, hipMemcpyDeviceToHost, s));
    if (loss)
        HIP_TRY(hipMemcpyAsync(loss, md->loss, sizeof(float),
                               on_dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
    if (!on_dev)
        HIP_TRY(hipStreamSynchronize(s));
    return PMP_OK;
}

}  // namespace

pmp_status pmp_model_grad(pmp_model *md, const float *x, const float *t, const float *w,
                          int32_t rows, float *grad, float *loss, uint32_t flags, void *stream)
{
    return model_steps(md, x, t, w, rows, 0.f, 1, grad, loss, flags, (hipStream_t)stream);
}

pmp_status pmp_model_train(pmp_model *md, const float *x, const float *t, const float *w,
                           int32_t rows, float lr, int32_t steps, float *loss, uint32_t flags,
                           void *stream)
{
    if (!(lr > 0.f) || steps < 1)
        return fail(PMP_EINVAL, "need lr > 0 and steps >= 1");
    return model_steps(md, x, t, w, rows, lr, steps, nullptr, loss, flags,
                       (hipStream_t)stream);
}

pmp_status pmp_ga_set_model(pmp_ga *ga, pmp_model *model, const pmp_learn_params *lp)
{
    if (!ga)
        return fail(PMP_EINVAL, "ga is NULL");
    HIP_TRY(hipDeviceSynchronize());
    if (ga->gexec) {
        (void)hipGraphExecDestroy(ga->gexec);
        ga->gexec = nullptr;
    }
    if (!model) {
        ga->model = nullptr;
        ga->free_learned();
        return PMP_OK;
    }
    if (ga->persistent)
        return fail(PMP_EUNSUPPORTED, "learned proposal in persistent-kernel mode");
    if (ga->inst->m > PMP_MAX_LEARNED_FACILITIES)
        return fail(PMP_EUNSUPPORTED, "m=%d above %d", ga->inst->m, PMP_MAX_LEARNED_FACILITIES);
    if (ga->inst->resolve_total() != hipSuccess)  // (a feature's denominator)
        return fail(PMP_EDEVICE, "sum of d of the instance");
    pmp_learn_params q{};
    if (lp)
        q = *lp;
    if (q.reserved[0] || q.reserved[1])
        return fail(PMP_EINVAL, "reserved fields must be 0");
    const int C = q.candidates ? q.candidates : PMP_MAX_CANDIDATES;
    if (C < 1 || C > PMP_MAX_CANDIDATES)
        return fail(PMP_EINVAL, "candidates %d outside 1..%d", C, PMP_MAX_CANDIDATES);
    if (ga->Y < 1)
        return fail(PMP_EINVAL, "the run has no mutation attempts");
    const int L = q.learned_iters ? q.learned_iters : (ga->Y + 1) / 2;
    if (L < 1 || L > C || L > ga->Y)
        return fail(PMP_EINVAL, "learned_iters %d outside 1..min(C=%d, Y=%d)", L, C, ga->Y);
    if (q.explore_permille < 0 || q.explore_permille > 1000)
        return fail(PMP_EINVAL, "explore_permille outside 0..1000");
    const int H = q.history ? q.history : 4;
    if (H < 1 || (int64_t)H * L * ga->prm.population > (1 << 24))
        return fail(PMP_EINVAL, "history %d: ring too large", H);
    if (q.train_every < 0)
        return fail(PMP_EINVAL, "train_every < 0");
    const float lr = q.lr == 0.f ? 1e-3f : q.lr;
    if (!(lr > 0.f) || lr > 1.f)
        return fail(PMP_EINVAL, "lr outside (0, 1]");
    ga->free_learned();
    ga->model = nullptr;
    const size_t P = ga->prm.population, R = (size_t)H * L * P;
    if (dalloc(&ga->swaps, P * L * 2) || dalloc(&ga->rep_x, R * kIn) || dalloc(&ga->rep_t, R) ||
        dalloc(&ga->rep_w, R) || dalloc(&ga->rep_jk, R * 2) || dalloc(&ga->rep_d, R * 2) ||
        dalloc(&ga->scores, P * C) || dalloc(&ga->cand, P * C * 2) ||
        dalloc(&ga->cbits, P * ga->inst->W) || dalloc(&ga->cpre, P * ga->inst->W) ||
        hipMalloc(&ga->sums, P * kSlots * (2 * sizeof(uint32_t) + 3 * sizeof(uint64_t))) ||
        dalloc(&ga->last_trained, 1)) {
        ga->free_learned();
        return fail(PMP_ENOMEM, "learned proposal buffers (%zu ring rows)", R);
    }
    hipError_t e = hipMemset(ga->rep_w, 0, sizeof(float) * R);
    if (e == hipSuccess)
        e = hipMemset(ga->rep_t, 0, sizeof(float) * R);
    if (e == hipSuccess)
        e = hipMemset(ga->rep_x, 0, sizeof(uint16_t) * R * kIn);
    if (e == hipSuccess)
        e = hipMemset(ga->rep_jk, 0, sizeof(int32_t) * R * 2);
    if (e == hipSuccess)
        e = hipMemset(ga->rep_d, 0, sizeof(long long) * R * 2);
    if (e == hipSuccess)
        e = hipMemset(ga->scores, 0, sizeof(float) * P * C);
    if (e == hipSuccess)
        e = hipMemset(ga->last_trained, 0, sizeof(unsigned long long));
    if (e == hipSuccess)
        e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        ga->free_learned();
        return fail(PMP_EDEVICE, "learned proposal init: %s", hipGetErrorString(e));
    }
    ga->walk_shape = env_int("PMP_WALK", 0);
    if (ga->walk_shape == 0) {
        // the two-pass walk's buffers and the facility index of the rows'
        // first positions (built once per run)
        const Tables t = ga->inst->tables();
        const size_t PN = P * (size_t)t.n;
        const int L = std::min(kNearL, t.K);
        const size_t E = (size_t)t.n * L;
        int32_t *cursor = nullptr;
        std::vector<int32_t> off((size_t)t.m + 1, 0);
        if (dalloc(&ga->s12, PN) || dalloc(&ga->c12, 2 * PN) ||
            dalloc(&ga->near_off, (size_t)t.m + 1) || dalloc(&ga->near_q, E) ||
            dalloc(&cursor, (size_t)t.m)) {
            dfree(cursor);
            ga->free_learned();
            return fail(PMP_ENOMEM, "two-pass walk buffers (%zu pairs)", PN);
        }
        e = hipMemset(cursor, 0, sizeof(int32_t) * t.m);
        if (e == hipSuccess)
            e = launch_near_count(t, cursor, nullptr);
        if (e == hipSuccess)
            e = hipMemcpy(off.data() + 1, cursor, sizeof(int32_t) * t.m, hipMemcpyDeviceToHost);
        for (int f = 0; f < t.m; ++f)
            off[f + 1] += off[f];
        if (e == hipSuccess)
            e = hipMemcpy(ga->near_off, off.data(), sizeof(int32_t) * off.size(),
                          hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(cursor, off.data(), sizeof(int32_t) * t.m, hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = launch_near_fill(t, cursor, ga->near_q, nullptr);
        if (e == hipSuccess)
            e = hipDeviceSynchronize();
        dfree(cursor);
        if (e != hipSuccess) {
            ga->free_learned();
            return fail(PMP_EDEVICE, "facility index: %s", hipGetErrorString(e));
        }
    }
    ga->model = model;
    ga->LC = C;
    ga->LL = L;
    ga->Lexp = q.explore_permille;
    ga->LH = H;
    ga->Levery = q.train_every;
    ga->Llr = lr;
    return PMP_OK;
}

pmp_status pmp_ga_replay(pmp_ga *ga, int32_t *rows, uint16_t *x, float *target,
                         float *weight, int32_t *swap, int64_t *delta, float *scores,
                         void *stream)
{
    if (!ga)
        return fail(PMP_EINVAL, "ga is NULL");
    if (!ga->model)
        return fail(PMP_EINVAL, "the run has no model");
    HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    const size_t R = (size_t)ga->ring_rows();
    if (rows)
        *rows = (int32_t)R;
    if (x)
        HIP_TRY(hipMemcpy(x, ga->rep_x, sizeof(uint16_t) * R * kIn, hipMemcpyDeviceToHost));
    if (target)
        HIP_TRY(hipMemcpy(target, ga->rep_t, sizeof(float) * R, hipMemcpyDeviceToHost));
    if (weight)
        HIP_TRY(hipMemcpy(weight, ga->rep_w, sizeof(float) * R, hipMemcpyDeviceToHost));
    if (swap)
        HIP_TRY(hipMemcpy(swap, ga->rep_jk, sizeof(int32_t) * R * 2, hipMemcpyDeviceToHost));
    if (delta)
        HIP_TRY(hipMemcpy(delta, ga->rep_d, sizeof(int64_t) * R * 2, hipMemcpyDeviceToHost));
    if (scores)
        HIP_TRY(hipMemcpy(scores, ga->scores, sizeof(float) * ga->prm.population * ga->LC,
                          hipMemcpyDeviceToHost));
    return PMP_OK;
}


pmp_status pmp_exhaustive(pmp_instance *inst, uint64_t *best_mask, int64_t *best_cost,
                          int64_t *count, void *stream)
{
    if (!inst)
        return fail(PMP_EINVAL, "instance is NULL");
    if (inst->m > PMP_MAX_FACILITIES)
        return fail(PMP_EUNSUPPORTED, "enumeration takes m <= %d", PMP_MAX_FACILITIES);
    const int m = inst->m, p = inst->p, n = inst->n, W = inst->W;
    std::vector<unsigned long long> binom;
    const unsigned long long total = binomial_table(m, p, binom);
    if (total >= (1ull << 62))
        return fail(PMP_EUNSUPPORTED, "C(%d, %d) is too large to enumerate", m, p);
    if (count)
        *count = (int64_t)total;
    hipStream_t s = (hipStream_t)stream;
    const int B = (int)std::min<unsigned long long>(total, 1ull << 18);
    const int nblk = (B + 255) / 256;
    EvalArgs a{};
    a.t = inst->tables();
    a.paired = paired_scans(inst->m, inst->p);
    a.P = B;
    a.active = nullptr;
    a.done = nullptr;
    a.err = inst->err;
    a.waves = eval_waves(n, B, m, p, W);
    a.clients_per_block = clients_per_block(n, B, m, p, W, false, a.waves);
    a.tiles_c = (B + kEvalTile - 1) / kEvalTile;
    a.tiles_i = (n + a.clients_per_block - 1) / a.clients_per_block;
    unsigned long long *d_binom = nullptr, *fit = nullptr, *bc = nullptr, *run = nullptr;
    uint64_t *masks = nullptr;
    unsigned long long *part = nullptr;
    int *bi = nullptr;
    pmp_status st = PMP_OK;
    do {
        if (dalloc(&d_binom, binom.size()) || dalloc(&fit, (size_t)B) || dalloc(&bc, (size_t)nblk) ||
            dalloc(&bi, (size_t)nblk) || dalloc(&run, 2) || dalloc(&masks, (size_t)B * W) ||
            dalloc(&part, (size_t)a.tiles_i * B)) {
            st = fail(PMP_ENOMEM, "enumeration buffers (batch %d)", B);
            break;
        }
        const unsigned long long init[2] = {~0ull, 0ull};
        hipError_t e = hipMemcpyAsync(d_binom, binom.data(), sizeof(unsigned long long) * binom.size(),
                                      hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(run, init, sizeof init, hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = launch_zero(inst->err, sizeof(uint32_t), s);
        a.masks = masks;
        a.part = part;
        a.spart = nullptr;
        for (unsigned long long r0 = 0; r0 < total && e == hipSuccess; r0 += (unsigned long long)B) {
            const int cnt = (int)std::min<unsigned long long>((unsigned long long)B, total - r0);
            EvalArgs b = a;
            b.P = cnt;
            b.tiles_c = (cnt + kEvalTile - 1) / kEvalTile;
            e = launch_unrank(d_binom, m, p, W, r0, cnt, masks, s);
            if (e == hipSuccess)
                e = launch_eval(b, s);
            if (e == hipSuccess)
                e = launch_reduce(b, fit, nullptr, s);
            if (e == hipSuccess)
                e = launch_argmin(fit, cnt, bc, bi, s);
            if (e == hipSuccess)
                e = launch_fold(bc, bi, (cnt + 255) / 256, r0, run, s);
        }
        unsigned long long res[2] = {0, 0};
        uint32_t herr = 0;
        if (e == hipSuccess)
            e = hipMemcpyAsync(res, run, sizeof res, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(&herr, inst->err, sizeof herr, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess)
            e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            st = fail(PMP_EDEVICE, "enumeration: %s", hipGetErrorString(e));
            break;
        }
        st = status_from_err(herr);
        if (st != PMP_OK)
            break;
        if (best_cost)
            *best_cost = (int64_t)res[0];
        if (best_mask) {
            // the winning rank, unranked on the host
            for (int w = 0; w < W; ++w)
                best_mask[w] = 0;
            unsigned long long r = res[1];
            int xx = 0;
            for (int i = 0; i < p; ++i) {
                for (;;) {
                    const unsigned long long c = binom[(size_t)(m - xx - 1) * (p + 1) + (p - i - 1)];
                    if (r < c)
                        break;
                    r -= c;
                    ++xx;
                }
                best_mask[xx >> 6] |= 1ull << (xx & 63);
                ++xx;
            }
        }
    } while (0);
    dfree(d_binom);
    dfree(fit);
    dfree(bc);
    dfree(bi);
    dfree(run);
    dfree(masks);
    dfree(part);
    return st;
}

}  // extern "C"
