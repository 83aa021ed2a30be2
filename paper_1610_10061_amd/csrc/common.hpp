// Shared definitions of the gfx950 p-median library: device state layout,
// error bits, kernel argument blocks and the internal launcher interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pmp.h"

namespace pmp {

// Error bits of an instance's device error word.
enum : uint32_t {
    ERR_NEGATIVE_DISTANCE = 1u << 0,  // some d_ij < 0
    ERR_POPCOUNT = 1u << 1,           // a chromosome without exactly p ones
    ERR_STRAY_BITS = 1u << 2,         // bits set at positions >= m
    ERR_SCAN_OVERRUN = 1u << 3,       // no open facility in a truncated row
    ERR_BARRIER_TIMEOUT = 1u << 4,    // a grid barrier waited past its bound
    ERR_HASH_TABLE = 1u << 5,         // reduced polynomial: no free slot
    ERR_HASH_COLLISION = 1u << 6,     // reduced polynomial: two sets, one key
};

// Device GA run state: 64-bit words.
enum GaSlot : int {
    GS_GEN = 0,   // generations run
    GS_SAT = 1,   // generations since the last strict improvement
    GS_DONE = 2,  // 1 once stopped
    GS_BEST = 3,  // global best cost
    GS_COUNT = 8
};

// Tables of one preprocessed instance (device pointers).
struct Tables {
    const uint16_t *pi;  // n x pitch, facility order (first K valid)
    const int32_t *ds;   // n x pitch, sorted distances D'
    int32_t n, m, p, K, W, pitch;
};

// One population evaluation (Eq. (6) by the walk of Section 4.2).  Output:
// part[ti * P + c] = chromosome c's cost summed over the clients of client
// tile ti (and spart the summed scan lengths), written for active c only.
struct EvalArgs {
    Tables t;
    const uint64_t *masks;            // P x W
    int32_t P;
    const uint8_t *active;            // optional: evaluate c only if active[c]
    unsigned long long *part;         // tiles_i x P partial costs
    uint32_t *spart;                  // optional tiles_i x P partial scan lengths
    const unsigned long long *done;   // optional: skip everything when *done
    uint32_t *err;                    // error word
    int32_t clients_per_block;
    int32_t tiles_c;                  // ceil(P / 64)
    int32_t tiles_i;                  // ceil(n / clients_per_block)
    // reduced-polynomial walk (k_hbp.hip), else null: row lengths K_i and
    // the int64 running sums replacing t.ds; c0 is added to every fitness
    const int32_t *rlen;
    const long long *e64;
    long long c0;
    // very short scans expected (m + 1 <= 4 (p + 1)): two clients per chunk
    int32_t paired;
    // waves per workgroup of k_eval: 4 (0 means 4), 8 or 16
    int32_t waves;
    // chromosomes wider than LDS staging allows (W > kMaxStagedWords): the
    // tiles' facility-major copies in device memory (tile tc at
    // tg + tc * tg_stride: 64 W words, then an all-zero and an all-ones word),
    // made and checked beforehand (launch_tile_major)
    const uint64_t *tg;
    int64_t tg_stride;
    // partial sums chromosome-major (part[c * tiles_i + ti]) instead of
    // tile-major (part[ti * P + c]): the fused crossover stages, whose
    // readers add up one chromosome's tiles at a time
    int32_t pcm;
};

// Widest chromosome the evaluation stages in LDS (words); wider ones use a
// facility-major copy in device memory.
constexpr int kMaxStagedWords = PMP_MAX_FACILITIES / 64;  // 128

// Reduced polynomial construction (k_hbp.hip).  t: the instance's tables.
struct HbpArgs {
    Tables t;
    uint64_t *key;                 // n x pitch term keys (0: zero term)
    int32_t *slot_of;              // n x pitch table slot of each term
    uint16_t *posinv;              // n x m position in the row (0xFFFF past K)
    uint64_t *slot_key;            // table: key (0 = free)
    int32_t *slot_row, *slot_tmin, *slot_tmax;
    unsigned long long *slot_sum;
    uint64_t mask;                 // table size - 1 (a power of two)
    long long *charged;            // n x pitch owned coefficient (0: none)
    long long *esum;               // n x pitch running sums of charged
    int32_t *rlen_full, *owned;    // per row: K_i, owned terms
    int32_t *maxlen;               // max K_i
    int32_t *kept_at, *term_at;    // per row: compacted row, first term
    int32_t *tot;                  // kept rows, terms
    uint16_t *rpi;                 // kept rows x rpitch walk order
    long long *re;                 // kept rows x rpitch running sums
    int32_t *rlen;                 // kept rows: K_i
    int32_t rpitch;
    int32_t *term_row, *term_deg;  // owned terms, row by row
    long long *term_coef;
    unsigned long long *npos;      // positive terms
    unsigned long long *c0;        // constant: sum of the rows' first terms
    uint32_t *err;
};
hipError_t launch_hbp_keys(const HbpArgs &h, hipStream_t s);
hipError_t launch_hbp_table(const HbpArgs &h, hipStream_t s);
hipError_t launch_hbp_emit(const HbpArgs &h, hipStream_t s);

// Index of the calling wave in its workgroup, as a wave-uniform (scalar)
// value: derived from threadIdx.x the compiler cannot prove it uniform and
// would keep everything computed from it in vector registers.
__device__ __forceinline__ int wave_id()
{
    return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

constexpr int kMaxPersistentBlocks = 4096;
constexpr int kBarrierWords = 32 * (kMaxPersistentBlocks + 1);

constexpr int kEvalTile = 64;     // chromosomes per block (one per lane)
constexpr int kEvalWaves = 4;     // waves per block

// Launchers (each lives with its kernels).
hipError_t launch_sort_rows(const int32_t *d, int64_t ld, int32_t n, int32_t m,
                            int32_t K, int32_t pitch, uint16_t *pi,
                            int32_t *delta, int32_t *ds, uint32_t *err,
                            hipStream_t s);
// e0/e1 (optional) are recorded at the kernel's start and end.
// Workgroups of the evaluation kernel for W words per chromosome (reduced
// or paired walk) that one CU holds at once.
int eval_workgroups_per_cu(int W, bool reduced, bool paired, int waves = kEvalWaves);
hipError_t launch_eval(const EvalArgs &a, hipStream_t s, hipEvent_t e0 = nullptr,
                       hipEvent_t e1 = nullptr);
hipError_t launch_reduce(const EvalArgs &a, unsigned long long *fitness,
                         unsigned long long *scan, hipStream_t s);
// Facility-major copies of the chromosome tiles of a.masks into tg (a.P
// chromosomes, a.t.W words each) and the feasibility check of every
// chromosome (error bits into a.err).
hipError_t launch_tile_major(const EvalArgs &a, uint64_t *tg, hipStream_t s);
// Rows wider than PMP_MAX_FACILITIES: the sort in device memory, `batch`
// rows at a time in `scratch` (batch x m2 keys, m2 = m rounded up to a power
// of two).
int wide_sort_rows_per_batch(int32_t m);
hipError_t launch_sort_rows_wide(const int32_t *d, int64_t ld, int32_t n, int32_t m,
                                 int32_t K, int32_t pitch, uint16_t *pi, int32_t *delta,
                                 int32_t *ds, uint32_t *err, uint64_t *scratch, int32_t batch,
                                 hipStream_t s);
hipError_t launch_zero(void *p, size_t bytes, hipStream_t s);
// The other thread mappings of the evaluation (k_eval_schemes.hip).
hipError_t launch_eval_per_chromosome(const EvalArgs &a, unsigned long long *fitness,
                                      unsigned long long *scan, hipStream_t s);
hipError_t launch_eval_per_client(const EvalArgs &a, hipStream_t s);
// All-pairs shortest paths (k_apsp.hip) on a padded uint32 work matrix.
int apsp_padded(int n);
hipError_t launch_apsp_in(const int32_t *w, int64_t ldw, int n, uint32_t *D, uint32_t *wmax,
                          hipStream_t s);
hipError_t launch_apsp_rounds(uint32_t *D, int n, hipStream_t s);
hipError_t launch_apsp_out(const uint32_t *D, int n, int32_t *d, int64_t ldd, hipStream_t s);

// Per-chromosome GA counters (summed on the host when read).
enum GaStat : int {
    CS_EVALS = 0,      // evaluations of this slot's chromosomes
    CS_SCAN = 1,       // Pi' entries those evaluations read
    CS_XO_FAIL = 2,    // crossovers without offspring
    CS_XO_TAKEN = 3,   // crossover offspring taken
    CS_MUT_TAKEN = 4,  // mutants taken
    CS_SWAP_TRIED = 5, // scored swaps evaluated
    CS_SWAP_TAKEN = 6, // scored swaps taken
    CS_SPEC_EVALS = 7, // mutants evaluated past the cycle's first improvement
    CS_SPEC_SCAN = 8,  // Pi' entries those evaluations read
    CS_COUNT = 9
};

// A run's report, gathered on the device so that the host reads it in one
// copy: the run state, the counters summed over the population, the error
// words (OR-ed), the best mask.
enum GaReport : int {
    RP_GS = 0,
    RP_TOT = RP_GS + GS_COUNT,
    RP_ERR = RP_TOT + CS_COUNT,
    RP_MASK = RP_ERR + 1  // then W words
};

// Kinds of the operator a stage kernel finishes (prev) and starts (op).
// OP_MUT_ALL: every attempt of the mutation cycle at once (the mutants of
// one parent; see ga_resolve_one).
enum GaOp : int { OP_NONE = 0, OP_INIT = 1, OP_XOVER = 2, OP_MUT = 3, OP_SWAP = 4, OP_MUT_ALL = 5 };

// Largest mutation cycle evaluated at once (lanes of a wave).
constexpr int kMaxSpec = 64;

// Operator finished (prev) and started (op) by stage step k of a generation
// with X crossover stages and S = X + Y stages, of which the first L
// mutation attempts take scored swaps; and the operator's index.
__device__ __host__ __forceinline__ int ga_stage_kind(int k, int X, int L)
{
    return k < X ? OP_XOVER : (k - X < L ? OP_SWAP : OP_MUT);
}

__device__ __host__ __forceinline__ void ga_stage_ops(int k, int X, int S,
                                                      int *prev, int *op,
                                                      int *index, int L = 0)
{
    *prev = k == 0 ? OP_INIT : ga_stage_kind(k - 1, X, L);
    *op = k == S ? OP_NONE : ga_stage_kind(k, X, L);
    *index = k < X ? k : k - X;
}

// The random draws of one operator application: crossover (a, b) = (r1,
// quota); mutation (a, b, c) = (lo, hi, move) of the rotated range.
struct __align__(16) OpDraw {
    int32_t a, b, c, d;
};

// Device state of one GA run.  Population, fitness, offspring and their
// "evaluate me" flags are double-buffered: a stage kernel reads buffer `in`
// and writes buffer `in ^ 1`, so every chromosome (and its crossover partner)
// is read as the previous stage left it.
struct GaArgs {
    Tables t;
    uint64_t seed;
    int32_t P, NT, NB, lg, X, Y, generations, saturation;
    int32_t migration;              // PMP_MIG_SAME_BLOCK or PMP_MIG_ONE_BLOCK
    int32_t init_rank;              // fresh chromosomes by lexicographic rank
    const unsigned long long *binom;// with init_rank: C(a, b) at a (p + 1) + b, a < m, b <= p
    uint64_t nsets;                 // with init_rank: C(m, p), below 2^63
    OpDraw *draws;                  // P x (X + Y) draws of this generation:
                                    // crossover stage k at k, mutation
                                    // attempt a at X + a
    // the mutation cycle evaluated at once: mutant a of chromosome c at
    // row c Y + a (P Y x W), its "differs from the parent" flag, and the
    // evaluation's partial sums (TI x P Y)
    uint64_t *mut;
    uint8_t *mut_ok;
    const unsigned long long *mpart;
    const uint32_t *mspart;
    int32_t TIm;                    // client tiles of the mutants' evaluation
    int32_t mpw;                    // mutants made per wave (>= 1)
    uint64_t *cur[2];               // P x W population
    unsigned long long *fit[2];     // P fitness of cur
    uint64_t *off[2];               // P x W offspring
    uint8_t *ok[2];                 // P: offspring exists and is evaluated
    uint8_t *improved;              // P: mutation cycle already succeeded
    const unsigned long long *part; // TI x P partial costs of the last evaluation
    const uint32_t *spart;          // TI x P partial scan lengths
    int32_t TI;                     // client tiles of the evaluation
    int32_t pcm;                    // part/spart chromosome-major (P x TI)
    uint64_t *gmask;                // NB x W group bests (migrants)
    unsigned long long *gcost;      // NB
    uint64_t *best_mask;            // W
    unsigned long long *gs;         // GS_COUNT run state
    unsigned long long *cstat;      // P x CS_COUNT counters
    uint32_t *arrive;               // group-best arrival counter
    uint32_t *bar;                  // grid barrier: epoch word, then one
                                    // flag per workgroup (32 words apart)
    uint32_t *err;
    // learned proposal (L = 0: none): the first L mutation attempts take
    // the swaps listed in `swaps` (P x L pairs j, k); each evaluated swap's
    // exact change of cost goes to the replay ring slot
    // ((generation mod H) L + attempt) P + chromosome.
    const int32_t *swaps;
    float *rep_t, *rep_w;           // normalised target, row weight (0/1)
    long long *rep_d;               // change of cost, parent cost
    int32_t L, H;
};

// Exhaustive enumeration (k_enum.hip).
hipError_t launch_unrank(const unsigned long long *binom, int m, int p, int W,
                         unsigned long long r0, int count, uint64_t *masks, hipStream_t s);
hipError_t launch_argmin(const unsigned long long *fit, int count, unsigned long long *best_cost,
                         int *best_idx, hipStream_t s);
hipError_t launch_fold(const unsigned long long *bc, const int *bi, int nblk,
                       unsigned long long r0, unsigned long long *run, hipStream_t s);

hipError_t launch_ga_init(const GaArgs &g, hipStream_t s);
// A crossover stage fused with the evaluation of its offspring (a: the
// evaluation's arguments; e0/e1 optional events stamped by the dispatch),
// for chromosomes of W <= 16 words (ga_stage_eval_fits).
bool ga_stage_eval_fits(int W);
hipError_t launch_ga_stage_eval(const GaArgs &g, const EvalArgs &a, int in, int prev,
                                int index, hipStream_t s, hipEvent_t e0 = nullptr,
                                hipEvent_t e1 = nullptr);
hipError_t launch_ga_stage(const GaArgs &g, int in, int prev, int op,
                           int index, hipStream_t s);
hipError_t launch_ga_best(const GaArgs &g, int fb, hipStream_t s, bool place_migrants = false);
hipError_t launch_ga_resolve(const GaArgs &g, int in, int out, hipStream_t s);
// launch_ga_resolve plus the next generation's population and draws
// (k_init's work) in the same launch; launch_ga_best must then place the
// migrants.  Only when the resolve reads and writes buffer 1.
hipError_t launch_ga_resolve_init(const GaArgs &g, int in, int out, hipStream_t s);
// The report (GaReport layout) into out; err1 may be null.
hipError_t launch_ga_report(const GaArgs &g, const uint32_t *err0, const uint32_t *err1,
                            unsigned long long *out, hipStream_t s);
// One instance of a batched (persistent) GA launch: its GA state and its
// evaluation tiling, with its offsets in the batch's global item ranges.
struct BatchItem {
    GaArgs g;
    EvalArgs e;       // masks / active are set per phase by the kernel
    int32_t X, S;     // crossover stages run, all stages (X + Y)
    int32_t fb;       // buffer holding the population after the last stage
};

struct BatchArgs {
    const BatchItem *items;
    const int32_t *chrom0;  // count + 1 prefix offsets of chromosomes
    const int32_t *tile0;   // ... of evaluation tiles
    const int32_t *group0;  // ... of groups
    // the run of every chromosome, evaluation tile and group of the batch
    const int32_t *chrom_run, *tile_run, *group_run;
    int32_t count, max_S;
    uint32_t *bar;          // grid barrier: epoch word, then one flag per
                            // workgroup (32 words apart)
    uint32_t *err;          // batch error word (barrier time-outs)
};

// One cooperative launch running `generations` generations of every
// instance of the batch.  max_blocks > 0 caps the grid; the grid used is
// returned.  max_w2 = largest 2*W of the batch (LDS sizing).
hipError_t launch_ga_batch(const BatchArgs &b, int generations, int max_w2,
                           int max_blocks, int want_blocks, hipStream_t s,
                           int *grid, bool cooperative);
// Events that bracket the batch-wide evaluation launches (profiling): pairs
// events[*used], events[*used + 1] while *used + 2 <= cap; none when null.
struct BatchEvents {
    hipEvent_t *events = nullptr;
    int cap = 0;
    int *used = nullptr;
};
// The same generations as a sequence of batch-wide kernels (one per phase).
hipError_t launch_ga_batch_kernels(const BatchArgs &b, int nchrom, int ntiles,
                                   int ngroups, int generations, int max_w2,
                                   hipStream_t s, const BatchEvents &ev = BatchEvents{});
// One batch-wide evaluation of every run's current population (buffer 0),
// as the first evaluation of a generation does (the batch autotuner's probe).
hipError_t launch_ga_batch_eval(const BatchArgs &b, int ntiles, int max_w2, hipStream_t s);

}  // namespace pmp
