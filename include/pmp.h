/*
 * pmp.h - C ABI of the MI355X (gfx950) p-median hot path.
 *
 * Method: AlBdaiwi & AboElFotoh, "A GPU-Based Genetic Algorithm for the
 * P-Median Problem" (arXiv 1610.10061).  An instance is an n x m matrix of
 * non-negative distances d_ij between client i and facility j and an integer
 * 0 < p < m (Section 1, Eq. (1)-(3)).  A chromosome is m bits, bit j set when
 * facility j is open (Section 4.1).
 *
 * Conventions for every entry point
 *  - Indices are 0-based (the paper's are 1-based).
 *  - Every call returns a pmp_status; nothing throws across the ABI.  On
 *    failure pmp_last_error() gives a thread-local message.
 *  - Chromosome masks are P x W little-endian uint64 words, W = ceil(m/64),
 *    row-major; bit j of word j/64 is facility j; bits at positions >= m
 *    must be zero.
 *  - Flags: PMP_ON_DEVICE says pointer arguments are device pointers and the
 *    work is enqueued on `stream` (a hipStream_t, NULL = default stream);
 *    without it pointers are host pointers and the call returns when the
 *    results are in host memory.  PMP_ASYNC (with PMP_ON_DEVICE) skips the
 *    final stream wait: errors found on the device are then kept in the
 *    instance's error word until pmp_instance_check().
 *  - Handles own all device memory they allocate until *_destroy.  Input
 *    buffers are borrowed for the duration of the call (for asynchronous
 *    calls: until the enqueued work has run); outputs go to caller buffers.
 *  - Handles are not thread-safe: calls on one handle must not overlap.
 */
#ifndef PMP_H
#define PMP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define PMP_API __attribute__((visibility("default")))
#else
#define PMP_API
#endif

typedef enum {
    PMP_OK = 0,
    PMP_EINVAL = 1,       /* bad argument: sizes, null pointers, d < 0, ... */
    PMP_ENOMEM = 2,       /* device or host allocation failed */
    PMP_EDEVICE = 3,      /* a HIP call failed; see pmp_last_error() */
    PMP_EINFEASIBLE = 4,  /* a chromosome without exactly p open facilities */
    PMP_EUNSUPPORTED = 5  /* a size or mode the library does not handle for that call */
} pmp_status;

#define PMP_ON_DEVICE 1u
#define PMP_ASYNC 2u
/* Thread mappings of pmp_eval_population other than the default tiled one
 * (at most one of them): one thread per chromosome walking every client, or
 * one thread per (client, chromosome) pair - the paper's "n threads"
 * scenario (Section 5, the observation on the Fitness bottleneck).  Same
 * results; kept to measure the load-balance argument. */
#define PMP_EVAL_PER_CHROMOSOME 4u
#define PMP_EVAL_PER_CLIENT 8u

/* Largest m of an instance: facility indices of Pi' are 16-bit. */
#define PMP_MAX_EVAL_FACILITIES 65535
/* Largest m of the GA, the reduced polynomial, the enumeration and the other
 * evaluation schemes (their kernels hold a tile of 64 chromosomes, or a
 * chromosome per wave, on chip: 64 x 1 KiB at m = 8192).  Preprocessing and
 * the tiled evaluation take wider instances: rows are then sorted in device
 * memory and the chromosome tiles are turned facility-major in device
 * memory (L2-resident) instead of LDS. */
#define PMP_MAX_FACILITIES 8192

typedef struct pmp_instance pmp_instance;
typedef struct pmp_ga pmp_ga;

/* ---------------------------------------------------------------------------
 * pmp_preprocess - Section 2.1 and Section 3.1 host step 3: for every client
 * i, the ordering Pi^i of the facilities by d_i. ascending (equal distances
 * ordered by lower facility index, the order Example 1 prints) and the gap
 * terms Delta^i (delta_i1 = d_{i pi_i1}, delta_ir = d_{i pi_ir} -
 * d_{i pi_i(r-1)}), both truncated to their first K = m - p + 1 columns, the
 * truncation argued after Eq. (6).  The sorted distances D'_ik = d_{i pi_ik}
 * (the running sums of Delta') are kept too; the evaluation reads them.
 *
 *  d       n x m int32, row stride ld >= m elements; host pointer, or device
 *          pointer with PMP_ON_DEVICE.  Copied; not kept.
 *  n, m, p 1 <= n, 2 <= m <= PMP_MAX_EVAL_FACILITIES, 1 <= p <= m - 1.
 *  flags   PMP_ON_DEVICE; with it, PMP_ASYNC (see below).
 *  out     receives a new instance handle (device tables, owned).
 * Errors: PMP_EINVAL for sizes (m above PMP_MAX_EVAL_FACILITIES included),
 * null pointers, PMP_ASYNC without PMP_ON_DEVICE, or any d_ij < 0 (the paper
 * assumes non-negative distances).
 * Rows wider than PMP_MAX_FACILITIES are sorted in device memory (a scratch
 * of up to 256 MB of keys, freed before returning).
 * Waits for its stream before returning, except with PMP_ASYNC: the tables
 * are then made on `stream` after the call returns (d must stay valid until
 * they are), negative distances are recorded in the instance's error word
 * for pmp_instance_check, and the sum of d (a learned-proposal feature) is
 * read back when first needed.  Many instances then preprocess back to
 * back on the device.
 * ------------------------------------------------------------------------- */
PMP_API pmp_status pmp_preprocess(const int32_t *d, int64_t ld, int32_t n, int32_t m,
                          int32_t p, uint32_t flags, void *stream,
                          pmp_instance **out);

/* Sizes of an instance: n, m, p, K = m - p + 1 and W = ceil(m/64).  Any
 * output pointer may be NULL. */
PMP_API pmp_status pmp_instance_info(const pmp_instance *inst, int32_t *n, int32_t *m,
                             int32_t *p, int32_t *K, int32_t *W);

/* Copy the truncated tables out (Section 2.1): pi (uint16), delta and
 * dsorted (int32), each n x K row-major.  NULL outputs are skipped.  Host
 * pointers, or device pointers with PMP_ON_DEVICE. */
PMP_API pmp_status pmp_instance_tables(const pmp_instance *inst, uint16_t *pi,
                               int32_t *delta, int32_t *dsorted,
                               uint32_t flags, void *stream);

/* ---------------------------------------------------------------------------
 * pmp_eval_population - Eq. (6) for every chromosome of a population, the
 * Fitness function of Section 4.2: for chromosome c and client i, walk
 * Pi'_i to the first open facility, position s*_{c,i} (1-based); the
 * client's cost is D'_{i,s*} (= the sum of the first s* gap terms), and
 *     fitness[c] = sum_i D'_{i, s*_{c,i}}   (int64, exact).
 *
 *  masks       P x W uint64 chromosomes (see conventions).
 *  P           >= 0 chromosomes.
 *  fitness     P int64 outputs.
 *  scan_total  optional (NULL = skip): P int64 outputs, sum_i s*_{c,i}, the
 *              number of Pi' entries the walk reads for chromosome c.
 *  flags       PMP_ON_DEVICE, PMP_ASYNC, and at most one of
 *              PMP_EVAL_PER_CHROMOSOME / PMP_EVAL_PER_CLIENT.
 * Errors: PMP_EINFEASIBLE if a chromosome's popcount is not p or it has bits
 * at positions >= m (the truncated walk is defined only for exactly p open
 * facilities); its fitness is then unspecified.  With PMP_ASYNC the error is
 * only recorded in the instance (see pmp_instance_check).  PMP_EINVAL for
 * both scheme flags at once; PMP_EUNSUPPORTED for a scheme flag when m >
 * PMP_MAX_FACILITIES.  For m > PMP_MAX_FACILITIES the instance keeps a device
 * buffer of the tiles' facility-major copies (P x W words, grown on demand).
 * ------------------------------------------------------------------------- */
PMP_API pmp_status pmp_eval_population(pmp_instance *inst, const uint64_t *masks,
                               int32_t P, int64_t *fitness,
                               int64_t *scan_total, uint32_t flags,
                               void *stream);

/* ---------------------------------------------------------------------------
 * pmp_eval_population_noalloc - pmp_eval_population (default tiled scheme)
 * for callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  It calls
 * no hipMalloc, hipFree or allocating library routine.  The evaluation's
 * client-tile partial sums go to a fixed workspace compiled into the
 * library (a static device array of PMP_NOALLOC_CELLS 12-byte cells, 6 MiB,
 * one copy on each GPU the library runs on, held until the process ends).
 *
 *  inst, masks, P, fitness, scan_total: as pmp_eval_population.
 *  flags   must hold PMP_ON_DEVICE (masks, fitness, scan_total are device
 *          pointers on `stream`); PMP_ASYNC as pmp_eval_population; no
 *          scheme flag.
 * Client tiles are widened when needed so that (client tiles) x P fits the
 * workspace; the results do not depend on the tiling (exact integer sums).
 * Errors: PMP_EINVAL for P > PMP_NOALLOC_CELLS, host pointers (no
 * PMP_ON_DEVICE) or a scheme flag; PMP_EUNSUPPORTED when scan_total is asked
 * for and a widened tile's scan sums could pass 2^32, or for m >
 * PMP_MAX_FACILITIES; otherwise as pmp_eval_population.  Every call on one GPU uses that GPU's workspace:
 * calls that overlap on one GPU (two streams, two threads) race and give
 * wrong results; the caller serialises them.  Nothing in the workspace
 * needs clearing between calls (every cell read is written first).
 * ------------------------------------------------------------------------- */
#define PMP_NOALLOC_CELLS (1 << 19)
PMP_API pmp_status pmp_eval_population_noalloc(pmp_instance *inst, const uint64_t *masks,
                                               int32_t P, int64_t *fitness,
                                               int64_t *scan_total, uint32_t flags,
                                               void *stream);

/* ---------------------------------------------------------------------------
 * The reduced Hammer-Beresnev polynomial (Section 2.1, after Eq. (6); Example
 * 1 reduces 15 terms to 7).  Term t >= 1 of client i has coefficient
 * Delta'_{i,t} and the monomial "the first t facilities of row i are all
 * closed" (0-based t); monomials are sets, so equal sets from different
 * clients merge into one term with the summed coefficient, and sets whose
 * coefficients are all 0 drop out.  The constant is sum_i Delta'_{i,0}.
 *
 * pmp_hbp_reduce builds it on the device from an instance's tables.  Each
 * merged term is charged to the lowest client row holding it with a
 * positive coefficient; row i keeps its first K_i positions, K_i - 1 being
 * the highest degree it is charged (rows charged nothing are dropped), so
 * that the polynomial is evaluated as walks: a kept row costs the running
 * sum of its charged coefficients up to min(first open position, K_i - 1),
 * and the cost is the constant plus the kept rows' costs - equal to Eq. (1)
 * for every feasible chromosome.  Sets are merged by 64-bit keys and every
 * merge is then checked exactly; a key collision (never expected) makes the
 * call fail with PMP_EUNSUPPORTED rather than merge different sets.
 *
 *  inst    a preprocessed instance (borrowed: it must outlive the handle).
 *  out     receives the handle (device tables, owned).
 * Errors: PMP_EINVAL (null), PMP_EUNSUPPORTED (key collision),
 * PMP_ENOMEM.  Waits for its stream.
 * ------------------------------------------------------------------------- */
typedef struct pmp_hbp pmp_hbp;
PMP_API pmp_status pmp_hbp_reduce(pmp_instance *inst, void *stream, pmp_hbp **out);

/* constant, number of non-constant monomials, kept rows and the longest
 * kept row (any pointer may be NULL). */
PMP_API pmp_status pmp_hbp_info(const pmp_hbp *h, int64_t *constant, int64_t *monomials,
                                int32_t *rows, int32_t *max_len);

/* The monomials as (row, degree, coefficient), row by row and by degree
 * within a row (the monomial is the set of the row's first `degree`
 * facilities), and K_i of every client row (n entries; 0 = dropped).  Each
 * output may be NULL; host pointers, or device pointers with PMP_ON_DEVICE.
 * Waits for its stream. */
PMP_API pmp_status pmp_hbp_terms(const pmp_hbp *h, int32_t *row, int32_t *degree,
                                 int64_t *coef, int32_t *row_len, uint32_t flags,
                                 void *stream);

/* The reduced polynomial at every chromosome of a population: arguments,
 * flags and errors as pmp_eval_population (no scheme flags); scan_total
 * counts the positions the truncated walks read. */
PMP_API pmp_status pmp_hbp_eval(pmp_hbp *h, const uint64_t *masks, int32_t P,
                                int64_t *fitness, int64_t *scan_total, uint32_t flags,
                                void *stream);
PMP_API void pmp_hbp_destroy(pmp_hbp *h);

/* ---------------------------------------------------------------------------
 * pmp_apsp - all-pairs shortest path lengths of a weighted directed graph
 * (blocked Floyd-Warshall on the device): the distance matrix of a graph
 * instance (the p-median benchmarks the paper uses give graphs, whose cost
 * d_ij is the length of a shortest path from i to j), ready for
 * pmp_preprocess.
 *
 *  w       n x n int32 weights, row stride ldw >= n: w_ij >= 0 is an arc
 *          i -> j (an undirected edge is two arcs), w_ij < 0 no arc; the
 *          diagonal is taken as 0.  Host pointer, or device pointer with
 *          PMP_ON_DEVICE.  Not modified.
 *  d       n x n int32 output, row stride ldd >= n (same memory kind as w):
 *          d_ij = length of a shortest path from i to j, or -1 if there is
 *          none.  d may not overlap w.
 *  n       1 <= n <= 32768.
 * The library keeps one padded n x n work matrix per device between calls
 * (grown on demand, held until the process ends); calls are serialised.
 * Errors: PMP_EINVAL for null pointers, n or strides out of range;
 * PMP_EUNSUPPORTED when (n - 1) * (largest weight) >= 2^31 - 1 (a path
 * length might not fit int32); PMP_ENOMEM.  Always waits for its stream.
 * ------------------------------------------------------------------------- */
PMP_API pmp_status pmp_apsp(const int32_t *w, int64_t ldw, int32_t n, int32_t *d,
                            int64_t ldd, uint32_t flags, void *stream);

/* Wait for `stream`, then return and clear the errors recorded on the device
 * by asynchronous calls on this instance (PMP_EINFEASIBLE or PMP_EINVAL). */
PMP_API pmp_status pmp_instance_check(pmp_instance *inst, void *stream);

PMP_API void pmp_instance_destroy(pmp_instance *inst);

/* ---------------------------------------------------------------------------
 * The genetic algorithm of Section 3 (host steps 7-16 around each Evolve call,
 * Evolve steps 1-8), with the operators of Section 4.  One generation:
 *  1. population: a uniform random p-subset in every slot (Section 4.1), but
 *     from the second generation on the group bests of the previous
 *     generation migrate (Section 4.5): group b's best to slot b*NT (the same
 *     block; default) or, with PMP_MIG_ONE_BLOCK, to slot b (the team of
 *     bests in one block, or the first ones when NB > NT);
 *  2. fitness of all (pmp_eval_population's kernel);
 *  3. crossover stages k = 0..X-1, stride NT >> (1 + k mod lg NT); slot t
 *     of a group pairs with t XOR stride; the pair's lower slot draws
 *     r1 in [0, m) and i in [1, floor(p/2)]; each partner forms its offspring
 *     from both parents as they were when the stage began (Section 4.3) and
 *     takes it if strictly fitter;
 *  4. up to Y mutation attempts (circular or block shift, Section 4.4),
 *     stopping at a chromosome's first strict improvement;
 *  5. group best (least fitness, lowest slot on ties; Evolve steps 7-8);
 *  6. global best, saturation count (reset on strict improvement), stop at
 *     S generations without improvement (S > 0) or at `generations`
 *     (EvolveLimit) generations (host steps 13-15).
 * All random choices come from Philox4x64-10 counter streams keyed by
 * (seed, role) and addressed by (generation, chromosome, tag, stage), so a
 * run is reproducible bit for bit and independent of launch shapes.
 * ------------------------------------------------------------------------- */
/* Migration variants (Section 4.5). */
#define PMP_MIG_SAME_BLOCK 0  /* group b's best -> slot b*NT (its own block) */
#define PMP_MIG_ONE_BLOCK 1   /* all group bests -> slots 0..NB-1 (one block) */
/* Generation of fresh chromosomes (Section 4.1). */
#define PMP_INIT_SUBSET 0     /* a uniform p-subset by Floyd's method */
#define PMP_INIT_RANK 1       /* a uniform rank below C(m, p), unranked in
                                 lexicographic order; needs C(m, p) < 2^63 */

typedef struct {
    uint64_t seed;
    int32_t population;       /* P = NB x NT */
    int32_t group_size;       /* NT: a power of two dividing P, <= 1024 */
    int32_t generations;      /* EvolveLimit, >= 1 */
    int32_t saturation;       /* S; 0 = off */
    int32_t crossover_iters;  /* X; 0 = lg NT */
    int32_t mutation_iters;   /* Y; 0 = lg NT */
    int32_t migration;        /* PMP_MIG_SAME_BLOCK (0) or PMP_MIG_ONE_BLOCK */
    int32_t init;             /* PMP_INIT_SUBSET (0) or PMP_INIT_RANK */
} pmp_ga_params;

typedef struct {
    int64_t generations;       /* generations run so far */
    int64_t saturation_count;  /* generations since the last improvement */
    int64_t done;              /* 1 once stopped */
    int64_t best_cost;         /* INT64_MAX before the first generation */
    int64_t chromosome_evals;  /* chromosomes evaluated */
    int64_t crossover_fail;    /* crossover operations with no offspring */
    int64_t crossover_taken;   /* offspring that replaced a parent */
    int64_t mutation_taken;    /* mutants that replaced a parent */
    int64_t scan_total;        /* Pi' entries read by all evaluations */
    int64_t pair_evals;        /* chromosome_evals x n */
    int64_t swap_tried;        /* scored swaps evaluated (learned proposal) */
    int64_t swap_taken;        /* scored swaps that replaced a parent */
    int64_t speculative_evals; /* mutants evaluated beyond the ones above: the
                                  per-step schedule evaluates a whole mutation
                                  cycle at once, also the attempts after its
                                  first improvement (results unchanged) */
} pmp_ga_stats;

/* Create a GA run on an instance (the instance must outlive it).
 * PMP_EINVAL: P < 1, NT not a power of two, NT > 1024, P % NT != 0,
 * generations < 1, negative counts, unknown migration or init.
 * PMP_EUNSUPPORTED: PMP_INIT_RANK with C(m, p) >= 2^63, or m >
 * PMP_MAX_FACILITIES. */
PMP_API pmp_status pmp_ga_create(pmp_instance *inst, const pmp_ga_params *params,
                         pmp_ga **out);

/* Enqueue `generations` more generations on `stream` (asynchronous).  Once
 * the run has stopped, further generations do nothing. */
PMP_API pmp_status pmp_ga_step(pmp_ga *ga, int32_t generations, void *stream);

/* Wait for `stream`; copy the best chromosome (W words, host), its cost and
 * the counters.  NULL outputs are skipped. */
PMP_API pmp_status pmp_ga_best(pmp_ga *ga, uint64_t *mask, int64_t *cost,
                       pmp_ga_stats *stats, void *stream);

/* Wait for `stream`; copy the state (host pointers; NULL = skip): the
 * population (P x W) and its fitness (P) as the last generation left them,
 * the group bests (NB x W masks, NB costs). */
PMP_API pmp_status pmp_ga_state(pmp_ga *ga, uint64_t *population, int64_t *fitness,
                        uint64_t *group_masks, int64_t *group_costs,
                        void *stream);

PMP_API void pmp_ga_destroy(pmp_ga *ga);

/* ---------------------------------------------------------------------------
 * pmp_ga_autotune (not in the paper) - choose the evaluation tile of a run
 * in two dimensions: how many clients one workgroup of the evaluation
 * kernel takes (its 64 chromosomes are fixed, one per lane), and how many
 * waves (4, 8 or 16) share that workgroup's staged chromosome tile.  The
 * shape's default is timed first, then every pair of candidate clients (4,
 * 8, 12, ..., 512) and waves, on a generation-0 population of this run with
 * HIP events; a pair replaces the default only when at least 3 % faster.
 * The choice is remembered for runs of similar shape (n, m/p, W, P) in this
 * process.  Results do not depend on it (integer sums).  Call it before the
 * first pmp_ga_step and before adding the run to a batch.  `clients` and
 * `waves` (optional) receive the choice.  PMP_EINVAL after the first
 * generation.
 * ------------------------------------------------------------------------- */
PMP_API pmp_status pmp_ga_autotune(pmp_ga *ga, int32_t *clients, int32_t *waves, void *stream);

/* ---------------------------------------------------------------------------
 * Batching (not in the paper): advance many GA runs, typically on different
 * instances of uneven n, m, p, together.  Each phase of a generation
 * (population, evaluation, each crossover/mutation stage, group and global
 * bests) spreads the work items of all runs over the whole GPU; runs that
 * have stopped, or have fewer stages, sit the later phases out.  Default:
 * one batch-wide kernel per phase; PMP_BATCH_MODE=persistent: one persistent
 * kernel with grid barriers between phases.  Either way a step is captured
 * once into a hipGraph and replayed.  Every run evolves exactly as
 * pmp_ga_step would evolve it alone (same Philox streams, same decisions).
 *
 * pmp_batch_create  gas: `count` distinct GA handles (borrowed; they must
 *                   outlive the batch and must not be stepped otherwise
 *                   while a batch step is in flight).  Tune a GA
 *                   (pmp_ga_autotune) before adding it to a batch.
 * pmp_batch_step    enqueue `generations` generations of every run on
 *                   `stream`, captured once per generation count into a
 *                   hipGraph and replayed (PMP_BATCH_GRAPH=0: launched
 *                   directly, the persistent kernel cooperatively).
 *                   Asynchronous.
 * pmp_batch_autotune  choose the batch evaluation's client tiling by
 *                   timing it: every run keeps its own tuned clients per
 *                   workgroup (scaled to the batch kernel's 16 waves) unless
 *                   one common count of clients per workgroup (64 ... 512;
 *                   more for a run whose partial sums would not fit) is
 *                   faster over the whole batch; the choice goes to
 *                   `*clients` (optional; 0 = each run's own).  The probe
 *                   evaluates each run's generation-0
 *                   population (made again by the first step, identically),
 *                   so every run must be before its first generation
 *                   (PMP_EINVAL otherwise, when the choice is timed).
 *                   Choices are cached per process by the runs' shapes.  Results of the runs do not depend on
 *                   the tiling.  Synchronous on `stream`.  PMP_BATCH_CLIENTS
 *                   sets the common count without timing (also at
 *                   pmp_batch_create).
 * pmp_batch_check   wait for `stream`; PMP_EDEVICE if a grid barrier timed
 *                   out (the kernel then drains without finishing); `grid`
 *                   (optional) receives the workgroups of the last launch.
 * pmp_ga_step_batch create, step once, check, destroy.
 * Results are read per run with pmp_ga_best / pmp_ga_state.
 * ------------------------------------------------------------------------- */
typedef struct pmp_batch pmp_batch;

PMP_API pmp_status pmp_batch_create(pmp_ga *const *gas, int32_t count,
                                    pmp_batch **out);
PMP_API pmp_status pmp_batch_step(pmp_batch *batch, int32_t generations,
                                  void *stream);
PMP_API pmp_status pmp_batch_autotune(pmp_batch *batch, int32_t *clients,
                                      void *stream);
PMP_API pmp_status pmp_batch_check(pmp_batch *batch, int32_t *grid, void *stream);
PMP_API void pmp_batch_destroy(pmp_batch *batch);
PMP_API pmp_status pmp_ga_step_batch(pmp_ga *const *gas, int32_t count,
                                     int32_t generations, void *stream);

/* ---------------------------------------------------------------------------
 * pmp_solve - the whole method on host data: preprocess, run the GA to its
 * stop, return the best open set.
 *  d      n x m int32 host matrix (row stride m).
 *  open   m bytes, 1 = open (host).  cost: its objective.  stats optional.
 * ------------------------------------------------------------------------- */
PMP_API pmp_status pmp_solve(const int32_t *d, int32_t n, int32_t m, int32_t p,
                     const pmp_ga_params *params, uint8_t *open,
                     int64_t *cost, pmp_ga_stats *stats);

/* ---------------------------------------------------------------------------
 * pmp_exhaustive (not in the paper's method; its ground truth) - the exact
 * optimum of Eq. (1)-(3) over all C(m, p) open sets, on the GPU: every
 * p-subset, in lexicographic order of its sorted facility indices, is built
 * by combinadic unranking and evaluated by the kernel of
 * pmp_eval_population, in batches.
 *  best_mask  W words (host; NULL = skip): the lexicographically first open
 *             set of least cost.
 *  best_cost  its cost (host; NULL = skip).   count  C(m, p) (NULL = skip).
 * Synchronous on `stream`.  PMP_EUNSUPPORTED when C(m, p) >= 2^62.
 * ------------------------------------------------------------------------- */
PMP_API pmp_status pmp_exhaustive(pmp_instance *inst, uint64_t *best_mask, int64_t *best_cost,
                                  int64_t *count, void *stream);

/* ---------------------------------------------------------------------------
 * Profiling of the kernels that evaluate fitness inside pmp_ga_step: when
 * enabled, every launch that runs evaluations (the evaluation kernel, or the
 * persistent GA kernel that contains the whole generation) is bracketed by
 * HIP events on the GA's stream.  pmp_ga_profile_read waits for the stream
 * and returns the summed milliseconds of those launches, their number, the
 * (chromosome, client) pairs they evaluated and the algorithmic bytes of
 * those evaluations: per pair 2*s* + 4 (the uint16 Pi' entries up to the
 * serving facility plus one int32 D' entry), plus 8*W + 8 per evaluated
 * chromosome (mask read, fitness write).  Enabling or reading resets the
 * totals.
 * ------------------------------------------------------------------------- */
typedef struct {
    double eval_ms;
    int64_t eval_launches;
    int64_t eval_bytes;
    int64_t eval_pairs;
} pmp_profile;

PMP_API pmp_status pmp_ga_profile(pmp_ga *ga, int32_t enable);
PMP_API pmp_status pmp_ga_profile_read(pmp_ga *ga, pmp_profile *out, void *stream);

/* The same for a batch (per-phase kernels only): while enabled,
 * pmp_batch_step launches its phases directly (no graph) and brackets every
 * launch of the batch-wide evaluation kernel with HIP events.
 * pmp_batch_profile_read waits for `stream` and returns the summed
 * milliseconds of those launches and their number; both reset the totals.
 * PMP_EUNSUPPORTED for a batch in persistent-kernel mode. */
PMP_API pmp_status pmp_batch_profile(pmp_batch *batch, int32_t enable);
PMP_API pmp_status pmp_batch_profile_read(pmp_batch *batch, double *eval_ms,
                                          int64_t *eval_launches, void *stream);

/* ===========================================================================
 * Learned swap proposal (not in the paper).  A small network scores swap
 * moves of a chromosome (close open facility j, open closed facility k) from
 * 16 features of j and 16 of k; the GA's mutation cycle (step 4 above) tries
 * the best-scored swaps before its plain mutation attempts, and every tried
 * swap is judged by the exact evaluation kernel and taken only if strictly
 * fitter, like any mutant.  Each judged swap yields a training tuple (the 32
 * inputs; the exact change of the objective), on which the network is
 * trained on the GPU.
 * ======================================================================== */
#define PMP_FEATURES 16
#define PMP_MLP_INPUTS 32
#define PMP_MLP_HIDDEN 128
#define PMP_MLP_PARAMS 20865
#define PMP_MAX_LEARNED_FACILITIES 4096
#define PMP_MAX_CANDIDATES 64

/* ---------------------------------------------------------------------------
 * pmp_features - the 16 features of every facility j of every chromosome x.
 * For client i, with positions in the truncated row Pi'_i (Section 2.1):
 * a_i, c1_i = first open facility and its cost (Eq. (6)'s term), b_i, c2_i =
 * the second open facility and its cost, or c2_i = D'_{i,K} and no b_i when
 * the truncated row holds no second open facility.  f = cost of x,
 * F = max(f, 1), T = max(sum of all d_ij, 1), L = ceil(m / p).
 *   0 1 if j is open          1 #{i : a_i = j} p / n
 *   2 sum_{a_i = j} c1_i p/F  3 sum_{a_i = j} (c2_i - c1_i) p / F
 *   4 #{i : b_i = j} p / n    5 sum_{b_i = j} (c2_i - c1_i) p / F
 *   6 #{i : j closed, before a_i in Pi'_i} p / n
 *   7 sum over those i of (c1_i - d_ij) p / F
 *   8 #{i : j closed, after a_i and before b_i (up to K without b_i)} p / n
 *   9 sum over those i of (c2_i - d_ij) p / F
 *  10 (sum_i d_ij) m / T      11 #{i : j among the first L of Pi'_i} m/(n L)
 *  12 p / m                   13 f m / T
 *  14 gen_frac                15 1
 * Each value is (float)(a * b / c) evaluated in double from the integers.
 *  masks    P x W chromosomes, exactly p open facilities each.
 *  out      P x m x 16 float32 (chromosome-major, then facility).
 * Errors: PMP_EUNSUPPORTED if m > PMP_MAX_LEARNED_FACILITIES; PMP_EINFEASIBLE
 * as pmp_eval_population.  Host pointers, or device with PMP_ON_DEVICE.
 * ------------------------------------------------------------------------- */
PMP_API pmp_status pmp_features(pmp_instance *inst, const uint64_t *masks, int32_t P,
                                float gen_frac, float *out, uint32_t flags, void *stream);

/* ---------------------------------------------------------------------------
 * The scoring network: 32 inputs -> 128 -> 128 -> 1, ReLU after each hidden
 * layer.  Parameters (PMP_MLP_PARAMS float32, in this order): W1 [128][32],
 * b1 [128], W2 [128][128], b2 [128], w3 [128], b3 [1];
 * y = w3 . relu(W2 h1 + b2) + b3 with h1 = relu(W1 x + b1).  Weights and
 * inputs are rounded to BF16 (nearest even) and h1 too; products accumulate
 * in FP32 on the matrix cores.  The training loss of rows (x_r, t_r, w_r) is
 * sum_r w_r (y_r - t_r)^2 / (2 sum_r w_r); gradients treat the BF16
 * roundings as identity; Adam (beta1 0.9, beta2 0.999, eps 1e-8) updates
 * FP32 master parameters.
 *
 * pmp_model_create   Glorot-uniform weights from Philox (seed), zero biases.
 * pmp_model_get/set  the FP32 master parameters (set clears Adam's state).
 * pmp_model_forward  y[rows] for x[rows x 32] (float32, rounded to BF16).
 * pmp_model_grad     gradient (PMP_MLP_PARAMS) and loss of the rows; w may
 *                    be NULL (all 1).  Rows whose weights sum to 0: no output.
 * pmp_model_train    `steps` Adam steps of size lr on the rows.
 * Host pointers, or device pointers with PMP_ON_DEVICE.  A model may be
 * shared by several GA runs; calls on one model must not overlap.
 * ------------------------------------------------------------------------- */
typedef struct pmp_model pmp_model;

PMP_API pmp_status pmp_model_create(uint64_t seed, pmp_model **out);
PMP_API pmp_status pmp_model_get(pmp_model *model, float *params, uint32_t flags,
                                 void *stream);
PMP_API pmp_status pmp_model_set(pmp_model *model, const float *params, uint32_t flags,
                                 void *stream);
PMP_API pmp_status pmp_model_forward(pmp_model *model, const float *x, int32_t rows,
                                     float *y, uint32_t flags, void *stream);
PMP_API pmp_status pmp_model_grad(pmp_model *model, const float *x, const float *t,
                                  const float *w, int32_t rows, float *grad, float *loss,
                                  uint32_t flags, void *stream);
PMP_API pmp_status pmp_model_train(pmp_model *model, const float *x, const float *t,
                                   const float *w, int32_t rows, float lr, int32_t steps,
                                   float *loss, uint32_t flags, void *stream);
PMP_API void pmp_model_destroy(pmp_model *model);

/* ---------------------------------------------------------------------------
 * pmp_ga_set_model - let a GA run use (and train) a model.  Each generation,
 * after the crossover stages, every chromosome x draws C candidates: for
 * candidate t, r_j uniform in [0, p) and r_k uniform in [0, m - p) from its
 * Philox stream (role 2, tag 5, stage t), j = the r_j-th open and k = the
 * r_k-th closed facility in index order; input row t = [features of j |
 * features of k] (pmp_features, gen_frac = generation / EvolveLimit), scored
 * by the network (the predicted normalised change of the cost).  Mutation
 * attempt a < L takes the swap of rank a (ascending score, ties to lower t),
 * or, when a draw in [0, 1000) of stream (role 2, tag 6, stage a) falls below
 * explore_permille, the candidate of a second draw uniform in [0, C).  The
 * remaining Y - L attempts are the plain mutations.  Each evaluated swap
 * stores (inputs, target) in a ring of H generations: target =
 * clamp((f(x') - f(x)) p / max(f(x), 1), -4, 4).  After every train_every-th
 * generation one Adam step (lr) is taken on the whole ring.
 *  model  borrowed, must outlive the run; NULL detaches (plain GA again).
 * PMP_EINVAL: bad parameters; PMP_EUNSUPPORTED: m above
 * PMP_MAX_LEARNED_FACILITIES, or a run in persistent-kernel mode.
 * ------------------------------------------------------------------------- */
typedef struct {
    int32_t candidates;        /* C, 1..PMP_MAX_CANDIDATES; 0 = 64 */
    int32_t learned_iters;     /* L, 1..min(C, Y); 0 = ceil(Y / 2) */
    int32_t explore_permille;  /* 0..1000 */
    int32_t history;           /* H generations kept for training; 0 = 4 */
    int32_t train_every;       /* 0 = never (frozen model) */
    float lr;                  /* Adam step size; 0 = 1e-3 */
    int32_t reserved[2];       /* must be 0 */
} pmp_learn_params;

PMP_API pmp_status pmp_ga_set_model(pmp_ga *ga, pmp_model *model,
                                    const pmp_learn_params *params);

/* pmp_ga_replay - wait for `stream`; copy the training ring of a learned run
 * (host pointers, NULL = skip).  Row ((g mod H) L + a) P + c holds attempt a
 * of chromosome c in generation g: x (32 BF16 inputs as uint16), target,
 * weight (1 = evaluated, 0 = not run), swap (j, k), delta (f(x') - f(x),
 * f(x)).  *rows receives H L P.  scores (P x C): the network's scores of the
 * candidates of the last generation. */
PMP_API pmp_status pmp_ga_replay(pmp_ga *ga, int32_t *rows, uint16_t *x, float *target,
                                 float *weight, int32_t *swap, int64_t *delta,
                                 float *scores, void *stream);

PMP_API const char *pmp_status_str(pmp_status s);
PMP_API const char *pmp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PMP_H */
