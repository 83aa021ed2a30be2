/*
 * CPU oracle for the p-median hot path (AlBdaiwi & AboElFotoh, "A GPU-Based
 * Genetic Algorithm for the P-Median Problem", arXiv 1610.10061).
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, slow, obviously correct C.  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load
 * this library.  It shares no code, header or table with the GPU library and
 * includes nothing from it.
 *
 * Conventions: indices are 0-based (the paper's math is 1-based); a
 * chromosome is m bits in W = ceil(m/64) little-endian 64-bit words, bit j of
 * word j/64 set when facility j is open (Section 4.1).  The oracle unpacks
 * chromosomes to one byte per facility before doing anything with them.
 *
 * Every function states the passage it follows.  Readings where the paper is
 * silent or garbled are listed beside the code that takes them.
 *
 * Return codes: 0 ok, 1 invalid argument, 2 infeasible chromosome
 * (popcount != p, or no open facility), 3 out of memory.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL 1
#define ORC_EINFEASIBLE 2
#define ORC_ENOMEM 3

static void unpack(const uint64_t *mask, int32_t m, uint8_t *bits)
{
    for (int32_t j = 0; j < m; ++j)
        bits[j] = (uint8_t)((mask[j / 64] >> (j % 64)) & 1u);
}

static void pack(const uint8_t *bits, int32_t m, int32_t W, uint64_t *mask)
{
    for (int32_t w = 0; w < W; ++w)
        mask[w] = 0;
    for (int32_t j = 0; j < m; ++j)
        if (bits[j])
            mask[j / 64] |= (uint64_t)1 << (j % 64);
}

/* number of threads a call with threads = 0 uses */
int orc_default_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static int set_threads(int32_t threads)
{
#ifdef _OPENMP
    return threads > 0 ? threads : omp_get_max_threads();
#else
    (void)threads;
    return 1;
#endif
}

/* ------------------------------------------------------------------------
 * Objective, Section 1, Eq. (1)-(3): every client is served by the open
 * facility nearest to it, so the cost of an open set O is
 *     f(O) = sum_i min_{j in O} d_ij .
 * Computed directly from d, never through the orderings.
 *
 * When scan_total is given, also the number of entries the paper's scan of
 * Section 4.2 reads for each client: with j* the open facility of least
 * (d_ij, j), the position of j* in the ordering of Section 2.1 (ties by
 * lower index) is 1 + #{ j : (d_ij, j) < (d_ij*, j*) }.  scan_total[c] is the
 * sum of these positions over clients.  This needs no ordering either.
 * ---------------------------------------------------------------------- */
static int64_t objective_one(const int32_t *d, int64_t ld, int32_t n,
                             int32_t m, const uint8_t *open,
                             const int32_t *olist, int32_t np,
                             int64_t *scan)
{
    int64_t total = 0, stotal = 0;
    for (int32_t i = 0; i < n; ++i) {
        const int32_t *row = d + (int64_t)i * ld;
        int32_t jbest = olist[0];
        for (int32_t k = 1; k < np; ++k) {
            int32_t j = olist[k];
            if (row[j] < row[jbest])  /* open list ascending: keeps lowest j */
                jbest = j;
        }
        total += row[jbest];
        if (scan) {
            int64_t before = 0;
            for (int32_t j = 0; j < m; ++j)
                if (row[j] < row[jbest] || (row[j] == row[jbest] && j < jbest))
                    ++before;
            stotal += before + 1;
        }
    }
    (void)open;
    if (scan)
        *scan = stotal;
    return total;
}

int orc_objective(const int32_t *d, int64_t ld, int32_t n, int32_t m,
                  int32_t p, const uint64_t *masks, int32_t P,
                  int64_t *cost, int64_t *scan_total, int32_t threads)
{
    if (!d || !masks || !cost || n < 1 || m < 1 || P < 0 || ld < m)
        return ORC_EINVAL;
    const int32_t W = (m + 63) / 64;
    int bad = 0;
    int nt = set_threads(threads);
#pragma omp parallel num_threads(nt) reduction(| : bad)
    {
        uint8_t *open = (uint8_t *)malloc((size_t)m);
        int32_t *olist = (int32_t *)malloc(sizeof(int32_t) * (size_t)m);
#pragma omp for schedule(dynamic, 1)
        for (int32_t c = 0; c < P; ++c) {
            unpack(masks + (int64_t)c * W, m, open);
            int32_t np = 0;
            for (int32_t j = 0; j < m; ++j)
                if (open[j])
                    olist[np++] = j;
            /* bits past m must be clear */
            for (int32_t j = m; j < W * 64; ++j)
                if ((masks[(int64_t)c * W + j / 64] >> (j % 64)) & 1u)
                    np = -1;
            if (np <= 0 || (p > 0 && np != p)) {
                bad = 1;
                cost[c] = -1;
                if (scan_total)
                    scan_total[c] = -1;
                continue;
            }
            int64_t s = 0;
            cost[c] = objective_one(d, ld, n, m, open, olist, np,
                                    scan_total ? &s : NULL);
            if (scan_total)
                scan_total[c] = s;
        }
        free(open);
        free(olist);
    }
    return bad ? ORC_EINFEASIBLE : ORC_OK;
}

/* ------------------------------------------------------------------------
 * Orderings and gap terms, Section 2.1.
 * Pi^i orders the facilities by d_i. ascending; among equal distances the
 * lower index comes first (the reading that reproduces rows 2 and 3 of the
 * printed Pi of Example 1).  delta_i1 = d_{i pi_i1}, delta_ir =
 * d_{i pi_ir} - d_{i pi_i(r-1)}.  Only the first K = m - p + 1 columns are
 * kept (the truncation argument after Eq. (6)).  dsorted is d_{i pi_ik}, the
 * running sum of the gaps.
 * ---------------------------------------------------------------------- */
typedef struct {
    int32_t dist;
    int32_t fac;
} orc_key;

static int cmp_key(const void *a, const void *b)
{
    const orc_key *x = (const orc_key *)a, *y = (const orc_key *)b;
    if (x->dist != y->dist)
        return x->dist < y->dist ? -1 : 1;
    return x->fac < y->fac ? -1 : (x->fac > y->fac ? 1 : 0);
}

int orc_tables(const int32_t *d, int64_t ld, int32_t n, int32_t m, int32_t p,
               int32_t ncols, int32_t *pi, int32_t *delta, int32_t *dsorted)
{
    if (!d || n < 1 || m < 2 || p < 1 || p >= m || ld < m)
        return ORC_EINVAL;
    const int32_t K = ncols > 0 ? ncols : m - p + 1;
    if (K > m)
        return ORC_EINVAL;
    orc_key *row = (orc_key *)malloc(sizeof(orc_key) * (size_t)m);
    if (!row)
        return ORC_ENOMEM;
    for (int32_t i = 0; i < n; ++i) {
        for (int32_t j = 0; j < m; ++j) {
            if (d[(int64_t)i * ld + j] < 0) {
                free(row);
                return ORC_EINVAL;
            }
            row[j].dist = d[(int64_t)i * ld + j];
            row[j].fac = j;
        }
        qsort(row, (size_t)m, sizeof(orc_key), cmp_key);
        for (int32_t k = 0; k < K; ++k) {
            int64_t o = (int64_t)i * K + k;
            if (pi)
                pi[o] = row[k].fac;
            if (delta)
                delta[o] = k == 0 ? row[0].dist : row[k].dist - row[k - 1].dist;
            if (dsorted)
                dsorted[o] = row[k].dist;
        }
    }
    free(row);
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * B_C(z), Eq. (6), evaluated the paper's way (Section 4.2, function
 * Fitness): for each client, walk its row of Pi' adding the gap terms of
 * Delta' until the facility just added is open.  z_j = 1 means facility j is
 * closed; the product of z over the first k-1 entries of Pi^i is 1 exactly
 * while none of them is open, which is what the walk tests.  The garbled
 * "until C_S" is read as "until facility pi_is is open".
 * Used by the tests to cross-check orc_objective, never by itself.
 * ---------------------------------------------------------------------- */
int orc_bc_eval(const int32_t *pi, const int32_t *delta, int32_t n, int32_t K,
                int32_t m, const uint64_t *masks, int32_t P, int64_t *cost,
                int64_t *scan_total)
{
    if (!pi || !delta || !masks || !cost || n < 1 || K < 1 || m < 1)
        return ORC_EINVAL;
    const int32_t W = (m + 63) / 64;
    uint8_t *open = (uint8_t *)malloc((size_t)m);
    int rc = ORC_OK;
    for (int32_t c = 0; c < P; ++c) {
        unpack(masks + (int64_t)c * W, m, open);
        int64_t fitness = 0, scanned = 0;
        for (int32_t i = 0; i < n; ++i) {
            int32_t s = 0;
            int found = 0;
            while (s < K) {
                fitness += delta[(int64_t)i * K + s];
                int32_t j = pi[(int64_t)i * K + s];
                ++s;
                if (open[j]) {
                    found = 1;
                    break;
                }
            }
            scanned += s;
            if (!found) {  /* fewer than p open: the truncated walk ran out */
                rc = ORC_EINFEASIBLE;
                fitness = -1;
                break;
            }
        }
        cost[c] = fitness;
        if (scan_total)
            scan_total[c] = fitness < 0 ? -1 : scanned;
    }
    free(open);
    return rc;
}

/* ------------------------------------------------------------------------
 * Exhaustive search over all C(m,p) open sets in lexicographic order
 * (Eq. (1)-(3)); the first set in that order among those of least cost is
 * returned.  A depth-first walk keeps, for each depth, every client's
 * least distance to the facilities chosen so far; the cost of a full set is
 * the sum of those minima, which is Eq. (1) with nearest assignment.
 * Work is split over the first chosen facility.
 * ---------------------------------------------------------------------- */
static void exh_walk(const int32_t *d, int64_t ld, int32_t n, int32_t m,
                     int32_t p, int32_t depth, int32_t next, int32_t *chosen,
                     int32_t *mins /* (p+1) x n */, int64_t *best,
                     int32_t *best_set, int64_t *count)
{
    if (depth == p) {
        int64_t s = 0;
        const int32_t *mn = mins + (int64_t)p * n;
        for (int32_t i = 0; i < n; ++i)
            s += mn[i];
        ++*count;
        if (s < *best) {
            *best = s;
            memcpy(best_set, chosen, sizeof(int32_t) * (size_t)p);
        }
        return;
    }
    for (int32_t j = next; j <= m - (p - depth); ++j) {
        chosen[depth] = j;
        const int32_t *prev = mins + (int64_t)depth * n;
        int32_t *cur = mins + (int64_t)(depth + 1) * n;
        for (int32_t i = 0; i < n; ++i) {
            int32_t v = d[(int64_t)i * ld + j];
            cur[i] = v < prev[i] ? v : prev[i];
        }
        exh_walk(d, ld, n, m, p, depth + 1, j + 1, chosen, mins, best,
                 best_set, count);
    }
}

int orc_exhaustive(const int32_t *d, int64_t ld, int32_t n, int32_t m,
                   int32_t p, int64_t *best_cost, uint64_t *best_mask,
                   int64_t *count, int32_t threads)
{
    if (!d || !best_cost || n < 1 || m < 1 || p < 1 || p > m || ld < m)
        return ORC_EINVAL;
    const int32_t W = (m + 63) / 64;
    const int32_t nfirst = m - p + 1;
    int64_t *bc = (int64_t *)malloc(sizeof(int64_t) * (size_t)nfirst);
    int32_t *bs = (int32_t *)malloc(sizeof(int32_t) * (size_t)nfirst * p);
    int64_t *cnt = (int64_t *)calloc((size_t)nfirst, sizeof(int64_t));
    int nt = set_threads(threads);
#pragma omp parallel for num_threads(nt) schedule(dynamic, 1)
    for (int32_t f = 0; f < nfirst; ++f) {
        int32_t *chosen = (int32_t *)malloc(sizeof(int32_t) * (size_t)p);
        int32_t *mins = (int32_t *)malloc(sizeof(int32_t) * (size_t)(p + 1) * n);
        for (int32_t i = 0; i < n; ++i)
            mins[i] = INT32_MAX;
        chosen[0] = f;
        for (int32_t i = 0; i < n; ++i)
            mins[n + i] = d[(int64_t)i * ld + f];
        bc[f] = INT64_MAX;
        exh_walk(d, ld, n, m, p, 1, f + 1, chosen, mins, &bc[f],
                 bs + (int64_t)f * p, &cnt[f]);
        free(chosen);
        free(mins);
    }
    int32_t fb = 0;
    int64_t total = 0;
    for (int32_t f = 0; f < nfirst; ++f) {
        total += cnt[f];
        if (bc[f] < bc[fb])  /* strict: earlier first element wins ties */
            fb = f;
    }
    *best_cost = bc[fb];
    if (best_mask) {
        for (int32_t w = 0; w < W; ++w)
            best_mask[w] = 0;
        for (int32_t k = 0; k < p; ++k) {
            int32_t j = bs[(int64_t)fb * p + k];
            best_mask[j / 64] |= (uint64_t)1 << (j % 64);
        }
    }
    if (count)
        *count = total;
    free(bc);
    free(bs);
    free(cnt);
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * Random numbers.  The paper draws from curand streams, one per thread
 * (Section 3.2, Init kernel), and keeps the host's generator independent of
 * the device's (Section 6, Observation 3).  Here every draw comes from the
 * counter-based Philox4x64-10 generator (Salmon, Moraes, Dror and Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC 2011), keyed by
 * (seed, role) with role 1 for population sampling and role 2 for the
 * evolution operators, and addressed by the counter
 *     (generation, chromosome, tag << 32 | stage, block).
 * A stream hands out the four 64-bit words of block 0, then of block 1, ...
 * ---------------------------------------------------------------------- */
#define ORC_PHILOX_M0 0xD2E7470EE14C6C93ull
#define ORC_PHILOX_M1 0xCA5A826395121157ull
#define ORC_PHILOX_W0 0x9E3779B97F4A7C15ull
#define ORC_PHILOX_W1 0xBB67AE8584CAA73Bull

void orc_philox4x64(const uint64_t ctr[4], const uint64_t key[2],
                    uint64_t out[4])
{
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        unsigned __int128 a = (unsigned __int128)ORC_PHILOX_M0 * x0;
        unsigned __int128 b = (unsigned __int128)ORC_PHILOX_M1 * x2;
        uint64_t y0 = (uint64_t)(b >> 64) ^ x1 ^ k0;
        uint64_t y1 = (uint64_t)b;
        uint64_t y2 = (uint64_t)(a >> 64) ^ x3 ^ k1;
        uint64_t y3 = (uint64_t)a;
        x0 = y0;
        x1 = y1;
        x2 = y2;
        x3 = y3;
        k0 += ORC_PHILOX_W0;
        k1 += ORC_PHILOX_W1;
    }
    out[0] = x0;
    out[1] = x1;
    out[2] = x2;
    out[3] = x3;
}

#define ORC_ROLE_INIT 1u
#define ORC_ROLE_EVOLVE 2u
#define ORC_TAG_INIT 1u
#define ORC_TAG_XOVER 2u
#define ORC_TAG_MUT 3u

typedef struct {
    uint64_t key[2];
    uint64_t ctr[4];
    uint64_t buf[4];
    int used;
} orc_stream;

static void stream_open(orc_stream *s, uint64_t seed, uint64_t role,
                        uint64_t gen, uint64_t chrom, uint64_t tag,
                        uint64_t stage)
{
    s->key[0] = seed;
    s->key[1] = role;
    s->ctr[0] = gen;
    s->ctr[1] = chrom;
    s->ctr[2] = (tag << 32) | (stage & 0xFFFFFFFFull);
    s->ctr[3] = 0;
    s->used = 4;
}

static uint64_t stream_next(orc_stream *s)
{
    if (s->used == 4) {
        orc_philox4x64(s->ctr, s->key, s->buf);
        s->ctr[3] += 1;
        s->used = 0;
    }
    return s->buf[s->used++];
}

/* Uniform integer in [0, r), r >= 1: Lemire's multiply-and-reject method
 * ("Fast random integer generation in an interval", ACM TOMACS 2019). */
static uint64_t stream_below(orc_stream *s, uint64_t r)
{
    uint64_t x = stream_next(s);
    unsigned __int128 prod = (unsigned __int128)x * r;
    uint64_t low = (uint64_t)prod;
    if (low < r) {
        uint64_t floor_ = (0 - r) % r;
        while (low < floor_) {
            x = stream_next(s);
            prod = (unsigned __int128)x * r;
            low = (uint64_t)prod;
        }
    }
    return (uint64_t)(prod >> 64);
}

/* test hook: n consecutive bounded draws from one stream */
int orc_stream_draws(uint64_t seed, uint64_t role, uint64_t gen, uint64_t chrom,
                     uint64_t tag, uint64_t stage, const uint64_t *bounds,
                     int32_t count, uint64_t *out)
{
    orc_stream s;
    stream_open(&s, seed, role, gen, chrom, tag, stage);
    for (int32_t k = 0; k < count; ++k)
        out[k] = bounds[k] == 0 ? stream_next(&s) : stream_below(&s, bounds[k]);
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * Chromosome generation, Section 4.1.  The paper draws one 64-bit rank below
 * C(m,p) and unranks it lexicographically; a 64-bit rank cannot be uniform
 * once C(m,p) exceeds 2^64 (already C(100,33) of Table 1 does).  The reading
 * taken: the intended law is a uniform p-subset, drawn with Floyd's
 * algorithm (Bentley and Floyd, "Programming pearls: a sample of
 * brilliance", CACM 1987): for j = m-p .. m-1 pick t uniform in [0, j];
 * take t unless it is already taken, else take j.
 * ---------------------------------------------------------------------- */
static void sample_subset(orc_stream *s, int32_t m, int32_t p, uint8_t *bits)
{
    memset(bits, 0, (size_t)m);
    for (int32_t j = m - p; j < m; ++j) {
        int32_t t = (int32_t)stream_below(s, (uint64_t)j + 1);
        if (bits[t])
            bits[j] = 1;
        else
            bits[t] = 1;
    }
}

/* ------------------------------------------------------------------------
 * Chromosome generation as Section 4.1 describes it: a uniform random rank
 * r in [0, C(m, p)) names the r-th p-subset in lexicographic order of its
 * sorted elements.  The GA takes it only when C(m, p) < 2^63, so that one
 * bounded 64-bit draw covers every subset.  Unranking walks the candidates x = 0, 1, ... for each
 * element in turn and skips x while the C(m - x - 1, p - i - 1) subsets
 * whose i-th element is x all come before r.
 * ---------------------------------------------------------------------- */
static uint64_t binom_u64(int32_t a, int32_t b)  /* exact; UINT64_MAX past 2^64 */
{
    if (b < 0 || b > a)
        return 0;
    if (b > a - b)
        b = a - b;
    unsigned __int128 c = 1;
    for (int32_t j = 1; j <= b; ++j) {
        c = c * (unsigned __int128)(a - b + j) / (unsigned __int128)j;
        if (c > (unsigned __int128)UINT64_MAX)
            return UINT64_MAX;
    }
    return (uint64_t)c;
}

static void unrank_subset(uint64_t r, int32_t m, int32_t p, uint8_t *bits)
{
    memset(bits, 0, (size_t)m);
    int32_t x = 0;
    for (int32_t i = 0; i < p; ++i) {
        for (;;) {
            const uint64_t c = binom_u64(m - x - 1, p - i - 1);
            if (r < c)
                break;
            r -= c;
            ++x;
        }
        bits[x] = 1;
        ++x;
    }
}

int orc_unrank(uint64_t r, int32_t m, int32_t p, uint64_t *mask)
{
    if (m < 1 || p < 1 || p > m || !mask || binom_u64(m, p) == UINT64_MAX ||
        r >= binom_u64(m, p))
        return ORC_EINVAL;
    uint8_t *bits = (uint8_t *)malloc((size_t)m);
    unrank_subset(r, m, p, bits);
    pack(bits, m, (m + 63) / 64, mask);
    free(bits);
    return ORC_OK;
}

int orc_sample_subset(uint64_t seed, uint64_t gen, uint64_t chrom, int32_t m,
                      int32_t p, uint64_t *mask)
{
    if (m < 1 || p < 1 || p > m || !mask)
        return ORC_EINVAL;
    orc_stream s;
    uint8_t *bits = (uint8_t *)malloc((size_t)m);
    stream_open(&s, seed, ORC_ROLE_INIT, gen, chrom, ORC_TAG_INIT, 0);
    sample_subset(&s, m, p, bits);
    pack(bits, m, (m + 63) / 64, mask);
    free(bits);
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * Crossover, Section 4.3.  Starting at r1 and wrapping past the end, visit
 * the positions where the two parents differ; turn on the first i of them
 * where the own parent A has a 0 and turn off the first i where A has a 1,
 * so the offspring keeps exactly p ones.  If a whole turn ends before both
 * counts reach i, the operator fails and there is no offspring.
 * ---------------------------------------------------------------------- */
static int crossover(const uint8_t *A, const uint8_t *B, int32_t m, int32_t r1,
                     int32_t i, uint8_t *F)
{
    memcpy(F, A, (size_t)m);
    int32_t on = 0, off = 0;
    for (int32_t t = 0; t < m && (on < i || off < i); ++t) {
        int32_t j = (r1 + t) % m;
        if (A[j] == B[j])
            continue;
        if (A[j] == 0 && on < i) {
            F[j] = 1;
            ++on;
        } else if (A[j] == 1 && off < i) {
            F[j] = 0;
            ++off;
        }
    }
    return on == i && off == i;
}

int orc_crossover(const uint64_t *a, const uint64_t *b, int32_t m, int32_t r1,
                  int32_t i, uint64_t *f)
{
    if (m < 1 || r1 < 0 || r1 >= m || i < 1)
        return -1;
    uint8_t *A = (uint8_t *)malloc((size_t)m * 3);
    uint8_t *B = A + m, *F = B + m;
    unpack(a, m, A);
    unpack(b, m, B);
    int ok = crossover(A, B, m, r1, i, F);
    pack(F, m, (m + 63) / 64, f);
    free(A);
    return ok;
}

/* ------------------------------------------------------------------------
 * Mutation, Section 4.4: a circular shift of the whole chromosome or a
 * block shift (a circular shift of a random subsequence), by a random
 * amount in a random direction.  Readings (the figures are not available):
 * each choice is uniform; "right" moves bit j to j + s, i.e. numpy.roll by
 * +s; a circular shift moves by s in [1, m-1]; a block is [a, b] with
 * a < b drawn as a uniform pair of distinct positions, shifted by s in
 * [1, b - a] inside the block.  Draw order: type, direction, then either
 * s, or the two block ends and s.
 * ---------------------------------------------------------------------- */
static void mutate(orc_stream *s, const uint8_t *A, int32_t m, uint8_t *F,
                   int32_t *desc /* type, dir, a, b, s */)
{
    int32_t type = (int32_t)stream_below(s, 2);
    int32_t dir = (int32_t)stream_below(s, 2);  /* 0 right, 1 left */
    if (type == 0) {
        int32_t sh = 1 + (int32_t)stream_below(s, (uint64_t)m - 1);
        int32_t move = dir == 0 ? sh : m - sh;
        for (int32_t j = 0; j < m; ++j)
            F[(j + move) % m] = A[j];
        if (desc) {
            desc[0] = 0; desc[1] = dir; desc[2] = 0; desc[3] = m - 1; desc[4] = sh;
        }
    } else {
        int32_t x = (int32_t)stream_below(s, (uint64_t)m);
        int32_t y = (int32_t)stream_below(s, (uint64_t)m - 1);
        if (y >= x)
            ++y;
        int32_t a = x < y ? x : y, b = x < y ? y : x;
        int32_t len = b - a + 1;
        int32_t sh = 1 + (int32_t)stream_below(s, (uint64_t)len - 1);
        int32_t move = dir == 0 ? sh : len - sh;
        memcpy(F, A, (size_t)m);
        for (int32_t q = 0; q < len; ++q)
            F[a + (q + move) % len] = A[a + q];
        if (desc) {
            desc[0] = 1; desc[1] = dir; desc[2] = a; desc[3] = b; desc[4] = sh;
        }
    }
}

int orc_mutate(uint64_t seed, uint64_t gen, uint64_t chrom, uint64_t attempt,
               const uint64_t *a, int32_t m, uint64_t *f, int32_t *desc)
{
    if (m < 2 || !a || !f)
        return ORC_EINVAL;
    orc_stream s;
    uint8_t *A = (uint8_t *)malloc((size_t)m * 2);
    unpack(a, m, A);
    stream_open(&s, seed, ORC_ROLE_EVOLVE, gen, chrom, ORC_TAG_MUT, attempt);
    mutate(&s, A, m, A + m, desc);
    pack(A + m, m, (m + 63) / 64, f);
    free(A);
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * The genetic algorithm, Section 3 (host steps 7-16 around one Evolve call,
 * Evolve steps 1-8), one generation = one Evolve call and the host steps
 * after it.  Population of P = NB x NT chromosomes; group b is chromosomes
 * b*NT .. b*NT+NT-1 (a thread block of the paper).
 *
 *  1. Population: a fresh uniform p-subset for every slot (Floyd's method, or
 *     with init 1 the subset of a uniform lexicographic rank), except that from
 *     the second generation on the group bests of the previous generation
 *     migrate (Section 4.5): group b's best to slot b*NT (to the same block,
 *     migration 0) or to slot b (the team of bests in one block, migration 1).
 *  2. Fitness of every chromosome.
 *  3. Crossover cycle: stages k = 0 .. X-1 with stride NT/2, NT/4, ..., 1
 *     (repeating if X > lg NT).  Chromosome t of a group pairs with t XOR
 *     stride (the pairing of Evolve step 3).  Both partners read each
 *     other's chromosome as it was when the stage began.  The pair's lower
 *     index draws r1 in [0, m) and i in [1, floor(p/2)] and both use them;
 *     each forms its own offspring and takes it if strictly fitter.  No
 *     crossover when p < 2.
 *  4. Mutation cycle: up to Y attempts (default lg NT); each attempt mutates
 *     the current chromosome and takes the offspring if strictly fitter,
 *     and the cycle stops at the first success.  An offspring equal to its
 *     parent is not evaluated.
 *  5. Group best: least fitness, lowest index on ties.
 *  6. Global best: least group best, lowest group on ties; the saturation
 *     count resets on a strict improvement and grows otherwise.  Stop when
 *     it reaches S (S > 0) or when EvolveLimit generations have run.
 *
 * The paper prints no trajectory (its Figures 1-3 are missing), so the
 * exact sequence of choices rests on the readings above.  The tests pin it
 * by a worked derivation of whole generations kept apart from this file
 * (every Philox word from numpy's generator, every operator parameter,
 * offspring and accept decision, the state after each generation, on
 * Example 1 and on an instance with many equal costs), and by invariants
 * (popcount p, fitness equal to the objective, non-increasing best,
 * saturation stop, optimum reached on a small instance, checkpoint/resume
 * equivalence).
 * ---------------------------------------------------------------------- */
typedef struct {
    uint64_t seed;
    int32_t population;
    int32_t group_size;
    int32_t generations;      /* EvolveLimit */
    int32_t saturation;       /* S, 0 = off */
    int32_t crossover_iters;  /* 0 = lg NT */
    int32_t mutation_iters;   /* 0 = lg NT */
    int32_t migration;        /* 0: to the same block, 1: all to one block */
    int32_t init;             /* 0: uniform subset (Floyd), 1: uniform rank, unranked */
} orc_ga_params;

/* state layout (int64): */
enum {
    ORC_ST_GEN = 0,        /* generations run */
    ORC_ST_SAT = 1,        /* saturation count */
    ORC_ST_DONE = 2,       /* 1 once stopped */
    ORC_ST_BEST = 3,       /* global best cost (INT64_MAX before any) */
    ORC_ST_CHROM_EVALS = 4,
    ORC_ST_XO_FAIL = 5,    /* crossover operations that failed */
    ORC_ST_XO_TAKEN = 6,
    ORC_ST_MUT_TAKEN = 7,
    ORC_ST_COUNT = 8
};

static int ilog2(int32_t v)
{
    int r = 0;
    while ((1 << (r + 1)) <= v)
        ++r;
    return r;
}

int orc_ga_run(const int32_t *d, int64_t ld, int32_t n, int32_t m, int32_t p,
               const orc_ga_params *prm, int32_t gens, uint64_t *pop,
               int64_t *fit, uint64_t *gbest_mask, int64_t *gbest_cost,
               uint64_t *best_mask, int64_t *state, int64_t *trace,
               int32_t threads)
{
    if (!d || !prm || !pop || !fit || !gbest_mask || !gbest_cost ||
        !best_mask || !state)
        return ORC_EINVAL;
    const int32_t P = prm->population, NT = prm->group_size;
    if (n < 1 || m < 2 || p < 1 || p >= m || P < 1 || NT < 1 ||
        (NT & (NT - 1)) || P % NT || prm->generations < 1)
        return ORC_EINVAL;
    const uint64_t nsets = binom_u64(m, p);
    if ((prm->init != 0 && prm->init != 1) || (prm->init == 1 && nsets >= (1ull << 63)))
        return ORC_EINVAL;
    const int32_t W = (m + 63) / 64, NB = P / NT, lg = ilog2(NT);
    const int32_t X = prm->crossover_iters > 0 ? prm->crossover_iters : lg;
    const int32_t Y = prm->mutation_iters > 0 ? prm->mutation_iters : lg;
    const int nt = set_threads(threads);

    uint8_t *bits = (uint8_t *)malloc((size_t)P * m);      /* current */
    uint8_t *snap = (uint8_t *)malloc((size_t)P * m);      /* stage start */
    uint8_t *offs = (uint8_t *)malloc((size_t)P * m);      /* offspring */
    uint8_t *ok = (uint8_t *)malloc((size_t)P);
    uint8_t *improved = (uint8_t *)malloc((size_t)P);
    int64_t *offfit = (int64_t *)malloc(sizeof(int64_t) * (size_t)P);
    uint64_t *tmp = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)P * W);
    int32_t *which = (int32_t *)malloc(sizeof(int32_t) * (size_t)P);
    int rc = ORC_OK;
    if (!bits || !snap || !offs || !ok || !improved || !offfit || !tmp || !which) {
        rc = ORC_ENOMEM;
        goto out;
    }

    /* the population carried over from the previous call (left unchanged
     * when this call runs no generation) */
    for (int32_t c = 0; c < P; ++c)
        unpack(pop + (int64_t)c * W, m, bits + (int64_t)c * m);

    for (int32_t step = 0; step < gens && !state[ORC_ST_DONE]; ++step) {
        const uint64_t g = (uint64_t)state[ORC_ST_GEN];

        /* 1. population of this Evolve call, with migrants */
#pragma omp parallel for num_threads(nt) schedule(static)
        for (int32_t c = 0; c < P; ++c) {
            const int one = prm->migration == 1;
            if (g > 0 && (one ? c < NB : c % NT == 0)) {
                unpack(gbest_mask + (int64_t)(one ? c : c / NT) * W, m,
                       bits + (int64_t)c * m);
            } else {
                orc_stream s;
                stream_open(&s, prm->seed, ORC_ROLE_INIT, g, (uint64_t)c,
                            ORC_TAG_INIT, 0);
                if (prm->init == 1)
                    unrank_subset(stream_below(&s, nsets), m, p, bits + (int64_t)c * m);
                else
                    sample_subset(&s, m, p, bits + (int64_t)c * m);
            }
        }
        /* 2. fitness */
        for (int32_t c = 0; c < P; ++c)
            pack(bits + (int64_t)c * m, m, W, tmp + (int64_t)c * W);
        if (orc_objective(d, ld, n, m, p, tmp, P, fit, NULL, nt)) {
            rc = ORC_EINFEASIBLE;
            goto out;
        }
        state[ORC_ST_CHROM_EVALS] += P;

        /* 3. crossover cycle */
        for (int32_t k = 0; k < X && p >= 2 && lg > 0; ++k) {
            const int32_t stride = NT >> (1 + k % lg);
            memcpy(snap, bits, (size_t)P * m);
            int32_t nok = 0;
            for (int32_t c = 0; c < P; ++c) {
                const int32_t partner = c ^ stride;
                const int32_t leader = c < partner ? c : partner;
                orc_stream s;
                stream_open(&s, prm->seed, ORC_ROLE_EVOLVE, g,
                            (uint64_t)leader, ORC_TAG_XOVER, (uint64_t)k);
                int32_t r1 = (int32_t)stream_below(&s, (uint64_t)m);
                int32_t i = 1 + (int32_t)stream_below(&s, (uint64_t)(p / 2));
                ok[c] = (uint8_t)crossover(snap + (int64_t)c * m,
                                           snap + (int64_t)partner * m, m, r1,
                                           i, offs + (int64_t)c * m);
                nok += ok[c];
            }
            /* evaluate the offspring that exist */
            int32_t q = 0;
            for (int32_t c = 0; c < P; ++c)
                if (ok[c]) {
                    pack(offs + (int64_t)c * m, m, W, tmp + (int64_t)q * W);
                    which[q++] = c;
                }
            if (orc_objective(d, ld, n, m, p, tmp, q, offfit, NULL, nt)) {
                rc = ORC_EINFEASIBLE;
                goto out;
            }
            state[ORC_ST_CHROM_EVALS] += q;
            state[ORC_ST_XO_FAIL] += P - nok;
            for (int32_t r = 0; r < q; ++r) {
                int32_t c = which[r];
                if (offfit[r] < fit[c]) {
                    memcpy(bits + (int64_t)c * m, offs + (int64_t)c * m,
                           (size_t)m);
                    fit[c] = offfit[r];
                    state[ORC_ST_XO_TAKEN] += 1;
                }
            }
        }

        /* 4. mutation cycle */
        memset(improved, 0, (size_t)P);
        for (int32_t a = 0; a < Y; ++a) {
            int32_t q = 0;
            for (int32_t c = 0; c < P; ++c) {
                if (improved[c])
                    continue;
                orc_stream s;
                stream_open(&s, prm->seed, ORC_ROLE_EVOLVE, g, (uint64_t)c,
                            ORC_TAG_MUT, (uint64_t)a);
                uint8_t *F = offs + (int64_t)c * m;
                mutate(&s, bits + (int64_t)c * m, m, F, NULL);
                if (memcmp(F, bits + (int64_t)c * m, (size_t)m) == 0)
                    continue;
                pack(F, m, W, tmp + (int64_t)q * W);
                which[q++] = c;
            }
            if (orc_objective(d, ld, n, m, p, tmp, q, offfit, NULL, nt)) {
                rc = ORC_EINFEASIBLE;
                goto out;
            }
            state[ORC_ST_CHROM_EVALS] += q;
            for (int32_t r = 0; r < q; ++r) {
                int32_t c = which[r];
                if (offfit[r] < fit[c]) {
                    memcpy(bits + (int64_t)c * m, offs + (int64_t)c * m,
                           (size_t)m);
                    fit[c] = offfit[r];
                    improved[c] = 1;
                    state[ORC_ST_MUT_TAKEN] += 1;
                }
            }
        }

        /* 5. group bests (Evolve steps 7-8) */
        for (int32_t b = 0; b < NB; ++b) {
            int32_t bi = b * NT;
            for (int32_t t = 1; t < NT; ++t)
                if (fit[b * NT + t] < fit[bi])
                    bi = b * NT + t;
            gbest_cost[b] = fit[bi];
            pack(bits + (int64_t)bi * m, m, W, gbest_mask + (int64_t)b * W);
        }
        /* 6. global best, saturation, stop (host steps 13-15) */
        int32_t bb = 0;
        for (int32_t b = 1; b < NB; ++b)
            if (gbest_cost[b] < gbest_cost[bb])
                bb = b;
        if (gbest_cost[bb] < state[ORC_ST_BEST]) {
            state[ORC_ST_BEST] = gbest_cost[bb];
            memcpy(best_mask, gbest_mask + (int64_t)bb * W,
                   sizeof(uint64_t) * (size_t)W);
            state[ORC_ST_SAT] = 0;
        } else {
            state[ORC_ST_SAT] += 1;
        }
        if (trace)
            trace[step] = state[ORC_ST_BEST];
        state[ORC_ST_GEN] += 1;
        if ((prm->saturation > 0 && state[ORC_ST_SAT] >= prm->saturation) ||
            state[ORC_ST_GEN] >= prm->generations)
            state[ORC_ST_DONE] = 1;
    }
    for (int32_t c = 0; c < P; ++c)
        pack(bits + (int64_t)c * m, m, W, pop + (int64_t)c * W);
out:
    free(bits);
    free(snap);
    free(offs);
    free(ok);
    free(improved);
    free(offfit);
    free(tmp);
    free(which);
    return rc;
}

/* ------------------------------------------------------------------------
 * All-pairs shortest path lengths (Floyd, CACM 1962), the step that turns a
 * graph instance into its cost matrix (the benchmark graphs the paper
 * evaluates on give costs as shortest-path lengths).  w: n x n, w_ij >= 0 an
 * arc i -> j, w_ij < 0 no arc, diagonal taken as 0.  d: n x n, -1 where
 * there is no path.  Plain triple loop over the intermediate vertex k in
 * 64-bit arithmetic.  Returns ORC_EINVAL when a path length exceeds int32.
 * ---------------------------------------------------------------------- */
int orc_apsp(const int32_t *w, int32_t n, int32_t *d)
{
    if (!w || !d || n < 1)
        return ORC_EINVAL;
    const int64_t INF = INT64_MAX / 4;
    int64_t *D = (int64_t *)malloc(sizeof(int64_t) * (size_t)n * (size_t)n);
    if (!D)
        return ORC_ENOMEM;
    for (int32_t i = 0; i < n; ++i)
        for (int32_t j = 0; j < n; ++j) {
            const int32_t x = w[(int64_t)i * n + j];
            D[(int64_t)i * n + j] = i == j ? 0 : (x >= 0 ? (int64_t)x : INF);
        }
    for (int32_t k = 0; k < n; ++k)
        for (int32_t i = 0; i < n; ++i) {
            const int64_t dik = D[(int64_t)i * n + k];
            if (dik >= INF)
                continue;
            for (int32_t j = 0; j < n; ++j) {
                const int64_t via = dik + D[(int64_t)k * n + j];
                if (via < D[(int64_t)i * n + j])
                    D[(int64_t)i * n + j] = via;
            }
        }
    int rc = ORC_OK;
    for (int64_t e = 0; e < (int64_t)n * n; ++e) {
        if (D[e] >= INF)
            d[e] = -1;
        else if (D[e] > INT32_MAX)
            rc = ORC_EINVAL;
        else
            d[e] = (int32_t)D[e];
    }
    free(D);
    return rc;
}
