// Shared definitions of the gfx950 p-median library: device state layout,
// error bits, kernel argument blocks and the internal launcher interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pmp {

// Error bits of an instance's device error word.
enum : uint32_t {
    ERR_NEGATIVE_DISTANCE = 1u << 0,  // some d_ij < 0
    ERR_POPCOUNT = 1u << 1,           // a chromosome without exactly p ones
    ERR_STRAY_BITS = 1u << 2,         // bits set at positions >= m
    ERR_SCAN_OVERRUN = 1u << 3,       // no open facility in a truncated row
};

// Device GA state: one array of 64-bit counters.
enum GaSlot : int {
    GS_GEN = 0,          // generations run
    GS_SAT = 1,          // generations since the last strict improvement
    GS_DONE = 2,         // 1 once stopped
    GS_BEST = 3,         // global best cost
    GS_CHROM_EVALS = 4,  // chromosomes evaluated
    GS_XO_FAIL = 5,
    GS_XO_TAKEN = 6,
    GS_MUT_TAKEN = 7,
    GS_SCAN_TOTAL = 8,   // sum of s* over evaluated pairs
    GS_COUNT = 16
};

// Tables of one preprocessed instance (device pointers).
struct Tables {
    const uint16_t *pi;  // n x pitch, facility order (first K valid)
    const int32_t *ds;   // n x pitch, sorted distances D'
    int32_t n, m, p, K, W, pitch;
};

// One population evaluation (Eq. (6) by the walk of Section 4.2).
struct EvalArgs {
    Tables t;
    const uint64_t *masks;            // P x W
    int32_t P;
    const uint8_t *active;            // optional: evaluate c only if active[c]
    unsigned long long *fitness;      // P, accumulated (caller zeroes)
    unsigned long long *scan;         // optional P, accumulated
    unsigned long long *gstate;       // optional GA counters (GS_*)
    uint32_t *err;                    // error word
    int32_t clients_per_block;
    int32_t tiles_c;                  // ceil(P / 64)
    int32_t tiles_i;                  // ceil(n / clients_per_block)
};

constexpr int kEvalTile = 64;     // chromosomes per block (one per lane)
constexpr int kEvalWaves = 4;     // waves per block

// Launchers (each lives with its kernels).
hipError_t launch_sort_rows(const int32_t *d, int64_t ld, int32_t n, int32_t m,
                            int32_t K, int32_t pitch, uint16_t *pi,
                            int32_t *delta, int32_t *ds, uint32_t *err,
                            hipStream_t s);
hipError_t launch_eval(const EvalArgs &a, hipStream_t s);
hipError_t launch_zero(void *p, size_t bytes, hipStream_t s);

struct GaArgs {
    Tables t;
    uint64_t seed;
    int32_t P, NT, NB, lg, X, Y, generations, saturation;
    uint64_t *cur;            // P x W current population
    uint64_t *off;            // P x W offspring
    unsigned long long *fit;  // P current fitness
    unsigned long long *ofit; // P offspring fitness
    uint8_t *ok;              // P: offspring exists / must be evaluated
    uint8_t *improved;        // P: mutation cycle succeeded
    uint64_t *gmask;          // NB x W group bests
    unsigned long long *gcost;// NB
    uint64_t *best_mask;      // W
    unsigned long long *gs;   // GS_COUNT counters
    uint32_t *err;
};

hipError_t launch_ga_init(const GaArgs &g, hipStream_t s);
hipError_t launch_ga_crossover(const GaArgs &g, int stage, hipStream_t s);
hipError_t launch_ga_mutate(const GaArgs &g, int attempt, hipStream_t s);
hipError_t launch_ga_accept(const GaArgs &g, int mutation, hipStream_t s);
hipError_t launch_ga_best(const GaArgs &g, hipStream_t s);
hipError_t launch_ga_state_init(const GaArgs &g, hipStream_t s);

}  // namespace pmp
