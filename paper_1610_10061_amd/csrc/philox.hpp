// Counter-based random streams for the GA operators.
//
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
// easy as 1, 2, 3", SC 2011): ten rounds of two 64x64->128 multiplications
// with Weyl-sequence key bumps.  A stream is keyed by (seed, role) and
// addressed by the counter (generation, chromosome, tag << 32 | stage, block);
// it yields the four words of block 0, then of block 1, and so on.  Every
// random choice of the GA is a function of these logical indices only, never
// of a thread or block id, so results do not depend on the launch shape.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pmp {

enum : uint64_t { ROLE_POPULATION = 1, ROLE_EVOLVE = 2, ROLE_MODEL = 3 };
enum : uint64_t {
    TAG_SAMPLE = 1,
    TAG_CROSSOVER = 2,
    TAG_MUTATION = 3,
    TAG_WEIGHTS = 4,  // initial network weights
    TAG_PROPOSE = 5,  // swap candidates of the learned proposal
    TAG_EXPLORE = 6,  // exploration draws of the learned proposal
};

struct PhiloxStream {
    uint64_t k0, k1;       // key
    uint64_t c0, c1, c2;   // fixed counter words
    uint64_t block;        // fourth counter word
    uint64_t buf[4];
    int used;

    __device__ __forceinline__ PhiloxStream(uint64_t seed, uint64_t role,
                                            uint64_t gen, uint64_t chrom,
                                            uint64_t tag, uint64_t stage)
        : k0(seed), k1(role), c0(gen), c1(chrom),
          c2((tag << 32) | (stage & 0xFFFFFFFFull)), block(0), used(4) {}

    __device__ __forceinline__ void refill()
    {
        const uint64_t kM0 = 0xD2E7470EE14C6C93ull, kM1 = 0xCA5A826395121157ull;
        const uint64_t kW0 = 0x9E3779B97F4A7C15ull, kW1 = 0xBB67AE8584CAA73Bull;
        uint64_t x0 = c0, x1 = c1, x2 = c2, x3 = block;
        uint64_t a = k0, b = k1;
#pragma unroll
        for (int r = 0; r < 10; ++r) {
            const uint64_t hi0 = __umul64hi(kM0, x0), lo0 = kM0 * x0;
            const uint64_t hi1 = __umul64hi(kM1, x2), lo1 = kM1 * x2;
            x0 = hi1 ^ x1 ^ a;
            x1 = lo1;
            x2 = hi0 ^ x3 ^ b;
            x3 = lo0;
            a += kW0;
            b += kW1;
        }
        buf[0] = x0;
        buf[1] = x1;
        buf[2] = x2;
        buf[3] = x3;
        ++block;
        used = 0;
    }

    __device__ __forceinline__ uint64_t next()
    {
        if (used == 4) refill();
        // select, not buf[used]: a run-time index would put buf in scratch
        const int k = used++;
        return k == 0 ? buf[0] : k == 1 ? buf[1] : k == 2 ? buf[2] : buf[3];
    }

    // Uniform integer in [0, r), r >= 1 (Lemire, ACM TOMACS 2019): the high
    // word of x * r, redrawn while the low word falls below 2^64 mod r.
    __device__ __forceinline__ uint64_t below(uint64_t r)
    {
        uint64_t x = next();
        uint64_t lo = x * r;
        if (lo < r) {
            const uint64_t thresh = (0ull - r) % r;
            while (lo < thresh) {
                x = next();
                lo = x * r;
            }
        }
        return __umul64hi(x, r);
    }
};

}  // namespace pmp
