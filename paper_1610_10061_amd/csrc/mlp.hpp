// Swap-scoring network shared by the proposal kernel and the training
// kernels: 32 inputs -> 128 -> 128 -> 1 with ReLU, BF16 weights and inputs,
// FP32 accumulation on the MFMA units (gfx950's v_mfma_f32_16x16x32_bf16:
// a 16 x 16 product over 32 values of k per instruction).
//
// MFMA 16x16x32 BF16 operand layout (wave64, lane l, g = l / 16):
//   A fragment: A[row l%16][k 8g + i], i = 0..7
//   B fragment: B[k 8g + i][col l%16], i = 0..7
//   C/D:        D[row 4g + i][col l%16], i = 0..3
//
// Parameter vector (FP32 master copy, kParams values):
//   W1 [128][32] | b1 [128] | W2 [128][128] | b2 [128] | w3 [128] | b3 [1]
// BF16 copies are kept of W1, W2, W2^T and w3.  The first hidden layer's
// activations are rounded to BF16 (they are the second product's operand);
// the second layer's activations and the output stay FP32.
#pragma once

#include "common.hpp"

namespace pmp {

constexpr int kIn = 32;
constexpr int kHidden = 128;
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kHidden * kIn;       // 4096
constexpr int kOffW2 = kOffB1 + kHidden;             // 4224
constexpr int kOffB2 = kOffW2 + kHidden * kHidden;   // 20608
constexpr int kOffW3 = kOffB2 + kHidden;             // 20736
constexpr int kOffB3 = kOffW3 + kHidden;             // 20864
constexpr int kParams = kOffB3 + 1;                  // 20865
static_assert(kParams == PMP_MLP_PARAMS, "parameter count");

// Header words of one training block's partial sums (after kParams values).
constexpr int kPartHead = 4;            // count, loss, step, unused
constexpr int kPartStride = kParams + kPartHead + 3;  // 20872, 16-byte multiple
// Partial vectors of at most kMaxTrainBlocks workgroups, stored by 64-value
// chunks: chunk k / 64 of workgroup b at (k / 64 * kMaxTrainBlocks + b) * 64,
// so a workgroup writes 64 consecutive values at a time and the update
// reads one chunk of every workgroup as one contiguous block.
constexpr int kMaxTrainBlocks = 256;
constexpr int kPartChunks = (kPartStride + 63) / 64;
constexpr size_t kPartFloats = (size_t)kPartChunks * kMaxTrainBlocks * 64;
__device__ __forceinline__ int64_t part_index(int b, int k)
{
    return ((int64_t)(k >> 6) * kMaxTrainBlocks + b) * 64 + (k & 63);
}

// Round-to-nearest-even FP32 -> BF16 (finite inputs).
__device__ __host__ __forceinline__ uint16_t f32_to_bf16(float x)
{
    uint32_t u;
    __builtin_memcpy(&u, &x, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h)
{
    return __uint_as_float((uint32_t)h << 16);
}

// Read-only view of a model for the forward pass.
struct MlpDev {
    const uint16_t *W1;   // [128][32]  BF16
    const uint16_t *W2;   // [128][128] BF16
    const uint16_t *W2T;  // [128][128] BF16, W2 transposed
    const uint16_t *w3;   // [128]      BF16
    const float *b1, *b2, *b3;
};

// Everything a model owns on the device.
struct MlpModelDev {
    float *master;  // kParams
    float *m1, *m2; // Adam moments
    uint16_t *W1, *W2, *W2T, *w3;
    uint32_t *step; // Adam steps taken
    MlpDev view() const
    {
        MlpDev v;
        v.W1 = W1;
        v.W2 = W2;
        v.W2T = W2T;
        v.w3 = w3;
        v.b1 = master + kOffB1;
        v.b2 = master + kOffB2;
        v.b3 = master + kOffB3;
        return v;
    }
};

// When a training step runs inside a GA's generation sequence: after
// generation counts divisible by `every`, once per generation count.
struct TrainGate {
    const unsigned long long *gen;  // null: always train
    unsigned long long *last;       // generation count of the last step
    int32_t every;
};

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 mfma_bf16(bf16x8 a, bf16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Eight consecutive BF16 values at an 8-byte aligned address.
__device__ __forceinline__ bf16x8 load_bf16x8(const uint16_t *p)
{
    const uint2 lo = *reinterpret_cast<const uint2 *>(p);
    const uint2 hi = *reinterpret_cast<const uint2 *>(p + 4);
    const uint4 v = {lo.x, lo.y, hi.x, hi.y};
    return __builtin_bit_cast(bf16x8, v);
}

// Order this wave's earlier LDS accesses before its later ones.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

constexpr int kXStride = kIn + 4;       // padded LDS row of inputs (BF16)
constexpr int kHStride = kHidden + 4;   // padded LDS row of activations

// The output layer's terms of hidden tiles 2q and 2q + 1 for one row (this
// lane's unit of each tile, z: pre-activations, w: output weights), summed
// over the 16 lanes of the row's group (every lane ends with the sum).
__device__ __forceinline__ float out_pair(float z_a, float z_b, float w_a, float w_b)
{
    float v = fmaxf(z_a, 0.f) * w_a;
    v += fmaxf(z_b, 0.f) * w_b;
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 4);
    v += __shfl_xor(v, 8);
    return v;
}

// The output from the four tile pairs' sums, added in this order by every
// kernel.
__device__ __forceinline__ float out_sum(const float s[4], float b3)
{
    return ((s[0] + s[1]) + (s[2] + s[3])) + b3;
}

// The network on the workgroup's 64 input rows x (LDS), by hidden tile
// pairs: wave q computes hidden tiles 2q and 2q + 1 of both layers for all 64
// rows, so each wave loads a quarter of the weights once and uses each
// weight fragment for four row tiles (the layers' weights are read once per
// workgroup, not once per wave).  h1: the first layer's BF16 activations of
// all rows (LDS); ys: per row the output sums of the four tile pairs, which
// out_sum adds.  The training kernel computes its forward with the same
// operations, so a row's output is the same bits in every kernel.
// Block-wide (four waves, q = the wave's number; one barrier inside).
static_assert(kIn == 32 && kHidden == 128, "four tile pairs, one K-step in layer 1");
__device__ __forceinline__ void mlp_forward64(const MlpDev &P, const uint16_t *x, uint16_t *h1,
                                            float *ys, int q, int lane)
{
    const int r = lane & 15, g = lane >> 4;
    {
        bf16x8 bw[2];
        float bias[2];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int t = 2 * q + j;
            bw[j] = load_bf16x8(P.W1 + (t * 16 + r) * kIn + 8 * g);
            bias[j] = P.b1[t * 16 + r];
        }
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const bf16x8 ax = load_bf16x8(x + (mt * 16 + r) * kXStride + 8 * g);
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                f32x4 acc = {0.f, 0.f, 0.f, 0.f};
                acc = mfma_bf16(ax, bw[j], acc);
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    acc[i] += bias[j];
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    h1[(mt * 16 + 4 * g + i) * kHStride + (2 * q + j) * 16 + r] =
                        f32_to_bf16(fmaxf(acc[i], 0.f));
            }
        }
    }
    __syncthreads();
    bf16x8 bw[2][kHidden / 32];
    float bias[2], w3[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int t = 2 * q + j;
#pragma unroll
        for (int kb = 0; kb < kHidden / 32; ++kb)
            bw[j][kb] = load_bf16x8(P.W2 + (t * 16 + r) * kHidden + kb * 32 + 8 * g);
        bias[j] = P.b2[t * 16 + r];
        w3[j] = bf16_to_f32(P.w3[t * 16 + r]);
    }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        bf16x8 ah[kHidden / 32];
#pragma unroll
        for (int kb = 0; kb < kHidden / 32; ++kb)
            ah[kb] = load_bf16x8(h1 + (mt * 16 + r) * kHStride + kb * 32 + 8 * g);
        f32x4 z[2];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < kHidden / 32; ++kb)
                acc = mfma_bf16(ah[kb], bw[j][kb], acc);
#pragma unroll
            for (int i = 0; i < 4; ++i)
                acc[i] += bias[j];
            z[j] = acc;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float v = out_pair(z[0][i], z[1][i], w3[0], w3[1]);
            if (r == 0)
                ys[(mt * 16 + 4 * g + i) * 4 + q] = v;
        }
    }
}

// Launchers (k_mlp.hip).
hipError_t launch_mlp_forward(const MlpDev &P, const uint16_t *X, int rows, float *y,
                              hipStream_t s);
// Partial gradient sums of L = sum_r w_r (y_r - t_r)^2 / (2 sum_r w_r) into
// `partials` (kPartFloats, by part_index; at most kMaxTrainBlocks blocks);
// returns the block count used.
hipError_t launch_mlp_grad(const MlpDev &P, const uint16_t *X, const float *T,
                           const float *Wt, int rows, float *partials, int max_blocks,
                           const MlpModelDev &M, TrainGate gate, int *blocks,
                           hipStream_t s);
// Sum the partials: gradient (and loss) out, and/or an Adam step when lr > 0.
hipError_t launch_mlp_update(const MlpModelDev &M, const float *partials, int blocks,
                             float lr, float *grad_out, float *loss_out, TrainGate gate,
                             hipStream_t s);
hipError_t launch_mlp_publish(const MlpModelDev &M, hipStream_t s);
hipError_t launch_mlp_init(const MlpModelDev &M, uint64_t seed, hipStream_t s);
hipError_t launch_to_bf16(const float *x, uint16_t *y, int64_t count, hipStream_t s);
hipError_t launch_from_bf16(const uint16_t *x, float *y, int64_t count, hipStream_t s);

}  // namespace pmp
