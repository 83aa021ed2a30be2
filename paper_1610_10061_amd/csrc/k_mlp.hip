// Inference and training kernels of the swap-scoring network (mlp.hpp).
//
// Training is deterministic: every workgroup sums its rows' gradient into
// registers (weight matrices on the MFMA units, with the rows as the
// contraction dimension) and writes one partial vector; the update kernel
// adds the partials in workgroup order and takes an Adam step (Kingma & Ba,
// ICLR 2015).  No floating-point atomics anywhere.
#include "mlp.hpp"
#include "philox.hpp"

namespace pmp {

namespace {

constexpr int kWaves = 4;
constexpr int kChunk = 16 * kWaves;   // rows per workgroup step
static_assert(kWaves == 4, "training splits the hidden layer into four tile pairs");
constexpr int kTStride = kChunk + 4;  // padded LDS row of a transposed tile

// Copy 16 input rows (row0..row0+15, zero past `rows`) into LDS x.
__device__ __forceinline__ void stage_rows16(const uint16_t *X, int64_t row0, int rows,
                                             uint16_t *x, int lane)
{
    const int r = lane >> 2, c = (lane & 3) * 8;
    uint4 v = {0u, 0u, 0u, 0u};
    if (row0 + r < rows)
        v = *reinterpret_cast<const uint4 *>(X + (row0 + r) * kIn + c);
    uint2 *d = reinterpret_cast<uint2 *>(x + r * kXStride + c);
    d[0] = uint2{v.x, v.y};
    d[1] = uint2{v.z, v.w};
}

// Forward of 64 rows per workgroup, split by hidden tile pairs over the
// four waves (mlp_forward64).
__global__ __launch_bounds__(64 * kWaves) void k_mlp_forward(MlpDev P, const uint16_t *X,
                                                            int rows, float *y)
{
    __shared__ __align__(16) uint16_t xs[kChunk * kXStride];
    __shared__ __align__(16) uint16_t hs[kChunk * kHStride];
    __shared__ float ys[kChunk * 4];
    const int wave = wave_id(), lane = threadIdx.x & 63;
    const int64_t row0 = (int64_t)blockIdx.x * kChunk;
    stage_rows16(X, row0 + wave * 16, rows, xs + wave * 16 * kXStride, lane);
    __syncthreads();
    mlp_forward64(P, xs, hs, ys, wave, lane);
    __syncthreads();
    const int64_t row = row0 + threadIdx.x;
    if (threadIdx.x < kChunk && row < rows)
        y[row] = out_sum(ys + threadIdx.x * 4, P.b3[0]);
}

struct GradLds {
    uint16_t xr[kChunk * kXStride];      // inputs, row-major
    uint16_t xt[kIn * kTStride];         // inputs, transposed
    uint16_t hr[kChunk * kHStride];      // h1 row-major, then dz2 row-major
    uint16_t ht[kHidden * kTStride];     // h1 transposed
    uint16_t z2t[kHidden * kTStride];    // dz2 transposed
    uint16_t z1t[kHidden * kTStride];    // dz1 transposed
    float ys[kChunk * 4];                // per row, the tile pairs' output sums
    float dy[kChunk];                    // per row, weight x output error
    int train;
};

// Gradient partial sums over the rows of this workgroup's chunks.
__global__ __launch_bounds__(64 * kWaves) void k_mlp_grad(MlpDev P, const uint16_t *X,
                                                         const float *T, const float *Wt,
                                                         int rows, float *partials,
                                                         const uint32_t *step,
                                                         TrainGate gate)
{
    __shared__ __align__(16) GradLds L;
    const int wave = wave_id(), lane = threadIdx.x & 63;
    const int r = lane & 15, g = lane >> 4;
    // value k of this workgroup's partial vector
    const int blk = (int)blockIdx.x;
    auto part = [partials, blk](int k) -> float & { return partials[part_index(blk, k)]; };
    if (threadIdx.x == 0) {
        int train = 1;
        if (gate.gen) {
            const unsigned long long gen = *gate.gen;
            train = gen > 0 && gen % (unsigned long long)gate.every == 0 && gen != *gate.last;
        }
        L.train = train;
        if (!train)
            part(kParams) = 0.f;  // no rows: the update kernel skips
    }
    __syncthreads();
    if (!L.train)
        return;

    f32x4 acc2[16], acc1[4];
#pragma unroll
    for (int k = 0; k < 16; ++k)
        acc2[k] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < 4; ++k)
        acc1[k] = f32x4{0.f, 0.f, 0.f, 0.f};
    // this wave's hidden tiles 2 wave and 2 wave + 1: bias and output-weight
    // gradients (per lane: unit r of each tile, over its rows)
    float db1[2], db2[2], dw3[2];
#pragma unroll
    for (int j = 0; j < 2; ++j)
        db1[j] = db2[j] = dw3[j] = 0.f;
    float db3 = 0.f, lsum = 0.f, wsum = 0.f;  // (threads of the chunk's rows)

    const int nchunks = (rows + kChunk - 1) / kChunk;
    for (int ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        const int64_t row0 = (int64_t)ch * kChunk;
        // inputs: row-major and transposed
        {
            const int tr = threadIdx.x >> 2, c = (threadIdx.x & 3) * 8;
            uint4 v = {0u, 0u, 0u, 0u};
            if (row0 + tr < rows)
                v = *reinterpret_cast<const uint4 *>(X + (row0 + tr) * kIn + c);
            uint2 *d = reinterpret_cast<uint2 *>(L.xr + tr * kXStride + c);
            d[0] = uint2{v.x, v.y};
            d[1] = uint2{v.z, v.w};
            const uint32_t w4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int e = 0; e < 8; ++e)
                L.xt[(c + e) * kTStride + tr] =
                    (uint16_t)((e & 1) ? (w4[e >> 1] >> 16) : (w4[e >> 1] & 0xFFFFu));
        }
        __syncthreads();

        // Forward and backward by hidden tile pairs: wave qp computes hidden
        // tiles 2 qp and 2 qp + 1 of every product for all 64 rows of the chunk
        // (a quarter of the weights per wave, each fragment used for four
        // row tiles), with the same operations per element as mlp_forward64.
        const int qp = wave;
        f32x4 z1[4][2], z2[4][2];
        {
            bf16x8 bw[2];
            float bias[2];
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int t = 2 * qp + j;
                bw[j] = load_bf16x8(P.W1 + (t * 16 + r) * kIn + 8 * g);
                bias[j] = P.b1[t * 16 + r];
            }
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                const bf16x8 ax = load_bf16x8(L.xr + (mt * 16 + r) * kXStride + 8 * g);
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const int t = 2 * qp + j;
                    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
                    acc = mfma_bf16(ax, bw[j], acc);
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        acc[i] += bias[j];
                    z1[mt][j] = acc;
                    uint16_t h[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        h[i] = f32_to_bf16(fmaxf(acc[i], 0.f));
                        L.hr[(mt * 16 + 4 * g + i) * kHStride + t * 16 + r] = h[i];
                    }
                    // h1 transposed (the D layout holds four consecutive rows)
                    *reinterpret_cast<uint2 *>(L.ht + (t * 16 + r) * kTStride + mt * 16 + 4 * g) =
                        uint2{h[0] | ((uint32_t)h[1] << 16), h[2] | ((uint32_t)h[3] << 16)};
                }
            }
        }
        __syncthreads();
        float w3[2];
        {
            bf16x8 bw[2][kHidden / 32];
            float bias[2];
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int t = 2 * qp + j;
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
                    ah[kb] = load_bf16x8(L.hr + (mt * 16 + r) * kHStride + kb * 32 + 8 * g);
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int kb = 0; kb < kHidden / 32; ++kb)
                        acc = mfma_bf16(ah[kb], bw[j][kb], acc);
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        acc[i] += bias[j];
                    z2[mt][j] = acc;
                }
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float v = out_pair(z2[mt][0][i], z2[mt][1][i], w3[0], w3[1]);
                    if (r == 0)
                        L.ys[(mt * 16 + 4 * g + i) * 4 + qp] = v;
                }
            }
        }
        __syncthreads();
        // output error and row weight of row `threadIdx.x`
        if (threadIdx.x < kChunk) {
            const int64_t row = row0 + threadIdx.x;
            float e = 0.f, w = 0.f;
            if (row < rows) {
                w = Wt ? Wt[row] : 1.f;
                e = out_sum(L.ys + threadIdx.x * 4, P.b3[0]) - T[row];
            }
            L.dy[threadIdx.x] = w * e;
            lsum += w * e * e;
            wsum += w;
            db3 += w * e;
        }
        __syncthreads();
        // dz2 = dy w3 relu'(z2); dw3 += dy h2; db2 += dz2 (dz2 row-major over
        // h1, whose last reader passed the barrier above, and transposed)
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int t = 2 * qp + j;
                uint16_t h[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int rw = mt * 16 + 4 * g + i;
                    const float dyv = L.dy[rw];
                    const float z = z2[mt][j][i];
                    dw3[j] += dyv * fmaxf(z, 0.f);
                    const float dz = z > 0.f ? dyv * w3[j] : 0.f;
                    db2[j] += dz;
                    h[i] = f32_to_bf16(dz);
                    L.hr[rw * kHStride + t * 16 + r] = h[i];
                }
                *reinterpret_cast<uint2 *>(L.z2t + (t * 16 + r) * kTStride + mt * 16 + 4 * g) =
                    uint2{h[0] | ((uint32_t)h[1] << 16), h[2] | ((uint32_t)h[3] << 16)};
            }
        __syncthreads();
        // dz1 = (dz2 W2) relu'(z1); db1 += dz1
        {
            bf16x8 bw[2][kHidden / 32];
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int kb = 0; kb < kHidden / 32; ++kb)
                    bw[j][kb] =
                        load_bf16x8(P.W2T + ((2 * qp + j) * 16 + r) * kHidden + kb * 32 + 8 * g);
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                bf16x8 a[kHidden / 32];
#pragma unroll
                for (int kb = 0; kb < kHidden / 32; ++kb)
                    a[kb] = load_bf16x8(L.hr + (mt * 16 + r) * kHStride + kb * 32 + 8 * g);
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const int t = 2 * qp + j;
                    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int kb = 0; kb < kHidden / 32; ++kb)
                        acc = mfma_bf16(a[kb], bw[j][kb], acc);
                    uint16_t h[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const float dz = z1[mt][j][i] > 0.f ? acc[i] : 0.f;
                        db1[j] += dz;
                        h[i] = f32_to_bf16(dz);
                    }
                    *reinterpret_cast<uint2 *>(L.z1t + (t * 16 + r) * kTStride + mt * 16 +
                                               4 * g) =
                        uint2{h[0] | ((uint32_t)h[1] << 16), h[2] | ((uint32_t)h[3] << 16)};
                }
            }
        }
        __syncthreads();
        // weight gradients over the chunk's rows: this wave owns output rows
        // (hidden units) 32 wave .. 32 wave + 31 of dW2 and dW1
#pragma unroll
        for (int kk = 0; kk < kChunk / 32; ++kk) {
            bf16x8 a2[2], a1[2];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int n = (2 * wave + q) * 16 + r;
                a2[q] = load_bf16x8(L.z2t + n * kTStride + kk * 32 + 8 * g);
                a1[q] = load_bf16x8(L.z1t + n * kTStride + kk * 32 + 8 * g);
            }
#pragma unroll
            for (int kt = 0; kt < 8; ++kt) {
                const bf16x8 b = load_bf16x8(L.ht + (kt * 16 + r) * kTStride + kk * 32 + 8 * g);
#pragma unroll
                for (int q = 0; q < 2; ++q)
                    acc2[q * 8 + kt] = mfma_bf16(a2[q], b, acc2[q * 8 + kt]);
            }
#pragma unroll
            for (int kt = 0; kt < 2; ++kt) {
                const bf16x8 b = load_bf16x8(L.xt + (kt * 16 + r) * kTStride + kk * 32 + 8 * g);
#pragma unroll
                for (int q = 0; q < 2; ++q)
                    acc1[q * 2 + kt] = mfma_bf16(a1[q], b, acc1[q * 2 + kt]);
            }
        }
        __syncthreads();
    }

    // weight matrices: plain stores of this workgroup's sums
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int n0 = (2 * wave + q) * 16 + 4 * g;
#pragma unroll
        for (int kt = 0; kt < 8; ++kt)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                part(kOffW2 + (n0 + i) * kHidden + kt * 16 + r) = acc2[q * 8 + kt][i];
#pragma unroll
        for (int kt = 0; kt < 2; ++kt)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                part(kOffW1 + (n0 + i) * kIn + kt * 16 + r) = acc1[q * 2 + kt][i];
    }
    // vectors: the wave's own tiles, summed over the four row groups
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        float a = db1[j], b = db2[j], c = dw3[j];
        a += __shfl_xor(a, 16);
        a += __shfl_xor(a, 32);
        b += __shfl_xor(b, 16);
        b += __shfl_xor(b, 32);
        c += __shfl_xor(c, 16);
        c += __shfl_xor(c, 32);
        if (g == 0) {
            const int u = (2 * wave + j) * 16 + r;
            part(kOffB1 + u) = a;
            part(kOffB2 + u) = b;
            part(kOffW3 + u) = c;
        }
    }
    // the output bias, loss and row-weight sums over the rows (wave 0)
    if (wave == 0) {
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            db3 += __shfl_xor(db3, o);
            lsum += __shfl_xor(lsum, o);
            wsum += __shfl_xor(wsum, o);
        }
        if (lane == 0) {
            part(kOffB3) = db3;
            part(kParams + 1) = lsum;
            part(kParams) = wsum;
        }
    }
    if (threadIdx.x == 0)
        part(kParams + 2) = __uint_as_float(*step + 1u);
}

// BF16 copies of parameter k from its master value.
__device__ __forceinline__ void publish(const MlpModelDev &M, int k, float v)
{
    if (k < kOffB1) {
        M.W1[k] = f32_to_bf16(v);
    } else if (k >= kOffW2 && k < kOffB2) {
        const int e = k - kOffW2, n = e / kHidden, c = e - n * kHidden;
        const uint16_t h = f32_to_bf16(v);
        M.W2[e] = h;
        M.W2T[c * kHidden + n] = h;
    } else if (k >= kOffW3 && k < kOffB3) {
        M.w3[k - kOffW3] = f32_to_bf16(v);
    }
}

// Sum the partials of `blocks` training workgroups: gradient = sum / (row
// weight sum).  With lr > 0, an Adam step on the master parameters and their
// BF16 copies.  Nothing happens when the row weights sum to zero.
// Workgroup layout: 64 parameters x 8 partial groups; thread (k, q) adds the
// partials of workgroups q, q + 8, ... in order, then the 8 group sums are
// added in order, so the result does not depend on scheduling.
constexpr int kUpdGroups = 8;
constexpr int kUpdMaxBlocks = kMaxTrainBlocks;

__global__ __launch_bounds__(64 * kUpdGroups) void k_mlp_update(MlpModelDev M,
                                                                 const float *partials,
                                                                 int blocks, float lr,
                                                                 float *grad_out,
                                                                 float *loss_out,
                                                                 TrainGate gate)
{
    __shared__ float hn[kUpdMaxBlocks], hl[kUpdMaxBlocks];
    __shared__ float red[kUpdGroups][64];
    __shared__ float tot[2];
    const int tx = threadIdx.x & 63, q = threadIdx.x >> 6;
    if (threadIdx.x < blocks) {
        hn[threadIdx.x] = partials[part_index(threadIdx.x, kParams)];
        hl[threadIdx.x] = partials[part_index(threadIdx.x, kParams + 1)];
    }
    const int k = blockIdx.x * 64 + tx;
    float s = 0.f;
    if (k < kParams) {
        float v[kUpdMaxBlocks / kUpdGroups];
#pragma unroll
        for (int r = 0; r < kUpdMaxBlocks / kUpdGroups; ++r) {
            const int b = q + kUpdGroups * r;
            v[r] = b < blocks ? partials[part_index(b, k)] : 0.f;
        }
#pragma unroll
        for (int r = 0; r < kUpdMaxBlocks / kUpdGroups; ++r)
            s += v[r];
    }
    red[q][tx] = s;
    __syncthreads();
    if (threadIdx.x < 64) {  // row-weight and loss sums: lane l adds 4 l .. 4 l + 3, then a
                             // butterfly (the same order in every workgroup)
        float n = 0.f, l = 0.f;
#pragma unroll
        for (int i = 0; i < kUpdMaxBlocks / 64; ++i) {
            const int b = (int)threadIdx.x * (kUpdMaxBlocks / 64) + i;
            n += b < blocks ? hn[b] : 0.f;
            l += b < blocks ? hl[b] : 0.f;
        }
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            n += __shfl_xor(n, o);
            l += __shfl_xor(l, o);
        }
        if (threadIdx.x == 0) {
            tot[0] = n;
            tot[1] = l;
        }
    }
    __syncthreads();
    const float n = tot[0];
    if (!(n > 0.f) || q != 0)
        return;
    if (blockIdx.x == 0 && tx == 0) {
        if (loss_out)
            *loss_out = tot[1] / (2.f * n);
        if (lr > 0.f) {
            *M.step = __float_as_uint(partials[part_index(0, kParams + 2)]);
            if (gate.last)
                *gate.last = *gate.gen;
        }
    }
    if (k >= kParams)
        return;
    float sum = 0.f;
#pragma unroll
    for (int g = 0; g < kUpdGroups; ++g)
        sum += red[g][tx];
    const float gk = sum / n;
    if (grad_out)
        grad_out[k] = gk;
    if (!(lr > 0.f))
        return;
    const float t = (float)__float_as_uint(partials[part_index(0, kParams + 2)]);
    const float beta1 = 0.9f, beta2 = 0.999f, eps = 1e-8f;
    const float m = beta1 * M.m1[k] + (1.f - beta1) * gk;
    const float v = beta2 * M.m2[k] + (1.f - beta2) * gk * gk;
    M.m1[k] = m;
    M.m2[k] = v;
    const float mh = m / (1.f - powf(beta1, t));
    const float vh = v / (1.f - powf(beta2, t));
    const float p = M.master[k] - lr * mh / (sqrtf(vh) + eps);
    M.master[k] = p;
    publish(M, k, p);
}

__global__ void k_mlp_publish(MlpModelDev M)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < kParams)
        publish(M, k, M.master[k]);
}

// Weight matrices uniform in [-a, a], a = sqrt(6 / (fan_in + fan_out))
// (Glorot & Bengio, AISTATS 2010), biases zero, Adam state cleared.
// Parameter k takes the top 24 bits of the first word of its own Philox
// stream: u = (x >> 40) / 2^24, value (2u - 1) a.
__global__ void k_mlp_init(MlpModelDev M, uint64_t seed)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k == 0)
        *M.step = 0;
    if (k >= kParams)
        return;
    float a = 0.f;
    if (k < kOffB1)
        a = sqrtf(6.f / (float)(kIn + kHidden));
    else if (k >= kOffW2 && k < kOffB2)
        a = sqrtf(6.f / (float)(kHidden + kHidden));
    else if (k >= kOffW3 && k < kOffB3)
        a = sqrtf(6.f / (float)(kHidden + 1));
    PhiloxStream st(seed, ROLE_MODEL, 0, (uint64_t)k, TAG_WEIGHTS, 0);
    const float u = (float)(st.next() >> 40) * (1.f / 16777216.f);
    const float v = (2.f * u - 1.f) * a;
    M.master[k] = v;
    M.m1[k] = 0.f;
    M.m2[k] = 0.f;
    publish(M, k, v);
}

__global__ void k_to_bf16(const float *x, uint16_t *y, int64_t count)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < count)
        y[k] = f32_to_bf16(x[k]);
}

__global__ void k_from_bf16(const uint16_t *x, float *y, int64_t count)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < count)
        y[k] = bf16_to_f32(x[k]);
}

unsigned grid_for(int64_t count, int per) { return (unsigned)((count + per - 1) / per); }

}  // namespace

hipError_t launch_mlp_forward(const MlpDev &P, const uint16_t *X, int rows, float *y,
                              hipStream_t s)
{
    if (rows <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_mlp_forward, dim3(grid_for(rows, 16 * kWaves)), dim3(64 * kWaves),
                       0, s, P, X, rows, y);
    return hipGetLastError();
}

hipError_t launch_mlp_grad(const MlpDev &P, const uint16_t *X, const float *T,
                           const float *Wt, int rows, float *partials, int max_blocks,
                           const MlpModelDev &M, TrainGate gate, int *blocks,
                           hipStream_t s)
{
    int nb = (int)grid_for(rows > 0 ? rows : 1, kChunk);
    if (nb > max_blocks)
        nb = max_blocks;
    if (nb > kMaxTrainBlocks)
        nb = kMaxTrainBlocks;
    *blocks = nb;
    hipLaunchKernelGGL(k_mlp_grad, dim3(nb), dim3(64 * kWaves), 0, s, P, X, T, Wt, rows,
                       partials, (const uint32_t *)M.step, gate);
    return hipGetLastError();
}

hipError_t launch_mlp_update(const MlpModelDev &M, const float *partials, int blocks,
                             float lr, float *grad_out, float *loss_out, TrainGate gate,
                             hipStream_t s)
{
    if (blocks > kUpdMaxBlocks)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mlp_update, dim3(grid_for(kParams, 64)), dim3(64 * kUpdGroups), 0, s,
                       M, partials, blocks, lr, grad_out, loss_out, gate);
    return hipGetLastError();
}

hipError_t launch_mlp_publish(const MlpModelDev &M, hipStream_t s)
{
    hipLaunchKernelGGL(k_mlp_publish, dim3(grid_for(kParams, 256)), dim3(256), 0, s, M);
    return hipGetLastError();
}

hipError_t launch_mlp_init(const MlpModelDev &M, uint64_t seed, hipStream_t s)
{
    hipLaunchKernelGGL(k_mlp_init, dim3(grid_for(kParams, 256)), dim3(256), 0, s, M, seed);
    return hipGetLastError();
}

hipError_t launch_to_bf16(const float *x, uint16_t *y, int64_t count, hipStream_t s)
{
    if (count <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_to_bf16, dim3(grid_for(count, 256)), dim3(256), 0, s, x, y, count);
    return hipGetLastError();
}

hipError_t launch_from_bf16(const uint16_t *x, float *y, int64_t count, hipStream_t s)
{
    if (count <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_from_bf16, dim3(grid_for(count, 256)), dim3(256), 0, s, x, y,
                       count);
    return hipGetLastError();
}

}  // namespace pmp
