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

__global__ __launch_bounds__(64 * kWaves) void k_mlp_forward(MlpDev P, const uint16_t *X,
                                                            int rows, float *y)
{
    __shared__ __align__(16) uint16_t xs[kWaves][16 * kXStride];
    __shared__ __align__(16) uint16_t hs[kWaves][16 * kHStride];
    const int wave = wave_id(), lane = threadIdx.x & 63;
    const int64_t row0 = ((int64_t)blockIdx.x * kWaves + wave) * 16;
    if (row0 >= rows)
        return;
    stage_rows16(X, row0, rows, xs[wave], lane);
    wave_lds_sync();
    f32x4 z1[8], z2[8];
    float out[4];
    mlp_forward16(P, xs[wave], hs[wave], lane, z1, z2, out);
    if ((lane & 15) == 0)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t row = row0 + 4 * (lane >> 4) + i;
            if (row < rows)
                y[row] = out[i];
        }
}

struct GradLds {
    uint16_t xr[kChunk * kXStride];      // inputs, row-major
    uint16_t xt[kIn * kTStride];         // inputs, transposed
    uint16_t hr[kChunk * kHStride];      // h1 row-major, then dz2 row-major
    uint16_t ht[kHidden * kTStride];     // h1 transposed
    uint16_t z2t[kHidden * kTStride];    // dz2 transposed
    uint16_t z1t[kHidden * kTStride];    // dz1 transposed
    float vec[kWaves][3 * kHidden + 4];  // per-wave vector partials
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
    float *part = partials + (int64_t)blockIdx.x * kPartStride;
    if (threadIdx.x == 0) {
        int train = 1;
        if (gate.gen) {
            const unsigned long long gen = *gate.gen;
            train = gen > 0 && gen % (unsigned long long)gate.every == 0 && gen != *gate.last;
        }
        L.train = train;
        if (!train)
            part[kParams] = 0.f;  // no rows: the update kernel skips
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
    float db1[8], db2[8], dw3[8];
#pragma unroll
    for (int t = 0; t < 8; ++t)
        db1[t] = db2[t] = dw3[t] = 0.f;
    float db3 = 0.f, lsum = 0.f, wsum = 0.f;

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

        const int wr = wave * 16;  // this wave's first row in the chunk
        f32x4 z1[8], z2[8];
        float y[4];
        mlp_forward16(P, L.xr + wr * kXStride, L.hr + wr * kHStride, lane, z1, z2, y);
        // h1 transposed (the D layout holds four consecutive rows per lane)
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const uint32_t lo = f32_to_bf16(fmaxf(z1[t][0], 0.f)) |
                                ((uint32_t)f32_to_bf16(fmaxf(z1[t][1], 0.f)) << 16);
            const uint32_t hi = f32_to_bf16(fmaxf(z1[t][2], 0.f)) |
                                ((uint32_t)f32_to_bf16(fmaxf(z1[t][3], 0.f)) << 16);
            *reinterpret_cast<uint2 *>(L.ht + (t * 16 + r) * kTStride + wr + 4 * g) =
                uint2{lo, hi};
        }
        // output error and row weights
        float dy[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t row = row0 + wr + 4 * g + i;
            float e = 0.f, w = 0.f;
            if (row < rows) {
                w = Wt ? Wt[row] : 1.f;
                e = y[i] - T[row];
            }
            dy[i] = w * e;
            if (r == 0) {
                lsum += w * e * e;
                wsum += w;
                db3 += w * e;
            }
        }
        // dz2 = dy w3 relu'(z2); dw3 += dy h2; db2 += dz2
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const float w = bf16_to_f32(P.w3[t * 16 + r]);
            uint16_t h[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float z = z2[t][i];
                dw3[t] += dy[i] * fmaxf(z, 0.f);
                const float dz = z > 0.f ? dy[i] * w : 0.f;
                db2[t] += dz;
                h[i] = f32_to_bf16(dz);
                L.hr[(wr + 4 * g + i) * kHStride + t * 16 + r] = h[i];
            }
            *reinterpret_cast<uint2 *>(L.z2t + (t * 16 + r) * kTStride + wr + 4 * g) =
                uint2{h[0] | ((uint32_t)h[1] << 16), h[2] | ((uint32_t)h[3] << 16)};
        }
        wave_lds_sync();
        // dz1 = (dz2 W2) relu'(z1); db1 += dz1
        {
            bf16x8 a[kHidden / 32];
#pragma unroll
            for (int kb = 0; kb < kHidden / 32; ++kb)
                a[kb] = load_bf16x8(L.hr + (wr + r) * kHStride + kb * 32 + 8 * g);
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kb = 0; kb < kHidden / 32; ++kb)
                    acc = mfma_bf16(a[kb],
                                    load_bf16x8(P.W2T + (t * 16 + r) * kHidden + kb * 32 + 8 * g),
                                    acc);
                uint16_t h[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float dz = z1[t][i] > 0.f ? acc[i] : 0.f;
                    db1[t] += dz;
                    h[i] = f32_to_bf16(dz);
                }
                *reinterpret_cast<uint2 *>(L.z1t + (t * 16 + r) * kTStride + wr + 4 * g) =
                    uint2{h[0] | ((uint32_t)h[1] << 16), h[2] | ((uint32_t)h[3] << 16)};
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
                part[kOffW2 + (n0 + i) * kHidden + kt * 16 + r] = acc2[q * 8 + kt][i];
#pragma unroll
        for (int kt = 0; kt < 2; ++kt)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                part[kOffW1 + (n0 + i) * kIn + kt * 16 + r] = acc1[q * 2 + kt][i];
    }
    // vectors: sum the four row groups of the wave, then the waves in order
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        float a = db1[t], b = db2[t], c = dw3[t];
        a += __shfl_xor(a, 16);
        a += __shfl_xor(a, 32);
        b += __shfl_xor(b, 16);
        b += __shfl_xor(b, 32);
        c += __shfl_xor(c, 16);
        c += __shfl_xor(c, 32);
        if (g == 0) {
            L.vec[wave][t * 16 + r] = a;
            L.vec[wave][kHidden + t * 16 + r] = b;
            L.vec[wave][2 * kHidden + t * 16 + r] = c;
        }
    }
    db3 += __shfl_xor(db3, 16);
    db3 += __shfl_xor(db3, 32);
    lsum += __shfl_xor(lsum, 16);
    lsum += __shfl_xor(lsum, 32);
    wsum += __shfl_xor(wsum, 16);
    wsum += __shfl_xor(wsum, 32);
    if (lane == 0) {
        L.vec[wave][3 * kHidden] = db3;
        L.vec[wave][3 * kHidden + 1] = lsum;
        L.vec[wave][3 * kHidden + 2] = wsum;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < 3 * kHidden + 3; k += blockDim.x) {
        float v = 0.f;
        for (int w = 0; w < kWaves; ++w)
            v += L.vec[w][k];
        if (k < kHidden)
            part[kOffB1 + k] = v;
        else if (k < 2 * kHidden)
            part[kOffB2 + k - kHidden] = v;
        else if (k < 3 * kHidden)
            part[kOffW3 + k - 2 * kHidden] = v;
        else if (k == 3 * kHidden)
            part[kOffB3] = v;
        else if (k == 3 * kHidden + 1)
            part[kParams + 1] = v;
        else
            part[kParams] = v;
    }
    if (threadIdx.x == 0)
        part[kParams + 2] = __uint_as_float(*step + 1u);
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
constexpr int kUpdMaxBlocks = 256;

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
        hn[threadIdx.x] = partials[(int64_t)threadIdx.x * kPartStride + kParams];
        hl[threadIdx.x] = partials[(int64_t)threadIdx.x * kPartStride + kParams + 1];
    }
    const int k = blockIdx.x * 64 + tx;
    float s = 0.f;
    if (k < kParams) {
        float v[kUpdMaxBlocks / kUpdGroups];
#pragma unroll
        for (int r = 0; r < kUpdMaxBlocks / kUpdGroups; ++r) {
            const int b = q + kUpdGroups * r;
            v[r] = b < blocks ? partials[(int64_t)b * kPartStride + k] : 0.f;
        }
#pragma unroll
        for (int r = 0; r < kUpdMaxBlocks / kUpdGroups; ++r)
            s += v[r];
    }
    red[q][tx] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        float n = 0.f, l = 0.f;
        for (int b = 0; b < blocks; ++b) {
            n += hn[b];
            l += hl[b];
        }
        tot[0] = n;
        tot[1] = l;
    }
    __syncthreads();
    const float n = tot[0];
    if (!(n > 0.f) || q != 0)
        return;
    if (blockIdx.x == 0 && tx == 0) {
        if (loss_out)
            *loss_out = tot[1] / (2.f * n);
        if (lr > 0.f) {
            *M.step = __float_as_uint(partials[kParams + 2]);
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
    const float t = (float)__float_as_uint(partials[kParams + 2]);
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
