// All-pairs shortest paths by blocked Floyd-Warshall (Floyd, CACM 1962;
// the three-phase tiling of Venkataraman et al., JEA 2003): the step that
// turns a graph instance (edge weights) into the distance matrix d that
// preprocessing sorts.  Distances are uint32 in a padded work matrix with
// INF = 0x7FFFFFFF for "no path"; every finite distance stays below INF (the
// host checks (n - 1) * max weight < INF), so a + b never wraps in 32 bits
// and min(d_ij, a + b) never exceeds d_ij <= INF: an update is one add and
// one min.
//
// Per round kb (tile 64 x 64):
//  - k_fw_panels: every workgroup first closes the diagonal tile (kb, kb)
//    over its own 64 intermediate vertices (redundantly, in LDS), then one
//    tile of row kb or of column kb through it; the workgroup of the
//    diagonal itself stores it;
//  - k_fw_rest: every other tile (i, j) takes min over k of
//    D(i, kb)[., k] + D(kb, j)[k, .] - a min-plus product of the two panel
//    tiles, staged in LDS, 4 x 4 elements per thread.
#include <algorithm>

#include "common.hpp"

namespace pmp {

namespace {

constexpr int kTile = 64;
constexpr uint32_t kInf = 0x7FFFFFFFu;

__device__ __forceinline__ uint32_t tile_at(const uint32_t *D, int ld, int ti, int tj, int r,
                                            int c)
{
    return D[(int64_t)(ti * kTile + r) * ld + tj * kTile + c];
}

// A thread's 4 x 4 block of a 64 x 64 tile: rows 4 ty .. 4 ty + 3, columns
// 4 tx .. 4 tx + 3 (ty = thread / 16, tx = thread % 16).
struct Block {
    uint32_t v[4][4];
};

__device__ __forceinline__ void load_block(Block &b, const uint32_t *D, int ld, int ti, int tj)
{
    const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const uint4 q = *reinterpret_cast<const uint4 *>(
            &D[(int64_t)(ti * kTile + 4 * ty + r) * ld + tj * kTile + 4 * tx]);
        b.v[r][0] = q.x;
        b.v[r][1] = q.y;
        b.v[r][2] = q.z;
        b.v[r][3] = q.w;
    }
}

__device__ __forceinline__ void store_block(const Block &b, uint32_t *D, int ld, int ti, int tj)
{
    const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
#pragma unroll
    for (int r = 0; r < 4; ++r)
        *reinterpret_cast<uint4 *>(&D[(int64_t)(ti * kTile + 4 * ty + r) * ld + tj * kTile + 4 * tx]) =
            make_uint4(b.v[r][0], b.v[r][1], b.v[r][2], b.v[r][3]);
}

// Row k and column k of a tile held in registers, published for step k:
// the threads holding column k write it to col[k & 1], those holding row k
// to row[k & 1].  Double buffering needs one barrier per step: a buffer is
// rewritten two steps later, after every thread has passed the next barrier.
struct Lines {
    uint32_t row[2][kTile];
    uint32_t col[2][kTile];
};

__device__ __forceinline__ void publish(const Block &b, Lines &L, int k, bool pub_row,
                                        bool pub_col)
{
    const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
    const int q = k & 3;  // selected, not indexed: a run-time index would spill the block
    if (pub_col && tx == (k >> 2)) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
            L.col[k & 1][4 * ty + r] =
                q == 0 ? b.v[r][0] : q == 1 ? b.v[r][1] : q == 2 ? b.v[r][2] : b.v[r][3];
    }
    if (pub_row && ty == (k >> 2)) {
#pragma unroll
        for (int c = 0; c < 4; ++c)
            L.row[k & 1][4 * tx + c] =
                q == 0 ? b.v[0][c] : q == 1 ? b.v[1][c] : q == 2 ? b.v[2][c] : b.v[3][c];
    }
}

__device__ __forceinline__ void relax(Block &b, const uint32_t a[4], const uint32_t c[4])
{
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q)
            b.v[r][q] = min(b.v[r][q], a[r] + c[q]);
}

__device__ __forceinline__ void read4(const uint32_t *p, uint32_t out[4])
{
    const uint4 q = *reinterpret_cast<const uint4 *>(p);
    out[0] = q.x;
    out[1] = q.y;
    out[2] = q.z;
    out[3] = q.w;
}

// Close the diagonal tile over its own 64 vertices, in registers: step k
// relaxes every entry through vertex k (row k and column k do not change
// during step k, the diagonal entry being 0).
__device__ __forceinline__ void close_diagonal(Block &g, Lines &L)
{
    const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
    for (int k = 0; k < kTile; ++k) {
        publish(g, L, k, true, true);
        __syncthreads();
        uint32_t a[4], c[4];
        read4(&L.col[k & 1][4 * ty], a);
        read4(&L.row[k & 1][4 * tx], c);
        relax(g, a, c);
    }
}

// Phases 1 and 2 of round kb.  Workgroup b < nb: row tile (kb, b);
// nb <= b < 2 nb: column tile (b - nb, kb).  Every workgroup closes the
// diagonal tile itself (no extra launch); the diagonal's own workgroups
// (b = kb and b = nb + kb) stop there, and b = kb stores it.  A row tile
// then relaxes through the closed diagonal's column k and its own row k, a
// column tile through its own column k and the diagonal's row k.
__global__ __launch_bounds__(256) void k_fw_panels(uint32_t *D, int ld, int nb, int kb)
{
    __shared__ __attribute__((aligned(16))) Lines L;
    // the closed diagonal: Gt[k][i] = G[i][k] (columns), G[k][j] (rows)
    __shared__ __attribute__((aligned(16))) uint32_t Gt[kTile][kTile + 4];
    __shared__ __attribute__((aligned(16))) uint32_t G[kTile][kTile + 4];
    const int b = blockIdx.x;
    const bool row = b < nb;
    const int other = row ? b : b - nb;
    const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
    const bool diag = other == kb;
    Block g, t;
    load_block(g, D, ld, kb, kb);
    if (!diag)
        load_block(t, D, ld, row ? kb : other, row ? other : kb);
    close_diagonal(g, L);
    if (diag) {
        if (row)
            store_block(g, D, ld, kb, kb);
        return;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            Gt[4 * tx + c][4 * ty + r] = g.v[r][c];
            G[4 * ty + r][4 * tx + c] = g.v[r][c];
        }
    __syncthreads();
    for (int k = 0; k < kTile; ++k) {
        publish(t, L, k, row, !row);
        __syncthreads();
        uint32_t a[4], c[4];
        if (row) {
            read4(&Gt[k][4 * ty], a);
            read4(&L.row[k & 1][4 * tx], c);
        } else {
            read4(&L.col[k & 1][4 * ty], a);
            read4(&G[k][4 * tx], c);
        }
        relax(t, a, c);
    }
    store_block(t, D, ld, row ? kb : other, row ? other : kb);
}

// Phase 3 of round kb: tile (i, j) off row and column kb.  The column-panel
// tile is staged transposed so each thread reads its 4 rows' entries of
// column k with one 16-byte LDS read, and the row-panel tile's 4 columns of
// row k likewise.
__global__ __launch_bounds__(256) void k_fw_rest(uint32_t *D, int ld, int nb, int kb)
{
    // rows padded by 4 words: the transposing stores spread over the banks,
    // and rows stay 16-byte aligned
    __shared__ __attribute__((aligned(16))) uint32_t At[kTile][kTile + 4];  // At[k][i] = D(i, kb)[i][k]
    __shared__ __attribute__((aligned(16))) uint32_t B[kTile][kTile + 4];   // B[k][j] = D(kb, j)[k][j]
    const int nrest = nb - 1;
    const int ii = blockIdx.x / nrest, jj = blockIdx.x - ii * nrest;
    const int ti = ii < kb ? ii : ii + 1, tj = jj < kb ? jj : jj + 1;
    for (int e = threadIdx.x; e < kTile * kTile; e += 256) {
        const int r = e >> 6, c = e & 63;
        At[c][r] = tile_at(D, ld, ti, kb, r, c);
        B[r][c] = tile_at(D, ld, kb, tj, r, c);
    }
    const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
    uint32_t acc[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const uint4 v = *reinterpret_cast<const uint4 *>(
            &D[(int64_t)(ti * kTile + 4 * ty + r) * ld + tj * kTile + 4 * tx]);
        acc[r][0] = v.x;
        acc[r][1] = v.y;
        acc[r][2] = v.z;
        acc[r][3] = v.w;
    }
    __syncthreads();
#pragma unroll 8
    for (int k = 0; k < kTile; ++k) {
        const uint4 a = *reinterpret_cast<const uint4 *>(&At[k][4 * ty]);
        const uint4 bb = *reinterpret_cast<const uint4 *>(&B[k][4 * tx]);
        const uint32_t av[4] = {a.x, a.y, a.z, a.w};
        const uint32_t bv[4] = {bb.x, bb.y, bb.z, bb.w};
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c)
                acc[r][c] = min(acc[r][c], av[r] + bv[c]);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
        *reinterpret_cast<uint4 *>(&D[(int64_t)(ti * kTile + 4 * ty + r) * ld + tj * kTile + 4 * tx]) =
            make_uint4(acc[r][0], acc[r][1], acc[r][2], acc[r][3]);
}

// Work matrix from the weights: INF where there is no edge (w < 0) and in the
// padding, 0 on the diagonal, and the largest weight into *wmax (a grid-stride
// loop, so that only a few thousand waves meet at the one atomic).
__global__ __launch_bounds__(256) void k_fw_in(const int32_t *w, int64_t ldw, int n, uint32_t *D,
                                               int ld, uint32_t *wmax)
{
    const int64_t cells = (int64_t)ld * ld;
    uint32_t mx = 0;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < cells;
         e += (int64_t)gridDim.x * 256) {
        const int i = (int)(e / ld), j = (int)(e - (int64_t)i * ld);
        uint32_t v = kInf;
        if (i < n && j < n) {
            const int32_t x = w[(int64_t)i * ldw + j];
            if (x >= 0) {
                v = (uint32_t)x;
                mx = max(mx, v);
            }
        }
        if (i == j)
            v = 0;
        D[e] = v;
    }
    // one atomic per wave (every lane takes part in the shuffles)
#pragma unroll
    for (int dd = 32; dd > 0; dd >>= 1)
        mx = max(mx, (uint32_t)__shfl_xor((int)mx, dd));
    if ((threadIdx.x & 63) == 0 && mx > 0)
        atomicMax(wmax, mx);
}

// Distances out: -1 for INF (no path).
__global__ __launch_bounds__(256) void k_fw_out(const uint32_t *D, int ld, int n, int32_t *d,
                                                int64_t ldd)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)n * n)
        return;
    const int i = (int)(e / n), j = (int)(e - (int64_t)i * n);
    const uint32_t v = D[(int64_t)i * ld + j];
    d[(int64_t)i * ldd + j] = v >= kInf ? -1 : (int32_t)v;
}

}  // namespace

int apsp_padded(int n)
{
    return ((n + kTile - 1) / kTile) * kTile;
}

hipError_t launch_apsp_in(const int32_t *w, int64_t ldw, int n, uint32_t *D, uint32_t *wmax,
                          hipStream_t s)
{
    const int ld = apsp_padded(n);
    const int64_t cells = (int64_t)ld * ld;
    const int64_t blocks = std::min<int64_t>((cells + 255) / 256, 2048);
    hipLaunchKernelGGL(k_fw_in, dim3((unsigned)blocks), dim3(256), 0, s, w, ldw, n, D, ld, wmax);
    return hipGetLastError();
}

hipError_t launch_apsp_rounds(uint32_t *D, int n, hipStream_t s)
{
    const int ld = apsp_padded(n), nb = ld / kTile;
    for (int kb = 0; kb < nb; ++kb) {
        hipLaunchKernelGGL(k_fw_panels, dim3(2 * nb), dim3(256), 0, s, D, ld, nb, kb);
        if (nb > 1)
            hipLaunchKernelGGL(k_fw_rest, dim3((nb - 1) * (nb - 1)), dim3(256), 0, s, D, ld, nb,
                               kb);
    }
    return hipGetLastError();
}

hipError_t launch_apsp_out(const uint32_t *D, int n, int32_t *d, int64_t ldd, hipStream_t s)
{
    const int ld = apsp_padded(n);
    const int64_t cells = (int64_t)n * n;
    hipLaunchKernelGGL(k_fw_out, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0, s, D, ld, n,
                       d, ldd);
    return hipGetLastError();
}

}  // namespace pmp
