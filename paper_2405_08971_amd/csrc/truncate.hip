// Truncation (Sec. 3.2) support kernels on gfx950: the FP64 Gram matrix M^T M of the
// downdate factor and the extraction of the leading eigenvectors.  The eigensolver
// itself (FP64) and the rotation M V_r (FP32 GEMM) are library calls made by the host.
#include "cakf_common.h"
#include "launchers.h"

namespace cakf {

constexpr int GT = 64;        // Gram tile side
constexpr int GROWS = 32;     // factor rows staged per LDS chunk

// Partial Gram tiles: block (tile, split) accumulates M[rows, c-block]^T M[rows, d-block]
// over its row range in FP64 (FP32 inputs; each product is exact in FP64), for
// lower-triangle tiles c-block >= d-block.  Each thread owns a 4 x 4 set of outputs and
// reads one float4 of each operand per staged row.
__global__ __launch_bounds__(256) void k_gram_partial(const float* __restrict__ M, int n,
                                                      int ldM, int K, int nsplit,
                                                      double* __restrict__ work) {
    __shared__ float As[GROWS][GT + 4], Bs[GROWS][GT + 4];
    const int tile = blockIdx.x / nsplit, split = blockIdx.x % nsplit;
    int tc = (int)((sqrtf(8.0f * (float)tile + 1.0f) - 1.0f) * 0.5f);
    while ((tc + 1) * (tc + 2) / 2 <= tile) ++tc;
    while (tc * (tc + 1) / 2 > tile) --tc;
    const int td = tile - tc * (tc + 1) / 2;       // td <= tc
    const int c0 = tc * GT, d0 = td * GT;
    const int rows_per = (n + nsplit - 1) / nsplit;
    const int r0 = split * rows_per, r1 = min(n, r0 + rows_per);
    const int tid = threadIdx.x;
    const int ti = tid >> 4, tj = tid & 15;
    double acc[4][4];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = 0.0;
    for (int p0 = r0; p0 < r1; p0 += GROWS) {
        __syncthreads();
#pragma unroll
        for (int u = 0; u < GROWS * GT / 256; ++u) {
            const int e = tid + 256 * u;
            const int rr = e / GT, cc = e % GT;
            const int p = p0 + rr;
            const bool okr = p < r1;
            As[rr][cc] = (okr && c0 + cc < K) ? M[(size_t)p * ldM + c0 + cc] : 0.0f;
            Bs[rr][cc] = (okr && d0 + cc < K) ? M[(size_t)p * ldM + d0 + cc] : 0.0f;
        }
        __syncthreads();
#pragma unroll 4
        for (int rr = 0; rr < GROWS; ++rr) {
            const float4 a = *reinterpret_cast<const float4*>(&As[rr][4 * ti]);
            const float4 b = *reinterpret_cast<const float4*>(&Bs[rr][4 * tj]);
            const double av[4] = {a.x, a.y, a.z, a.w};
            const double bv[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < 4; ++y) acc[x][y] = __builtin_fma(av[x], bv[y], acc[x][y]);
        }
    }
    double* w = work + (size_t)split * K * K;
#pragma unroll
    for (int x = 0; x < 4; ++x) {
        const int c = c0 + 4 * ti + x;
        if (c >= K) continue;
#pragma unroll
        for (int y = 0; y < 4; ++y) {
            const int dd = d0 + 4 * tj + y;
            if (dd < K) w[(size_t)c * K + dd] = acc[x][y];
        }
    }
}

// G = sum over splits (fixed order), lower tiles mirrored to the full symmetric matrix.
__global__ void k_gram_reduce(const double* __restrict__ work, int K, int nsplit,
                              double* __restrict__ G) {
    const size_t total = (size_t)K * K;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(e / K), d = (int)(e % K);
        if (c / GT < d / GT) continue;                  // upper tiles: mirrored below
        double s = 0.0;
        for (int sp = 0; sp < nsplit; ++sp) s += work[(size_t)sp * total + e];
        G[e] = s;
        if (c / GT != d / GT) G[(size_t)d * K + c] = s;
    }
}

void launch_gram64(const float* M, int n, int ldM, int K, double* G, double* work,
                   size_t work_elems, hipStream_t st) {
    const int nt = (K + GT - 1) / GT;
    const int tiles = nt * (nt + 1) / 2;
    int nsplit = std::max(1, (2048 + tiles - 1) / tiles);
    nsplit = std::min(nsplit, std::max(1, n / 256));
    while (nsplit > 1 && (size_t)nsplit * K * K > work_elems) --nsplit;
    hipLaunchKernelGGL(k_gram_partial, dim3(tiles * nsplit), dim3(256), 0, st, M, n, ldM, K,
                       nsplit, work);
    const size_t total = (size_t)K * K;
    const int blocks = (int)std::min<size_t>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(k_gram_reduce, dim3(blocks), dim3(256), 0, st, work, K, nsplit, G);
}

// The eigensolver returns eigenvalues in ascending order with eigenvectors as columns
// of E (column-major K x K).  V_r keeps the r leading ones in descending order:
// Vr (FP32, column-major K x r) and, optionally, rot_out (FP64, row-major K x r).
__global__ void k_pick_rotation(const double* __restrict__ E, int K, int r,
                                float* __restrict__ Vr, double* __restrict__ rot_out) {
    const size_t total = (size_t)K * r;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(e / K), k = (int)(e % K);
        const double v = E[(size_t)(K - 1 - c) * K + k];
        Vr[(size_t)c * K + k] = (float)v;
        if (rot_out) rot_out[(size_t)k * r + c] = v;
    }
}

void launch_pick_rotation(const double* E, int K, int r, float* Vr, double* rot_out,
                          hipStream_t st) {
    const size_t total = (size_t)K * r;
    const int blocks = (int)std::min<size_t>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(k_pick_rotation, dim3(blocks), dim3(256), 0, st, E, K, r, Vr, rot_out);
}

}  // namespace cakf
