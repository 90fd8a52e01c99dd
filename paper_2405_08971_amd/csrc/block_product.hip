// Block product of the CAKF update on gfx950:  Y = sigma_f2 * K(X, Xo) B  (n x b),
// the matrix-free Sigma H^T [W w] of Alg. 2 (the kernel part of P^- H^T [W w]).  The
// kernel matrix is generated tile by tile in registers/LDS and never stored.
#include "cakf_common.h"
#include "launchers.h"

namespace cakf {

// ------------------------------------------------------------------- FP32 (VALU) form
// Block: 64 state rows x up to 160 columns; the observation axis is walked in chunks of
// 64.  Each chunk: the 64 x 64 kernel tile is evaluated once into LDS (16 entries per
// thread), then every thread accumulates 1 row x 40 columns (columns g + 4 k).
constexpr int BP_ROWS = 64;
constexpr int BP_CHUNK = 64;
constexpr int BP_COLS = 160;
constexpr int BP_CB = BP_COLS / 4;

template <int NU2, int DIST>
__global__ __launch_bounds__(256) void k_block_fp32(const float4* __restrict__ Xs, int n,
                                                    const float4* __restrict__ Xo, int m,
                                                    const float* __restrict__ B, int ldb,
                                                    int col0, int ncols, float sigma_f2,
                                                    float* __restrict__ out, int ldo) {
    __shared__ float4 xo[BP_CHUNK];
    __shared__ float4 Bs[BP_CHUNK][4][BP_CB / 4];      // [q][g][k/4], columns g + 4k
    __shared__ float Kt[BP_ROWS][BP_CHUNK + 1];
    const int tid = threadIdx.x;
    const int row0 = blockIdx.x * BP_ROWS;
    // kernel-tile role: row tr (4 threads per row), 16 observation points each
    const int tr = tid >> 2, tq = (tid & 3) * 16;
    const int prow = min(row0 + tr, n - 1);
    const float4 xr = Xs[prow];
    // contraction role: row cr, column group g
    const int cr = tid & 63, g = tid >> 6;
    float acc[BP_CB];
#pragma unroll
    for (int k = 0; k < BP_CB; ++k) acc[k] = 0.0f;

    for (int q0 = 0; q0 < m; q0 += BP_CHUNK) {
        const int qn = min(BP_CHUNK, m - q0);
        __syncthreads();
        if (tid < BP_CHUNK) xo[tid] = Xo[q0 + min(tid, qn - 1)];
        // B chunk: qn rows x ncols columns into the [q][g][k] layout (zero padded)
        for (int e = tid; e < BP_CHUNK * BP_COLS; e += 256) {
            const int q = e / BP_COLS, c = e % BP_COLS;
            float v = 0.0f;
            if (q < qn && c < ncols) v = B[(size_t)(q0 + q) * ldb + col0 + c];
            float* dst = reinterpret_cast<float*>(&Bs[q][c & 3][0]);
            dst[c >> 2] = v;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 16; ++u) Kt[tr][tq + u] = kval<NU2, DIST>(xr, xo[tq + u]);
        __syncthreads();
        for (int q = 0; q < qn; ++q) {
            const float kv = Kt[cr][q];
#pragma unroll
            for (int k4 = 0; k4 < BP_CB / 4; ++k4) {
                const float4 b = Bs[q][g][k4];
                acc[4 * k4 + 0] = __builtin_fmaf(kv, b.x, acc[4 * k4 + 0]);
                acc[4 * k4 + 1] = __builtin_fmaf(kv, b.y, acc[4 * k4 + 1]);
                acc[4 * k4 + 2] = __builtin_fmaf(kv, b.z, acc[4 * k4 + 2]);
                acc[4 * k4 + 3] = __builtin_fmaf(kv, b.w, acc[4 * k4 + 3]);
            }
        }
    }
    const int p = row0 + cr;
    if (p < n) {
        float* orow = out + (size_t)p * ldo + col0;
#pragma unroll
        for (int k = 0; k < BP_CB; ++k) {
            const int c = g + 4 * k;
            if (c < ncols) orow[c] = sigma_f2 * acc[k];
        }
    }
}

void launch_block_product(int nu2, int dist, int prec, const float4* Xs, int n,
                          const float4* Xo, int m, const float* B, int ldb, int bcols,
                          float sigma_f2, float* out, int ldo, hipStream_t st) {
    (void)prec;
    const int blocks = (n + BP_ROWS - 1) / BP_ROWS;
    for (int c0 = 0; c0 < bcols; c0 += BP_COLS) {
        const int nc = std::min(BP_COLS, bcols - c0);
        CAKF_DISPATCH_KERNEL(nu2, dist,
            hipLaunchKernelGGL((k_block_fp32<NU2, DIST>), dim3(blocks), dim3(256), 0, st, Xs, n,
                               Xo, m, B, ldb, c0, nc, sigma_f2, out, ldo));
    }
}

}  // namespace cakf
