// Truncation (Sec. 3.2) support kernels on gfx950: the FP64 Gram matrix M^T M of the
// downdate factor and the extraction of the leading eigenvectors.  The eigensolver
// itself (FP64) and the rotation M V_r (FP32 GEMM) are library calls made by the host.
#include "cakf_common.h"
#include "launchers.h"

namespace cakf {

constexpr int GT = 64;        // Gram tile side
constexpr int GROWS = 64;     // factor rows staged per LDS chunk
constexpr int GLD = GT + 16;  // LDS row stride (floats): a wave's 4 x 16 operand reads
                              // fall on distinct banks

typedef double f64x4 __attribute__((ext_vector_type(4)));

// Partial Gram tiles: block (tile, split) accumulates M[rows, c-block]^T M[rows, d-block]
// over its row range in FP64 (FP32 inputs; each product is exact in FP64), for
// lower-triangle tiles c-block >= d-block.  The products run on FP64 MFMA
// (v_mfma_f64_16x16x4f64, D = A B + D over 4 factor rows): wave w owns the 32 x 32
// quarter at rows 32 (w / 2), columns 32 (w % 2) of the 64 x 64 tile as 2 x 2 products.
// Lane l supplies A[l % 16][l / 16] = M[row l / 16, column l % 16 of the c sub-block]
// and B[l / 16][l % 16] = M[row l / 16, column l % 16 of the d sub-block], widened to
// FP64, and holds D[l / 16 + 4 i][l % 16] in register i (rows interleaved by 4, unlike
// the FP32 16 x 16 x 4 form).
//
// Tiles are enumerated row block by row block (tile = tc (tc + 1) / 2 + td); the first
// tile_off of them (the leading columns whose Gram is known, below) are not launched.
__global__ __launch_bounds__(256) void k_gram_partial(const float* __restrict__ M, int n,
                                                      int ldM, int K, int nsplit, int tile_off,
                                                      double* __restrict__ work) {
    __shared__ float As[GROWS][GLD], Bs[GROWS][GLD];
    const int tile = blockIdx.x / nsplit + tile_off, split = blockIdx.x % nsplit;
    int tc = (int)((sqrtf(8.0f * (float)tile + 1.0f) - 1.0f) * 0.5f);
    while ((tc + 1) * (tc + 2) / 2 <= tile) ++tc;
    while (tc * (tc + 1) / 2 > tile) --tc;
    const int td = tile - tc * (tc + 1) / 2;       // td <= tc
    const int c0 = tc * GT, d0 = td * GT;
    const int rows_per = (n + nsplit - 1) / nsplit;
    const int r0 = split * rows_per, r1 = min(n, r0 + rows_per);
    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int cb = 32 * (w >> 1), db = 32 * (w & 1);
    f64x4 acc[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int i = 0; i < 4; ++i) acc[x][y][i] = 0.0;
    // staging: 16-byte loads (factor rows are 16-byte aligned, ldM a multiple of 4), the
    // next chunk's loads issued into registers before the current chunk's products
    constexpr int LD4 = GROWS * GT / 4 / 256;      // float4 loads per operand per thread
    float4 ra[LD4], rb[LD4];
    auto load_chunk = [&](int p0) {
#pragma unroll
        for (int u = 0; u < LD4; ++u) {
            const int e = tid + 256 * u;
            const int rr = e / (GT / 4), c4 = 4 * (e % (GT / 4));
            const int p = p0 + rr;
            float4 a = make_float4(0.0f, 0.0f, 0.0f, 0.0f), b = a;
            if (p < r1) {
                if (c0 + c4 < K) a = *reinterpret_cast<const float4*>(M + (size_t)p * ldM + c0 + c4);
                if (d0 + c4 < K) b = *reinterpret_cast<const float4*>(M + (size_t)p * ldM + d0 + c4);
            }
            // columns at or beyond K (inside the row's 16-byte group) read as zero
            if (c0 + c4 + 3 >= K) {
                if (c0 + c4 + 1 >= K) a.y = 0.0f;
                if (c0 + c4 + 2 >= K) a.z = 0.0f;
                a.w = 0.0f;
            }
            if (d0 + c4 + 3 >= K) {
                if (d0 + c4 + 1 >= K) b.y = 0.0f;
                if (d0 + c4 + 2 >= K) b.z = 0.0f;
                b.w = 0.0f;
            }
            ra[u] = a;
            rb[u] = b;
        }
    };
    if (r0 < r1) load_chunk(r0);
    for (int p0 = r0; p0 < r1; p0 += GROWS) {
        __syncthreads();
#pragma unroll
        for (int u = 0; u < LD4; ++u) {
            const int e = tid + 256 * u;
            const int rr = e / (GT / 4), c4 = 4 * (e % (GT / 4));
            *reinterpret_cast<float4*>(&As[rr][c4]) = ra[u];
            *reinterpret_cast<float4*>(&Bs[rr][c4]) = rb[u];
        }
        __syncthreads();
        if (p0 + GROWS < r1) load_chunk(p0 + GROWS);
#pragma unroll
        for (int ks = 0; ks < GROWS / 4; ++ks) {
            const int rr = 4 * ks + lk;
            double a[2], b[2];
#pragma unroll
            for (int x = 0; x < 2; ++x) a[x] = (double)As[rr][cb + 16 * x + li];
#pragma unroll
            for (int y = 0; y < 2; ++y) b[y] = (double)Bs[rr][db + 16 * y + li];
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y)
                    acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], b[y], acc[x][y], 0, 0, 0);
        }
    }
    double* wk = work + (size_t)split * K * K;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int c = c0 + cb + 16 * x + lk + 4 * i;
                const int dd = d0 + db + 16 * y + li;
                if (c < K && dd < K) wk[(size_t)c * K + dd] = acc[x][y][i];
            }
}

// G = sum over splits (fixed order), lower tiles mirrored to the full symmetric matrix;
// the leading kk x kk block (kk > 0) is the diagonal matrix scale * lam.
__global__ void k_gram_reduce(const double* __restrict__ work, int K, int nsplit, int kk,
                              const double* __restrict__ lam, double scale,
                              double* __restrict__ G) {
    const size_t total = (size_t)K * K;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(e / K), d = (int)(e % K);
        if (c < kk && d < kk) {
            G[e] = c == d ? scale * lam[c] : 0.0;
            continue;
        }
        if (c / GT < d / GT) continue;                  // upper tiles: mirrored below
        double s = 0.0;
        for (int sp = 0; sp < nsplit; ++sp) s += work[(size_t)sp * total + e];
        G[e] = s;
        if (c / GT != d / GT) G[(size_t)d * K + c] = s;
    }
}

// M must be 16-byte aligned with ldM a multiple of 4 (true of every factor buffer: device
// allocations with leading dimensions rounded up to 4), and K <= ldM.  With lam, the first
// orth columns of M are mutually orthogonal with squared norms scale * lam[c] (the columns
// of a truncated factor, M V_r, scaled by the predictions since): the Gram tiles inside
// that block are not computed but taken as that diagonal.
void launch_gram64(const float* M, int n, int ldM, int K, double* G, double* work,
                   size_t work_elems, hipStream_t st, int orth, const double* lam,
                   double scale) {
    const int nt = (K + GT - 1) / GT;
    const int ot = lam ? std::min(std::min(orth, K) / GT, nt) : 0;
    const int tile_off = ot * (ot + 1) / 2;
    const int tiles = nt * (nt + 1) / 2 - tile_off;
    int nsplit = 1;
    if (tiles > 0) {
        nsplit = std::max(1, (2048 + tiles - 1) / tiles);
        nsplit = std::min(nsplit, std::max(1, n / 256));
        while (nsplit > 1 && (size_t)nsplit * K * K > work_elems) --nsplit;
        hipLaunchKernelGGL(k_gram_partial, dim3(tiles * nsplit), dim3(256), 0, st, M, n, ldM,
                           K, nsplit, tile_off, work);
    }
    const size_t total = (size_t)K * K;
    const int blocks = (int)std::min<size_t>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(k_gram_reduce, dim3(blocks), dim3(256), 0, st, work, K, nsplit, ot * GT,
                       lam, scale, G);
}

// lam[c] (c < r) = src[K - 1 - c] (ascending src, the library solver's order) or src[c]
__global__ void k_store_lam(const double* __restrict__ src, int K, int r, int ascending,
                            double* __restrict__ lam) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < r) lam[c] = ascending ? src[K - 1 - c] : src[c];
}

void launch_store_lam(const double* src, int K, int r, int ascending, double* lam,
                      hipStream_t st) {
    hipLaunchKernelGGL(k_store_lam, dim3((r + 255) / 256), dim3(256), 0, st, src, K, r,
                       ascending, lam);
}

// The eigensolver returns eigenvalues in ascending order with eigenvectors as columns
// of E (column-major K x K).  V_r keeps the r leading ones in descending order:
// Vr (FP32, row-major K x r) and, optionally, rot_out (FP64, row-major K x r).
__global__ void k_pick_rotation(const double* __restrict__ E, int K, int r,
                                float* __restrict__ Vr, double* __restrict__ rot_out) {
    const size_t total = (size_t)K * r;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(e / K), k = (int)(e % K);
        const double v = E[(size_t)(K - 1 - c) * K + k];
        Vr[(size_t)k * r + c] = (float)v;
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
