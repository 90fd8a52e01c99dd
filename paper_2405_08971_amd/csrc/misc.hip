// Elementwise and row kernels of libcakf: point pre-scaling, predict, mean update,
// marginal variances.
#include "cakf_common.h"
#include "launchers.h"

namespace cakf {

// Euclidean: (c x, c y, c z, c^2 |x|^2); great-circle: (x, y, z, c), with
// c = log2(e) sqrt(2 nu) / ell (see cakf_common.h).
__global__ void k_prescale(const float* __restrict__ X, int n, int dim, float c, int dist,
                           float4* __restrict__ Xs) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const float x = X[(size_t)p * dim + 0];
    const float y = X[(size_t)p * dim + 1];
    const float z = dim == 3 ? X[(size_t)p * dim + 2] : 0.0f;
    if (dist == DIST_EUCLID) {
        const float sx = c * x, sy = c * y, sz = c * z;
        const double w = (double)sx * sx + (double)sy * sy + (double)sz * sz;
        Xs[p] = make_float4(sx, sy, sz, (float)w);
    } else {
        Xs[p] = make_float4(x, y, z, c);
    }
}

void launch_prescale(const float* X, int n, int dim, float c, int dist, float4* Xs,
                     hipStream_t st) {
    hipLaunchKernelGGL(k_prescale, dim3((n + 255) / 256), dim3(256), 0, st, X, n, dim, c, dist,
                       Xs);
}

// Predict of Alg. 1 for A = a I, b = 0: m <- a m, M <- a M (first rank columns).
__global__ void k_scale_state(float* __restrict__ mean, float* __restrict__ M, int n, int ld,
                              int rank, float a) {
    const size_t total = (size_t)n * rank;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
        const size_t p = e / rank, c = e % rank;
        M[p * ld + c] *= a;
    }
    for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < (size_t)n; p += stride)
        mean[p] *= a;
}

void launch_scale_state(float* mean, float* M, int n, int ld, int rank, float a, hipStream_t st) {
    const size_t total = std::max<size_t>((size_t)n * rank, (size_t)n);
    const int blocks = (int)std::min<size_t>((total + 255) / 256, 8192);
    hipLaunchKernelGGL(k_scale_state, dim3(blocks), dim3(256), 0, st, mean, M, n, ld, rank, a);
}

// Predict of the Matérn-3/2 temporal state (value rows 0..n-1, scaled-derivative rows
// n..2n-1): each point's pair of rows (p, n + p) of the mean and of the factor's first
// rank columns is multiplied by the 2x2 transition [[t00, t01], [t10, t11]].
__global__ void k_predict_pairs(float* __restrict__ mean, float* __restrict__ M, int n, int ld,
                                int rank, float t00, float t01, float t10, float t11) {
    const size_t total = (size_t)n * (rank + 1);
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
        const size_t p = e / (rank + 1), c = e % (rank + 1);
        float* v0 = c < (size_t)rank ? M + p * ld + c : mean + p;
        float* v1 = c < (size_t)rank ? M + (p + n) * ld + c : mean + p + n;
        const float a = *v0, b = *v1;
        *v0 = __builtin_fmaf(t00, a, t01 * b);
        *v1 = __builtin_fmaf(t10, a, t11 * b);
    }
}

void launch_predict_pairs(float* mean, float* M, int n, int ld, int rank, const float t[4],
                          hipStream_t st) {
    const size_t total = (size_t)n * (rank + 1);
    const int blocks = (int)std::min<size_t>((total + 255) / 256, 8192);
    hipLaunchKernelGGL(k_predict_pairs, dim3(blocks), dim3(256), 0, st, mean, M, n, ld, rank,
                       t[0], t[1], t[2], t[3]);
}

// M[p, c0 + c] = 0 for p < rows, c < cols (the scaled-derivative rows of new columns).
__global__ void k_zero_cols(float* __restrict__ M, int ld, int rows, int cols) {
    const size_t total = (size_t)rows * cols;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x)
        M[(e / cols) * ld + e % cols] = 0.0f;
}

void launch_zero_cols(float* M, int ld, int rows, int cols, hipStream_t st) {
    const size_t total = (size_t)rows * cols;
    if (total == 0) return;
    hipLaunchKernelGGL(k_zero_cols, dim3((int)std::min<size_t>((total + 255) / 256, 8192)),
                       dim3(256), 0, st, M, ld, rows, cols);
}

// p[e] = 0 for e < count: clears workspace with a kernel rather than a memset node.
__global__ void k_fill_zero(float* __restrict__ p, size_t count) {
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
         e += (size_t)gridDim.x * blockDim.x)
        p[e] = 0.0f;
}

void launch_fill_zero(float* p, size_t count, hipStream_t st) {
    if (count == 0) return;
    hipLaunchKernelGGL(k_fill_zero, dim3((int)std::min<size_t>((count + 255) / 256, 8192)),
                       dim3(256), 0, st, p, count);
}

// m <- m + M[:, col]  (the mean column of the block product).
__global__ void k_mean_add(float* __restrict__ mean, const float* __restrict__ M, int n, int ld,
                           int col) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) mean[p] += M[(size_t)p * ld + col];
}

void launch_mean_add(float* mean, const float* M, int n, int ld, int col, hipStream_t st) {
    hipLaunchKernelGGL(k_mean_add, dim3((n + 255) / 256), dim3(256), 0, st, mean, M, n, ld, col);
}

// diag(Sigma - M M^T) at the requested rows: sigma_f2 - sum_c M[p, c]^2 (one wave per row,
// FP64 accumulation).
__global__ __launch_bounds__(256) void k_marginal_var(const float* __restrict__ M, int n, int ld,
                                                      int rank, float sigma_f2,
                                                      const int32_t* __restrict__ rows,
                                                      int count, float* __restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int e = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (e >= count) return;
    const int p = rows ? rows[e] : e;
    if (p < 0 || p >= n) {
        if (lane == 0) out[e] = __builtin_nanf("");
        return;
    }
    const float* row = M + (size_t)p * ld;
    double s = 0.0;
    for (int c = lane; c < rank; c += 64) {
        const double v = row[c];
        s = __builtin_fma(v, v, s);
    }
    s = wave_sum(s);
    if (lane == 0) out[e] = (float)((double)sigma_f2 - s);
}

void launch_marginal_var(const float* M, int n, int ld, int rank, float sigma_f2,
                         const int32_t* rows, int count, float* out, hipStream_t st) {
    hipLaunchKernelGGL(k_marginal_var, dim3((count + 3) / 4), dim3(256), 0, st, M, n, ld, rank,
                       sigma_f2, rows, count, out);
}

// dst[p, 0:cols] = src[p, 0:cols].
__global__ void k_copy_rows(const float* __restrict__ src, int lds, float* __restrict__ dst,
                            int ldd, int rows, int cols) {
    const size_t total = (size_t)rows * cols;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
        const size_t p = e / cols, c = e % cols;
        dst[p * ldd + c] = src[p * lds + c];
    }
}

void launch_copy_rows(const float* src, int lds, float* dst, int ldd, int rows, int cols,
                      hipStream_t st) {
    const size_t total = (size_t)rows * cols;
    if (total == 0) return;
    const int blocks = (int)std::min<size_t>((total + 255) / 256, 8192);
    hipLaunchKernelGGL(k_copy_rows, dim3(blocks), dim3(256), 0, st, src, lds, dst, ldd, rows, cols);
}

}  // namespace cakf
