// Element kernels of the computation-aware RTS smoother (Alg. 3) on gfx950.  The
// kernel-matrix product Sigma A^T [ws Ws] runs in the block-product kernels; the dense
// low-rank products are library GEMMs.
#include "cakf_common.h"
#include "launchers.h"

namespace cakf {

// Bs = a [ws | Ws] (rows >= n and columns >= 1 + rs are zero), row-major np x ldb.
__global__ void k_smooth_pack(const float* __restrict__ ws, const float* __restrict__ Ws,
                              int ldw, int n, int np, int rs, float a, float* __restrict__ Bs,
                              int ldb) {
    const size_t total = (size_t)np * ldb;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int p = (int)(e / ldb), c = (int)(e % ldb);
        float v = 0.0f;
        if (p < n) {
            if (c == 0) v = a * ws[p];
            else if (c <= rs) v = a * Ws[(size_t)p * ldw + c - 1];
        }
        Bs[e] = v;
    }
}

void launch_smooth_pack(const float* ws, const float* Ws, int ldw, int n, int np, int rs,
                        float a, float* Bs, int ldb, hipStream_t st) {
    const size_t total = (size_t)np * ldb;
    hipLaunchKernelGGL(k_smooth_pack, dim3((int)std::min<size_t>((total + 255) / 256, 8192)),
                       dim3(256), 0, st, ws, Ws, ldw, n, np, rs, a, Bs, ldb);
}

// Smoothed moments of step k from Z = P_k A^T [ws Ws] (n x b, ld ldz), with the filter
// moments scaled by g (1 at a step; A(t, t_k) at an interpolated time t):
//   mean_out = g m_k + Z[:, 0];  factor_out = [g M_k | Z[:, 1:b]];
//   var_out = sigma_f2 - |g M_k[p, :]|^2 - |Z[p, 1:b]|^2   (FP64 accumulation).
// Z == nullptr: the filter moments alone (b ignored).
__global__ __launch_bounds__(256) void k_smooth_out(const float* __restrict__ mean,
                                                    const float* __restrict__ M, int ldm,
                                                    int rank, float g,
                                                    const float* __restrict__ Z,
                                                    int ldz, int b, int n, float sigma_f2,
                                                    float* __restrict__ mean_out,
                                                    float* __restrict__ factor_out, int ldo,
                                                    float* __restrict__ var_out) {
    const int lane = threadIdx.x & 63;
    const int p = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (p >= n) return;
    const float* Mr = M + (size_t)p * ldm;
    const float* Zr = Z ? Z + (size_t)p * ldz : nullptr;
    double s = 0.0;
    for (int c = lane; c < rank; c += 64) {
        const float v = g * Mr[c];
        s = __builtin_fma((double)v, (double)v, s);
        if (factor_out) factor_out[(size_t)p * ldo + c] = v;
    }
    if (Zr) {
        for (int c = 1 + lane; c < b; c += 64) {
            const float v = Zr[c];
            s = __builtin_fma((double)v, (double)v, s);
            if (factor_out) factor_out[(size_t)p * ldo + rank + c - 1] = v;
        }
    }
    s = wave_sum(s);
    if (lane == 0) {
        if (mean_out) mean_out[p] = g * mean[p] + (Zr ? Zr[0] : 0.0f);
        if (var_out) var_out[p] = (float)((double)sigma_f2 - s);
    }
}

void launch_smooth_out(const float* mean, const float* M, int ldm, int rank, float g,
                       const float* Z, int ldz, int b, int n, float sigma_f2, float* mean_out,
                       float* factor_out, int ldo, float* var_out, hipStream_t st) {
    hipLaunchKernelGGL(k_smooth_out, dim3((n + 3) / 4), dim3(256), 0, st, mean, M, ldm, rank, g,
                       Z, ldz, b, n, sigma_f2, mean_out, factor_out, ldo, var_out);
}

// Gather rows of a row-major matrix: out[q, 0:cols] = A[idx[q], 0:cols].
__global__ void k_gather_rows(const float* __restrict__ A, int lda, const int32_t* __restrict__ idx,
                              int m, int n, int cols, float* __restrict__ out, int ldo) {
    const size_t total = (size_t)m * cols;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int q = (int)(e / cols), c = (int)(e % cols);
        int p = idx[q];
        p = (p < 0 || p >= n) ? 0 : p;
        out[(size_t)q * ldo + c] = A[(size_t)p * lda + c];
    }
}

void launch_gather_rows(const float* A, int lda, const int32_t* idx, int m, int n, int cols,
                        float* out, int ldo, hipStream_t st) {
    const size_t total = (size_t)m * cols;
    if (total == 0) return;
    hipLaunchKernelGGL(k_gather_rows, dim3((int)std::min<size_t>((total + 255) / 256, 8192)),
                       dim3(256), 0, st, A, lda, idx, m, n, cols, out, ldo);
}

// Next smoother messages before truncation (distinct indices idx):
//   ws[p]           = Bs[p, 0]                      (then + w_obs[q] - WR[q, 0] at p = idx[q])
//   Wc[p, 0:i]      = 0                              (then W_obs[q, :] at p = idx[q])
//   Wc[p, i:i+rs]   = Bs[p, 1:1+rs]                 (then - WR[q, 1:1+rs] at p = idx[q])
__global__ void k_smooth_dense(const float* __restrict__ Bs, int ldb, int n, int i, int rs,
                               float* __restrict__ ws, float* __restrict__ Wc, int ldw) {
    const size_t total = (size_t)n * (i + rs + 1);
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int p = (int)(e / (i + rs + 1)), c = (int)(e % (i + rs + 1));
        if (c == i + rs) ws[p] = Bs[(size_t)p * ldb];
        else Wc[(size_t)p * ldw + c] = c < i ? 0.0f : Bs[(size_t)p * ldb + 1 + c - i];
    }
}

__global__ void k_smooth_scatter(const int32_t* __restrict__ idx, int m, int n, int i, int rs,
                                 const float* __restrict__ w_obs,
                                 const float* __restrict__ W_obs, int imax,
                                 const float* __restrict__ WR, int ldr,
                                 float* __restrict__ ws, float* __restrict__ Wc, int ldw) {
    const size_t total = (size_t)m * (i + rs + 1);
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int q = (int)(e / (i + rs + 1)), c = (int)(e % (i + rs + 1));
        const int p = idx[q];
        if (p < 0 || p >= n) continue;
        if (c == i + rs) {
            ws[p] += w_obs[q] - (WR ? WR[(size_t)q * ldr] : 0.0f);
        } else if (c < i) {
            Wc[(size_t)p * ldw + c] = W_obs[(size_t)q * imax + c];
        } else if (WR) {
            Wc[(size_t)p * ldw + c] -= WR[(size_t)q * ldr + 1 + c - i];
        }
    }
}

void launch_smooth_messages(const float* Bs, int ldb, int n, const int32_t* idx, int m, int i,
                            int rs, const float* w_obs, const float* W_obs, int imax,
                            const float* WR, int ldr, float* ws, float* Wc, int ldw,
                            hipStream_t st) {
    const size_t total = (size_t)n * (i + rs + 1);
    hipLaunchKernelGGL(k_smooth_dense, dim3((int)std::min<size_t>((total + 255) / 256, 8192)),
                       dim3(256), 0, st, Bs, ldb, n, i, rs, ws, Wc, ldw);
    if (m > 0) {
        const size_t t2 = (size_t)m * (i + rs + 1);
        hipLaunchKernelGGL(k_smooth_scatter, dim3((int)std::min<size_t>((t2 + 255) / 256, 8192)),
                           dim3(256), 0, st, idx, m, n, i, rs, w_obs, W_obs, imax, WR, ldr, ws,
                           Wc, ldw);
    }
}

// Pad the pre-scaled points to np entries (copies of the last point; the matching rows
// of the block operand are zero).
__global__ void k_pad_points(const float4* __restrict__ Xs, int n, int np, float4* __restrict__ Xp) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < np) Xp[p] = Xs[p < n ? p : n - 1];
}

void launch_pad_points(const float4* Xs, int n, int np, float4* Xp, hipStream_t st) {
    hipLaunchKernelGGL(k_pad_points, dim3((np + 255) / 256), dim3(256), 0, st, Xs, n, np, Xp);
}

}  // namespace cakf
