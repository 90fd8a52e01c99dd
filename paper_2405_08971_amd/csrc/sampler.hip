// Elementwise and small kernels of the path sampler (App. C, CAKF/CAKS sampler) on gfx950.
// ns paths are the columns of row-major n x ns (state) and m x ns (observation) arrays;
// the kernel-matrix and low-rank products of the sampler go through the block product
// and rocBLAS, driven from cakf_api.hip:
//   forward   x^-   = a x_{k-1} + q                                  (k_sample_predict)
//             d     = y - x^-[idx] - sigma e                         (k_sample_innov)
//             z     = L^{-1} (S^T d)                                 (k_sample_solve)
//             wobs  = W_obs z,  x = x^- + Sigma H^T wobs - M^- (M^-^T H^T wobs)
//   backward  B     = a ws_{k+1}                                     (k_sample_scale_pad)
//             xs    = x + Sigma B - M (M^T B)
//             ws    = B + H^T (wobs - W_obs (W_obs^T (P^- B)[idx]))  (k_sample_messages)
#include "cakf_common.h"
#include "launchers.h"

namespace cakf {

static int grid_for(size_t total) { return (int)std::min<size_t>((total + 255) / 256, 8192); }

// out[p, s] = a x[p, s] + q[p, s]   (n x ns, leading dimension ld)
__global__ void k_sample_predict(const float* __restrict__ x, const float* __restrict__ q,
                                 float a, int n, int ns, int ld, float* __restrict__ out) {
    const size_t total = (size_t)n * ns;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const size_t o = (e / ns) * ld + e % ns;
        out[o] = __builtin_fmaf(a, x[o], q[o]);
    }
}

void launch_sample_predict(const float* x, const float* q, float a, int n, int ns, int ld,
                           float* out, hipStream_t st) {
    hipLaunchKernelGGL(k_sample_predict, dim3(grid_for((size_t)n * ns)), dim3(256), 0, st, x, q,
                       a, n, ns, ld, out);
}

// d[p, s] = y[p] - x[idx[p], s] - sigma e[p, s] for p < m (x: ld ldx, e: ld lde, d: ld ldd).
// An index outside [0, n) reads row 0.
__global__ void k_sample_innov(const float* __restrict__ y, const int32_t* __restrict__ idx,
                               const float* __restrict__ x, int ldx, const float* __restrict__ e,
                               int lde, float sigma, int n, int m, int ns,
                               float* __restrict__ d, int ldd) {
    const size_t total = (size_t)m * ns;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (size_t)gridDim.x * blockDim.x) {
        const int p = (int)(t / ns), s = (int)(t % ns);
        int r = idx[p];
        r = (r < 0 || r >= n) ? 0 : r;
        d[(size_t)p * ldd + s] =
            y[p] - x[(size_t)r * ldx + s] - sigma * e[(size_t)p * lde + s];
    }
}

void launch_sample_innov(const float* y, const int32_t* idx, const float* x, int ldx,
                         const float* e, int lde, float sigma, int n, int m, int ns, float* d,
                         int ldd, hipStream_t st) {
    hipLaunchKernelGGL(k_sample_innov, dim3(grid_for((size_t)m * ns)), dim3(256), 0, st, y, idx,
                       x, ldx, e, lde, sigma, n, m, ns, d, ldd);
}

// z[l, s] = sum_k Linv[l, k] r[k, s]  (Linv: FP64 row-major imax x imax, lower triangular;
// r, z: FP32 imax x ns with leading dimension ld).  One thread per output, FP64 sums.
__global__ void k_sample_solve(const double* __restrict__ Linv, int imax,
                               const float* __restrict__ r, int ns, int ld,
                               float* __restrict__ z) {
    const int total = imax * ns;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < total; t += gridDim.x * blockDim.x) {
        const int l = t / ns, s = t % ns;
        double acc = 0.0;
        for (int k = 0; k <= l; ++k)
            acc = __builtin_fma(Linv[(size_t)l * imax + k], (double)r[(size_t)k * ld + s], acc);
        z[(size_t)l * ld + s] = (float)acc;
    }
}

void launch_sample_solve(const double* Linv, int imax, const float* r, int ns, int ld, float* z,
                         hipStream_t st) {
    hipLaunchKernelGGL(k_sample_solve, dim3(grid_for((size_t)imax * ns)), dim3(256), 0, st, Linv,
                       imax, r, ns, ld, z);
}

// out[p, s] (ld ldo) += Y[p, s] (ld ldy) for p < n, s < ns
__global__ void k_add_cols(const float* __restrict__ Y, int ldy, int n, int ns,
                           float* __restrict__ out, int ldo) {
    const size_t total = (size_t)n * ns;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const size_t p = e / ns, s = e % ns;
        out[p * ldo + s] += Y[p * ldy + s];
    }
}

void launch_add_cols(const float* Y, int ldy, int n, int ns, float* out, int ldo,
                     hipStream_t st) {
    hipLaunchKernelGGL(k_add_cols, dim3(grid_for((size_t)n * ns)), dim3(256), 0, st, Y, ldy, n,
                       ns, out, ldo);
}

// out (rows x ld, the first ns columns) = a * in (n x ns, ld ldi) in rows < n, 0 in the
// padding rows n .. rows-1 and in columns ns .. ld-1.
__global__ void k_sample_scale_pad(const float* __restrict__ in, int ldi, float a, int n,
                                   int rows, int ns, float* __restrict__ out, int ld) {
    const size_t total = (size_t)rows * ld;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const size_t p = e / ld;
        const int s = (int)(e % ld);
        out[e] = (p < (size_t)n && s < ns) ? a * in[p * ldi + s] : 0.0f;
    }
}

void launch_sample_scale_pad(const float* in, int ldi, float a, int n, int rows, int ns,
                             float* out, int ld, hipStream_t st) {
    hipLaunchKernelGGL(k_sample_scale_pad, dim3(grid_for((size_t)rows * ld)), dim3(256), 0, st,
                       in, ldi, a, n, rows, ns, out, ld);
}

// H^T v into a zeroed n-row array: out[idx[p], s] += v[p, s] - (WR ? WR[p, s] : 0) for p < m.
// The indices of a step are distinct, so no two threads add to one entry.
__global__ void k_sample_scatter(const int32_t* __restrict__ idx, int n, int m, int ns,
                                 const float* __restrict__ v, int ldv,
                                 const float* __restrict__ WR, int ldr, float* __restrict__ out,
                                 int ldo) {
    const size_t total = (size_t)m * ns;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (size_t)gridDim.x * blockDim.x) {
        const int p = (int)(t / ns), s = (int)(t % ns);
        const int r = idx[p];
        if (r < 0 || r >= n) continue;
        float val = v[(size_t)p * ldv + s];
        if (WR) val -= WR[(size_t)p * ldr + s];
        out[(size_t)r * ldo + s] += val;
    }
}

void launch_sample_scatter(const int32_t* idx, int n, int m, int ns, const float* v, int ldv,
                           const float* WR, int ldr, float* out, int ldo, hipStream_t st) {
    if ((size_t)m * ns == 0) return;
    hipLaunchKernelGGL(k_sample_scatter, dim3(grid_for((size_t)m * ns)), dim3(256), 0, st, idx, n,
                       m, ns, v, ldv, WR, ldr, out, ldo);
}

// out (rows x ld, the first ns columns) = in (n x ns, ld ldi) in rows < n, zero elsewhere
// (the padding rows and the columns ns .. ld-1).
void launch_sample_copy_pad(const float* in, int ldi, int n, int rows, int ns, float* out,
                            int ld, hipStream_t st) {
    launch_sample_scale_pad(in, ldi, 1.0f, n, rows, ns, out, ld, st);
}

// Xo[q] = Xs[idx[q]] for q < mp (rows m .. mp-1 repeat idx[0]; an index outside [0, n)
// reads point 0)
__global__ void k_gather_points(const float4* __restrict__ Xs, int n,
                                const int32_t* __restrict__ idx, int m, int mp,
                                float4* __restrict__ Xo) {
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < mp; q += gridDim.x * blockDim.x) {
        int p = idx[q < m ? q : 0];
        p = (p < 0 || p >= n) ? 0 : p;
        Xo[q] = Xs[p];
    }
}

void launch_gather_points(const float4* Xs, int n, const int32_t* idx, int m, int mp,
                          float4* Xo, hipStream_t st) {
    hipLaunchKernelGGL(k_gather_points, dim3(grid_for((size_t)mp)), dim3(256), 0, st, Xs, n, idx,
                       m, mp, Xo);
}

}  // namespace cakf
