// Reverse-mode derivative of the projected log-likelihood on gfx950.
//
// The likelihood is the sum over updates of
//     l_k = -1/2 [ i log 2 pi + 2 sum_j log L_jj - log det S^T S + alpha^T alpha ],
// C = S^T Ghat S = L L^T, alpha = L^{-1} S^T r0, with the actions S_k and the truncation
// rotations V_r,k held fixed (the paper leaves evidence maximisation to future work,
// Sec. 8; this is the derivative of the filter as run).  The backward sweep visits the
// steps in reverse and carries the adjoints of the filter mean and of the truncated
// factor.  Per step (Alg. 1 and Alg. 2 read backwards), with Ybar the adjoint of the
// new factor columns and of the mean increment, B = [W w] = [S L^{-T}, S L^{-T} alpha]:
//   Y = sigma_f2 K(X, Xo) B - M^- Mo^T B   gives   Bbar = sigma_f2 K(Xo, X) Ybar + Mo Qbar,
//       Qbar = -M^-T Ybar,  Mbar^- -= Ybar (Mo^T B)^T,  Mobar = B Qbar^T, and the
//       parameter terms sum K o (Ybar B^T) (signal variance), sum dK/dell o (Ybar B^T);
//   the Cholesky form (App. B) gives Cbar, cbar = L^{-T} alphabar in FP64;
//   C = S^T Ghat S gives the parameter terms sum K o (S Cbar S^T), sum dK/dell o
//       (S Cbar S^T), <Cbar, S^T S> (noise), and Mobar -= 2 S Cbar (Mo^T S)^T;
//   r0 = y - m^-[idx], Mo = M^-[idx] scatter back; m^- = a m, M^- = a M^+ give the
//       derivative in a and the adjoints of the previous step.
// The kernel-matrix terms are evaluated tile by tile and never stored
// (k_adj_tiles): each 32 x 32 tile of kernel values and their lengthscale derivatives is
// computed on the VALU in the register layout of an FP32 MFMA result, the rank-b
// products Ybar B^T are formed on the MFMA units in that same layout, and (for the
// state x observation sweep) the transposed product K^T Ybar reuses the kernel values
// as the A operand of further MFMAs.
#include "cakf_common.h"
#include "launchers.h"

namespace cakf {

typedef float f32x16 __attribute__((ext_vector_type(16)));

// Matern correlation k(u) and -u dk/du, as functions of u' = log2(e) u (unit variance);
// dk/dell = (-u dk/du) / ell since u is proportional to 1 / ell.
//   nu = 1/2: k = e^-u,                     -u k' = u e^-u
//   nu = 3/2: k = (1 + u) e^-u,             -u k' = u^2 e^-u
//   nu = 5/2: k = (1 + u + u^2 / 3) e^-u,   -u k' = (u^2 / 3)(1 + u) e^-u
template <int NU2>
__device__ __forceinline__ void matern_and_dlog(float up, float& k, float& kd) {
    const float e = __builtin_amdgcn_exp2f(-up);
    const float u = up * LN2;
    if constexpr (NU2 == 1) {
        k = e;
        kd = u * e;
    } else if constexpr (NU2 == 3) {
        k = __builtin_fmaf(u, e, e);
        kd = (u * u) * e;
    } else {
        k = __builtin_fmaf(u, __builtin_fmaf(u, 1.0f / 3.0f, 1.0f), 1.0f) * e;
        kd = (u * u * (1.0f / 3.0f)) * __builtin_fmaf(u, e, e);
    }
}

template <int NU2, int DIST>
__device__ __forceinline__ float pair_dist(const float4 ap, const float4 b) {
    if constexpr (DIST == DIST_EUCLID) return scaled_dist_diff(ap, b);
    else return scaled_dist<DIST>(ap, b);
}

// ------------------------------------------------------------------------ k_adj_tiles
// For a block of 32 q-points (Xq, rows of Bq) and one slice of p-points (Xp, rows of Yp):
//   sK  = sum_{p,q} k(x_p, x_q) (Yp Bq^T)_pq,   sKd = sum (-u dk/du)(x_p, x_q) (Yp Bq^T)_pq
// (per-block FP64 partials in spart[2 * block + {0, 1}]) and, with BBAR, the partial
// products sum_p k(x_p, x_q) Yp[p, c] for this slice into bpart.  b columns are used
// (zero padded to W = 32 CT in LDS); bk = b rounded up to even is the MFMA depth of
// Yp Bq^T.  Four waves take 32 rows each of a staged chunk of AT_CHUNK rows.
constexpr int AT_CHUNK = 128;
constexpr int AT_MAXCOL = 160;   // columns per launch (LDS: 128 + 32 staged rows of them)

template <int NU2, int DIST, bool BBAR, int CT>
__global__ __launch_bounds__(256) void k_adj_tiles(const float4* __restrict__ Xp, int np_,
                                                   const float* __restrict__ Yp, int ldy,
                                                   const float4* __restrict__ Xq, int mq,
                                                   const float* __restrict__ Bq, int ldb,
                                                   int b, int bk, int rows_per_slice,
                                                   float* __restrict__ bpart, int ldbp,
                                                   size_t slice_stride,
                                                   double* __restrict__ spart) {
    constexpr int W = 32 * CT;
    __shared__ float Yl[AT_CHUNK][W + 1];
    __shared__ float Bl[32][W + 1];
    __shared__ float4 Xl[AT_CHUNK];
    __shared__ double sred[2][4];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int l32 = lane & 31, hi = lane >> 5;
    const int q0 = blockIdx.x * 32;
    const int pbeg = blockIdx.y * rows_per_slice;
    const int pend = min(np_, pbeg + rows_per_slice);
    for (int e = tid; e < 32 * W; e += 256) {
        const int r = e / W, c = e % W;
        const int q = q0 + r;
        Bl[r][c] = (q < mq && c < b) ? Bq[(size_t)q * ldb + c] : 0.0f;
    }
    const bool qvalid = q0 + l32 < mq;
    const float4 xq = Xq[min(q0 + l32, mq - 1)];
    f32x16 acc[BBAR ? CT : 1];
#pragma unroll
    for (int t = 0; t < (BBAR ? CT : 1); ++t)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[t][i] = 0.0f;
    double aK = 0.0, aKd = 0.0;
    for (int c0 = pbeg; c0 < pend; c0 += AT_CHUNK) {
        __syncthreads();
        if (tid < AT_CHUNK) Xl[tid] = Xp[min(c0 + tid, np_ - 1)];
        for (int e = tid; e < AT_CHUNK * W; e += 256) {
            const int r = e / W, c = e % W;
            const int p = c0 + r;
            Yl[r][c] = (p < pend && c < b) ? Yp[(size_t)p * ldy + c] : 0.0f;
        }
        __syncthreads();
        const int pb = 32 * w;
        if (c0 + pb >= pend) continue;
        float kv[16], kd[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int r = pb + 8 * (i / 4) + 4 * hi + (i % 4);
            float k, d;
            matern_and_dlog<NU2>(pair_dist<NU2, DIST>(prep_row<DIST>(Xl[r]), xq), k, d);
            const bool ok = qvalid && c0 + r < pend;
            kv[i] = ok ? k : 0.0f;
            kd[i] = ok ? d : 0.0f;
        }
        f32x16 d1;
#pragma unroll
        for (int i = 0; i < 16; ++i) d1[i] = 0.0f;
        for (int cc = 0; cc < bk; cc += 2)
            d1 = __builtin_amdgcn_mfma_f32_32x32x2f32(Yl[pb + l32][cc + hi], Bl[l32][cc + hi], d1,
                                                      0, 0, 0);
        float s1 = 0.0f, s2 = 0.0f;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            s1 = __builtin_fmaf(kv[i], d1[i], s1);
            s2 = __builtin_fmaf(kd[i], d1[i], s2);
        }
        aK += (double)s1;
        aKd += (double)s2;
        if constexpr (BBAR) {
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int r = pb + 8 * (i / 4) + (i % 4) + 4 * hi;
#pragma unroll
                for (int t = 0; t < CT; ++t)
                    acc[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(kv[i], Yl[r][32 * t + l32],
                                                                  acc[t], 0, 0, 0);
            }
        }
    }
    aK = wave_sum(aK);
    aKd = wave_sum(aKd);
    if (lane == 0) {
        sred[0][w] = aK;
        sred[1][w] = aKd;
    }
    __syncthreads();
    if constexpr (BBAR) {
        // cross-wave sum of the K^T Yp partials through LDS (reusing the Y staging area)
        float* red = &Yl[0][0];
#pragma unroll
        for (int t = 0; t < CT; ++t)
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int q = 8 * (j / 4) + 4 * hi + (j % 4);
                red[(w * 32 + q) * W + 32 * t + l32] = acc[t][j];
            }
        __syncthreads();
        float* out = bpart + (size_t)blockIdx.y * slice_stride;
        for (int e = tid; e < 32 * W; e += 256) {
            const int r = e / W, c = e % W;
            const float s = (red[r * W + c] + red[(32 + r) * W + c]) +
                            (red[(64 + r) * W + c] + red[(96 + r) * W + c]);
            if (q0 + r < mq && c < b) out[(size_t)(q0 + r) * ldbp + c] = s;
        }
    }
    if (tid == 0) {
        const size_t blk = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
        spart[2 * blk] = (sred[0][0] + sred[0][1]) + (sred[0][2] + sred[0][3]);
        spart[2 * blk + 1] = (sred[1][0] + sred[1][1]) + (sred[1][2] + sred[1][3]);
    }
}

int adj_tiles_slices(int np_, int mq) {
    const int qblk = (mq + 31) / 32;
    int ns = (2048 + qblk - 1) / qblk;
    const int maxs = (np_ + AT_CHUNK - 1) / AT_CHUNK;
    ns = std::max(1, std::min(ns, maxs));
    return ns;
}

template <int NU2, int DIST, bool BBAR>
static int launch_adj_ct(int ct, dim3 grid, const float4* Xp, int np_, const float* Yp,
                         int ldy, const float4* Xq, int mq, const float* Bq, int ldb, int b,
                         int bk, int rps, float* bpart, int ldbp, size_t sstride,
                         double* spart, hipStream_t st) {
#define CAKF_ADJ_CT(N)                                                                      \
    case N:                                                                                 \
        hipLaunchKernelGGL((k_adj_tiles<NU2, DIST, BBAR, N>), grid, dim3(256), 0, st, Xp,   \
                           np_, Yp, ldy, Xq, mq, Bq, ldb, b, bk, rps, bpart, ldbp, sstride, \
                           spart);                                                          \
        return 0;
    switch (ct) {
        CAKF_ADJ_CT(1)
        CAKF_ADJ_CT(2)
        CAKF_ADJ_CT(3)
        CAKF_ADJ_CT(4)
        CAKF_ADJ_CT(5)
        default:
            return -1;
    }
#undef CAKF_ADJ_CT
}

void adj_tiles_geometry(int np_, int mq, int* gx, int* gy, int* rps) {
    const int ns = adj_tiles_slices(np_, mq);
    *rps = ((np_ + ns - 1) / ns + AT_CHUNK - 1) / AT_CHUNK * AT_CHUNK;
    *gx = (mq + 31) / 32;
    *gy = (np_ + *rps - 1) / *rps;
}

// One launch over at most AT_MAXCOL columns.
static int launch_adj_block(int nu2, int dist, bool bbar, const float4* Xp, int np_,
                            const float* Yp, int ldy, const float4* Xq, int mq, const float* Bq,
                            int ldb, int b, float* bpart, int ldbp, size_t slice_stride,
                            double* spart, int* nblocks, hipStream_t st) {
    const int ct = (b + 31) / 32;
    if (ct < 1 || ct > 5 || mq < 1 || np_ < 1) return -1;
    const int bk = (b + 1) & ~1;
    int gx = 0, gy = 0, rps = 0;
    adj_tiles_geometry(np_, mq, &gx, &gy, &rps);
    const dim3 grid(gx, gy);
    *nblocks = grid.x * grid.y;
    int rc = -1;
#define CAKF_ADJ_LAUNCH(NU, DI)                                                               \
    rc = bbar ? launch_adj_ct<NU, DI, true>(ct, grid, Xp, np_, Yp, ldy, Xq, mq, Bq, ldb, b, bk, \
                                            rps, bpart, ldbp, slice_stride, spart, st)        \
              : launch_adj_ct<NU, DI, false>(ct, grid, Xp, np_, Yp, ldy, Xq, mq, Bq, ldb, b,  \
                                             bk, rps, bpart, ldbp, slice_stride, spart, st)
    if (dist == DIST_EUCLID) {
        if (nu2 == 1) CAKF_ADJ_LAUNCH(1, 0);
        else if (nu2 == 3) CAKF_ADJ_LAUNCH(3, 0);
        else CAKF_ADJ_LAUNCH(5, 0);
    } else {
        if (nu2 == 1) CAKF_ADJ_LAUNCH(1, 1);
        else if (nu2 == 3) CAKF_ADJ_LAUNCH(3, 1);
        else CAKF_ADJ_LAUNCH(5, 1);
    }
#undef CAKF_ADJ_LAUNCH
    return rc ? rc : (int)grid.y;
}

// Both sums are linear in the columns: more than AT_MAXCOL columns are taken in blocks of
// AT_MAXCOL, each launch writing its own columns of bpart and its own run of per-block
// partials after the previous launch's (spart then holds *nblocks partials in all).
int launch_adj_tiles(int nu2, int dist, bool bbar, const float4* Xp, int np_, const float* Yp,
                     int ldy, const float4* Xq, int mq, const float* Bq, int ldb, int b,
                     float* bpart, int ldbp, size_t slice_stride, double* spart,
                     int* nblocks, hipStream_t st) {
    if (b < 1) return -1;
    int total = 0, ns = -1;
    for (int c0 = 0; c0 < b; c0 += AT_MAXCOL) {
        int nb = 0;
        ns = launch_adj_block(nu2, dist, bbar, Xp, np_, Yp + c0, ldy, Xq, mq, Bq + c0, ldb,
                              std::min(AT_MAXCOL, b - c0), bbar ? bpart + c0 : bpart, ldbp,
                              slice_stride, spart + 2 * (size_t)total, &nb, st);
        if (ns < 0) return ns;
        total += nb;
    }
    *nblocks = total;
    return ns;
}

// Bbar[q, c] = scale * sum over the slices of bpart (fixed order), c < b; zero for rows
// >= m up to mp and columns b..ldo.
__global__ void k_adj_bbar_reduce(const float* __restrict__ bpart, size_t slice_stride,
                                  int ldbp, int ns, int m, int mp, int b, float scale,
                                  float* __restrict__ out, int ldo) {
    const size_t total = (size_t)mp * ldo;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int q = (int)(e / ldo), c = (int)(e % ldo);
        float v = 0.0f;
        if (q < m && c < b) {
            double s = 0.0;
            for (int k = 0; k < ns; ++k) s += bpart[(size_t)k * slice_stride + (size_t)q * ldbp + c];
            v = (float)(scale * s);
        }
        out[e] = v;
    }
}

void launch_adj_bbar_reduce(const float* bpart, size_t slice_stride, int ldbp, int ns, int m,
                            int mp, int b, float scale, float* out, int ldo, hipStream_t st) {
    const size_t total = (size_t)mp * ldo;
    const int blocks = (int)std::min<size_t>((total + 255) / 256, 8192);
    hipLaunchKernelGGL(k_adj_bbar_reduce, dim3(blocks), dim3(256), 0, st, bpart, slice_stride,
                       ldbp, ns, m, mp, b, scale, out, ldo);
}

// grad[ik] += ck * sum sK, grad[id] += cd * sum sKd over the blocks (one block, fixed
// order: each thread a strided subset, then a fixed tree over the threads).
__global__ __launch_bounds__(256) void k_adj_scalars(const double* __restrict__ spart,
                                                     int nblk, double ck, double cd,
                                                     double* __restrict__ grad, int ik,
                                                     int id) {
    __shared__ double r0[256], r1[256];
    double a = 0.0, d = 0.0;
    for (int k = threadIdx.x; k < nblk; k += 256) {
        a += spart[2 * k];
        d += spart[2 * k + 1];
    }
    r0[threadIdx.x] = a;
    r1[threadIdx.x] = d;
    __syncthreads();
    for (int s = 128; s >= 1; s >>= 1) {
        if ((int)threadIdx.x < s) {
            r0[threadIdx.x] += r0[threadIdx.x + s];
            r1[threadIdx.x] += r1[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        grad[ik] += ck * r0[0];
        grad[id] += cd * r1[0];
    }
}

void launch_adj_scalars(const double* spart, int nblk, double ck, double cd, double* grad,
                        int ik, int id, hipStream_t st) {
    hipLaunchKernelGGL(k_adj_scalars, dim3(1), dim3(256), 0, st, spart, nblk, ck, cd, grad, ik,
                       id);
}

// ------------------------------------------------------------------ packing kernels
// Ybar (n x bp): columns 0..imax-1 from the factor adjoint's new columns
// Mb[:, rank .. rank + imax), column imax from the mean adjoint, zero beyond.
__global__ void k_adj_pack_ybar(const float* __restrict__ Mb, int ldM, int rank, int imax,
                                const float* __restrict__ mb, int n, float* __restrict__ Yb,
                                int bp) {
    const size_t total = (size_t)n * bp;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int p = (int)(e / bp), c = (int)(e % bp);
        float v = 0.0f;
        if (c < imax) v = Mb[(size_t)p * ldM + rank + c];
        else if (c == imax) v = mb[p];
        Yb[e] = v;
    }
}

void launch_adj_pack_ybar(const float* Mb, int ldM, int rank, int imax, const float* mb, int n,
                          float* Yb, int bp, hipStream_t st) {
    const size_t total = (size_t)n * bp;
    const int blocks = (int)std::min<size_t>((total + 255) / 256, 8192);
    hipLaunchKernelGGL(k_adj_pack_ybar, dim3(blocks), dim3(256), 0, st, Mb, ldM, rank, imax, mb,
                       n, Yb, bp);
}

// One wave per observation row q < mp: Xo, Mo = a M^+_{k-1}[idx] (rank columns, ld ldmo),
// B = [W_obs w_obs] (FP32, bp columns, zero padded), W64 = W_obs (FP64),
// Sr64 = [S r0] (FP64, imax + 1 columns), r0 = y - a m_{k-1}[idx].  Rows >= m are zero.
__global__ __launch_bounds__(256) void k_adj_obs_prep(
    const float4* __restrict__ Xs, int n, const int32_t* __restrict__ idx,
    const float* __restrict__ y, int m, int mp, float a, const float* __restrict__ mprev, const float* __restrict__ Mprev,
    int ldprev, int rank, const float* __restrict__ W_obs, const float* __restrict__ w_obs,
    const float* __restrict__ S, int imax, int bp, int ldmo, float4* __restrict__ Xo,
    float* __restrict__ Mo, float* __restrict__ Bq, double* __restrict__ W64,
    double* __restrict__ Sr64) {
    const int lane = threadIdx.x & 63;
    const int q = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (q >= mp) return;
    const bool real = q < m;
    int p = real ? idx[q] : 0;
    if (p < 0 || p >= n) p = 0;     // as the forward gather reads an invalid index
    if (lane == 0) Xo[q] = Xs[p];
    for (int c = lane; c < ldmo; c += 64)
        Mo[(size_t)q * ldmo + c] = (real && c < rank) ? a * Mprev[(size_t)p * ldprev + c] : 0.0f;
    for (int c = lane; c < bp; c += 64) {
        float v = 0.0f;
        if (real) {
            if (c < imax) v = W_obs[(size_t)q * imax + c];
            else if (c == imax) v = w_obs[q];
        }
        Bq[(size_t)q * bp + c] = v;
    }
    if (!real) return;
    for (int c = lane; c <= imax; c += 64) {
        if (c < imax) {
            W64[(size_t)q * imax + c] = (double)W_obs[(size_t)q * imax + c];
            Sr64[(size_t)q * (imax + 1) + c] = (double)S[(size_t)q * imax + c];
        } else {
            const double mp_ = mprev ? (double)a * (double)mprev[p] : 0.0;
            Sr64[(size_t)q * (imax + 1) + imax] = (double)y[q] - mp_;
        }
    }
}

void launch_adj_obs_prep(const float4* Xs, int n, const int32_t* idx, const float* y, int m,
                         int mp, float a, const float* mprev, const float* Mprev, int ldprev, int rank,
                         const float* W_obs, const float* w_obs, const float* S, int imax,
                         int bp, int ldmo, float4* Xo, float* Mo, float* Bq, double* W64,
                         double* Sr64, hipStream_t st) {
    hipLaunchKernelGGL(k_adj_obs_prep, dim3((mp + 3) / 4), dim3(256), 0, st, Xs, n, idx, y, m,
                       mp, a, mprev, Mprev, ldprev, rank, W_obs, w_obs, S, imax, bp, ldmo, Xo, Mo,
                       Bq, W64, Sr64);
}

// FP64 copy of the first cols columns of an FP32 matrix (rows x cols, row-major).
__global__ void k_to_f64(const float* __restrict__ A, int lda, int rows, int cols,
                         double* __restrict__ out, int ldo) {
    const size_t total = (size_t)rows * cols;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int r = (int)(e / cols), c = (int)(e % cols);
        out[(size_t)r * ldo + c] = (double)A[(size_t)r * lda + c];
    }
}

void launch_to_f64(const float* A, int lda, int rows, int cols, double* out, int ldo,
                   hipStream_t st) {
    const size_t total = (size_t)rows * cols;
    if (!total) return;
    const int blocks = (int)std::min<size_t>((total + 255) / 256, 8192);
    hipLaunchKernelGGL(k_to_f64, dim3(blocks), dim3(256), 0, st, A, lda, rows, cols, out, ldo);
}

// FP32 copy of an FP64 matrix (rows x cols, row-major, packed).
__global__ void k_to_f32(const double* __restrict__ A, size_t total, float* __restrict__ out) {
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x)
        out[e] = (float)A[e];
}

void launch_to_f32(const double* A, size_t total, float* out, hipStream_t st) {
    if (!total) return;
    const int blocks = (int)std::min<size_t>((total + 255) / 256, 8192);
    hipLaunchKernelGGL(k_to_f32, dim3(blocks), dim3(256), 0, st, A, total, out);
}

// out[c * rows + r] = A[r * cols + c]: an FP64 row-major rows x cols matrix as its FP32
// transpose (row-major cols x rows).
__global__ void k_to_f32_t(const double* __restrict__ A, int rows, int cols,
                           float* __restrict__ out) {
    const size_t total = (size_t)rows * cols;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(e / rows), r = (int)(e % rows);
        out[e] = (float)A[(size_t)r * cols + c];
    }
}

void launch_to_f32_t(const double* A, int rows, int cols, float* out, hipStream_t st) {
    const size_t total = (size_t)rows * cols;
    if (!total) return;
    const int blocks = (int)std::min<size_t>((total + 255) / 256, 8192);
    hipLaunchKernelGGL(k_to_f32_t, dim3(blocks), dim3(256), 0, st, A, rows, cols, out);
}

// ------------------------------------------------------------------------ k_adj_small
// One block, FP64: the Cholesky-form adjoint of one update with J kept actions.
// G1 = W^T [Bbar_W wbar] and G2 = S^T [S r0] (imax x (imax + 1), row-major).
//   alpha = L^{-1} S^T r0,  alphabar = W^T wbar - alpha,  cbar = L^{-T} alphabar,
//   Lbar  = -tril(L^{-T} Wbar^T W) - tril(cbar alpha^T) - diag(1 / L_jj),
//           Wbar^T W = (W^T Bbar_W)^T + alpha (W^T wbar)^T,
//   Cbar  = sym(L^{-T} Phi(L^T Lbar) L^{-1}),  Phi = lower triangle, diagonal halved
//           (the adjoint of C = L L^T),
//   grad[noise] += <Cbar, S^T S>.
// Out: Cc = [Cbar cbar] in FP32 (imax x (imax + 1), zero beyond J).  X1, X2: imax x imax
// FP64 scratch.
constexpr int AS_THREADS = 1024;

__global__ __launch_bounds__(AS_THREADS) void k_adj_small(
    int J, int imax, const double* __restrict__ G1, const double* __restrict__ G2,
    const double* __restrict__ L, const double* __restrict__ Linv, double* __restrict__ X1,
    double* __restrict__ X2, float* __restrict__ Cc, double* __restrict__ grad, int inoise) {
    __shared__ double al[256], ab[256], cb[256];
    __shared__ double red[AS_THREADS / 64];
    const int tid = threadIdx.x;
    const int ld = imax, lg = imax + 1;
    // alpha = L^{-1} (S^T r0)
    if (tid < J) {
        double s = 0.0;
        for (int b = 0; b <= tid; ++b) s = __builtin_fma(Linv[(size_t)tid * ld + b], G2[(size_t)b * lg + imax], s);
        al[tid] = s;
    }
    __syncthreads();
    if (tid < J) ab[tid] = G1[(size_t)tid * lg + imax] - al[tid];
    __syncthreads();
    // cbar = L^{-T} alphabar
    if (tid < J) {
        double s = 0.0;
        for (int b = tid; b < J; ++b) s = __builtin_fma(Linv[(size_t)b * ld + tid], ab[b], s);
        cb[tid] = s;
    }
    // X1 = Wbar^T W
    for (int e = tid; e < J * J; e += AS_THREADS) {
        const int a = e / J, b = e % J;
        X1[(size_t)a * ld + b] = G1[(size_t)b * lg + a] + al[a] * G1[(size_t)b * lg + imax];
    }
    __syncthreads();
    // X2 = Lbar (lower triangle)
    for (int e = tid; e < J * J; e += AS_THREADS) {
        const int a = e / J, b = e % J;
        double v = 0.0;
        if (a >= b) {
            double s = 0.0;
#pragma unroll 4
            for (int c = a; c < J; ++c) s = __builtin_fma(Linv[(size_t)c * ld + a], X1[(size_t)c * ld + b], s);
            v = -s - cb[a] * al[b];
            if (a == b) v -= 1.0 / L[(size_t)a * ld + a];
        }
        X2[(size_t)a * ld + b] = v;
    }
    __syncthreads();
    // X1 = Phi(L^T Lbar)
    for (int e = tid; e < J * J; e += AS_THREADS) {
        const int a = e / J, b = e % J;
        double v = 0.0;
        if (a >= b) {
            double s = 0.0;
#pragma unroll 4
            for (int c = a; c < J; ++c) s = __builtin_fma(L[(size_t)c * ld + a], X2[(size_t)c * ld + b], s);
            v = a == b ? 0.5 * s : s;
        }
        X1[(size_t)a * ld + b] = v;
    }
    __syncthreads();
    // X2 = Phi(.) L^{-1}
    for (int e = tid; e < J * J; e += AS_THREADS) {
        const int a = e / J, b = e % J;
        double s = 0.0;
#pragma unroll 4
        for (int c = b; c <= a; ++c) s = __builtin_fma(X1[(size_t)a * ld + c], Linv[(size_t)c * ld + b], s);
        X2[(size_t)a * ld + b] = s;
    }
    __syncthreads();
    // X1 = L^{-T} X2  (Cbar before symmetrising)
    for (int e = tid; e < J * J; e += AS_THREADS) {
        const int a = e / J, b = e % J;
        double s = 0.0;
#pragma unroll 4
        for (int c = a; c < J; ++c) s = __builtin_fma(Linv[(size_t)c * ld + a], X2[(size_t)c * ld + b], s);
        X1[(size_t)a * ld + b] = s;
    }
    __syncthreads();
    double gn = 0.0;
    for (int e = tid; e < imax * lg; e += AS_THREADS) {
        const int a = e / lg, b = e % lg;
        float v = 0.0f;
        if (a < J) {
            if (b < J) {
                const double cs = 0.5 * (X1[(size_t)a * ld + b] + X1[(size_t)b * ld + a]);
                gn = __builtin_fma(cs, G2[(size_t)a * lg + b], gn);
                v = (float)cs;
            } else if (b == imax) {
                v = (float)cb[a];
            }
        }
        Cc[e] = v;
    }
    gn = wave_sum(gn);
    if ((tid & 63) == 0) red[tid >> 6] = gn;
    __syncthreads();
    if (tid == 0) {
        double s = 0.0;
        for (int k = 0; k < AS_THREADS / 64; ++k) s += red[k];
        grad[inoise] += s;
    }
}

void launch_adj_small(int J, int imax, const double* G1, const double* G2, const double* L,
                      const double* Linv, double* X1, double* X2, float* Cc, double* grad,
                      int inoise, hipStream_t st) {
    hipLaunchKernelGGL(k_adj_small, dim3(1), dim3(AS_THREADS), 0, st, J, imax, G1, G2, L, Linv,
                       X1, X2, Cc, grad, inoise);
}

// ---------------------------------------------------------------- scatter and predict
// Mb[idx[q], c] += Mob[q, c] (c < rank), mb[idx[q]] -= Zr[q, imax]; one wave per row.
// The indices of a step are distinct, so no two rows write the same entries.
__global__ __launch_bounds__(256) void k_adj_scatter(const int32_t* __restrict__ idx, int m, int n,
                                                     const float* __restrict__ Mob, int ldmo,
                                                     int rank, const float* __restrict__ Zr,
                                                     int ldz, int imax, float* __restrict__ Mb,
                                                     int ldM, float* __restrict__ mb) {
    const int lane = threadIdx.x & 63;
    const int q = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (q >= m) return;
    int p = idx[q];
    if (p < 0 || p >= n) p = 0;
    for (int c = lane; c < rank; c += 64) Mb[(size_t)p * ldM + c] += Mob[(size_t)q * ldmo + c];
    if (lane == 0) mb[p] -= Zr[(size_t)q * ldz + imax];
}

void launch_adj_scatter(const int32_t* idx, int m, int n, const float* Mob, int ldmo, int rank,
                        const float* Zr, int ldz, int imax, float* Mb, int ldM, float* mb,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_adj_scatter, dim3((m + 3) / 4), dim3(256), 0, st, idx, m, n, Mob, ldmo,
                       rank, Zr, ldz, imax, Mb, ldM, mb);
}

// Predict adjoint of m^- = a m_{k-1}, M^- = a M^+_{k-1}: per-block FP64 partials of
// <mb, m_{k-1}> + <Mb[:, :rank], M^+_{k-1}>, then mb *= a, Mb[:, :rank] *= a.  One wave
// per row.
__global__ __launch_bounds__(256) void k_adj_predict(float* __restrict__ mb,
                                                     const float* __restrict__ mprev,
                                                     float* __restrict__ Mb, int ldM,
                                                     const float* __restrict__ Mprev,
                                                     int ldprev, int rank, int n, float a,
                                                     double* __restrict__ part) {
    __shared__ double red[4];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int p = blockIdx.x * 4 + w;
    double s = 0.0;
    if (p < n) {
        for (int c = lane; c < rank; c += 64) {
            const float v = Mb[(size_t)p * ldM + c];
            s = __builtin_fma((double)v, (double)Mprev[(size_t)p * ldprev + c], s);
            Mb[(size_t)p * ldM + c] = a * v;
        }
        if (lane == 0) {
            const float v = mb[p];
            if (mprev) s = __builtin_fma((double)v, (double)mprev[p], s);
            mb[p] = a * v;
        }
    }
    s = wave_sum(s);
    if (lane == 0) red[w] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

int launch_adj_predict(float* mb, const float* mprev, float* Mb, int ldM, const float* Mprev,
                       int ldprev, int rank, int n, float a, double* part, hipStream_t st) {
    const int blocks = (n + 3) / 4;
    hipLaunchKernelGGL(k_adj_predict, dim3(blocks), dim3(256), 0, st, mb, mprev, Mb, ldM, Mprev,
                       ldprev, rank, n, a, part);
    return blocks;
}

// grad[i] += sum of part[0..nblk) (one block, fixed order).
__global__ __launch_bounds__(256) void k_sum_into(const double* __restrict__ part, int nblk,
                                                  double* __restrict__ grad, int i) {
    __shared__ double r[256];
    double a = 0.0;
    for (int k = threadIdx.x; k < nblk; k += 256) a += part[k];
    r[threadIdx.x] = a;
    __syncthreads();
    for (int s = 128; s >= 1; s >>= 1) {
        if ((int)threadIdx.x < s) r[threadIdx.x] += r[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) grad[i] += r[0];
}

void launch_sum_into(const double* part, int nblk, double* grad, int i, hipStream_t st) {
    hipLaunchKernelGGL(k_sum_into, dim3(1), dim3(256), 0, st, part, nblk, grad, i);
}

}  // namespace cakf
