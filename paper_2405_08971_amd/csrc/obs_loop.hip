// Observation-space part of the CAKF update on gfx950: gather, the action loop and the
// Cholesky form of the projected update.
//
// The update conditions the predictive belief on S^T y (Sec. 3.1) with the projected
// Gram matrix C = S^T Ghat S, Ghat = H P^- H^T + Lambda = sigma_f2 K(Xo, Xo)
// - Mo Mo^T + noise_var I, Mo = H M^-.  Actions are chosen one at a time (the iterative
// update of App. B); with the CG policy the next action is the current residual
// (Sec. 3.3).  The kernels keep, per action s_j,
//     u_j = sigma_f2 K(Xo, Xo) s_j   (U, m x i),   t_j = Mo^T s_j   (T, r x i),
// so that column j of C is  S^T u_j - T^T t_j + noise_var S^T s_j  and the residual
// after j+1 actions is r0 - (U - Mo T + noise_var S) beta with beta = C^{-1} S^T r0.  C is factorised incrementally in FP64 (C = L L^T with L^{-1}
// kept explicitly); the Ghat-orthonormal directions of the iterative update are
// S L^{-T} (App. B), which is what the block product consumes.
//
// One iteration j launches: sym_tiles (u_j), form_u (u_j and the Gram partial sums),
// tail (one FP64 block), next_action (CG only: s_{j+1} and partial sums of Mo^T s_{j+1}).
#include "cakf_common.h"
#include "launchers.h"

namespace cakf {

// ------------------------------------------------------------------------------ gather
// One wave per observation row q in [0, mp): Xo, r0 = y - m^-[idx], Mo = M^-[idx, :rank],
// and the action rows (zero, then s_0 = r0 for CG or the given actions).  An index
// outside [0, n) is counted in the loop state and read as index 0.
__global__ __launch_bounds__(256) void k_gather(const float4* __restrict__ Xs, int n,
                                                const float* __restrict__ mean,
                                                const float* __restrict__ M, int ldM,
                                                const int32_t* __restrict__ idx,
                                                const float* __restrict__ y,
                                                const float* __restrict__ given, int cg,
                                                ObsDims d, float4* __restrict__ Xo,
                                                float* __restrict__ r0,
                                                float* __restrict__ Mo,
                                                float* __restrict__ S,
                                                float* __restrict__ U,
                                                LoopState* __restrict__ ls) {
    const int lane = threadIdx.x & 63;
    const int q = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (q >= d.mp) return;
    const bool real = q < d.m;
    int p = real ? idx[q] : idx[0];
    if (p < 0 || p >= n) {
        if (real && lane == 0) atomicAdd(&ls->bad_index, 1);
        p = 0;
    }
    float rq = 0.0f;
    if (real) rq = y[q] - mean[p];
    if (lane == 0) {
        Xo[q] = Xs[p];
        r0[q] = rq;
    }
    const float* Mrow = M + (size_t)p * ldM;
    float* Morow = Mo + (size_t)q * d.ldmo;
    for (int c = lane; c < d.ldmo; c += 64) Morow[c] = (real && c < d.rank) ? Mrow[c] : 0.0f;
    float* Srow = S + (size_t)q * d.imax;
    float* Urow = U + (size_t)q * d.imax;
    for (int l = lane; l < d.imax; l += 64) {
        float v = 0.0f;
        if (real) {
            if (cg) v = (l == 0) ? rq : 0.0f;
            else v = given[(size_t)q * d.imax + l];
        }
        Srow[l] = v;
        Urow[l] = 0.0f;
    }
}

void launch_gather(const float4* Xs, int n, const float* mean, const float* M, int ldM,
                   const int32_t* idx, const float* y, const float* given, int cg,
                   const ObsDims& d, float4* Xo, float* r0, float* Mo, float* S, float* U,
                   LoopState* ls, hipStream_t st) {
    const int blocks = (d.mp + 3) / 4;
    hipLaunchKernelGGL(k_gather, dim3(blocks), dim3(256), 0, st, Xs, n, mean, M, ldM, idx, y,
                       given, cg, d, Xo, r0, Mo, S, U, ls);
}

// ------------------------------------------------------------- column sums A^T x (det.)
// partial[b, c] = sum over the 256 rows of block b of A[p, c] * x[p].
__global__ __launch_bounds__(256) void k_colsum_partial(const float* __restrict__ A, int lda,
                                                        int rows, int cols,
                                                        const float* __restrict__ x,
                                                        int ldx,
                                                        float* __restrict__ partial,
                                                        int ldp) {
    __shared__ float red[4][1024];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int p0 = (blockIdx.x * 4 + w) * 64;
    float acc[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) acc[u] = 0.0f;
    const int pend = min(rows, p0 + 64);
    for (int p = p0; p < pend; ++p) {
        const float xv = x[(size_t)p * ldx];
        const float* row = A + (size_t)p * lda;
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int c = lane + 64 * u;
            if (c < cols) acc[u] = __builtin_fmaf(row[c], xv, acc[u]);
        }
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int c = lane + 64 * u;
        if (c < cols) red[w][c] = acc[u];
    }
    __syncthreads();
    for (int c = threadIdx.x; c < cols; c += 256)
        partial[(size_t)blockIdx.x * ldp + c] = (red[0][c] + red[1][c]) + (red[2][c] + red[3][c]);
}

void launch_colsum_partial(const float* A, int lda, int rows, int cols, const float* x,
                           int ldx, float* partial, int ldp, hipStream_t st, int* nblk_out) {
    const int blocks = (rows + 255) / 256;
    *nblk_out = blocks;
    hipLaunchKernelGGL(k_colsum_partial, dim3(blocks), dim3(256), 0, st, A, lda, rows, cols,
                       x, ldx, partial, ldp);
}

__global__ __launch_bounds__(256) void k_colsum_final(const float* __restrict__ partial,
                                                      int ldp, int nblk, int cols,
                                                      float* __restrict__ out, int ldo) {
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= cols) return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += partial[(size_t)b * ldp + c];
    out[(size_t)c * ldo] = (float)s;
}

void launch_colsum_final(const float* partial, int ldp, int nblk, int cols, float* out,
                         int ldo, hipStream_t st) {
    if (cols <= 0) return;
    hipLaunchKernelGGL(k_colsum_final, dim3((cols + 255) / 256), dim3(256), 0, st, partial,
                       ldp, nblk, cols, out, ldo);
}

// ----------------------------------------------------------- symmetric kernel matvec
// u_j = K(Xo, Xo) s_j over the upper triangle of SYM_TILE x SYM_TILE tiles.  Tile (P, Q),
// P <= Q, adds its row sums K_PQ s_Q to slot Q of block P and (P < Q) its column sums
// K_PQ^T s_P to slot P of block Q; every (slot, block) pair is written exactly once, so
// the reduction in form_u is deterministic.  Each thread evaluates an 8 x 8 set of
// entries.  Blocks below n_extra instead finish t_j = Mo^T s_j from next_action's
// partial sums.
template <int NU2, int DIST>
__global__ __launch_bounds__(256) void k_sym_tiles(const float4* __restrict__ Xo,
                                                   const float* __restrict__ S, ObsDims d,
                                                   int j, float* __restrict__ part,
                                                   const float* __restrict__ mpart,
                                                   int nmpart, int n_extra,
                                                   float* __restrict__ T,
                                                   double* __restrict__ ttpart,
                                                   const LoopState* __restrict__ ls) {
    if (ls->stop) return;
    if ((int)blockIdx.x < n_extra) {
        // t_j = Mo^T s_j for the 256 rows c of this block's slice of T (finished from
        // next_action's partial sums for CG, precomputed otherwise), then the slice's
        // contribution to (T^T t_j)_l for l <= j.
        __shared__ float tj[256];
        const int c = blockIdx.x * 256 + threadIdx.x;
        float v = 0.0f;
        if (c < d.rank) {
            if (mpart) {
                double s = 0.0;
                for (int b = 0; b < nmpart; ++b) s += mpart[(size_t)b * d.ldmo + c];
                v = (float)s;
                T[(size_t)c * d.imax + j] = v;
            } else {
                v = T[(size_t)c * d.imax + j];
            }
        }
        tj[threadIdx.x] = v;
        __syncthreads();
        const int cend = min(256, d.rank - (int)blockIdx.x * 256);
        for (int l = threadIdx.x; l <= j; l += 256) {
            double acc = 0.0;
            const float* Tc = T + (size_t)blockIdx.x * 256 * d.imax + l;
            for (int cc = 0; cc < cend; ++cc) {
                const float tl = (l == j) ? tj[cc] : Tc[(size_t)cc * d.imax];
                acc = __builtin_fma((double)tl, (double)tj[cc], acc);
            }
            ttpart[(size_t)blockIdx.x * d.imax + l] = acc;
        }
        return;
    }
    const int t = blockIdx.x - n_extra;
    // column-major enumeration of the upper triangle: t = Q (Q + 1) / 2 + P
    int Q = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
    while ((Q + 1) * (Q + 2) / 2 <= t) ++Q;
    while (Q * (Q + 1) / 2 > t) --Q;
    const int P = t - Q * (Q + 1) / 2;

    __shared__ float4 xr[SYM_TILE], xc[SYM_TILE];
    __shared__ float sr[SYM_TILE], sc[SYM_TILE];
    __shared__ float red[2][16][SYM_TILE + 1];
    const int tid = threadIdx.x;
    const int P0 = P * SYM_TILE, Q0 = Q * SYM_TILE;
    if (tid < SYM_TILE) {
        xr[tid] = Xo[P0 + tid];
        sr[tid] = S[(size_t)(P0 + tid) * d.imax + j];
    } else {
        const int u = tid - SYM_TILE;
        xc[u] = Xo[Q0 + u];
        sc[u] = S[(size_t)(Q0 + u) * d.imax + j];
    }
    __syncthreads();
    const int tr = tid >> 4, tc = tid & 15;
    float4 a[8], b[8];
    float sa[8], sb[8], ra[8], cb[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        a[i] = xr[tr + 16 * i];
        sa[i] = sr[tr + 16 * i];
        b[i] = xc[tc + 16 * i];
        sb[i] = sc[tc + 16 * i];
        ra[i] = 0.0f;
        cb[i] = 0.0f;
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const float kv = kval<NU2, DIST>(a[i], b[k]);
            ra[i] = __builtin_fmaf(kv, sb[k], ra[i]);
            cb[k] = __builtin_fmaf(kv, sa[i], cb[k]);
        }
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        red[0][tc][tr + 16 * i] = ra[i];
        red[1][tr][tc + 16 * i] = cb[i];
    }
    __syncthreads();
    if (tid < SYM_TILE) {
        float s = 0.0f;
#pragma unroll
        for (int g = 0; g < 16; ++g) s += red[0][g][tid];
        part[(size_t)Q * d.mp + P0 + tid] = s;
    } else if (P != Q) {
        const int u = tid - SYM_TILE;
        float s = 0.0f;
#pragma unroll
        for (int g = 0; g < 16; ++g) s += red[1][g][u];
        part[(size_t)P * d.mp + Q0 + u] = s;
    }
}

void launch_sym_tiles(int nu2, int dist, const float4* Xo, const float* S, const ObsDims& d,
                      int j, float* part, const float* mpart, int nmpart, float* T,
                      double* ttpart, const LoopState* ls, hipStream_t st) {
    const int nb = d.mp / SYM_TILE;
    const int tiles = nb * (nb + 1) / 2;
    const int n_extra = (d.rank + 255) / 256;
    CAKF_DISPATCH_KERNEL(nu2, dist,
        hipLaunchKernelGGL((k_sym_tiles<NU2, DIST>), dim3(tiles + n_extra), dim3(256), 0, st,
                           Xo, S, d, j, part, mpart, nmpart, n_extra, T, ttpart, ls));
}

// ------------------------------------------------------------------------- form_u
// u_j[p] = sigma_f2 * (sum over the nb slots of the tile partial sums, FP64), i.e.
// U = Sigma[idx, idx] S, stored in U[:, j];
// per-block partial sums (FP64) of g_l = s_l^T u_j, q_l = s_l^T s_j (l <= j) and
// c = r0^T s_j.  Layout of one block's partials: [g (imax) | q (imax) | c].
__global__ __launch_bounds__(256) void k_form_u(const float* __restrict__ part,
                                                const float* __restrict__ S,
                                                float* __restrict__ U,
                                                const float* __restrict__ r0, ObsDims d,
                                                int j, double sigma_f2,
                                                double* __restrict__ gpart,
                                                const LoopState* __restrict__ ls) {
    if (ls->stop) return;
    __shared__ double red[4][2 * 256 + 1];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int p0 = (blockIdx.x * 4 + w) * 64;
    const int nb = d.mp / SYM_TILE;
    const int p = p0 + lane;
    float u = 0.0f, sp = 0.0f;
    double cc = 0.0;
    if (p < d.m) {
        double acc = 0.0;
        for (int s = 0; s < nb; ++s) acc += part[(size_t)s * d.mp + p];
        u = (float)(sigma_f2 * acc);
        U[(size_t)p * d.imax + j] = u;
        sp = S[(size_t)p * d.imax + j];
        cc = (double)r0[p] * (double)sp;
    }
    double g[4] = {0.0, 0.0, 0.0, 0.0}, q[4] = {0.0, 0.0, 0.0, 0.0};
    const int rows = min(64, d.m - p0);
    for (int rr = 0; rr < rows; ++rr) {
        const double ur = (double)__shfl(u, rr, 64);
        const double srr = (double)__shfl(sp, rr, 64);
        const float* Srow = S + (size_t)(p0 + rr) * d.imax;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int l = lane + 64 * v;
            if (l <= j) {
                const double sl = (double)Srow[l];
                g[v] = __builtin_fma(sl, ur, g[v]);
                q[v] = __builtin_fma(sl, srr, q[v]);
            }
        }
    }
    cc = wave_sum(cc);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int l = lane + 64 * v;
        if (l <= j) {
            red[w][l] = g[v];
            red[w][256 + l] = q[v];
        }
    }
    if (lane == 0) red[w][512] = cc;
    __syncthreads();
    const int gs = 2 * d.imax + 1;
    double* out = gpart + (size_t)blockIdx.x * gs;
    for (int l = threadIdx.x; l <= j; l += 256) {
        out[l] = (red[0][l] + red[1][l]) + (red[2][l] + red[3][l]);
        out[d.imax + l] = (red[0][256 + l] + red[1][256 + l]) + (red[2][256 + l] + red[3][256 + l]);
    }
    if (threadIdx.x == 0) out[2 * d.imax] = (red[0][512] + red[1][512]) + (red[2][512] + red[3][512]);
}

void launch_form_u(const float* part, const float* S, float* U, const float* r0,
                   const ObsDims& d, int j, double sigma_f2, double* gpart,
                   const LoopState* ls, hipStream_t st, int* nblk_out) {
    const int blocks = (d.m + 255) / 256;
    *nblk_out = blocks;
    hipLaunchKernelGGL(k_form_u, dim3(blocks), dim3(256), 0, st, part, S, U, r0, d, j,
                       sigma_f2, gpart, ls);
}

// --------------------------------------------------------------------------- tail
// One block, FP64.  Finishes column j of C = S^T Ghat S, extends its Cholesky factor
// (with the explicit inverse L^{-1}), alpha = L^{-1} S^T r0, beta = L^{-T} alpha, the
// Cholesky factor of S^T S (log det only) and the log-likelihood term.  Stops the loop
// on breakdown (pivot) or residual tolerance.
__global__ __launch_bounds__(256) void k_tail(const double* __restrict__ gpart, int nblk,
                                              const double* __restrict__ ttpart, int ntt,
                                              ObsDims d, int j, double noise_var,
                                              double resid_tol, double pivot_tol,
                                              double* __restrict__ Linv,
                                              double* __restrict__ L,
                                              double* __restrict__ LSinv,
                                              double* __restrict__ alpha,
                                              double* __restrict__ beta,
                                              LoopState* __restrict__ ls) {
    __shared__ double Ccol[1024], Qcol[1024], lrow[1024], lsrow[1024], sred[256];
    __shared__ double s_c, s_d2, s_ds2;
    __shared__ int s_stop;
    const int tid = threadIdx.x;
    if (ls->stop) return;
    const int gs = 2 * d.imax + 1;
    const int ld = d.imax;
    // column j of S^T K S and S^T S, and c_j = s_j^T r0
    for (int l = tid; l <= j; l += 256) {
        double g = 0.0, q = 0.0;
        for (int b = 0; b < nblk; ++b) {
            g += gpart[(size_t)b * gs + l];
            q += gpart[(size_t)b * gs + d.imax + l];
        }
        double tt = 0.0;   // (T^T t_j)_l
        for (int b = 0; b < ntt; ++b) tt += ttpart[(size_t)b * d.imax + l];
        Ccol[l] = g - tt + noise_var * q;
        Qcol[l] = q;
    }
    if (tid == 0) {
        double c = 0.0;
        for (int b = 0; b < nblk; ++b) c += gpart[(size_t)b * gs + 2 * d.imax];
        s_c = c;
        s_stop = 0;
    }
    __syncthreads();
    if (tid == 0) {
        if (j == 0) {
            ls->q00 = Qcol[0];
        } else if (resid_tol > 0.0 && Qcol[j] <= resid_tol * resid_tol * ls->q00) {
            s_stop = 1;
        }
    }
    __syncthreads();
    if (s_stop) {
        if (tid == 0) ls->stop = 1;
        return;
    }
    // new row of L: l = L^{-1} C[0:j, j]
    for (int k = tid; k < j; k += 256) {
        double acc = 0.0;
        for (int p = 0; p <= k; ++p) acc = __builtin_fma(Linv[(size_t)k * ld + p], Ccol[p], acc);
        lrow[k] = acc;
    }
    for (int k = tid; k < j; k += 256) {
        double acc = 0.0;
        for (int p = 0; p <= k; ++p) acc = __builtin_fma(LSinv[(size_t)k * ld + p], Qcol[p], acc);
        lsrow[k] = acc;
    }
    __syncthreads();
    double part = 0.0, parts = 0.0;
    for (int k = tid; k < j; k += 256) {
        part = __builtin_fma(lrow[k], lrow[k], part);
        parts = __builtin_fma(lsrow[k], lsrow[k], parts);
    }
    sred[tid] = part;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (tid < off) sred[tid] += sred[tid + off];
        __syncthreads();
    }
    if (tid == 0) s_d2 = Ccol[j] - sred[0];
    __syncthreads();
    sred[tid] = parts;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (tid < off) sred[tid] += sred[tid + off];
        __syncthreads();
    }
    if (tid == 0) {
        s_ds2 = Qcol[j] - sred[0];
        const double d2 = s_d2;
        const bool finite = isfinite(d2) && isfinite(Ccol[j]);
        if (!(finite && d2 > pivot_tol * Ccol[j] && d2 > 0.0)) {
            s_stop = 1;
            ls->stop = 1;
            ls->dropped += 1;
            if (!finite) ls->nonfinite += 1;
        }
    }
    __syncthreads();
    if (s_stop) return;
    const double dj = sqrt(s_d2);
    const double inv_d = 1.0 / dj;
    // L^{-1} new row: -(l^T L^{-1}) / d and 1 / d; L new row for the record
    for (int p = tid; p < j; p += 256) {
        double acc = 0.0;
        for (int k = p; k < j; ++k) acc = __builtin_fma(lrow[k], Linv[(size_t)k * ld + p], acc);
        Linv[(size_t)j * ld + p] = -acc * inv_d;
        L[(size_t)j * ld + p] = lrow[p];
    }
    const double ds = sqrt(fmax(s_ds2, 1e-300));
    for (int p = tid; p < j; p += 256) {
        double acc = 0.0;
        for (int k = p; k < j; ++k) acc = __builtin_fma(lsrow[k], LSinv[(size_t)k * ld + p], acc);
        LSinv[(size_t)j * ld + p] = -acc / ds;
    }
    if (tid == 0) {
        Linv[(size_t)j * ld + j] = inv_d;
        L[(size_t)j * ld + j] = dj;
        LSinv[(size_t)j * ld + j] = 1.0 / ds;
        double acc = 0.0;
        for (int k = 0; k < j; ++k) acc = __builtin_fma(lrow[k], alpha[k], acc);
        const double aj = (s_c - acc) * inv_d;
        alpha[j] = aj;
        ls->logdet_c += 2.0 * log(dj);
        ls->logdet_s += 2.0 * log(ds);
        ls->alpha2 += aj * aj;
        ls->i_eff = j + 1;
        ls->loglik = -0.5 * ((double)(j + 1) * 1.8378770664093453 + ls->logdet_c -
                             ls->logdet_s + ls->alpha2);
    }
    __syncthreads();
    __threadfence_block();
    // beta = L^{-T} alpha over the kept actions
    for (int p = tid; p <= j; p += 256) {
        double acc = 0.0;
        for (int k = p; k <= j; ++k) acc = __builtin_fma(Linv[(size_t)k * ld + p], alpha[k], acc);
        beta[p] = acc;
    }
}

void launch_tail(const double* gpart, int nblk, const double* ttpart, const ObsDims& d,
                 int j, double noise_var, double resid_tol, double pivot_tol, double* Linv,
                 double* L, double* LSinv, double* alpha, double* beta, LoopState* ls,
                 hipStream_t st) {
    const int ntt = (d.rank + 255) / 256;
    hipLaunchKernelGGL(k_tail, dim3(1), dim3(256), 0, st, gpart, nblk, ttpart, ntt, d, j,
                       noise_var, resid_tol, pivot_tol, Linv, L, LSinv, alpha, beta, ls);
}

// ---------------------------------------------------------------------- next_action
// CG policy: s_{j+1} = r0 - Ghat S beta = r0 - (U - Mo T + noise_var S) beta (the
// residual after j+1 actions), stored unnormalised in S[:, j+1], and per-block partial
// sums of Mo^T s_{j+1} (finished by the next sym_tiles launch).  T beta is formed by
// every block from the small r x (j+1) matrix T.
__global__ __launch_bounds__(256) void k_next_action(const float* __restrict__ U,
                                                     const float* __restrict__ Mo,
                                                     const float* __restrict__ r0,
                                                     float* __restrict__ S,
                                                     const double* __restrict__ beta,
                                                     const float* __restrict__ T,
                                                     float noise_var, ObsDims d, int j,
                                                     float* __restrict__ mpart,
                                                     const LoopState* __restrict__ ls) {
    if (ls->stop) return;
    __shared__ float red[4][1024];
    __shared__ float Tbeta[1024];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int p0 = (blockIdx.x * 4 + w) * 64;
    for (int c = threadIdx.x; c < d.rank; c += 256) {
        double acc = 0.0;
        const float* Tc = T + (size_t)c * d.imax;
        for (int l = 0; l <= j; ++l) acc = __builtin_fma((double)Tc[l], beta[l], acc);
        Tbeta[c] = (float)acc;
    }
    __syncthreads();
    float bl[4], tb[16], acc[16];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int l = lane + 64 * v;
        bl[v] = (l <= j) ? (float)beta[l] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int c = lane + 64 * u;
        tb[u] = (c < d.rank) ? Tbeta[c] : 0.0f;
        acc[u] = 0.0f;
    }
    const int rows = min(64, d.m - p0);
    for (int rr = 0; rr < rows; ++rr) {
        const int p = p0 + rr;
        const float* Urow = U + (size_t)p * d.imax;
        const float* Srow = S + (size_t)p * d.imax;
        const float* Mrow = Mo + (size_t)p * d.ldmo;
        float part = 0.0f;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int l = lane + 64 * v;
            if (l <= j) part -= __builtin_fmaf(noise_var, Srow[l], Urow[l]) * bl[v];
        }
        float mo[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int c = lane + 64 * u;
            mo[u] = (c < d.rank) ? Mrow[c] : 0.0f;
            part = __builtin_fmaf(mo[u], tb[u], part);
        }
        const float rho = r0[p] + wave_sum(part);
        if (lane == 0) S[(size_t)p * d.imax + j + 1] = rho;
#pragma unroll
        for (int u = 0; u < 16; ++u) acc[u] = __builtin_fmaf(mo[u], rho, acc[u]);
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int c = lane + 64 * u;
        if (c < d.rank) red[w][c] = acc[u];
    }
    __syncthreads();
    for (int c = threadIdx.x; c < d.rank; c += 256)
        mpart[(size_t)blockIdx.x * d.ldmo + c] = (red[0][c] + red[1][c]) + (red[2][c] + red[3][c]);
}

void launch_next_action(const float* U, const float* Mo, const float* r0, float* S,
                        const double* beta, const float* T, float noise_var,
                        const ObsDims& d, int j, float* mpart, const LoopState* ls,
                        hipStream_t st, int* nblk_out) {
    const int blocks = (d.m + 255) / 256;
    *nblk_out = blocks;
    hipLaunchKernelGGL(k_next_action, dim3(blocks), dim3(256), 0, st, U, Mo, r0, S, beta, T,
                       noise_var, d, j, mpart, ls);
}

// ----------------------------------------------------------------------- build_block
// B = [S L^{-T} | S beta | 0] (mp x bp, row-major) for the block product, plus the
// optional record copies (m rows).  FP64 accumulation.
__global__ __launch_bounds__(256) void k_build_block(const float* __restrict__ S,
                                                     const double* __restrict__ Linv,
                                                     const double* __restrict__ beta,
                                                     ObsDims d, float* __restrict__ B,
                                                     int ldb, int bp,
                                                     float* __restrict__ rec_W,
                                                     float* __restrict__ rec_w,
                                                     float* __restrict__ rec_S,
                                                     const LoopState* __restrict__ ls) {
    const int kept = ls->i_eff;
    const size_t total = (size_t)d.mp * bp;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < total;
         e += (size_t)gridDim.x * 256) {
        const int p = (int)(e / bp), c = (int)(e % bp);
        const float* Srow = S + (size_t)p * d.imax;
        double acc = 0.0;
        if (p < d.m) {
            if (c < d.imax) {
                const double* Lrow = Linv + (size_t)c * d.imax;
                for (int l = 0; l <= c; ++l) acc = __builtin_fma((double)Srow[l], Lrow[l], acc);
            } else if (c == d.imax) {
                for (int l = 0; l < d.imax; ++l) acc = __builtin_fma((double)Srow[l], beta[l], acc);
            }
        }
        const float v = (float)acc;
        B[(size_t)p * ldb + c] = v;
        if (p < d.m) {
            if (c < d.imax) {
                if (rec_W) rec_W[(size_t)p * d.imax + c] = v;
                if (rec_S) rec_S[(size_t)p * d.imax + c] = c < kept ? Srow[c] : 0.0f;
            } else if (c == d.imax && rec_w) {
                rec_w[p] = v;
            }
        }
    }
}

void launch_build_block(const float* S, const double* Linv, const double* beta,
                        const ObsDims& d, float* B, int ldb, int bp, float* rec_W,
                        float* rec_w, float* rec_S, const LoopState* ls, hipStream_t st) {
    const size_t total = (size_t)d.mp * bp;
    const int blocks = (int)std::min<size_t>((total + 255) / 256, 65536);
    hipLaunchKernelGGL(k_build_block, dim3(blocks), dim3(256), 0, st, S, Linv, beta, d, B, ldb,
                       bp, rec_W, rec_w, rec_S, ls);
}

// Record outputs that live in the loop state.
__global__ void k_finish_record(const LoopState* __restrict__ ls, const double* __restrict__ L,
                                int imax, double* __restrict__ rec_chol,
                                double* __restrict__ rec_loglik, int* __restrict__ rec_n) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    if (rec_chol) {
        for (int e = tid; e < imax * imax; e += gridDim.x * blockDim.x) rec_chol[e] = L[e];
    }
    if (tid == 0) {
        if (rec_loglik) *rec_loglik = ls->loglik;
        if (rec_n) *rec_n = ls->i_eff;
    }
}

void launch_finish_record(const LoopState* ls, const double* L, int imax, double* rec_chol,
                          double* rec_loglik, int* rec_n, hipStream_t st) {
    hipLaunchKernelGGL(k_finish_record, dim3(64), dim3(256), 0, st, ls, L, imax, rec_chol,
                       rec_loglik, rec_n);
}

}  // namespace cakf
