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
// tail (one FP64 block), next_action (CG only: s_{j+1}, V[:, j] = Mo t_j and partial
// sums of Mo^T s_{j+1}).
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
// entries.  With mpart (CG policy, j > 0) the first n_extra blocks instead finish
// t_j = Mo^T s_j (column j of T, stored column-major: T[l * ldmo + c]) from
// next_action's per-block partial sums, 64 factor columns per block.
template <int NU2, int DIST>
__global__ __launch_bounds__(256) void k_sym_tiles(const float4* __restrict__ Xo,
                                                   const float* __restrict__ S, ObsDims d,
                                                   int j, float* __restrict__ part,
                                                   const float* __restrict__ mpart,
                                                   int nmpart, int n_extra,
                                                   float* __restrict__ T,
                                                   const LoopState* __restrict__ ls) {
    if (ls->stop) return;
    if ((int)blockIdx.x < n_extra) {
        __shared__ double tred[4][64];
        const int cl = threadIdx.x & 63, grp = threadIdx.x >> 6;
        const int c = blockIdx.x * 64 + cl;
        double a8[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) a8[u] = 0.0;
        if (c < d.rank) {
            int b = grp;
            for (; b + 28 < nmpart; b += 32) {
#pragma unroll
                for (int u = 0; u < 8; ++u) a8[u] += mpart[(size_t)(b + 4 * u) * d.ldmo + c];
            }
            for (; b < nmpart; b += 4) a8[0] += mpart[(size_t)b * d.ldmo + c];
        }
        tred[grp][cl] = ((a8[0] + a8[1]) + (a8[2] + a8[3])) + ((a8[4] + a8[5]) + (a8[6] + a8[7]));
        __syncthreads();
        if (grp == 0 && c < d.rank)
            T[(size_t)j * d.ldmo + c] =
                (float)((tred[0][cl] + tred[1][cl]) + (tred[2][cl] + tred[3][cl]));
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
        a[i] = prep_row<DIST>(xr[tr + 16 * i]);
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
                      const LoopState* ls, hipStream_t st) {
    const int nb = d.mp / SYM_TILE;
    const int tiles = nb * (nb + 1) / 2;
    const int n_extra = (mpart && nmpart > 0) ? (d.rank + 63) / 64 : 0;
    CAKF_DISPATCH_KERNEL(nu2, dist,
        hipLaunchKernelGGL((k_sym_tiles<NU2, DIST>), dim3(tiles + n_extra), dim3(256), 0, st,
                           Xo, S, d, j, part, mpart, nmpart, n_extra, T, ls));
}

// ------------------------------------------------------------------------- form_u
// u_j[p] = sigma_f2 * (sum over the nb slots of the tile partial sums, FP64), i.e.
// U = Sigma[idx, idx] S, stored in U[:, j]; per-block partial sums (FP64) of
// g_l = s_l^T u_j, q_l = s_l^T s_j (l <= j) and c = r0^T s_j.  A row block covers
// FU_CHUNKS chunks of FU_ROWS rows; each chunk stages its action rows in LDS with all
// loads in flight at once.  Layout of one block's partials: [g (imax) | q (imax) | c].
// The TT_COLS-wide column blocks after the row blocks compute (T^T t_j)_l = t_l^T t_j
// for l <= j (FP64), one wave per column group.
constexpr int FU_ROWS = 64;
constexpr int FU_CHUNKS = 2;
constexpr int TT_COLS = 16;

__global__ __launch_bounds__(256) void k_form_u(const float* __restrict__ part,
                                                const float* __restrict__ S,
                                                float* __restrict__ U,
                                                const float* __restrict__ r0,
                                                const float* __restrict__ T, ObsDims d,
                                                int j, double sigma_f2, int n_rowblk,
                                                double* __restrict__ gpart,
                                                double* __restrict__ ttv,
                                                const LoopState* __restrict__ ls) {
    if (ls->stop) return;
    const int tid = threadIdx.x;
    const int J = j + 1;
    if ((int)blockIdx.x >= n_rowblk) {
        // (T^T t_j)_l for l in this block's TT_COLS columns, 4 per wave
        const int lane = tid & 63, w = tid >> 6;
        const int l0 = (blockIdx.x - n_rowblk) * TT_COLS + w * (TT_COLS / 4);
        const float* tj = T + (size_t)j * d.ldmo;
        double acc[TT_COLS / 4];
#pragma unroll
        for (int u = 0; u < TT_COLS / 4; ++u) acc[u] = 0.0;
        for (int c0 = 0; c0 < d.rank; c0 += 64) {
            const int c = c0 + lane;
            const float tv = c < d.rank ? tj[c] : 0.0f;
#pragma unroll
            for (int u = 0; u < TT_COLS / 4; ++u) {
                const int l = l0 + u;
                const float tl = (l < J && c < d.rank) ? T[(size_t)l * d.ldmo + c] : 0.0f;
                acc[u] = __builtin_fma((double)tl, (double)tv, acc[u]);
            }
        }
#pragma unroll
        for (int u = 0; u < TT_COLS / 4; ++u) {
            const double v = wave_sum(acc[u]);
            if (lane == 0 && l0 + u < J) ttv[l0 + u] = v;
        }
        return;
    }
    __shared__ float Ss[FU_ROWS][257];
    __shared__ double ured[4][FU_ROWS];
    __shared__ float uu[FU_ROWS], ss[FU_ROWS], rr[FU_ROWS];
    const int nb = d.mp / SYM_TILE;
    double g = 0.0, q = 0.0, cc = 0.0;
    for (int chunk = 0; chunk < FU_CHUNKS; ++chunk) {
        const int p0 = (blockIdx.x * FU_CHUNKS + chunk) * FU_ROWS;
        if (p0 >= d.m) break;
        {
            const int row = tid & 63, grp = tid >> 6;
            const int p = p0 + row;
            double a8[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) a8[u] = 0.0;
            if (p < d.m) {
                int s = grp;
                for (; s + 28 < nb; s += 32) {
#pragma unroll
                    for (int u = 0; u < 8; ++u) a8[u] += part[(size_t)(s + 4 * u) * d.mp + p];
                }
                for (; s < nb; s += 4) a8[0] += part[(size_t)s * d.mp + p];
            }
            ured[grp][row] = ((a8[0] + a8[1]) + (a8[2] + a8[3])) + ((a8[4] + a8[5]) + (a8[6] + a8[7]));
        }
        const int total = FU_ROWS * J;
        for (int e0 = 0; e0 < total; e0 += 256 * 8) {
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int e = e0 + 256 * u + tid;
                v[u] = 0.0f;
                if (e < total) {
                    const int row = e / J, col = e - row * J;
                    const int p = p0 + row;
                    if (p < d.m) v[u] = S[(size_t)p * d.imax + col];
                }
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int e = e0 + 256 * u + tid;
                if (e < total) {
                    const int row = e / J, col = e - row * J;
                    Ss[row][col] = v[u];
                }
            }
        }
        __syncthreads();
        if (tid < FU_ROWS) {
            const int p = p0 + tid;
            float uf = (float)(sigma_f2 * ((ured[0][tid] + ured[1][tid]) + (ured[2][tid] + ured[3][tid])));
            float rv = 0.0f;
            if (p < d.m) {
                U[(size_t)p * d.imax + j] = uf;
                rv = r0[p];
            } else {
                uf = 0.0f;
            }
            uu[tid] = uf;
            ss[tid] = Ss[tid][j];
            rr[tid] = rv;
        }
        __syncthreads();
        if (tid < J) {
#pragma unroll 8
            for (int row = 0; row < FU_ROWS; ++row) {
                const double sl = (double)Ss[row][tid];
                g = __builtin_fma(sl, (double)uu[row], g);
                q = __builtin_fma(sl, (double)ss[row], q);
            }
        }
        if (tid >= 192) {
            const int row = tid - 192;
            cc = __builtin_fma((double)rr[row], (double)ss[row], cc);
        }
        __syncthreads();
    }
    const int gs = 2 * d.imax + 1;
    double* out = gpart + (size_t)blockIdx.x * gs;
    if (tid < J) {
        out[tid] = g;
        out[d.imax + tid] = q;
    }
    if (tid >= 192) {
        cc = wave_sum(cc);
        if (tid == 192) out[2 * d.imax] = cc;
    }
}

void launch_form_u(const float* part, const float* S, float* U, const float* r0,
                   const float* T, const ObsDims& d, int j, double sigma_f2, double* gpart,
                   double* ttv, const LoopState* ls, hipStream_t st, int* nblk_out) {
    const int rowblk = (d.m + FU_ROWS * FU_CHUNKS - 1) / (FU_ROWS * FU_CHUNKS);
    const int ttblk = d.rank > 0 ? (j + 1 + TT_COLS - 1) / TT_COLS : 0;
    *nblk_out = rowblk;
    hipLaunchKernelGGL(k_form_u, dim3(rowblk + ttblk), dim3(256), 0, st, part, S, U, r0, T, d,
                       j, sigma_f2, rowblk, gpart, ttv, ls);
}

// --------------------------------------------------------------------------- tail
// One block of 1024 threads, FP64.  Finishes column j of C = S^T Ghat S, extends its
// Cholesky factor C = L L^T (L^{-1} kept explicitly, row-major Linv and column-major
// LinvT so that every triangular product reads coalesced), alpha = L^{-1} S^T r0,
// beta = L^{-T} alpha, the Cholesky factor of S^T S (log det only) and the
// log-likelihood term.  Every reduction and triangular product splits its terms over
// several threads of a row and combines them with lane shuffles.  Stops the loop on
// breakdown (pivot) or residual tolerance.
constexpr int TAIL_THREADS = 1024;

__device__ __forceinline__ double tail_block_sum(double v, double* red) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < TAIL_THREADS / 64; ++k) s += red[k];
    return s;
}

// sum of v over groups of tpr consecutive lanes (tpr a power of two <= 64)
__device__ __forceinline__ double group_sum(double v, int tpr) {
    for (int off = tpr >> 1; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ int pow2_at_least(int v) {
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

__global__ __launch_bounds__(TAIL_THREADS) void k_tail(const double* __restrict__ gpart,
                                                       int nblk,
                                                       const double* __restrict__ ttv,
                                                       ObsDims d, int j, double noise_var,
                                                       double resid_tol, double pivot_tol,
                                                       double* __restrict__ Linv,
                                                       double* __restrict__ LinvT,
                                                       double* __restrict__ L,
                                                       double* __restrict__ LSinv,
                                                       double* __restrict__ LSinvT,
                                                       double* __restrict__ alpha,
                                                       double* __restrict__ beta,
                                                       LoopState* __restrict__ ls) {
    __shared__ double Ccol[256], Qcol[256], lrow[256], lsrow[256], nrow[256], alph[256];
    __shared__ double red[TAIL_THREADS / 64];
    const int tid = threadIdx.x;
    if (ls->stop) return;
    const int gs = 2 * d.imax + 1;
    const int ld = d.imax;
    const int J = j + 1;
    // 1. column j of S^T U and S^T S: pairs (array, l), tpp threads per pair
    {
        const int np = pow2_at_least(2 * J);
        const int tpp = TAIL_THREADS / np >= 64 ? 64 : TAIL_THREADS / np;
        const int pair = tid / tpp, sub = tid % tpp;
        double acc = 0.0;
        const bool live = pair < 2 * J;
        if (live) {
            const int off = pair < J ? pair : d.imax + (pair - J);
            double a4[4] = {0.0, 0.0, 0.0, 0.0};
            int b = sub;
            for (; b + 3 * tpp < nblk; b += 4 * tpp) {
#pragma unroll
                for (int u = 0; u < 4; ++u) a4[u] += gpart[(size_t)(b + u * tpp) * gs + off];
            }
            for (; b < nblk; b += tpp) a4[0] += gpart[(size_t)b * gs + off];
            acc = (a4[0] + a4[1]) + (a4[2] + a4[3]);
        }
        acc = group_sum(acc, tpp);
        if (live && sub == 0) {
            if (pair < J) Ccol[pair] = acc;
            else Qcol[pair - J] = acc;
        }
    }
    double cpart = 0.0;
    for (int b = tid; b < nblk; b += TAIL_THREADS) cpart += gpart[(size_t)b * gs + 2 * d.imax];
    const double c_j = tail_block_sum(cpart, red);        // includes __syncthreads
    if (tid < J) {
        const double tt = d.rank > 0 ? ttv[tid] : 0.0;
        Ccol[tid] = Ccol[tid] - tt + noise_var * Qcol[tid];
        alph[tid] = (tid < j) ? alpha[tid] : 0.0;
    }
    __syncthreads();
    if (j == 0) {
        if (tid == 0) ls->q00 = Qcol[0];
    } else if (resid_tol > 0.0 && Qcol[j] <= resid_tol * resid_tol * ls->q00) {
        if (tid == 0) ls->stop = 1;
        return;
    }
    // rows per triangular product: j (or J) rows, tpr threads per row
    const int tpr = j > 0 ? std::min(64, TAIL_THREADS / pow2_at_least(J)) : 1;
    const int row = tid / tpr, sub = tid % tpr;
    // 2. l = L^{-1} C[0:j, j] and ls = LS^{-1} Q[0:j, j]
    {
        double lk = 0.0, lsk = 0.0;
        if (row < j) {
            for (int p = sub; p <= row; p += tpr) {
                lk = __builtin_fma(LinvT[(size_t)p * ld + row], Ccol[p], lk);
                lsk = __builtin_fma(LSinvT[(size_t)p * ld + row], Qcol[p], lsk);
            }
        }
        lk = group_sum(lk, tpr);
        lsk = group_sum(lsk, tpr);
        if (row < j && sub == 0) {
            lrow[row] = lk;
            lsrow[row] = lsk;
        }
    }
    __syncthreads();
    double v1 = 0.0, v2 = 0.0, v3 = 0.0;
    if (tid < j) {
        v1 = lrow[tid] * lrow[tid];
        v2 = lsrow[tid] * lsrow[tid];
        v3 = lrow[tid] * alph[tid];
    }
    const double l2 = tail_block_sum(v1, red);
    const double ls2 = tail_block_sum(v2, red);
    const double la = tail_block_sum(v3, red);
    const double d2 = Ccol[j] - l2;
    const bool finite = isfinite(d2) && isfinite(Ccol[j]);
    if (!(finite && d2 > pivot_tol * Ccol[j] && d2 > 0.0)) {
        if (tid == 0) {
            ls->stop = 1;
            ls->dropped += 1;
            if (!finite) ls->nonfinite += 1;
        }
        return;
    }
    const double dj = sqrt(d2);
    const double inv_d = 1.0 / dj;
    const double ds = sqrt(fmax(Qcol[j] - ls2, 1e-300));
    const double aj = (c_j - la) * inv_d;
    // 3. new row j of L^{-1} (and of LS^{-1}): -(l^T L^{-1}) / d, 1 / d
    {
        double acc = 0.0, accs = 0.0;
        if (row < j) {
            for (int k = row + sub; k < j; k += tpr) {
                acc = __builtin_fma(lrow[k], Linv[(size_t)k * ld + row], acc);
                accs = __builtin_fma(lsrow[k], LSinv[(size_t)k * ld + row], accs);
            }
        }
        acc = group_sum(acc, tpr);
        accs = group_sum(accs, tpr);
        if (row < j && sub == 0) {
            const double v = -acc * inv_d, vs = -accs / ds;
            Linv[(size_t)j * ld + row] = v;
            LinvT[(size_t)row * ld + j] = v;
            LSinv[(size_t)j * ld + row] = vs;
            LSinvT[(size_t)row * ld + j] = vs;
            L[(size_t)j * ld + row] = lrow[row];
            nrow[row] = v;
        }
    }
    if (tid == 0) {
        Linv[(size_t)j * ld + j] = inv_d;
        LinvT[(size_t)j * ld + j] = inv_d;
        LSinv[(size_t)j * ld + j] = 1.0 / ds;
        LSinvT[(size_t)j * ld + j] = 1.0 / ds;
        L[(size_t)j * ld + j] = dj;
        nrow[j] = inv_d;
        alph[j] = aj;
        alpha[j] = aj;
        ls->logdet_c += 2.0 * log(dj);
        ls->logdet_s += 2.0 * log(ds);
        ls->alpha2 += aj * aj;
        ls->i_eff = J;
        ls->loglik = -0.5 * ((double)J * 1.8378770664093453 + ls->logdet_c - ls->logdet_s +
                             ls->alpha2);
    }
    __syncthreads();
    // 4. beta = L^{-T} alpha over the kept actions (row j of L^{-1} from LDS)
    {
        const int tprb = std::min(64, TAIL_THREADS / pow2_at_least(J));
        const int rb = tid / tprb, sb = tid % tprb;
        double acc = 0.0;
        if (rb < J) {
            for (int k = rb + sb; k < j; k += tprb)
                acc = __builtin_fma(Linv[(size_t)k * ld + rb], alph[k], acc);
        }
        acc = group_sum(acc, tprb);
        if (rb < J && sb == 0) beta[rb] = acc + nrow[rb] * alph[j];
    }
}

void launch_tail(const double* gpart, int nblk, const double* ttv, const ObsDims& d, int j,
                 double noise_var, double resid_tol, double pivot_tol, double* Linv,
                 double* LinvT, double* L, double* LSinv, double* LSinvT, double* alpha,
                 double* beta, LoopState* ls, hipStream_t st) {
    hipLaunchKernelGGL(k_tail, dim3(1), dim3(TAIL_THREADS), 0, st, gpart, nblk, ttv, d, j,
                       noise_var, resid_tol, pivot_tol, Linv, LinvT, L, LSinv, LSinvT, alpha,
                       beta, ls);
}

// ---------------------------------------------------------------------- next_action
// CG policy: s_{j+1} = r0 - Ghat S beta = r0 - (U - Mo T + noise_var S) beta (the
// residual after j+1 actions), stored unnormalised in S[:, j+1].  The low-rank part is
// kept per row as V = Mo T: this launch adds column j, V[:, j] = Mo t_j, from the same
// pass over the rows of Mo that also forms the per-block partial sums of Mo^T s_{j+1}
// (finished by the next sym_tiles launch).  One wave per row, lanes over the action and
// factor columns, NA_ROWS rows per wave loaded NA_BATCH at a time.
constexpr int NA_ROWS = 16;
constexpr int NA_BATCH = 4;

__global__ __launch_bounds__(256) void k_next_action(const float* __restrict__ U,
                                                     const float* __restrict__ Mo,
                                                     const float* __restrict__ r0,
                                                     float* __restrict__ S,
                                                     float* __restrict__ V,
                                                     const double* __restrict__ beta,
                                                     const float* __restrict__ T,
                                                     float noise_var, ObsDims d, int j,
                                                     float* __restrict__ mpart,
                                                     const LoopState* __restrict__ ls) {
    if (ls->stop) return;
    __shared__ float red[4][1024];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int p0 = (blockIdx.x * 4 + w) * NA_ROWS;
    float bl[4], tj[16], acc[16];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int l = lane + 64 * v;
        bl[v] = (l <= j) ? (float)beta[l] : 0.0f;
    }
    const float* tcol = T + (size_t)j * d.ldmo;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int c = lane + 64 * u;
        tj[u] = (c < d.rank) ? tcol[c] : 0.0f;
        acc[u] = 0.0f;
    }
    const int rows = min(NA_ROWS, d.m - p0);
    for (int rr = 0; rr < rows; rr += NA_BATCH) {
        float mo[NA_BATCH][16], part[NA_BATCH], vj[NA_BATCH];
#pragma unroll
        for (int b = 0; b < NA_BATCH; ++b) {
            const int p = p0 + min(rr + b, rows - 1);
            const float* Mrow = Mo + (size_t)p * d.ldmo;
            vj[b] = 0.0f;
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int c = lane + 64 * u;
                mo[b][u] = (c < d.rank) ? Mrow[c] : 0.0f;
                vj[b] = __builtin_fmaf(mo[b][u], tj[u], vj[b]);
            }
            const float* Urow = U + (size_t)p * d.imax;
            const float* Srow = S + (size_t)p * d.imax;
            const float* Vrow = V + (size_t)p * d.imax;
            part[b] = 0.0f;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int l = lane + 64 * v;
                if (l < j)
                    part[b] -= (__builtin_fmaf(noise_var, Srow[l], Urow[l]) - Vrow[l]) * bl[v];
                else if (l == j)
                    part[b] -= __builtin_fmaf(noise_var, Srow[l], Urow[l]) * bl[v];
            }
        }
#pragma unroll
        for (int b = 0; b < NA_BATCH; ++b) {
            const bool live = rr + b < rows;
            const int p = p0 + rr + b;
            const float vpj = wave_sum(vj[b]);
            // the V[:, j] term of row p, held by the lane that owns column j
            const int lj = j & 63, vj_slot = j >> 6;
            float extra = 0.0f;
#pragma unroll
            for (int v = 0; v < 4; ++v)
                if (v == vj_slot && lane == lj) extra = vpj * bl[v];
            const float rho = live ? r0[p] + wave_sum(part[b] + extra) : 0.0f;
            if (live && lane == 0) {
                S[(size_t)p * d.imax + j + 1] = rho;
                V[(size_t)p * d.imax + j] = vpj;
            }
#pragma unroll
            for (int u = 0; u < 16; ++u) acc[u] = __builtin_fmaf(mo[b][u], rho, acc[u]);
        }
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

void launch_next_action(const float* U, const float* Mo, const float* r0, float* S, float* V,
                        const double* beta, const float* T, float noise_var,
                        const ObsDims& d, int j, float* mpart, const LoopState* ls,
                        hipStream_t st, int* nblk_out) {
    const int blocks = (d.m + 4 * NA_ROWS - 1) / (4 * NA_ROWS);
    *nblk_out = blocks;
    hipLaunchKernelGGL(k_next_action, dim3(blocks), dim3(256), 0, st, U, Mo, r0, S, V, beta, T,
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
