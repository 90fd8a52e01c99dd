// Observation-space part of the CAKF update on gfx950: gather, the action loop and the
// Cholesky form of the projected update.
//
// The update conditions the predictive belief on S^T y (Sec. 3.1) with the projected
// Gram matrix C = S^T Ghat S, Ghat = H P^- H^T + Lambda = sigma_f2 K(Xo, Xo)
// - Mo Mo^T + noise_var I, Mo = H M^-.  Actions are chosen one at a time (the iterative
// update of App. B); with the CG policy the next action is the current residual
// (Sec. 3.3).  The kernels keep, per action s_l,
//     u_l = sigma_f2 K(Xo, Xo) s_l   (U, m x i),   t_l = Mo^T s_l   (T, r x i),
// so that entry (l, j) of C is  g_l - t_l^T t_j + noise_var s_l^T s_j  with
// g_l = s_l^T u_j = u_l^T s_j (K is symmetric).  The residual after j+1 actions is
// r0 - (U - Mo T + noise_var S) beta with beta = C^{-1} S^T r0.  C is factorised
// incrementally in FP64 (C = L L^T with L^{-1} kept explicitly); the Ghat-orthonormal
// directions of the iterative update are S L^{-T} (App. B), which is what the block
// product consumes.
//
// Column j of C needs u_j only in its diagonal entry: every other entry, u_l^T s_j and
// s_l^T s_j for l < j, and s_j^T s_j, r0^T s_j, is formed from rows that are already
// loaded when s_j is produced.  One iteration j launches:
//   sym_tiles    u_j tile sums; its first blocks finish the column products of s_j
//                (and, CG, t_j = Mo^T s_j) from the previous launch's block partials;
//                through arrival counters, the last tile of each row block forms those
//                rows of u_j (and of s_j^T u_j), the last spare block the triangular
//                products of the Cholesky step, and the last arrival of all the FP64
//                Cholesky step itself: column j of C, row j of L^{-1}, alpha and beta
//                (sym_tiles.hip);
//   next_action  CG: s_{j+1} = the residual, V[:, j] = Mo t_j, partial sums of
//                Mo^T s_{j+1}; both policies: the column products of s_{j+1}.
// The block-residual policy forms the Gram columns of a round of actions in one product
// instead and takes the round's Cholesky steps in one launch of the tail kernel.
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
// partial[b, c] = sum over the CS_ROWS rows of block b of A[p, c] * x[p] (cols <= 1024):
// each wave takes CS_ROWS / 4 rows, four rows' loads in flight at a time, in row order.
constexpr int CS_ROWS = 64;

__global__ __launch_bounds__(256) void k_colsum_partial(const float* __restrict__ A, int lda,
                                                        int rows, int cols,
                                                        const float* __restrict__ x,
                                                        int ldx,
                                                        float* __restrict__ partial,
                                                        int ldp) {
    __shared__ float red[4][1024];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int p0 = blockIdx.x * CS_ROWS + w * (CS_ROWS / 4);
    float acc[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) acc[u] = 0.0f;
    const int pend = min(rows, p0 + CS_ROWS / 4);
    for (int pb = p0; pb < pend; pb += 4) {
        float v[4][16], xv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int p = pb + q;
            const bool ok = p < pend;
            const float* row = A + (size_t)min(p, pend - 1) * lda;
            xv[q] = ok ? x[(size_t)min(p, pend - 1) * ldx] : 0.0f;
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int c = lane + 64 * u;
                v[q][u] = (ok && c < cols) ? row[c] : 0.0f;
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int u = 0; u < 16; ++u) acc[u] = __builtin_fmaf(v[q][u], xv[q], acc[u]);
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
    const int blocks = (rows + CS_ROWS - 1) / CS_ROWS;
    *nblk_out = blocks;
    hipLaunchKernelGGL(k_colsum_partial, dim3(blocks), dim3(256), 0, st, A, lda, rows, cols,
                       x, ldx, partial, ldp);
}

// out[c * ldo] = sum over b < nblk of partial[b, c] (FP64, fixed order): 32 columns per
// block, 8 row groups of 32 threads with 8 loads in flight each, groups added in order.
__global__ __launch_bounds__(256) void k_colsum_final(const float* __restrict__ partial,
                                                      int ldp, int nblk, int cols,
                                                      float* __restrict__ out, int ldo) {
    __shared__ double red[8][33];
    const int cl = threadIdx.x & 31, grp = threadIdx.x >> 5;
    const int c = blockIdx.x * 32 + cl;
    double a[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] = 0.0;
    if (c < cols) {
        int b = grp;
        for (; b + 56 < nblk; b += 64) {
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = partial[(size_t)(b + 8 * u) * ldp + c];
#pragma unroll
            for (int u = 0; u < 8; ++u) a[u] += (double)v[u];
        }
        for (; b < nblk; b += 8) a[0] += (double)partial[(size_t)b * ldp + c];
    }
    red[grp][cl] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    __syncthreads();
    if (grp == 0 && c < cols) {
        double t = 0.0;
#pragma unroll
        for (int g = 0; g < 8; ++g) t += red[g][cl];
        out[(size_t)c * ldo] = (float)t;
    }
}

void launch_colsum_final(const float* partial, int ldp, int nblk, int cols, float* out,
                         int ldo, hipStream_t st) {
    if (cols <= 0) return;
    hipLaunchKernelGGL(k_colsum_final, dim3((cols + 31) / 32), dim3(256), 0, st, partial, ldp,
                       nblk, cols, out, ldo);
}

// ------------------------------------------------------------------------- form_u
// u_j[p] = sigma_f2 * (sum over the nb slots of the tile partial sums, FP64), stored in
// U[:, j], and per-block partial sums (FP64) of s_j^T u_j, FU_ROWS rows per block.
constexpr int FU_ROWS = 64;
constexpr int FU_LOADS = 8;

__global__ __launch_bounds__(256) void k_form_u(const float* __restrict__ part,
                                                const float* __restrict__ S,
                                                float* __restrict__ U, ObsDims d, int j,
                                                double sigma_f2, double* __restrict__ fupart,
                                                const LoopState* __restrict__ ls) {
    if (ls->stop) return;
    // thread (quad, grp) sums rows 4 quad .. 4 quad + 3 of the block over the slots grp,
    // grp + 16, ... with 16-byte loads, FU_LOADS slots in flight at a time; the 16 slot
    // groups are then combined in a fixed order
    __shared__ double ured[16][FU_ROWS + 1];
    const int tid = threadIdx.x;
    const int nb = d.mp / SYM_TILE;
    const int quad = tid & 15, grp = tid >> 4;
    const int p0 = blockIdx.x * FU_ROWS + 4 * quad;    // < mp (mp a multiple of 128)
    const int prow = blockIdx.x * FU_ROWS + tid;
    const float sj = (tid < FU_ROWS && prow < d.m) ? S[(size_t)prow * d.imax + j] : 0.0f;
    double a4[4] = {0.0, 0.0, 0.0, 0.0};
    for (int s0 = grp; s0 < nb; s0 += 16 * FU_LOADS) {
        float4 v[FU_LOADS];
#pragma unroll
        for (int u = 0; u < FU_LOADS; ++u) {
            const int sl = s0 + 16 * u;
            v[u] = sl < nb ? *reinterpret_cast<const float4*>(part + (size_t)sl * d.mp + p0)
                           : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        }
#pragma unroll
        for (int u = 0; u < FU_LOADS; ++u) {
            a4[0] += (double)v[u].x;
            a4[1] += (double)v[u].y;
            a4[2] += (double)v[u].z;
            a4[3] += (double)v[u].w;
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) ured[grp][4 * quad + r] = a4[r];
    __syncthreads();
    if (tid < FU_ROWS) {
        double t = 0.0;
#pragma unroll
        for (int g = 0; g < 16; ++g) t += ured[g][tid];
        double prod = 0.0;
        if (prow < d.m) {
            const float uf = (float)(sigma_f2 * t);
            U[(size_t)prow * d.imax + j] = uf;
            prod = (double)sj * (double)uf;
        }
        prod = wave_sum(prod);
        if (tid == 0) fupart[blockIdx.x] = prod;
    }
}

void launch_form_u(const float* part, const float* S, float* U, const ObsDims& d, int j,
                   double sigma_f2, double* fupart, const LoopState* ls, hipStream_t st,
                   int* nblk_out) {
    const int rowblk = (d.m + FU_ROWS - 1) / FU_ROWS;
    *nblk_out = rowblk;
    hipLaunchKernelGGL(k_form_u, dim3(rowblk), dim3(256), 0, st, part, S, U, d, j, sigma_f2,
                       fupart, ls);
}

// ---------------------------------------------------------------- Cholesky step, O(j)
// The rest of the Cholesky step of action j once u_j and the triangular products are
// formed: C_jj = s_j^T u_j + noise_var s_j^T s_j - t_j^T t_j, the pivot
// d^2 = C_jj - |lrow|^2 (breakdown stops the loop and drops the action),
// alpha_j = (r0^T s_j - lrow^T alpha) / d, row j of L (lrow, d) and of L^{-1}
// (-nrow / d, 1 / d), beta_j = beta_{j-1} + alpha_j (row j of L^{-1}); the
// residual-tolerance stop.  Every wave of every block that takes it computes the same
// scalars (the same loads, sums in a fixed order).
struct TailScalars {
    double inv_d, aj, dj;
    int outcome;      // 0: keep action j; 1: tolerance stop; 2: breakdown; 3: non-finite
};

// The step's loads (issued before anything that depends on them, so that a caller can put
// them in flight together with its own): this lane's share of s_j^T u_j and the scalars.
struct TailIn {
    double fu, qjj, c_j, l2, la, tt, q00;
};

__device__ __forceinline__ TailIn tail_load(const TailArgs& ta, int j, const LoopState* ls) {
    const int lane = threadIdx.x & 63, ld = ta.imax;
    TailIn in;
    in.fu = 0.0;
    for (int b = lane; b < ta.nfu; b += 64) in.fu += ta.fupart[b];
    in.qjj = ta.colvec[2 * j];
    in.c_j = ta.colvec[2 * j + 1];
    in.l2 = ta.tri[tri_scal(ld)];
    in.la = ta.tri[tri_scal(ld) + 1];
    in.tt = ta.tri[tri_scal(ld) + 2];
    in.q00 = j > 0 ? ls->q00 : 0.0;
    return in;
}

__device__ TailScalars tail_finish(const TailArgs& ta, int j, const TailIn& in) {
    const double fu = wave_sum(in.fu);
    const double qjj = in.qjj;
    const double cjj = fu - in.tt + ta.noise_var * qjj;
    TailScalars r{0.0, 0.0, 0.0, 0};
    if (j > 0 && ta.resid_tol > 0.0 && qjj <= ta.resid_tol * ta.resid_tol * in.q00) {
        r.outcome = 1;
        return r;
    }
    const double d2 = cjj - in.l2;
    const bool finite = isfinite(d2) && isfinite(cjj);
    if (!(finite && d2 > ta.pivot_tol * cjj && d2 > 0.0)) {
        r.outcome = finite ? 2 : 3;
        return r;
    }
    r.dj = sqrt(d2);
    r.inv_d = 1.0 / r.dj;
    r.aj = (in.c_j - in.la) * r.inv_d;
    return r;
}

__device__ TailScalars tail_scalars(const TailArgs& ta, int j, const LoopState* ls) {
    return tail_finish(ta, j, tail_load(ta, j, ls));
}

// entry l <= j of row j of L^{-1} and of beta_j
__device__ __forceinline__ double tail_linv(const TailArgs& ta, const TailScalars& ts, int j,
                                            int l) {
    return l < j ? -ta.tri[tri_nrow(ta.imax) + l] * ts.inv_d : ts.inv_d;
}

__device__ __forceinline__ double tail_beta(const TailArgs& ta, const TailScalars& ts, int j,
                                            int l) {
    const double prev = l < j ? ta.beta_in[l] : 0.0;
    return __builtin_fma(ts.aj, tail_linv(ta, ts, j, l), prev);
}

// The stores of the step (one workgroup of at least j + 1 threads, the same scalars in
// every thread): the loop state, and for a kept action row j of L, L^{-1}, S^T S,
// alpha_j and beta_j (into beta_out).
__device__ void tail_store(const TailArgs& ta, const TailScalars& ts, int j, LoopState* ls) {
    const int tid = threadIdx.x, ld = ta.imax, J = j + 1;
    if (ts.outcome != 0) {
        if (tid == 0) {
            ls->stop = 1;
            if (ts.outcome >= 2) ls->dropped += 1;
            if (ts.outcome == 3) ls->nonfinite += 1;
        }
        return;
    }
    if (tid < J) {
        const double v = tail_linv(ta, ts, j, tid);
        ta.Linv[(size_t)j * ld + tid] = v;
        ta.LinvT[(size_t)tid * ld + j] = v;
        ta.L[(size_t)j * ld + tid] = tid < j ? ta.tri[tri_lrow(ld) + tid] : ts.dj;
        ta.SS[(size_t)j * ld + tid] = ta.colvec[j + tid];
        ta.beta_out[tid] = tail_beta(ta, ts, j, tid);
    }
    if (tid == 0) {
        if (j == 0) ls->q00 = ta.colvec[0];
        ta.alpha[j] = ts.aj;
        ls->logdet_c += 2.0 * log(ts.dj);
        ls->alpha2 += ts.aj * ts.aj;
        ls->i_eff = J;
    }
}

// After the loop (one workgroup of TF_THREADS threads): the step of the last action when
// the loop ran to it (no next action follows), the final beta into beta_final when the
// last kept action left it in the other buffer, then log det S^T S over the kept actions
// (right-looking Cholesky of the leading block, FP64; pivots floored at 1e-300 as in the
// block-policy step) and the projected log-likelihood term
//     -1/2 (i log 2 pi + log det S^T Ghat S - log det S^T S + |L^{-1} S^T r0|^2).
// The factorisation runs in LDS up to TF_LDS_N actions (row stride TF_LDS_N + 1 doubles,
// so that a column's entries fall in different banks), column by column: thread (r, c)
// of a 32 x 32 grid updates the trailing entries (i, l) with i = r, l = c (mod 32).  Above
// TF_LDS_N it runs in work (imax^2 doubles, global memory), blocked by panels of TF_NB
// columns: wave 0 factors the panel's diagonal block in an LDS copy (lane i owns row i;
// the lanes only wait on one another within the wave), each row below solves for its
// panel entries against that block (one thread per row), and the trailing lower triangle
// takes the panel's outer products on the same 32 x 32 grid: three block barriers and
// one pass over the trailing matrix per panel instead of per column (1.69 -> 1.29 ms at
// 256 actions; in LDS, where each pass is cheap, the column form is faster: 0.13 against
// 0.23 ms at 128).  The pivots are kept and their logs summed at the end.
constexpr int TF_LDS_N = 128;
constexpr int TF_THREADS = 1024;
constexpr int TF_NB = 32;

// Cholesky pivots of the lower triangle A (row stride la) of order ie, in place, by the
// 32 x 32 thread grid.  In LDS: the thread's entries row by row (the loads' latency is
// short).
__device__ void tf_cholesky_lds(double* A, int la, int ie, double* piv) {
    const int tid = threadIdx.x, r = tid >> 5, c = tid & 31;
    for (int k = 0; k < ie; ++k) {
        const double dk = sqrt(fmax(A[k * la + k], 1e-300));
        const double rk = 1.0 / dk;
        if (tid == 0) piv[k] = dk;
        // this thread's first trailing row and column (i = r, l = c modulo 32)
        const int i0 = k + 1 + ((r - (k + 1)) & 31), l0 = k + 1 + ((c - (k + 1)) & 31);
        for (int i = k + 1 + tid; i < ie; i += TF_THREADS) A[i * la + k] *= rk;
        __syncthreads();
        for (int i = i0; i < ie; i += 32) {
            const double aik = A[i * la + k];
            for (int l = l0; l <= i; l += 32) A[i * la + l] -= aik * A[l * la + k];
        }
        __syncthreads();
    }
}

// orders the LDS accesses of one wave's lanes around it (no block barrier)
__device__ __forceinline__ void tf_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Cholesky pivots of the lower triangle A (global memory, row stride la) of order ie, in
// place.  D: LDS scratch of TF_NB x (TF_NB + 1) doubles, dinv: TF_NB doubles.
__device__ __forceinline__ void tf_cholesky_blocked(double* A, int la, int ie, double* piv,
                                                    double (*D)[TF_NB + 1], double* dinv) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int r = tid >> 5, c = tid & 31;
    for (int kb = 0; kb < ie; kb += TF_NB) {
        const int nb = min(TF_NB, ie - kb);
        // 1. the diagonal block, factored by wave 0 in D
        for (int e = tid; e < nb * nb; e += TF_THREADS) {
            const int i = e / nb, l = e % nb;
            if (l <= i) D[i][l] = A[(size_t)(kb + i) * la + kb + l];
        }
        __syncthreads();
        if (w == 0) {
            for (int k = 0; k < nb; ++k) {
                const double dk = sqrt(fmax(D[k][k], 1e-300));
                const double rk = 1.0 / dk;
                double lik = 0.0;
                if (lane > k && lane < nb) {
                    lik = D[lane][k] * rk;
                    D[lane][k] = lik;
                }
                if (lane == 0) {
                    piv[kb + k] = dk;
                    dinv[k] = rk;
                }
                tf_wave_sync();
                if (lane > k && lane < nb)
                    for (int l = k + 1; l <= lane; ++l) D[lane][l] -= lik * D[l][k];
                tf_wave_sync();
            }
        }
        __syncthreads();
        // 2. the panel rows below: x = a L^{-T} by forward substitution against D, each
        //    entry written back before the next one reads it
        for (int i = kb + nb + tid; i < ie; i += TF_THREADS) {
            double* ai = A + (size_t)i * la + kb;
            for (int q = 0; q < nb; ++q) {
                double sq = ai[q];
                for (int p = 0; p < q; ++p) sq = __builtin_fma(-ai[p], D[q][p], sq);
                ai[q] = sq * dinv[q];
            }
        }
        __syncthreads();
        // 3. the trailing lower triangle minus the panel's outer products
        const int t0 = kb + nb;
        const int i0 = t0 + ((r - t0) & 31), l0 = t0 + ((c - t0) & 31);
        for (int i = i0; i < ie; i += 32)
            for (int l = l0; l <= i; l += 32) {
                const double* ai = A + (size_t)i * la + kb;
                const double* al = A + (size_t)l * la + kb;
                double s = 0.0;
#pragma unroll 8
                for (int q = 0; q < nb; ++q) s = __builtin_fma(ai[q], al[q], s);
                A[(size_t)i * la + l] -= s;
            }
        __syncthreads();
    }
}

__global__ __launch_bounds__(TF_THREADS) void k_tail_final(TailArgs ta, int j,
                                                           const double* __restrict__ beta_odd,
                                                           double* __restrict__ beta_final,
                                                           double* __restrict__ work,
                                                           LoopState* __restrict__ ls) {
    __shared__ double Al[TF_LDS_N * (TF_LDS_N + 1)];
    __shared__ double piv[256];
    __shared__ double Dl[TF_NB][TF_NB + 1], dinv[TF_NB];
    __shared__ double red[TF_THREADS / 64];
    const int tid = threadIdx.x, ld = ta.imax;
    if (!ls->stop) {
        const TailScalars ts = tail_scalars(ta, j, ls);
        tail_store(ta, ts, j, ls);
    }
    __syncthreads();
    const int ie = ls->i_eff;
    if (ie > 0 && ((ie - 1) & 1))
        for (int l = tid; l < ie; l += TF_THREADS) beta_final[l] = beta_odd[l];
    const int r = tid >> 5, c = tid & 31;
    if (ie <= TF_LDS_N) {
        constexpr int la = TF_LDS_N + 1;
        for (int i = r; i < ie; i += 32)
            for (int l = c; l <= i; l += 32) Al[i * la + l] = ta.SS[(size_t)i * ld + l];
        __syncthreads();
        tf_cholesky_lds(Al, la, ie, piv);
    } else {
        for (int i = r; i < ie; i += 32)
            for (int l = c; l <= i; l += 32) work[i * ld + l] = ta.SS[(size_t)i * ld + l];
        __syncthreads();
        tf_cholesky_blocked(work, ld, ie, piv, Dl, dinv);
    }
    double lg = 0.0;
    for (int t = tid; t < ie; t += TF_THREADS) lg += 2.0 * log(piv[t]);
    lg = wave_sum(lg);
    if ((tid & 63) == 0) red[tid >> 6] = lg;
    __syncthreads();
    if (tid == 0) {
        double logdet = 0.0;
        for (int w = 0; w < TF_THREADS / 64; ++w) logdet += red[w];
        ls->logdet_s = logdet;
        ls->loglik = -0.5 * ((double)ie * 1.8378770664093453 + ls->logdet_c - logdet +
                             ls->alpha2);
    }
}

void launch_tail_final(const TailArgs& ta, int j, const double* beta_odd, double* beta_final,
                       double* work, LoopState* ls, hipStream_t st) {
    hipLaunchKernelGGL(k_tail_final, dim3(1), dim3(TF_THREADS), 0, st, ta, j, beta_odd,
                       beta_final, work, ls);
}

// --------------------------------------------------------------------------- tail
// The Cholesky steps of a block-policy round: one block of 1024 threads, FP64, actions
// jfirst .. jfirst + nj - 1 in turn.  Takes column j of C = S^T Ghat S from the round's
// Gram product, extends its Cholesky factor C = L L^T (L^{-1} kept explicitly,
// row-major Linv and column-major LinvT so that every triangular product reads
// coalesced), alpha = L^{-1} S^T r0, beta = L^{-T} alpha (updated in place: the new row
// of L^{-1} times alpha_j is all that changes), the Cholesky factor of S^T S (log det
// only) and the log-likelihood term.  Each triangular product splits a row over tpr
// threads, issues its loads TAIL_BATCH at a time and combines the threads with lane
// shuffles.  Stops the loop on breakdown (pivot) or residual tolerance.
constexpr int TAIL_THREADS = 1024;
constexpr int TAIL_BATCH = 8;      // loads in flight per thread in the triangular products

// sums of three values over the block (same result in every thread)
__device__ __forceinline__ void block_sum3(double& a, double& b, double& c, double (*red)[16]) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_sum(c);
    __syncthreads();
    if (lane == 0) {
        red[0][w] = a;
        red[1][w] = b;
        red[2][w] = c;
    }
    __syncthreads();
    a = b = c = 0.0;
#pragma unroll 2
    for (int k = 0; k < TAIL_THREADS / 64; ++k) {
        a += red[0][k];
        b += red[1][k];
        c += red[2][k];
    }
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

__global__ __launch_bounds__(TAIL_THREADS) void k_tail(ObsDims d, int jfirst, double noise_var,
                                                       double resid_tol, double pivot_tol,
                                                       double* __restrict__ Linv,
                                                       double* __restrict__ LinvT,
                                                       double* __restrict__ L,
                                                       double* __restrict__ LSinv,
                                                       double* __restrict__ LSinvT,
                                                       double* __restrict__ alpha,
                                                       double* __restrict__ beta,
                                                       LoopState* __restrict__ ls,
                                                       TailDirect td, int nj) {
    __shared__ double Ccol[256], Qcol[256], lrow[256], lsrow[256], nrow[256], alph[256];
    __shared__ double red[3][TAIL_THREADS / 64];
    const int tid = threadIdx.x;
    if (ls->stop) return;
    const int ld = d.imax;
    // every exit below is taken by the whole workgroup and ends the loop with the stop
    // flag set
    const double* gdir = td.G;
    for (int g = 0; g < nj; ++g) {
        const int j = jfirst + g;
        const int J = j + 1;
        // 1. column j: s_l^T u_j, s_l^T s_j, s_l^T v_j and s_j^T r0 from columns uc + g,
        //    sc + g, vc + g and rc of td.G
        double cj = 0.0, unused0 = 0.0, unused1 = 0.0;
        if (tid == 0) cj = gdir[(size_t)j * td.ld + td.rc];
        double gcol = 0.0, qcol = 0.0, al = 0.0;
        if (tid < J) {
            const double* row = gdir + (size_t)tid * td.ld;
            qcol = row[td.sc + g];
            gcol = row[td.uc + g] + noise_var * qcol - row[td.vc + g];
            al = tid < j ? alpha[tid] : 0.0;
        }
        block_sum3(cj, unused0, unused1, red);
        const double c_j = cj;
        if (tid < J) {
            Ccol[tid] = gcol;
            Qcol[tid] = qcol;
            alph[tid] = al;
        }
        __syncthreads();
        if (j == 0) {
            if (tid == 0) ls->q00 = Qcol[0];
        } else if (resid_tol > 0.0 && Qcol[j] <= resid_tol * resid_tol * ls->q00) {
            if (tid == 0) ls->stop = 1;
            return;
        }
        // rows of the triangular products: j rows, tpr threads per row
        const int tpr = j > 0 ? std::min(64, TAIL_THREADS / pow2_at_least(j)) : 1;
        const int row = tid / tpr, sub = tid % tpr;
        // 2. l = L^{-1} C[0:j, j] and ls = LS^{-1} Q[0:j, j]
        {
            double lk = 0.0, lsk = 0.0;
            if (row < j) {
                for (int p0 = sub; p0 <= row; p0 += TAIL_BATCH * tpr) {
                    double a[TAIL_BATCH], b[TAIL_BATCH];
    #pragma unroll
                    for (int u = 0; u < TAIL_BATCH; ++u) {
                        const int p = p0 + u * tpr;
                        a[u] = p <= row ? LinvT[(size_t)p * ld + row] : 0.0;
                        b[u] = p <= row ? LSinvT[(size_t)p * ld + row] : 0.0;
                    }
    #pragma unroll
                    for (int u = 0; u < TAIL_BATCH; ++u) {
                        const int p = p0 + u * tpr;
                        if (p <= row) {
                            lk = __builtin_fma(a[u], Ccol[p], lk);
                            lsk = __builtin_fma(b[u], Qcol[p], lsk);
                        }
                    }
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
        double l2 = 0.0, ls2 = 0.0, la = 0.0;
        if (tid < j) {
            l2 = lrow[tid] * lrow[tid];
            ls2 = lsrow[tid] * lsrow[tid];
            la = lrow[tid] * alph[tid];
        }
        block_sum3(l2, ls2, la, red);
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
                for (int k0 = row + sub; k0 < j; k0 += TAIL_BATCH * tpr) {
                    double a[TAIL_BATCH], b[TAIL_BATCH];
    #pragma unroll
                    for (int u = 0; u < TAIL_BATCH; ++u) {
                        const int k = k0 + u * tpr;
                        a[u] = k < j ? Linv[(size_t)k * ld + row] : 0.0;
                        b[u] = k < j ? LSinv[(size_t)k * ld + row] : 0.0;
                    }
    #pragma unroll
                    for (int u = 0; u < TAIL_BATCH; ++u) {
                        const int k = k0 + u * tpr;
                        if (k < j) {
                            acc = __builtin_fma(lrow[k], a[u], acc);
                            accs = __builtin_fma(lsrow[k], b[u], accs);
                        }
                    }
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
            alpha[j] = aj;
            ls->logdet_c += 2.0 * log(dj);
            ls->logdet_s += 2.0 * log(ds);
            ls->alpha2 += aj * aj;
            ls->i_eff = J;
            ls->loglik = -0.5 * ((double)J * 1.8378770664093453 + ls->logdet_c - ls->logdet_s +
                                 ls->alpha2);
        }
        __syncthreads();
        // 4. beta = L^{-T} alpha: the previous beta plus alpha_j times row j of L^{-1}
        if (tid < J) {
            const double prev = tid < j ? beta[tid] : 0.0;
            beta[tid] = __builtin_fma(aj, nrow[tid], prev);
        }
        // the next action reads this one's rows of L^{-1}, alpha_j and beta
        __syncthreads();
    }
}

void launch_tail(const ObsDims& d, int jfirst, double noise_var, double resid_tol,
                 double pivot_tol, double* Linv, double* LinvT, double* L, double* LSinv,
                 double* LSinvT, double* alpha, double* beta, LoopState* ls, hipStream_t st,
                 const TailDirect& td, int nj) {
    hipLaunchKernelGGL(k_tail, dim3(1), dim3(TAIL_THREADS), 0, st, d, jfirst, noise_var,
                       resid_tol, pivot_tol, Linv, LinvT, L, LSinv, LSinvT, alpha, beta, ls, td,
                       nj);
}

// ---------------------------------------------------------------------- next_action
// Produces (RESID: the CG policy) or reads (given actions, and s_0) action s_jt, and forms
// the per-block partial sums (FP64) of its column products
//     u_l^T s_jt (l < jt),  s_l^T s_jt (l <= jt),  r0^T s_jt,
// laid out as [u^T s (jt) | s^T s (jt + 1) | r0^T s] in cpart[block * gs + pos].
// With tail (jt >= 1) the launch first finishes the Cholesky step of action j = jt - 1
// (tail_scalars in every wave, tail_store in block 0), and stops on its outcome.
// RESID, with j = jt - 1: s_jt = r0 - Ghat S beta = r0 - (U - Mo T + noise_var S) beta,
// the residual after jt actions, stored unnormalised in S[:, jt]; V[:, j] = Mo t_j (the
// low-rank part kept per row, V = Mo T) and the per-block partial sums of Mo^T s_jt
// (finished by the next sym_tiles launch) come from the same pass over the rows of Mo.
// Each wave takes RW rows with all their loads in flight at once; lanes own CPL
// consecutive factor columns and the action columns lane + 64 v, v < LPL.
template <bool RESID, int CPL, int LPL, int RW>
__global__ __launch_bounds__(256) void k_next_action(const float* __restrict__ U,
                                                     const float* __restrict__ Mo,
                                                     const float* __restrict__ r0,
                                                     float* __restrict__ S,
                                                     float* __restrict__ V,
                                                     const float* __restrict__ T,
                                                     float noise_var, ObsDims d, int jt,
                                                     int mopart,
                                                     float* __restrict__ mpart,
                                                     double* __restrict__ cpart, int gs,
                                                     LoopState* __restrict__ ls, TailArgs ta,
                                                     int tail) {
    if (ls->stop) return;
    __shared__ float mred[4][64 * CPL];
    __shared__ double gred[4][64 * LPL], qred[4][64 * LPL];
    __shared__ double sred[2][4];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int p0 = (blockIdx.x * 4 + w) * RW;
    const int j = jt - 1;
    // the O(j) rest of the Cholesky step of action j (every block; block 0 stores it)
    // lowrank: this pass also forms the partial sums of Mo^T s_jt (mopart; the CG residual
    // needs Mo t_j as well)
    const bool lowrank = (RESID || mopart) && d.rank > 0;
    float tj[CPL], acc[CPL], bl[LPL];
    double g[LPL], q[LPL];
#pragma unroll
    for (int k = 0; k < CPL; ++k) {
        const int c = lane * CPL + k;
        tj[k] = (RESID && lowrank && c < d.rank) ? T[(size_t)j * d.ldmo + c] : 0.0f;
        acc[k] = 0.0f;
    }
#pragma unroll
    for (int v = 0; v < LPL; ++v) {
        g[v] = 0.0;
        q[v] = 0.0;
    }
    // loads of all RW rows (issued before the Cholesky step's loads and its exit, which
    // the row loads do not depend on)
    float mo[RW][CPL], uu[RW][LPL], sv[RW][LPL], vv[RW][LPL], r0v[RW], sr[RW];
#pragma unroll
    for (int b = 0; b < RW; ++b) {
        const int p = min(p0 + b, d.m - 1);
        r0v[b] = r0[p];
        sr[b] = RESID ? 0.0f : S[(size_t)p * d.imax + jt];
#pragma unroll
        for (int v = 0; v < LPL; ++v) {
            const int l = lane + 64 * v;
            uu[b][v] = l < jt ? U[(size_t)p * d.imax + l] : 0.0f;
            sv[b][v] = l < jt ? S[(size_t)p * d.imax + l] : 0.0f;
            vv[b][v] = (RESID && l < j) ? V[(size_t)p * d.imax + l] : 0.0f;
        }
#pragma unroll
        for (int k4 = 0; k4 < CPL / 4; ++k4) {
            const int c = lane * CPL + 4 * k4;
            float4 x = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if (lowrank && c < d.ldmo)
                x = *reinterpret_cast<const float4*>(Mo + (size_t)p * d.ldmo + c);
            mo[b][4 * k4] = x.x;
            mo[b][4 * k4 + 1] = x.y;
            mo[b][4 * k4 + 2] = x.z;
            mo[b][4 * k4 + 3] = x.w;
        }
    }
    // the Cholesky step's inputs and, for the residual, beta_{j-1} and row j of the
    // triangular products, loaded with the rows above
    TailIn tin{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    double bprev[LPL], nrw[LPL];
    if (tail) tin = tail_load(ta, j, ls);
#pragma unroll
    for (int v = 0; v < LPL; ++v) {
        const int l = lane + 64 * v;
        const bool in = RESID && tail && l < j;
        bprev[v] = in ? ta.beta_in[l] : 0.0;
        nrw[v] = in ? ta.tri[tri_nrow(ta.imax) + l] : 0.0;
    }
    TailScalars ts{0.0, 0.0, 0.0, 0};
    if (tail) {
        ts = tail_finish(ta, j, tin);
        if (blockIdx.x == 0) tail_store(ta, ts, j, ls);
        if (ts.outcome != 0) return;
    }
    // beta_j = beta_{j-1} + alpha_j (row j of L^{-1}), as in tail_beta
#pragma unroll
    for (int v = 0; v < LPL; ++v) {
        const int l = lane + 64 * v;
        const double lv = l < j ? -nrw[v] * ts.inv_d : ts.inv_d;
        bl[v] = (RESID && l <= j) ? (float)__builtin_fma(ts.aj, lv, bprev[v]) : 0.0f;
    }
    const float bj = RESID ? (float)(ts.aj * ts.inv_d) : 0.0f;
    float rho[RW];
    if constexpr (RESID) {
        float dotp[RW], part[RW];
#pragma unroll
        for (int b = 0; b < RW; ++b) {
            dotp[b] = 0.0f;
#pragma unroll
            for (int k = 0; k < CPL; ++k) dotp[b] = __builtin_fmaf(mo[b][k], tj[k], dotp[b]);
            part[b] = 0.0f;
#pragma unroll
            for (int v = 0; v < LPL; ++v)
                part[b] = __builtin_fmaf(vv[b][v] - __builtin_fmaf(noise_var, sv[b][v], uu[b][v]),
                                         bl[v], part[b]);
        }
#pragma unroll
        for (int b = 0; b < RW; ++b) {
            const float vs = wave_sum(dotp[b]);
            const float ps = wave_sum(part[b]);
            const bool live = p0 + b < d.m;
            rho[b] = live ? r0v[b] + ps + bj * vs : 0.0f;
            if (live && lane == b) {
                S[(size_t)(p0 + b) * d.imax + jt] = rho[b];
                V[(size_t)(p0 + b) * d.imax + j] = vs;
            }
        }
    } else {
#pragma unroll
        for (int b = 0; b < RW; ++b) rho[b] = p0 + b < d.m ? sr[b] : 0.0f;
    }
    double qq = 0.0, cc = 0.0;
#pragma unroll
    for (int b = 0; b < RW; ++b) {
        const double rd = rho[b];
        if (lowrank) {
#pragma unroll
            for (int k = 0; k < CPL; ++k) acc[k] = __builtin_fmaf(mo[b][k], rho[b], acc[k]);
        }
#pragma unroll
        for (int v = 0; v < LPL; ++v) {
            g[v] = __builtin_fma((double)uu[b][v], rd, g[v]);
            q[v] = __builtin_fma((double)sv[b][v], rd, q[v]);
        }
        qq = __builtin_fma(rd, rd, qq);
        cc = __builtin_fma((double)r0v[b], rd, cc);
    }
    // block sums over the 4 waves, fixed order
    if (lowrank) {
#pragma unroll
        for (int k = 0; k < CPL; ++k) mred[w][lane * CPL + k] = acc[k];
    }
#pragma unroll
    for (int v = 0; v < LPL; ++v) {
        gred[w][lane + 64 * v] = g[v];
        qred[w][lane + 64 * v] = q[v];
    }
    if (lane == 0) {
        sred[0][w] = qq;
        sred[1][w] = cc;
    }
    __syncthreads();
    if (lowrank) {
        for (int c = threadIdx.x; c < d.rank; c += 256)
            mpart[(size_t)blockIdx.x * d.ldmo + c] = (mred[0][c] + mred[1][c]) + (mred[2][c] + mred[3][c]);
    }
    double* out = cpart + (size_t)blockIdx.x * gs;
    for (int pos = threadIdx.x; pos < 2 * jt + 2; pos += 256) {
        double v;
        if (pos < jt) {
            v = (gred[0][pos] + gred[1][pos]) + (gred[2][pos] + gred[3][pos]);
        } else if (pos < 2 * jt) {
            const int l = pos - jt;
            v = (qred[0][l] + qred[1][l]) + (qred[2][l] + qred[3][l]);
        } else {
            const int k = pos - 2 * jt;
            v = (sred[k][0] + sred[k][1]) + (sred[k][2] + sred[k][3]);
        }
        out[pos] = v;
    }
}

template <bool RESID, int CPL, int LPL>
static void launch_na(int blocks, const float* U, const float* Mo, const float* r0, float* S,
                      float* V, const float* T, float noise_var, const ObsDims& d, int jt,
                      int mopart, float* mpart, double* cpart, int gs, LoopState* ls,
                      const TailArgs& ta, int tail, hipStream_t st) {
    constexpr int RW = next_action_rows_per_wave(CPL, LPL);
    hipLaunchKernelGGL((k_next_action<RESID, CPL, LPL, RW>), dim3(blocks), dim3(256), 0, st, U,
                       Mo, r0, S, V, T, noise_var, d, jt, mopart, mpart, cpart, gs, ls, ta,
                       tail);
}

template <bool RESID, int CPL>
static void launch_na_l(int lpl, int blocks, const float* U, const float* Mo, const float* r0,
                        float* S, float* V, const float* T, float noise_var, const ObsDims& d,
                        int jt, int mopart, float* mpart, double* cpart, int gs, LoopState* ls,
                        const TailArgs& ta, int tail, hipStream_t st) {
    if (lpl == 1)
        launch_na<RESID, CPL, 1>(blocks, U, Mo, r0, S, V, T, noise_var, d, jt, mopart, mpart,
                                 cpart, gs, ls, ta, tail, st);
    else if (lpl == 2)
        launch_na<RESID, CPL, 2>(blocks, U, Mo, r0, S, V, T, noise_var, d, jt, mopart, mpart,
                                 cpart, gs, ls, ta, tail, st);
    else
        launch_na<RESID, CPL, 4>(blocks, U, Mo, r0, S, V, T, noise_var, d, jt, mopart, mpart,
                                 cpart, gs, ls, ta, tail, st);
}

template <bool RESID>
static void launch_na_c(int cpl, int lpl, int blocks, const float* U, const float* Mo,
                        const float* r0, float* S, float* V, const float* T, float noise_var,
                        const ObsDims& d, int jt, int mopart, float* mpart, double* cpart,
                        int gs, LoopState* ls, const TailArgs& ta, int tail, hipStream_t st) {
    if (cpl == 4)
        launch_na_l<RESID, 4>(lpl, blocks, U, Mo, r0, S, V, T, noise_var, d, jt, mopart, mpart,
                              cpart, gs, ls, ta, tail, st);
    else if (cpl == 8)
        launch_na_l<RESID, 8>(lpl, blocks, U, Mo, r0, S, V, T, noise_var, d, jt, mopart, mpart,
                              cpart, gs, ls, ta, tail, st);
    else
        launch_na_l<RESID, 16>(lpl, blocks, U, Mo, r0, S, V, T, noise_var, d, jt, mopart, mpart,
                               cpart, gs, ls, ta, tail, st);
}

void launch_next_action(int resid, int mopart, const float* U, const float* Mo,
                        const float* r0, float* S, float* V, const float* T, float noise_var,
                        const ObsDims& d, int jt, float* mpart, double* cpart, int gs,
                        LoopState* ls, const TailArgs* ta, hipStream_t st, int* nblk_out) {
    // the lanes cover the factor columns whenever Mo is read (CG residual or mopart)
    const bool reads_mo = (resid || mopart) && d.rank > 0;
    const int lpl = next_action_lpl(d.imax);
    const int cpl = reads_mo ? next_action_cpl(d.ldmo) : 4;
    const int blocks = next_action_blocks(d.m, cpl, lpl);
    *nblk_out = blocks;
    const TailArgs none{};
    const int tail = ta != nullptr ? 1 : 0;
    if (resid)
        launch_na_c<true>(cpl, lpl, blocks, U, Mo, r0, S, V, T, noise_var, d, jt, 1, mpart,
                          cpart, gs, ls, tail ? *ta : none, tail, st);
    else
        launch_na_c<false>(cpl, lpl, blocks, U, Mo, r0, S, V, T, noise_var, d, jt,
                           mopart ? 1 : 0, mpart, cpart, gs, ls, tail ? *ta : none, tail, st);
}

// ------------------------------------------------------------------ block-residual policy
// Start of a round of bt actions at action index j0: the residual
// rho = r0 - (U - Mo T + noise_var S) beta over the j0 actions taken so far, split over bt
// contiguous observation groups: S[p, j0 + g] = rho[p] if p lies in
// [floor(g m / bt), floor((g + 1) m / bt)), else 0.  One wave per observation row.
__global__ __launch_bounds__(256) void k_block_residual(const float* __restrict__ U,
                                                        const float* __restrict__ V,
                                                        float* __restrict__ S,
                                                        const float* __restrict__ r0,
                                                        const double* __restrict__ beta,
                                                        float noise_var, ObsDims d, int j0,
                                                        int bt, const LoopState* __restrict__ ls) {
    if (ls->stop) return;
    const int lane = threadIdx.x & 63;
    const int p = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (p >= d.mp) return;
    float rho = 0.0f;
    if (p < d.m) {
        float part = 0.0f;
        for (int l = lane; l < j0; l += 64) {
            const size_t o = (size_t)p * d.imax + l;
            const float lr = d.rank > 0 ? V[o] : 0.0f;
            part = __builtin_fmaf(lr - __builtin_fmaf(noise_var, S[o], U[o]), (float)beta[l], part);
        }
        rho = r0[p] + wave_sum(part);
    }
    for (int g = lane; g < bt; g += 64) {
        const int g0 = (int)((long long)g * d.m / bt), g1 = (int)((long long)(g + 1) * d.m / bt);
        S[(size_t)p * d.imax + j0 + g] = (p >= g0 && p < g1) ? rho : 0.0f;
    }
}

void launch_block_residual(const float* U, const float* V, float* S, const float* r0,
                           const double* beta, float noise_var, const ObsDims& d, int j0, int bt,
                           const LoopState* ls, hipStream_t st) {
    hipLaunchKernelGGL(k_block_residual, dim3((d.mp + 3) / 4), dim3(256), 0, st, U, V, S, r0,
                       beta, noise_var, d, j0, bt, ls);
}

// Skinny products of a round, C (P x Q) = sum over the observation rows p of
// A[p, c] B[p, q] with few columns and m rows: the rows are cut into slabs of ATB_RB, each
// workgroup forms one slab's products for 64 columns of A and 64 of B (FP32 operands
// staged in LDS, accumulation in Acc), and a second kernel sums the slabs in a fixed
// order.  Two instances:
//   Gram:  A = S[:, 0:P] (all actions so far), B = [U_r | S_r | V_r | r0] over the round's
//          columns r (FP64 accumulation; C[l, q] then gives s_l^T Ghat s_g =
//          s_l^T u_g + noise_var s_l^T s_g - s_l^T v_g, s_l^T s_g and s_l^T r0);
//   Mo^T:  A = Mo (P = rank), B = S_r (FP32 accumulation), C = T[:, r].
constexpr int ATB_RB = 64;    // rows per slab (one LDS chunk)
constexpr int ATB_PC = 64;    // columns of A per workgroup
constexpr int ATB_LD = ATB_RB * ATB_PC / 256;   // elements of A each thread loads

struct RowsA {
    const float* A;
    int ld;
    __device__ float operator()(int p, int c) const { return A[(size_t)p * ld + c]; }
};
struct RowsA64 {
    const double* A;
    int ld;
    __device__ double operator()(int p, int c) const { return A[(size_t)p * ld + c]; }
};
struct RoundGramB {
    const float *U, *S, *V, *r0;
    int ld, j0, bt, lowrank;
    __device__ float operator()(int p, int q) const {
        const size_t o = (size_t)p * ld + j0;
        if (q < bt) return U[o + q];
        if (q < 2 * bt) return S[o + q - bt];
        if (q < 3 * bt) return lowrank ? V[o + q - 2 * bt] : 0.0f;
        return r0[p];
    }
};

__device__ __forceinline__ float fma_acc(float a, float b, float c) {
    return __builtin_fmaf(a, b, c);
}
__device__ __forceinline__ double fma_acc(double a, double b, double c) {
    return __builtin_fma(a, b, c);
}

// QC columns of B per workgroup (16, 32 or 64; the smallest that holds Q, else 64 and
// more workgroups along z): thread (cl, qg) accumulates C[c0 + cl, q0 + qg + 4 k].  The
// operands are staged in the type the loaders return (FP32, or FP64 for FP64 sources).
template <typename Acc, int QC, class LA, class LB>
__global__ __launch_bounds__(256) void k_atb_partial(LA la, LB lb, int m, int P, int Q,
                                                     Acc* __restrict__ part) {
    using TA = decltype(la(0, 0));
    using TB = decltype(lb(0, 0));
    constexpr int BLD = ATB_RB * QC / 256;      // elements of B each thread loads
    __shared__ TA As[ATB_RB][ATB_PC + 1];
    __shared__ TB Bs[ATB_RB][QC + 1];
    const int tid = threadIdx.x;
    const int c0 = blockIdx.y * ATB_PC, q0 = blockIdx.z * QC;
    const int p0 = blockIdx.x * ATB_RB;
    const int cl = tid & 63, qg = tid >> 6;
    // all of the slab's loads are issued before any of them is used
    TA av[ATB_LD];
    TB bv[BLD];
#pragma unroll
    for (int u = 0; u < ATB_LD; ++u) {
        const int p = p0 + u * 4 + qg;
        av[u] = (p < m && c0 + cl < P) ? la(p, c0 + cl) : TA(0);
    }
#pragma unroll
    for (int u = 0; u < BLD; ++u) {
        const int e = u * 256 + tid, r = e / QC, q = e % QC, p = p0 + r;
        bv[u] = (p < m && q0 + q < Q) ? lb(p, q0 + q) : TB(0);
    }
#pragma unroll
    for (int u = 0; u < ATB_LD; ++u) As[u * 4 + qg][cl] = av[u];
#pragma unroll
    for (int u = 0; u < BLD; ++u) {
        const int e = u * 256 + tid;
        Bs[e / QC][e % QC] = bv[u];
    }
    __syncthreads();
    Acc acc[QC / 4];
#pragma unroll
    for (int k = 0; k < QC / 4; ++k) acc[k] = Acc(0);
#pragma unroll 4
    for (int r = 0; r < ATB_RB; ++r) {
        const Acc a = (Acc)As[r][cl];
#pragma unroll
        for (int k = 0; k < QC / 4; ++k) acc[k] = fma_acc(a, (Acc)Bs[r][qg + 4 * k], acc[k]);
    }
    const int c = c0 + cl;
    if (c < P) {
        Acc* out = part + ((size_t)blockIdx.x * P + c) * Q;
#pragma unroll
        for (int k = 0; k < QC / 4; ++k) {
            const int q = q0 + qg + 4 * k;
            if (q < Q) out[q] = acc[k];
        }
    }
}

template <typename Acc, class LA, class LB>
static void launch_atb_partial(LA la, LB lb, int m, int P, int Q, Acc* part, hipStream_t st) {
    const int nslab = (m + ATB_RB - 1) / ATB_RB, pc = (P + ATB_PC - 1) / ATB_PC;
    if (Q <= 16)
        hipLaunchKernelGGL((k_atb_partial<Acc, 16, LA, LB>), dim3(nslab, pc, 1), dim3(256), 0,
                           st, la, lb, m, P, Q, part);
    else if (Q <= 32)
        hipLaunchKernelGGL((k_atb_partial<Acc, 32, LA, LB>), dim3(nslab, pc, 1), dim3(256), 0,
                           st, la, lb, m, P, Q, part);
    else
        hipLaunchKernelGGL((k_atb_partial<Acc, 64, LA, LB>), dim3(nslab, pc, (Q + 63) / 64),
                           dim3(256), 0, st, la, lb, m, P, Q, part);
}

// C[c, q] = sum over the slabs of part, written to G[c * ldg + q] (FP64) or, for the
// Mo^T instance, to T[(j0 + q) * ldt + c] (FP32, column-major).  A workgroup takes 64
// consecutive outputs; wave w sums the w-th quarter of the slabs (8 loads in flight, added
// in slab order) and the four quarters are added in order: a fixed summation order.
template <typename Acc, bool TOUT>
__global__ __launch_bounds__(256) void k_atb_reduce(const Acc* __restrict__ part, int nslab,
                                                    int P, int Q, double* __restrict__ G,
                                                    int ldg, float* __restrict__ T, int ldt,
                                                    int j0) {
    __shared__ Acc quarter[4][64];
    const int total = P * Q;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int e = blockIdx.x * 64 + lane;
    const int per = (nslab + 3) / 4;
    const int b0 = w * per, b1 = min(nslab, b0 + per);
    Acc v = Acc(0);
    if (e < total) {
        for (int b = b0; b < b1; b += 8) {
            Acc x[8];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                x[u] = b + u < b1 ? part[(size_t)(b + u) * total + e] : Acc(0);
#pragma unroll
            for (int u = 0; u < 8; ++u) v += x[u];
        }
    }
    quarter[w][lane] = v;
    __syncthreads();
    if (w == 0 && e < total) {
        const Acc sum = ((quarter[0][lane] + quarter[1][lane]) + quarter[2][lane]) +
                        quarter[3][lane];
        const int c = e / Q, q = e % Q;
        if constexpr (TOUT) T[(size_t)(j0 + q) * ldt + c] = (float)sum;
        else G[(size_t)c * ldg + q] = (double)sum;
    }
}

size_t round_products_elems(int m, int P, int Q) {
    return (size_t)((m + ATB_RB - 1) / ATB_RB) * P * Q;
}

void launch_round_gram(const float* U, const float* V, const float* S, const float* r0,
                       const ObsDims& d, int j0, int bt, double* part, double* G, int ldg,
                       hipStream_t st) {
    const int P = j0 + bt, Q = 3 * bt + 1;
    const int nslab = (d.m + ATB_RB - 1) / ATB_RB;
    launch_atb_partial<double>(RowsA{S, d.imax},
                               RoundGramB{U, S, V, r0, d.imax, j0, bt, d.rank > 0 ? 1 : 0}, d.m,
                               P, Q, part, st);
    const int blocks = (P * Q + 63) / 64;
    hipLaunchKernelGGL((k_atb_reduce<double, false>), dim3(blocks), dim3(256), 0, st, part,
                       nslab, P, Q, G, ldg, nullptr, 0, 0);
}

size_t atb64_part_elems(int m, int P, int Q) {
    return (size_t)((m + ATB_RB - 1) / ATB_RB) * P * Q;
}

void launch_atb64(const double* A, int lda, const double* B, int ldb, int m, int P, int Q,
                  double* part, double* G, int ldg, hipStream_t st) {
    if (m <= 0 || P <= 0 || Q <= 0) return;
    const int nslab = (m + ATB_RB - 1) / ATB_RB;
    launch_atb_partial<double>(RowsA64{A, lda}, RowsA64{B, ldb}, m, P, Q, part, st);
    const int blocks = (P * Q + 63) / 64;
    hipLaunchKernelGGL((k_atb_reduce<double, false>), dim3(blocks), dim3(256), 0, st, part,
                       nslab, P, Q, G, ldg, nullptr, 0, 0);
}

void launch_round_mot(const float* Mo, const float* S, const ObsDims& d, int j0, int bt,
                      float* part, float* T, hipStream_t st) {
    const int P = d.rank, Q = bt;
    const int nslab = (d.m + ATB_RB - 1) / ATB_RB;
    launch_atb_partial<float>(RowsA{Mo, d.ldmo}, RowsA{S + j0, d.imax}, d.m, P, Q, part, st);
    const int blocks = (P * Q + 63) / 64;
    hipLaunchKernelGGL((k_atb_reduce<float, true>), dim3(blocks), dim3(256), 0, st, part, nslab,
                       P, Q, nullptr, 0, T, d.ldmo, j0);
}

// ----------------------------------------------------------------------- build_block
// B = [S L^{-T} | S beta | 0] (mp x bp, row-major) for the block product, plus the
// optional record copies (m rows).  FP64 accumulation in the order l = 0, 1, ...  A block
// stages BB_ROWS rows of S in LDS; thread c computes column c of them, so each load of
// (L^{-1})[c][l] = LinvT[l][c] (consecutive threads, consecutive words) feeds BB_ROWS
// products.
constexpr int BB_ROWS = 16;
constexpr int BB_MAXI = 256;      // max_actions

__global__ __launch_bounds__(256) void k_build_block(const float* __restrict__ S,
                                                     const double* __restrict__ LinvT,
                                                     const double* __restrict__ beta,
                                                     ObsDims d, float* __restrict__ B,
                                                     int ldb, int bp,
                                                     float* __restrict__ rec_W,
                                                     float* __restrict__ rec_w,
                                                     float* __restrict__ rec_S,
                                                     const LoopState* __restrict__ ls) {
    __shared__ float Ss[BB_ROWS][BB_MAXI];
    const int kept = ls->i_eff;
    const int p0 = blockIdx.x * BB_ROWS;
    const int imax = d.imax;
    for (int e = threadIdx.x; e < BB_ROWS * imax; e += blockDim.x) {
        const int r = e / imax, l = e % imax, p = p0 + r;
        Ss[r][l] = p < d.m ? S[(size_t)p * imax + l] : 0.0f;
    }
    __syncthreads();
    for (int c = threadIdx.x; c < bp; c += blockDim.x) {
        double acc[BB_ROWS];
#pragma unroll
        for (int r = 0; r < BB_ROWS; ++r) acc[r] = 0.0;
        if (c < imax) {
            for (int l = 0; l <= c; ++l) {
                const double lv = LinvT[(size_t)l * imax + c];
#pragma unroll
                for (int r = 0; r < BB_ROWS; ++r) acc[r] = __builtin_fma((double)Ss[r][l], lv, acc[r]);
            }
        } else if (c == imax) {
            for (int l = 0; l < imax; ++l) {
                const double bv = beta[l];
#pragma unroll
                for (int r = 0; r < BB_ROWS; ++r) acc[r] = __builtin_fma((double)Ss[r][l], bv, acc[r]);
            }
        }
#pragma unroll
        for (int r = 0; r < BB_ROWS; ++r) {
            const int p = p0 + r;
            if (p >= d.mp) break;
            const float v = (float)acc[r];
            B[(size_t)p * ldb + c] = v;
            if (p < d.m) {
                if (c < imax) {
                    if (rec_W) rec_W[(size_t)p * imax + c] = v;
                    if (rec_S) rec_S[(size_t)p * imax + c] = c < kept ? Ss[r][c] : 0.0f;
                } else if (c == imax && rec_w) {
                    rec_w[p] = v;
                }
            }
        }
    }
}

void launch_build_block(const float* S, const double* LinvT, const double* beta,
                        const ObsDims& d, float* B, int ldb, int bp, float* rec_W,
                        float* rec_w, float* rec_S, const LoopState* ls, hipStream_t st) {
    const int blocks = (d.mp + BB_ROWS - 1) / BB_ROWS;
    hipLaunchKernelGGL(k_build_block, dim3(blocks), dim3(256), 0, st, S, LinvT, beta, d, B, ldb,
                       bp, rec_W, rec_w, rec_S, ls);
}

// Record outputs that live in the loop state.
__global__ void k_finish_record(const LoopState* __restrict__ ls, const double* __restrict__ L,
                                const double* __restrict__ Linv, int imax,
                                double* __restrict__ rec_chol, double* __restrict__ rec_chol_inv,
                                double* __restrict__ rec_loglik, int* __restrict__ rec_n) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    for (int e = tid; e < imax * imax; e += gridDim.x * blockDim.x) {
        if (rec_chol) rec_chol[e] = L[e];
        if (rec_chol_inv) rec_chol_inv[e] = Linv[e];
    }
    if (tid == 0) {
        if (rec_loglik) *rec_loglik = ls->loglik;
        if (rec_n) *rec_n = ls->i_eff;
    }
}

void launch_finish_record(const LoopState* ls, const double* L, const double* Linv, int imax,
                          double* rec_chol, double* rec_chol_inv, double* rec_loglik, int* rec_n,
                          hipStream_t st) {
    hipLaunchKernelGGL(k_finish_record, dim3(64), dim3(256), 0, st, ls, L, Linv, imax, rec_chol,
                       rec_chol_inv, rec_loglik, rec_n);
}

}  // namespace cakf
