// The symmetric kernel matvec of the CAKF action loop on gfx950: the tile sums of
// u_j = sigma_f2 K(Xo, Xo) s_j over the upper triangle of 128 x 128 tiles (each off-diagonal
// tile serves its row block and, transposed, its column block), with the reductions of the
// previous launch's column products in spare blocks, the last of which (through an arrival
// counter) takes the triangular products of the action's Cholesky step while the tiles
// run.  Part of the observation-space loop described in obs_loop.hip.
#include <hip/hip_ext.h>

#include "cakf_common.h"
#include "launchers.h"

namespace cakf {

// ----------------------------------------------------------- symmetric kernel matvec
// out[pos] = sum over rows b < nrows of in[b * ld + pos] for the CR_POS positions pos0 +
// [0, CR_POS) below npos: CR_GRP row groups with 8 independent FP64 accumulators each,
// combined in a fixed order.  The result is valid in the threads of group 0.
constexpr int CR_POS = 32, CR_GRP = 8;

template <typename Tin>
__device__ __forceinline__ double column_reduce(const Tin* __restrict__ in, size_t ld,
                                                int nrows, int npos, int pos0,
                                                double (*red)[CR_POS + 1]) {
    const int pl = threadIdx.x % CR_POS, grp = threadIdx.x / CR_POS;
    const int pos = pos0 + pl;
    double a[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] = 0.0;
    if (pos < npos) {
        int b = grp;
        for (; b + 7 * CR_GRP < nrows; b += 8 * CR_GRP) {
            Tin v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = in[(size_t)(b + u * CR_GRP) * ld + pos];
#pragma unroll
            for (int u = 0; u < 8; ++u) a[u] += (double)v[u];
        }
        for (; b < nrows; b += CR_GRP) a[0] += (double)in[(size_t)b * ld + pos];
    }
    red[grp][pl] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    __syncthreads();
    double s = 0.0;
    if (grp == 0) {
#pragma unroll
        for (int g = 0; g < CR_GRP; ++g) s += red[g][pl];
    }
    return s;
}

// The first n_t + n_c blocks of a sym_tiles launch: (n_t) t_j = Mo^T s_j into column j
// of T (column-major, T[l * ldmo + c]) from next_action's per-block partial sums, and the
// block's share of t_l^T t_j (l <= j, FP64, over its CR_POS factor rows) into
// ttpart[block * imax + l]; (n_c) the column products of s_j into colvec, laid out as
// [u_l^T s_j (l < j) | s_l^T s_j (l <= j) | r0^T s_j].
__device__ __forceinline__ void sym_extra_block(const ObsDims& d, int j,
                                                const float* __restrict__ mpart, int nmpart,
                                                int n_t, float* __restrict__ T,
                                                const double* __restrict__ cpart, int ncpart,
                                                int gs, double* __restrict__ colvec,
                                                double* __restrict__ ttpart,
                                                double (*cred)[CR_POS + 1], float* tchunk) {
    const int tid = threadIdx.x;
    if ((int)blockIdx.x < n_t) {
        const int pos0 = blockIdx.x * CR_POS;
        const double v = column_reduce(mpart, (size_t)d.ldmo, nmpart, d.rank, pos0, cred);
        if (tid < CR_POS) {
            const bool in = pos0 + tid < d.rank;
            if (in) T[(size_t)j * d.ldmo + pos0 + tid] = (float)v;
            tchunk[tid] = in ? (float)v : 0.0f;
        }
        __syncthreads();
        // thread l: its column's CR_POS rows of this chunk (16-byte loads; rows at or
        // beyond the rank are masked); column j is the chunk itself
        const int l = tid;
        if (l <= j) {
            double acc = 0.0;
            if (l == j) {
#pragma unroll
                for (int c = 0; c < CR_POS; ++c)
                    acc = __builtin_fma((double)tchunk[c], (double)tchunk[c], acc);
            } else {
                const float4* col =
                    reinterpret_cast<const float4*>(T + (size_t)l * d.ldmo + pos0);
                float4 x[CR_POS / 4];
#pragma unroll
                for (int k = 0; k < CR_POS / 4; ++k) x[k] = col[k];
#pragma unroll
                for (int k = 0; k < CR_POS / 4; ++k) {
                    const int c = 4 * k;
                    const bool i0 = pos0 + c < d.rank, i1 = pos0 + c + 1 < d.rank;
                    const bool i2 = pos0 + c + 2 < d.rank, i3 = pos0 + c + 3 < d.rank;
                    acc = __builtin_fma(i0 ? (double)x[k].x : 0.0, (double)tchunk[c], acc);
                    acc = __builtin_fma(i1 ? (double)x[k].y : 0.0, (double)tchunk[c + 1], acc);
                    acc = __builtin_fma(i2 ? (double)x[k].z : 0.0, (double)tchunk[c + 2], acc);
                    acc = __builtin_fma(i3 ? (double)x[k].w : 0.0, (double)tchunk[c + 3], acc);
                }
            }
            ttpart[(size_t)blockIdx.x * d.imax + l] = acc;
        }
    } else {
        const int pos0 = (blockIdx.x - n_t) * CR_POS;
        const int npos = 2 * j + 2;
        const double v = column_reduce(cpart, (size_t)gs, ncpart, npos, pos0, cred);
        if ((int)threadIdx.x < CR_POS && pos0 + (int)threadIdx.x < npos)
            colvec[pos0 + threadIdx.x] = v;
    }
}

// ------------------------------------------------------------------ rest of the step
// Arrival at a counter whose n-th arrival within a launch continues with work that needs
// the writes of every earlier arrival.  The block barrier orders the workgroup's writes
// before thread 0's agent-scope release; the last arrival acquires with an agent-scope
// fence and resets the counter to zero for the next launch.  No workgroup waits for
// another.  Returns the same flag in every thread.  (A release makes the XCD's L2 write
// back: worth it for the few spare blocks of a launch, far too costly for every tile.)
__device__ __forceinline__ bool arrive(unsigned* ctr, unsigned n, int* flag) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const unsigned old =
            __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int last = old + 1u == n;
        if (last) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            __hip_atomic_store(ctr, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        *flag = last;
    }
    __syncthreads();
    return *flag != 0;
}

// sum over the workgroup (256 threads), the same in every thread; red: 4 doubles of LDS
__device__ __forceinline__ double block_sum(double v, double* red) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    const double s = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
    return s;
}

// y[t] = sum over p of A[t lda + p] x[p] for t < j, over p <= t (LOWER) or t <= p < j:
// A row-major FP64, x and y in LDS, j < 64 QN.  Rows t and j - 1 - t hold j + 1 entries
// together, so a wave reads them as one vector of 64 QN lanes (coalesced, none masked off
// by the triangle) and splits the sum at the boundary; a wave takes RB such pairs at a
// time with their loads in flight (RB QN doubles per lane: the code shares the tile
// kernel's register budget).
template <bool LOWER, int QN, int RB>
__device__ void tri_matvec_q(const double* __restrict__ A, int lda, const double* x, int j,
                             double* y) {
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int npair = (j + 1) / 2;
#pragma unroll 1
    for (int q0 = RB * w; q0 < npair; q0 += 4 * RB) {
        double s1[RB], s2[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const int t = q0 + r, t2 = j - 1 - t;
            // entry e < len1 belongs to row t, the rest to row t2 (none when t == t2)
            const int len1 = LOWER ? t + 1 : j - t;
            double a1 = 0.0, a2 = 0.0;
#pragma unroll
            for (int q = 0; q < QN; ++q) {
                const int e = lane + 64 * q;
                const bool valid = t < npair && e <= j;
                const bool first = e < len1;
                const int row = first ? t : t2;
                const int p = LOWER ? (first ? e : e - len1) : (first ? t + e : e - 1);
                if (valid && (first || t2 != t)) {
                    const double v = A[(size_t)row * lda + p] * x[p];
                    if (first)
                        a1 += v;
                    else
                        a2 += v;
                }
            }
            s1[r] = a1;
            s2[r] = a2;
        }
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const int t = q0 + r, t2 = j - 1 - t;
            const double v1 = wave_sum(s1[r]);
            const double v2 = wave_sum(s2[r]);
            if (lane == 0 && t < npair) {
                y[t] = v1;
                if (t2 != t) y[t2] = v2;
            }
        }
    }
}

template <bool LOWER>
__device__ void tri_matvec(const double* __restrict__ A, int lda, const double* x, int j,
                           double* y) {
    if (j < 64)
        tri_matvec_q<LOWER, 1, 8>(A, lda, x, j, y);
    else if (j < 128)
        tri_matvec_q<LOWER, 2, 4>(A, lda, x, j, y);
    else
        tri_matvec_q<LOWER, 4, 2>(A, lda, x, j, y);
}

// The triangular products of the Cholesky step of action j (one workgroup, after every
// spare block has written T[:, j] and colvec), into ta.tri (offsets tri_*):
//   c_l = u_l^T s_j + noise_var s_l^T s_j - t_l^T t_j (l < j),  tt = t_j^T t_j,
//   lrow = L^{-1} c,  nrow = lrow^T L^{-1},  l2 = |lrow|^2,  la = lrow^T alpha.
// sm: 1028 doubles.
__device__ void tri_products(const ObsDims& d, int j, int n_t, const float* __restrict__ T,
                             const double* __restrict__ colvec, const TriArgs& ta,
                             double* sm) {
    double* cv = sm;
    double* tt = sm + 256;
    double* lr = sm + 512;
    double* nr = sm + 768;
    double* red = sm + 1024;
    const int tid = threadIdx.x;
    const int ld = d.imax;
    double* tri = ta.tri;
    // t_l^T t_j for l <= j: the sum of the n_t spare blocks' shares (fixed order); at
    // j = 0 (column 0 of T formed before the loop) the one product directly
    if (d.rank > 0 && n_t > 0) {
        if (tid <= j) {
            double a = 0.0;
            for (int b = 0; b < n_t; ++b) a += ta.ttpart[(size_t)b * ld + tid];
            tt[tid] = a;
        }
    } else if (d.rank > 0 && j == 0) {
        const float* t0 = T;
        double a = 0.0;
        for (int c = tid; c < d.rank; c += 256) a = __builtin_fma((double)t0[c], (double)t0[c], a);
        a = block_sum(a, red);
        if (tid == 0) tt[0] = a;
    } else if (tid <= j) {
        tt[tid] = 0.0;
    }
    __syncthreads();
    if (tid < j) cv[tid] = colvec[tid] + ta.noise_var * colvec[j + tid] - tt[tid];
    __syncthreads();
    tri_matvec<true>(ta.Linv, ld, cv, j, lr);
    __syncthreads();
    tri_matvec<false>(ta.LinvT, ld, lr, j, nr);
    __syncthreads();
    double l2 = 0.0, la = 0.0;
    if (tid < j) {
        l2 = lr[tid] * lr[tid];
        la = lr[tid] * ta.alpha[tid];
        tri[tri_lrow(ld) + tid] = lr[tid];
        tri[tri_nrow(ld) + tid] = nr[tid];
    }
    l2 = block_sum(l2, red);
    la = block_sum(la, red);
    if (tid == 0) {
        tri[tri_scal(ld) + 0] = l2;
        tri[tri_scal(ld) + 1] = la;
        tri[tri_scal(ld) + 2] = tt[j];
    }
}

// The spare blocks of a launch: the reductions, then (the last spare block to finish)
// the triangular products of the Cholesky step of action j.
__device__ void step_spare(const ObsDims& d, int j, const float* mpart, int nmpart, int n_t,
                           float* T, const double* cpart, int ncpart, int gs, int n_c,
                           double* colvec, const TriArgs& ta, double* sm, int* flags) {
    sym_extra_block(d, j, mpart, nmpart, n_t, T, cpart, ncpart, gs, colvec, ta.ttpart,
                    reinterpret_cast<double(*)[CR_POS + 1]>(sm),
                    reinterpret_cast<float*>(sm + CR_GRP * (CR_POS + 1)));
    if (!arrive(ta.ctr, (unsigned)(n_t + n_c), flags)) return;
    // the block shares its SIMDs with tile waves: issue its instructions first
    __builtin_amdgcn_s_setprio(3);
    tri_products(d, j, n_t, T, colvec, ta, sm);
}

// u_j = K(Xo, Xo) s_j over the upper triangle of SYM_TILE x SYM_TILE tiles.  Tile (P, Q),
// P <= Q, adds its row sums K_PQ s_Q to slot Q of block P and (P < Q) its column sums
// K_PQ^T s_P to slot P of block Q; every (slot, block) pair is written exactly once, and
// the reduction in form_u is deterministic.  Each thread evaluates an 8 x 8 set of
// entries.  The first n_t + n_c blocks instead finish, from next_action's per-block
// partial sums: (n_t) t_j = Mo^T s_j into column j of T (column-major, T[l * ldmo + c]);
// (n_c) the column products of s_j into colvec, laid out as
// [u_l^T s_j (l < j) | s_l^T s_j (l <= j) | r0^T s_j]; the last of them then takes the
// triangular products (step_spare).
template <int NU2, int DIST>
__global__ __launch_bounds__(256) void k_sym_tiles(const float4* __restrict__ Xo,
                                                   const float* __restrict__ S, ObsDims d,
                                                   int j, float* __restrict__ part,
                                                   const float* __restrict__ mpart,
                                                   int nmpart, int n_t,
                                                   float* __restrict__ T,
                                                   const double* __restrict__ cpart,
                                                   int ncpart, int gs, int n_c,
                                                   double* __restrict__ colvec,
                                                   const LoopState* __restrict__ ls,
                                                   TriArgs ta) {
    __shared__ __align__(16) float red[2][16][SYM_TILE + 1];   // also FP64 scratch
    __shared__ int flags[1];
    double* sm = reinterpret_cast<double*>(&red[0][0][0]);
    if (ls->stop) return;
    const int n_extra = n_t + n_c;
    if ((int)blockIdx.x < n_extra) {
        step_spare(d, j, mpart, nmpart, n_t, T, cpart, ncpart, gs, n_c, colvec, ta, sm, flags);
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

// Euclidean Matern-3/2 and -5/2 form of k_sym_tiles: the squared scaled distance of a
// 16 x 16 sub-tile is one v_mfma_f32_16x16x4f32, D = A B + C with
// A[i] = (-2 c x_i, -2 c y_i, -2 c z_i, 1), B[:, j] = (c x_j, c y_j, c z_j, c^2 |x_j|^2) and
// C[i, j] = c^2 |x_i|^2, so the VALU is left with the square root, exp2, the polynomial
// and the two products of every entry.  Lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16] and receives D[4 (l / 16) + r][l % 16] in register r.  Wave w covers
// the tile's rows 32 w .. 32 w + 31 (two row sub-tiles) against all 128 columns (eight
// column sub-tiles).  The 16 partial sums per row (one per lane column) and per column
// (four lane rows times four waves) are combined in a fixed order as in k_sym_tiles.
// The dot-product form of the distance (flat kernels at u' = 0 only) carries the larger
// entry error described with the point layout: it serves the BF16 modes, while the FP32
// mode, Matern-1/2 and the great-circle distance take k_sym_tiles (difference form).
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int NU2>
__global__ __launch_bounds__(256) void k_sym_tiles_mfma(const float4* __restrict__ Xo,
                                                        const float* __restrict__ S, ObsDims d,
                                                        int j, float* __restrict__ part,
                                                        const float* __restrict__ mpart,
                                                        int nmpart, int n_t,
                                                        float* __restrict__ T,
                                                        const double* __restrict__ cpart,
                                                        int ncpart, int gs, int n_c,
                                                        double* __restrict__ colvec,
                                                        const LoopState* __restrict__ ls,
                                                        TriArgs ta) {
    static_assert(NU2 == 3 || NU2 == 5, "the dot-product distance needs a flat kernel at 0");
    __shared__ __align__(16) float red[2][16][SYM_TILE + 1];   // also FP64 scratch
    __shared__ int flags[1];
    double* sm = reinterpret_cast<double*>(&red[0][0][0]);
    if (ls->stop) return;
    const int n_extra = n_t + n_c;
    if ((int)blockIdx.x < n_extra) {
        step_spare(d, j, mpart, nmpart, n_t, T, cpart, ncpart, gs, n_c, colvec, ta, sm, flags);
        return;
    }
    const int t = blockIdx.x - n_extra;
    int Q = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
    while ((Q + 1) * (Q + 2) / 2 <= t) ++Q;
    while (Q * (Q + 1) / 2 > t) --Q;
    const int P = t - Q * (Q + 1) / 2;

    __shared__ float4 xr[SYM_TILE], xc[SYM_TILE];
    __shared__ float sr[SYM_TILE], sc[SYM_TILE];
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
    const int lane = tid & 63, w = tid >> 6;
    const int li = lane & 15, lg = lane >> 4;
    float aop[2], sa[2][4], ra[2][4];
    f32x4 cw[2];
#pragma unroll
    for (int R = 0; R < 2; ++R) {
        const int rb = 32 * w + 16 * R;
        const float comp = reinterpret_cast<const float*>(&xr[rb + li])[lg];
        aop[R] = lg < 3 ? -2.0f * comp : 1.0f;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            cw[R][r] = xr[rb + 4 * lg + r].w;
            sa[R][r] = sr[rb + 4 * lg + r];
            ra[R][r] = 0.0f;
        }
    }
    float bop[8], sb[8], cb[8];
#pragma unroll
    for (int C = 0; C < 8; ++C) {
        bop[C] = reinterpret_cast<const float*>(&xc[16 * C + li])[lg];
        sb[C] = sc[16 * C + li];
        cb[C] = 0.0f;
    }
#pragma unroll
    for (int C = 0; C < 8; ++C) {
#pragma unroll
        for (int R = 0; R < 2; ++R) {
            const f32x4 u2 = __builtin_amdgcn_mfma_f32_16x16x4f32(aop[R], bop[C], cw[R], 0, 0, 0);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float kv = matern_u<NU2>(__builtin_amdgcn_sqrtf(__builtin_fabsf(u2[r])));
                ra[R][r] = __builtin_fmaf(kv, sb[C], ra[R][r]);
                cb[C] = __builtin_fmaf(kv, sa[R][r], cb[C]);
            }
        }
    }
#pragma unroll
    for (int R = 0; R < 2; ++R)
#pragma unroll
        for (int r = 0; r < 4; ++r) red[0][li][32 * w + 16 * R + 4 * lg + r] = ra[R][r];
#pragma unroll
    for (int C = 0; C < 8; ++C) red[1][4 * w + lg][16 * C + li] = cb[C];
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

void launch_sym_tiles(int nu2, int dist, bool mfma_dist, const float4* Xo, const float* S,
                      const ObsDims& d, int j, float* part, const float* mpart, int nmpart,
                      float* T, const double* cpart, int ncpart, int gs, double* colvec,
                      const LoopState* ls, const TriArgs& ta, hipStream_t st,
                      hipEvent_t ev_start, hipEvent_t ev_stop) {
    const int nb = d.mp / SYM_TILE;
    const int tiles = nb * (nb + 1) / 2;
    const int n_t = (mpart && nmpart > 0) ? (d.rank + CR_POS - 1) / CR_POS : 0;
    const int n_c = (2 * j + 2 + CR_POS - 1) / CR_POS;
    // with events: the launch's own start and stop timestamps (kernel duration only)
#define CAKF_SYM_MFMA(NUV)                                                                    \
    hipExtLaunchKernelGGL((k_sym_tiles_mfma<NUV>), dim3(tiles + n_t + n_c), dim3(256), 0, st, \
                          ev_start, ev_stop, 0, Xo, S, d, j, part, mpart, nmpart, n_t, T,     \
                          cpart, ncpart, gs, n_c, colvec, ls, ta)
    if (mfma_dist && dist == DIST_EUCLID && nu2 == 5) { CAKF_SYM_MFMA(5); return; }
    if (mfma_dist && dist == DIST_EUCLID && nu2 == 3) { CAKF_SYM_MFMA(3); return; }
#undef CAKF_SYM_MFMA
    CAKF_DISPATCH_KERNEL(nu2, dist,
        hipExtLaunchKernelGGL((k_sym_tiles<NU2, DIST>), dim3(tiles + n_t + n_c), dim3(256), 0,
                              st, ev_start, ev_stop, 0, Xo, S, d, j, part, mpart, nmpart, n_t, T,
                              cpart, ncpart, gs, n_c, colvec, ls, ta));
}

}  // namespace cakf
