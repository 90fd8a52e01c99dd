// The symmetric kernel matvec of the CAKF action loop on gfx950: the tile sums of
// u_j = sigma_f2 K(Xo, Xo) s_j over the upper triangle of 128 x 128 tiles (each off-diagonal
// tile serves its row block and, transposed, its column block), with the reductions of the
// previous launch's column products in spare blocks.  Part of the observation-space loop
// described in obs_loop.hip.
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
// of T (column-major, T[l * ldmo + c]) from next_action's per-block partial sums; (n_c)
// the column products of s_j into colvec, laid out as
// [u_l^T s_j (l < j) | s_l^T s_j (l <= j) | r0^T s_j].
__device__ __forceinline__ void sym_extra_block(const ObsDims& d, int j,
                                                const float* __restrict__ mpart, int nmpart,
                                                int n_t, float* __restrict__ T,
                                                const double* __restrict__ cpart, int ncpart,
                                                int gs, double* __restrict__ colvec) {
    __shared__ double cred[CR_GRP][CR_POS + 1];
    if ((int)blockIdx.x < n_t) {
        const int pos0 = blockIdx.x * CR_POS;
        const double v = column_reduce(mpart, (size_t)d.ldmo, nmpart, d.rank, pos0, cred);
        if ((int)threadIdx.x < CR_POS && pos0 + (int)threadIdx.x < d.rank)
            T[(size_t)j * d.ldmo + pos0 + threadIdx.x] = (float)v;
    } else {
        const int pos0 = (blockIdx.x - n_t) * CR_POS;
        const int npos = 2 * j + 2;
        const double v = column_reduce(cpart, (size_t)gs, ncpart, npos, pos0, cred);
        if ((int)threadIdx.x < CR_POS && pos0 + (int)threadIdx.x < npos)
            colvec[pos0 + threadIdx.x] = v;
    }
}

// u_j = K(Xo, Xo) s_j over the upper triangle of SYM_TILE x SYM_TILE tiles.  Tile (P, Q),
// P <= Q, adds its row sums K_PQ s_Q to slot Q of block P and (P < Q) its column sums
// K_PQ^T s_P to slot P of block Q; every (slot, block) pair is written exactly once, so
// the reduction in form_u is deterministic.  Each thread evaluates an 8 x 8 set of
// entries.  The first n_t + n_c blocks instead finish, from next_action's per-block
// partial sums: (n_t) t_j = Mo^T s_j into column j of T (column-major, T[l * ldmo + c]);
// (n_c) the column products of s_j into colvec, laid out as
// [u_l^T s_j (l < j) | s_l^T s_j (l <= j) | r0^T s_j].
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
                                                   const LoopState* __restrict__ ls) {
    if (ls->stop) return;
    const int n_extra = n_t + n_c;
    if ((int)blockIdx.x < n_extra) {
        sym_extra_block(d, j, mpart, nmpart, n_t, T, cpart, ncpart, gs, colvec);
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
                                                        const LoopState* __restrict__ ls) {
    static_assert(NU2 == 3 || NU2 == 5, "the dot-product distance needs a flat kernel at 0");
    if (ls->stop) return;
    const int n_extra = n_t + n_c;
    if ((int)blockIdx.x < n_extra) {
        sym_extra_block(d, j, mpart, nmpart, n_t, T, cpart, ncpart, gs, colvec);
        return;
    }
    const int t = blockIdx.x - n_extra;
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
                      const LoopState* ls, hipStream_t st, hipEvent_t ev_start,
                      hipEvent_t ev_stop) {
    const int nb = d.mp / SYM_TILE;
    const int tiles = nb * (nb + 1) / 2;
    const int n_t = (mpart && nmpart > 0) ? (d.rank + CR_POS - 1) / CR_POS : 0;
    const int n_c = (2 * j + 2 + CR_POS - 1) / CR_POS;
    // with events: the launch's own start and stop timestamps (kernel duration only)
#define CAKF_SYM_MFMA(NUV)                                                                    \
    hipExtLaunchKernelGGL((k_sym_tiles_mfma<NUV>), dim3(tiles + n_t + n_c), dim3(256), 0, st, \
                          ev_start, ev_stop, 0, Xo, S, d, j, part, mpart, nmpart, n_t, T,     \
                          cpart, ncpart, gs, n_c, colvec, ls)
    if (mfma_dist && dist == DIST_EUCLID && nu2 == 5) { CAKF_SYM_MFMA(5); return; }
    if (mfma_dist && dist == DIST_EUCLID && nu2 == 3) { CAKF_SYM_MFMA(3); return; }
#undef CAKF_SYM_MFMA
    CAKF_DISPATCH_KERNEL(nu2, dist,
        hipExtLaunchKernelGGL((k_sym_tiles<NU2, DIST>), dim3(tiles + n_t + n_c), dim3(256), 0,
                              st, ev_start, ev_stop, 0, Xo, S, d, j, part, mpart, nmpart, n_t, T,
                              cpart, ncpart, gs, n_c, colvec, ls));
}

}  // namespace cakf
