// Block product of the CAKF update on gfx950:  Y = sigma_f2 * K(X, Xo) B  (n x b),
// the matrix-free Sigma H^T [W w] of Alg. 2 (the kernel part of P^- H^T [W w]).  The
// kernel matrix is generated tile by tile in registers/LDS and never stored.
#include "cakf_common.h"
#include "launchers.h"

namespace cakf {

// ------------------------------------------------------------------- BF16 MFMA form
// v_mfma_f32_32x32x16_bf16 (D = A B, A 32 x 16, B 16 x 32): lane l supplies
// A[l % 32][8 (l / 32) + t] and B[8 (l / 32) + t][l % 32], t = 0..7, and holds
// D[8 (i / 4) + 4 (l / 32) + i % 4][l % 32] in accumulator register i.
//
// A is the kernel tile: each lane evaluates its 8 entries (its state row against 8
// observation points) in FP32 on the VALU and rounds them to BF16 in registers, so the
// tile never reaches LDS or memory.  B = [W w] arrives pre-split and transposed
// (column-major, BF16): the chunk for 64 observations is staged in LDS and shared by the
// workgroup's 4 waves.  Each wave owns one 32-row tile of state rows and NT 32-column
// tiles.  With X3 the products are
// Kh Bh + Kl Bh + Kh Bl on K = Kh + Kl, B = Bh + Bl (each part BF16), which restores
// close to FP32 accuracy at 3x the MFMA work.
//
// For the Euclidean Matern-3/2 and -5/2 kernels (MD) the squared scaled distances come from
// FP32 MFMA instead of the VALU: v_mfma_f32_32x32x2f32 twice (coordinates x, y, then z and
// the norm term) per 32 observations gives D'[o][p] = <(c x_o, c y_o, c z_o, c^2 |x_o|^2),
// (-2 c x_p, -2 c y_p, -2 c z_p, 1)> + c^2 |x_p|^2 with the observations as rows, so lane l
// receives its own state row l % 32 against the observations
// 8 (i / 4) + 4 (l / 32) + i % 4 (i = 0..15) of the group.  Taken 8 at a time these are the
// lane's A values for two BF16 k-steps, in the observation order that swaps the middle two
// 4-blocks of every 16 (positions 4..7 <-> 8..11); B is stored in that order (k_split_bt),
// so the products are unchanged.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// observation at stored position q of the MD order (an involution within blocks of 16)
__host__ __device__ __forceinline__ int md_perm(int q) {
    const int o = q & 15;
    return ((o >> 2) == 1 || (o >> 2) == 2) ? (q ^ 12) : q;
}
constexpr int MF_KC = 64;        // observations per LDS chunk (4 MFMA k-steps)
constexpr int MF_ROWS = 128;     // state rows per workgroup (4 waves x 32)
constexpr int MF_MAXNT = 8;      // tiles of a single launch (B parts in LDS: 2 x 37 KB at 8)
constexpr int MF_SPLITNT = 5;    // tiles per launch when they need more than one launch

template <int NU2, int DIST, int NT, bool X3>
__global__ __launch_bounds__(256) void k_block_mfma(const float4* __restrict__ Xs, int n,
                                                    const float4* __restrict__ Xo, int mp,
                                                    const __bf16* __restrict__ Bth,
                                                    const __bf16* __restrict__ Btl, int ldbt,
                                                    int tile0, int ncols, int coff,
                                                    float sigma_f2,
                                                    float* __restrict__ out, int ldo,
                                                    int qchunk, size_t part_stride,
                                                    const float* __restrict__ Bf, int ldbf,
                                                    int fcol) {
    __shared__ float4 xo[MF_KC];
    __shared__ bf16x8 bh[NT * 32][MF_KC / 8 + 1];
    __shared__ bf16x8 bl[X3 ? NT * 32 : 1][MF_KC / 8 + 1];
    __shared__ float wf[MF_KC];       // the FP32 column's chunk, in stored order
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int rl = lane & 31, half = lane >> 5;
    const int row0 = blockIdx.x * MF_ROWS + w * 32;
    const float4 xa = prep_row<DIST>(Xs[min(row0 + rl, n - 1)]);
    constexpr bool MD = DIST == DIST_EUCLID && NU2 != 1;
    // MD operands of the state-row side: coordinates (half, 2 + half) of the prepared row
    const float rb1 = half == 0 ? xa.x : xa.y, rb2 = half == 0 ? xa.z : 1.0f;
    f32x16 acc[NT];
#pragma unroll
    for (int c = 0; c < NT; ++c)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[c][i] = 0.0f;
    // column fcol (>= 0) of out is summed in FP32 from the FP32 kernel entries, one chunk at
    // a time, the chunk sums added in FP64 (when it is also one of the MFMA columns, it
    // replaces that column's MFMA result)
    const bool fp = fcol >= 0;
    double fsum = 0.0;
    // observation range of this split (qchunk a multiple of MF_KC)
    const int qend = min(mp, (int)(blockIdx.y + 1) * qchunk);
    out += blockIdx.y * part_stride;
    for (int q0 = blockIdx.y * qchunk; q0 < qend; q0 += MF_KC) {
        __syncthreads();
        if (threadIdx.x < MF_KC) xo[threadIdx.x] = Xo[q0 + threadIdx.x];
        if (fp && threadIdx.x >= 64 && threadIdx.x < 64 + MF_KC) {
            const int q = q0 + threadIdx.x - 64;
            wf[threadIdx.x - 64] = Bf[(size_t)(MD ? md_perm(q) : q) * ldbf + fcol];
        }
        for (int e = threadIdx.x; e < NT * 32 * (MF_KC / 8); e += 256) {
            const int c = e / (MF_KC / 8), g = e % (MF_KC / 8);
            const size_t off = (size_t)(tile0 * 32 + c) * ldbt + q0 + 8 * g;
            bh[c][g] = *reinterpret_cast<const bf16x8*>(Bth + off);
            if constexpr (X3) bl[c][g] = *reinterpret_cast<const bf16x8*>(Btl + off);
        }
        __syncthreads();
        f32x16 dd;
        float fchunk = 0.0f;
#pragma unroll
        for (int ks = 0; ks < MF_KC / 16; ++ks) {
            bf16x8 ah, al;
            float kv[8];
            if constexpr (MD) {
                if (ks % 2 == 0) {
                    // squared distances of the 32 observations of k-steps ks, ks + 1
                    const float4 xg = xo[ks * 16 + rl];
                    const float a1 = half == 0 ? xg.x : xg.y, a2 = half == 0 ? xg.z : xg.w;
#pragma unroll
                    for (int i = 0; i < 16; ++i) dd[i] = xa.w;
                    dd = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, rb1, dd, 0, 0, 0);
                    dd = __builtin_amdgcn_mfma_f32_32x32x2f32(a2, rb2, dd, 0, 0, 0);
                }
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    const float ka =
                        matern_u<NU2>(__builtin_amdgcn_sqrtf(__builtin_fabsf(dd[8 * (ks % 2) + t])));
                    kv[t] = ka;
                    ah[t] = (__bf16)ka;
                    if constexpr (X3) al[t] = (__bf16)(ka - (float)ah[t]);
                }
            } else {
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    const float ka = kval<NU2, DIST>(xa, xo[ks * 16 + 8 * half + t]);
                    kv[t] = ka;
                    ah[t] = (__bf16)ka;
                    if constexpr (X3) al[t] = (__bf16)(ka - (float)ah[t]);
                }
            }
            // the lane's 8 entries sit at stored positions ks * 16 + 8 half + t
            if (fp) {
#pragma unroll
                for (int t = 0; t < 8; ++t)
                    fchunk = __builtin_fmaf(kv[t], wf[ks * 16 + 8 * half + t], fchunk);
            }
            // the three products of each column tile are issued NT apart, so that no
            // MFMA waits on the result of the one before it
#pragma unroll
            for (int c = 0; c < NT; ++c)
                acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                    ah, bh[c * 32 + rl][ks * 2 + half], acc[c], 0, 0, 0);
            if constexpr (X3) {
#pragma unroll
                for (int c = 0; c < NT; ++c)
                    acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                        al, bh[c * 32 + rl][ks * 2 + half], acc[c], 0, 0, 0);
#pragma unroll
                for (int c = 0; c < NT; ++c)
                    acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                        ah, bl[c * 32 + rl][ks * 2 + half], acc[c], 0, 0, 0);
            }
        }
        fsum += (double)fchunk;
    }
#pragma unroll
    for (int c = 0; c < NT; ++c) {
        // MFMA column cm (of ncols) is column coff + cm of out
        const int cm = (tile0 + c) * 32 + rl, col = coff + cm;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int row = row0 + 8 * (i / 4) + 4 * half + (i % 4);
            if (row < n && cm < ncols && col != fcol)
                out[(size_t)row * ldo + col] = sigma_f2 * acc[c][i];
        }
    }
    if (fp) {
        // the two half-waves hold the same row over complementary observations
        const double other = __shfl_xor(fsum, 32, 64);
        const double tot = half == 0 ? fsum + other : other + fsum;
        if (half == 0 && row0 + rl < n)
            out[(size_t)(row0 + rl) * ldo + fcol] = (float)((double)sigma_f2 * tot);
    }
}

template <int NU2, int DIST, bool X3>
static void launch_mfma_tiles(int nt, int tile0, const float4* Xs, int n, const float4* Xo,
                              int mp, const __bf16* Bth, const __bf16* Btl, int ldbt,
                              int ncols, int coff, float sigma_f2, float* out, int ldo,
                              int nsplit,
                              int qchunk, size_t part_stride, const float* Bf, int ldbf,
                              int fcol, hipStream_t st) {
    const dim3 grid((n + MF_ROWS - 1) / MF_ROWS, nsplit), block(256);
#define CAKF_MF(NTV)                                                                       \
    hipLaunchKernelGGL((k_block_mfma<NU2, DIST, NTV, X3>), grid, block, 0, st, Xs, n, Xo, mp, \
                       Bth, Btl, ldbt, tile0, ncols, coff, sigma_f2, out, ldo, qchunk,        \
                       part_stride, Bf, ldbf, fcol)
    switch (nt) {
        case 1: CAKF_MF(1); break;
        case 2: CAKF_MF(2); break;
        case 3: CAKF_MF(3); break;
        case 4: CAKF_MF(4); break;
        case 5: CAKF_MF(5); break;
        case 6: CAKF_MF(6); break;
        case 7: CAKF_MF(7); break;
        default: CAKF_MF(8); break;
    }
#undef CAKF_MF
}

// FP32 MFMA form of the same product (v_mfma_f32_32x32x2f32, full FP32 operands): lane l
// supplies A[l % 32][l / 32] = K(row l % 32, observation l / 32 of the k-step), evaluated
// on the VALU (difference form of the distance), and B[l / 32][l % 32] from the LDS chunk,
// and holds D[8 (i / 4) + 4 (l / 32) + i % 4][l % 32] in register i.  Each wave owns 32
// state rows and NT 32-column tiles; a workgroup's four waves share the chunk of 64
// observations of B.  The MFMA accumulates one chunk in FP32; the chunk sums are added
// into FP64 accumulators, so the rounding error grows with the chunk length (64) rather
// than with m: the columns of [W w] are Ghat-orthonormal search directions whose products
// with the kernel matrix cancel by two to three orders of magnitude, and a plain FP32
// sum over m = 600 observations already left ~1e-5 in the posterior variance.
constexpr int F32_KC = 64;
constexpr int F32_MAXNT = 3;     // column tiles per launch (FP64 accumulators: 32 VGPRs each;
                                 // 5 tiles need 256 VGPRs, one wave per SIMD: 9.0 ms
                                 // against 5.0 ms at n = 65536)
template <int NU2, int DIST, int NT>
__global__ __launch_bounds__(256) void k_block_mfma32(const float4* __restrict__ Xs, int n,
                                                      const float4* __restrict__ Xo, int m,
                                                      const float* __restrict__ B, int ldb,
                                                      int col0, int ncols, float sigma_f2,
                                                      float* __restrict__ out, int ldo,
                                                      int qchunk, size_t part_stride) {
    constexpr int BC = NT * 32;
    constexpr int BLD = F32_KC * BC / 256;          // B elements each thread stages
    __shared__ float4 xo[F32_KC];
    __shared__ float Bs[F32_KC][BC];
    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int rl = lane & 31, half = lane >> 5;
    const int row0 = blockIdx.x * MF_ROWS + w * 32;
    const float4 xa = prep_row<DIST>(Xs[min(row0 + rl, n - 1)]);
    f32x16 acc[NT];
    double dacc[NT][16];
#pragma unroll
    for (int c = 0; c < NT; ++c)
#pragma unroll
        for (int i = 0; i < 16; ++i) dacc[c][i] = 0.0;
    const int qend = min(m, (int)(blockIdx.y + 1) * qchunk);
    out += blockIdx.y * part_stride;
    for (int q0 = blockIdx.y * qchunk; q0 < qend; q0 += F32_KC) {
        const int qn = min(F32_KC, qend - q0);
        __syncthreads();
        if (tid < F32_KC) xo[tid] = Xo[q0 + min(tid, qn - 1)];
        float bv[BLD];
#pragma unroll
        for (int u = 0; u < BLD; ++u) {
            const int e = tid + 256 * u, q = e / BC, c = e % BC;
            const float x = B[(size_t)(q0 + min(q, qn - 1)) * ldb + col0 + min(c, ncols - 1)];
            bv[u] = (q < qn && c < ncols) ? x : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < BLD; ++u) (&Bs[0][0])[tid + 256 * u] = bv[u];
        __syncthreads();
#pragma unroll
        for (int c = 0; c < NT; ++c)
#pragma unroll
            for (int i = 0; i < 16; ++i) acc[c][i] = 0.0f;
#pragma unroll 4
        for (int ks = 0; ks < F32_KC / 2; ++ks) {
            const int k = 2 * ks + half;
            const float a = kval<NU2, DIST>(xa, xo[k]);
#pragma unroll
            for (int c = 0; c < NT; ++c)
                acc[c] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, Bs[k][32 * c + rl], acc[c], 0, 0, 0);
        }
#pragma unroll
        for (int c = 0; c < NT; ++c)
#pragma unroll
            for (int i = 0; i < 16; ++i) dacc[c][i] += (double)acc[c][i];
    }
#pragma unroll
    for (int c = 0; c < NT; ++c) {
        const int col = 32 * c + rl;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int row = row0 + 8 * (i / 4) + 4 * half + (i % 4);
            if (row < n && col < ncols)
                out[(size_t)row * ldo + col0 + col] = (float)((double)sigma_f2 * dacc[c][i]);
        }
    }
}

template <int NU2, int DIST>
static void launch_mfma32_tiles(int nt, dim3 grid, hipStream_t st, const float4* Xs, int n,
                                const float4* Xo, int m, const float* B, int ldb, int col0,
                                int ncols, float sigma_f2, float* out, int ldo, int qchunk,
                                size_t part_stride) {
#define CAKF_F32(NTV)                                                                        \
    hipLaunchKernelGGL((k_block_mfma32<NU2, DIST, NTV>), grid, dim3(256), 0, st, Xs, n, Xo, m, \
                       B, ldb, col0, ncols, sigma_f2, out, ldo, qchunk, part_stride)
    switch (nt) {
        case 1: CAKF_F32(1); break;
        case 2: CAKF_F32(2); break;
        case 3: CAKF_F32(3); break;
        case 4: CAKF_F32(4); break;
        default: CAKF_F32(5); break;
    }
#undef CAKF_F32
}

// Split B (FP32, row-major mp x ldb, columns 0..bp) into transposed BF16 parts:
// Bth[c * mp + q] = bf16(B[o, c]), Btl = bf16(B - Bth), o = q or, with perm, md_perm(q).
__global__ void k_split_bt(const float* __restrict__ B, int mp, int ldb, int bcols, int bp,
                           int perm, __bf16* __restrict__ Bth, __bf16* __restrict__ Btl) {
    const size_t total = (size_t)mp * bp;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(e / mp), q = (int)(e % mp);
        const int o = perm ? md_perm(q) : q;
        const float v = c < bcols ? B[(size_t)o * ldb + c] : 0.0f;
        const __bf16 h = (__bf16)v;
        Bth[e] = h;
        Btl[e] = (__bf16)(v - (float)h);
    }
}

// Sum of the nsplit partial products part[s] (n x ldp, s-major) into out (fixed order).
__global__ void k_split_sum(const float* __restrict__ part, int nsplit, size_t stride, int n,
                            int ncols, int ldp, float* __restrict__ out, int ldo) {
    const size_t total = (size_t)n * ncols;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int row = (int)(e / ncols), col = (int)(e % ncols);
        const float* p = part + (size_t)row * ldp + col;
        float v = 0.0f;
        for (int s = 0; s < nsplit; ++s) v += p[s * stride];
        out[(size_t)row * ldo + col] = v;
    }
}

int block_product_splits(int n, int mp, int bcols, size_t part_elems) {
    // enough workgroups to fill the 256 CUs several times over (about 1024), at least 512
    // observations per range, within the partial buffer
    const int rowblocks = (n + MF_ROWS - 1) / MF_ROWS;
    if (rowblocks >= 256) return 1;     // the row blocks alone fill the chip
    int ns = std::max(1, 1024 / std::max(rowblocks, 1));
    ns = std::min(ns, std::max(1, mp / 512));
    const size_t per = (size_t)n * (size_t)bcols;
    while (ns > 1 && (size_t)ns * per > part_elems) --ns;
    return ns;
}

void launch_block_product(int nu2, int dist, int prec, const float4* Xs, int n,
                          const float4* Xo, int m, int mp, const float* B, int ldb, int bcols,
                          __bf16* Bth, __bf16* Btl, float sigma_f2, float* out, int ldo,
                          hipStream_t st, int nsplit, float* part, int fp32_col) {
    // With nsplit > 1 the observation axis is cut into nsplit ranges (multiples of 512
    // observations), each range's product goes to part (n x bcols per range) and the ranges
    // are summed into out afterwards.
    if (nsplit < 1 || !part) nsplit = 1;
    const int qchunk = nsplit > 1 ? ((mp + 511) / 512 + nsplit - 1) / nsplit * 512 : mp;
    float* dst = nsplit > 1 ? part : out;
    const int ldd = nsplit > 1 ? bcols : ldo;
    const size_t stride = nsplit > 1 ? (size_t)n * bcols : 0;
    if (prec == 0) {
        const int blocks = (n + MF_ROWS - 1) / MF_ROWS;
        for (int c0 = 0; c0 < bcols; c0 += 32 * F32_MAXNT) {
            const int nc = std::min(32 * F32_MAXNT, bcols - c0);
            const int nt = (nc + 31) / 32;
            CAKF_DISPATCH_KERNEL(nu2, dist,
                (launch_mfma32_tiles<NU2, DIST>(nt, dim3(blocks, nsplit), st, Xs, n, Xo, m, B,
                                                ldb, c0, nc, sigma_f2, dst, ldd,
                                                nsplit > 1 ? qchunk : m, stride)));
        }
    } else {
        // the FP32 column, when it is the first or the last one, is left out of the MFMA
        // columns altogether (no tile carries it as a padded or discarded column): the first
        // launch sums it on the VALU from the same kernel entries
        int coff = 0, mcols = bcols;
        if (fp32_col >= 0 && bcols >= 2 && (fp32_col == 0 || fp32_col == bcols - 1)) {
            mcols = bcols - 1;
            coff = fp32_col == 0 ? 1 : 0;
        }
        const int ntiles = (mcols + 31) / 32;
        const size_t total = (size_t)mp * ntiles * 32;
        hipLaunchKernelGGL(k_split_bt, dim3((int)std::min<size_t>((total + 255) / 256, 8192)),
                           dim3(256), 0, st, B + coff, mp, ldb, mcols, ntiles * 32,
                           (dist == DIST_EUCLID && nu2 != 1) ? 1 : 0, Bth, Btl);
        // up to MF_MAXNT tiles in one launch (the kernel entries evaluated once); more in
        // launches of at most MF_SPLITNT tiles, as even as possible (measured: 8-tile
        // launches at two workgroups per CU beat two launches over the same 8 tiles, but
        // lose to 5-tile launches at three per CU once several launches are needed anyway)
        const int nl = ntiles <= MF_MAXNT ? 1 : (ntiles + MF_SPLITNT - 1) / MF_SPLITNT;
        for (int l = 0, t0 = 0; l < nl; ++l) {
            const int nt = (ntiles - t0) / (nl - l) + ((ntiles - t0) % (nl - l) != 0 ? 1 : 0);
            // the FP32 column: the first launch when it is outside the MFMA columns, else
            // the launch whose tiles hold it
            const int fc = mcols < bcols ? (t0 == 0 ? fp32_col : -1)
                           : (fp32_col >= 32 * t0 && fp32_col < std::min(32 * (t0 + nt), bcols))
                               ? fp32_col : -1;
            if (prec == 2) {
                CAKF_DISPATCH_KERNEL(nu2, dist,
                    (launch_mfma_tiles<NU2, DIST, true>(nt, t0, Xs, n, Xo, mp, Bth, Btl, mp,
                                                        mcols, coff, sigma_f2, dst, ldd, nsplit,
                                                        qchunk, stride, B, ldb, fc, st)));
            } else {
                CAKF_DISPATCH_KERNEL(nu2, dist,
                    (launch_mfma_tiles<NU2, DIST, false>(nt, t0, Xs, n, Xo, mp, Bth, Btl, mp,
                                                         mcols, coff, sigma_f2, dst, ldd, nsplit,
                                                         qchunk, stride, B, ldb, fc, st)));
            }
            t0 += nt;
        }
    }
    if (nsplit > 1) {
        const size_t total = (size_t)n * bcols;
        hipLaunchKernelGGL(k_split_sum, dim3((int)std::min<size_t>((total + 255) / 256, 4096)),
                           dim3(256), 0, st, part, nsplit, stride, n, bcols, bcols, out, ldo);
    }
}

}  // namespace cakf
