// Householder tridiagonalisation of the truncation's FP64 Gram matrix on gfx950 (one
// cooperative launch), the first stage of the symmetric eigensolver behind Truncate
// (Sec. 3.2): G = Q T Q^T with T tridiagonal, Q = H_0 H_1 ... H_{K-3},
// H_j = I - tau_j v_j v_j^T, and the back-transformation Q Z of the leading
// eigenvectors of T.
//
// Why one launch: the reduction is a chain of K - 2 dependent steps, each a symmetric
// matrix-vector product with the trailing matrix and a rank-2 update.  As separate
// kernels every step costs several launches; here the K x K matrix is distributed by
// rows over the registers of a few workgroups (row i lives in workgroup i mod G, lane l
// of the owning wave holds its entries l + 64 t), each step's matrix work is local, and
// the workgroups exchange only two vectors per step through global memory, separated by
// one grid-wide barrier:
//   after barrier j every wave holds v_j, tau_j and reads p_j = tau_j A v_j (each owner
//   wrote its rows' entries) and row j+1 of the matrix before update j (written by its
//   owner); it forms w_j = p_j - (tau_j / 2)(p_j^T v_j) v_j, the updated row j+1
//   (row - v_{j+1} w_j - w_{j+1} v_j) and from it v_{j+1}, tau_{j+1} (identically in
//   every wave: same data, same reduction order); then it applies update j to its own
//   rows and forms their entries of p_{j+1}; the owner of row j+2 publishes it.
// Vectors are double-buffered by the parity of j, so a workgroup one step ahead never
// overwrites what a slower one still reads.  The reflector of step j follows LAPACK's
// convention (dlarfg: v_j[j+1] = 1, beta = -sign(alpha) ||x||).
//
// The barrier is a monotonically increasing counter (one device-scope atomic add per
// workgroup and step).  Co-residency of all workgroups is guaranteed by the cooperative
// launch (which fails instead of starting otherwise).  Every wait is bounded: a wait
// that exceeds its spin limit raises an abort flag that ends every later wait, so the
// launch always finishes; the flag turns the output into NaN.
#include <hip/hip_cooperative_groups.h>

#include "cakf_common.h"
#include "launchers.h"

namespace cakf {

int tridiag_max_k() { return TD_MAXK; }

// Shapes of the register-resident reduction: KC column chunks of 64 per row, WAVES waves
// per workgroup, R rows per wave (the rows and four chunked vectors stay in registers).
template <int KC, int WAVES, int R>
struct TdShape {
    static constexpr int kc = KC, waves = WAVES, rows = R;
    static int workgroups(int K) { return (K + WAVES * R - 1) / (WAVES * R); }
};
using TdSmall = TdShape<10, 8, 5>;     // K <= 640: 40 rows per workgroup
using TdLarge = TdShape<20, 4, 5>;     // K <= 1280: 20 rows per workgroup (64 at K = 1280)

int tridiag_workgroups(int K) {
    return K <= 64 * TdSmall::kc ? TdSmall::workgroups(K) : TdLarge::workgroups(K);
}

// The arrival is a release (the workgroup's writes, ordered before it by the block
// barrier, become visible at agent scope); the wait polls with relaxed loads and ends
// with one acquire fence, so the cache invalidation of an acquire happens once per step
// and not once per poll.
__device__ __forceinline__ void td_barrier(unsigned* ctr, unsigned target, int* abort_flag) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        unsigned spins = 0;
        while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
            if (++spins > (1u << 24)) {
                __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
}

// G: K x K symmetric (both triangles).  Out: V (column-major K x K; column j holds v_j
// in rows j+2 .. K-1), tau, d (K), e (K - 1).  pbuf, rowbuf: 2K doubles each; ctr and
// abort_flag zero on entry.
template <int KC, int WAVES, int R>
__global__ __launch_bounds__(WAVES * 64) void k_tridiag(const double* __restrict__ G, int K,
                                                        double* __restrict__ V,
                                                        double* __restrict__ tau,
                                                        double* __restrict__ d,
                                                        double* __restrict__ e,
                                                        double* __restrict__ pbuf,
                                                        double* __restrict__ rowbuf,
                                                        unsigned* ctr, int* abort_flag) {
    // LDS copies of v (by parity), w and the new row, for the lookups of single entries
    __shared__ double vs[2][64 * KC], ws[64 * KC], xs[64 * KC];
    const int NWG = gridDim.x, wg = blockIdx.x, tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    double a[R][KC];
    int rowi[R];
#pragma unroll
    for (int s = 0; s < R; ++s) {
        const int i = wg + (wave + WAVES * s) * NWG;
        rowi[s] = i < K ? i : -1;
#pragma unroll
        for (int t = 0; t < KC; ++t) {
            const int k = lane + 64 * t;
            a[s][t] = (i < K && k < K) ? G[(size_t)i * K + k] : 0.0;
        }
    }
    // reflector of column 0 from row 0
    double v[KC], w[KC];
    double tj;
    {
        double x[KC], s2 = 0.0;
#pragma unroll
        for (int t = 0; t < KC; ++t) {
            const int k = lane + 64 * t;
            x[t] = k < K ? G[k] : 0.0;
            if (k >= 2) s2 += x[t] * x[t];
        }
        const double xn2 = wave_sum(s2);
        const double alpha = G[1];
        double beta = alpha, scale = 0.0;
        tj = 0.0;
        if (xn2 != 0.0) {
            beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
            tj = (beta - alpha) / beta;
            scale = 1.0 / (alpha - beta);
        }
#pragma unroll
        for (int t = 0; t < KC; ++t) {
            const int k = lane + 64 * t;
            v[t] = k == 1 ? 1.0 : (k > 1 ? x[t] * scale : 0.0);
        }
        if (wg == 0 && tid == 0) {
            d[0] = G[0];
            e[0] = beta;
            tau[0] = tj;
        }
    }
    if (wave == 0)
#pragma unroll
        for (int t = 0; t < KC; ++t) vs[0][lane + 64 * t] = v[t];
#pragma unroll
    for (int s = 0; s < R; ++s) {
        double acc = 0.0;
#pragma unroll
        for (int t = 0; t < KC; ++t) acc += a[s][t] * v[t];
        acc = wave_sum(acc);
        if (lane == 0 && rowi[s] > 0) pbuf[rowi[s]] = tj * acc;
        if (rowi[s] == 1)
#pragma unroll
            for (int t = 0; t < KC; ++t) {
                const int k = lane + 64 * t;
                if (k >= 1 && k < K) rowbuf[k] = a[s][t];
            }
    }
    for (int j = 0; j < K - 2; ++j) {
        const int b = j & 1;
        // v_j into column j of V (one workgroup per step)
        if (wg == j % NWG && wave == 0)
#pragma unroll
            for (int t = 0; t < KC; ++t) {
                const int k = lane + 64 * t;
                if (k >= j + 2 && k < K) V[(size_t)j * K + k] = v[t];
            }
        td_barrier(ctr, (unsigned)(j + 1) * NWG, abort_flag);
        const double* pb = pbuf + b * K;
        const double* rb = rowbuf + b * K;
        double x[KC], s2 = 0.0;
#pragma unroll
        for (int t = 0; t < KC; ++t) {
            const int k = lane + 64 * t;
            const bool in = k > j && k < K;
            const double pk = in ? pb[k] : 0.0;
            x[t] = in ? rb[k] : 0.0;
            w[t] = pk;
            s2 += pk * v[t];
        }
        const double kk = 0.5 * tj * wave_sum(s2);
        // w_{j+1} = p_{j+1} - kk (v_j[j+1] = 1)
        const double w1 = pb[j + 1] - kk;
        double sx = 0.0;
#pragma unroll
        for (int t = 0; t < KC; ++t) {
            const int k = lane + 64 * t;
            w[t] -= kk * v[t];
            // row j+1 after update j
            x[t] = k > j ? x[t] - w[t] - w1 * v[t] : 0.0;
            if (k >= j + 3) sx += x[t] * x[t];
        }
        const double xn2 = wave_sum(sx);
        if (wave == 0)
#pragma unroll
            for (int t = 0; t < KC; ++t) {
                ws[lane + 64 * t] = w[t];
                xs[lane + 64 * t] = x[t];
            }
        __syncthreads();
        const int j1 = j + 1;
        const double alpha = xs[j1 + 1];
        double beta = alpha, scale = 0.0, tn = 0.0;
        if (xn2 != 0.0) {
            beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
            tn = (beta - alpha) / beta;
            scale = 1.0 / (alpha - beta);
        }
        if (wg == 0 && tid == 0) {
            d[j1] = xs[j1];
            e[j1] = beta;
            tau[j1] = tn;
        }
        // the new reflector (into x)
#pragma unroll
        for (int t = 0; t < KC; ++t) {
            const int k = lane + 64 * t;
            x[t] = k == j1 + 1 ? 1.0 : (k > j1 + 1 ? x[t] * scale : 0.0);
        }
        // update j of the own rows, then their entries of p_{j+1}
        const double* vprev = vs[b];
#pragma unroll
        for (int s = 0; s < R; ++s) {
            const int i = rowi[s];
            if (i <= j) continue;                  // wave-uniform
            const double vi = vprev[i], wi = ws[i];
            double acc = 0.0;
#pragma unroll
            for (int t = 0; t < KC; ++t) {
                a[s][t] -= vi * w[t] + wi * v[t];
                acc += a[s][t] * x[t];
            }
            acc = wave_sum(acc);
            if (lane == 0 && i > j1) pbuf[(1 - b) * K + i] = tn * acc;
            if (i == j1 + 1)
#pragma unroll
                for (int t = 0; t < KC; ++t) {
                    const int k = lane + 64 * t;
                    if (k >= j1 + 1 && k < K) rowbuf[(1 - b) * K + k] = a[s][t];
                }
        }
#pragma unroll
        for (int t = 0; t < KC; ++t) v[t] = x[t];
        if (wave == 0)
#pragma unroll
            for (int t = 0; t < KC; ++t) vs[1 - b][lane + 64 * t] = v[t];
        tj = tn;
    }
    const bool failed = __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    if (wg == 0 && tid == 0) {
        const double dk2 = xs[K - 2], ek2 = xs[K - 1];
        d[K - 2] = failed ? __builtin_nan("") : dk2;
        e[K - 2] = failed ? __builtin_nan("") : ek2;
        tau[K - 2] = 0.0;
    }
#pragma unroll
    for (int s = 0; s < R; ++s)
        if (rowi[s] == K - 1)
#pragma unroll
            for (int t = 0; t < KC; ++t)
                if (lane + 64 * t == K - 1) d[K - 1] = failed ? __builtin_nan("") : a[s][t];
}

// Zero the barrier counter and the abort flag before a launch (a kernel rather than a
// memset node, so that a captured stream replays it correctly).
__global__ void k_clear_barrier(unsigned* ctr, int* abort_flag) {
    *ctr = 0u;
    *abort_flag = 0;
}

// Returns hipSuccess or the launch error (e.g. when the grid cannot be co-resident).
hipError_t launch_tridiag(const double* G, int K, double* V, double* tau, double* d, double* e,
                          double* pbuf, double* rowbuf, unsigned* ctr, int* abort_flag,
                          hipStream_t st) {
    if (K < 3 || K > TD_MAXK) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_clear_barrier, dim3(1), dim3(1), 0, st, ctr, abort_flag);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    const int nwg = tridiag_workgroups(K);
    void* args[] = {(void*)&G, (void*)&K, (void*)&V, (void*)&tau, (void*)&d, (void*)&e,
                    (void*)&pbuf, (void*)&rowbuf, (void*)&ctr, (void*)&abort_flag};
    if (K <= 64 * TdSmall::kc)
        return hipLaunchCooperativeKernel(
            (const void*)k_tridiag<TdSmall::kc, TdSmall::waves, TdSmall::rows>, dim3(nwg),
            dim3(TdSmall::waves * 64), args, 0, st);
    return hipLaunchCooperativeKernel(
        (const void*)k_tridiag<TdLarge::kc, TdLarge::waves, TdLarge::rows>, dim3(nwg),
        dim3(TdLarge::waves * 64), args, 0, st);
}

// ------------------------------------------------------ tridiagonal eigenproblem (top r)
// The r largest eigenpairs of the symmetric tridiagonal T (diagonal d, off-diagonal e),
// computed independently of one another:
//   eigenvalues  by bisection on Sturm counts (the number of negative pivots of the
//                LDL^T factorisation of T - sigma I is the number of eigenvalues below
//                sigma), two waves per eigenvalue; each lane follows two shifts at once,
//                so a round tests 256 shifts and shrinks the bracket 257-fold;
//   eigenvectors by the twisted factorisation of T - lambda I: the forward factor
//                L D L^T and the backward factor U D' U^T meet at the index k where the
//                twist element gamma_k = D_k + D'_k - (d_k - lambda) is smallest in
//                magnitude, and z is obtained from z_k = 1 outwards with the two factors'
//                multipliers (two lanes per eigenvector, the pivots kept in LDS);
//   ties         eigenvalues within TRI_CTOL ||T|| of a neighbour (repeated eigenvalues)
//                are recomputed by inverse iteration from distinct starting vectors, each
//                iterate orthogonalised against the tie's earlier vectors (one wave per
//                tie), since their twisted vectors can coincide.
// Vectors of distinct eigenvalues that lie close together (absolute gaps far below ||T||,
// as in the graded spectra of a truncation Gram matrix) carry errors of order
// eps ||T|| / gap and are left slightly non-orthogonal; the caller restores orthogonality
// with the symmetric correction Z (Z^T Z)^{-1/2} (launch_lowdin_x).
// Output: Zr (row-major K x r, column c the eigenvector of the c-th largest eigenvalue).
constexpr double TRI_CTOL = 1e-13;
constexpr int TRI_ITERS = 3;
constexpr int TRI_MAXK = 1280;         // LDS of the cluster kernel (6 K doubles)
// the twisted kernel keeps 3 VPB K pivots and vector entries in LDS: VPB = 8 eigenvectors
// per workgroup for K <= 640, 4 for K <= 1280
constexpr int TW_LDS = 5120;           // VPB * largest K

// Gershgorin bounds of T widened by rounding, ||T|| and the pivot floor, per workgroup.
__device__ void tri_bounds(const double* __restrict__ d, const double* __restrict__ e, int K,
                           double* red, double& glo, double& ghi, double& tnorm,
                           double& pivmin) {
    double lo = 1e300, hi = -1e300, emax = 0.0;
    for (int i = threadIdx.x; i < K; i += blockDim.x) {
        const double a = i > 0 ? fabs(e[i - 1]) : 0.0, b = i + 1 < K ? fabs(e[i]) : 0.0;
        lo = fmin(lo, d[i] - a - b);
        hi = fmax(hi, d[i] + a + b);
        emax = fmax(emax, b * b);
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int off = 32; off >= 1; off >>= 1) {
        lo = fmin(lo, __shfl_xor(lo, off, 64));
        hi = fmax(hi, __shfl_xor(hi, off, 64));
        emax = fmax(emax, __shfl_xor(emax, off, 64));
    }
    if (lane == 0) {
        red[3 * w] = lo;
        red[3 * w + 1] = hi;
        red[3 * w + 2] = emax;
    }
    __syncthreads();
    lo = red[0];
    hi = red[1];
    emax = red[2];
    for (int k = 1; k < nw; ++k) {
        lo = fmin(lo, red[3 * k]);
        hi = fmax(hi, red[3 * k + 1]);
        emax = fmax(emax, red[3 * k + 2]);
    }
    __syncthreads();
    tnorm = fmax(fabs(lo), fabs(hi));
    pivmin = 2.2250738585072014e-308 * fmax(1.0, emax);
    const double pad = 2.0 * 2.220446049250313e-16 * tnorm + 2.0 * pivmin;
    glo = lo - pad;
    ghi = hi + pad;
}

// 1 / q by the hardware reciprocal estimate and two Newton steps.
__device__ __forceinline__ double tri_rcp(double q) {
    double r = __builtin_amdgcn_rcp(q);
    r = __builtin_fma(__builtin_fma(-q, r, 1.0), r, r);
    return __builtin_fma(__builtin_fma(-q, r, 1.0), r, r);
}

// One Sturm step of the bisection: the reciprocal estimate with one Newton step (the
// count needs the pivots' signs; the hardware estimate alone is good to about 2^-24
// relative, one step brings it to about 11 ulp over 4M random inputs, a relative
// perturbation of e^2 far below the eps ||T|| the bisection resolves).
__device__ __forceinline__ double bis_pivot(double dmin, double e2, double q, double pivmin) {
    double r = __builtin_amdgcn_rcp(q);
    r = __builtin_fma(__builtin_fma(-q, r, 1.0), r, r);
    const double v = __builtin_fma(-e2, r, dmin);
    return fabs(v) < pivmin ? -pivmin : v;
}

// lam[c] (c < r) = the c-th largest eigenvalue; info[0..1] = ||T||, pivot floor.  Two
// eigenvalues per workgroup, two waves per eigenvalue, two shifts per lane: a round tests
// 256 shifts and shrinks the bracket 257-fold; the two waves meet in LDS once per round.
__global__ __launch_bounds__(256) void k_tri_bisect(const double* __restrict__ d,
                                                    const double* __restrict__ e, int K, int r,
                                                    double* __restrict__ lam,
                                                    double* __restrict__ info) {
    __shared__ double dl[TRI_MAXK], e2[TRI_MAXK];
    __shared__ double red[12];
    __shared__ int pick[4];
    for (int i = threadIdx.x; i < K; i += blockDim.x) {
        dl[i] = d[i];
        e2[i] = i + 1 < K ? e[i] * e[i] : 0.0;
    }
    double glo, ghi, tnorm, pivmin;
    tri_bounds(d, e, K, red, glo, ghi, tnorm, pivmin);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        info[0] = tnorm;
        info[1] = pivmin;
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int pair = w >> 1, half = w & 1;
    const int c = blockIdx.x * 2 + pair;
    const bool live = c < r;
    const int t = K - 1 - c;                 // ascending index of the eigenvalue
    double lo = glo, hi = ghi;
    // to an absolute accuracy of about eps ||T|| (the accuracy to which the Householder
    // reduction determines the eigenvalues of the Gram matrix)
    const double abstol = 2.220446049250313e-16 * tnorm + pivmin;
    for (int round = 0; round < 12; ++round) {
        const bool done =
            !live || hi - lo <= 2.0 * 2.220446049250313e-16 * fmax(fabs(lo), fabs(hi)) + abstol;
        const double h = (hi - lo) / 257.0;
        int gw = 128;                        // this wave's first shift above t, of 128
        if (!done) {
            // shifts g = 128 half + 2 lane + u, u = 0, 1, at lo + (hi - lo) (g + 1) / 257
            double sg[2], q[2];
            int cnt[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                sg[u] = lo + h * (double)(128 * half + 2 * lane + u + 1);
                q[u] = dl[0] - sg[u];
                if (fabs(q[u]) < pivmin) q[u] = -pivmin;
                cnt[u] = q[u] < 0.0;
            }
            for (int i = 1; i < K; ++i) {
                const double di = dl[i], ei = e2[i - 1];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    q[u] = bis_pivot(di - sg[u], ei, q[u], pivmin);
                    cnt[u] += q[u] < 0.0;
                }
            }
            const int first = cnt[0] >= t + 1 ? 0 : (cnt[1] >= t + 1 ? 1 : 2);
            const unsigned long long above = __ballot(first < 2);
            const int l = above ? __builtin_ctzll(above) : 64;
            const int fl = l < 64 ? __shfl(first, l, 64) : 2;
            gw = l < 64 ? 2 * l + fl : 128;
        }
        if (lane == 0) pick[w] = gw;
        __syncthreads();
        const int g0 = pick[2 * pair], g1 = pick[2 * pair + 1];
        __syncthreads();
        if (!done) {
            const int g = g0 < 128 ? g0 : (g1 < 128 ? 128 + g1 : 256);   // 0..256
            const double nlo = g == 0 ? lo : lo + h * (double)g;
            const double nhi = g == 256 ? hi : lo + h * (double)(g + 1);
            lo = nlo;
            hi = nhi;
        }
    }
    if (live && half == 0 && lane == 0) lam[c] = 0.5 * (lo + hi);
}

// Twisted-factorisation eigenvectors, TW_VPB per workgroup of one wave: lane 2v runs the
// forward factorisation of eigenvector v and lane 2v + 1 the backward one, the pivots
// kept in LDS; the twist index is chosen by the whole wave, then the same two lanes
// extend z below and above it, and the wave normalises.
template <int TW_VPB>
__global__ __launch_bounds__(64) void k_tri_twisted(const double* __restrict__ d,
                                                    const double* __restrict__ e, int K, int r,
                                                    const double* __restrict__ lam,
                                                    const double* __restrict__ info,
                                                    double* __restrict__ Zr) {
    constexpr int TW_MAXK = TW_LDS / TW_VPB;
    __shared__ double dl[TW_MAXK], el[TW_MAXK];
    __shared__ double Dv[TW_VPB][TW_MAXK], Dpv[TW_VPB][TW_MAXK], zv[TW_VPB][TW_MAXK];
    __shared__ int kb_s[TW_VPB];
    const int lane = threadIdx.x;
    for (int i = lane; i < K; i += 64) {
        dl[i] = d[i];
        el[i] = i + 1 < K ? e[i] : 0.0;
    }
    __syncthreads();
    const double pivmin = info[1];
    const int v = lane >> 1, side = lane & 1;
    const int c = blockIdx.x * TW_VPB + v;
    const bool act = v < TW_VPB && c < r;
    const double lm = act ? lam[c] : 0.0;
    if (act) {
        if (side == 0) {
            // forward: T - lm I = L D L^T,  D_{i+1} = (d_{i+1} - lm) - e_i^2 / D_i
            double Dc = dl[0] - lm;
            for (int i = 0; i + 1 < K; ++i) {
                if (fabs(Dc) < pivmin) Dc = pivmin;
                Dv[v][i] = Dc;
                Dc = __builtin_fma(-el[i] * el[i], tri_rcp(Dc), dl[i + 1] - lm);
            }
            Dv[v][K - 1] = Dc;
        } else {
            // backward: T - lm I = U D' U^T,  D'_{i-1} = (d_{i-1} - lm) - e_{i-1}^2 / D'_i
            double Dc = dl[K - 1] - lm;
            for (int i = K - 1; i >= 1; --i) {
                if (fabs(Dc) < pivmin) Dc = pivmin;
                Dpv[v][i] = Dc;
                Dc = __builtin_fma(-el[i - 1] * el[i - 1], tri_rcp(Dc), dl[i - 1] - lm);
            }
            Dpv[v][0] = Dc;
        }
    }
    __syncthreads();
    // twist index of each vector: smallest |gamma_k|, ties to the lowest k (wave argmin)
    for (int vv = 0; vv < TW_VPB; ++vv) {
        const int cc = blockIdx.x * TW_VPB + vv;
        if (cc >= r) break;
        const double lv = lam[cc];
        double best = 1e308;
        int kbest = K;
        for (int k = lane; k < K; k += 64) {
            const double g = fabs(Dv[vv][k] + Dpv[vv][k] - (dl[k] - lv));
            if (g < best) {
                best = g;
                kbest = k;
            }
        }
        for (int off = 32; off >= 1; off >>= 1) {
            const double ob = __shfl_xor(best, off, 64);
            const int ok = __shfl_xor(kbest, off, 64);
            if (ob < best || (ob == best && ok < kbest)) {
                best = ob;
                kbest = ok;
            }
        }
        if (lane == 0) kb_s[vv] = kbest;
    }
    __syncthreads();
    if (act) {
        const int kb = kb_s[v];
        if (side == 0) {
            // below the twist: z_i = -(e_i / D_i) z_{i+1}
            double z = 1.0;
            zv[v][kb] = 1.0;
            for (int i = kb - 1; i >= 0; --i) {
                z = -el[i] * tri_rcp(Dv[v][i]) * z;
                zv[v][i] = z;
            }
        } else {
            // above the twist: z_i = -(e_{i-1} / D'_i) z_{i-1}
            double z = 1.0;
            for (int i = kb + 1; i < K; ++i) {
                z = -el[i - 1] * tri_rcp(Dpv[v][i]) * z;
                zv[v][i] = z;
            }
        }
    }
    __syncthreads();
    for (int vv = 0; vv < TW_VPB; ++vv) {
        const int cc = blockIdx.x * TW_VPB + vv;
        if (cc >= r) break;
        double nn = 0.0;
        for (int k = lane; k < K; k += 64) nn = __builtin_fma(zv[vv][k], zv[vv][k], nn);
        nn = wave_sum(nn);
        const double sc = 1.0 / sqrt(nn);
        for (int k = lane; k < K; k += 64) Zr[(size_t)k * r + cc] = zv[vv][k] * sc;
    }
}

// A reproducible starting vector entry in (-1, 1) for inverse iteration.
__device__ __forceinline__ double tri_start(int i, int t) {
    unsigned long long x = (unsigned long long)(i + 1) * 0x9E3779B97F4A7C15ull ^
                           (unsigned long long)(t + 1) * 0xD1B54A32D192ED03ull;
    x ^= x >> 31;
    x *= 0xBF58476D1CE4E5B9ull;
    x ^= x >> 29;
    return (double)(x >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// Clusters among the top r: consecutive eigenvalues with lam[c] - lam[c+1] <= TRI_CTOL ||T||.
// One wave per cluster (workgroups take clusters blockIdx.x, + gridDim.x, ...): for each
// member t, the tridiagonal LU factorisation of T - lam_t I with partial pivoting (in LDS),
// TRI_ITERS solves from a distinct starting vector, each result orthogonalised against the
// cluster's earlier members and normalised; the member's column of Zr is replaced.
__global__ __launch_bounds__(64) void k_tri_clusters(const double* __restrict__ d,
                                                     const double* __restrict__ e, int K, int r,
                                                     const double* __restrict__ lam,
                                                     const double* __restrict__ info,
                                                     double* __restrict__ Zr) {
    __shared__ double fd[TRI_MAXK], fs1[TRI_MAXK], fs2[TRI_MAXK], fm[TRI_MAXK], x[TRI_MAXK];
    __shared__ unsigned char pv[TRI_MAXK];
    __shared__ int cl_start, cl_end;
    const int lane = threadIdx.x;
    const double tnorm = info[0];
    const double ctol = TRI_CTOL * tnorm;
    const double pert = 2.220446049250313e-16 * fmax(tnorm, 1e-300);
    // no tie at all (the usual case): every lane checks its gaps, the wave leaves
    {
        bool tie = false;
        for (int c = lane; c + 1 < r; c += 64) tie |= lam[c] - lam[c + 1] <= ctol;
        if (!__ballot(tie)) return;
    }
    // the cluster this workgroup takes: count cluster starts in order (lane 0, r steps)
    for (int want = blockIdx.x;; want += gridDim.x) {
        if (lane == 0) {
            int found = -1, cs = 0, ce = 0, idx = 0;
            int c = 0;
            while (c < r) {
                int c1 = c;
                while (c1 + 1 < r && lam[c1] - lam[c1 + 1] <= ctol) ++c1;
                if (c1 > c) {
                    if (idx == want) {
                        found = 1;
                        cs = c;
                        ce = c1;
                        break;
                    }
                    ++idx;
                }
                c = c1 + 1;
            }
            cl_start = found > 0 ? cs : -1;
            cl_end = ce;
        }
        __syncthreads();
        const int cs = cl_start, ce = cl_end;
        __syncthreads();
        if (cs < 0) return;
        for (int t = cs; t <= ce; ++t) {
            const double lm = lam[t];
            // LU with partial pivoting of T - lm I: row i after elimination holds
            // fd[i] (diagonal), fs1[i], fs2[i] (superdiagonals); fm[i] the multiplier of
            // step i, pv[i] whether rows i, i+1 were swapped
            if (lane == 0) {
                double dg = d[0] - lm, s1 = K > 1 ? e[0] : 0.0, s2 = 0.0;
                for (int i = 0; i + 1 < K; ++i) {
                    const double sub = e[i];
                    const double nd = d[i + 1] - lm, ns1 = i + 2 < K ? e[i + 1] : 0.0;
                    if (fabs(sub) > fabs(dg)) {
                        // swap rows i and i + 1
                        const double m = dg / sub;
                        fd[i] = sub;
                        fs1[i] = nd;
                        fs2[i] = ns1;
                        fm[i] = m;
                        pv[i] = 1;
                        dg = s1 - m * nd;
                        s1 = s2 - m * ns1;
                        s2 = 0.0;
                    } else {
                        if (dg == 0.0) dg = pert;
                        const double m = sub / dg;
                        fd[i] = dg;
                        fs1[i] = s1;
                        fs2[i] = s2;
                        fm[i] = m;
                        pv[i] = 0;
                        dg = nd - m * s1;
                        s1 = ns1 - m * s2;
                        s2 = 0.0;
                    }
                }
                fd[K - 1] = dg == 0.0 ? pert : dg;
                fs1[K - 1] = 0.0;
                fs2[K - 1] = 0.0;
            }
            for (int i = lane; i < K; i += 64) x[i] = tri_start(i, t);
            __syncthreads();
            for (int it = 0; it < TRI_ITERS; ++it) {
                if (lane == 0) {
                    // forward elimination of the right-hand side, then back substitution
                    for (int i = 0; i + 1 < K; ++i) {
                        double a = x[i], b = x[i + 1];
                        if (pv[i]) {
                            const double tmp = a;
                            a = b;
                            b = tmp;
                        }
                        x[i] = a;
                        x[i + 1] = b - fm[i] * a;
                    }
                    for (int i = K - 1; i >= 0; --i) {
                        double s = x[i];
                        if (i + 1 < K) s -= fs1[i] * x[i + 1];
                        if (i + 2 < K) s -= fs2[i] * x[i + 2];
                        const double dv = fabs(fd[i]) > pert ? fd[i] : (fd[i] >= 0.0 ? pert : -pert);
                        x[i] = s / dv;
                    }
                }
                __syncthreads();
                // orthogonalise against the cluster's earlier members, then normalise
                for (int s = cs; s < t; ++s) {
                    double dot = 0.0;
                    for (int i = lane; i < K; i += 64) dot = __builtin_fma(Zr[(size_t)i * r + s], x[i], dot);
                    dot = wave_sum(dot);
                    for (int i = lane; i < K; i += 64) x[i] = __builtin_fma(-dot, Zr[(size_t)i * r + s], x[i]);
                    __syncthreads();
                }
                double nn = 0.0;
                for (int i = lane; i < K; i += 64) nn = __builtin_fma(x[i], x[i], nn);
                nn = wave_sum(nn);
                const double sc = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
                for (int i = lane; i < K; i += 64) x[i] *= sc;
                __syncthreads();
            }
            for (int i = lane; i < K; i += 64) Zr[(size_t)i * r + t] = x[i];
            __syncthreads();
        }
    }
}

int tri_eigen_work_elems(int K, int r) { return r + 2; }
int tri_eigen_max_k() { return TW_LDS / 4; }

void launch_tri_eigen(const double* d, const double* e, int K, int r, double* work, double* Zr,
                      hipStream_t st) {
    double* lam = work;
    double* info = work + r;
    hipLaunchKernelGGL(k_tri_bisect, dim3((r + 1) / 2), dim3(256), 0, st, d, e, K, r, lam, info);
    if (K <= TW_LDS / 8)
        hipLaunchKernelGGL(k_tri_twisted<8>, dim3((r + 7) / 8), dim3(64), 0, st, d, e, K, r, lam,
                           info, Zr);
    else
        hipLaunchKernelGGL(k_tri_twisted<4>, dim3((r + 3) / 4), dim3(64), 0, st, d, e, K, r, lam,
                           info, Zr);
    hipLaunchKernelGGL(k_tri_clusters, dim3(32), dim3(64), 0, st, d, e, K, r, lam, info, Zr);
}

// X = I - E/2 + (3/8) E2 for the symmetric correction Z X ~ Z (Z^T Z)^{-1/2}, given
// E = Z^T Z - I (E holds Z^T Z on entry and is turned into E in place, E2 = E E is formed
// by the caller in between: mode 0 subtracts I, mode 1 forms X into E2).
__global__ void k_lowdin(double* __restrict__ E, double* __restrict__ E2, int r, int mode) {
    const size_t total = (size_t)r * r;
    for (size_t x = (size_t)blockIdx.x * blockDim.x + threadIdx.x; x < total;
         x += (size_t)gridDim.x * blockDim.x) {
        const bool diag = x / r == x % r;
        if (mode == 0) {
            if (diag) E[x] -= 1.0;
        } else {
            E2[x] = (diag ? 1.0 : 0.0) - 0.5 * E[x] + 0.375 * E2[x];
        }
    }
}

void launch_lowdin(double* E, double* E2, int r, int mode, hipStream_t st) {
    const size_t total = (size_t)r * r;
    hipLaunchKernelGGL(k_lowdin, dim3((int)std::min<size_t>((total + 255) / 256, 2048)), dim3(256),
                       0, st, E, E2, r, mode);
}

// ------------------------------------------------------------------ back-transformation
// V_r = Q Z_r for the r leading eigenvectors of T: Z holds T's eigenvectors as columns
// (column-major, ascending eigenvalues), so output column c (descending order) starts as
// Z's column K - 1 - c; the reflectors are applied last-to-first, z <- z - tau_j v_j
// (v_j^T z).  Each wave keeps one column in registers (lane l holds rows l + 64 u), so r
// waves run at once; a workgroup stages BT_CHUNK reflectors at a time in LDS for its four
// waves, the next chunk's loads in flight while the current one is applied.  Writes
// Vr (FP32, row-major K x r) and, if asked, rot (FP64, row-major K x r).
constexpr int BT_CHUNK = 8;

template <int U>
__global__ __launch_bounds__(256) void k_backtransform(const double* __restrict__ Z,
                                                       long long zrs, long long zcs,
                                                       const double* __restrict__ Vh,
                                                       const double* __restrict__ tau, int K,
                                                       int r, float* __restrict__ Vr,
                                                       double* __restrict__ rot) {
    constexpr int CH = BT_CHUNK * 64 * U;          // doubles of one staged chunk
    constexpr int PER = (CH + 255) / 256;          // of them loaded per thread
    __shared__ double vs[BT_CHUNK * 64 * U];
    __shared__ double ts[BT_CHUNK];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int col = blockIdx.x * 4 + wave;
    double z[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int k = lane + 64 * u;
        z[u] = (col < r && k < K) ? Z[(long long)k * zrs + (long long)col * zcs] : 0.0;
    }
    // the chunk of reflectors j0, j0 - 1, .. (v_j[j + 1] = 1, zero above) into registers
    double pv[PER], pt = 0.0;
    auto fetch = [&](int j0) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int e = tid + 256 * i;
            const int jj = e / (64 * U), k = e % (64 * U), j = j0 - jj;
            double v = 0.0;
            if (e < CH && j >= 0 && k < K && k >= j + 1) v = (k == j + 1) ? 1.0 : Vh[(size_t)j * K + k];
            pv[i] = v;
        }
        pt = (tid < BT_CHUNK && j0 - tid >= 0) ? tau[j0 - tid] : 0.0;
    };
    fetch(K - 3);
    for (int j0 = K - 3; j0 >= 0; j0 -= BT_CHUNK) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int e = tid + 256 * i;
            if (e < CH) vs[e] = pv[i];
        }
        if (tid < BT_CHUNK) ts[tid] = pt;
        __syncthreads();
        if (j0 - BT_CHUNK >= 0) fetch(j0 - BT_CHUNK);      // in flight during the products
        const int njj = min(BT_CHUNK, j0 + 1);
        for (int jj = 0; jj < njj; ++jj) {
            const double t = ts[jj];
            double vl[U];
#pragma unroll
            for (int u = 0; u < U; ++u) vl[u] = vs[jj * 64 * U + lane + 64 * u];
            double d0 = 0.0;
#pragma unroll
            for (int u = 0; u < U; ++u) d0 = __builtin_fma(vl[u], z[u], d0);
            const double f0 = t * wave_sum(d0);
#pragma unroll
            for (int u = 0; u < U; ++u) z[u] = __builtin_fma(-f0, vl[u], z[u]);
        }
    }
    if (col < r) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = lane + 64 * u;
            if (k < K) {
                Vr[(size_t)k * r + col] = (float)z[u];
                if (rot) rot[(size_t)k * r + col] = z[u];
            }
        }
    }
}

void launch_backtransform(const double* Z, long long zrs, long long zcs, const double* Vh,
                          const double* tau, int K, int r, float* Vr, double* rot,
                          hipStream_t st) {
    const int blocks = (r + 3) / 4;
    const int u = (K + 63) / 64;
#define CAKF_BT(N)                                                                          \
    hipLaunchKernelGGL(k_backtransform<N>, dim3(blocks), dim3(256), 0, st, Z, zrs, zcs, Vh,  \
                       tau, K, r, Vr, rot)
    if (u <= 2) CAKF_BT(2);
    else if (u <= 4) CAKF_BT(4);
    else if (u <= 6) CAKF_BT(6);
    else if (u <= 8) CAKF_BT(8);
    else if (u <= 10) CAKF_BT(10);
    else CAKF_BT(20);
#undef CAKF_BT
}

}  // namespace cakf
