// Householder tridiagonalisation of the truncation's FP64 Gram matrix on gfx950 (one
// cooperative launch), the first stage of the symmetric eigensolver behind Truncate
// (Sec. 3.2): G = Q T Q^T with T tridiagonal, Q = H_0 H_1 ... H_{K-3},
// H_j = I - tau_j v_j v_j^T, and the back-transformation Q Z of the leading
// eigenvectors of T.  The tridiagonal eigenproblem itself (divide and conquer) is a
// rocSOLVER call made by the host.
//
// Why one launch: the reduction is a chain of K - 2 dependent steps, each a symmetric
// matrix-vector product with the trailing matrix and a rank-2 update.  As separate
// kernels every step costs several launches; here the K x K matrix is distributed by
// rows over the LDS of a few workgroups (row i lives in workgroup i mod G), each step's
// matrix work is local, and the workgroups exchange only two vectors per step through
// global memory, separated by one grid-wide barrier:
//   after barrier j every workgroup holds v_j, tau_j and reads p_j = tau_j A v_j (each
//   owner wrote its rows' entries) and row j+1 of the matrix before update j (written by
//   its owner); it forms w_j = p_j - (tau_j / 2)(p_j^T v_j) v_j, the updated row j+1
//   (row - v_{j+1} w_j - w_{j+1} v_j) and from it v_{j+1}, tau_{j+1} (identically in
//   every workgroup: same data, same reduction order); then one pass over its own rows
//   applies update j and forms its rows of p_{j+1}; the owner of row j+2 publishes it.
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

constexpr int TD_THREADS = 512;
constexpr int TD_LDS = 12800;           // doubles of matrix rows per workgroup (100 KiB)

int tridiag_max_k() { return TD_MAXK; }

int tridiag_workgroups(int K) {
    const int rows = TD_LDS / K;
    return (K + rows - 1) / rows;
}

__device__ __forceinline__ double td_block_sum(double v, double* red) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < TD_THREADS / 64; ++w) s += red[w];
    __syncthreads();
    return s;
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
__global__ __launch_bounds__(TD_THREADS) void k_tridiag(const double* __restrict__ G, int K,
                                                        double* __restrict__ V,
                                                        double* __restrict__ tau,
                                                        double* __restrict__ d,
                                                        double* __restrict__ e,
                                                        double* __restrict__ pbuf,
                                                        double* __restrict__ rowbuf,
                                                        unsigned* ctr, int* abort_flag) {
    __shared__ double Al[TD_LDS];
    __shared__ double xr[TD_MAXK], vv[TD_MAXK], ww[TD_MAXK];
    __shared__ double red[TD_THREADS / 64];
    const int NWG = gridDim.x, wg = blockIdx.x, tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int nloc = (K - wg + NWG - 1) / NWG;      // rows wg, wg + NWG, ...
    for (int rr = wave; rr < nloc; rr += TD_THREADS / 64)
        for (int k = lane; k < K; k += 64) Al[rr * K + k] = G[(size_t)(wg + rr * NWG) * K + k];
    for (int k = tid; k < K; k += TD_THREADS) xr[k] = G[k];
    __syncthreads();
    // reflector of column 0 from row 0
    double tj = 0.0;
    {
        double s = 0.0;
        for (int k = 2 + tid; k < K; k += TD_THREADS) s += xr[k] * xr[k];
        const double xn2 = td_block_sum(s, red);
        const double alpha = xr[1];
        double beta = alpha, scale = 0.0;
        if (xn2 != 0.0) {
            beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
            tj = (beta - alpha) / beta;
            scale = 1.0 / (alpha - beta);
        }
        for (int k = 1 + tid; k < K; k += TD_THREADS) vv[k] = (k == 1) ? 1.0 : xr[k] * scale;
        if (wg == 0 && tid == 0) {
            d[0] = xr[0];
            e[0] = beta;
            tau[0] = tj;
        }
        __syncthreads();
    }
    for (int rr = wave; rr < nloc; rr += TD_THREADS / 64) {
        const int i = wg + rr * NWG;
        double acc = 0.0;
        if (i > 0)
            for (int k = 1 + lane; k < K; k += 64) acc += Al[rr * K + k] * vv[k];
        acc = wave_sum(acc);
        if (lane == 0 && i > 0) pbuf[i] = tj * acc;
    }
    if (1 % NWG == wg)
        for (int k = 1 + tid; k < K; k += TD_THREADS) rowbuf[k] = Al[(1 / NWG) * K + k];
    for (int j = 0; j < K - 2; ++j) {
        const int b = j & 1;
        // v_j into column j of V, spread over the workgroups
        for (int k = j + 2 + wg * TD_THREADS + tid; k < K; k += NWG * TD_THREADS)
            V[(size_t)j * K + k] = vv[k];
        td_barrier(ctr, (unsigned)(j + 1) * NWG, abort_flag);
        double s2 = 0.0;
        for (int k = j + 1 + tid; k < K; k += TD_THREADS) {
            const double pk = pbuf[b * K + k];
            ww[k] = pk;
            xr[k] = rowbuf[b * K + k];
            s2 += pk * vv[k];
        }
        const double kk = 0.5 * tj * td_block_sum(s2, red);
        for (int k = j + 1 + tid; k < K; k += TD_THREADS) ww[k] -= kk * vv[k];
        __syncthreads();
        // row j+1 after update j (v_j[j+1] = 1), and the reflector of column j+1
        const double w1 = ww[j + 1];
        double s = 0.0;
        for (int k = j + 1 + tid; k < K; k += TD_THREADS) {
            const double x = xr[k] - ww[k] - w1 * vv[k];
            xr[k] = x;
            if (k >= j + 3) s += x * x;
        }
        const double xn2 = td_block_sum(s, red);
        const int j1 = j + 1;
        const double alpha = xr[j1 + 1];
        double beta = alpha, scale = 0.0, tn = 0.0;
        if (xn2 != 0.0) {
            beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
            tn = (beta - alpha) / beta;
            scale = 1.0 / (alpha - beta);
        }
        if (wg == 0 && tid == 0) {
            d[j1] = xr[j1];
            e[j1] = beta;
            tau[j1] = tn;
        }
        // one pass over the own rows: update j, then this row's entry of p_{j+1}
        for (int rr = wave; rr < nloc; rr += TD_THREADS / 64) {
            const int i = wg + rr * NWG;
            if (i <= j) continue;
            const double vi = vv[i], wi = ww[i];
            double acc = 0.0;
            for (int k = j + 1 + lane; k < K; k += 64) {
                const double a = Al[rr * K + k] - (vi * ww[k] + wi * vv[k]);
                Al[rr * K + k] = a;
                if (k > j1) acc += a * ((k == j1 + 1) ? 1.0 : xr[k] * scale);
            }
            acc = wave_sum(acc);
            if (lane == 0 && i > j1) pbuf[(1 - b) * K + i] = tn * acc;
        }
        if ((j1 + 1) % NWG == wg && j1 + 1 < K) {
            __syncthreads();
            const int rr = (j1 + 1) / NWG;
            for (int k = j1 + 1 + tid; k < K; k += TD_THREADS) rowbuf[(1 - b) * K + k] = Al[rr * K + k];
        }
        __syncthreads();
        for (int k = j1 + 1 + tid; k < K; k += TD_THREADS) vv[k] = (k == j1 + 1) ? 1.0 : xr[k] * scale;
        tj = tn;
        __syncthreads();
    }
    const bool failed = __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (wg == 0 && tid == 0) {
        d[K - 2] = failed ? __builtin_nan("") : xr[K - 2];
        e[K - 2] = failed ? __builtin_nan("") : xr[K - 1];
        tau[K - 2] = 0.0;
    }
    if ((K - 1) % NWG == wg && tid == 0)
        d[K - 1] = failed ? __builtin_nan("") : Al[((K - 1) / NWG) * K + K - 1];
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
    return hipLaunchCooperativeKernel((const void*)k_tridiag, dim3(nwg), dim3(TD_THREADS), args,
                                      0, st);
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
        z[u] = (col < r && k < K) ? Z[(size_t)(K - 1 - col) * K + k] : 0.0;
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

void launch_backtransform(const double* Z, const double* Vh, const double* tau, int K, int r,
                          float* Vr, double* rot, hipStream_t st) {
    const int blocks = (r + 3) / 4;
    const int u = (K + 63) / 64;
#define CAKF_BT(N)                                                                          \
    hipLaunchKernelGGL(k_backtransform<N>, dim3(blocks), dim3(256), 0, st, Z, Vh, tau, K, r, \
                       Vr, rot)
    if (u <= 2) CAKF_BT(2);
    else if (u <= 4) CAKF_BT(4);
    else if (u <= 6) CAKF_BT(6);
    else if (u <= 8) CAKF_BT(8);
    else CAKF_BT(10);
#undef CAKF_BT
}

}  // namespace cakf
