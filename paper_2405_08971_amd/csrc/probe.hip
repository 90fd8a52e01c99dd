// Issue-rate probes of the VALU instructions the kernel-matrix products are made of
// (measurement support for the roofline figures, not part of the filter): v_exp_f32,
// v_sqrt_f32 and v_fma_f32 in dependent chains, eight independent chains per lane and
// enough waves to fill every SIMD, so that the launch time is set by the issue rate.
#include "cakf_common.h"

namespace cakf {

constexpr int PR_CHAINS = 8;
constexpr int PR_THREADS = 256;

// OP 0: v = exp2(-v) (stays in [0.5, 1]); 1: v = sqrt(v) (tends to 1); 2: v = v a + b.
template <int OP>
__global__ __launch_bounds__(PR_THREADS) void k_rate(float* __restrict__ out, int iters) {
    float v[PR_CHAINS];
#pragma unroll
    for (int c = 0; c < PR_CHAINS; ++c) v[c] = 0.5f + 0.05f * (float)((threadIdx.x + c) & 7);
#pragma unroll 4
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < PR_CHAINS; ++c) {
            if constexpr (OP == 0) v[c] = __builtin_amdgcn_exp2f(-v[c]);
            else if constexpr (OP == 1) v[c] = __builtin_amdgcn_sqrtf(v[c]);
            else v[c] = __builtin_fmaf(v[c], 0.999f, 0.001f);
        }
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < PR_CHAINS; ++c) s += v[c];
    out[blockIdx.x * PR_THREADS + threadIdx.x] = s;
}

// Lane operations per second of each probe on the current device (best of three
// launches).  out: 3 doubles (exp2, sqrt, fma).
hipError_t probe_rates(double* out) {
    int dev = 0, cus = 0;
    hipError_t err = hipGetDevice(&dev);
    if (err == hipSuccess) err = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (err != hipSuccess) return err;
    const int blocks = cus * 16;           // 16 workgroups of 4 waves per CU: 16 waves/SIMD
    const int iters = 2048;
    float* buf = nullptr;
    err = hipMalloc((void**)&buf, (size_t)blocks * PR_THREADS * sizeof(float));
    if (err != hipSuccess) return err;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    for (int op = 0; op < 3 && err == hipSuccess; ++op) {
        float best = 0.0f;
        for (int rep = 0; rep < 4 && err == hipSuccess; ++rep) {
            (void)hipEventRecord(e0, nullptr);
            if (op == 0) hipLaunchKernelGGL(k_rate<0>, dim3(blocks), dim3(PR_THREADS), 0, nullptr, buf, iters);
            else if (op == 1) hipLaunchKernelGGL(k_rate<1>, dim3(blocks), dim3(PR_THREADS), 0, nullptr, buf, iters);
            else hipLaunchKernelGGL(k_rate<2>, dim3(blocks), dim3(PR_THREADS), 0, nullptr, buf, iters);
            (void)hipEventRecord(e1, nullptr);
            err = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
            if (rep > 0 && (best == 0.0f || ms < best)) best = ms;   // the first launch warms up
        }
        out[op] = (double)blocks * PR_THREADS * iters * PR_CHAINS / (best * 1e-3);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(buf);
    return err;
}

}  // namespace cakf
