// Shared device helpers of libcakf (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define CAKF_WAVE 64

namespace cakf {

// Points are stored pre-scaled as float4.  Euclidean distance: (c x, c y, c z, 0) with
// c = sqrt(2 nu) / ell, so that u = sqrt(2 nu) d / ell is the plain Euclidean distance
// of the stored vectors.  Great-circle distance: (x, y, z, c) with unit (x, y, z) and
// u = c * theta, theta = 2 arcsin(|x - x'| / 2) (the angle arccos(<x, x'>) written in
// its chord form, which stays well conditioned for nearby points in FP32).
enum { DIST_EUCLID = 0, DIST_GEODESIC = 1 };

// Matern(nu) correlation as a function of u = sqrt(2 nu) d / ell (unit variance):
//   nu = 1/2 : exp(-u);  nu = 3/2 : (1 + u) exp(-u);  nu = 5/2 : (1 + u + u^2/3) exp(-u).
template <int NU2>
__device__ __forceinline__ float matern_u(float u) {
    const float e = __builtin_amdgcn_exp2f(-u * 1.4426950408889634f);
    if constexpr (NU2 == 1) {
        return e;
    } else if constexpr (NU2 == 3) {
        return __builtin_fmaf(u, e, e);
    } else {
        const float p = __builtin_fmaf(u, __builtin_fmaf(u, 0.333333343f, 1.0f), 1.0f);
        return p * e;
    }
}

template <int DIST>
__device__ __forceinline__ float scaled_dist(const float4 a, const float4 b) {
    if constexpr (DIST == DIST_EUCLID) {
        const float dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z;
        return __builtin_amdgcn_sqrtf(__builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz)));
    } else {
        const float dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z;
        const float h = __builtin_amdgcn_sqrtf(__builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz)));
        return a.w * 2.0f * asinf(fminf(1.0f, 0.5f * h));
    }
}

template <int NU2, int DIST>
__device__ __forceinline__ float kval(const float4 a, const float4 b) {
    return matern_u<NU2>(scaled_dist<DIST>(a, b));
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, CAKF_WAVE);
    return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, CAKF_WAVE);
    return v;
}

}  // namespace cakf

// Dispatch a templated launcher over (kernel, distance).
#define CAKF_DISPATCH_KERNEL(nu2, dist, CALL)                                   \
    do {                                                                        \
        if ((dist) == cakf::DIST_EUCLID) {                                      \
            if ((nu2) == 1) { constexpr int NU2 = 1, DIST = 0; CALL; }          \
            else if ((nu2) == 3) { constexpr int NU2 = 3, DIST = 0; CALL; }     \
            else { constexpr int NU2 = 5, DIST = 0; CALL; }                     \
        } else {                                                                \
            if ((nu2) == 1) { constexpr int NU2 = 1, DIST = 1; CALL; }          \
            else if ((nu2) == 3) { constexpr int NU2 = 3, DIST = 1; CALL; }     \
            else { constexpr int NU2 = 5, DIST = 1; CALL; }                     \
        }                                                                       \
    } while (0)
