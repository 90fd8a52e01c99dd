// Shared device helpers of libcakf (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define CAKF_WAVE 64

namespace cakf {

// Points are stored pre-scaled as float4 by c = log2(e) sqrt(2 nu) / ell, so that the
// scaled distance u' = log2(e) u (u = sqrt(2 nu) d / ell) feeds exp2 directly.
//  Euclidean:    (c x, c y, c z, c^2 |x|^2); a row point is prepared once as
//                (-2 c x, -2 c y, -2 c z, c^2 |x|^2).  Two forms of u'^2 use this layout:
//                the dot-product form w_a + w_b - 2 <a, b> (one add and three FMAs, or one
//                FP32 MFMA per tile) and the difference form |b - a|^2 (three roundings of
//                the differences).  The dot-product form leaves an absolute error of order
//                eps (w_a + w_b) in u'^2, i.e. relative errors up to ~1e-5 in single kernel
//                entries at the lengthscales used here, which ill-conditioned projected Gram
//                matrices amplify to ~2e-5 in the posterior; the difference form keeps every
//                entry within a few ulp.  kval (every FP32 product) takes the difference
//                form; the dot-product form is kept for the BF16 block product and the
//                BF16-mode action loop, whose MFMA distance it allows.
//  Great-circle: (x, y, z, c) with unit (x, y, z) and u' = c theta,
//                theta = 2 arcsin(|x - x'| / 2), the chord form of arccos(<x, x'>) that
//                stays well conditioned for nearby points in FP32.
enum { DIST_EUCLID = 0, DIST_GEODESIC = 1 };

constexpr float LN2 = 0.6931471805599453f;

// Matern(nu) correlation as a function of u' = log2(e) u (unit variance):
//   nu = 1/2 : 2^-u';  nu = 3/2 : (1 + ln2 u') 2^-u';
//   nu = 5/2 : (1 + ln2 u' + ln2^2 u'^2 / 3) 2^-u'.
template <int NU2>
__device__ __forceinline__ float matern_u(float up) {
    const float e = __builtin_amdgcn_exp2f(-up);
    if constexpr (NU2 == 1) {
        return e;
    } else if constexpr (NU2 == 3) {
        return __builtin_fmaf(up * LN2, e, e);
    } else {
        const float p = __builtin_fmaf(up, __builtin_fmaf(up, LN2 * LN2 / 3.0f, LN2), 1.0f);
        return p * e;
    }
}

template <int DIST>
__device__ __forceinline__ float4 prep_row(const float4 a) {
    if constexpr (DIST == DIST_EUCLID) return make_float4(-2.0f * a.x, -2.0f * a.y, -2.0f * a.z, a.w);
    else return a;
}

// u' between a prepared row point and a stored point.
template <int DIST>
__device__ __forceinline__ float scaled_dist(const float4 ap, const float4 b) {
    if constexpr (DIST == DIST_EUCLID) {
        const float t = __builtin_fmaf(ap.x, b.x, __builtin_fmaf(ap.y, b.y,
                        __builtin_fmaf(ap.z, b.z, ap.w + b.w)));
        return __builtin_amdgcn_sqrtf(__builtin_fabsf(t));
    } else {
        const float dx = ap.x - b.x, dy = ap.y - b.y, dz = ap.z - b.z;
        const float h = __builtin_amdgcn_sqrtf(__builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz)));
        return ap.w * 2.0f * asinf(fminf(1.0f, 0.5f * h));
    }
}

// u' from coordinate differences (Euclidean): b - a = b + ap / 2 with one rounding per
// coordinate (ap / 2 = -c a exactly).  Unlike the dot-product form it has no error of order
// sqrt(eps) |x| in u' near u' = 0 and no cancellation against the norms.
__device__ __forceinline__ float scaled_dist_diff(const float4 ap, const float4 b) {
    const float dx = __builtin_fmaf(0.5f, ap.x, b.x);
    const float dy = __builtin_fmaf(0.5f, ap.y, b.y);
    const float dz = __builtin_fmaf(0.5f, ap.z, b.z);
    return __builtin_amdgcn_sqrtf(__builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz)));
}

// Kernel entry k(a, b) for a prepared row point ap = prep_row(a) and a stored point b
// (Euclidean distances in the difference form).
template <int NU2, int DIST>
__device__ __forceinline__ float kval(const float4 ap, const float4 b) {
    if constexpr (DIST == DIST_EUCLID) return matern_u<NU2>(scaled_dist_diff(ap, b));
    else return matern_u<NU2>(scaled_dist<DIST>(ap, b));
}

// Wave-wide sums with the result in every lane.  Within each row of 16 lanes the sum is
// formed with DPP lane permutes (quad swaps, half-row and row mirrors); the four row sums
// are then read out with readlane and added in a fixed order, so the result is
// deterministic and identical in all lanes.
namespace dpp {
constexpr int QUAD_1032 = 0xB1;     // quad_perm [1, 0, 3, 2]
constexpr int QUAD_2301 = 0x4E;     // quad_perm [2, 3, 0, 1]
constexpr int ROW_HALF_MIRROR = 0x141;
constexpr int ROW_MIRROR = 0x140;
template <int CTRL>
__device__ __forceinline__ float perm(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double perm(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xFFFFFFFFLL), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <typename F>
__device__ __forceinline__ F row_sum(F v) {
    v += perm<QUAD_1032>(v);
    v += perm<QUAD_2301>(v);
    v += perm<ROW_HALF_MIRROR>(v);
    v += perm<ROW_MIRROR>(v);
    return v;
}
__device__ __forceinline__ float lane(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double lane(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xFFFFFFFFLL), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
}  // namespace dpp

__device__ __forceinline__ float wave_sum(float v) {
    v = dpp::row_sum(v);
    return (dpp::lane(v, 0) + dpp::lane(v, 16)) + (dpp::lane(v, 32) + dpp::lane(v, 48));
}

__device__ __forceinline__ double wave_sum(double v) {
    v = dpp::row_sum(v);
    return (dpp::lane(v, 0) + dpp::lane(v, 16)) + (dpp::lane(v, 32) + dpp::lane(v, 48));
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
