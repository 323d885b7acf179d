// soft.h -- cubic-spline softening of the near-field pair force (Sec. 2.4.3).
//
// a_a -= m_b F(r, h_ab) (r_a - r_b), h_ab = (h_a + h_b) / 2, q = r / h_ab:
//   F = h^-3 (4/3 - 6/5 q^2 + 1/2 q^3)                      q < 1
//   F = h^-3 (8/3 - 3 q + 6/5 q^2 - 1/6 q^3) - r^-3 / 15   1 <= q < 2
//   F = r^-3                                               q >= 2
// and, for the backward pass, dF/dr / r:
//   h^-5 (-12/5 + 3/2 q)                                   q < 1
//   h^-5 (12/5 - 1/2 q) - 3 h^-4 / r + r^-5 / 5            1 <= q < 2
//   -3 r^-5                                                q >= 2
// The two inner pieces share one polynomial whose coefficients are selected
// by q < 1 (no branch). Arguments are r^2, h_a + h_b and the caller's powers
// of 1/r.
#pragma once

#include "far_math.h"

namespace rcb {

// smallest normal numbers: below them r^2 counts as 0 (the hardware
// reciprocal square root flushes subnormal inputs to zero and returns inf)
template <typename T>
__device__ __forceinline__ constexpr T r2_min();
template <>
__device__ __forceinline__ constexpr float r2_min<float>() { return 1.17549435e-38f; }
template <>
__device__ __forceinline__ constexpr double r2_min<double>() { return 2.2250738585072014e-308; }

__device__ __forceinline__ float rsq_t(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsq_t(double x) { return rcbfar::rsqrt64(x); }
__device__ __forceinline__ float rcp_t(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_t(double x) { return rcbfar::rcp64(x); }

// True when the pair is certainly outside the kernel support whatever the
// rounding of q: r^2 >= (h_a + h_b)^2 (1 + 2^-16) + r2_min. F is then r^-3
// and dF/dr / r is -3 r^-5, as soft_F and soft_FdF would return them; the
// margin (far above the few-ulp errors of q) keeps the two identical.
template <typename T>
__device__ __forceinline__ bool soft_outside(T r2, T hsum) {
    return r2 >= (hsum * (T)(1.0 + 1.0 / 65536.0)) * hsum + r2_min<T>();
}

// The callers compute rinv = rsq_t(r2), r3 = rinv^3 (and r5 = r3 rinv^2) for
// every pair and call these only for pairs not certainly outside, which reuse
// them. r^2 below r2_min is taken as 0 here (rinv is inf there): q = 0, and
// the pair, whose offset is then zero or below 1e-19, adds nothing.
template <typename T>
__device__ __forceinline__ T soft_F(T r2, T rinv, T r3, T hsum) {
    const T ri = r2 >= r2_min<T>() ? rinv : (T)0;
    const T hinv = (T)2 * rcp_t(hsum);
    const T q = r2 * ri * hinv;
    const T h3 = hinv * hinv * hinv;
    const bool in = q < (T)1;
    const T k0 = in ? (T)(4.0 / 3.0) : (T)(8.0 / 3.0);
    const T k1 = in ? (T)0 : (T)-3;
    const T k2 = in ? (T)(-6.0 / 5.0) : (T)(6.0 / 5.0);
    const T k3 = in ? (T)0.5 : (T)(-1.0 / 6.0);
    const T poly = k0 + q * (k1 + q * (k2 + q * k3));
    const T tail = in ? (T)0 : r3 * (T)(1.0 / 15.0);
    return q < (T)2 ? h3 * poly - tail : r3;
}

template <typename T>
__device__ __forceinline__ void soft_FdF(T r2, T rinv, T r3, T r5, T hsum, T &F, T &dFr) {
    const T ri = r2 >= r2_min<T>() ? rinv : (T)0;
    const T hinv = (T)2 * rcp_t(hsum);
    const T q = r2 * ri * hinv;
    const T h2 = hinv * hinv;
    const T h3 = h2 * hinv;
    const T h4 = h2 * h2;
    const T h5 = h4 * hinv;
    const bool in = q < (T)1, near = q < (T)2;
    const T k0 = in ? (T)(4.0 / 3.0) : (T)(8.0 / 3.0);
    const T k1 = in ? (T)0 : (T)-3;
    const T k2 = in ? (T)(-6.0 / 5.0) : (T)(6.0 / 5.0);
    const T k3 = in ? (T)0.5 : (T)(-1.0 / 6.0);
    const T d0 = in ? (T)(-12.0 / 5.0) : (T)(12.0 / 5.0);
    const T d1 = in ? (T)1.5 : (T)-0.5;
    const T poly = k0 + q * (k1 + q * (k2 + q * k3));
    const T tail = in ? (T)0 : r3 * (T)(1.0 / 15.0);
    const T dtail = in ? (T)0 : (T)0.2 * r5 - (T)3 * h4 * ri;
    F = near ? h3 * poly - tail : r3;
    dFr = near ? h5 * (d0 + d1 * q) + dtail : (T)-3 * r5;
}

}  // namespace rcb
