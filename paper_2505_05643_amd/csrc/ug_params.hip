// The three covariance parameterisations Section 4.2 compares, evaluated
// per Gaussian in float or double: scale and unit quaternion (Sigma =
// R diag(s^2) R^T), a symmetric M with Sigma^-1 = M M^T + beta I (Eq. 10),
// and the triangular L of Eq. 11 (Sigma^-1 = L L^T).  For each route the
// kernel forms what resampling and rendering need: the covariance (written
// out from L^-1 for Eq. 11; the explicit 3x3 inverse for Eq. 10; the
// product for quaternions), a draw F z with F F^T = Sigma (back
// substitution with L^T; the Cholesky factor of the inverted precision;
// R diag(s)), and the squared Mahalanobis distance of an offset.  The float
// instance measures each route's rounding; the double one is its
// reference.  For Eq. 10 the reference inverts the precision through its
// Cholesky factor (error about condition x eps) instead of the adjugate
// the float route uses, whose cofactors cancel terms of the size of the
// largest eigenvalue squared (error about condition^2 x eps, which even in
// double is 1e-4 at an anisotropy of 1000).  One thread per Gaussian,
// contraction off (each operation rounds once, in the order written).
#include <type_traits>

#include "ug_kernels.h"

namespace ug {

template <typename T>
__device__ __forceinline__ T sqrt_t(T x) {
  if constexpr (std::is_same_v<T, float>) {
    return sqrtf(x);
  } else {
    return sqrt(x);
  }
}

// Sigma = L^-T L^-1 of a lower-triangular L, from L^-1 written out.
template <typename T>
__device__ __forceinline__ void tri_covariance(T l11, T l21, T l31, T l22, T l32, T l33, T (&S)[6]) {
#pragma clang fp contract(off)
  const T i11 = (T)1 / l11, i22 = (T)1 / l22, i33 = (T)1 / l33;
  const T i21 = -l21 * i11 * i22;
  const T i32 = -l32 * i22 * i33;
  const T i31 = (l21 * l32 - l22 * l31) * i11 * i22 * i33;
  S[0] = i11 * i11 + i21 * i21 + i31 * i31;
  S[1] = i21 * i22 + i31 * i32;
  S[2] = i31 * i33;
  S[3] = i22 * i22 + i32 * i32;
  S[4] = i32 * i33;
  S[5] = i33 * i33;
}

template <int KIND, typename T>
__global__ __launch_bounds__(256) void k_param_eval(const float* __restrict__ raw, const float* __restrict__ z,
                                                    const float* __restrict__ delta, int64_t n, float beta_f,
                                                    T* __restrict__ sigma, T* __restrict__ draw,
                                                    T* __restrict__ d2) {
#pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const T beta = (T)beta_f;
  T r[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) r[k] = (T)raw[8 * i + k];
  const T z1 = (T)z[3 * i], z2 = (T)z[3 * i + 1], z3 = (T)z[3 * i + 2];
  const T d1 = (T)delta[3 * i], d2v = (T)delta[3 * i + 1], d3 = (T)delta[3 * i + 2];
  T S[6], y[3], q;
  if constexpr (KIND == UG_PARAM_TRI) {
    const T l11 = r[0] * r[0] + beta, l21 = r[1], l31 = r[2];
    const T l22 = r[3] * r[3] + beta, l32 = r[4], l33 = r[5] * r[5] + beta;
    tri_covariance(l11, l21, l31, l22, l32, l33, S);
    // L^-T z by back substitution
    y[2] = z3 / l33;
    y[1] = (z2 - l32 * y[2]) / l22;
    y[0] = (z1 - l21 * y[1] - l31 * y[2]) / l11;
    // |L^T delta|^2
    const T a1 = l11 * d1 + l21 * d2v + l31 * d3, a2 = l22 * d2v + l32 * d3, a3 = l33 * d3;
    q = a1 * a1 + a2 * a2 + a3 * a3;
  } else if constexpr (KIND == UG_PARAM_SYM) {
    const T m11 = r[0], m12 = r[1], m13 = r[2], m22 = r[3], m23 = r[4], m33 = r[5];
    // precision P = M M + beta I (M symmetric)
    const T p11 = m11 * m11 + m12 * m12 + m13 * m13 + beta;
    const T p12 = m11 * m12 + m12 * m22 + m13 * m23;
    const T p13 = m11 * m13 + m12 * m23 + m13 * m33;
    const T p22 = m12 * m12 + m22 * m22 + m23 * m23 + beta;
    const T p23 = m12 * m13 + m22 * m23 + m23 * m33;
    const T p33 = m13 * m13 + m23 * m23 + m33 * m33 + beta;
    if constexpr (std::is_same_v<T, float>) {
      // Sigma = P^-1 = adj(P) / det(P), the explicit inverse
      const T c11 = p22 * p33 - p23 * p23, c12 = p13 * p23 - p12 * p33, c13 = p12 * p23 - p13 * p22;
      const T c22 = p11 * p33 - p13 * p13, c23 = p12 * p13 - p11 * p23, c33 = p11 * p22 - p12 * p12;
      const T det = p11 * c11 + p12 * c12 + p13 * c13;
      const T id = (T)1 / det;
      S[0] = c11 * id;
      S[1] = c12 * id;
      S[2] = c13 * id;
      S[3] = c22 * id;
      S[4] = c23 * id;
      S[5] = c33 * id;
    } else {
      // reference: P = G G^T (Cholesky), Sigma = G^-T G^-1
      const T g11 = sqrt_t(p11);
      const T g21 = p12 / g11, g31 = p13 / g11;
      const T g22 = sqrt_t(p22 - g21 * g21);
      const T g32 = (p23 - g31 * g21) / g22;
      const T g33 = sqrt_t(p33 - g31 * g31 - g32 * g32);
      tri_covariance(g11, g21, g31, g22, g32, g33, S);
    }
    // lower Cholesky factor C of Sigma, y = C z (NaN where a pivot is not positive)
    const T C11 = sqrt_t(S[0]);
    const T C21 = S[1] / C11, C31 = S[2] / C11;
    const T C22 = sqrt_t(S[3] - C21 * C21);
    const T C32 = (S[4] - C31 * C21) / C22;
    const T C33 = sqrt_t(S[5] - C31 * C31 - C32 * C32);
    y[0] = C11 * z1;
    y[1] = C21 * z1 + C22 * z2;
    y[2] = C31 * z1 + C32 * z2 + C33 * z3;
    // |M delta|^2 + beta |delta|^2
    const T b1 = m11 * d1 + m12 * d2v + m13 * d3, b2 = m12 * d1 + m22 * d2v + m23 * d3;
    const T b3 = m13 * d1 + m23 * d2v + m33 * d3;
    q = b1 * b1 + b2 * b2 + b3 * b3 + beta * (d1 * d1 + d2v * d2v + d3 * d3);
  } else {
    // unit quaternion (w, x, y, z) -> R; Sigma = R diag(s^2) R^T
    const T nq = sqrt_t(r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + r[3] * r[3]);
    const T w = r[0] / nq, x = r[1] / nq, yy = r[2] / nq, zz = r[3] / nq;
    T R[3][3];
    R[0][0] = (T)1 - (T)2 * (yy * yy + zz * zz);
    R[0][1] = (T)2 * (x * yy - w * zz);
    R[0][2] = (T)2 * (x * zz + w * yy);
    R[1][0] = (T)2 * (x * yy + w * zz);
    R[1][1] = (T)1 - (T)2 * (x * x + zz * zz);
    R[1][2] = (T)2 * (yy * zz - w * x);
    R[2][0] = (T)2 * (x * zz - w * yy);
    R[2][1] = (T)2 * (yy * zz + w * x);
    R[2][2] = (T)1 - (T)2 * (x * x + yy * yy);
    const T s[3] = {r[4], r[5], r[6]};
    const T s2[3] = {s[0] * s[0], s[1] * s[1], s[2] * s[2]};
    const int jj[6] = {0, 0, 0, 1, 1, 2}, kk[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
    for (int e = 0; e < 6; ++e)
      S[e] = R[jj[e]][0] * s2[0] * R[kk[e]][0] + R[jj[e]][1] * s2[1] * R[kk[e]][1] +
             R[jj[e]][2] * s2[2] * R[kk[e]][2];
    const T sz[3] = {s[0] * z1, s[1] * z2, s[2] * z3};
#pragma unroll
    for (int k = 0; k < 3; ++k) y[k] = R[k][0] * sz[0] + R[k][1] * sz[1] + R[k][2] * sz[2];
    // |diag(1/s) R^T delta|^2
    q = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const T t = (R[0][k] * d1 + R[1][k] * d2v + R[2][k] * d3) / s[k];
      q += t * t;
    }
  }
#pragma unroll
  for (int e = 0; e < 6; ++e) sigma[6 * i + e] = S[e];
#pragma unroll
  for (int k = 0; k < 3; ++k) draw[3 * i + k] = y[k];
  d2[i] = q;
}

template <typename T>
hipError_t launch_param_eval_t(int32_t kind, const float* raw, const float* z, const float* delta, int64_t n,
                               float beta, T* sigma, T* draw, T* d2, hipStream_t s) {
  const dim3 grid((unsigned)((n + 255) / 256)), block(256);
  if (kind == UG_PARAM_TRI)
    hipLaunchKernelGGL((k_param_eval<UG_PARAM_TRI, T>), grid, block, 0, s, raw, z, delta, n, beta, sigma, draw, d2);
  else if (kind == UG_PARAM_SYM)
    hipLaunchKernelGGL((k_param_eval<UG_PARAM_SYM, T>), grid, block, 0, s, raw, z, delta, n, beta, sigma, draw, d2);
  else
    hipLaunchKernelGGL((k_param_eval<UG_PARAM_QUAT, T>), grid, block, 0, s, raw, z, delta, n, beta, sigma, draw,
                       d2);
  return hipGetLastError();
}

hipError_t launch_param_eval(int32_t kind, bool fp64, const float* raw, const float* z, const float* delta,
                             int64_t n, float beta, void* sigma, void* draw, void* d2, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (fp64)
    return launch_param_eval_t<double>(kind, raw, z, delta, n, beta, static_cast<double*>(sigma),
                                       static_cast<double*>(draw), static_cast<double*>(d2), s);
  return launch_param_eval_t<float>(kind, raw, z, delta, n, beta, static_cast<float*>(sigma),
                                    static_cast<float*>(draw), static_cast<float*>(d2), s);
}

}  // namespace ug
