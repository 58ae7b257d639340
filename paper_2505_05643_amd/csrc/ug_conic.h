// FP64 per-(Gaussian, plane) geometry: Eq. 9 transform, Eq. 11 factor,
// Eq. 12/13 culling and boxes, and the in-plane conic of Eq. 8 restricted
// to the probe plane x3 = 0, plus its adjoint.
//
// Derivation (probe frame of one plane, R = [e1 e2 n], m = R^-1 (mu - o)):
//   d^2(x) = |M (x|0 - m)|^2 with M = L^T R, columns b1, b2, b3.
//   G = M^-T = L^-1 R^-T has columns g_k = L^-1 (row k of R^-1); the
//   probe-frame covariance is Sigma'_jk = g_j . g_k, so the Eq. 13 box
//   half-widths are sqrt(chi^2 Sigma'_kk) (the cofactor-over-determinant of
//   the probe-frame precision) and the plane misses the ellipsoid iff
//   r^2 = m3^2 / Sigma'_33 > chi^2.
//   Restricted to x3 = 0 the quadratic is |R_B (x - c)|^2 + r^2 where
//   R_B = [[T11, T12], [0, T22]] is the Cholesky factor of B^T B, B = [b1 b2]:
//   T11 = |b1|, T12 = b1.b2 / T11, T22 = |b1 x b2| / T11 = |det M| |g3| / T11
//   (b1 x b2 = det(M) g3), and the centre is the conditional mean
//   c = m12 - m3 (Sigma'_13, Sigma'_23) / Sigma'_33.
// Everything is evaluated in double precision from the float32 inputs and
// rounded once into the float32 record.
#pragma once

#include "ug_internal.h"

namespace ug {

// Gaussian parameters in scalar type T (double for the record construction,
// float for its adjoint, whose tolerance is far looser).
template <typename T>
struct GaussT {
  T mu[3];
  T l[6];  // raw (l11, l21, l31, l22, l32, l33)
  T a, c;
  T L11, L21, L31, L22, L32, L33;
  T iL11, iL22, iL33;  // reciprocals of the diagonal
  T alpha, log2a;
  bool finite;
};
using GaussIn = GaussT<double>;

template <typename T>
struct ConicT {
  T m1, m2, m3;
  T g1[3], g2[3], g3[3];
  T b1[3], b2[3];
  T S11, S22, S33, S13, S23, iS;  // iS = 1 / S33
  T T11, T12, T22, detL, n3;
  T c1, c2, r2;
};
using Conic = ConicT<double>;

// Plane pose in scalar type T.
template <typename T>
struct PlaneT {
  T o[3], rinv[9], e1[3], e2[3], absdet, sx, sy;
};

template <typename T>
__device__ __forceinline__ PlaneT<T> plane_as(const PlaneConst& P) {
  PlaneT<T> q;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    q.o[k] = (T)P.o[k];
    q.e1[k] = (T)P.e1[k];
    q.e2[k] = (T)P.e2[k];
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) q.rinv[k] = (T)P.rinv[k];
  q.absdet = (T)P.absdet;
  q.sx = (T)P.sx;
  q.sy = (T)P.sy;
  return q;
}

// A Gaussian's stored parameters as loaded (split from their set-up so a
// kernel can issue the loads early, beside other loads it waits for).
struct GaussRaw {
  float mu[3], l[6], a, c;
};

__device__ __forceinline__ GaussRaw load_gauss_raw(const ug_gaussians& g, int i) {
  GaussRaw r;
#pragma unroll
  for (int k = 0; k < 3; ++k) r.mu[k] = g.means[3 * i + k];
#pragma unroll
  for (int k = 0; k < 6; ++k) r.l[k] = g.lraw[6 * i + k];
  r.a = g.opacity[i];
  r.c = g.intensity[i];
  return r;
}

template <typename T>
__device__ __forceinline__ void gauss_setup(const GaussRaw& r, T beta, GaussT<T>& G) {
  bool fin = true;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    G.mu[k] = (T)r.mu[k];
    fin = fin && __builtin_isfinite(G.mu[k]);
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    G.l[k] = (T)r.l[k];
    fin = fin && __builtin_isfinite(G.l[k]);
  }
  G.a = (T)r.a;
  G.c = (T)r.c;
  fin = fin && __builtin_isfinite(G.a) && __builtin_isfinite(G.c);
  G.finite = fin;
  // Eq. 11: diagonal entries squared plus beta.
  G.L11 = G.l[0] * G.l[0] + beta;
  G.L21 = G.l[1];
  G.L31 = G.l[2];
  G.L22 = G.l[3] * G.l[3] + beta;
  G.L32 = G.l[4];
  G.L33 = G.l[5] * G.l[5] + beta;
  G.iL11 = (T)1 / G.L11;
  G.iL22 = (T)1 / G.L22;
  G.iL33 = (T)1 / G.L33;
  // alpha = sigmoid(a); log2(alpha) = -softplus(-a) / ln 2, stable for any
  // a.  In single precision for both types: the records hold it in float
  // (e0 and emin), so a double evaluation would only cost time.
  const float na = -(float)G.a;
  const float sp = fmaxf(na, 0.f) + log1pf(expf(-fabsf(na)));
  G.log2a = (T)(-sp * (float)(1.0 / kLn2));
  G.alpha = (T)(1.f / (1.f + expf(na)));
}

template <typename T>
__device__ __forceinline__ void load_gauss(const ug_gaussians& g, int i, T beta, GaussT<T>& G) {
  gauss_setup(load_gauss_raw(g, i), beta, G);
}

// Forward substitution y = L^-1 q.
template <typename T>
__device__ __forceinline__ void fsub(const GaussT<T>& G, T q0, T q1, T q2, T* y) {
  y[0] = q0 * G.iL11;
  y[1] = (q1 - G.L21 * y[0]) * G.iL22;
  y[2] = (q2 - G.L31 * y[0] - G.L32 * y[1]) * G.iL33;
}

// Back substitution h = L^-T d.
template <typename T>
__device__ __forceinline__ void bsub(const GaussT<T>& G, const T* d, T* h) {
  h[2] = d[2] * G.iL33;
  h[1] = (d[1] - G.L32 * h[2]) * G.iL22;
  h[0] = (d[0] - G.L21 * h[1] - G.L31 * h[2]) * G.iL11;
}

// Phase 1 of Section 4.4: probe coordinates of the mean and the distance of
// the plane from the ellipsoid.  Returns false if the plane misses the
// chi^2 ellipsoid (|m3| > sqrt(chi^2 Sigma'_33), i.e. r^2 > chi^2).
template <typename T>
__device__ __forceinline__ bool conic_cull(const GaussT<T>& G, const PlaneT<T>& P, T chi2, ConicT<T>& k) {
  const T d0 = G.mu[0] - P.o[0], d1 = G.mu[1] - P.o[1], d2 = G.mu[2] - P.o[2];
  k.m3 = P.rinv[6] * d0 + P.rinv[7] * d1 + P.rinv[8] * d2;
  fsub(G, P.rinv[6], P.rinv[7], P.rinv[8], k.g3);
  k.S33 = k.g3[0] * k.g3[0] + k.g3[1] * k.g3[1] + k.g3[2] * k.g3[2];
  return k.m3 * k.m3 <= chi2 * k.S33;  // false for NaN as well
}

// The rest of the conic, after conic_cull accepted the pair.
template <typename T>
__device__ __forceinline__ void conic_full(const GaussT<T>& G, const PlaneT<T>& P, ConicT<T>& k) {
  const T d0 = G.mu[0] - P.o[0], d1 = G.mu[1] - P.o[1], d2 = G.mu[2] - P.o[2];
  k.m1 = P.rinv[0] * d0 + P.rinv[1] * d1 + P.rinv[2] * d2;
  k.m2 = P.rinv[3] * d0 + P.rinv[4] * d1 + P.rinv[5] * d2;
  fsub(G, P.rinv[0], P.rinv[1], P.rinv[2], k.g1);
  fsub(G, P.rinv[3], P.rinv[4], P.rinv[5], k.g2);
  const T iS = (T)1 / k.S33;
  k.iS = iS;
  k.r2 = k.m3 * k.m3 * iS;
  k.S11 = k.g1[0] * k.g1[0] + k.g1[1] * k.g1[1] + k.g1[2] * k.g1[2];
  k.S22 = k.g2[0] * k.g2[0] + k.g2[1] * k.g2[1] + k.g2[2] * k.g2[2];
  k.S13 = k.g1[0] * k.g3[0] + k.g1[1] * k.g3[1] + k.g1[2] * k.g3[2];
  k.S23 = k.g2[0] * k.g3[0] + k.g2[1] * k.g3[1] + k.g2[2] * k.g3[2];
  // b_k = L^T e_k
  k.b1[0] = G.L11 * P.e1[0] + G.L21 * P.e1[1] + G.L31 * P.e1[2];
  k.b1[1] = G.L22 * P.e1[1] + G.L32 * P.e1[2];
  k.b1[2] = G.L33 * P.e1[2];
  k.b2[0] = G.L11 * P.e2[0] + G.L21 * P.e2[1] + G.L31 * P.e2[2];
  k.b2[1] = G.L22 * P.e2[1] + G.L32 * P.e2[2];
  k.b2[2] = G.L33 * P.e2[2];
  k.T11 = sqrt(k.b1[0] * k.b1[0] + k.b1[1] * k.b1[1] + k.b1[2] * k.b1[2]);
  const T iT11 = (T)1 / k.T11;
  k.T12 = (k.b1[0] * k.b2[0] + k.b1[1] * k.b2[1] + k.b1[2] * k.b2[2]) * iT11;
  k.detL = G.L11 * G.L22 * G.L33;
  k.n3 = sqrt(k.S33);
  k.T22 = k.detL * P.absdet * k.n3 * iT11;
  k.c1 = k.m1 - k.m3 * k.S13 * iS;
  k.c2 = k.m2 - k.m3 * k.S23 * iS;
}

__device__ __forceinline__ double cross_norm2(const double* a, const double* b) {
  const double x = a[1] * b[2] - a[2] * b[1];
  const double y = a[2] * b[0] - a[0] * b[2];
  const double z = a[0] * b[1] - a[1] * b[0];
  return x * x + y * y + z * z;
}

// Inclusive pixel-index range covered by [centre - half, centre + half],
// padded so float rounding never drops a pixel the record's own test keeps.
__device__ __forceinline__ bool pixel_range(double centre, double half, int32_t size, int& lo, int& hi) {
  const double pad = 1e-3 + 1e-5 * half;
  double a = centre - half - pad, b = centre + half + pad;
  if (!(a <= b)) return false;  // NaN
  if (b < 0.0 || a > (double)(size - 1)) return false;
  a = a > 0.0 ? a : 0.0;
  b = b < (double)(size - 1) ? b : (double)(size - 1);
  lo = (int)ceil(a);
  hi = (int)floor(b);
  return lo <= hi;
}

struct Footprint {
  RecAcc acc;
  RecGeo geo;
  uint32_t keys;
  uint32_t spans[kRowSpans];  // ROWS mode: as in Rec
};

// Column ranges of the record's ellipse over bands of pixel rows.  The
// ellipse is (t11 du + t12 dv)^2 + (t22 dv)^2 <= e0 - emin (du, dv relative
// to the record's centre); its right edge is concave in dv and its left edge
// convex, so the extreme columns over a row band sit at the clamped
// stationary points.  The per-record constants are float (relative error
// ~1e-7, far inside the 1e-5 relative padding); the per-band remainders,
// where cancellation happens near the ellipse's top and bottom, are double,
// with their square roots in float.  Contraction is off, so every kernel
// that calls these gets the same answer bit for bit.
struct BandPrep {
  double thr, t12, t22, inv_t11, u0, v0, vext, dvr;
  bool inf;
};

__device__ __forceinline__ bool band_prep(const RecAcc& ra, int ub, int vb, BandPrep& b) {
#pragma clang fp contract(off)
  b.thr = (double)ra.e0 - (double)ra.emin;  // exact
  if (!(b.thr >= 0.0)) return false;
  b.inf = __builtin_isinf(b.thr);
  if (b.inf) return true;
  b.t12 = ra.t12;
  b.t22 = ra.t22;
  b.inv_t11 = (double)(1.0f / ra.t11);
  b.u0 = (double)ub + (double)ra.fu;
  b.v0 = (double)vb + (double)ra.fv;
  const float sq = __builtin_amdgcn_sqrtf((float)b.thr);
  b.vext = (double)(sq / ra.t22) * (1.0 + 1e-6) + 1e-3;
  const float S = __builtin_amdgcn_sqrtf(ra.t12 * ra.t12 + ra.t22 * ra.t22);
  b.dvr = (double)(-ra.t12 * sq / (ra.t22 * S));  // row offset of the rightmost point; the leftmost is -dvr
  return true;
}

// Column range [ua, uz] of the ellipse over pixel rows [ya, yb], clipped to
// [umin, umax] and padded so float rounding in the accumulation never keeps
// a pixel outside it; false if empty.
__device__ __forceinline__ bool band_cols(const BandPrep& b, int ya, int yb, int umin, int umax, int& ua, int& uz) {
#pragma clang fp contract(off)
  if (b.inf) {
    ua = umin;
    uz = umax;
    return umin <= umax;
  }
  double lo = (double)ya - b.v0, hi = (double)yb - b.v0;
  lo = lo > -b.vext ? lo : -b.vext;
  hi = hi < b.vext ? hi : b.vext;
  if (!(lo <= hi)) return false;
  const double dvr = b.dvr < lo ? lo : (b.dvr > hi ? hi : b.dvr);
  const double dvl = -b.dvr < lo ? lo : (-b.dvr > hi ? hi : -b.dvr);
  double qr = b.thr - b.t22 * b.t22 * dvr * dvr;
  double ql = b.thr - b.t22 * b.t22 * dvl * dvl;
  qr = qr > 0.0 ? qr : 0.0;
  ql = ql > 0.0 ? ql : 0.0;
  const double ur = b.u0 + (-b.t12 * dvr + (double)__builtin_amdgcn_sqrtf((float)qr)) * b.inv_t11;
  const double ul = b.u0 + (-b.t12 * dvl - (double)__builtin_amdgcn_sqrtf((float)ql)) * b.inv_t11;
  const double pad = 1e-3 + 1e-5 * (ur - ul);
  double a = ul - pad, c = ur + pad;
  a = a > (double)umin ? a : (double)umin;
  c = c < (double)umax ? c : (double)umax;
  if (!(a <= c)) return false;
  ua = (int)ceil(a);
  uz = (int)floor(c);
  return ua <= uz;
}

// Column ranges of the bands of tile row ty (TH / 8 <= kMaxBands bands) over
// the record's column span [umin, umax].  Empty bands get ua > uz.
constexpr int kMaxBands = 4;
__device__ __forceinline__ void band_ranges(const BandPrep& bp, int ty, int TH, int H, int umin, int umax,
                                            int (&ua)[kMaxBands], int (&uz)[kMaxBands]) {
#pragma unroll
  for (int b = 0; b < kMaxBands; ++b) {
    const int ya = ty * TH + b * kSubBlock;
    const int yb = min(ya + kSubBlock - 1, H - 1);
    ua[b] = 1;
    uz[b] = 0;
    if (b * kSubBlock < TH && ya <= yb) {
      int a, z;
      if (band_cols(bp, ya, yb, umin, umax, a, z)) {
        ua[b] = a;
        uz[b] = z;
      }
    }
  }
}

// Mask of the sub-blocks of tile column tx touched by the band ranges
// (TW / 8 column blocks per band).
__device__ __forceinline__ uint32_t tile_mask(const int (&ua)[kMaxBands], const int (&uz)[kMaxBands], int tx, int TW) {
  const int K = TW / kSubBlock;
  const int x0 = tx * TW;
  uint32_t m = 0;
#pragma unroll
  for (int b = 0; b < kMaxBands; ++b) {
    const int lo = max(ua[b], x0) - x0, hi = min(uz[b], x0 + TW - 1) - x0;
    if (lo <= hi) {
      const uint32_t bits = ((2u << (hi / kSubBlock)) - 1u) & ~((1u << (lo / kSubBlock)) - 1u);
      m |= bits << (b * K);
    }
  }
  return m;
}

// Tile index of pixel index px >= 0 for a tile size T that is a power of two
// (8, 16 or 32): a shift, where an integer division by the runtime T would
// cost a few dozen instructions.
__device__ __forceinline__ int tile_of(int px, int T) { return px >> (31 - __builtin_clz((unsigned)T)); }

// Tiles [tx0, tx1] of tile row ty that a ROWS-mode record covers: those under
// the column range of the ellipse over the whole tile row; false if none.
__device__ __forceinline__ bool rows_span(const BandPrep& bp, int ty, int TW, int TH, int H, int umin, int umax,
                                          int& tx0, int& tx1) {
  const int ya = ty * TH, yb = min(ya + TH - 1, H - 1);
  int ua, uz;
  if (!band_cols(bp, ya, yb, umin, umax, ua, uz)) return false;
  tx0 = tile_of(ua, TW);
  tx1 = tile_of(uz, TW);
  return true;
}

// Key count of a ROWS-mode record over its tile rectangle (rows_span summed
// over its tile rows), and the spans of its first kRowSpans tile rows.
__device__ __forceinline__ uint32_t rows_count(const RecAcc& ra, const RecGeo& geo, int W, int H, int TW, int TH,
                                               uint32_t (&spans)[kRowSpans]) {
#pragma unroll
  for (int i = 0; i < kRowSpans; ++i) spans[i] = kNoSpan;
  const int umin = geo.tx0 * TW;
  const int umax = min(geo.tx1 * TW + TW - 1, W - 1);
  BandPrep bp;
  if (!band_prep(ra, geo.ub, geo.vb, bp)) return 0;
  uint32_t keys = 0;
  for (int ty = geo.ty0; ty <= geo.ty1; ++ty) {
    int tx0, tx1;
    if (rows_span(bp, ty, TW, TH, H, umin, umax, tx0, tx1)) {
      keys += (uint32_t)(tx1 - tx0 + 1);
      const int i = ty - geo.ty0;
#pragma unroll
      for (int k = 0; k < kRowSpans; ++k)
        if (i == k) spans[k] = (uint32_t)tx0 | (uint32_t)tx1 << 16;
    }
  }
  return keys;
}

// The float record of an accepted pair: the in-plane factor scaled to pixel
// units, the conic centre (u0, v0) split into an integer base pixel and a
// fraction, the exponent offset and cut-off, the intensity.
__device__ __forceinline__ void record_conic(const GaussIn& G, const PlaneConst& P, const Conic& k, double chi2,
                                             double u0, double v0, Footprint& f) {
  const double ks = sqrt(kHalfLog2e);
  double ubd = floor(u0 + 0.5), vbd = floor(v0 + 0.5);
  ubd = ubd < -1.0e9 ? -1.0e9 : (ubd > 1.0e9 ? 1.0e9 : ubd);
  vbd = vbd < -1.0e9 ? -1.0e9 : (vbd > 1.0e9 ? 1.0e9 : vbd);
  f.acc.t11 = (float)(ks * k.T11 * P.sx);
  f.acc.t12 = (float)(ks * k.T12 * P.sy);
  f.acc.t22 = (float)(ks * k.T22 * P.sy);
  f.acc.fu = (float)(u0 - ubd);
  f.acc.fv = (float)(v0 - vbd);
  f.acc.e0 = (float)(G.log2a - kHalfLog2e * k.r2);
  f.acc.emin = (float)(G.log2a - kHalfLog2e * chi2);
  f.acc.c = (float)G.c;
  f.geo.ub = (int32_t)ubd;
  f.geo.vb = (int32_t)vbd;
}

// Pixels [lo, hi] (clipped to the image) whose index lies in
// [centre - half, centre + half], edges included, with no padding; false if
// none.
__device__ __forceinline__ bool box_pixels(double centre, double half, int32_t size, int& lo, int& hi) {
  double a = centre - half, b = centre + half;
  if (!(a <= b)) return false;  // NaN
  if (b < 0.0 || a > (double)(size - 1)) return false;
  a = a > 0.0 ? ceil(a) : 0.0;
  b = b < (double)(size - 1) ? floor(b) : (double)(size - 1);
  lo = (int)a;
  hi = (int)b;
  return lo <= hi;
}

// Record of a pair under the paper-literal Phase-2 support (the plane meets
// the Eq. 13 box, decided by the caller): the rectangle fields hold the
// pixels whose centres lie in the in-plane part of the box, b_{1:2} = m_{1:2}
// -/+ sqrt(chi^2 Sigma'_kk), and the cut-off is -inf, so every pixel of the
// rectangle takes its Eq. 8 weight.  Pixel u's centre is at
// (u - cu) sx in the plane, hence the index interval below.  No keys.
__device__ __forceinline__ bool make_box_record(const GaussIn& G, const PlaneConst& P, const PlaneInt& PI,
                                                const Conic& k, double chi2, Footprint& f) {
  int ulo, uhi, vlo, vhi;
  if (!box_pixels(k.m1 / P.sx + P.cu, sqrt(chi2 * k.S11) / P.sx, PI.W, ulo, uhi)) return false;
  if (!box_pixels(k.m2 / P.sy + P.cv, sqrt(chi2 * k.S22) / P.sy, PI.H, vlo, vhi)) return false;
  record_conic(G, P, k, chi2, k.c1 / P.sx + P.cu, k.c2 / P.sy + P.cv, f);
  f.acc.emin = -INFINITY;
  f.geo.tx0 = (uint16_t)ulo;
  f.geo.tx1 = (uint16_t)uhi;
  f.geo.ty0 = (uint16_t)vlo;
  f.geo.ty1 = (uint16_t)vhi;
  f.keys = 0;
  return true;
}

// Record, tile rectangle and key count of an accepted pair (conic_full done).
// Returns false if the footprint misses the image.
__device__ __forceinline__ bool make_footprint(const GaussIn& G, const PlaneConst& P, const PlaneInt& PI,
                                               const Conic& k, double chi2, int box_mode, int TW, int TH,
                                               Footprint& f) {
  const double u0 = k.c1 / P.sx + P.cu;
  const double v0 = k.c2 / P.sy + P.cv;
  int ulo, uhi, vlo, vhi;
  if (box_mode == UG_BOX_PAPER) {
    // Eq. 13: b_{1:2} = m_{1:2} -/+ sqrt(chi^2 Sigma'_kk).
    if (!pixel_range(k.m1 / P.sx + P.cu, sqrt(chi2 * k.S11) / P.sx, PI.W, ulo, uhi)) return false;
    if (!pixel_range(k.m2 / P.sy + P.cv, sqrt(chi2 * k.S22) / P.sy, PI.H, vlo, vhi)) return false;
  } else {
    // Box of the ellipse cut by the plane: conditional variances
    // Sigma'_kk - Sigma'_k3^2 / Sigma'_33 = |g_k x g3|^2 / |g3|^2.
    double q = chi2 - k.r2;
    q = q > 0.0 ? q : 0.0;
    if (!pixel_range(u0, sqrt(q * cross_norm2(k.g1, k.g3) * k.iS) / P.sx, PI.W, ulo, uhi)) return false;
    if (!pixel_range(v0, sqrt(q * cross_norm2(k.g2, k.g3) * k.iS) / P.sy, PI.H, vlo, vhi)) return false;
  }
  record_conic(G, P, k, chi2, u0, v0, f);
  f.geo.tx0 = (uint16_t)tile_of(ulo, TW);
  f.geo.tx1 = (uint16_t)tile_of(uhi, TW);
  f.geo.ty0 = (uint16_t)tile_of(vlo, TH);
  f.geo.ty1 = (uint16_t)tile_of(vhi, TH);
  if (box_mode == UG_BOX_ROWS) {
    f.keys = rows_count(f.acc, f.geo, PI.W, PI.H, TW, TH, f.spans);
  } else {
    f.keys = (uint32_t)(f.geo.tx1 - f.geo.tx0 + 1) * (uint32_t)(f.geo.ty1 - f.geo.ty0 + 1);
  }
  return f.keys > 0;
}

// Adjoint of make_footprint's float record with respect to the Gaussian's
// raw parameters, holding the cut-off set fixed.  dr = (dt11, dt12, dt22,
// dfu, dfv, de0, dc).  Accumulates into dmu[3], dL[6] (L11, L21, L31, L22,
// L32, L33), da, dc.
template <typename T>
__device__ __forceinline__ void footprint_adjoint(const GaussT<T>& G, const PlaneT<T>& P, const ConicT<T>& k,
                                                  const float* dr, T* dmu, T* dL, T& da, T& dc) {
  const T ks = (T)0.84932180028801904272;  // sqrt(log2(e) / 2)
  const T dT11 = ks * P.sx * (T)dr[0];
  const T dT12 = ks * P.sy * (T)dr[1];
  const T dT22 = ks * P.sy * (T)dr[2];
  const T dc1 = (T)dr[3] / P.sx;
  const T dc2 = (T)dr[4] / P.sy;
  const T de0 = (T)dr[5];
  dc += (T)dr[6];
  // e0 = log2(sigmoid(a)) - kHalfLog2e r^2
  da += de0 * ((T)1 - G.alpha) / (T)kLn2;
  const T dr2 = -(T)kHalfLog2e * de0;
  // T22 = detM n3 / T11, T12 = b1.b2 / T11, T11 = |b1|
  const T iT11 = (T)1 / k.T11;
  const T detM = k.detL * P.absdet;
  const T dT11t = dT11 - (dT12 * k.T12 + dT22 * k.T22) * iT11;
  const T ddetL = dT22 * P.absdet * k.n3 * iT11;
  const T dn3 = dT22 * detM * iT11;
  T db1[3], db2[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    db1[j] = (dT11t * k.b1[j] + dT12 * k.b2[j]) * iT11;
    db2[j] = dT12 * k.b1[j] * iT11;
  }
  // c1 = m1 - m3 S13/S33, c2 = m2 - m3 S23/S33, r2 = m3^2 / S33
  const T iS = k.iS;
  T dm[3];
  dm[0] = dc1;
  dm[1] = dc2;
  dm[2] = (-dc1 * k.S13 - dc2 * k.S23 + dr2 * (T)2 * k.m3) * iS;
  const T dS13 = -dc1 * k.m3 * iS;
  const T dS23 = -dc2 * k.m3 * iS;
  const T dS33 = (dc1 * k.m3 * k.S13 + dc2 * k.m3 * k.S23 - dr2 * k.m3 * k.m3) * iS * iS;
  const T in3 = (T)1 / k.n3;
  T dg1[3], dg2[3], dg3[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    dg1[j] = dS13 * k.g3[j];
    dg2[j] = dS23 * k.g3[j];
    dg3[j] = dS13 * k.g1[j] + dS23 * k.g2[j] + (T)2 * dS33 * k.g3[j] + dn3 * k.g3[j] * in3;
  }
  // g = L^-1 q  ->  dL_ij -= h_i g_j with h = L^-T dg (lower triangle)
  T h[3];
  bsub(G, dg1, h);
  dL[0] -= h[0] * k.g1[0]; dL[1] -= h[1] * k.g1[0]; dL[2] -= h[2] * k.g1[0];
  dL[3] -= h[1] * k.g1[1]; dL[4] -= h[2] * k.g1[1]; dL[5] -= h[2] * k.g1[2];
  bsub(G, dg2, h);
  dL[0] -= h[0] * k.g2[0]; dL[1] -= h[1] * k.g2[0]; dL[2] -= h[2] * k.g2[0];
  dL[3] -= h[1] * k.g2[1]; dL[4] -= h[2] * k.g2[1]; dL[5] -= h[2] * k.g2[2];
  bsub(G, dg3, h);
  dL[0] -= h[0] * k.g3[0]; dL[1] -= h[1] * k.g3[0]; dL[2] -= h[2] * k.g3[0];
  dL[3] -= h[1] * k.g3[1]; dL[4] -= h[2] * k.g3[1]; dL[5] -= h[2] * k.g3[2];
  // b_j = sum_i L_ij e_i  ->  dL_ij += e_i db_j
  dL[0] += P.e1[0] * db1[0] + P.e2[0] * db2[0];
  dL[1] += P.e1[1] * db1[0] + P.e2[1] * db2[0];
  dL[2] += P.e1[2] * db1[0] + P.e2[2] * db2[0];
  dL[3] += P.e1[1] * db1[1] + P.e2[1] * db2[1];
  dL[4] += P.e1[2] * db1[1] + P.e2[2] * db2[1];
  dL[5] += P.e1[2] * db1[2] + P.e2[2] * db2[2];
  // detL = L11 L22 L33
  dL[0] += ddetL * G.L22 * G.L33;
  dL[3] += ddetL * G.L11 * G.L33;
  dL[5] += ddetL * G.L11 * G.L22;
  // m = R^-1 (mu - o)  ->  dmu = R^-T dm
#pragma unroll
  for (int j = 0; j < 3; ++j) dmu[j] += P.rinv[j] * dm[0] + P.rinv[3 + j] * dm[1] + P.rinv[6 + j] * dm[2];
}

}  // namespace ug
