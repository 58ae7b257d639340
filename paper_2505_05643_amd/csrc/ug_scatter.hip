// The paper's own accumulation (Section 4.4, Phase 2) as an alternative to
// the tile-binned gather: every accepted (Gaussian, plane) record adds its
// weight w and w c to per-pixel sums with atomic adds over the pixels of
// its box, then a pass normalises (Eq. 5-7).  The per-pair predicate is
// the same Eq. 12 test as the gather's, so the image agrees with it to
// float rounding; the order of the atomic additions is not fixed, so the
// last bits may differ from run to run.  Forward only: the adjoint needs
// the tile binning.
//
// Work split: one wave per record (a grid-stride loop over records), lanes
// walk the record's pixel box 64 at a time.  The box is the record's tile
// rectangle (from the chosen binning) cut to the ellipse's bounding box,
// padded so float rounding never drops a pixel the per-pair test keeps.
//
// With the paper-literal box support the records hold the exact pixel
// rectangle of their Eq. 13 box and a cut-off of -inf: the same kernel,
// launched with a 1 x 1 "tile", adds every pixel of the rectangle (the
// ellipse cut is skipped because the cut-off is unbounded).
#include "ug_kernels.h"

namespace ug {

// Sums start at zero (a fill kernel, so the step can be graph-captured).
__global__ __launch_bounds__(256) void k_scatter_zero(float* __restrict__ num, float* __restrict__ den,
                                                      uint64_t m) {
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < m; i += (uint64_t)gridDim.x * 256) {
    num[i] = 0.f;
    den[i] = 0.f;
  }
}

__global__ __launch_bounds__(256) void k_scatter(const Ctrl* __restrict__ ctrl, const uint2* __restrict__ rec_pair,
                                                 const PlaneInt* __restrict__ pint, const Rec* __restrict__ recs,
                                                 int TW, int TH,
                                                 float* __restrict__ num, float* __restrict__ den) {
  const uint32_t nrec = ctrl->n_rec_eff;
  const int lane = threadIdx.x & 63;
  const uint32_t nw = gridDim.x * 4u;
  for (uint32_t r = blockIdx.x * 4u + (threadIdx.x >> 6); r < nrec; r += nw) {
    const RecGeo g = recs[r].geo;
    if (g.tx0 > g.tx1 || g.ty0 > g.ty1) continue;  // footprint off the image (uniform)
    const RecAcc A = recs[r].acc;
    const PlaneInt PI = pint[rec_pair[r].y];
    // tile rectangle of the record, cut to the plane
    int u0 = g.tx0 * TW, u1 = min(g.tx1 * TW + TW - 1, PI.W - 1);
    int v0 = g.ty0 * TH, v1 = min(g.ty1 * TH + TH - 1, PI.H - 1);
    // the ellipse (t11 du + t12 dv)^2 + (t22 dv)^2 <= e0 - emin has
    // |dv| <= s / t22 and |du| <= s |(t22, -t12)| / (t11 t22), s = sqrt(e0 - emin)
    const float thr = A.e0 - A.emin;
    if (!(thr >= 0.f)) continue;  // uniform
    if (thr < INFINITY && A.t11 > 0.f && A.t22 > 0.f) {
      const float s = sqrtf(thr);
      const float ve = s / A.t22 * 1.0001f + 0.01f;
      const float ue = s * sqrtf(A.t12 * A.t12 + A.t22 * A.t22) / (A.t11 * A.t22) * 1.0001f + 0.01f;
      const float cu = (float)g.ub + A.fu, cv = (float)g.vb + A.fv;
      if (ue < 1e9f && ve < 1e9f) {
        u0 = max(u0, (int)floorf(cu - ue));
        u1 = min(u1, (int)ceilf(cu + ue));
        v0 = max(v0, (int)floorf(cv - ve));
        v1 = min(v1, (int)ceilf(cv + ve));
      }
    }
    if (u0 > u1 || v0 > v1) continue;
    const uint32_t bw = (uint32_t)(u1 - u0 + 1), npx = bw * (uint32_t)(v1 - v0 + 1);
    const size_t base = ((size_t)PI.pix_off_hi << 32) | PI.pix_off_lo;
    for (uint32_t k = (uint32_t)lane; k < npx; k += 64) {
      const int u = u0 + (int)(k % bw), v = v0 + (int)(k / bw);
      const float du = (float)(u - g.ub) - A.fu, dv = (float)(v - g.vb) - A.fv;
      const float t1 = fmaf(A.t11, du, A.t12 * dv);
      const float t2 = A.t22 * dv;
      const float ee = fmaf(-t1, t1, fmaf(-t2, t2, A.e0));
      if (ee >= A.emin) {
        const float w = __builtin_amdgcn_exp2f(ee);
        const size_t idx = base + (size_t)v * PI.W + u;
        atomicAdd(&num[idx], w * A.c);
        atomicAdd(&den[idx], w);
      }
    }
  }
}

// c_hat = (sum w c + alpha_BG c_BG) / (sum w + alpha_BG), in place; the
// denominator is kept for the record.
__global__ __launch_bounds__(256) void k_scatter_norm(float* __restrict__ image, float* __restrict__ dsave, uint64_t m,
                                                      float bg_alpha, float bg_color) {
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < m; i += (uint64_t)gridDim.x * 256) {
    const float D = dsave[i] + bg_alpha;
    image[i] = (image[i] + bg_alpha * bg_color) / D;
    dsave[i] = D;
  }
}

hipError_t launch_scatter_zero(float* num, float* den, uint64_t m, hipStream_t s) {
  const uint64_t want = (m + 255) / 256;
  const unsigned blocks = (unsigned)(want < 1 ? 1 : (want > 8192 ? 8192 : want));
  hipLaunchKernelGGL(k_scatter_zero, dim3(blocks), dim3(256), 0, s, num, den, m);
  return hipGetLastError();
}

hipError_t launch_scatter(const Ctrl* ctrl, const uint2* rec_pair, const PlaneInt* pint, const Rec* recs,
                          int tile_w, int tile_h, uint32_t rec_cap, float* num, float* den,
                          hipStream_t s) {
  const uint32_t want = (rec_cap + 3u) / 4u;  // four records (waves) per block
  const unsigned blocks = want < 1u ? 1u : (want > 65536u ? 65536u : want);
  hipLaunchKernelGGL(k_scatter, dim3(blocks), dim3(256), 0, s, ctrl, rec_pair, pint, recs, tile_w, tile_h,
                     num, den);
  return hipGetLastError();
}

hipError_t launch_scatter_norm(float* image, float* dsave, uint64_t m, float bg_alpha, float bg_color,
                               hipStream_t s) {
  const uint64_t want = (m + 255) / 256;
  const unsigned blocks = (unsigned)(want < 1 ? 1 : (want > 8192 ? 8192 : want));
  hipLaunchKernelGGL(k_scatter_norm, dim3(blocks), dim3(256), 0, s, image, dsave, m, bg_alpha, bg_color);
  return hipGetLastError();
}

}  // namespace ug
