// Image-quality scores of rendered planes against references, for
// evaluating reconstructions (Section 5.2 reports SSIM and PSNR).  Per
// plane: the mean SSIM (Wang et al. 2004; 11 x 11 Gaussian window of
// standard deviation 1.5, weighted population moments, C1 = (0.01 L)^2,
// C2 = (0.03 L)^2) over the window positions that lie inside the image, and
// the MSE over every pixel, from which PSNR = 10 log10(L^2 / MSE).
//
// One wave per 8-pixel-wide column strip of a plane, sliding down it 8 rows
// at a time.  The five moment sums of the row pass (x, y, x^2, y^2, x y
// filtered along the row, FP64) are kept in an LDS ring of 24 rows (three
// groups of 8 starting at row -5), so each step filters only one new group
// and the column pass reads the 18 rows its windows span; the group after
// it is loaded before the column pass and filtered at the next step.  Each
// wave writes its two sums (SSIM over its valid window positions, squared
// differences over its pixels) to a partial array, and a second launch adds
// each plane's strips in a fixed order: the result is deterministic.
#include "ug_kernels.h"

namespace ug {

constexpr int kQRad = 5, kQWin = 2 * kQRad + 1;
constexpr int kQStrip = 8;                   // output columns per wave
constexpr int kQCols = kQStrip + 2 * kQRad;  // input columns a strip reads
constexpr int kQRing = 24;                   // three 8-row groups of row-pass sums
constexpr int kQLoads = (kQStrip * kQCols + 63) / 64;  // loads per lane for 8 input rows

// Row ring slot of image row r (r >= -kQRad).
__device__ __forceinline__ int qslot(int r) { return (r + 2 * kQRing) % kQRing; }

__global__ __launch_bounds__(64) void k_quality_strip(const PlaneInt* __restrict__ pint, uint32_t max_strips,
                                                      const float* __restrict__ img, const float* __restrict__ ref,
                                                      QualityConst q, double2* __restrict__ part) {
  __shared__ double s_h[5][kQRing][kQStrip];        // row-pass sums of the ring's rows
  __shared__ float s_x[kQStrip][kQCols], s_y[kQStrip][kQCols];  // 8 new input rows
  const uint32_t p = blockIdx.y, strip = blockIdx.x;
  const PlaneInt PI = pint[p];
  const int x0 = (int)strip * kQStrip;
  const int lane = (int)threadIdx.x;
  double s_ssim = 0.0, s_se = 0.0;
  if (x0 < PI.W) {  // uniform: the strip has pixels
    const size_t base = ((size_t)PI.pix_off_hi << 32) | PI.pix_off_lo;
    // input rows [ya, ya + 8), columns x0 - 5 .. x0 + 12, zero outside the image
    float ax[kQLoads], ay[kQLoads];
    auto load_rows = [&](int ya) {
#pragma unroll
      for (int k = 0; k < kQLoads; ++k) {
        const int i = lane + 64 * k;
        ax[k] = 0.f;
        ay[k] = 0.f;
        if (i < kQStrip * kQCols) {
          const int y = ya + i / kQCols, x = x0 - kQRad + i % kQCols;
          if (x >= 0 && x < PI.W && y >= 0 && y < PI.H) {
            const size_t idx = base + (size_t)y * (size_t)PI.W + (size_t)x;
            ax[k] = img[idx];
            ay[k] = ref[idx];
          }
        }
      }
    };
    // stores the loaded rows, adds their squared differences (the strip's own
    // columns, rows inside the image) and filters them along the row into the
    // ring
    auto filter_rows = [&](int ya) {
#pragma unroll
      for (int k = 0; k < kQLoads; ++k) {
        const int i = lane + 64 * k;
        if (i < kQStrip * kQCols) {
          const int rr = i / kQCols, cc = i % kQCols;
          s_x[rr][cc] = ax[k];
          s_y[rr][cc] = ay[k];
          const int y = ya + rr, x = x0 - kQRad + cc;
          if (cc >= kQRad && cc < kQRad + kQStrip && x < PI.W && y >= 0 && y < PI.H) {
            const double d = (double)ax[k] - (double)ay[k];
            s_se += d * d;
          }
        }
      }
      wave_lds_sync();
      const int rr = lane / kQStrip, c = lane % kQStrip;  // 64 lanes = 8 rows x 8 columns
      double sx = 0.0, sy = 0.0, sxx = 0.0, syy = 0.0, sxy = 0.0;
#pragma unroll
      for (int t = 0; t < kQWin; ++t) {
        const double a = s_x[rr][c + t], b = s_y[rr][c + t], w = q.taps[t];
        const double wa = w * a, wb = w * b;
        sx += wa;
        sy += wb;
        sxx += wa * a;
        syy += wb * b;
        sxy += wa * b;
      }
      const int sl = qslot(ya + rr);
      s_h[0][sl][c] = sx;
      s_h[1][sl][c] = sy;
      s_h[2][sl][c] = sxx;
      s_h[3][sl][c] = syy;
      s_h[4][sl][c] = sxy;
      wave_lds_sync();
    };
    // groups start at rows -5 + 8 k; the windows of output rows y0 .. y0 + 7
    // (y0 = 8 j) span rows y0 - 5 .. y0 + 12, i.e. groups j, j + 1, j + 2.
    // Rows outside the image filter to zero.
    load_rows(-kQRad);
    filter_rows(-kQRad);
    load_rows(-kQRad + kQStrip);
    filter_rows(-kQRad + kQStrip);
    load_rows(-kQRad + 2 * kQStrip);
    for (int y0 = 0; y0 < PI.H; y0 += kQStrip) {
      filter_rows(y0 - kQRad + 2 * kQStrip);  // group j + 2, loaded at the previous step
      load_rows(y0 - kQRad + 3 * kQStrip);    // group j + 3, for the next step
      const int r = lane / kQStrip, c = lane % kQStrip;
      const int x = x0 + c, y = y0 + r;
      if (x >= kQRad && y >= kQRad && x < PI.W - kQRad && y < PI.H - kQRad) {
        double m[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int t = 0; t < kQWin; ++t) {
          const double w = q.taps[t];
          const int sl = qslot(y - kQRad + t);
#pragma unroll
          for (int j = 0; j < 5; ++j) m[j] += w * s_h[j][sl][c];
        }
        const double mx = m[0], my = m[1];
        const double vx = m[2] - mx * mx, vy = m[3] - my * my, cxy = m[4] - mx * my;
        s_ssim += ((2.0 * mx * my + q.c1) * (2.0 * cxy + q.c2)) / ((mx * mx + my * my + q.c1) * (vx + vy + q.c2));
      }
      wave_lds_sync();  // the next group takes the ring rows of group j
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    s_ssim += __shfl_xor(s_ssim, o, 64);
    s_se += __shfl_xor(s_se, o, 64);
  }
  if (lane == 0) part[(size_t)p * max_strips + strip] = make_double2(s_ssim, s_se);
}

// One block per plane: its strips' sums added in a fixed order.
__global__ __launch_bounds__(256) void k_quality_plane(const PlaneInt* __restrict__ pint,
                                                       const double2* __restrict__ part, uint32_t max_strips,
                                                       double* __restrict__ ssim, double* __restrict__ mse) {
  __shared__ double s_a[256], s_b[256];
  const PlaneInt PI = pint[blockIdx.x];
  const uint32_t ns = (uint32_t)((PI.W + kQStrip - 1) / kQStrip);
  const double2* pp = part + (size_t)blockIdx.x * max_strips;
  double a = 0.0, b = 0.0;
  for (uint32_t i = threadIdx.x; i < ns; i += 256) {
    a += pp[i].x;
    b += pp[i].y;
  }
  s_a[threadIdx.x] = a;
  s_b[threadIdx.x] = b;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      s_a[threadIdx.x] += s_a[threadIdx.x + o];
      s_b[threadIdx.x] += s_b[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double nw = (double)(PI.W - 2 * kQRad) * (double)(PI.H - 2 * kQRad);
    ssim[blockIdx.x] = (PI.W >= kQWin && PI.H >= kQWin) ? s_a[0] / nw : __builtin_nan("");
    mse[blockIdx.x] = s_b[0] / ((double)PI.W * (double)PI.H);
  }
}

uint32_t quality_strips(int32_t max_width) { return (uint32_t)((max_width + kQStrip - 1) / kQStrip); }

hipError_t launch_quality(const PlaneInt* pint, int32_t p, uint32_t max_strips, const float* img, const float* ref,
                          const QualityConst& q, double2* part, double* ssim, double* mse, hipStream_t s) {
  if (p <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_quality_strip, dim3(max_strips, (uint32_t)p), dim3(64), 0, s, pint, max_strips, img, ref, q,
                     part);
  hipLaunchKernelGGL(k_quality_plane, dim3((uint32_t)p), dim3(256), 0, s, pint, part, max_strips, ssim, mse);
  return hipGetLastError();
}

}  // namespace ug
