// Image-quality scores of rendered planes against references, for
// evaluating reconstructions (Section 5.2 reports SSIM and PSNR).  Per
// plane: the mean SSIM (Wang et al. 2004; 11 x 11 Gaussian window of
// standard deviation 1.5, weighted population moments, C1 = (0.01 L)^2,
// C2 = (0.03 L)^2) over the window positions that lie inside the image, and
// the MSE over every pixel, from which PSNR = 10 log10(L^2 / MSE).
//
// One wave per 8 x 8 block of pixels of the plan's tiles (grid: tiles x
// sub-blocks per tile).  The wave stages the 18 x 18 patch of both images in
// LDS, filters its rows with the 11 taps (five moment sums in FP64, so
// E[x^2] - mu^2 loses nothing that matters next to C2), then its columns,
// and scores its 64 pixels; the two per-block sums go to a partial array.
// A second launch adds each plane's partials in a fixed order: the result
// is deterministic.
#include "ug_kernels.h"

namespace ug {

constexpr int kQRad = 5, kQWin = 2 * kQRad + 1;
constexpr int kQSub = 8, kQPatch = kQSub + 2 * kQRad;

__global__ __launch_bounds__(64) void k_quality_block(const PlaneInt* __restrict__ pint,
                                                      const uint32_t* __restrict__ tile_plane,
                                                      const uint32_t* __restrict__ tile_org, int TW,
                                                      const float* __restrict__ img, const float* __restrict__ ref,
                                                      QualityConst q, double2* __restrict__ part) {
  __shared__ float s_x[kQPatch * kQPatch], s_y[kQPatch * kQPatch];
  __shared__ double s_h[5][kQPatch * kQSub];
  const uint32_t tile = blockIdx.x;
  const int sub = (int)blockIdx.y, kx = TW / kQSub;
  const PlaneInt PI = pint[tile_plane[tile]];
  const uint32_t org = tile_org[tile];
  const int x0 = (int)(org & 0xffffu) + (sub % kx) * kQSub;
  const int y0 = (int)(org >> 16) + (sub / kx) * kQSub;
  const size_t base = ((size_t)PI.pix_off_hi << 32) | PI.pix_off_lo;
  const int t = (int)threadIdx.x;
  double s_ssim = 0.0, s_se = 0.0;
  if (x0 < PI.W && y0 < PI.H) {  // uniform: the sub-block has pixels
    // patch rows y0-5 .. y0+12, columns x0-5 .. x0+12; zero outside the
    // image (read only by positions whose window is not inside it)
    for (int i = t; i < kQPatch * kQPatch; i += 64) {
      const int y = y0 - kQRad + i / kQPatch, x = x0 - kQRad + i % kQPatch;
      float a = 0.f, b = 0.f;
      if (x >= 0 && x < PI.W && y >= 0 && y < PI.H) {
        const size_t k = base + (size_t)y * (size_t)PI.W + (size_t)x;
        a = img[k];
        b = ref[k];
      }
      s_x[i] = a;
      s_y[i] = b;
    }
    __syncthreads();
    // rows: 18 patch rows x 8 output columns
    for (int i = t; i < kQPatch * kQSub; i += 64) {
      const int r = i / kQSub, c = i % kQSub;
      double sx = 0.0, sy = 0.0, sxx = 0.0, syy = 0.0, sxy = 0.0;
#pragma unroll
      for (int k = 0; k < kQWin; ++k) {
        const double a = s_x[r * kQPatch + c + k], b = s_y[r * kQPatch + c + k], w = q.taps[k];
        const double wa = w * a, wb = w * b;
        sx += wa;
        sy += wb;
        sxx += wa * a;
        syy += wb * b;
        sxy += wa * b;
      }
      s_h[0][i] = sx;
      s_h[1][i] = sy;
      s_h[2][i] = sxx;
      s_h[3][i] = syy;
      s_h[4][i] = sxy;
    }
    __syncthreads();
    // columns and scores: lane t owns pixel (x0 + t % 8, y0 + t / 8)
    const int c = t % kQSub, r = t / kQSub;
    const int x = x0 + c, y = y0 + r;
    if (x < PI.W && y < PI.H) {
      const double d = (double)s_x[(r + kQRad) * kQPatch + c + kQRad] - (double)s_y[(r + kQRad) * kQPatch + c + kQRad];
      s_se = d * d;
      if (x >= kQRad && y >= kQRad && x < PI.W - kQRad && y < PI.H - kQRad) {
        double m[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < kQWin; ++k) {
          const double w = q.taps[k];
#pragma unroll
          for (int j = 0; j < 5; ++j) m[j] += w * s_h[j][(r + k) * kQSub + c];
        }
        const double mx = m[0], my = m[1];
        const double vx = m[2] - mx * mx, vy = m[3] - my * my, cxy = m[4] - mx * my;
        s_ssim = ((2.0 * mx * my + q.c1) * (2.0 * cxy + q.c2)) / ((mx * mx + my * my + q.c1) * (vx + vy + q.c2));
      }
    }
  }
  // wave sums, butterfly order (deterministic)
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    s_ssim += __shfl_xor(s_ssim, o, 64);
    s_se += __shfl_xor(s_se, o, 64);
  }
  if (t == 0) part[(size_t)tile * gridDim.y + blockIdx.y] = make_double2(s_ssim, s_se);
}

// One block per plane: its partials (tiles tile_off .. tile_off + ntx nty - 1,
// all sub-blocks) summed in a fixed order.
__global__ __launch_bounds__(256) void k_quality_plane(const PlaneInt* __restrict__ pint,
                                                       const double2* __restrict__ part, uint32_t subs,
                                                       double* __restrict__ ssim, double* __restrict__ mse) {
  __shared__ double s_a[256], s_b[256];
  const PlaneInt PI = pint[blockIdx.x];
  const size_t b0 = (size_t)PI.tile_off * subs;
  const size_t nb = (size_t)PI.ntx * (size_t)PI.nty * subs;
  double a = 0.0, b = 0.0;
  for (size_t i = threadIdx.x; i < nb; i += 256) {
    const double2 v = part[b0 + i];
    a += v.x;
    b += v.y;
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

uint32_t quality_subs(int tile_w, int tile_h) { return (uint32_t)((tile_w / kQSub) * (tile_h / kQSub)); }

hipError_t launch_quality(const PlaneInt* pint, const uint32_t* tile_plane, const uint32_t* tile_org,
                          uint32_t num_tiles, int32_t p, int tile_w, int tile_h, const float* img, const float* ref,
                          const QualityConst& q, double2* part, double* ssim, double* mse, hipStream_t s) {
  const uint32_t subs = quality_subs(tile_w, tile_h);
  hipLaunchKernelGGL(k_quality_block, dim3(num_tiles, subs), dim3(64), 0, s, pint, tile_plane, tile_org, tile_w, img,
                     ref, q, part);
  hipLaunchKernelGGL(k_quality_plane, dim3((uint32_t)p), dim3(256), 0, s, pint, part, subs, ssim, mse);
  return hipGetLastError();
}

}  // namespace ug
