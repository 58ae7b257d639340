// Training-step helpers: the MSE loss gradient and a fused Adam update.
#include "ug_kernels.h"

namespace ug {

constexpr int kMseBlocks = 1024;

// Each block: d_image over a contiguous chunk and the chunk's squared-error
// sum (fixed-order tree), written to loss[1 + block].
__global__ __launch_bounds__(256) void k_mse_part(const float* __restrict__ image, const float* __restrict__ target,
                                                  int64_t m, float* __restrict__ d_image, float* __restrict__ loss) {
  __shared__ float sh[256];
  const int64_t chunk = (m + gridDim.x - 1) / gridDim.x;
  const int64_t a = (int64_t)blockIdx.x * chunk;
  const int64_t b = a + chunk < m ? a + chunk : m;
  const float scale = 2.0f / (float)m;
  float acc = 0.f;
  for (int64_t i = a + threadIdx.x; i < b; i += 256) {
    const float d = image[i] - target[i];
    d_image[i] = scale * d;
    acc = fmaf(d, d, acc);
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[1 + blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void k_mse_final(int nparts, int64_t m, float* __restrict__ loss) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nparts; i += 256) acc += (double)loss[1 + i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = (float)(sh[0] / (double)m);
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ mo, float* __restrict__ ve, int64_t n, float lr,
                                              float b1, float b2, float eps, float c1, float c2) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const float gi = g[i];
    const float m = fmaf(b1, mo[i], (1.f - b1) * gi);
    const float v = fmaf(b2, ve[i], (1.f - b2) * gi * gi);
    mo[i] = m;
    ve[i] = v;
    p[i] -= lr * (m * c1) / (sqrtf(v * c2) + eps);
  }
}

hipError_t launch_mse(const float* image, const float* target, int64_t m, float* d_image, float* loss,
                      hipStream_t s) {
  int64_t want = (m + 4095) / 4096;
  const int blocks = (int)(want < 1 ? 1 : (want > kMseBlocks ? kMseBlocks : want));
  hipLaunchKernelGGL(k_mse_part, dim3(blocks), dim3(256), 0, s, image, target, m, d_image, loss);
  hipLaunchKernelGGL(k_mse_final, dim3(1), dim3(256), 0, s, blocks, m, loss);
  return hipGetLastError();
}

hipError_t launch_adam(float* param, const float* grad, float* mo, float* ve, int64_t count, float lr, float b1,
                       float b2, float eps, int32_t t, hipStream_t s) {
  const double c1 = 1.0 / (1.0 - pow((double)b1, (double)t));
  const double c2 = 1.0 / (1.0 - pow((double)b2, (double)t));
  int64_t want = (count + 255) / 256;
  const int blocks = (int)(want < 1 ? 1 : (want > 8192 ? 8192 : want));
  hipLaunchKernelGGL(k_adam, dim3(blocks), dim3(256), 0, s, param, grad, mo, ve, count, lr, b1, b2, eps, (float)c1,
                     (float)c2);
  return hipGetLastError();
}

}  // namespace ug
