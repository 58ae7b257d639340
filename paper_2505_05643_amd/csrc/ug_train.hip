// Training-step helpers: the MSE loss gradient and a fused Adam update.
#include "ug_kernels.h"

namespace ug {

constexpr int kMseBlocks = 1024;

// Each block: d_image over a contiguous chunk (a multiple of 1024 pixels)
// and the chunk's squared-error sum (fixed-order tree), written to
// loss[1 + block]; the last block to finish (a counter in
// loss[1 + kMseBlocks], left at zero) adds the block sums in block order in
// double and writes the mean to loss[0].  With 16-byte aligned arrays (vec)
// a thread takes four pixels per step.
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ image, const float* __restrict__ target,
                                             int64_t m, float* __restrict__ d_image, float* __restrict__ loss,
                                             int vec) {
  __shared__ float sh[256];
  __shared__ double shd[256];
  __shared__ bool last;
  const int64_t chunk = ((m + gridDim.x - 1) / gridDim.x + 1023) / 1024 * 1024;
  const int64_t a = (int64_t)blockIdx.x * chunk;
  const int64_t b = a + chunk < m ? a + chunk : m;
  const float scale = 2.0f / (float)m;
  float acc = 0.f;
  if (vec) {
    const int64_t b4 = a < b ? a + (b - a) / 4 * 4 : a;  // whole groups of four
#pragma unroll 4
    for (int64_t i = a + 4 * (int64_t)threadIdx.x; i < b4; i += 1024) {
      const float4 x = *reinterpret_cast<const float4*>(image + i);
      const float4 y = *reinterpret_cast<const float4*>(target + i);
      const float4 d = make_float4(x.x - y.x, x.y - y.y, x.z - y.z, x.w - y.w);
      *reinterpret_cast<float4*>(d_image + i) = make_float4(scale * d.x, scale * d.y, scale * d.z, scale * d.w);
      acc = fmaf(d.x, d.x, acc);
      acc = fmaf(d.y, d.y, acc);
      acc = fmaf(d.z, d.z, acc);
      acc = fmaf(d.w, d.w, acc);
    }
    const int64_t i = b4 + threadIdx.x;  // fewer than four left at the end
    if (i < b) {
      const float d = image[i] - target[i];
      d_image[i] = scale * d;
      acc = fmaf(d, d, acc);
    }
  } else {
    for (int64_t i = a + threadIdx.x; i < b; i += 256) {
      const float d = image[i] - target[i];
      d_image[i] = scale * d;
      acc = fmaf(d, d, acc);
    }
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  unsigned int* counter = reinterpret_cast<unsigned int*>(loss + 1 + kMseBlocks);
  if (threadIdx.x == 0) {
    loss[1 + blockIdx.x] = sh[0];
    __threadfence();
    last = atomicAdd(counter, 1u) == gridDim.x - 1u;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  double s = 0.0;
  for (int i = threadIdx.x; i < (int)gridDim.x; i += 256)
    s += (double)__hip_atomic_load(&loss[1 + i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  shd[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) shd[threadIdx.x] += shd[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    loss[0] = (float)(shd[0] / (double)m);
    *counter = 0u;
  }
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

// Adam over the concatenation [means | lraw | intensity | opacity] (11 n
// floats); the step number comes from device memory.
struct AdamPtrs {
  float* p[4];
  const float* g[4];
  float* m[4];
  float* v[4];
};

__global__ __launch_bounds__(256) void k_adam_gaussians(AdamPtrs A, int64_t n, ug_adam_params hp,
                                                        const int32_t* __restrict__ step_dev,
                                                        const Ctrl* __restrict__ ctrl) {
  if (ctrl && (ctrl->flags & (kFlagRecCap | kFlagKeyCap))) return;
  const int t = *step_dev + 1;
  const float c1 = 1.f / (1.f - powf(hp.beta1, (float)t));
  const float c2 = 1.f / (1.f - powf(hp.beta2, (float)t));
  const float frac = fminf((float)(t - 1) / (float)hp.decay_steps, 1.f);
  const float lr_mu = hp.lr_means * powf(hp.lr_means_final / hp.lr_means, frac);
  const int64_t total = 11 * n;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
    int seg;
    int64_t j;
    if (i < 3 * n) {
      seg = 0;
      j = i;
    } else if (i < 9 * n) {
      seg = 1;
      j = i - 3 * n;
    } else if (i < 10 * n) {
      seg = 2;
      j = i - 9 * n;
    } else {
      seg = 3;
      j = i - 10 * n;
    }
    const float lr = seg == 0 ? lr_mu : hp.lr;
    const float gi = A.g[seg][j];
    const float m = fmaf(hp.beta1, A.m[seg][j], (1.f - hp.beta1) * gi);
    const float v = fmaf(hp.beta2, A.v[seg][j], (1.f - hp.beta2) * gi * gi);
    A.m[seg][j] = m;
    A.v[seg][j] = v;
    A.p[seg][j] -= lr * (m * c1) / (sqrtf(v * c2) + hp.eps);
  }
}

__global__ void k_step_increment(int32_t* __restrict__ step_dev, const Ctrl* __restrict__ ctrl) {
  if (ctrl && (ctrl->flags & (kFlagRecCap | kFlagKeyCap))) return;
  *step_dev += 1;
}

hipError_t launch_adam_gaussians(float* const p[4], const float* const g[4], float* const m[4], float* const v[4],
                                 int64_t n, const ug_adam_params& hp, int32_t* step_dev, const Ctrl* ctrl,
                                 hipStream_t s) {
  AdamPtrs A;
  for (int k = 0; k < 4; ++k) {
    A.p[k] = p[k];
    A.g[k] = g[k];
    A.m[k] = m[k];
    A.v[k] = v[k];
  }
  const int64_t want = (11 * n + 255) / 256;
  const int blocks = (int)(want < 1 ? 1 : (want > 8192 ? 8192 : want));
  hipLaunchKernelGGL(k_adam_gaussians, dim3(blocks), dim3(256), 0, s, A, n, hp, step_dev, ctrl);
  hipLaunchKernelGGL(k_step_increment, dim3(1), dim3(1), 0, s, step_dev, ctrl);
  return hipGetLastError();
}

hipError_t launch_mse(const float* image, const float* target, int64_t m, float* d_image, float* loss,
                      hipStream_t s) {
  int64_t want = (m + 4095) / 4096;  // few blocks: each one's release fence is costly
  const int blocks = (int)(want < 1 ? 1 : (want > kMseBlocks ? kMseBlocks : want));
  const int vec = (reinterpret_cast<uintptr_t>(image) | reinterpret_cast<uintptr_t>(target) |
                   reinterpret_cast<uintptr_t>(d_image)) % 16 == 0;
  hipLaunchKernelGGL(k_mse, dim3(blocks), dim3(256), 0, s, image, target, m, d_image, loss, vec);
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
