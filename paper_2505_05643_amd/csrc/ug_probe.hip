// Throughput probes of the chip, for the roofline figures the benchmark
// reports: independent FMA chains (scalar FP32 VALU peak), chains of
// v_exp_f32 (transcendental rate), the forward accumulate's per-pair
// instruction mix with no memory traffic, and a streaming copy (HBM).
// Measurement only; no part of the render or its adjoint.
#include "ug_kernels.h"

namespace ug {

constexpr int kProbeChains = 8;

// 2 flop per FMA, kProbeChains independent chains per thread.
__global__ __launch_bounds__(256) void k_probe_fma(float* __restrict__ out, int iters, float a, float b) {
  float v[kProbeChains];
#pragma unroll
  for (int k = 0; k < kProbeChains; ++k) v[k] = (float)(threadIdx.x + k) * 1e-3f;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < kProbeChains; ++k) v[k] = fmaf(v[k], a, b);
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < kProbeChains; ++k) s += v[k];
  out[(size_t)blockIdx.x * 256 + threadIdx.x] = s;
}

// One v_exp_f32 per step (the negation is a source modifier); values stay
// in [1/2, 1].
__global__ __launch_bounds__(256) void k_probe_exp(float* __restrict__ out, int iters) {
  float v[kProbeChains];
#pragma unroll
  for (int k = 0; k < kProbeChains; ++k) v[k] = (float)((threadIdx.x + k) & 63) * (1.f / 64.f);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < kProbeChains; ++k) v[k] = __builtin_amdgcn_exp2f(-v[k]);
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < kProbeChains; ++k) s += v[k];
  out[(size_t)blockIdx.x * 256 + threadIdx.x] = s;
}

// The forward's pair evaluation (t1, exponent, cut-off, exp2, two sums) on
// register-resident records: kProbeChains pixels per thread, one record per
// iteration whose row term moves by a step each time.
__global__ __launch_bounds__(256) void k_probe_pairs(float* __restrict__ out, int iters, float t11, float emin,
                                                     float c, float dstep) {
  float u[kProbeChains], D[kProbeChains], N[kProbeChains];
#pragma unroll
  for (int k = 0; k < kProbeChains; ++k) {
    u[k] = (float)((threadIdx.x & 7) + 8 * k);
    D[k] = 0.f;
    N[k] = 0.f;
  }
  float B = -4.f, erow = 0.f;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < kProbeChains; ++k) {
      const float t1 = fmaf(t11, u[k], B);
      const float ee = fmaf(-t1, t1, erow);
      const float w = ee >= emin ? __builtin_amdgcn_exp2f(ee) : 0.f;
      D[k] += w;
      N[k] = fmaf(w, c, N[k]);
    }
    B += dstep;
    B = B > 4.f ? -4.f : B;
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < kProbeChains; ++k) s += D[k] + N[k];
  out[(size_t)blockIdx.x * 256 + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_probe_copy(const float4* __restrict__ src, float4* __restrict__ dst,
                                                    size_t n4) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n4; i += (size_t)gridDim.x * 256) dst[i] = src[i];
}

hipError_t launch_probe(int kind, int blocks, int iters, const float* src, float* dst, int64_t n, hipStream_t s) {
  switch (kind) {
    case UG_PROBE_FMA:
      hipLaunchKernelGGL(k_probe_fma, dim3(blocks), dim3(256), 0, s, dst, iters, 0.9999f, 1e-4f);
      break;
    case UG_PROBE_EXP:
      hipLaunchKernelGGL(k_probe_exp, dim3(blocks), dim3(256), 0, s, dst, iters);
      break;
    case UG_PROBE_PAIRS:
      hipLaunchKernelGGL(k_probe_pairs, dim3(blocks), dim3(256), 0, s, dst, iters, 0.3f, -5.6f, 0.5f, 0.01f);
      break;
    case UG_PROBE_COPY:
      hipLaunchKernelGGL(k_probe_copy, dim3(blocks), dim3(256), 0, s, reinterpret_cast<const float4*>(src),
                         reinterpret_cast<float4*>(dst), (size_t)n / 4);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace ug
