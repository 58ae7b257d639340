// Densification and pruning between training steps.  Section 4.2 draws new
// means from a Gaussian through its triangular factor (y = mu + L^-T z, a
// back substitution: no general inverse); the clone / split / prune rule is
// only referenced by the paper, so the one here is a stated choice (see
// include/ug.h, ug_densify).  The decisions are integer outcomes of float32
// arithmetic written out operation by operation with contraction off, so a
// float32 reference reproduces them exactly.
//
// Three launches: per-block counts of the outputs, a one-block scan of the
// block counts (which also publishes the total), and the write, which
// decides again and places each Gaussian's outputs at its block offset plus
// its rank in the block: Gaussian order, deterministic.
#include <cmath>

#include "ug_kernels.h"

namespace ug {

constexpr int kDensifyThreads = 256;

struct DensifyRule {
  float beta, amin, gthr, split2, max2, phi;  // amin = logit(min_opacity); sizes squared
};

// 0 = prune, 1 = keep, 2 = clone, 3 = split (two outputs for 2 and 3).
__device__ __forceinline__ int densify_decide(const float* __restrict__ r, float a, float acc, int32_t cnt,
                                              const DensifyRule& q) {
#pragma clang fp contract(off)
  const float l11 = r[0] * r[0] + q.beta, l21 = r[1], l31 = r[2];
  const float l22 = r[3] * r[3] + q.beta, l32 = r[4], l33 = r[5] * r[5] + q.beta;
  // L^-1, lower triangular, entry by entry; size^2 = trace(Sigma) = |L^-1|_F^2
  const float i11 = 1.f / l11, i22 = 1.f / l22, i33 = 1.f / l33;
  const float i21 = -l21 * i11 * i22;
  const float i32 = -l32 * i22 * i33;
  const float i31 = (l21 * l32 - l22 * l31) * i11 * i22 * i33;
  const float s2 = i11 * i11 + i21 * i21 + i22 * i22 + i31 * i31 + i32 * i32 + i33 * i33;
  if (!(a >= q.amin)) return 0;  // opacity below the floor (or NaN)
  if (q.max2 > 0.f && !(s2 <= q.max2)) return 0;
  if (cnt > 0 && acc >= q.gthr * (float)cnt) return s2 > q.split2 ? 3 : 2;
  return 1;
}

__device__ __forceinline__ uint32_t densify_outputs(int d) { return d == 0 ? 0u : (d == 1 ? 1u : 2u); }

__global__ __launch_bounds__(kDensifyThreads) void k_densify_count(ug_gaussians g, const float* __restrict__ acc,
                                                                   const int32_t* __restrict__ cnt, DensifyRule q,
                                                                   uint32_t* __restrict__ blk) {
  __shared__ uint32_t s_tot;
  if (threadIdx.x == 0) s_tot = 0u;
  __syncthreads();
  const int i = (int)(blockIdx.x * kDensifyThreads + threadIdx.x);
  uint32_t c = 0u;
  if (i < g.n) c = densify_outputs(densify_decide(g.lraw + 6 * (size_t)i, g.opacity[i], acc[i], cnt[i], q));
  if (c) atomicAdd(&s_tot, c);
  __syncthreads();
  if (threadIdx.x == 0) blk[blockIdx.x] = s_tot;
}

// One block: exclusive scan of the block counts in place, the total to
// *count.  Thread t owns a contiguous run of the block counts; the run sums
// are scanned across the block (wave prefix by shuffles, then the 16 wave
// totals), and each thread rewrites its run from its exclusive prefix.
__global__ __launch_bounds__(1024) void k_densify_scan(uint32_t* __restrict__ blk, uint32_t nblk,
                                                       int64_t* __restrict__ count) {
  __shared__ unsigned long long s_wave[16];
  const uint32_t t = threadIdx.x;
  const int lane = (int)(t & 63u), wave = (int)(t >> 6);
  const uint32_t per = (nblk + 1023u) / 1024u;
  const uint32_t b0 = min(t * per, nblk), b1 = min(b0 + per, nblk);
  unsigned long long s = 0;
  for (uint32_t b = b0; b < b1; ++b) s += blk[b];
  unsigned long long x = s;  // inclusive prefix within the wave
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned long long y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) s_wave[wave] = x;
  __syncthreads();
  unsigned long long before = 0, total = 0;
  for (int w = 0; w < 16; ++w) {
    const unsigned long long v = s_wave[w];
    if (w < wave) before += v;
    total += v;
  }
  if (t == 0) *count = (int64_t)total;
  unsigned long long run = before + x - s;
  for (uint32_t b = b0; b < b1; ++b) {
    const uint32_t v = blk[b];
    blk[b] = (uint32_t)run;
    run += v;
  }
}

__global__ __launch_bounds__(kDensifyThreads) void k_densify_write(ug_gaussians g, const float* __restrict__ acc,
                                                                   const int32_t* __restrict__ cnt,
                                                                   const float* __restrict__ z, DensifyRule q,
                                                                   const uint32_t* __restrict__ blk,
                                                                   ug_gaussians_mut out, int64_t cap) {
#pragma clang fp contract(off)
  __shared__ uint32_t s_w[kDensifyThreads / 64];
  const int i = (int)(blockIdx.x * kDensifyThreads + threadIdx.x);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int d = 0;
  if (i < g.n) d = densify_decide(g.lraw + 6 * (size_t)i, g.opacity[i], acc[i], cnt[i], q);
  const uint32_t c = densify_outputs(d);
  // in-block exclusive scan of the output counts
  uint32_t x = c;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) s_w[wave] = x;
  __syncthreads();
  uint32_t before = 0;
  for (int w = 0; w < wave; ++w) before += s_w[w];
  if (!c) return;
  const int64_t o = (int64_t)blk[blockIdx.x] + before + x - c;
  const float* r = g.lraw + 6 * (size_t)i;
  const float mu[3] = {g.means[3 * i], g.means[3 * i + 1], g.means[3 * i + 2]};
  for (uint32_t k = 0; k < c; ++k) {
    const int64_t j = o + k;
    if (j >= cap) break;
    float m[3] = {mu[0], mu[1], mu[2]};
    float rr[6] = {r[0], r[1], r[2], r[3], r[4], r[5]};
    if (d == 3) {
      // Section 4.2: y = mu + L^-T z, back substitution with L^T
      const float l11 = r[0] * r[0] + q.beta, l21 = r[1], l31 = r[2];
      const float l22 = r[3] * r[3] + q.beta, l32 = r[4], l33 = r[5] * r[5] + q.beta;
      const float* zz = z + 6 * (size_t)i + 3 * k;
      const float y3 = zz[2] / l33;
      const float y2 = (zz[1] - l32 * y3) / l22;
      const float y1 = (zz[0] - l21 * y2 - l31 * y3) / l11;
      m[0] += y1;
      m[1] += y2;
      m[2] += y3;
      // L' = phi L (every std divided by phi): diagonal l'^2 + beta = phi (l^2 + beta)
      rr[0] = sqrtf(q.phi * l11 - q.beta);
      rr[1] = q.phi * r[1];
      rr[2] = q.phi * r[2];
      rr[3] = sqrtf(q.phi * l22 - q.beta);
      rr[4] = q.phi * r[4];
      rr[5] = sqrtf(q.phi * l33 - q.beta);
    }
#pragma unroll
    for (int e = 0; e < 3; ++e) out.means[3 * j + e] = m[e];
#pragma unroll
    for (int e = 0; e < 6; ++e) out.lraw[6 * j + e] = rr[e];
    out.intensity[j] = g.intensity[i];
    out.opacity[j] = g.opacity[i];
  }
}

// y[j] = means[idx[j]] + L^-T z[j]; out-of-range indices give NaN.
__global__ __launch_bounds__(256) void k_sample(ug_gaussians g, float beta, const int32_t* __restrict__ idx,
                                                const float* __restrict__ z, int64_t k, float* __restrict__ out) {
#pragma clang fp contract(off)
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < k; j += (int64_t)gridDim.x * 256) {
    const int i = idx[j];
    if (i < 0 || i >= g.n) {
      out[3 * j] = out[3 * j + 1] = out[3 * j + 2] = NAN;
      continue;
    }
    const float* r = g.lraw + 6 * (size_t)i;
    const float l11 = r[0] * r[0] + beta, l21 = r[1], l31 = r[2];
    const float l22 = r[3] * r[3] + beta, l32 = r[4], l33 = r[5] * r[5] + beta;
    const float y3 = z[3 * j + 2] / l33;
    const float y2 = (z[3 * j + 1] - l32 * y3) / l22;
    const float y1 = (z[3 * j] - l21 * y2 - l31 * y3) / l11;
    out[3 * j] = g.means[3 * i] + y1;
    out[3 * j + 1] = g.means[3 * i + 1] + y2;
    out[3 * j + 2] = g.means[3 * i + 2] + y3;
  }
}

// Skipped when the render that produced the gradients overflowed (ctrl).
__global__ __launch_bounds__(256) void k_grad_norm(const Ctrl* __restrict__ ctrl, const float* __restrict__ d_means,
                                                   int32_t n, float* __restrict__ acc, int32_t* __restrict__ cnt) {
  if (ctrl && (ctrl->flags & (kFlagRecCap | kFlagKeyCap))) return;
  for (int i = (int)(blockIdx.x * 256 + threadIdx.x); i < n; i += (int)(gridDim.x * 256)) {
    const float x = d_means[3 * i], y = d_means[3 * i + 1], w = d_means[3 * i + 2];
    acc[i] += sqrtf(x * x + y * y + w * w);
    cnt[i] += 1;
  }
}

uint32_t densify_blocks(int32_t n) { return (uint32_t)((n + kDensifyThreads - 1) / kDensifyThreads); }

hipError_t launch_densify(const ug_gaussians& g, const float* acc, const int32_t* cnt, const float* z,
                          const ug_densify_params& dp, const ug_gaussians_mut& out, int64_t cap, int64_t* count,
                          uint32_t* blk, hipStream_t s) {
  DensifyRule q;
  q.beta = dp.beta;
  const double t = (double)dp.min_opacity;
  q.amin = t <= 0.0 ? -INFINITY : (t >= 1.0 ? INFINITY : (float)std::log(t / (1.0 - t)));
  q.gthr = dp.grad_thresh;
  q.split2 = dp.split_size * dp.split_size;
  q.max2 = dp.max_size * dp.max_size;
  q.phi = dp.split_factor;
  const uint32_t nb = densify_blocks(g.n);
  if (nb > 0)
    hipLaunchKernelGGL(k_densify_count, dim3(nb), dim3(kDensifyThreads), 0, s, g, acc, cnt, q, blk);
  hipLaunchKernelGGL(k_densify_scan, dim3(1), dim3(1024), 0, s, blk, nb, count);
  if (nb > 0)
    hipLaunchKernelGGL(k_densify_write, dim3(nb), dim3(kDensifyThreads), 0, s, g, acc, cnt, z, q, blk, out, cap);
  return hipGetLastError();
}

hipError_t launch_sample(const ug_gaussians& g, float beta, const int32_t* idx, const float* z, int64_t k, float* out,
                         hipStream_t s) {
  if (k <= 0) return hipSuccess;
  const int64_t want = (k + 255) / 256;
  const unsigned blocks = (unsigned)(want > 8192 ? 8192 : want);
  hipLaunchKernelGGL(k_sample, dim3(blocks), dim3(256), 0, s, g, beta, idx, z, k, out);
  return hipGetLastError();
}

hipError_t launch_grad_norm(const Ctrl* ctrl, const float* d_means, int32_t n, float* acc, int32_t* cnt,
                            hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int want = (n + 255) / 256;
  hipLaunchKernelGGL(k_grad_norm, dim3(want > 8192 ? 8192 : want), dim3(256), 0, s, ctrl, d_means, n, acc, cnt);
  return hipGetLastError();
}

}  // namespace ug
