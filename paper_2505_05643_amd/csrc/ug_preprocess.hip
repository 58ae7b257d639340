// Preprocess kernels: plane set-up, the Phase-1 cull with record counting
// (Section 4.4), record writing, key emission (tile binning), and the
// per-Gaussian adjoint of the record construction.
#include "ug_conic.h"
#include "ug_kernels.h"

namespace ug {

// ---------------------------------------------------------------- plane set-up
// One thread per plane: FP64 constants of the pose (an invalid pose is
// marked and skipped by the count pass, which raises the flag); thread 0
// clears the control block of this render.
__global__ __launch_bounds__(256) void k_init(ug_planes pl, const PlaneInt* __restrict__ pint,
                                              PlaneConst* __restrict__ pc, Ctrl* __restrict__ ctrl) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p == 0) {
    ctrl->n_rec = 0;
    ctrl->n_key = 0;
    ctrl->n_eval = 0;
    ctrl->flags = 0;
    ctrl->n_rec_eff = 0;
    ctrl->n_key_eff = 0;
  }
  if (p >= pl.p) return;
  double R[9];
  bool fin = true;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    R[k] = (double)pl.rot[9 * p + k];
    fin = fin && isfinite_d(R[k]);
  }
  PlaneConst c;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    c.o[k] = (double)pl.origin[3 * p + k];
    fin = fin && isfinite_d(c.o[k]);
    c.e1[k] = R[3 * k + 0];
    c.e2[k] = R[3 * k + 1];
  }
  c.sx = (double)pl.spacing[2 * p + 0];
  c.sy = (double)pl.spacing[2 * p + 1];
  fin = fin && isfinite_d(c.sx) && isfinite_d(c.sy) && c.sx > 0.0 && c.sy > 0.0;
  // R^-1 = adj(R) / det(R)
  const double a = R[0], b = R[1], cc = R[2], d = R[3], e = R[4], f = R[5], g = R[6], h = R[7], i = R[8];
  const double A = e * i - f * h, B = -(d * i - f * g), C = d * h - e * g;
  const double det = a * A + b * B + cc * C;
  fin = fin && isfinite_d(det) && det > 0.0;
  const double id = 1.0 / det;
  c.rinv[0] = A * id;
  c.rinv[1] = -(b * i - cc * h) * id;
  c.rinv[2] = (b * f - cc * e) * id;
  c.rinv[3] = B * id;
  c.rinv[4] = (a * i - cc * g) * id;
  c.rinv[5] = -(a * f - cc * d) * id;
  c.rinv[6] = C * id;
  c.rinv[7] = -(a * h - b * g) * id;
  c.rinv[8] = (a * e - b * d) * id;
  c.absdet = fabs(det);
  c.cu = 0.5 * (double)pint[p].W - 0.5;
  c.cv = 0.5 * (double)pint[p].H - 0.5;
  c.valid = fin ? 1 : 0;
  c.pad = 0;
  pc[p] = c;
}

// ---------------------------------------------------------------- block scans
// Exclusive scan of one uint32 per thread over a 256-thread block.
__device__ __forceinline__ uint32_t block_exscan_256(uint32_t v, uint32_t* sh /*[4]*/, uint32_t& total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh[wave] = x;
  __syncthreads();
  uint32_t before = 0;
  total = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const uint32_t s = sh[w];
    if (w < wave) before += s;
    total += s;
  }
  __syncthreads();
  return before + x - v;
}

// ---------------------------------------------------------------- count pass
// One thread per Gaussian, looping over all planes: Phase-1 cull, then the
// footprint's key count.  Writes per-Gaussian counts and per-block sums.
__global__ __launch_bounds__(256) void k_count(ug_gaussians g, const PlaneConst* __restrict__ pc,
                                               const PlaneInt* __restrict__ pint, RenderParams rp,
                                               uint32_t* __restrict__ cnt_rec, uint32_t* __restrict__ cnt_key,
                                               uint32_t* __restrict__ blk_rec, uint32_t* __restrict__ blk_key,
                                               Ctrl* __restrict__ ctrl) {
  __shared__ uint32_t sh[8];
  const int i = blockIdx.x * 256 + threadIdx.x;
  uint32_t nr = 0, nk = 0;
  if (i < rp.n) {
    GaussIn G;
    load_gauss(g, i, (double)rp.beta, G);
    if (!G.finite) {
      atomicOr(&ctrl->flags, kFlagNonfinite);
    } else {
      const double chi2 = (double)rp.chi2;
      bool bad_plane = false;
      for (int p = 0; p < rp.p; ++p) {
        if (!pc[p].valid) {
          bad_plane = true;
          continue;
        }
        const PlaneConst& P = pc[p];
        Conic k;
        if (!conic_cull(G, P, chi2, k)) continue;
        conic_full(G, P, k);
        Footprint f;
        if (!make_footprint(G, P, pint[p], k, chi2, rp.box_mode, rp.tile_w, rp.tile_h, f)) continue;
        nr += 1;
        nk += f.keys;
      }
      if (bad_plane && i == 0) atomicOr(&ctrl->flags, kFlagNonfinite);
    }
    cnt_rec[i] = nr;
    cnt_key[i] = nk;
  }
  uint32_t tr, tk;
  block_exscan_256(nr, sh, tr);
  block_exscan_256(nk, sh + 4, tk);
  if (threadIdx.x == 0) {
    blk_rec[blockIdx.x] = tr;
    blk_key[blockIdx.x] = tk;
  }
}

// ---------------------------------------------------------------- top scan
// Single block: exclusive scan of the per-block sums (64-bit), totals,
// capacity check.
__global__ __launch_bounds__(1024) void k_top_scan(const uint32_t* __restrict__ blk_rec,
                                                   const uint32_t* __restrict__ blk_key,
                                                   unsigned long long* __restrict__ blk_rec_off,
                                                   unsigned long long* __restrict__ blk_key_off, int nblk,
                                                   Ctrl* __restrict__ ctrl, uint32_t rec_cap, uint32_t key_cap,
                                                   uint32_t* __restrict__ rec_koff) {
  __shared__ unsigned long long sr[1024], sk[1024];
  const int t = threadIdx.x;
  const int per = (nblk + 1023) / 1024;
  const int b0 = t * per, b1 = min(b0 + per, nblk);
  unsigned long long r = 0, k = 0;
  for (int b = b0; b < b1; ++b) {
    r += blk_rec[b];
    k += blk_key[b];
  }
  sr[t] = r;
  sk[t] = k;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const unsigned long long ar = t >= o ? sr[t - o] : 0ull;
    const unsigned long long ak = t >= o ? sk[t - o] : 0ull;
    __syncthreads();
    sr[t] += ar;
    sk[t] += ak;
    __syncthreads();
  }
  unsigned long long er = sr[t] - r, ek = sk[t] - k;
  for (int b = b0; b < b1; ++b) {
    blk_rec_off[b] = er;
    blk_key_off[b] = ek;
    er += blk_rec[b];
    ek += blk_key[b];
  }
  if (t == 1023) {
    const unsigned long long nr = sr[1023], nk = sk[1023];
    ctrl->n_rec = nr;
    ctrl->n_key = nk;
    unsigned f = 0;
    if (nr > rec_cap) f |= kFlagRecCap;
    if (nk > key_cap) f |= kFlagKeyCap;
    if (f) atomicOr(&ctrl->flags, f);
    const bool ok = (f == 0);
    ctrl->n_rec_eff = ok ? (uint32_t)nr : 0u;
    ctrl->n_key_eff = ok ? (uint32_t)nk : 0u;
    if (rec_koff) rec_koff[ok ? nr : 0] = ok ? (uint32_t)nk : 0u;
  }
}

// ---------------------------------------------------------------- write pass
// Same blocking as k_count.  Each thread recomputes its accepted pairs and
// writes them Gaussian-major at its scanned offsets.
__global__ __launch_bounds__(256) void k_write(ug_gaussians g, const PlaneConst* __restrict__ pc,
                                               const PlaneInt* __restrict__ pint, RenderParams rp,
                                               const uint32_t* __restrict__ cnt_rec,
                                               const uint32_t* __restrict__ cnt_key,
                                               const unsigned long long* __restrict__ blk_rec_off,
                                               const unsigned long long* __restrict__ blk_key_off,
                                               uint32_t* __restrict__ off_rec, RecAcc* __restrict__ racc,
                                               RecGeo* __restrict__ rgeo, uint32_t* __restrict__ rec_pid,
                                               uint32_t* __restrict__ rec_koff) {
  __shared__ uint32_t sh[8];
  const int i = blockIdx.x * 256 + threadIdx.x;
  const uint32_t nr = i < rp.n ? cnt_rec[i] : 0u;
  const uint32_t nk = i < rp.n ? cnt_key[i] : 0u;
  uint32_t tr, tk;
  const uint32_t er = block_exscan_256(nr, sh, tr);
  const uint32_t ek = block_exscan_256(nk, sh + 4, tk);
  if (i >= rp.n) return;
  unsigned long long r = blk_rec_off[blockIdx.x] + er;
  unsigned long long kk = blk_key_off[blockIdx.x] + ek;
  off_rec[i] = (uint32_t)(r < rp.rec_cap ? r : rp.rec_cap);
  if (nr == 0) return;
  GaussIn G;
  load_gauss(g, i, (double)rp.beta, G);
  const double chi2 = (double)rp.chi2;
  uint32_t written = 0;
  for (int p = 0; p < rp.p && written < nr; ++p) {
    if (!pc[p].valid) continue;
    const PlaneConst& P = pc[p];
    Conic k;
    if (!conic_cull(G, P, chi2, k)) continue;
    conic_full(G, P, k);
    Footprint f;
    if (!make_footprint(G, P, pint[p], k, chi2, rp.box_mode, rp.tile_w, rp.tile_h, f)) continue;
    if (r < rp.rec_cap) {
      racc[r] = f.acc;
      rgeo[r] = f.geo;
      rec_pid[r] = (uint32_t)p;
      rec_koff[r] = (uint32_t)(kk < rp.key_cap ? kk : rp.key_cap);
    }
    ++r;
    ++written;
    kk += f.keys;
  }
}

// ---------------------------------------------------------------- key emission
// One thread per record: (global tile id, emission index) for every tile the
// footprint covers, in row-major tile order.
__global__ __launch_bounds__(256) void k_emit(const Ctrl* __restrict__ ctrl, const RecAcc* __restrict__ racc,
                                              const RecGeo* __restrict__ rgeo,
                                              const uint32_t* __restrict__ rec_pid,
                                              const uint32_t* __restrict__ rec_koff,
                                              const PlaneInt* __restrict__ pint, RenderParams rp,
                                              uint32_t* __restrict__ key_tile, uint32_t* __restrict__ rec_of_key) {
  const uint32_t nrec = ctrl->n_rec_eff;
  const int TW = rp.tile_w, TH = rp.tile_h;
  for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < nrec; r += gridDim.x * blockDim.x) {
    const RecGeo geo = rgeo[r];
    uint32_t pid = rec_pid[r];
    uint32_t e = rec_koff[r];
    const uint32_t e_end = rec_koff[r + 1];
    if (pid >= (uint32_t)rp.p) {  // never: the write pass stores every record
      atomicOr(const_cast<unsigned int*>(&ctrl->flags), kFlagInternal);
      pid = 0;
    }
    const PlaneInt PI = pint[pid];
    if (rp.box_mode != UG_BOX_ROWS) {
      for (int ty = geo.ty0; ty <= geo.ty1; ++ty) {
        const uint32_t rowbase = PI.tile_off + (uint32_t)ty * (uint32_t)PI.ntx;
        for (int tx = geo.tx0; tx <= geo.tx1; ++tx) {
          if (e < e_end) {
            key_tile[e] = rowbase + (uint32_t)tx;
            rec_of_key[e] = r;
          }
          ++e;
        }
      }
    } else {
      const RecAcc ra = racc[r];
      const int umin = geo.tx0 * TW;
      const int umax = min(geo.tx1 * TW + TW - 1, PI.W - 1);
      for (int ty = geo.ty0; ty <= geo.ty1; ++ty) {
        const int ya = ty * TH, yb = min(ya + TH - 1, PI.H - 1);
        int ua, uz;
        if (!rows_band(ra, geo.ub, geo.vb, ya, yb, umin, umax, ua, uz)) continue;
        const uint32_t rowbase = PI.tile_off + (uint32_t)ty * (uint32_t)PI.ntx;
        for (int tx = ua / TW; tx <= uz / TW; ++tx) {
          if (e < e_end) {
            key_tile[e] = rowbase + (uint32_t)tx;
            rec_of_key[e] = r;
          }
          ++e;
        }
      }
    }
    // The count pass sized this record's key range with the same footprint
    // code, so e == e_end here.  Keep every slot defined regardless.
    if (e != e_end) {
      atomicOr(const_cast<unsigned int*>(&ctrl->flags), kFlagInternal);
      for (; e < e_end; ++e) {
        key_tile[e] = PI.tile_off;
        rec_of_key[e] = r;
      }
    }
  }
}

// ---------------------------------------------------------------- adjoint
// Sum of the per-key partial derivatives of each record (its keys are
// contiguous in emission order).  One thread per record, deterministic.
__global__ __launch_bounds__(256) void k_reduce_partials(const Ctrl* __restrict__ ctrl,
                                                         const uint32_t* __restrict__ rec_koff,
                                                         const float4* __restrict__ partial,
                                                         float4* __restrict__ drec) {
  const uint32_t nrec = ctrl->n_rec_eff;
  for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < nrec; r += gridDim.x * blockDim.x) {
    const uint32_t k0 = rec_koff[r], k1 = rec_koff[r + 1];
    float4 a = make_float4(0.f, 0.f, 0.f, 0.f), b = a;
    for (uint32_t k = k0; k < k1; ++k) {
      const float4 x = partial[2 * (size_t)k], y = partial[2 * (size_t)k + 1];
      a.x += x.x; a.y += x.y; a.z += x.z; a.w += x.w;
      b.x += y.x; b.y += y.y; b.z += y.z; b.w += y.w;
    }
    drec[2 * (size_t)r] = a;
    drec[2 * (size_t)r + 1] = b;
  }
}

// One thread per Gaussian: chain rule from its records' derivatives to the
// raw parameters (mu, l, c, a).  No atomics: each Gaussian's records are
// contiguous.
__global__ __launch_bounds__(256) void k_preprocess_bwd(ug_gaussians g, const PlaneConst* __restrict__ pc,
                                                        RenderParams rp, const Ctrl* __restrict__ ctrl,
                                                        const uint32_t* __restrict__ cnt_rec,
                                                        const uint32_t* __restrict__ off_rec,
                                                        const uint32_t* __restrict__ rec_pid,
                                                        const float* __restrict__ drec, float* __restrict__ d_means,
                                                        float* __restrict__ d_lraw, float* __restrict__ d_int,
                                                        float* __restrict__ d_op, int accumulate) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rp.n) return;
  const bool ok = (ctrl->flags & (kFlagRecCap | kFlagKeyCap)) == 0;
  const uint32_t nr = ok ? cnt_rec[i] : 0u;
  double dmu[3] = {0, 0, 0}, dL[6] = {0, 0, 0, 0, 0, 0}, da = 0.0, dc = 0.0;
  if (nr > 0) {
    GaussIn G;
    load_gauss(g, i, (double)rp.beta, G);
    const double chi2 = (double)rp.chi2;
    const uint32_t r0 = off_rec[i];
    for (uint32_t j = 0; j < nr; ++j) {
      const uint32_t r = r0 + j;
      const PlaneConst& P = pc[rec_pid[r]];
      Conic k;
      conic_cull(G, P, chi2, k);
      conic_full(G, P, k);
      footprint_adjoint(G, P, k, drec + 8 * (size_t)r, dmu, dL, da, dc);
    }
    // Eq. 11: dL_kk / dl_kk = 2 l_kk
    dL[0] *= 2.0 * G.l[0];
    dL[3] *= 2.0 * G.l[3];
    dL[5] *= 2.0 * G.l[5];
  }
  if (accumulate) {
    for (int j = 0; j < 3; ++j) d_means[3 * i + j] += (float)dmu[j];
    for (int j = 0; j < 6; ++j) d_lraw[6 * i + j] += (float)dL[j];
    d_int[i] += (float)dc;
    d_op[i] += (float)da;
  } else {
    for (int j = 0; j < 3; ++j) d_means[3 * i + j] = (float)dmu[j];
    for (int j = 0; j < 6; ++j) d_lraw[6 * i + j] = (float)dL[j];
    d_int[i] = (float)dc;
    d_op[i] = (float)da;
  }
}

// ---------------------------------------------------------------- launchers
hipError_t launch_init(const ug_planes& pl, const PlaneInt* pint, PlaneConst* pc, Ctrl* ctrl, hipStream_t s) {
  const int blocks = (pl.p + 255) / 256;
  hipLaunchKernelGGL(k_init, dim3(blocks), dim3(256), 0, s, pl, pint, pc, ctrl);
  return hipGetLastError();
}

hipError_t launch_count(const ug_gaussians& g, const PlaneConst* pc, const PlaneInt* pint, const RenderParams& rp,
                        uint32_t* cnt_rec, uint32_t* cnt_key, uint32_t* blk_rec, uint32_t* blk_key, Ctrl* ctrl,
                        hipStream_t s) {
  const int blocks = (rp.n + 255) / 256;
  if (blocks > 0)
    hipLaunchKernelGGL(k_count, dim3(blocks), dim3(256), 0, s, g, pc, pint, rp, cnt_rec, cnt_key, blk_rec, blk_key,
                       ctrl);
  return hipGetLastError();
}

hipError_t launch_top_scan(const uint32_t* blk_rec, const uint32_t* blk_key, unsigned long long* blk_rec_off,
                           unsigned long long* blk_key_off, int nblk, Ctrl* ctrl, uint32_t rec_cap,
                           uint32_t key_cap, uint32_t* rec_koff, hipStream_t s) {
  hipLaunchKernelGGL(k_top_scan, dim3(1), dim3(1024), 0, s, blk_rec, blk_key, blk_rec_off, blk_key_off, nblk, ctrl,
                     rec_cap, key_cap, rec_koff);
  return hipGetLastError();
}

hipError_t launch_write(const ug_gaussians& g, const PlaneConst* pc, const PlaneInt* pint, const RenderParams& rp,
                        const uint32_t* cnt_rec, const uint32_t* cnt_key, const unsigned long long* blk_rec_off,
                        const unsigned long long* blk_key_off, uint32_t* off_rec, RecAcc* racc, RecGeo* rgeo,
                        uint32_t* rec_pid, uint32_t* rec_koff, hipStream_t s) {
  const int blocks = (rp.n + 255) / 256;
  if (blocks > 0)
    hipLaunchKernelGGL(k_write, dim3(blocks), dim3(256), 0, s, g, pc, pint, rp, cnt_rec, cnt_key, blk_rec_off,
                       blk_key_off, off_rec, racc, rgeo, rec_pid, rec_koff);
  return hipGetLastError();
}

hipError_t launch_emit(const Ctrl* ctrl, const RecAcc* racc, const RecGeo* rgeo, const uint32_t* rec_pid,
                       const uint32_t* rec_koff, const PlaneInt* pint, const RenderParams& rp, uint32_t* key_tile,
                       uint32_t* rec_of_key, hipStream_t s) {
  const uint32_t want = (rp.rec_cap + 255) / 256;
  const uint32_t blocks = want < 4096 ? (want > 0 ? want : 1) : 4096;
  hipLaunchKernelGGL(k_emit, dim3(blocks), dim3(256), 0, s, ctrl, racc, rgeo, rec_pid, rec_koff, pint, rp, key_tile,
                     rec_of_key);
  return hipGetLastError();
}

hipError_t launch_reduce_partials(const Ctrl* ctrl, const uint32_t* rec_koff, const float* partial, float* drec,
                                  uint32_t rec_cap, hipStream_t s) {
  const uint32_t want = (rec_cap + 255) / 256;
  const uint32_t blocks = want < 4096 ? (want > 0 ? want : 1) : 4096;
  hipLaunchKernelGGL(k_reduce_partials, dim3(blocks), dim3(256), 0, s, ctrl, rec_koff,
                     reinterpret_cast<const float4*>(partial), reinterpret_cast<float4*>(drec));
  return hipGetLastError();
}

hipError_t launch_preprocess_bwd(const ug_gaussians& g, const PlaneConst* pc, const RenderParams& rp,
                                 const Ctrl* ctrl, const uint32_t* cnt_rec, const uint32_t* off_rec,
                                 const uint32_t* rec_pid, const float* drec, float* d_means, float* d_lraw,
                                 float* d_int, float* d_op, int accumulate, hipStream_t s) {
  const int blocks = (rp.n + 255) / 256;
  if (blocks > 0)
    hipLaunchKernelGGL(k_preprocess_bwd, dim3(blocks), dim3(256), 0, s, g, pc, rp, ctrl, cnt_rec, off_rec, rec_pid,
                       drec, d_means, d_lraw, d_int, d_op, accumulate);
  return hipGetLastError();
}

}  // namespace ug
