// Preprocess kernels: plane set-up, the Phase-1 cull with record compaction
// (Section 4.4: reject the pairs whose box misses the plane, then compact
// the accepted ones), the per-record in-plane conic with key offsets and key
// emission (tile binning), and the adjoint of the record construction.
//
// Each compaction is a count kernel and a write kernel.  The count kernel
// leaves one total per block; a block of the write kernel adds up the totals
// of the blocks before it (at most 2048 of them, read coalesced), so offsets
// never depend on scheduling and no block waits on another: records are
// Gaussian-major with planes in order, and keys are in record order.
#include "ug_conic.h"
#include "ug_kernels.h"

namespace ug {

// ---------------------------------------------------------------- plane set-up
// One thread per plane: FP64 constants of the pose (an invalid pose is marked
// and skipped; the cull raises the flag).  Thread 0 clears the control block.
__global__ __launch_bounds__(256) void k_init(ug_planes pl, const PlaneInt* __restrict__ pint,
                                              PlaneConst* __restrict__ pc, Ctrl* __restrict__ ctrl) {
  const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid == 0) {
    ctrl->n_rec = 0;
    ctrl->n_key = 0;
    ctrl->n_eval = 0;
    ctrl->flags = 0;
    ctrl->n_rec_eff = 0;
    ctrl->n_key_eff = 0;
  }
  const int p = (int)gid;
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

// ---------------------------------------------------------------- block scan
// Exclusive scan of one value per thread over a 256-thread block.
template <typename T>
__device__ __forceinline__ T block_exscan_256(T v, T* sh /*[4]*/, T& total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  T x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const T y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh[wave] = x;
  __syncthreads();
  T before = 0;
  total = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const T s = sh[w];
    if (w < wave) before += s;
    total += s;
  }
  __syncthreads();
  return before + x - v;
}

// Sum of the first b block totals, by the whole block (coalesced reads).
__device__ __forceinline__ unsigned long long block_prefix(const uint32_t* __restrict__ tot, uint32_t b,
                                                           unsigned long long* sh /*[4]*/) {
  unsigned long long s = 0;
  for (uint32_t i = threadIdx.x; i < b; i += 256) s += tot[i];
  unsigned long long t;
  block_exscan_256<unsigned long long>(s, sh, t);
  return t;
}

// ---------------------------------------------------------------- cull pass
// Lanes = (Gaussian, plane) pairs.  A wave holds 64 / pw Gaussians, each
// owning a segment of pw lanes (pw = plane count rounded up to a power of
// two, at most 64) that walks the Gaussian's planes in chunks of pw; a block
// covers gpb consecutive Gaussians in rounds of 4 * 64 / pw.  A pair is a
// record iff the plane meets the Eq. 12 ellipsoid (the Phase-1 test of
// Eq. 13's box along the normal).
struct CullLane {
  int per_wave, seg, pl, gl;
  unsigned long long segmask;
};

__device__ __forceinline__ CullLane cull_lane(int pw) {
  CullLane c;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  c.per_wave = 64 / pw;
  c.seg = lane / pw;
  c.pl = lane - c.seg * pw;
  c.gl = wave * c.per_wave + c.seg;
  c.segmask = (pw == 64 ? ~0ull : ((1ull << pw) - 1ull)) << (c.seg * pw);
  return c;
}

// Counts: per-Gaussian records and the block's total.
__global__ __launch_bounds__(256) void k_cull_count(ug_gaussians g, const PlaneConst* __restrict__ pc,
                                                    RenderParams rp, int pw, int gpb, uint32_t* __restrict__ cnt_rec,
                                                    uint32_t* __restrict__ blk_tot, Ctrl* __restrict__ ctrl) {
  __shared__ uint32_t s_tot;
  const CullLane L = cull_lane(pw);
  if (threadIdx.x == 0) s_tot = 0;
  __syncthreads();
  const double chi2 = (double)rp.chi2;
  const int round = 4 * L.per_wave;
  uint32_t mine = 0;
  for (int r0 = 0; r0 < gpb; r0 += round) {
    const int gi = blockIdx.x * gpb + r0 + L.gl;
    const bool has = gi < rp.n;
    GaussIn G;
    G.finite = false;
    if (has) load_gauss(g, gi, (double)rp.beta, G);
    if (has && !G.finite && L.pl == 0) atomicOr(&ctrl->flags, kFlagNonfinite);
    uint32_t count = 0;
    for (int p0 = 0; p0 < rp.p; p0 += pw) {
      const int p = p0 + L.pl;
      bool acc = false;
      if (has && G.finite && p < rp.p) {
        if (pc[p].valid) {
          Conic k;
          acc = conic_cull(G, pc[p], chi2, k);
        } else if (gi == 0) {
          atomicOr(&ctrl->flags, kFlagNonfinite);
        }
      }
      count += (uint32_t)__popcll(__ballot(acc) & L.segmask);
    }
    if (has && L.pl == 0) {
      cnt_rec[gi] = count;
      mine += count;
    }
  }
  if (mine) atomicAdd(&s_tot, mine);
  __syncthreads();
  if (threadIdx.x == 0) blk_tot[blockIdx.x] = s_tot;
}

// Offsets and the compact (Gaussian, plane) list, Gaussian-major with planes
// ascending.  The last block publishes the total and the capacity check.
__global__ __launch_bounds__(256) void k_cull_write(ug_gaussians g, const PlaneConst* __restrict__ pc,
                                                    RenderParams rp, int pw, int gpb, uint32_t nblk,
                                                    const uint32_t* __restrict__ cnt_rec,
                                                    const uint32_t* __restrict__ blk_tot,
                                                    unsigned long long* __restrict__ off_rec,
                                                    uint2* __restrict__ rec_pair, Ctrl* __restrict__ ctrl) {
  __shared__ unsigned long long s_sh[4];
  __shared__ uint32_t s_sh32[4];
  __shared__ uint32_t s_cnt[256];
  const CullLane L = cull_lane(pw);
  unsigned long long carry = block_prefix(blk_tot, blockIdx.x, s_sh);
  const double chi2 = (double)rp.chi2;
  const int round = 4 * L.per_wave;
  for (int r0 = 0; r0 < gpb; r0 += round) {
    const int gi = blockIdx.x * gpb + r0 + L.gl;
    const bool has = gi < rp.n;
    s_cnt[threadIdx.x] = 0;
    __syncthreads();
    if (has && L.pl == 0) s_cnt[L.gl] = cnt_rec[gi];
    __syncthreads();
    uint32_t rtot;
    const uint32_t ex = block_exscan_256<uint32_t>(s_cnt[threadIdx.x], s_sh32, rtot);
    __syncthreads();
    s_cnt[threadIdx.x] = ex;
    __syncthreads();
    const unsigned long long base = carry + s_cnt[L.gl];
    carry += rtot;
    GaussIn G;
    G.finite = false;
    if (has) {
      load_gauss(g, gi, (double)rp.beta, G);
      if (L.pl == 0) off_rec[gi] = base;
    }
    unsigned long long r = base;
    for (int p0 = 0; p0 < rp.p; p0 += pw) {
      const int p = p0 + L.pl;
      bool acc = false;
      if (has && G.finite && p < rp.p && pc[p].valid) {
        Conic k;
        acc = conic_cull(G, pc[p], chi2, k);
      }
      const unsigned long long m = __ballot(acc) & L.segmask;
      if (acc) {
        const unsigned long long ri = r + lanemask_lt_popc(m);
        if (ri < rp.rec_cap) rec_pair[ri] = make_uint2((uint32_t)gi, (uint32_t)p);
      }
      r += (unsigned long long)__popcll(m);
    }
    __syncthreads();
  }
  if (blockIdx.x == nblk - 1 && threadIdx.x == 0) {
    ctrl->n_rec = carry;
    if (carry > rp.rec_cap) atomicOr(&ctrl->flags, kFlagRecCap);
    ctrl->n_rec_eff = carry <= rp.rec_cap ? (uint32_t)carry : 0u;
  }
}

// ---------------------------------------------------------------- record pass
// Lanes = records (every lane an accepted pair: no divergence); a block
// covers rpb consecutive records in rounds of 256.
__device__ __forceinline__ void emit_keys(const RecAcc& ra, const RecGeo& geo, const PlaneInt& PI, int box_mode,
                                          int TW, int TH, uint32_t r, uint32_t e, uint32_t e_end,
                                          uint32_t* __restrict__ key_tile, uint32_t* __restrict__ rec_of_key) {
  if (box_mode != UG_BOX_ROWS) {
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
}

// FP64 in-plane conic and footprint of each record; key counts and the
// block's total.
__global__ __launch_bounds__(256) void k_record(ug_gaussians g, const PlaneConst* __restrict__ pc,
                                                const PlaneInt* __restrict__ pint, RenderParams rp, int rpb,
                                                const uint2* __restrict__ rec_pair, RecAcc* __restrict__ racc,
                                                RecGeo* __restrict__ rgeo, uint32_t* __restrict__ rec_nkey,
                                                uint32_t* __restrict__ blk_tot, const Ctrl* __restrict__ ctrl) {
  __shared__ uint32_t s_tot;
  const uint32_t nrec = ctrl->n_rec_eff;
  const uint32_t r_begin = blockIdx.x * (uint32_t)rpb;
  if (r_begin >= nrec) return;  // uniform
  if (threadIdx.x == 0) s_tot = 0;
  __syncthreads();
  const double chi2 = (double)rp.chi2;
  uint32_t mine = 0;
  const uint32_t r_end = min(r_begin + (uint32_t)rpb, nrec);
  for (uint32_t r = r_begin + threadIdx.x; r < r_end; r += 256) {
    const uint2 gp = rec_pair[r];
    GaussIn G;
    load_gauss(g, (int)gp.x, (double)rp.beta, G);
    const PlaneConst& P = pc[gp.y];
    Conic k;
    conic_cull(G, P, chi2, k);
    conic_full(G, P, k);
    Footprint f;
    if (!make_footprint(G, P, pint[gp.y], k, chi2, rp.box_mode, rp.tile_w, rp.tile_h, f)) {
      // the plane cuts the ellipsoid outside the image: a record with no keys
      f.keys = 0;
      f.acc = RecAcc{0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      f.geo = RecGeo{0, 0, 1, 0, 1, 0};
    }
    racc[r] = f.acc;
    rgeo[r] = f.geo;
    rec_nkey[r] = f.keys;
    mine += f.keys;
  }
  if (mine) atomicAdd(&s_tot, mine);
  __syncthreads();
  if (threadIdx.x == 0) blk_tot[blockIdx.x] = s_tot;
}

// Key offsets (block prefix + in-block scan) and key emission.  The last
// active block publishes the key total and the capacity check.
__global__ __launch_bounds__(256) void k_emit(const PlaneInt* __restrict__ pint, RenderParams rp, int rpb,
                                              const uint2* __restrict__ rec_pair, const RecAcc* __restrict__ racc,
                                              const RecGeo* __restrict__ rgeo, const uint32_t* __restrict__ rec_nkey,
                                              const uint32_t* __restrict__ blk_tot, uint32_t* __restrict__ rec_koff,
                                              Ctrl* __restrict__ ctrl, uint32_t* __restrict__ key_tile,
                                              uint32_t* __restrict__ rec_of_key) {
  __shared__ unsigned long long s_sh[4];
  const uint32_t nrec = ctrl->n_rec_eff;
  const uint32_t r_begin = blockIdx.x * (uint32_t)rpb;
  if (r_begin >= nrec) return;  // uniform
  const uint32_t nact = (nrec + (uint32_t)rpb - 1) / (uint32_t)rpb;
  unsigned long long carry = block_prefix(blk_tot, blockIdx.x, s_sh);
  const uint32_t r_end = min(r_begin + (uint32_t)rpb, nrec);
  for (uint32_t r0 = r_begin; r0 < r_end; r0 += 256) {
    const uint32_t r = r0 + threadIdx.x;
    const bool act = r < r_end;
    const uint32_t nk = act ? rec_nkey[r] : 0u;
    unsigned long long tot;
    const unsigned long long koff = carry + block_exscan_256<unsigned long long>(nk, s_sh, tot);
    carry += tot;
    if (act) {
      rec_koff[r] = (uint32_t)(koff < rp.key_cap ? koff : rp.key_cap);
      if (nk > 0 && koff + nk <= rp.key_cap)
        emit_keys(racc[r], rgeo[r], pint[rec_pair[r].y], rp.box_mode, rp.tile_w, rp.tile_h, r, (uint32_t)koff,
                  (uint32_t)(koff + nk), key_tile, rec_of_key);
    }
  }
  if (blockIdx.x == nact - 1 && threadIdx.x == 0) {
    ctrl->n_key = carry;
    const bool ok = carry <= rp.key_cap;
    if (!ok) atomicOr(&ctrl->flags, kFlagKeyCap);
    ctrl->n_key_eff = ok ? (uint32_t)carry : 0u;
    rec_koff[nrec] = ok ? (uint32_t)carry : 0u;
  }
}

// ---------------------------------------------------------------- adjoint
// One thread per record: sum of its keys' partial derivatives (its keys are
// contiguous in emission order), then the FP64 chain rule through the record
// construction; the Gaussian's share is written to contrib[r] (12 floats).
__global__ __launch_bounds__(256) void k_record_adjoint(ug_gaussians g, const PlaneConst* __restrict__ pc,
                                                        RenderParams rp, const Ctrl* __restrict__ ctrl,
                                                        const uint2* __restrict__ rec_pair,
                                                        const uint32_t* __restrict__ rec_koff,
                                                        const float4* __restrict__ partial,
                                                        float* __restrict__ contrib) {
  const bool ok = (ctrl->flags & (kFlagRecCap | kFlagKeyCap)) == 0;
  const uint32_t nrec = ok ? ctrl->n_rec_eff : 0u;
  const double chi2 = (double)rp.chi2;
  for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < nrec; r += gridDim.x * blockDim.x) {
    const uint32_t k0 = rec_koff[r], k1 = rec_koff[r + 1];
    float4 a = make_float4(0.f, 0.f, 0.f, 0.f), c = a;
    for (uint32_t k = k0; k < k1; ++k) {
      const float4 x = partial[2 * (size_t)k], y = partial[2 * (size_t)k + 1];
      a.x += x.x; a.y += x.y; a.z += x.z; a.w += x.w;
      c.x += y.x; c.y += y.y; c.z += y.z; c.w += y.w;
    }
    double dmu[3] = {0, 0, 0}, dL[6] = {0, 0, 0, 0, 0, 0}, da = 0.0, dc = 0.0;
    if (k1 > k0) {
      const float dr[8] = {a.x, a.y, a.z, a.w, c.x, c.y, c.z, c.w};
      const uint2 gp = rec_pair[r];
      GaussIn G;
      load_gauss(g, (int)gp.x, (double)rp.beta, G);
      const PlaneConst& P = pc[gp.y];
      Conic k;
      conic_cull(G, P, chi2, k);
      conic_full(G, P, k);
      footprint_adjoint(G, P, k, dr, dmu, dL, da, dc);
    }
    float4* out = reinterpret_cast<float4*>(contrib + 12 * (size_t)r);
    out[0] = make_float4((float)dmu[0], (float)dmu[1], (float)dmu[2], (float)dL[0]);
    out[1] = make_float4((float)dL[1], (float)dL[2], (float)dL[3], (float)dL[4]);
    out[2] = make_float4((float)dL[5], (float)da, (float)dc, 0.f);
  }
}

// One thread per Gaussian: sum of its records' contributions (contiguous),
// then dL_kk / dl_kk = 2 l_kk (Eq. 11).  Deterministic, no atomics.
__global__ __launch_bounds__(256) void k_gauss_grad(ug_gaussians g, RenderParams rp, const Ctrl* __restrict__ ctrl,
                                                    const uint32_t* __restrict__ cnt_rec,
                                                    const unsigned long long* __restrict__ off_rec,
                                                    const float* __restrict__ contrib, float* __restrict__ d_means,
                                                    float* __restrict__ d_lraw, float* __restrict__ d_int,
                                                    float* __restrict__ d_op, int accumulate) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rp.n) return;
  const bool ok = (ctrl->flags & (kFlagRecCap | kFlagKeyCap)) == 0;
  const uint32_t nr = ok ? cnt_rec[i] : 0u;
  double acc[11] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  if (nr > 0) {
    const float4* c = reinterpret_cast<const float4*>(contrib + 12 * (size_t)off_rec[i]);
    for (uint32_t j = 0; j < nr; ++j) {
      const float4 x = c[3 * j], y = c[3 * j + 1], z = c[3 * j + 2];
      acc[0] += x.x; acc[1] += x.y; acc[2] += x.z; acc[3] += x.w;
      acc[4] += y.x; acc[5] += y.y; acc[6] += y.z; acc[7] += y.w;
      acc[8] += z.x; acc[9] += z.y; acc[10] += z.z;
    }
    acc[3] *= 2.0 * (double)g.lraw[6 * i + 0];
    acc[6] *= 2.0 * (double)g.lraw[6 * i + 3];
    acc[8] *= 2.0 * (double)g.lraw[6 * i + 5];
  }
  if (accumulate) {
    for (int j = 0; j < 3; ++j) d_means[3 * i + j] += (float)acc[j];
    for (int j = 0; j < 6; ++j) d_lraw[6 * i + j] += (float)acc[3 + j];
    d_op[i] += (float)acc[9];
    d_int[i] += (float)acc[10];
  } else {
    for (int j = 0; j < 3; ++j) d_means[3 * i + j] = (float)acc[j];
    for (int j = 0; j < 6; ++j) d_lraw[6 * i + j] = (float)acc[3 + j];
    d_op[i] = (float)acc[9];
    d_int[i] = (float)acc[10];
  }
}

// ---------------------------------------------------------------- launchers
constexpr uint32_t kMaxScanBlocks = 2048;

int pair_width(int p) {
  int pw = 1;
  while (pw < p && pw < 64) pw <<= 1;
  return pw;
}

// Gaussians per cull block: whole rounds of 4 * 64 / pw, at most 2048 blocks.
int cull_gpb(int n, int p) {
  const int round = 4 * (64 / pair_width(p));
  const long rounds = ((long)n + round - 1) / round;
  const long per = (rounds + kMaxScanBlocks - 1) / kMaxScanBlocks;
  return (int)((per < 1 ? 1 : per) * round);
}

uint32_t cull_blocks(int n, int p) {
  const int gpb = cull_gpb(n, p);
  return (uint32_t)((n + gpb - 1) / gpb);
}

// Records per record block: whole rounds of 256, at most 2048 blocks.
int record_rpb(uint32_t rec_cap) {
  const uint32_t rounds = (rec_cap + 255u) / 256u;
  const uint32_t per = (rounds + kMaxScanBlocks - 1) / kMaxScanBlocks;
  return (int)((per < 1 ? 1 : per) * 256u);
}

uint32_t record_blocks(uint32_t rec_cap) {
  const uint32_t rpb = (uint32_t)record_rpb(rec_cap);
  const uint32_t nb = (rec_cap + rpb - 1) / rpb;
  return nb < 1 ? 1 : nb;
}

hipError_t launch_init(const ug_planes& pl, const PlaneInt* pint, PlaneConst* pc, Ctrl* ctrl, hipStream_t s) {
  const uint32_t blocks = ((uint32_t)pl.p + 255) / 256;
  hipLaunchKernelGGL(k_init, dim3(blocks < 1 ? 1 : blocks), dim3(256), 0, s, pl, pint, pc, ctrl);
  return hipGetLastError();
}

hipError_t launch_cull(const ug_gaussians& g, const PlaneConst* pc, const RenderParams& rp, uint32_t* cnt_rec,
                       unsigned long long* off_rec, uint2* rec_pair, uint32_t* blk_tot, Ctrl* ctrl, hipStream_t s) {
  const uint32_t nb = cull_blocks(rp.n, rp.p);
  const int pw = pair_width(rp.p), gpb = cull_gpb(rp.n, rp.p);
  if (nb == 0) {  // no Gaussians: still publish the (zero) record total
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_cull_count, dim3(nb), dim3(256), 0, s, g, pc, rp, pw, gpb, cnt_rec, blk_tot, ctrl);
  hipLaunchKernelGGL(k_cull_write, dim3(nb), dim3(256), 0, s, g, pc, rp, pw, gpb, nb, cnt_rec, blk_tot, off_rec,
                     rec_pair, ctrl);
  return hipGetLastError();
}

hipError_t launch_record(const ug_gaussians& g, const PlaneConst* pc, const PlaneInt* pint, const RenderParams& rp,
                         const uint2* rec_pair, RecAcc* racc, RecGeo* rgeo, uint32_t* rec_nkey, uint32_t* rec_koff,
                         uint32_t* blk_tot, Ctrl* ctrl, uint32_t* key_tile, uint32_t* rec_of_key, hipStream_t s,
                         bool emit_stage_split) {
  (void)emit_stage_split;
  const uint32_t nb = record_blocks(rp.rec_cap);
  const int rpb = record_rpb(rp.rec_cap);
  hipLaunchKernelGGL(k_record, dim3(nb), dim3(256), 0, s, g, pc, pint, rp, rpb, rec_pair, racc, rgeo, rec_nkey,
                     blk_tot, ctrl);
  hipLaunchKernelGGL(k_emit, dim3(nb), dim3(256), 0, s, pint, rp, rpb, rec_pair, racc, rgeo, rec_nkey, blk_tot,
                     rec_koff, ctrl, key_tile, rec_of_key);
  return hipGetLastError();
}

hipError_t launch_record_adjoint(const ug_gaussians& g, const PlaneConst* pc, const RenderParams& rp,
                                 const Ctrl* ctrl, const uint2* rec_pair, const uint32_t* rec_koff,
                                 const float* partial, float* contrib, hipStream_t s) {
  uint32_t want = (rp.rec_cap + 255u) / 256u;
  const uint32_t blocks = want < 1 ? 1 : (want > 8192 ? 8192 : want);
  hipLaunchKernelGGL(k_record_adjoint, dim3(blocks), dim3(256), 0, s, g, pc, rp, ctrl, rec_pair, rec_koff,
                     reinterpret_cast<const float4*>(partial), contrib);
  return hipGetLastError();
}

hipError_t launch_gauss_grad(const ug_gaussians& g, const RenderParams& rp, const Ctrl* ctrl, const uint32_t* cnt_rec,
                             const unsigned long long* off_rec, const float* contrib, float* d_means, float* d_lraw,
                             float* d_int, float* d_op, int accumulate, hipStream_t s) {
  const int blocks = (rp.n + 255) / 256;
  if (blocks > 0)
    hipLaunchKernelGGL(k_gauss_grad, dim3(blocks), dim3(256), 0, s, g, rp, ctrl, cnt_rec, off_rec, contrib, d_means,
                       d_lraw, d_int, d_op, accumulate);
  return hipGetLastError();
}

}  // namespace ug
