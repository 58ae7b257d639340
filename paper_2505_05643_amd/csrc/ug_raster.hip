// Per-tile accumulation of the ultrasound image formation (Eq. 5-8, 12) and
// its adjoint.
//
// Forward: one workgroup per tile, lanes = pixels.  The tile's records
// (sorted by record id, so every pixel sums its Gaussians in the same order
// whatever the tile shape) are staged through LDS in batches and every lane
// walks the batch: per pixel-record pair two FMAs give the exponent, one
// compare applies the Eq. 12 cut-off, one v_exp_f32 gives the weight.
//
// Adjoint: lanes = keys (one record in one tile).  Each lane walks its
// tile's pixels and accumulates the record's seven partial derivatives in
// registers, so no cross-lane reduction or atomic is needed; rows that no
// lane's ellipse reaches are skipped with a wave vote.
#include "ug_kernels.h"

namespace ug {

__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }

// ---------------------------------------------------------------- forward
// Lane layout: each wave owns a sub-tile LW*K pixels wide and 64/LW rows tall
// (LW = lanes per pixel row, at most 8); a lane owns K pixels of one row,
// LW apart.  Per staged record a wave first tests the record's bounding box
// (from its own conic factor) against its sub-tile and then its row bound,
// and skips the record when either shows no pixel of the wave in support.
template <int TW, int TH, int K>
struct FwdLayout {
  static constexpr int NT = TW * TH / K;
  static constexpr int LW = (TW / K) < 8 ? (TW / K) : 8;
  static constexpr int SW = LW * K;  // sub-tile width
  static constexpr int SH = 64 / LW; // sub-tile height
  static constexpr int NWX = TW / SW;
  static_assert(NT % 64 == 0 && TW % SW == 0 && TH % SH == 0 && (TW / SW) * (TH / SH) == NT / 64, "layout");
};

// CNT: also count the in-support pairs of pixels inside the plane (a
// measurement variant; the counter costs one VALU op per pair).
template <int TW, int TH, int K, int BG, bool CNT>
__global__ __launch_bounds__(TW* TH / K) void k_accum_fwd(const PlaneInt* __restrict__ pint,
                                                          const uint32_t* __restrict__ tile_plane,
                                                          const uint32_t* __restrict__ tile_start,
                                                          const uint32_t* __restrict__ srec,
                                                          const RecAcc* __restrict__ racc,
                                                          const RecGeo* __restrict__ rgeo, float* __restrict__ image,
                                                          float* __restrict__ dsave, float bg_alpha, float bg_color,
                                                          unsigned long long* __restrict__ n_eval) {
  using Lay = FwdLayout<TW, TH, K>;
  constexpr int NT = Lay::NT, LW = Lay::LW, SW = Lay::SW, SH = Lay::SH, NWX = Lay::NWX;
  __shared__ float4 sA[BG];
  __shared__ float4 sB[BG];
  __shared__ float4 sC[BG];

  const uint32_t t = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t p = tile_plane[t];
  const PlaneInt PI = pint[p];
  const uint32_t lt = t - PI.tile_off;
  const int tx = (int)(lt % (uint32_t)PI.ntx), ty = (int)(lt / (uint32_t)PI.ntx);
  const int x0 = tx * TW, y0 = ty * TH;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int sx0 = (wave % NWX) * SW, sy0 = (wave / NWX) * SH;
  const int row = sy0 + lane / LW, col0 = sx0 + lane % LW;
  const float vrow = (float)row;
  const float wx_lo = (float)sx0, wx_hi = (float)(sx0 + SW - 1);
  const float wy_lo = (float)sy0, wy_hi = (float)(sy0 + SH - 1);
  float ucol[K], Nacc[K], Dacc[K];
  uint32_t cnt[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    ucol[k] = (float)(col0 + k * LW);
    Nacc[k] = 0.f;
    Dacc[k] = 0.f;
    cnt[k] = 0u;
  }
  const uint32_t s = tile_start[t], e = tile_start[t + 1];
  // Records are staged through LDS in batches of BG; the next batch is
  // fetched into registers while the current one is evaluated.
  constexpr int PER = (BG + NT - 1) / NT;  // records each thread stages per batch
  RecAcc pa[PER];
  RecGeo pg[PER];
  auto fetch = [&](uint32_t base) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const uint32_t j = tid + q * NT;
      if (j < (uint32_t)BG && base + j < e) {
        const uint32_t r = srec[base + j];
        pa[q] = racc[r];
        pg[q] = rgeo[r];
      }
    }
  };
  if (s < e) fetch(s);
  for (uint32_t base = s; base < e; base += BG) {
    const uint32_t nb = min((uint32_t)BG, e - base);
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const uint32_t j = tid + q * NT;
      if (j < nb) {
        const RecAcc& A = pa[q];
        const float du0 = (float)(pg[q].ub - x0) + A.fu;
        const float dv0 = (float)(pg[q].vb - y0) + A.fv;
        sA[j] = make_float4(A.t11, A.t12, A.t22, -A.t11 * du0);
        sB[j] = make_float4(dv0, A.e0, A.emin, A.c);
        // bounding box of (t11 du + t12 dv)^2 + (t22 dv)^2 <= e0 - emin,
        // padded well beyond float rounding (an empty support gives an
        // inverted box, which every wave skips)
        const float thr = A.e0 - A.emin;
        const float sq = sqrtf(fmaxf(thr, 0.f));
        const float hv = sq / A.t22 * 1.001f + 0.01f;
        const float hu = sq * sqrtf(A.t12 * A.t12 + A.t22 * A.t22) / (A.t11 * A.t22) * 1.001f + 0.01f;
        sC[j] = thr >= 0.f ? make_float4(du0 - hu, du0 + hu, dv0 - hv, dv0 + hv)
                           : make_float4(1.f, -1.f, 1.f, -1.f);
      }
    }
    __syncthreads();
    if (base + BG < e) fetch(base + BG);
    for (uint32_t j = 0; j < nb; ++j) {
      const float4 bb = sC[j];
      if (bb.x > wx_hi || bb.y < wx_lo || bb.z > wy_hi || bb.w < wy_lo) continue;  // uniform
      const float4 a = sA[j];
      const float4 b = sB[j];
      const float dv = vrow - b.x;
      const float t2 = a.z * dv;
      const float erow = fmaf(-t2, t2, b.y);
      // e <= erow on the whole pixel row: skip when no lane's row reaches
      // the support (wave-uniform branch).
      if (!__any(erow >= b.z)) continue;
      const float B = fmaf(a.y, dv, a.w);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const float t1 = fmaf(a.x, ucol[k], B);
        const float ee = fmaf(-t1, t1, erow);
        const float w = ee >= b.z ? fast_exp2(ee) : 0.f;
        Dacc[k] += w;
        Nacc[k] = fmaf(w, b.w, Nacc[k]);
        if constexpr (CNT) cnt[k] += ee >= b.z ? 1u : 0u;
      }
    }
    __syncthreads();
  }
  const int v = y0 + row;
  if (v < PI.H) {
    const size_t rowbase = (((size_t)PI.pix_off_hi << 32) | PI.pix_off_lo) + (size_t)v * PI.W;
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int u = x0 + col0 + k * LW;
      if (u < PI.W) {
        const float Dt = Dacc[k] + bg_alpha;
        image[rowbase + u] = (Nacc[k] + bg_alpha * bg_color) / Dt;
        dsave[rowbase + u] = Dt;
        c += cnt[k];
      }
    }
    if constexpr (CNT) {
      if (c) atomicAdd(n_eval, (unsigned long long)c);
    }
  }
}

// ---------------------------------------------------------------- backward prep
// Tile-major padded per-pixel adjoint inputs: gamma = dL/dc_hat / D and
// gamma * c_hat (zero outside the plane).
template <int TW, int TH>
__global__ __launch_bounds__(256) void k_bwd_prep(const PlaneInt* __restrict__ pint,
                                                  const uint32_t* __restrict__ tile_plane,
                                                  const float* __restrict__ image, const float* __restrict__ d_image,
                                                  const float* __restrict__ dsave, float2* __restrict__ gq,
                                                  uint32_t num_tiles) {
  const size_t gidx = (size_t)blockIdx.x * 256 + threadIdx.x;
  const uint32_t t = (uint32_t)(gidx / (TW * TH));
  if (t >= num_tiles) return;
  const int j = (int)(gidx % (TW * TH));
  const PlaneInt PI = pint[tile_plane[t]];
  const uint32_t lt = t - PI.tile_off;
  const int u = (int)(lt % (uint32_t)PI.ntx) * TW + j % TW;
  const int v = (int)(lt / (uint32_t)PI.ntx) * TH + j / TW;
  float2 out = make_float2(0.f, 0.f);
  if (u < PI.W && v < PI.H) {
    const size_t idx = (((size_t)PI.pix_off_hi << 32) | PI.pix_off_lo) + (size_t)v * PI.W + u;
    const float gam = d_image[idx] / dsave[idx];
    out = make_float2(gam, gam * image[idx]);
  }
  gq[gidx] = out;
}

// ---------------------------------------------------------------- backward
template <int TW, int TH>
__global__ __launch_bounds__(256) void k_accum_bwd(const Ctrl* __restrict__ ctrl, const PlaneInt* __restrict__ pint,
                                                   const uint32_t* __restrict__ tile_plane,
                                                   const uint32_t* __restrict__ skey,
                                                   const uint32_t* __restrict__ sval,
                                                   const uint32_t* __restrict__ srec,
                                                   const RecAcc* __restrict__ racc, const RecGeo* __restrict__ rgeo,
                                                   const float2* __restrict__ gq, float4* __restrict__ partial) {
  const uint32_t n = ctrl->n_key_eff;
  const float ln2 = (float)kLn2;
  const uint32_t nchunks = (n + 255u) / 256u;
  const uint32_t G = gridDim.x;
  for (uint32_t it = 0; it * G < nchunks; ++it) {
    const uint32_t chunk = it * G + xcd_remap(blockIdx.x, G);
    if (chunk >= nchunks) break;  // uniform over the block
    const uint32_t i = chunk * 256u + threadIdx.x;
    const bool act = i < n;
    float t11 = 0.f, t12 = 0.f, t22 = 0.f, P = 0.f, du0 = 0.f, dv0 = 0.f, e0 = 0.f, emin = INFINITY, c = 0.f;
    uint32_t t = 0;
    if (act) {
      t = skey[i];
      const uint32_t r = srec[i];
      const RecAcc A = racc[r];
      const RecGeo Gg = rgeo[r];
      const PlaneInt PI = pint[tile_plane[t]];
      const uint32_t lt = t - PI.tile_off;
      const int x0 = (int)(lt % (uint32_t)PI.ntx) * TW;
      const int y0 = (int)(lt / (uint32_t)PI.ntx) * TH;
      du0 = (float)(Gg.ub - x0) + A.fu;
      dv0 = (float)(Gg.vb - y0) + A.fv;
      t11 = A.t11;
      t12 = A.t12;
      t22 = A.t22;
      P = -A.t11 * du0;
      e0 = A.e0;
      emin = A.emin;
      c = A.c;
    }
    const float2* __restrict__ px = gq + (size_t)t * (TW * TH);
    float Sge = 0.f, Sa = 0.f, Sau = 0.f, S12 = 0.f, S22 = 0.f, Sb = 0.f, Sdc = 0.f;
    for (int y = 0; y < TH; ++y) {
      const float dv = (float)y - dv0;
      const float B = fmaf(t12, dv, P);
      const float t2 = t22 * dv;
      const float erow = fmaf(-t2, t2, e0);
      if (!__any(erow >= emin)) continue;  // no lane's ellipse reaches this row
      float rge = 0.f, ra = 0.f;
#pragma unroll 4
      for (int x = 0; x < TW; ++x) {
        const float xf = (float)x;
        const float t1 = fmaf(t11, xf, B);
        const float ee = fmaf(-t1, t1, erow);
        const float w = ee >= emin ? fast_exp2(ee) : 0.f;
        const float2 gg = px[y * TW + x];
        const float gw = fmaf(gg.x, c, -gg.y);  // dL/dw = gamma (c - c_hat)
        const float ge = w * gw;
        rge += ge;
        Sdc = fmaf(gg.x, w, Sdc);
        const float a = ge * t1;
        ra += a;
        Sau = fmaf(a, xf, Sau);
      }
      Sge += rge;
      Sa += ra;
      S12 = fmaf(dv, ra, S12);
      Sb = fmaf(t2, rge, Sb);
      S22 = fmaf(t2 * dv, rge, S22);
    }
    if (act) {
      // w = 2^(e0 - t1^2 - t2^2):  dL/ds = -ln2 w dL/dw, s = t1^2 + t2^2.
      const float k2 = 2.f * ln2;
      const uint32_t eidx = sval[i];
      partial[2 * (size_t)eidx] = make_float4(-k2 * (Sau - du0 * Sa), -k2 * S12, -k2 * S22, k2 * t11 * Sa);
      partial[2 * (size_t)eidx + 1] = make_float4(k2 * (t12 * Sa + t22 * Sb), ln2 * Sge, Sdc, 0.f);
    }
  }
}

// ---------------------------------------------------------------- dispatch
template <int TW, int TH, int K>
static hipError_t fwd_bg(int bg, dim3 grid, hipStream_t s, const PlaneInt* pint, const uint32_t* tp,
                         const uint32_t* ts, const uint32_t* srec, const RecAcc* ra, const RecGeo* rg, float* img,
                         float* ds, float ba, float bc, unsigned long long* n_eval) {
  constexpr int NT = TW * TH / K;
  switch (bg) {
#define UG_BG(B)                                                                                                  \
  case B:                                                                                                         \
    if (n_eval)                                                                                                   \
      hipLaunchKernelGGL((k_accum_fwd<TW, TH, K, B, true>), grid, dim3(NT), 0, s, pint, tp, ts, srec, ra, rg, img, \
                         ds, ba, bc, n_eval);                                                                     \
    else                                                                                                          \
      hipLaunchKernelGGL((k_accum_fwd<TW, TH, K, B, false>), grid, dim3(NT), 0, s, pint, tp, ts, srec, ra, rg,     \
                         img, ds, ba, bc, n_eval);                                                                \
    return hipGetLastError();
    UG_BG(32)
    UG_BG(64)
    UG_BG(128)
    UG_BG(256)
#undef UG_BG
    default:
      return hipErrorInvalidValue;
  }
}

// (tile_w, tile_h, pixels per lane) combinations compiled in.
#define UG_FWD_SHAPES(X) \
  X(8, 8, 1)             \
  X(16, 8, 1)            \
  X(16, 8, 2)            \
  X(16, 16, 1)           \
  X(16, 16, 2)           \
  X(16, 16, 4)           \
  X(32, 8, 1)            \
  X(32, 8, 2)            \
  X(32, 8, 4)            \
  X(32, 16, 2)           \
  X(32, 16, 4)           \
  X(32, 16, 8)

int accum_default_ppl(int tile_w, int tile_h) {
  const int px = tile_w * tile_h;
  return px >= 512 ? px / 256 : 1;
}

bool accum_config_supported(int tile_w, int tile_h, int ppl, int lds_batch) {
  if (!(lds_batch == 32 || lds_batch == 64 || lds_batch == 128 || lds_batch == 256)) return false;
#define UG_OK_SHAPE(W, H, K) \
  if (tile_w == W && tile_h == H && ppl == K) return true;
  UG_FWD_SHAPES(UG_OK_SHAPE)
#undef UG_OK_SHAPE
  return false;
}

hipError_t launch_accum_fwd(int tile_w, int tile_h, int ppl, int lds_batch, const PlaneInt* pint,
                            const uint32_t* tile_plane, const uint32_t* tile_start, const uint32_t* srec,
                            const RecAcc* racc, const RecGeo* rgeo, float* image, float* dsave, float bg_alpha,
                            float bg_color, uint32_t num_tiles, unsigned long long* n_eval, hipStream_t s) {
  const dim3 grid(num_tiles);
#define UG_LAUNCH_SHAPE(W, H, K)                                                                            \
  if (tile_w == W && tile_h == H && ppl == K)                                                               \
    return fwd_bg<W, H, K>(lds_batch, grid, s, pint, tile_plane, tile_start, srec, racc, rgeo, image, dsave, \
                           bg_alpha, bg_color, n_eval);
  UG_FWD_SHAPES(UG_LAUNCH_SHAPE)
#undef UG_LAUNCH_SHAPE
  return hipErrorInvalidValue;
}

hipError_t launch_bwd_prep(int tile_w, int tile_h, const PlaneInt* pint, const uint32_t* tile_plane,
                           const float* image, const float* d_image, const float* dsave, float* gq,
                           uint32_t num_tiles, hipStream_t s) {
  const size_t total = (size_t)num_tiles * tile_w * tile_h;
  const dim3 grid((unsigned)((total + 255) / 256));
  float2* g2 = reinterpret_cast<float2*>(gq);
#define UG_PREP(W, H)                                                                                              \
  if (tile_w == W && tile_h == H) {                                                                                \
    hipLaunchKernelGGL((k_bwd_prep<W, H>), grid, dim3(256), 0, s, pint, tile_plane, image, d_image, dsave, g2,     \
                       num_tiles);                                                                                 \
    return hipGetLastError();                                                                                      \
  }
  UG_PREP(8, 8)
  UG_PREP(16, 8)
  UG_PREP(16, 16)
  UG_PREP(32, 8)
  UG_PREP(32, 16)
#undef UG_PREP
  return hipErrorInvalidValue;
}

hipError_t launch_accum_bwd(int tile_w, int tile_h, const Ctrl* ctrl, const PlaneInt* pint,
                            const uint32_t* tile_plane, const uint32_t* skey, const uint32_t* sval,
                            const uint32_t* srec, const RecAcc* racc, const RecGeo* rgeo, const float* gq,
                            float* partial, uint32_t key_cap, hipStream_t s) {
  uint32_t want = (key_cap + 255u) / 256u;
  if (want < 1) want = 1;
  const uint32_t blocks = want < 16384u ? want : 16384u;
  const float2* g2 = reinterpret_cast<const float2*>(gq);
  float4* p4 = reinterpret_cast<float4*>(partial);
#define UG_BWD(W, H)                                                                                         \
  if (tile_w == W && tile_h == H) {                                                                          \
    hipLaunchKernelGGL((k_accum_bwd<W, H>), dim3(blocks), dim3(256), 0, s, ctrl, pint, tile_plane, skey, sval, \
                       srec, racc, rgeo, g2, p4);                                                            \
    return hipGetLastError();                                                                                \
  }
  UG_BWD(8, 8)
  UG_BWD(16, 8)
  UG_BWD(16, 16)
  UG_BWD(32, 8)
  UG_BWD(32, 16)
#undef UG_BWD
  return hipErrorInvalidValue;
}

}  // namespace ug
