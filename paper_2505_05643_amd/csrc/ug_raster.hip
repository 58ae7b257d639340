// Per-tile accumulation of the ultrasound image formation (Eq. 5-8, 12) and
// its adjoint.
//
// Tiles are split into 8x8-pixel sub-blocks; every key carries the mask of
// the sub-blocks its record's ellipse touches (Eq. 12 support, computed at
// key emission), so both passes evaluate (record, pixel) pairs only inside
// touched sub-blocks.
//
// Forward: one workgroup per tile, one wave per band of 8 pixel rows (or two,
// SPLIT = 2, taking alternate rounds of the tile's records and adding their
// sums at the end), lanes = pixels (a lane owns one pixel in each of the
// band's TW/8 sub-blocks).
// Each wave streams the tile's records (sorted by record id, so every pixel
// sums its Gaussians in the same order whatever the launch shape), keeps
// those whose mask touches its band in a wave-private LDS list and walks the
// list: per pixel-record pair two FMAs give the exponent, one compare
// applies the cut-off and one v_exp_f32 gives the weight.
//
// Adjoint: a wave takes 64 keys and expands them into (key, sub-block)
// items through an LDS queue in key order; lanes = items, each walking its
// 64 pixels and accumulating the record's seven partial derivatives in
// registers.  The items of a key are summed in sub-block order into the
// key's partial, so no atomic is needed and the result is deterministic.
#include <cfloat>

#include "ug_kernels.h"

namespace ug {

__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }

// A pair's weight 2^(e0 - t1^2 - t2^2) (Eq. 8 in log2 units) is evaluated as
// s 2^x with x = d - t1^2 - t2^2, d = e0 - sig and s = 2^sig per record.
// Under a cut-off (Eq. 12) sig = emin, so the support is x >= 0, and one
// signed-integer max of x's bits against the bits of -inf (kCutBits) maps
// every x < 0 to -inf, whose 2^x is 0: the compare and select of the test
// become one instruction.  sig stays within 64 of e0, so the scaled weights
// stay below 2^64 (for chi^2 > 64 / (log2(e) / 2) = 88.7 the cut then drops
// only weights below 2^-64 of the Gaussian's peak instead of those beyond
// chi^2).  Without a cut-off sig = e0 and the max is against INT_MIN (no
// operation).  A record whose sig is -inf (zero amplitude) gets d = -inf.
constexpr int kCutBits = (int)0xff800000u;  // bits of -inf
constexpr int kNoCutBits = (int)0x80000000u;

struct WeightScale {
  float d, s;
};

__device__ __forceinline__ WeightScale weight_scale(float e0, float emin, bool cut) {
  const float sig = cut ? fmaxf(emin, e0 - 64.f) : e0;
  if (!(sig > -INFINITY)) return {-INFINITY, 0.f};
  return {e0 - sig, exp2f(sig)};
}

// x with every value outside the support mapped to -inf (see above).
__device__ __forceinline__ float support_clamp(float x, int kcut) {
  return __int_as_float(max(__float_as_int(x), kcut));
}

// ---------------------------------------------------------------- forward
// CNT: also count the in-support pairs of pixels inside the plane and the
// evaluated pairs (64 per evaluated wave sub-block) into counters[0] and
// counters[1] (a measurement variant; one more VALU op per pair).  BG records
// are staged per wave and round (PER per lane; lanes beyond BG idle when
// BG < 64).
template <int TW, int TH, int BG, bool CNT, int SPLIT>
__global__ __launch_bounds__(64 * (TH / kSubBlock) * SPLIT) void k_accum_fwd(
    const PlaneInt* __restrict__ pint, const uint32_t* __restrict__ tile_plane,
    const uint32_t* __restrict__ tile_start, const uint32_t* __restrict__ skey, const uint32_t* __restrict__ srec,
    const Rec* __restrict__ recs, float* __restrict__ image,
    float* __restrict__ dsave, float bg_alpha, float bg_color, int kcut, unsigned long long* __restrict__ counters) {
  constexpr int K = TW / kSubBlock;   // pixels per lane = sub-blocks per band
  constexpr int NB = TH / kSubBlock;  // bands = waves
  constexpr int PER = BG >= 64 ? BG / 64 : 1;
  constexpr int CAP = PER * 64;
  static_assert(TW % kSubBlock == 0 && TH % kSubBlock == 0 && K * NB <= 32, "tile shape");
  static_assert(SPLIT == 1 || SPLIT == 2, "waves per band");
  // per kept record: (t11, s, s c, mask) and, per pixel row of the band,
  // (scaled exponent d - t2^2 at the row, t1 offset of the row) -- the row
  // set-up is done once per record while staging instead of once per record
  // and lane
  __shared__ float4 cA[NB * SPLIT][CAP];
  __shared__ float2 cR[NB * SPLIT][CAP][kSubBlock];

  const uint32_t t = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t p = tile_plane[t];
  const PlaneInt PI = pint[p];
  const uint32_t lt = t - PI.tile_off;
  const int x0 = (int)(lt % (uint32_t)PI.ntx) * TW, y0 = (int)(lt / (uint32_t)PI.ntx) * TH;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int band = wv % NB, half = wv / NB;  // half: which alternate rounds
  const int lrow = lane / kSubBlock, col0 = lane % kSubBlock;
  const int row = band * kSubBlock + lrow;
  constexpr int kMaskShift = key_mask_shift(TW, TH);
  const uint32_t bshift = (uint32_t)(kMaskShift + band * K), bmask = (1u << K) - 1u;
  float ucol[K], Nacc[K], Dacc[K];
  uint32_t cnt[K];
  uint32_t nexec = 0;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    ucol[k] = (float)(col0 + k * kSubBlock);
    Nacc[k] = 0.f;
    Dacc[k] = 0.f;
    cnt[k] = 0u;
  }
  const bool cut = kcut != kNoCutBits;
  const uint32_t s = tile_start[t], e = tile_start[t + 1];
  RecAcc pa[PER];
  RecGeo pg[PER];
  uint32_t pm[PER];
  // key words and record ids are loaded together (not the id behind the
  // mask test), then the records whose mask touches the band
  auto fetch = [&](uint32_t base) {
    uint32_t kw[PER], rid[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const uint32_t j = base + (uint32_t)(q * 64 + lane);
      const bool in = q * 64 + lane < BG && j < e;
      kw[q] = in ? skey[j] : 0u;
      rid[q] = in ? srec[j] : 0u;
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const uint32_t m = (kw[q] >> bshift) & bmask;
      pm[q] = m;
      if (m) {
        pa[q] = recs[rid[q]].acc;
        pg[q] = recs[rid[q]].geo;
      }
    }
  };
  const uint32_t s0 = s + (uint32_t)(half * BG);
  if (s0 < e) fetch(s0);
  for (uint32_t base = s0; base < e; base += SPLIT * BG) {
    // keep this round's records that touch the band, in order
    uint32_t n = 0;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const uint32_t m = pm[q];
      const unsigned long long bal = __ballot(m != 0u);
      if (m) {
        const uint32_t slot = n + lanemask_lt_popc(bal);
        const RecAcc& A = pa[q];
        const float du0 = (float)(pg[q].ub - x0) + A.fu;
        const float dv0 = (float)(pg[q].vb - y0) + A.fv;
        const float P = -A.t11 * du0;
        const WeightScale ws = weight_scale(A.e0, A.emin, cut);
        cA[wv][slot] = make_float4(A.t11, ws.s, ws.s * A.c, __uint_as_float(m));
#pragma unroll
        for (int y = 0; y < kSubBlock; ++y) {
          const float dv = (float)(band * kSubBlock + y) - dv0;
          const float t2 = A.t22 * dv;
          cR[wv][slot][y] = make_float2(fmaf(-t2, t2, ws.d), fmaf(A.t12, dv, P));
        }
      }
      n += (uint32_t)__popcll(bal);
    }
    if (base + SPLIT * BG < e) fetch(base + SPLIT * BG);
    wave_lds_sync();
    auto eval_rec = [&](const float4& a, const float2& rb) {
      const uint32_t m = __builtin_amdgcn_readfirstlane(__float_as_uint(a.w));
      const float erow = rb.x, B = rb.y;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (K > 1 && !((m >> k) & 1u)) continue;  // uniform
        const float t1 = fmaf(a.x, ucol[k], B);
        const float xs = support_clamp(fmaf(-t1, t1, erow), kcut);
        const float w = fast_exp2(xs);  // the weight over s
        Dacc[k] = fmaf(w, a.y, Dacc[k]);
        Nacc[k] = fmaf(w, a.z, Nacc[k]);
        if constexpr (CNT) {
          cnt[k] += xs != -INFINITY ? 1u : 0u;
          ++nexec;
        }
      }
    };
    // two records per iteration so their LDS reads overlap
    uint32_t j = 0;
    for (; j + 1 < n; j += 2) {
      const float4 a0 = cA[wv][j], a1 = cA[wv][j + 1];
      const float2 r0 = cR[wv][j][lrow], r1 = cR[wv][j + 1][lrow];
      eval_rec(a0, r0);
      eval_rec(a1, r1);
    }
    if (j < n) eval_rec(cA[wv][j], cR[wv][j][lrow]);
    wave_lds_sync();
  }
  if constexpr (SPLIT == 2) {
    // the band's second wave hands its sums over through its own staging
    // area; the first adds them to its own (first half + second half)
    float* xch = reinterpret_cast<float*>(&cR[NB + band][0][0]);
    if (half == 1) {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        xch[(2 * k) * 64 + lane] = Nacc[k];
        xch[(2 * k + 1) * 64 + lane] = Dacc[k];
      }
    }
    __syncthreads();
    if (half == 0) {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        Nacc[k] += xch[(2 * k) * 64 + lane];
        Dacc[k] += xch[(2 * k + 1) * 64 + lane];
      }
    }
  }
  const int v = y0 + row;
  if (v < PI.H) {
    const size_t rowbase = (((size_t)PI.pix_off_hi << 32) | PI.pix_off_lo) + (size_t)v * PI.W;
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int u = x0 + col0 + k * kSubBlock;
      if (u < PI.W) {
        if (half == 0) {
          const float Dt = Dacc[k] + bg_alpha;
          image[rowbase + u] = (Nacc[k] + bg_alpha * bg_color) / Dt;
          dsave[rowbase + u] = Dt;
        }
        c += cnt[k];
      }
    }
    if constexpr (CNT) {
      if (c) atomicAdd(&counters[0], (unsigned long long)c);
    }
  }
  if constexpr (CNT) {
    if (lane == 0 && nexec) atomicAdd(&counters[1], 64ull * nexec);
  }
}

// ---------------------------------------------------------------- backward prep
// Tile-major padded per-pixel adjoint inputs: gamma = dL/dc_hat / D and
// gamma * c_hat (zero outside the plane).  Four consecutive pixels of a tile
// row per thread: 16-byte loads where the arrays (vec) and the plane row are
// aligned and the row holds all four, single loads otherwise.
//
// MSE: the second array is the target and dL/dc_hat = scale (c_hat - target)
// is formed here, with the same float operations as the separate gradient
// kernel (so the same gamma bit for bit); each block also writes the sum of
// its squared differences to loss_part[block] (a fixed-order reduction).
template <int TW, int TH, bool MSE>
__global__ __launch_bounds__(256) void k_bwd_prep(const PlaneInt* __restrict__ pint,
                                                  const uint32_t* __restrict__ tile_plane,
                                                  const float* __restrict__ image, const float* __restrict__ second,
                                                  const float* __restrict__ dsave, float4* __restrict__ gq,
                                                  uint32_t num_tiles, int vec, float scale,
                                                  float* __restrict__ loss_part) {
  static_assert(TW % 4 == 0, "four pixels per thread within a tile row");
  const size_t gidx = (size_t)blockIdx.x * 256 + threadIdx.x;  // group of four pixels
  const uint32_t t = (uint32_t)(gidx / (TW * TH / 4));
  float sq = 0.f;  // MSE: this thread's squared differences
  if (t < num_tiles) {
    const int j = (int)(gidx % (TW * TH / 4)) * 4;
    const PlaneInt PI = pint[tile_plane[t]];
    const uint32_t lt = t - PI.tile_off;
    const int u = (int)(lt % (uint32_t)PI.ntx) * TW + j % TW;
    const int v = (int)(lt / (uint32_t)PI.ntx) * TH + j / TW;
    float gam[4] = {0.f, 0.f, 0.f, 0.f}, gc[4] = {0.f, 0.f, 0.f, 0.f};
    if (v < PI.H && u < PI.W) {
      const size_t idx = (((size_t)PI.pix_off_hi << 32) | PI.pix_off_lo) + (size_t)v * PI.W + u;
      if (vec && u + 3 < PI.W && (idx & 3u) == 0) {
        const float4 S2 = *reinterpret_cast<const float4*>(second + idx);
        const float4 Dt = *reinterpret_cast<const float4*>(dsave + idx);
        const float4 I = *reinterpret_cast<const float4*>(image + idx);
        const float s2[4] = {S2.x, S2.y, S2.z, S2.w}, dt[4] = {Dt.x, Dt.y, Dt.z, Dt.w};
        const float im[4] = {I.x, I.y, I.z, I.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          float dI = s2[q];
          if constexpr (MSE) {
            const float d = im[q] - s2[q];
            dI = scale * d;
            sq = fmaf(d, d, sq);
          }
          gam[q] = dI / dt[q];
          gc[q] = gam[q] * im[q];
        }
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (u + q < PI.W) {
            const float im = image[idx + q];
            float dI = second[idx + q];
            if constexpr (MSE) {
              const float d = im - dI;
              dI = scale * d;
              sq = fmaf(d, d, sq);
            }
            gam[q] = dI / dsave[idx + q];
            gc[q] = gam[q] * im;
          }
        }
      }
    }
    gq[2 * gidx] = make_float4(gam[0], gc[0], gam[1], gc[1]);
    gq[2 * gidx + 1] = make_float4(gam[2], gc[2], gam[3], gc[3]);
  }
  if constexpr (MSE) {
    __shared__ float s_w[4];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) sq += __shfl_xor(sq, o, 64);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = sq;
    __syncthreads();
    if (threadIdx.x == 0) loss_part[blockIdx.x] = ((s_w[0] + s_w[1]) + s_w[2]) + s_w[3];
  }
}

// ---------------------------------------------------------------- backward
// A wave loads 64 keys.  Each key's touched 8x8 sub-blocks become items
// (key, sub-block), queued in key order.  For every item a first pass over
// the queue (lanes = items) finds the rows of its sub-block that can hold a
// pixel inside the record's ellipse: row y can only if the larger of the
// exponents at the strip's two end columns -- or the row exponent itself
// when t1 changes sign across the strip -- passes the cut-off (t1 is
// monotone along the row, so no pixel between the ends does better); the
// first and last such rows bound the item.  Items are then ranked by their
// row count, largest first, and the evaluation pass (lanes = items in that
// order) walks 64 items with similar row counts together, each lane
// accumulating the record's seven sums over its rows in registers into the
// item's LDS slot.  Once a sub-chunk's items are done each key adds its
// slots in sub-block order.  A sub-chunk is the longest run of the wave's
// keys whose items fit the slots (at least one key: a key has at most 16
// items).  Rows an item skips would only add exact zeros, so the sums are
// those of walking all 64 pixels of every touched sub-block.
constexpr int kBwdSlots = 192;

template <int TW, int TH, bool GT>
__global__ __launch_bounds__(256) void k_accum_bwd(const Ctrl* __restrict__ ctrl,
                                                   const uint32_t* __restrict__ tile_org,
                                                   const uint32_t* __restrict__ skey,
                                                   const uint32_t* __restrict__ sval,
                                                   const uint32_t* __restrict__ srec,
                                                   const Rec* __restrict__ recs,
                                                   const float2* __restrict__ gq, float4* __restrict__ partial,
                                                   int kcut) {
  constexpr int K = TW / kSubBlock, Q = K * (TH / kSubBlock);
  constexpr int kMaskShift = key_mask_shift(TW, TH);
  static_assert(Q <= 16 && kBwdSlots >= Q && kBwdSlots <= 256, "sub-blocks per tile; slot ids fit a byte");
  __shared__ float4 kpA[4][64];     // t11, t12, t22, -t11 du0
  __shared__ float4 kpB[4][64];     // du0, dv0, d, s (the weight's scaled form)
  __shared__ float kpC[4][64];      // c
  __shared__ uint32_t kpT[4][64];   // tile
  __shared__ uint32_t qoff[4][65];  // first item of each key
  __shared__ uint32_t queue[4][kBwdSlots];   // key | sub-block << 6 | first row << 10 | rows << 13
  __shared__ uint8_t order[4][kBwdSlots];    // items with rows, by row count (largest first)
  __shared__ float slot[4][7][kBwdSlots];
  // GT (tiles of at most 512 pixels, launches with many keys): each wave
  // copies the gamma of its chunk's first tile (at most 4 KB) into LDS, and
  // items of that tile (nearly all: a tile holds many chunks) read their
  // rows there instead of through the L1, whose accesses otherwise set the
  // kernel's pace.  It costs a wave per SIMD of occupancy (LDS), which
  // small launches feel more than they gain; larger tiles would take too
  // much LDS.  Without it every row is read from memory.
  static_assert(!GT || TW * TH <= 512, "staged tile size");
  constexpr bool kGT = GT;
  constexpr int kGTQ = kGT ? TW * TH / 2 : 1;  // float4 per staged tile
  constexpr int kGTL = (kGTQ + 63) / 64;       // of them per lane
  __shared__ float4 gt[4][kGTQ];
  const uint32_t n = ctrl->n_key_eff;
  const float ln2 = (float)kLn2;
  const bool cut = kcut != kNoCutBits;
  // rows pass the pre-pass test iff their best pixel is in the support;
  // without a cut-off only zero-amplitude records (d = -inf) fail it
  const float thr = cut ? 0.f : -FLT_MAX;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t nchunks = (n + 63u) / 64u;
  const uint32_t W = gridDim.x * 4u;
  const uint32_t wid = xcd_remap(blockIdx.x, gridDim.x) * 4u + (uint32_t)wave;
  // The wave's chunks are fetched two ahead: while a chunk is processed,
  // the records and tile origins of the wave's next chunk (a random gather)
  // and the key words and record ids of the one after are in flight.  Lanes
  // past the last key read record 0 and tile 0 (both exist whenever there
  // is a key) and are masked off.
  const uint32_t kmask = (1u << kMaskShift) - 1u;
  auto fetch_keys = [&](uint32_t ch, uint32_t& kw, uint32_t& r) {
    const uint32_t j = ch * 64u + (uint32_t)lane;
    kw = j < n ? skey[j] : 0u;
    r = j < n ? srec[j] : 0u;
  };
  uint32_t chunk = wid;
  uint32_t kwN = 0u, rN = 0u, kwNN = 0u, rNN = 0u, orgN = 0u;
  RecAcc AN{};
  RecGeo GN{};
  if (chunk < nchunks) {
    fetch_keys(chunk, kwN, rN);
    AN = recs[rN].acc;
    GN = recs[rN].geo;
    orgN = tile_org[kwN & kmask];
    fetch_keys(chunk + W, kwNN, rNN);
  }
  for (; chunk < nchunks; chunk += W) {
    // ---- the chunk's keys; item offsets in key order
    const uint32_t i = chunk * 64u + (uint32_t)lane;
    const bool act = i < n;
    uint32_t eidx = act ? sval[i] : 0u;  // where the key's partial goes
    const uint32_t m = act ? kwN >> kMaskShift : 0u;
    // the staged tile: lane 0's key's (the wave's LDS syncs below order
    // these writes before the evaluation reads them)
    const uint32_t t0 = __builtin_amdgcn_readfirstlane(kwN & kmask);
    if constexpr (kGT) {
      const float4* __restrict__ src = reinterpret_cast<const float4*>(gq + (size_t)t0 * (TW * TH));
#pragma unroll
      for (int j = 0; j < kGTL; ++j)
        if (j * 64 + lane < kGTQ) gt[wave][j * 64 + lane] = src[j * 64 + lane];
    }
    if (act) {
      const uint32_t t = kwN & kmask;
      const RecAcc A = AN;
      const RecGeo Gg = GN;
      const uint32_t org = orgN;  // x0 | y0 << 16
      const int x0 = (int)(org & 0xffffu), y0 = (int)(org >> 16);
      const float du0 = (float)(Gg.ub - x0) + A.fu;
      const float dv0 = (float)(Gg.vb - y0) + A.fv;
      const WeightScale ws = weight_scale(A.e0, A.emin, cut);
      kpA[wave][lane] = make_float4(A.t11, A.t12, A.t22, -A.t11 * du0);
      kpB[wave][lane] = make_float4(du0, dv0, ws.d, ws.s);
      kpC[wave][lane] = A.c;
      kpT[wave][lane] = t;
    }
    const uint32_t pop = (uint32_t)__popc(m);
    uint32_t x = pop;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    const uint32_t off = x - pop;
    qoff[wave][lane] = off;
    if (lane == 63) qoff[wave][64] = x;
    // the next chunk's records (its keys arrived during the previous chunk)
    // and the keys of the one after
    AN = recs[rNN].acc;
    GN = recs[rNN].geo;
    orgN = tile_org[kwNN & kmask];
    kwN = kwNN;
    fetch_keys(chunk + 2u * W, kwNN, rNN);
    wave_lds_sync();
    float acc[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < 64;) {
      // ---- the sub-chunk: keys [k0, k1) whose items fit the slots
      const uint32_t base = qoff[wave][k0];
      const bool fits = lane >= k0 && qoff[wave][lane + 1] - base <= (uint32_t)kBwdSlots;
      const int k1 = k0 + (int)__popcll(__ballot(fits));
      const uint32_t L = qoff[wave][k1] - base;
      if (lane >= k0 && lane < k1) {
        uint32_t mm = m;
        uint32_t q = off - base;
        while (mm) {
          const uint32_t sb = (uint32_t)__builtin_ctz(mm);
          queue[wave][q++] = (uint32_t)lane | sb << 6;
          mm &= mm - 1u;
        }
      }
      wave_lds_sync();
      // ---- lanes = items: the rows each item can reach; counts per row count
      uint32_t bucket_tot[kSubBlock + 1];
#pragma unroll
      for (int b = 0; b <= kSubBlock; ++b) bucket_tot[b] = 0u;
      for (uint32_t q0 = 0; q0 < L; q0 += 64) {
        const uint32_t q = q0 + (uint32_t)lane;
        const bool has = q < L;
        const uint32_t ent = has ? queue[wave][q] : (uint32_t)k0;
        const int kl = (int)(ent & 63u), sb = (int)((ent >> 6) & 15u);
        const float4 a = kpA[wave][kl];
        const float4 b = kpB[wave][kl];
        const float xa = (float)((sb % K) * kSubBlock);
        const int by = (sb / K) * kSubBlock;
        uint32_t rows = 0u;
#pragma unroll
        for (int y = 0; y < kSubBlock; ++y) {
          const float dv = (float)(by + y) - b.y;
          const float B = fmaf(a.y, dv, a.w);
          const float t2 = a.z * dv;
          const float erow = fmaf(-t2, t2, b.z);
          // t1 at the strip's end columns, as the evaluation forms them; the
          // median of (ta, 0, tb) is the end value nearest zero, or zero when
          // t1 changes sign in between
          const float ta = fmaf(a.x, xa, B), tb = fmaf(a.x, (float)(kSubBlock - 1), ta);
          const float tm = __builtin_amdgcn_fmed3f(ta, 0.f, tb);
          rows |= (fmaf(-tm, tm, erow) >= thr ? 1u : 0u) << y;
        }
        const int ya = rows ? __builtin_ctz(rows) : 0, yb = rows ? 31 - __builtin_clz(rows) : -1;
        const int nr = has && rows ? yb - ya + 1 : 0;
        if (has) {
          queue[wave][q] = ent | (uint32_t)(nr ? ya : 0) << 10 | (uint32_t)nr << 13;
          if (nr == 0) {  // no pixel of the sub-block is inside: its sums are zero
#pragma unroll
            for (int f = 0; f < 7; ++f) slot[wave][f][q] = 0.f;
          }
        }
#pragma unroll
        for (int r = 1; r <= kSubBlock; ++r) bucket_tot[r] += (uint32_t)__popcll(__ballot(nr == r));
      }
      // bucket starts, largest row count first
      uint32_t bstart[kSubBlock + 1];
      uint32_t run = 0u;
#pragma unroll
      for (int r = kSubBlock; r >= 1; --r) {
        bstart[r] = run;
        run += bucket_tot[r];
      }
      const uint32_t Ls = run;  // items with rows
      wave_lds_sync();
      for (uint32_t q0 = 0; q0 < L; q0 += 64) {
        const uint32_t q = q0 + (uint32_t)lane;
        const uint32_t nr = q < L ? queue[wave][q] >> 13 : 0u;
        uint32_t pos = 0u;
#pragma unroll
        for (int r = 1; r <= kSubBlock; ++r) {
          const unsigned long long bal = __ballot(nr == (uint32_t)r);
          if (nr == (uint32_t)r) pos = bstart[r] + lanemask_lt_popc(bal);
          bstart[r] += (uint32_t)__popcll(bal);
        }
        if (nr) order[wave][pos] = (uint8_t)q;
      }
      wave_lds_sync();
      // ---- lanes = items by row count: the rows of one key's sub-block
      for (uint32_t s0 = 0; s0 < Ls; s0 += 64) {
        const uint32_t sidx = s0 + (uint32_t)lane;
        const bool has = sidx < Ls;
        const uint32_t q = has ? (uint32_t)order[wave][sidx] : 0u;
        const uint32_t ent = has ? queue[wave][q] : (uint32_t)k0;
        const int kl = (int)(ent & 63u), sb = (int)((ent >> 6) & 15u);
        const int ry = (int)((ent >> 10) & 7u), nr = has ? (int)(ent >> 13) : 0;
        const float4 a = kpA[wave][kl];
        const float4 b = kpB[wave][kl];
        const float c = kpC[wave][kl];
        const uint32_t t = kpT[wave][kl];
        const float t11 = a.x, t12 = a.y, t22 = a.z, P = a.w;
        const float d = b.z;
        const int bx0 = (sb % K) * kSubBlock, by = (sb / K) * kSubBlock + ry;
        const float bxf = (float)bx0;
        const float4* __restrict__ pq = reinterpret_cast<const float4*>(gq + (size_t)t * (TW * TH) + by * TW + bx0);
        const bool staged = kGT && t == t0;
        const int gbase = by * (TW / 2) + bx0 / 2;  // the item's first row in the staged tile (float4)
        float Sge = 0.f, Sa = 0.f, Sau = 0.f, S12 = 0.f, S22 = 0.f, Sb = 0.f, Sdc = 0.f;
        // row y of the item for y < nr; later rows (and lanes without an
        // item) re-read the item's last row (or the key's first) with a
        // row exponent of -inf, so they add exact zeros.  The loop ends
        // once no lane of the wave has rows left.  Each row's gamma is
        // loaded at the row's start: with four waves per SIMD the wait is
        // mostly hidden, and loading it a row ahead measured slower.
        const int nlast = nr > 0 ? nr - 1 : 0;
#pragma unroll
        for (int y = 0; y < kSubBlock; ++y) {
          if (!__any(y < nr)) break;  // uniform
          const int yl = y < nlast ? y : nlast;
          float4 cur[kSubBlock / 2];
          if (staged) {
#pragma unroll
            for (int x2 = 0; x2 < kSubBlock / 2; ++x2) cur[x2] = gt[wave][gbase + yl * (TW / 2) + x2];
          } else {
#pragma unroll
            for (int x2 = 0; x2 < kSubBlock / 2; ++x2) cur[x2] = pq[yl * (TW / 2) + x2];
          }
          const float dv = (float)(by + y) - b.y;
          const float B0 = fmaf(t11, bxf, fmaf(t12, dv, P));  // t1 at the strip's first column
          const float t2 = t22 * dv;
          const float erow = y < nr ? fmaf(-t2, t2, d) : -INFINITY;
          // per row: sum ge, sum ge j, sum ge j^2 over the strip's columns
          // j = 0..7; with t1 = B0 + t11 j the row's sum ge t1 and sum ge t1 x
          // (x = bx0 + j) follow from them, which saves the per-pixel
          // product ge t1 and the sums over it
          float rge = 0.f, rj = 0.f, rjj = 0.f;
#pragma unroll
          for (int x2 = 0; x2 < kSubBlock / 2; ++x2) {
            const float4 gg2 = cur[x2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              const int j = 2 * x2 + h;
              const float gx = h ? gg2.z : gg2.x, gy = h ? gg2.w : gg2.y;
              const float t1 = j ? fmaf(t11, (float)j, B0) : B0;
              const float w = fast_exp2(support_clamp(fmaf(-t1, t1, erow), kcut));  // the weight over s
              const float gw = fmaf(gx, c, -gy);  // dL/dw = gamma (c - c_hat)
              const float ge = w * gw;
              rge += ge;
              Sdc = fmaf(gx, w, Sdc);
              if (j) {
                rj = fmaf(ge, (float)j, rj);
                rjj = fmaf(ge, (float)(j * j), rjj);
              }
            }
          }
          const float ra = fmaf(t11, rj, B0 * rge);  // sum ge t1
          Sau = fmaf(bxf, ra, Sau);                   // + sum ge t1 x = bx0 ra + t11 rjj + B0 rj
          Sau = fmaf(t11, rjj, Sau);
          Sau = fmaf(B0, rj, Sau);
          Sge += rge;
          Sa += ra;
          S12 = fmaf(dv, ra, S12);
          Sb = fmaf(t2, rge, Sb);
          S22 = fmaf(t2 * dv, rge, S22);
        }
        if (has) {
          slot[wave][0][q] = Sge;
          slot[wave][1][q] = Sa;
          slot[wave][2][q] = Sau;
          slot[wave][3][q] = S12;
          slot[wave][4][q] = S22;
          slot[wave][5][q] = Sb;
          slot[wave][6][q] = Sdc;
        }
      }
      wave_lds_sync();
      // ---- each key adds its items in sub-block order
      if (lane >= k0 && lane < k1) {
        const uint32_t q1 = off - base + pop;
        for (uint32_t q = off - base; q < q1; ++q) {
#pragma unroll
          for (int f = 0; f < 7; ++f) acc[f] += slot[wave][f][q];
        }
      }
      wave_lds_sync();  // the next sub-chunk rewrites the queue and the slots
      k0 = k1;
    }
    if (act) {
      const float4 a = kpA[wave][lane];
      const float du0 = kpB[wave][lane].x, sw = kpB[wave][lane].w;
      // every sum is linear in the weights: scale them back by s once
      const float Sge = acc[0] * sw, Sa = acc[1] * sw, Sau = acc[2] * sw, S12 = acc[3] * sw, S22 = acc[4] * sw,
                  Sb = acc[5] * sw, Sdc = acc[6] * sw;
      // w = 2^(e0 - t1^2 - t2^2):  dL/ds = -ln2 w dL/dw, s = t1^2 + t2^2.
      const float k2 = 2.f * ln2;
      // keeps the address arithmetic here: moved up beside the load, it
      // would wait for it at the chunk's start
      asm volatile("" : "+v"(eidx));
      partial[2 * (size_t)eidx] = make_float4(-k2 * (Sau - du0 * Sa), -k2 * S12, -k2 * S22, k2 * a.x * Sa);
      partial[2 * (size_t)eidx + 1] = make_float4(k2 * (a.y * Sa + a.z * Sb), ln2 * Sge, Sdc, 0.f);
    }
    wave_lds_sync();  // the next chunk rewrites this wave's LDS
  }
}

// ---------------------------------------------------------------- dispatch
// Tile shapes compiled in (multiples of the 8x8 sub-block).
#define UG_TILE_SHAPES(X) \
  X(8, 8)                 \
  X(16, 8)                \
  X(8, 16)                \
  X(16, 16)               \
  X(32, 8)                \
  X(32, 16)               \
  X(16, 32)               \
  X(32, 32)

template <int TW, int TH, int SPLIT>
static hipError_t fwd_bg(int bg, dim3 grid, hipStream_t s, const PlaneInt* pint, const uint32_t* tp,
                         const uint32_t* ts, const uint32_t* skey, const uint32_t* srec, const Rec* rc,
                         float* img, float* ds, float ba, float bc, int kcut, unsigned long long* n_eval) {
  constexpr int NT = 64 * (TH / kSubBlock) * SPLIT;
  switch (bg) {
#define UG_BG(B)                                                                                                   \
  case B:                                                                                                          \
    if (n_eval)                                                                                                    \
      hipLaunchKernelGGL((k_accum_fwd<TW, TH, B, true, SPLIT>), grid, dim3(NT), 0, s, pint, tp, ts, skey, srec,    \
                         rc, img, ds, ba, bc, kcut, n_eval);                                                       \
    else                                                                                                           \
      hipLaunchKernelGGL((k_accum_fwd<TW, TH, B, false, SPLIT>), grid, dim3(NT), 0, s, pint, tp, ts, skey, srec,   \
                         rc, img, ds, ba, bc, kcut, n_eval);                                                       \
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

int accum_default_ppl(int tile_w, int tile_h) {
  (void)tile_h;
  return tile_w / kSubBlock;
}

bool accum_config_supported(int tile_w, int tile_h, int ppl, int lds_batch) {
  if (!(lds_batch == 32 || lds_batch == 64 || lds_batch == 128 || lds_batch == 256)) return false;
  if (ppl != tile_w / kSubBlock) return false;
#define UG_OK_SHAPE(W, H) \
  if (tile_w == W && tile_h == H) return true;
  UG_TILE_SHAPES(UG_OK_SHAPE)
#undef UG_OK_SHAPE
  return false;
}

hipError_t launch_accum_fwd(int tile_w, int tile_h, int lds_batch, int split, const PlaneInt* pint,
                            const uint32_t* tile_plane, const uint32_t* tile_start, const uint32_t* skey,
                            const uint32_t* srec, const Rec* recs, float* image, float* dsave,
                            float bg_alpha, float bg_color, bool cut, uint32_t num_tiles,
                            unsigned long long* n_eval, hipStream_t s) {
  const dim3 grid(num_tiles);
  const int kcut = cut ? kCutBits : kNoCutBits;
#define UG_LAUNCH_SHAPE(W, H)                                                                                    \
  if (tile_w == W && tile_h == H)                                                                                \
    return split == 2 ? fwd_bg<W, H, 2>(lds_batch, grid, s, pint, tile_plane, tile_start, skey, srec, recs,       \
                                        image, dsave, bg_alpha, bg_color, kcut, n_eval)                          \
                      : fwd_bg<W, H, 1>(lds_batch, grid, s, pint, tile_plane, tile_start, skey, srec, recs,       \
                                        image, dsave, bg_alpha, bg_color, kcut, n_eval);
  UG_TILE_SHAPES(UG_LAUNCH_SHAPE)
#undef UG_LAUNCH_SHAPE
  return hipErrorInvalidValue;
}

uint32_t bwd_prep_blocks(int tile_w, int tile_h, uint32_t num_tiles) {
  const size_t groups = (size_t)num_tiles * tile_w * tile_h / 4;  // four pixels per thread
  return (uint32_t)((groups + 255) / 256);
}

hipError_t launch_bwd_prep(int tile_w, int tile_h, const PlaneInt* pint, const uint32_t* tile_plane,
                           const float* image, const float* second, bool mse, float scale, float* loss_part,
                           const float* dsave, float* gq, uint32_t num_tiles, hipStream_t s) {
  const dim3 grid(bwd_prep_blocks(tile_w, tile_h, num_tiles));
  float4* g4 = reinterpret_cast<float4*>(gq);
  const int vec = (reinterpret_cast<uintptr_t>(image) | reinterpret_cast<uintptr_t>(second) |
                   reinterpret_cast<uintptr_t>(dsave)) % 16 == 0;
#define UG_PREP(W, H)                                                                                              \
  if (tile_w == W && tile_h == H) {                                                                                \
    if (mse)                                                                                                       \
      hipLaunchKernelGGL((k_bwd_prep<W, H, true>), grid, dim3(256), 0, s, pint, tile_plane, image, second, dsave,  \
                         g4, num_tiles, vec, scale, loss_part);                                                    \
    else                                                                                                           \
      hipLaunchKernelGGL((k_bwd_prep<W, H, false>), grid, dim3(256), 0, s, pint, tile_plane, image, second, dsave, \
                         g4, num_tiles, vec, scale, loss_part);                                                    \
    return hipGetLastError();                                                                                      \
  }
  UG_TILE_SHAPES(UG_PREP)
#undef UG_PREP
  return hipErrorInvalidValue;
}

// Launches with at least this key capacity (about 100,000 64-key chunks)
// stage their chunks' gamma tiles in LDS when the tile fits.
constexpr uint32_t kGTMinKeys = 1u << 22;

template <int TW, int TH>
static hipError_t bwd_launch(bool gt, uint32_t blocks, hipStream_t s, const Ctrl* ctrl, const uint32_t* tile_org,
                             const uint32_t* skey, const uint32_t* sval, const uint32_t* srec, const Rec* recs,
                             const float2* g2, float4* p4, int kcut) {
  if constexpr (TW * TH <= 512) {
    if (gt) {
      hipLaunchKernelGGL((k_accum_bwd<TW, TH, true>), dim3(blocks), dim3(256), 0, s, ctrl, tile_org, skey, sval,
                         srec, recs, g2, p4, kcut);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((k_accum_bwd<TW, TH, false>), dim3(blocks), dim3(256), 0, s, ctrl, tile_org, skey, sval, srec,
                     recs, g2, p4, kcut);
  return hipGetLastError();
}

hipError_t launch_accum_bwd(int tile_w, int tile_h, const Ctrl* ctrl, const uint32_t* tile_org,
                            const uint32_t* skey, const uint32_t* sval,
                            const uint32_t* srec, const Rec* recs,
                            const float* gq, float* partial, bool cut, uint32_t key_cap, hipStream_t s) {
  const float2* g2 = reinterpret_cast<const float2*>(gq);
  float4* p4 = reinterpret_cast<float4*>(partial);
  uint32_t want = (key_cap / 64u + 4u) / 4u;
  const uint32_t blocks = want < 1u ? 1u : (want > 16384u ? 16384u : want);
  const bool gt = key_cap >= kGTMinKeys;
#define UG_BWD(W, H)                                                                                          \
  if (tile_w == W && tile_h == H) return bwd_launch<W, H>(gt, blocks, s, ctrl, tile_org, skey, sval, srec, recs, \
                                                          g2, p4, cut ? kCutBits : kNoCutBits);
  UG_TILE_SHAPES(UG_BWD)
#undef UG_BWD
  return hipErrorInvalidValue;
}

}  // namespace ug
