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
#include <cfloat>

#include "ug_conic.h"
#include "ug_kernels.h"

namespace ug {

// ---------------------------------------------------------------- plane set-up
// FP64 constants of plane p's pose (an invalid pose is marked and skipped; the
// cull raises the flag) and the float constants of its cull.
__device__ __forceinline__ PlaneCull plane_setup(const ug_planes& pl, const PlaneInt* __restrict__ pint, int p,
                                                 PlaneConst* __restrict__ pc, PlaneCull* __restrict__ pcf) {
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
  PlaneCull q;
  for (int k = 0; k < 3; ++k) {
    q.o[k] = pl.origin[3 * p + k];
    q.r3[k] = (float)c.rinv[6 + k] + 0.f;  // -0 as +0 (same test; one group key per normal)
  }
  q.valid = c.valid;
  q.pad = 0;
  pcf[p] = q;
  return q;
}

// Bits of a float in the order of its value (-0 before +0).
__device__ __forceinline__ uint32_t float_order(float x) {
  const uint32_t b = __float_as_uint(x);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

// Whether two planes' group keys (validity, r3, o[0], o[1]) agree bit for bit.
__device__ __forceinline__ bool group_key_eq(const PlaneCull& a, const PlaneCull& b) {
  return a.valid == b.valid && __float_as_uint(a.r3[0]) == __float_as_uint(b.r3[0]) &&
         __float_as_uint(a.r3[1]) == __float_as_uint(b.r3[1]) && __float_as_uint(a.r3[2]) == __float_as_uint(b.r3[2]) &&
         __float_as_uint(a.o[0]) == __float_as_uint(b.o[0]) && __float_as_uint(a.o[1]) == __float_as_uint(b.o[1]);
}

// A 32-bit mix of the group key's bits (equal keys, equal hashes).
__device__ __forceinline__ uint32_t group_key_hash(const PlaneCull& q) {
  const uint32_t w[6] = {(uint32_t)q.valid, __float_as_uint(q.r3[0]), __float_as_uint(q.r3[1]),
                         __float_as_uint(q.r3[2]), __float_as_uint(q.o[0]), __float_as_uint(q.o[1])};
  uint32_t h = 0x811c9dc5u;
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    h = (h ^ w[i]) * 0x9e3779b1u;
    h ^= h >> 15;
  }
  return h;
}

// Groups of at least this many planes are searched by the cull.
constexpr uint32_t kGroupSearch = 8;

// One thread per plane; thread 0 clears the control block.  With group (a
// launch of one block, at most kGroupMaxPlanes planes) the planes are also
// ordered by (hash of the group key, o[2], index): each plane counts the
// planes before it in that order (its position), those with a smaller hash
// (its group's first position) and those with its hash (the group's size).
// Every plane then checks that its key equals that of its group's first
// plane; if two keys ever share a hash, the cull tests every plane instead.
__global__ __launch_bounds__(256) void k_init(ug_planes pl, const PlaneInt* __restrict__ pint,
                                              PlaneConst* __restrict__ pc, PlaneCull* __restrict__ pcf,
                                              PlaneGroups* __restrict__ pg, int group, Ctrl* __restrict__ ctrl) {
  __shared__ PlaneCull s_q[kGroupMaxPlanes];
  __shared__ unsigned long long s_hz[kGroupMaxPlanes];  // hash << 32 | order bits of o[2]
  __shared__ uint32_t s_first[kGroupMaxPlanes];         // plane at each group's first position
  __shared__ uint32_t s_big, s_bad;
  const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid == 0) {
    ctrl->n_rec = 0;
    ctrl->n_key = 0;
    ctrl->n_eval = 0;
    ctrl->n_exec = 0;
    ctrl->flags = 0;
    ctrl->n_rec_eff = 0;
    ctrl->n_key_eff = 0;
  }
  const int p = (int)gid;
  const bool mine = p < pl.p;
  PlaneCull q{};
  if (mine) q = plane_setup(pl, pint, p, pc, pcf);
  if (!group) {  // uniform (a launch argument)
    if (gid == 0) pg->use = 0u;
    return;
  }
  const uint32_t h = group_key_hash(q);
  const unsigned long long hz = (unsigned long long)h << 32 | float_order(q.o[2]);
  if (mine) {
    s_q[p] = q;
    s_hz[p] = hz;
  }
  if (threadIdx.x == 0) {
    s_big = 0u;
    s_bad = 0u;
  }
  __syncthreads();
  uint32_t rank = 0u, below = 0u, same = 0u;
  if (mine) {
#pragma unroll 8
    for (int j = 0; j < pl.p; ++j) {  // the same j in every lane: broadcast reads
      const unsigned long long o = s_hz[j];
      rank += (o < hz || (o == hz && j < p)) ? 1u : 0u;
      const uint32_t oh = (uint32_t)(o >> 32);
      below += oh < h ? 1u : 0u;
      same += oh == h ? 1u : 0u;
    }
    pg->perm[rank] = (uint32_t)p;
    pg->oz[rank] = q.o[2];
    pg->end[rank] = below + same;
    if (rank == below) s_first[below] = (uint32_t)p;
    if (q.valid && same >= kGroupSearch) atomicOr(&s_big, 1u);
  }
  __syncthreads();
  if (mine && !group_key_eq(q, s_q[s_first[below]])) atomicOr(&s_bad, 1u);
  __syncthreads();
  if (threadIdx.x == 0) pg->use = (s_big && !s_bad) ? 1u : 0u;
}

// Conservative float pre-test of Phase 1: false only if the exact (double)
// test surely rejects the pair.  The float m3 is off by at most a few ulps of
// sum |r3_i (mu_i - o_i)|, the float Sigma'_33 by a few ulps relative; the
// margins below are ten times larger.
// Split in two: Sigma'_33 depends on the plane through r3 only, so planes
// sharing r3 share it.
__device__ __forceinline__ float cull_s33(const GaussT<float>& G, const PlaneCull& P) {
  float g3[3];
  fsub(G, P.r3[0], P.r3[1], P.r3[2], g3);
  return g3[0] * g3[0] + g3[1] * g3[1] + g3[2] * g3[2];
}
__device__ __forceinline__ bool cull_test(const GaussT<float>& G, const PlaneCull& P, float S33, float chi2) {
  const float d0 = G.mu[0] - P.o[0], d1 = G.mu[1] - P.o[1], d2 = G.mu[2] - P.o[2];
  const float m3 = P.r3[0] * d0 + P.r3[1] * d1 + P.r3[2] * d2;
  const float slack = 2e-6f * (fabsf(P.r3[0] * d0) + fabsf(P.r3[1] * d1) + fabsf(P.r3[2] * d2));
  const float a = fmaxf(fabsf(m3) - slack, 0.f);
  return a * a <= chi2 * S33 * 1.0002f;  // false for NaN as well
}
__device__ __forceinline__ bool cull_maybe(const GaussT<float>& G, const PlaneCull& P, float chi2) {
  return cull_test(G, P, cull_s33(G, P), chi2);
}

// Sorted positions [lo, hi) of a plane group (planes sharing r3, o[0] and
// o[1], sorted by o[2]; P0 one of them) outside which cull_maybe rejects G.
// It accepts only if |m3| - slack <= sqrt(chi2 S33 1.0002) up to float
// rounding, where |m3| >= |r3_2 d2| - A with A = |r3_0 d0| + |r3_1 d1| (the
// same for the whole group) and slack <= 2e-6 (A + |r3_2 d2|), so
// |mu_2 - o_2| <= (sqrt(chi2 S33 1.0002) + A) (1 + 3e-6) / |r3_2|; the factors
// below widen that well beyond every rounding of this bound, and an infinite
// or undefined bound (no cut-off, r3_2 = 0) keeps the whole group.
__device__ __forceinline__ void group_window(const GaussT<float>& G, const PlaneCull& P0, float S33, float chi2,
                                             const float* oz, int& lo, int& hi) {
  const float d0 = G.mu[0] - P0.o[0], d1 = G.mu[1] - P0.o[1];
  const float A = fabsf(P0.r3[0] * d0) + fabsf(P0.r3[1] * d1);
  const float D = (sqrtf(chi2 * S33 * 1.0002f) + A) * 1.001f / fabsf(P0.r3[2]);
  const float mu = G.mu[2];
  const float Dw = D * 1.001f + 1e-6f * fabsf(mu);
  if (!(Dw <= FLT_MAX)) return;
  const float vlo = mu - Dw, vhi = mu + Dw;
  int a = lo, b = hi;  // first position with oz >= vlo
  while (a < b) {
    const int m = (a + b) >> 1;
    if (oz[m] < vlo) a = m + 1; else b = m;
  }
  int c = a, d = hi;  // first position with oz > vhi
  while (c < d) {
    const int m = (c + d) >> 1;
    if (oz[m] <= vhi) c = m + 1; else d = m;
  }
  lo = a;
  hi = c;
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
// A group of LPG lanes per Gaussian, lane k of a group testing planes k,
// k + LPG, ...; the group ORs its bits.  A block covers gpb Gaussians in
// rounds of 256 / LPG.  Small inputs spread a Gaussian over several lanes
// (and blocks over fewer Gaussians) so enough waves run; large ones use one
// lane per Gaussian, whose plane loads are then uniform (scalar).  A pair
// becomes a record iff the conservative float test
// of Phase 1 (Eq. 13's box along the normal meets the plane, i.e. the plane
// meets the Eq. 12 ellipsoid) passes; the test only errs towards accepting a
// pair whose plane narrowly misses the ellipsoid, and such a record has an
// empty support, so it adds exactly zero everywhere.  Acceptance is kept as
// one bit per (Gaussian, plane), 64 planes per word.
template <int LPG>
__global__ __launch_bounds__(256) void k_cull_count(ug_gaussians g, const PlaneCull* __restrict__ pcf,
                                                    const PlaneGroups* __restrict__ pg, RenderParams rp, int gpb,
                                                    uint32_t* __restrict__ cnt_rec,
                                                    unsigned long long* __restrict__ accbits,
                                                    uint32_t* __restrict__ blk_tot, Ctrl* __restrict__ ctrl) {
  __shared__ uint32_t s_tot;
  // grouped planes (one lane per Gaussian): each group is searched for the
  // window of planes the pre-test can accept, and only those are tested
  __shared__ uint16_t s_perm[kGroupMaxPlanes], s_end[kGroupMaxPlanes];
  __shared__ float s_oz[kGroupMaxPlanes];
  const bool grouped = LPG == 1 && pg->use != 0u;  // uniform
  if (grouped) {
    for (int j = (int)threadIdx.x; j < rp.p; j += 256) {
      s_perm[j] = (uint16_t)pg->perm[j];
      s_end[j] = (uint16_t)pg->end[j];
      s_oz[j] = pg->oz[j];
    }
  }
  if (threadIdx.x == 0) s_tot = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    for (int p = 0; p < rp.p; ++p)
      if (!pcf[p].valid) {
        atomicOr(&ctrl->flags, kFlagNonfinite);
        break;
      }
  }
  __syncthreads();
  const int nch = (rp.p + 63) / 64;
  const int sub = LPG == 1 ? 0 : (int)threadIdx.x % LPG;
  uint32_t mine = 0;
  for (int r0 = 0; r0 < gpb; r0 += 256 / LPG) {
    const int gi = blockIdx.x * gpb + r0 + (int)threadIdx.x / LPG;
    const bool has = gi < rp.n;
    GaussT<float> G;
    G.finite = false;
    if (has) load_gauss<float>(g, gi, rp.beta, G);
    if (has && sub == 0 && !G.finite) atomicOr(&ctrl->flags, kFlagNonfinite);
    const bool live = has && G.finite;
    uint32_t count = 0;
    if (grouped) {
      // at most 256 planes: four acceptance words, the word of plane q picked
      // by compares (no indexed register array)
      unsigned long long w0 = 0ull, w1 = 0ull, w2 = 0ull, w3 = 0ull;
      if (live) {
        for (int i = 0; i < rp.p;) {  // uniform: the groups in order
          const int e = min(max((int)s_end[i], i + 1), rp.p);  // a group ends past its start
          // the group's shared constants; each plane differs only in o[2]
          PlaneCull pf = pcf[s_perm[i]];
          const float S33 = cull_s33(G, pf);
          int lo = i, hi = pf.valid ? e : i;
          if ((uint32_t)(e - i) >= kGroupSearch) group_window(G, pf, S33, rp.chi2, s_oz, lo, hi);
          for (int j = lo; j < hi; ++j) {
            const int q = s_perm[j];
            pf.o[2] = s_oz[j];
            if (cull_test(G, pf, S33, rp.chi2)) {
              const unsigned long long bit = 1ull << (q & 63);
              const int w = q >> 6;
              w0 |= w == 0 ? bit : 0ull;
              w1 |= w == 1 ? bit : 0ull;
              w2 |= w == 2 ? bit : 0ull;
              w3 |= w == 3 ? bit : 0ull;
            }
          }
          i = e;
        }
      }
      if (has) {
        for (int c = 0; c < nch; ++c)
          accbits[(size_t)gi * nch + c] = c == 0 ? w0 : (c == 1 ? w1 : (c == 2 ? w2 : w3));
        count = (uint32_t)(__popcll(w0) + __popcll(w1) + __popcll(w2) + __popcll(w3));
        cnt_rec[gi] = count;
        mine += count;
      }
      continue;
    }
    for (int c = 0; c < nch; ++c) {
      const int pend = min(64, rp.p - c * 64);
      unsigned long long bits = 0;
      for (int j = sub; j < pend; j += LPG) {
        const PlaneCull pf = pcf[c * 64 + j];
        if (live && pf.valid && cull_maybe(G, pf, rp.chi2)) bits |= 1ull << j;
      }
#pragma unroll
      for (int o = 1; o < LPG; o <<= 1) bits |= __shfl_xor(bits, o, 64);
      if (has && sub == 0) accbits[(size_t)gi * nch + c] = bits;
      count += (uint32_t)__popcll(bits);
    }
    if (has && sub == 0) {
      cnt_rec[gi] = count;
      mine += count;
    }
  }
  if (mine) atomicAdd(&s_tot, mine);
  __syncthreads();
  if (threadIdx.x == 0) blk_tot[blockIdx.x] = s_tot;
}

// Offsets and the compact (Gaussian, plane) list, Gaussian-major with planes
// ascending.  A block covers m consecutive count blocks (gpb Gaussians in
// all).  The last block publishes the total and the capacity check.
__global__ __launch_bounds__(256) void k_cull_write(RenderParams rp, int gpb, uint32_t m, uint32_t nblk,
                                                    const uint32_t* __restrict__ cnt_rec,
                                                    const unsigned long long* __restrict__ accbits,
                                                    const uint32_t* __restrict__ blk_tot,
                                                    unsigned long long* __restrict__ off_rec,
                                                    uint2* __restrict__ rec_pair, Ctrl* __restrict__ ctrl) {
  __shared__ unsigned long long s_sh[4];
  const int nch = (rp.p + 63) / 64;
  // the first round's counts and first acceptance word do not depend on the
  // block prefix: load them before it so the two round trips overlap
  const int gi0 = blockIdx.x * gpb + threadIdx.x;
  const bool has0 = (int)threadIdx.x < gpb && gi0 < rp.n;
  const unsigned long long cnt0 = has0 ? cnt_rec[gi0] : 0ull;
  const unsigned long long bits0 = has0 ? accbits[(size_t)gi0 * nch] : 0ull;
  unsigned long long carry = block_prefix(blk_tot, blockIdx.x * m, s_sh);
  for (int r0 = 0; r0 < gpb; r0 += 256) {
    const int gi = blockIdx.x * gpb + r0 + threadIdx.x;
    const bool has = r0 + (int)threadIdx.x < gpb && gi < rp.n;
    const unsigned long long cnt = r0 == 0 ? cnt0 : (has ? cnt_rec[gi] : 0ull);
    unsigned long long tot;
    const unsigned long long base = carry + block_exscan_256<unsigned long long>(cnt, s_sh, tot);
    carry += tot;
    if (!has) continue;
    off_rec[gi] = base;
    unsigned long long r = base;
    for (int c = 0; c < nch; ++c) {
      unsigned long long bits = (r0 == 0 && c == 0) ? bits0 : accbits[(size_t)gi * nch + c];
      while (bits) {
        const int j = __builtin_ctzll(bits);
        bits &= bits - 1ull;
        if (r < rp.rec_cap) rec_pair[r] = make_uint2((uint32_t)gi, (uint32_t)(c * 64 + j));
        ++r;
      }
    }
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

// Records per block from the device-side record count: whole rounds of 256
// spread evenly over the grid (sized by the host for the capacity), so every
// block has a share whatever the head-room.  The record and emission kernels
// use the same split (the emission's block prefix reads the record blocks'
// totals).
__device__ __forceinline__ uint32_t record_rpb_dev(uint32_t nrec, uint32_t grid) {
  const uint32_t rounds = (nrec + 255u) / 256u;
  const uint32_t per = (rounds + grid - 1u) / grid;
  return (per < 1u ? 1u : per) * 256u;
}
__device__ __forceinline__ void emit_keys(const RecAcc& ra, const RecGeo& geo, const uint4& spans, const PlaneInt& PI,
                                          int box_mode, int TW, int TH, uint32_t r, uint32_t e, uint32_t e_end,
                                          uint32_t* __restrict__ key_tile, uint32_t* __restrict__ rec_of_key) {
  const int mshift = key_mask_shift(TW, TH);
  const int umin = geo.tx0 * TW;
  const int umax = min(geo.tx1 * TW + TW - 1, PI.W - 1);
  BandPrep bp;
  const bool ok = band_prep(ra, geo.ub, geo.vb, bp);
  if (box_mode == UG_BOX_ROWS && !ok) return;
  for (int ty = geo.ty0; ty <= geo.ty1; ++ty) {
    int tx0 = geo.tx0, tx1 = geo.tx1;
    if (box_mode == UG_BOX_ROWS) {
      // the record kernel's span for the first kRowSpans rows, else recomputed
      const int i = ty - (int)geo.ty0;
      if (i < kRowSpans) {
        const uint32_t w = i == 0 ? spans.x : (i == 1 ? spans.y : (i == 2 ? spans.z : spans.w));
        tx0 = (int)(w & 0xffffu);
        tx1 = (int)(w >> 16);
        if (tx0 > tx1) continue;
      } else if (!rows_span(bp, ty, TW, TH, PI.H, umin, umax, tx0, tx1)) {
        continue;
      }
    }
    int bua[kMaxBands], buz[kMaxBands];
    if (ok) {
      band_ranges(bp, ty, TH, PI.H, umin, umax, bua, buz);
    } else {
#pragma unroll
      for (int b = 0; b < kMaxBands; ++b) {
        bua[b] = 1;
        buz[b] = 0;
      }
    }
    const uint32_t rowbase = PI.tile_off + (uint32_t)ty * (uint32_t)PI.ntx;
    for (int tx = tx0; tx <= tx1; ++tx) {
      if (e < e_end) {
        key_tile[e] = (rowbase + (uint32_t)tx) | (tile_mask(bua, buz, tx, TW) << mshift);
        rec_of_key[e] = r;
      }
      ++e;
    }
  }
}

// Launches with up to kStagePlanes planes give the record kernel and the
// record adjoint their planes' constants from LDS (copied once per block)
// instead of gathering each record's plane from memory: a wave's 64 records
// touch many planes, and those gathers queue on the vector-memory address
// path.
constexpr int kStagePlanes = 256;
static_assert(sizeof(PlaneConst) % 8 == 0 && sizeof(PlaneInt) % 8 == 0, "LDS plane staging layout");

// FP64 in-plane conic and footprint of each record; key counts and the
// block's total.  STAGE (launches of up to kStagePlanes planes): the planes'
// constants are copied to LDS once per block (512 threads, so the 56 KB of
// a 256-plane launch still leaves the 16 waves per CU the registers allow)
// instead of being gathered per record from memory.
template <bool STAGE>
__global__ __launch_bounds__(STAGE ? 512 : 256) void k_record(ug_gaussians g, const PlaneConst* __restrict__ pc,
                                                              const PlaneInt* __restrict__ pint, RenderParams rp,
                                                              const uint2* __restrict__ rec_pair,
                                                              Rec* __restrict__ recs, uint32_t* __restrict__ rec_nkey,
                                                              uint32_t* __restrict__ blk_tot,
                                                              const Ctrl* __restrict__ ctrl) {
  constexpr uint32_t NT = STAGE ? 512u : 256u;
  extern __shared__ double s_planes[];  // STAGE: rp.p PlaneConst, then rp.p PlaneInt
  __shared__ uint32_t s_tot;
  const uint32_t nrec = ctrl->n_rec_eff;
  const uint32_t rpb = record_rpb_dev(nrec, gridDim.x);
  const uint32_t r_begin = blockIdx.x * rpb;
  if (r_begin >= nrec) return;  // uniform
  PlaneConst* s_pc = reinterpret_cast<PlaneConst*>(s_planes);
  PlaneInt* s_pi = reinterpret_cast<PlaneInt*>(s_pc + rp.p);
  if (STAGE) {
    for (int q = (int)threadIdx.x; q < rp.p; q += (int)NT) {
      s_pc[q] = pc[q];
      s_pi[q] = pint[q];
    }
  }
  if (threadIdx.x == 0) s_tot = 0;
  __syncthreads();
  const double chi2 = (double)rp.chi2;
  const bool rows = rp.box_mode == UG_BOX_ROWS && !rp.box_support;  // the records carry their row spans
  uint32_t mine = 0;
  const uint32_t r_end = min(r_begin + rpb, nrec);
  for (uint32_t r = r_begin + threadIdx.x; r < r_end; r += NT) {
    const uint2 gp = rec_pair[r];
    GaussIn G;
    load_gauss(g, (int)gp.x, (double)rp.beta, G);
    const PlaneConst& P = STAGE ? s_pc[gp.y] : pc[gp.y];
    const PlaneInt& PI = STAGE ? s_pi[gp.y] : pint[gp.y];
    const PlaneT<double> Pd = plane_as<double>(P);
    Conic k;
    const bool meets = conic_cull(G, Pd, chi2, k);
    conic_full(G, Pd, k);
    Footprint f;
    // Box support: the FP64 Phase-1 decision is final (a pair the
    // conservative float cull let through would otherwise fill its box).
    const bool ok = rp.box_support ? (meets && make_box_record(G, P, PI, k, chi2, f))
                                   : make_footprint(G, P, PI, k, chi2, rp.box_mode, rp.tile_w, rp.tile_h, f);
    if (!ok) {
      // the plane cuts the ellipsoid (or box) outside the image: a record with no keys
      f.keys = 0;
      f.acc = RecAcc{0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      f.geo = RecGeo{0, 0, 1, 0, 1, 0};
    }
    recs[r].acc = f.acc;
    recs[r].geo = f.geo;
    if (rows) *reinterpret_cast<uint4*>(recs[r].spans) = make_uint4(f.spans[0], f.spans[1], f.spans[2], f.spans[3]);
    rec_nkey[r] = f.keys;
    mine += f.keys;
  }
  if (mine) atomicAdd(&s_tot, mine);
  __syncthreads();
  if (threadIdx.x == 0) blk_tot[blockIdx.x] = s_tot;
}

// Key offsets (block prefix + in-block scan) and key emission.  The last
// active block publishes the key total and the capacity check.
__global__ __launch_bounds__(256) void k_emit(const PlaneInt* __restrict__ pint, RenderParams rp,
                                              const uint2* __restrict__ rec_pair, const Rec* __restrict__ recs,
                                              const uint32_t* __restrict__ rec_nkey,
                                              const uint32_t* __restrict__ blk_tot, uint32_t* __restrict__ rec_koff,
                                              Ctrl* __restrict__ ctrl, uint32_t* __restrict__ key_tile,
                                              uint32_t* __restrict__ rec_of_key) {
  __shared__ unsigned long long s_sh[4];
  const uint32_t nrec = ctrl->n_rec_eff;
  const uint32_t rpb = record_rpb_dev(nrec, gridDim.x);
  const uint32_t r_begin = blockIdx.x * rpb;
  if (r_begin >= nrec) return;  // uniform
  const uint32_t nact = (nrec + rpb - 1) / rpb;
  const uint32_t r_end = min(r_begin + rpb, nrec);
  // Each round's record data is loaded one round ahead (the first round's
  // before the block prefix), so its round trip overlaps the previous
  // round's scan and emission.  Lanes past the block's records load its last
  // record and drop it (no branch around the loads: the wait at a branch's
  // join would take every load in flight).  The plane lookup needs the plane
  // index first; it is issued at the end of the previous round, before the
  // next prefetch, so the emission waits for it and not for the prefetch
  // (loads complete in issue order as far as the waits can tell).
  uint32_t r = r_begin + threadIdx.x;
  bool act = r < r_end;
  uint32_t pl, nk;
  RecAcc ra;
  RecGeo ge;
  uint4 sp;
  {
    const uint32_t rl = act ? r : r_end - 1u;
    pl = rec_pair[rl].y;
    ra = recs[rl].acc;
    ge = recs[rl].geo;
    sp = *reinterpret_cast<const uint4*>(recs[rl].spans);
    nk = act ? rec_nkey[rl] : 0u;
  }
  unsigned long long carry = block_prefix(blk_tot, blockIdx.x, s_sh);
  PlaneInt PI = pint[pl];
  for (uint32_t r0 = r_begin; r0 < r_end; r0 += 256) {
    const uint32_t rn = r + 256u;
    const bool actn = rn < r_end;
    const uint32_t rl = actn ? rn : r_end - 1u;
    const uint32_t pln = rec_pair[rl].y;
    const RecAcc ran = recs[rl].acc;
    const RecGeo gen = recs[rl].geo;
    const uint4 spn = *reinterpret_cast<const uint4*>(recs[rl].spans);
    const uint32_t nkl = rec_nkey[rl];
    const uint32_t nkn = actn ? nkl : 0u;
    unsigned long long tot;
    const unsigned long long koff = carry + block_exscan_256<unsigned long long>(nk, s_sh, tot);
    carry += tot;
    if (act) {
      rec_koff[r] = (uint32_t)(koff < rp.key_cap ? koff : rp.key_cap);
      if (nk > 0 && koff + nk <= rp.key_cap)
        emit_keys(ra, ge, sp, PI, rp.box_mode, rp.tile_w, rp.tile_h, r, (uint32_t)koff, (uint32_t)(koff + nk),
                  key_tile, rec_of_key);
    }
    r = rn;
    act = actn;
    nk = nkn;
    ra = ran;
    ge = gen;
    sp = spn;
    PI = pint[pln];
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
// Final gradient of Gaussian i from the sum of its records' contributions
// (dmu[3], dL[6], da, dc): dL_kk / dl_kk = 2 l_kk (Eq. 11).
__device__ __forceinline__ void write_gauss_grad(const ug_gaussians& g, int i, const float (&acc)[kGradFields],
                                                 float* __restrict__ d_means, float* __restrict__ d_lraw,
                                                 float* __restrict__ d_int, float* __restrict__ d_op, int accumulate) {
  float v[kGradFields];
#pragma unroll
  for (int j = 0; j < kGradFields; ++j) v[j] = acc[j];
  v[3] *= 2.f * g.lraw[6 * i + 0];
  v[6] *= 2.f * g.lraw[6 * i + 3];
  v[8] *= 2.f * g.lraw[6 * i + 5];
  if (accumulate) {
    for (int j = 0; j < 3; ++j) d_means[3 * i + j] += v[j];
    for (int j = 0; j < 6; ++j) d_lraw[6 * i + j] += v[3 + j];
    d_op[i] += v[9];
    d_int[i] += v[10];
  } else {
    for (int j = 0; j < 3; ++j) d_means[3 * i + j] = v[j];
    for (int j = 0; j < 6; ++j) d_lraw[6 * i + j] = v[3 + j];
    d_op[i] = v[9];
    d_int[i] = v[10];
  }
}

// Lanes = records, 64 consecutive records per wave: the sum of the record's
// keys' partial derivatives (contiguous in emission order), the chain rule
// through the record construction (FP32: the adjoint's tolerance is 1e-3),
// then the per-Gaussian sum.  A Gaussian's records are contiguous, so equal
// Gaussian ids are added with a segmented scan across the wave; a Gaussian
// whose records all sit in one wave gets its gradient here.  Each wave also
// leaves its first and last segment sums in side[] for the Gaussians that
// span waves (k_gauss_grad).  Deterministic, no atomics.
// Float plane constants as the record adjoint stages them in LDS (o, R^-1,
// e1, e2, |det R|, sx, sy).
constexpr int kPlaneFloats = 21;

__device__ __forceinline__ void plane_to_lds(const PlaneT<float>& P, float* d) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    d[k] = P.o[k];
    d[12 + k] = P.e1[k];
    d[15 + k] = P.e2[k];
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) d[3 + k] = P.rinv[k];
  d[18] = P.absdet;
  d[19] = P.sx;
  d[20] = P.sy;
}

__device__ __forceinline__ PlaneT<float> plane_from_lds(const float* d) {
  PlaneT<float> P;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    P.o[k] = d[k];
    P.e1[k] = d[12 + k];
    P.e2[k] = d[15 + k];
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) P.rinv[k] = d[3 + k];
  P.absdet = d[18];
  P.sx = d[19];
  P.sy = d[20];
  return P;
}

__global__ __launch_bounds__(256) void k_record_adjoint(ug_gaussians g, const PlaneConst* __restrict__ pc,
                                                        RenderParams rp, const Ctrl* __restrict__ ctrl,
                                                        const uint2* __restrict__ rec_pair,
                                                        const uint32_t* __restrict__ rec_koff,
                                                        const float4* __restrict__ partial,
                                                        const uint32_t* __restrict__ cnt_rec,
                                                        const unsigned long long* __restrict__ off_rec,
                                                        float* __restrict__ side, float* __restrict__ d_means,
                                                        float* __restrict__ d_lraw, float* __restrict__ d_int,
                                                        float* __restrict__ d_op, int accumulate) {
  extern __shared__ float s_plane[];  // rp.p x kPlaneFloats when staged
  const bool staged = rp.p <= kStagePlanes;
  if (staged) {
    for (int q = threadIdx.x; q < rp.p; q += 256) plane_to_lds(plane_as<float>(pc[q]), s_plane + q * kPlaneFloats);
    __syncthreads();
  }
  const bool ok = (ctrl->flags & (kFlagRecCap | kFlagKeyCap)) == 0;
  const uint32_t nrec = ok ? ctrl->n_rec_eff : 0u;
  const uint32_t nw = (nrec + 63u) / 64u;
  const float chi2 = rp.chi2;
  const int lane = threadIdx.x & 63;
  for (uint32_t w = blockIdx.x * 4u + (threadIdx.x >> 6); w < nw; w += gridDim.x * 4u) {
    const uint32_t r = w * 64u + (uint32_t)lane;
    const bool act = r < nrec;
    float v[kGradFields];
#pragma unroll
    for (int j = 0; j < kGradFields; ++j) v[j] = 0.f;
    uint32_t gid = 0xffffffffu;
    if (act) {
      const uint2 gp = rec_pair[r];
      gid = gp.x;
      const uint32_t k0 = rec_koff[r], k1 = rec_koff[r + 1];
      // the Gaussian's parameters are loaded with the key range, so the two
      // round trips overlap
      const GaussRaw gr = load_gauss_raw(g, (int)gp.x);
      float4 a = make_float4(0.f, 0.f, 0.f, 0.f), c = a;
      // two keys per step, both loaded before either is added (same order
      // of additions as one key at a time)
      for (uint32_t k = k0; k < k1; k += 2) {
        const float4 x0 = partial[2 * (size_t)k], y0 = partial[2 * (size_t)k + 1];
        const bool two = k + 1 < k1;
        float4 x1 = make_float4(0.f, 0.f, 0.f, 0.f), y1 = x1;
        if (two) {
          x1 = partial[2 * (size_t)k + 2];
          y1 = partial[2 * (size_t)k + 3];
        }
        a.x += x0.x; a.y += x0.y; a.z += x0.z; a.w += x0.w;
        c.x += y0.x; c.y += y0.y; c.z += y0.z; c.w += y0.w;
        if (two) {
          a.x += x1.x; a.y += x1.y; a.z += x1.z; a.w += x1.w;
          c.x += y1.x; c.y += y1.y; c.z += y1.z; c.w += y1.w;
        }
      }
      if (k1 > k0) {
        const float dr[8] = {a.x, a.y, a.z, a.w, c.x, c.y, c.z, c.w};
        GaussT<float> G;
        gauss_setup(gr, rp.beta, G);
        const PlaneT<float> P = staged ? plane_from_lds(s_plane + gp.y * kPlaneFloats) : plane_as<float>(pc[gp.y]);
        ConicT<float> k;
        conic_cull(G, P, chi2, k);
        conic_full(G, P, k);
        float dmu[3] = {0, 0, 0}, dL[6] = {0, 0, 0, 0, 0, 0}, da = 0.f, dc = 0.f;
        footprint_adjoint(G, P, k, dr, dmu, dL, da, dc);
        v[0] = dmu[0]; v[1] = dmu[1]; v[2] = dmu[2];
        for (int j = 0; j < 6; ++j) v[3 + j] = dL[j];
        v[9] = da;
        v[10] = dc;
      }
    }
    // segmented inclusive scan over equal Gaussian ids (ids are sorted)
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t gu = __shfl_up(gid, o, 64);
      const bool add = lane >= o && gu == gid;
#pragma unroll
      for (int j = 0; j < kGradFields; ++j) {
        const float y = __shfl_up(v[j], o, 64);
        if (add) v[j] += y;
      }
    }
    const uint32_t gnext = __shfl_down(gid, 1, 64);
    const uint32_t g0 = __shfl(gid, 0, 64);
    const bool seg_end = act && (lane == 63 || gnext != gid);
    if (seg_end) {
      const uint64_t o = off_rec[gid];
      const uint64_t e = o + cnt_rec[gid];
      if (o >= (uint64_t)w * 64u && e <= (uint64_t)w * 64u + 64u)
        write_gauss_grad(g, (int)gid, v, d_means, d_lraw, d_int, d_op, accumulate);
      float* sd = side + (size_t)w * 2 * kGradFields;
      if (gid == g0) {
#pragma unroll
        for (int j = 0; j < kGradFields; ++j) sd[j] = v[j];
      }
      if (lane == 63 || r + 1 == nrec) {
#pragma unroll
        for (int j = 0; j < kGradFields; ++j) sd[kGradFields + j] = v[j];
      }
    }
  }
}

// One thread per Gaussian: zero gradient for a Gaussian without records,
// and the sum of the wave pieces for one whose records span waves (the
// first wave's last segment, whole middle waves, the last wave's first
// segment); the others were written by k_record_adjoint.
// With loss_out, block 0 also adds the backward prep's per-block squared
// differences (nparts floats, in order, in FP64) into the mean squared error.
__global__ __launch_bounds__(256) void k_gauss_grad(ug_gaussians g, RenderParams rp, const Ctrl* __restrict__ ctrl,
                                                    const uint32_t* __restrict__ cnt_rec,
                                                    const unsigned long long* __restrict__ off_rec,
                                                    const float* __restrict__ side, float* __restrict__ d_means,
                                                    float* __restrict__ d_lraw, float* __restrict__ d_int,
                                                    float* __restrict__ d_op, int accumulate,
                                                    const float* __restrict__ loss_part, uint32_t nparts,
                                                    double inv_m, float* __restrict__ loss_out) {
  if (loss_out && blockIdx.x == 0) {  // uniform
    __shared__ double s_l[256];
    double a = 0.0;
    for (uint32_t k = threadIdx.x; k < nparts; k += 256) a += (double)loss_part[k];
    s_l[threadIdx.x] = a;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) s_l[threadIdx.x] += s_l[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) loss_out[0] = (float)(s_l[0] * inv_m);
  }
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rp.n) return;
  const bool ok = (ctrl->flags & (kFlagRecCap | kFlagKeyCap)) == 0;
  const uint32_t nr = ok ? cnt_rec[i] : 0u;
  float acc[kGradFields];
#pragma unroll
  for (int j = 0; j < kGradFields; ++j) acc[j] = 0.f;
  if (nr > 0) {
    const uint64_t o = off_rec[i];
    const uint64_t wa = o / 64u, wb = (o + nr - 1u) / 64u;
    if (wa == wb) return;  // finished by k_record_adjoint
    const float* sa = side + (size_t)wa * 2 * kGradFields + kGradFields;
#pragma unroll
    for (int j = 0; j < kGradFields; ++j) acc[j] = sa[j];
    for (uint64_t w = wa + 1; w <= wb; ++w) {
      const float* sw = side + (size_t)w * 2 * kGradFields;
#pragma unroll
      for (int j = 0; j < kGradFields; ++j) acc[j] += sw[j];
    }
  }
  write_gauss_grad(g, i, acc, d_means, d_lraw, d_int, d_op, accumulate);
}

// ---------------------------------------------------------------- launchers
constexpr uint32_t kMaxScanBlocks = 2048;

// Lanes per Gaussian (log2) in the cull count: doubled while the lanes stay
// under 2^18 (a few waves per SIMD), up to one lane per plane and 64.
int cull_lpg_log2(int n, int p) {
  int l = 0;
  while (l < 6 && (1 << l) < p && ((long)n << l) < (1L << 18)) ++l;
  return l;
}

// Gaussians per cull block: whole count rounds (256 lanes), at most 2048
// blocks.
int cull_gpb(int n, int p) {
  const long unit = 256 >> cull_lpg_log2(n, p);
  const long rounds = ((long)n + unit - 1) / unit;
  const long per = (rounds + kMaxScanBlocks - 1) / kMaxScanBlocks;
  return (int)((per < 1 ? 1 : per) * unit);
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

hipError_t launch_init(const ug_planes& pl, const PlaneInt* pint, PlaneConst* pc, PlaneCull* pcf, PlaneGroups* pg,
                       bool group, Ctrl* ctrl, hipStream_t s) {
  const bool grp = group && pl.p >= 1 && pl.p <= kGroupMaxPlanes;  // one block
  const uint32_t blocks = grp ? 1u : ((uint32_t)pl.p + 255) / 256;
  hipLaunchKernelGGL(k_init, dim3(blocks < 1 ? 1 : blocks), dim3(256), 0, s, pl, pint, pc, pcf, pg, grp ? 1 : 0,
                     ctrl);
  return hipGetLastError();
}

size_t accbits_words(int n, int p) { return (size_t)n * (size_t)((p + 63) / 64); }

hipError_t launch_cull_count(const ug_gaussians& g, const PlaneCull* pcf, const PlaneGroups* pg,
                             const RenderParams& rp, uint32_t* cnt_rec, unsigned long long* accbits, uint32_t* blk_tot,
                             Ctrl* ctrl, hipStream_t s) {
  const uint32_t nb = cull_blocks(rp.n, rp.p);
  if (nb == 0) return hipGetLastError();  // no Gaussians: the zeroed totals stand
  const int gpb = cull_gpb(rp.n, rp.p);
  switch (cull_lpg_log2(rp.n, rp.p)) {
#define UG_CULL(L)                                                                                              \
  case L:                                                                                                       \
    hipLaunchKernelGGL(k_cull_count<(1 << L)>, dim3(nb), dim3(256), 0, s, g, pcf, pg, rp, gpb, cnt_rec, accbits, \
                       blk_tot, ctrl);                                                                              \
    break;
    UG_CULL(0)
    UG_CULL(1)
    UG_CULL(2)
    UG_CULL(3)
    UG_CULL(4)
    UG_CULL(5)
    UG_CULL(6)
#undef UG_CULL
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_cull_write(const RenderParams& rp, const uint32_t* cnt_rec, const unsigned long long* accbits,
                             const uint32_t* blk_tot, unsigned long long* off_rec, uint2* rec_pair, Ctrl* ctrl,
                             hipStream_t s) {
  const uint32_t nb = cull_blocks(rp.n, rp.p);
  if (nb == 0) return hipGetLastError();
  // count blocks of fewer than 256 Gaussians are written m at a time
  const int gpb = cull_gpb(rp.n, rp.p);
  const uint32_t m = gpb < 256 ? (uint32_t)(256 / gpb) : 1u;
  const uint32_t nbw = (nb + m - 1) / m;
  hipLaunchKernelGGL(k_cull_write, dim3(nbw), dim3(256), 0, s, rp, gpb * (int)m, m, nbw, cnt_rec, accbits, blk_tot,
                     off_rec, rec_pair, ctrl);
  return hipGetLastError();
}

hipError_t launch_record(const ug_gaussians& g, const PlaneConst* pc, const PlaneInt* pint, const RenderParams& rp,
                         const uint2* rec_pair, Rec* recs, uint32_t* rec_nkey, uint32_t* blk_tot,
                         Ctrl* ctrl, hipStream_t s) {
  if (rp.p <= kStagePlanes) {
    const size_t lds = (size_t)rp.p * (sizeof(PlaneConst) + sizeof(PlaneInt));
    hipLaunchKernelGGL(k_record<true>, dim3(record_blocks(rp.rec_cap)), dim3(512), lds, s, g, pc, pint, rp,
                       rec_pair, recs, rec_nkey, blk_tot, ctrl);
  } else {
    hipLaunchKernelGGL(k_record<false>, dim3(record_blocks(rp.rec_cap)), dim3(256), 0, s, g, pc, pint, rp,
                       rec_pair, recs, rec_nkey, blk_tot, ctrl);
  }
  return hipGetLastError();
}

hipError_t launch_emit(const PlaneInt* pint, const RenderParams& rp, const uint2* rec_pair, const Rec* recs,
                       const uint32_t* rec_nkey, const uint32_t* blk_tot, uint32_t* rec_koff,
                       Ctrl* ctrl, uint32_t* key_tile, uint32_t* rec_of_key, hipStream_t s) {
  hipLaunchKernelGGL(k_emit, dim3(record_blocks(rp.rec_cap)), dim3(256), 0, s, pint, rp,
                     rec_pair, recs, rec_nkey, blk_tot, rec_koff, ctrl, key_tile, rec_of_key);
  return hipGetLastError();
}

size_t adjoint_side_floats(uint32_t rec_cap) { return ((size_t)rec_cap + 63) / 64 * 2 * kGradFields; }

hipError_t launch_record_adjoint(const ug_gaussians& g, const PlaneConst* pc, const RenderParams& rp,
                                 const Ctrl* ctrl, const uint2* rec_pair, const uint32_t* rec_koff,
                                 const float* partial, const uint32_t* cnt_rec, const unsigned long long* off_rec,
                                 float* side, float* d_means, float* d_lraw, float* d_int, float* d_op,
                                 int accumulate, hipStream_t s) {
  uint32_t want = (rp.rec_cap + 255u) / 256u;
  // with staged planes every block loads them once: fewer, longer blocks
  const bool staged = rp.p <= kStagePlanes;
  const uint32_t cap = staged ? 2048u : 8192u;
  const uint32_t blocks = want < 1 ? 1 : (want > cap ? cap : want);
  const size_t lds = staged ? (size_t)rp.p * kPlaneFloats * sizeof(float) : 0;
  hipLaunchKernelGGL(k_record_adjoint, dim3(blocks), dim3(256), lds, s, g, pc, rp, ctrl, rec_pair, rec_koff,
                     reinterpret_cast<const float4*>(partial), cnt_rec, off_rec, side, d_means, d_lraw, d_int, d_op,
                     accumulate);
  return hipGetLastError();
}

hipError_t launch_gauss_grad(const ug_gaussians& g, const RenderParams& rp, const Ctrl* ctrl, const uint32_t* cnt_rec,
                             const unsigned long long* off_rec, const float* side, float* d_means, float* d_lraw,
                             float* d_int, float* d_op, int accumulate, const float* loss_part, uint32_t nparts,
                             double inv_m, float* loss_out, hipStream_t s) {
  int blocks = (rp.n + 255) / 256;
  if (loss_out && blocks < 1) blocks = 1;  // the loss is written even with no Gaussians
  if (blocks > 0)
    hipLaunchKernelGGL(k_gauss_grad, dim3(blocks), dim3(256), 0, s, g, rp, ctrl, cnt_rec, off_rec, side, d_means,
                       d_lraw, d_int, d_op, accumulate, loss_part, nparts, inv_m, loss_out);
  return hipGetLastError();
}

}  // namespace ug
