// Internal definitions shared by the HIP translation units of libug.
// Everything here is device-side layout and small helpers; the C ABI is
// include/ug.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ug.h"

namespace ug {

constexpr double kLog2e = 1.4426950408889634074;
constexpr double kLn2 = 0.69314718055994530942;
// d^2 enters the weight as exp(-d^2/2) = 2^(-kHalfLog2e * d^2).
constexpr double kHalfLog2e = 0.5 * kLog2e;

// ---------------------------------------------------------------- control block
// Written by the culling pass; read by every later kernel of the same render.
struct Ctrl {
  unsigned long long n_rec;   // accepted (Gaussian, plane) records
  unsigned long long n_key;   // (record, tile) keys
  unsigned long long n_eval;  // in-support pairs (counted only on request)
  unsigned long long n_exec;  // evaluated pairs, n_eval's companion
  unsigned int flags;         // kFlag* bits
  unsigned int n_rec_eff;     // records the later kernels process (0 on overflow)
  unsigned int n_key_eff;     // keys the later kernels process (0 on overflow)
  unsigned int pad[5];
};
static_assert(sizeof(Ctrl) == 64, "Ctrl layout");

constexpr unsigned kFlagRecCap = 1u;
constexpr unsigned kFlagKeyCap = 2u;
constexpr unsigned kFlagNonfinite = 4u;
constexpr unsigned kFlagInternal = 8u;  // an internal consistency check failed

// ---------------------------------------------------------------- planes
// Integer layout of one plane inside the launch (host-computed at plan time).
struct PlaneInt {
  int32_t W, H;        // pixels
  int32_t ntx, nty;    // tiles
  uint32_t tile_off;   // first global tile id of the plane
  uint32_t pix_off_lo; // first pixel index of the plane (low/high words)
  uint32_t pix_off_hi;
  uint32_t pad;
};
static_assert(sizeof(PlaneInt) == 32, "PlaneInt layout");

// FP64 constants of one plane pose (computed on device from the float32 pose).
// R = [e1 e2 n] maps probe -> world; m = R^-1 (mu - o) are probe coordinates.
struct PlaneConst {
  double o[3];
  double rinv[9];   // R^-1, row-major
  double e1[3];     // first two columns of R
  double e2[3];
  double absdet;    // |det R|
  double sx, sy;    // pixel spacing
  double cu, cv;    // W/2 - 1/2, H/2 - 1/2: pixel index of the in-plane origin
  int32_t valid;
  int32_t pad;
};

// Float copy of what the Phase-1 pre-test needs: origin and the third row
// of R^-1 (probe-frame normal coordinate m3 = r3 . (mu - o)).
struct PlaneCull {
  float o[3];
  float r3[3];
  int32_t valid;
  int32_t pad;
};
static_assert(sizeof(PlaneCull) == 32, "PlaneCull layout");

// Planes grouped for the Phase-1 cull: a group holds the valid planes whose
// cull constants agree bit for bit except the origin's third coordinate
// (r3, o[0], o[1]), sorted by that coordinate; written by the plane set-up
// for launches of up to kGroupMaxPlanes planes (use = 0 otherwise, or when
// no group is large enough to be worth a search).
constexpr int kGroupMaxPlanes = 256;
struct PlaneGroups {
  uint32_t use;
  uint32_t pad[3];
  uint32_t perm[kGroupMaxPlanes];  // plane at each sorted position
  float oz[kGroupMaxPlanes];       // its origin's third coordinate
  uint32_t end[kGroupMaxPlanes];   // one past the last position of its group
};

// ---------------------------------------------------------------- records
// One accepted (Gaussian, plane) pair as the accumulate kernels use it.
// In pixel-index units, with du = u - (ub + fu), dv = v - (vb + fv):
//   t1 = t11 du + t12 dv,  t2 = t22 dv,  e = e0 - t1^2 - t2^2,
//   weight = 2^e if e >= emin else 0.
// (t11, t12, t22) is the upper-triangular factor of the in-plane precision
// scaled by sqrt(log2(e)/2); e0 = log2(alpha) - log2(e)/2 * r^2 with r^2 the
// squared distance of the plane from the Gaussian; emin = log2(alpha) -
// log2(e)/2 * chi^2, so e >= emin is exactly d^2 <= chi^2 (Eq. 12).
// Per-Gaussian gradient fields: dmu (3), dL (6), d opacity logit, d intensity.
constexpr int kGradFields = 11;

// Side of the square pixel sub-blocks that tiles are split into (tile widths
// and heights are multiples of it).
constexpr int kSubBlock = 8;

// A key word holds the tile id in its low bits and the tile's sub-block
// coverage mask (Q = (TW / 8) (TH / 8) bits) in its top Q bits, so the sort
// moves the mask with the key; tile ids must stay below 2^(32 - Q).
__host__ __device__ constexpr int key_mask_shift(int tile_w, int tile_h) {
  return 32 - (tile_w / kSubBlock) * (tile_h / kSubBlock);
}

struct RecAcc {
  float t11, t12, t22, fu;
  float fv, e0, emin, c;
};
static_assert(sizeof(RecAcc) == 32, "RecAcc layout");

// Integer part of the record: conic centre base pixel and the tile rectangle.
struct RecGeo {
  int32_t ub, vb;
  uint16_t tx0, tx1, ty0, ty1;
};
static_assert(sizeof(RecGeo) == 16, "RecGeo layout");

// A record as stored: both parts in one 64-byte slot, so the accumulate
// kernels' gathers (one record per key, in tile order: random in record
// order) fetch one 64-byte segment per key instead of two.  The slot's last
// 16 bytes carry, for ROWS-mode binning, the tile span of each of the
// record's first kRowSpans tile rows as counted by the record kernel
// (tx0 | tx1 << 16; kNoSpan for a row the ellipse misses), so the emission
// reuses them instead of recomputing them; unused in the other modes.
constexpr int kRowSpans = 4;
constexpr uint32_t kNoSpan = 1u;  // tx0 = 1 > tx1 = 0
struct Rec {
  RecAcc acc;
  RecGeo geo;
  uint32_t spans[kRowSpans];
};
static_assert(sizeof(Rec) == 64, "Rec layout");

// Per-key partial derivatives written by the adjoint accumulate
// (dt11, dt12, dt22, dfu, dfv, de0, dc, unused).
struct Partial {
  float v[8];
};

// ---------------------------------------------------------------- launch params
struct RenderParams {
  float beta, chi2, bg_alpha, bg_color;
  int32_t tile_w, tile_h, box_mode;
  int32_t box_support;  // paper-literal Phase-2 support (records carry pixel boxes)
  int32_t n, p;
  uint32_t num_tiles;
  uint32_t rec_cap, key_cap;
};

// ---------------------------------------------------------------- helpers
__device__ __forceinline__ uint32_t lanemask_lt_popc(unsigned long long m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Blocks are dispatched round-robin over the 8 XCDs (block b -> XCD b % 8).
// Give each XCD a contiguous range of work items so neighbouring tiles share
// that XCD's L2.  Bijective on [0, nblocks).
__device__ __forceinline__ uint32_t xcd_remap(uint32_t b, uint32_t nblocks) {
  const uint32_t x = b & 7u, q = nblocks >> 3, r = nblocks & 7u;
  const uint32_t start = x * q + (x < r ? x : r);
  return start + (b >> 3);
}

__device__ __forceinline__ bool isfinite_d(double v) { return __builtin_isfinite(v); }

// Orders LDS writes and reads between the lanes of one wave (LDS operations
// of a wave execute in order; this keeps the compiler from moving them).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace ug
