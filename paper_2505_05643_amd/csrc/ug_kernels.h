// Host-side launchers of the HIP kernels (one translation unit per stage).
#pragma once

#include "ug_internal.h"

namespace ug {

// ---- preprocess (ug_preprocess.hip)
uint32_t cull_blocks(int n, int p);
uint32_t record_blocks(uint32_t rec_cap);
hipError_t launch_init(const ug_planes& pl, const PlaneInt* pint, PlaneConst* pc, PlaneCull* pcf, PlaneGroups* pg,
                       bool group, Ctrl* ctrl, hipStream_t s);
// Phase-1 cull: per-(Gaussian, plane) acceptance bits and per-Gaussian record
// counts, then record offsets and the compact (Gaussian, plane) pair list.
size_t accbits_words(int n, int p);
hipError_t launch_cull_count(const ug_gaussians& g, const PlaneCull* pcf, const PlaneGroups* pg,
                             const RenderParams& rp, uint32_t* cnt_rec, unsigned long long* accbits, uint32_t* blk_tot,
                             Ctrl* ctrl, hipStream_t s);
hipError_t launch_cull_write(const RenderParams& rp, const uint32_t* cnt_rec, const unsigned long long* accbits,
                             const uint32_t* blk_tot, unsigned long long* off_rec, uint2* rec_pair, Ctrl* ctrl,
                             hipStream_t s);
// Records (conic + footprint and per-record key counts), then key offsets and
// key emission: per key its key word (tile id and sub-block mask) and record
// id.
hipError_t launch_record(const ug_gaussians& g, const PlaneConst* pc, const PlaneInt* pint, const RenderParams& rp,
                         const uint2* rec_pair, Rec* recs, uint32_t* rec_nkey, uint32_t* blk_tot,
                         Ctrl* ctrl, hipStream_t s);
hipError_t launch_emit(const PlaneInt* pint, const RenderParams& rp, const uint2* rec_pair, const Rec* recs,
                       const uint32_t* rec_nkey, const uint32_t* blk_tot, uint32_t* rec_koff,
                       Ctrl* ctrl, uint32_t* key_tile, uint32_t* rec_of_key, hipStream_t s);
// Backward of the record construction and the per-Gaussian sums: the record
// adjoint finishes every Gaussian whose records sit in one wave of 64 and
// leaves per-wave segment sums in side (adjoint_side_floats floats); the
// Gaussian pass finishes the rest and zeroes Gaussians without records.
size_t adjoint_side_floats(uint32_t rec_cap);
hipError_t launch_record_adjoint(const ug_gaussians& g, const PlaneConst* pc, const RenderParams& rp,
                                 const Ctrl* ctrl, const uint2* rec_pair, const uint32_t* rec_koff,
                                 const float* partial, const uint32_t* cnt_rec, const unsigned long long* off_rec,
                                 float* side, float* d_means, float* d_lraw, float* d_int, float* d_op,
                                 int accumulate, hipStream_t s);
// loss_out (may be null): the mean squared error, inv_m times the sum of the
// nparts per-block sums in loss_part.
hipError_t launch_gauss_grad(const ug_gaussians& g, const RenderParams& rp, const Ctrl* ctrl, const uint32_t* cnt_rec,
                             const unsigned long long* off_rec, const float* side, float* d_means, float* d_lraw,
                             float* d_int, float* d_op, int accumulate, const float* loss_part, uint32_t nparts,
                             double inv_m, float* loss_out, hipStream_t s);

// ---- tile binning sort (ug_sort.hip)
// Stable LSD radix sort of the key words on their low `bits` bits (the tile
// id), moving two payload words per key: emission index (generated in the
// first pass) and record id.  Digits: the whole tile id in one pass when it
// has at most 10 bits and there are at most 256 sort blocks, else at most 8
// bits per pass with the bits split evenly (sort_digit_bits, sort_passes).
// Arrays are given as {key, val, rec}; passes alternate between two such
// sets.  Per pass: block-major digit histograms (hist holds
// sort_digit_slots * (nblocks + 1) words), their column scan, then the
// stable scatter.
int sort_digit_bits(int bits, uint32_t nblocks);
int sort_passes(int bits, uint32_t nblocks);
uint32_t sort_digit_slots(int bits, uint32_t nblocks);
hipError_t launch_radix_hist(const Ctrl* ctrl, const uint32_t* keys, uint32_t* hist, uint32_t nblocks, int bits,
                             int pass, hipStream_t s);
hipError_t launch_radix_colscan(uint32_t* hist, uint32_t nblocks, int bits, hipStream_t s);
// With a single pass (the digit is the whole tile id) the scatter also
// writes tile_start (if not null; num_tiles + 1 entries), which the column
// totals give directly.
hipError_t launch_radix_scatter(const Ctrl* ctrl, const uint32_t* const in[3], uint32_t* const out[3],
                                const uint32_t* hist, uint32_t nblocks, int bits, int pass, uint32_t* tile_start,
                                uint32_t num_tiles, hipStream_t s);
// tile_start[t] for t in [0, T] from the sorted key words (tile id = the key
// word's bits below mask_shift).
hipError_t launch_tile_ranges(const Ctrl* ctrl, const uint32_t* skeys, uint32_t num_tiles, uint32_t key_cap,
                              int mask_shift, uint32_t* tile_start, hipStream_t s);
uint32_t sort_blocks_for(uint32_t key_cap);

// ---- Phase-2 atomic scatter forward (ug_scatter.hip): zero the sums, one
// wave per record adds w c and w over its box, normalise in place.
hipError_t launch_scatter_zero(float* num, float* den, uint64_t m, hipStream_t s);
hipError_t launch_scatter(const Ctrl* ctrl, const uint2* rec_pair, const PlaneInt* pint, const Rec* recs,
                          int tile_w, int tile_h, uint32_t rec_cap, float* num, float* den,
                          hipStream_t s);
hipError_t launch_scatter_norm(float* image, float* dsave, uint64_t m, float bg_alpha, float bg_color,
                               hipStream_t s);

// ---- densification (ug_densify.hip)
uint32_t densify_blocks(int32_t n);
hipError_t launch_densify(const ug_gaussians& g, const float* acc, const int32_t* cnt, const float* z,
                          const ug_densify_params& dp, const ug_gaussians_mut& out, int64_t cap, int64_t* count,
                          uint32_t* blk, hipStream_t s);
hipError_t launch_sample(const ug_gaussians& g, float beta, const int32_t* idx, const float* z, int64_t k, float* out,
                         hipStream_t s);
hipError_t launch_grad_norm(const Ctrl* ctrl, const float* d_means, int32_t n, float* acc, int32_t* cnt,
                            hipStream_t s);

// ---- image-quality scores (ug_quality.hip)
struct QualityConst {
  double taps[11];  // normalised 1D Gaussian window
  double c1, c2;
};
uint32_t quality_strips(int32_t max_width);  // 8-pixel column strips of the widest plane
// part: p x max_strips double2 of workspace
hipError_t launch_quality(const PlaneInt* pint, int32_t p, uint32_t max_strips, const float* img, const float* ref,
                          const QualityConst& q, double2* part, double* ssim, double* mse, hipStream_t s);

// ---- covariance parameterisation study (ug_params.hip)
hipError_t launch_param_eval(int32_t kind, bool fp64, const float* raw, const float* z, const float* delta,
                             int64_t n, float beta, void* sigma, void* draw, void* d2, hipStream_t s);

// ---- throughput probes (ug_probe.hip)
hipError_t launch_probe(int kind, int blocks, int iters, const float* src, float* dst, int64_t n, hipStream_t s);

// ---- accumulate (ug_raster.hip)
int accum_default_ppl(int tile_w, int tile_h);
bool accum_config_supported(int tile_w, int tile_h, int ppl, int lds_batch);
// split = 2: two waves per 8-row band, taking alternate rounds of records.
// cut: the launch has a finite chi^2 cut-off (Eq. 12); the same flag goes to
// the adjoint.
hipError_t launch_accum_fwd(int tile_w, int tile_h, int lds_batch, int split, const PlaneInt* pint,
                            const uint32_t* tile_plane, const uint32_t* tile_start, const uint32_t* skey,
                            const uint32_t* srec, const Rec* recs, float* image, float* dsave,
                            float bg_alpha, float bg_color, bool cut, uint32_t num_tiles,
                            unsigned long long* n_eval, hipStream_t s);
// second = dL/dc_hat, or (mse) the target with dL/dc_hat = scale (image -
// target) formed inside and per-block squared-difference sums in loss_part
// (bwd_prep_blocks floats).
uint32_t bwd_prep_blocks(int tile_w, int tile_h, uint32_t num_tiles);
hipError_t launch_bwd_prep(int tile_w, int tile_h, const PlaneInt* pint, const uint32_t* tile_plane,
                           const float* image, const float* second, bool mse, float scale, float* loss_part,
                           const float* dsave, float* gq, uint32_t num_tiles, hipStream_t s);
// tile_org[t] = pixel origin of tile t, x0 | y0 << 16.
hipError_t launch_accum_bwd(int tile_w, int tile_h, const Ctrl* ctrl, const uint32_t* tile_org,
                            const uint32_t* skey, const uint32_t* sval,
                            const uint32_t* srec, const Rec* recs,
                            const float* gq, float* partial, bool cut, uint32_t key_cap, hipStream_t s);

// ---- training helpers (ug_train.hip)
hipError_t launch_mse(const float* image, const float* target, int64_t m, float* d_image, float* loss,
                      hipStream_t s);
hipError_t launch_adam(float* param, const float* grad, float* mo, float* ve, int64_t count, float lr, float b1,
                       float b2, float eps, int32_t t, hipStream_t s);
hipError_t launch_adam_gaussians(float* const p[4], const float* const g[4], float* const m[4], float* const v[4],
                                 int64_t n, const ug_adam_params& hp, int32_t* step_dev, const Ctrl* ctrl,
                                 hipStream_t s);

}  // namespace ug
