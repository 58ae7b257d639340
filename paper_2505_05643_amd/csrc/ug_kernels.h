// Host-side launchers of the HIP kernels (one translation unit per stage).
#pragma once

#include "ug_internal.h"

namespace ug {

// ---- preprocess (ug_preprocess.hip)
hipError_t launch_init(const ug_planes& pl, const PlaneInt* pint, PlaneConst* pc, Ctrl* ctrl, hipStream_t s);
hipError_t launch_count(const ug_gaussians& g, const PlaneConst* pc, const PlaneInt* pint, const RenderParams& rp,
                        uint32_t* cnt_rec, uint32_t* cnt_key, uint32_t* blk_rec, uint32_t* blk_key, Ctrl* ctrl,
                        hipStream_t s);
hipError_t launch_top_scan(const uint32_t* blk_rec, const uint32_t* blk_key, unsigned long long* blk_rec_off,
                           unsigned long long* blk_key_off, int nblk, Ctrl* ctrl, uint32_t rec_cap,
                           uint32_t key_cap, uint32_t* rec_koff, hipStream_t s);
hipError_t launch_write(const ug_gaussians& g, const PlaneConst* pc, const PlaneInt* pint, const RenderParams& rp,
                        const uint32_t* cnt_rec, const uint32_t* cnt_key, const unsigned long long* blk_rec_off,
                        const unsigned long long* blk_key_off, uint32_t* off_rec, RecAcc* racc, RecGeo* rgeo,
                        uint32_t* rec_pid, uint32_t* rec_koff, hipStream_t s);
hipError_t launch_emit(const Ctrl* ctrl, const RecAcc* racc, const RecGeo* rgeo, const uint32_t* rec_pid,
                       const uint32_t* rec_koff, const PlaneInt* pint, const RenderParams& rp, uint32_t* key_tile,
                       uint32_t* rec_of_key, hipStream_t s);
hipError_t launch_reduce_partials(const Ctrl* ctrl, const uint32_t* rec_koff, const float* partial, float* drec,
                                  uint32_t rec_cap, hipStream_t s);
hipError_t launch_preprocess_bwd(const ug_gaussians& g, const PlaneConst* pc, const RenderParams& rp,
                                 const Ctrl* ctrl, const uint32_t* cnt_rec, const uint32_t* off_rec,
                                 const uint32_t* rec_pid, const float* drec, float* d_means, float* d_lraw,
                                 float* d_int, float* d_op, int accumulate, hipStream_t s);

// ---- tile binning sort (ug_sort.hip)
// Stable LSD radix sort of (tile id, emission index) pairs on `bits` key
// bits, 8 bits per pass.  keys/vals are ping-pong buffers; on return
// *final_buf (0 or 1) names the buffer holding the sorted pairs, and srec
// holds rec_of_key[] gathered in sorted order.
hipError_t launch_sort(const Ctrl* ctrl, uint32_t* keys0, uint32_t* keys1, uint32_t* vals0, uint32_t* vals1,
                       const uint32_t* rec_of_key, uint32_t* srec, uint32_t* hist, uint32_t nblocks, int bits,
                       int* final_buf, hipStream_t s);
hipError_t launch_tile_ranges(const Ctrl* ctrl, const uint32_t* skeys, uint32_t num_tiles, uint32_t* tile_start,
                              hipStream_t s);
uint32_t sort_blocks_for(uint32_t key_cap);

// ---- accumulate (ug_raster.hip)
int accum_default_ppl(int tile_w, int tile_h);
bool accum_config_supported(int tile_w, int tile_h, int ppl, int lds_batch);
hipError_t launch_accum_fwd(int tile_w, int tile_h, int ppl, int lds_batch, const PlaneInt* pint, const uint32_t* tile_plane,
                            const uint32_t* tile_start, const uint32_t* srec, const RecAcc* racc,
                            const RecGeo* rgeo, float* image, float* dsave, float bg_alpha, float bg_color,
                            uint32_t num_tiles, unsigned long long* n_eval, hipStream_t s);
hipError_t launch_bwd_prep(int tile_w, int tile_h, const PlaneInt* pint, const uint32_t* tile_plane,
                           const float* image, const float* d_image, const float* dsave, float* gq,
                           uint32_t num_tiles, hipStream_t s);
hipError_t launch_accum_bwd(int tile_w, int tile_h, const Ctrl* ctrl, const PlaneInt* pint,
                            const uint32_t* tile_plane, const uint32_t* skey, const uint32_t* sval,
                            const uint32_t* srec, const RecAcc* racc, const RecGeo* rgeo, const float* gq,
                            float* partial, uint32_t key_cap, hipStream_t s);

// ---- training helpers (ug_train.hip)
hipError_t launch_mse(const float* image, const float* target, int64_t m, float* d_image, float* loss,
                      hipStream_t s);
hipError_t launch_adam(float* param, const float* grad, float* mo, float* ve, int64_t count, float lr, float b1,
                       float b2, float eps, int32_t t, hipStream_t s);

}  // namespace ug
