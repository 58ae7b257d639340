/*
 * ug.h - C ABI of the UltraGauss probe-plane rasterizer for AMD MI355X (gfx950).
 *
 * The operation (UltraGauss, Section 4.1-4.4):
 *   For every probe plane p and pixel x of its grid, lift x to 3D (Section 4.1),
 *   evaluate every Gaussian i by its 3D squared Mahalanobis distance d^2
 *   (Eq. 8, after the rigid world->probe transform of Eq. 9), keep the pair
 *   only if d^2 <= chi^2 (Eq. 12), weight it by alpha_i exp(-d^2/2), and
 *   normalise with a background component (Eq. 5-7):
 *       c(x) = (sum_i w_i c_i + a_BG c_BG) / (sum_i w_i + a_BG).
 *   Precisions use the lower-triangular factor of Eq. 11 (Section 4.2):
 *   Sigma^-1 = L L^T, L = [[l11^2+b, 0, 0], [l21, l22^2+b, 0], [l31, l32, l33^2+b]]
 *   (the entry printed at (3,2) is read as an independent l32).
 *   Gaussians are culled per plane and binned to tiles with the bounding box
 *   of Eq. 13 (Section 4.3-4.4; the matrix there is read as the precision).
 *
 * Conventions for every entry point:
 *   - All array arguments are DEVICE pointers to float32, C-contiguous, owned
 *     by the caller, unless marked "host".  Nothing is freed or retained.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is enqueued asynchronously; render and backward never synchronise
 *     and never allocate, so they can be captured in a hipGraph.
 *   - Arguments are validated on the host before anything is enqueued; an
 *     invalid call returns a negative UG_ERR_* code and enqueues nothing.
 *   - Conditions only the device can see (capacity overflow, non-finite
 *     inputs) are recorded in the workspace and read with ug_plan_status.
 *     On a capacity overflow the render draws background only and the
 *     backward writes zero gradients; re-plan with larger capacities.
 *   - Thread safety: a plan may be used from one host thread at a time;
 *     concurrent calls that share a workspace race.
 */
#ifndef UG_H
#define UG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define UG_OK 0
#define UG_ERR_INVALID_ARG (-1) /* bad pointer, size or parameter            */
#define UG_ERR_CAPACITY (-2)    /* records or keys exceeded the plan's capacity */
#define UG_ERR_NONFINITE (-3)   /* a Gaussian or plane held NaN/Inf (it was skipped) */
#define UG_ERR_HIP (-4)         /* a HIP runtime call failed                 */
#define UG_ERR_NO_DEVICE (-5)   /* no usable gfx950 device                   */
#define UG_ERR_INTERNAL (-6)    /* a device-side consistency check failed    */
#define UG_ERR_SCRATCH_SIZE (-7) /* the plan needs more workspace than ug_render_planes_noalloc holds */

/* ---- binning boxes (all give identical images) ------------------------ */
#define UG_BOX_PAPER 0 /* Eq. 13 box of the chi^2 ellipsoid, in-plane part b_{1:2} */
#define UG_BOX_CONIC 1 /* bounding box of the ellipse cut by the plane (tighter)  */
#define UG_BOX_ROWS 2  /* exact extent of that ellipse per row of tiles (tightest) */

/* ---- params.flags bits ------------------------------------------------ */
#define UG_FLAG_COUNT_EVALS 1 /* forward also counts in-support (Gaussian, pixel) pairs */
#define UG_FLAG_SCATTER 2     /* forward by the paper's Phase 2 (Sec. 4.4): every record
                                 adds to per-pixel sums with atomic adds over its box,
                                 instead of the tile-binned gather; same per-pair test,
                                 so the same image to float rounding (the order of the
                                 atomic additions is not fixed).  Forward only: the
                                 backward of such a plan returns UG_ERR_INVALID_ARG, and
                                 no keys are emitted (key_capacity may be 0)          */
#define UG_FLAG_BOX_SUPPORT 4 /* with UG_FLAG_SCATTER only: the paper-literal support of
                                 Phase 2 (Sec. 4.4).  A (Gaussian, plane) pair is kept
                                 iff the plane meets the Eq. 13 box (decided in FP64,
                                 with no slack), and then every pixel whose centre lies
                                 in the in-plane part of that box, edges included, takes
                                 the Eq. 8 weight: there is no per-pair Eq. 12 test, so
                                 box corners outside the chi^2 ellipse count and the
                                 image differs from the ellipsoid support.  box_mode is
                                 ignored.  Without UG_FLAG_SCATTER: UG_ERR_INVALID_ARG */
#define UG_FLAG_SPLIT_FORWARD 8 /* launch shape of the gather forward: two waves per 8-row
                                 band of a tile, each summing alternate rounds of lds_batch
                                 records, their sums added at the end (first + second).
                                 More waves for launches with few tiles; each pixel's sum
                                 is then grouped differently, so the image may differ from
                                 the one-wave form in the last bits (still deterministic).
                                 Not with tile_h = 32 and lds_batch = 256 (the staging
                                 would exceed 128 KB of LDS): UG_ERR_INVALID_ARG */
#define UG_FLAG_CULL_EACH_PLANE 16 /* Phase-1 cull (Sec. 4.4) by testing every (Gaussian,
                                 plane) pair.  Without it, launches of up to 256 planes
                                 group the planes that differ only in the origin's third
                                 coordinate (a stack of parallel slices) and test, per
                                 Gaussian, only the planes of a group inside a window
                                 that bounds the test's acceptance; the same test then
                                 decides each of them, so the records are the same
                                 either way.  A test and measurement switch            */

/* ---- pipeline stages (measurement hooks) ------------------------------- */
#define UG_STAGE_SETUP 0         /* plane pose set-up                                  */
#define UG_STAGE_CULL_COUNT 1    /* Phase-1 cull (Sec. 4.4): acceptance bits, counts    */
#define UG_STAGE_CULL_WRITE 2    /* record offsets and the compact pair list            */
#define UG_STAGE_RECORD 3        /* in-plane conic, footprint, per-record key counts    */
#define UG_STAGE_EMIT 4          /* key offsets and key emission                        */
#define UG_STAGE_SORT_HIST 5     /* radix sort: digit histograms (once per pass)        */
#define UG_STAGE_SORT_SCAN 6     /* radix sort: histogram column scan (once per pass)   */
#define UG_STAGE_SORT_SCATTER 7  /* radix sort: stable scatter (once per pass)          */
#define UG_STAGE_RANGES 8        /* per-tile key ranges (a one-pass sort writes them)   */
#define UG_STAGE_ACCUM 9         /* per-tile accumulation, Eq. 5-8 and 12               */
#define UG_STAGE_BWD_PREP 10     /* per-pixel adjoint inputs                            */
#define UG_STAGE_ACCUM_BWD 11    /* per-key adjoint of the accumulation                 */
#define UG_STAGE_RECORD_ADJ 12   /* per-record adjoint of the conic construction        */
#define UG_STAGE_GAUSS_GRAD 13   /* per-Gaussian sum of its records' adjoints           */
#define UG_STAGE_SCATTER 14      /* UG_FLAG_SCATTER forward: zero, scatter, normalise   */
#define UG_NUM_STAGES 15

typedef struct ug_plan ug_plan; /* opaque, host-side */

/* Gaussians, Section 4.2 and 4.5.  Device pointers. */
typedef struct {
  const float *means;     /* [n][3] world-space centres mu_i                  */
  const float *lraw;      /* [n][6] raw (l11, l21, l31, l22, l32, l33), Eq. 11 */
  const float *intensity; /* [n]    grey level c_i                            */
  const float *opacity;   /* [n]    logit a_i; alpha_i = 1/(1+exp(-a_i))      */
  int32_t n;
} ug_gaussians;

/* Probe planes, Section 4.1 / Eq. 9.  Device pointers.
 * rot is row-major 3x3 with columns (e1, e2, n): the probe->world rotation
 * (the inverse of W's rotation part), right-handed.  Pixel (u, v) of a W x H
 * plane lies at world point origin + x1 e1 + x2 e2 with
 * x1 = (u + 1/2 - W/2) sx, x2 = (v + 1/2 - H/2) sy. */
typedef struct {
  const float *rot;     /* [p][9] */
  const float *origin;  /* [p][3] world position of the image centre */
  const float *spacing; /* [p][2] (sx, sy) world units per pixel     */
  int32_t p;
} ug_planes;

typedef struct {
  float beta;      /* Eq. 11 diagonal shift, > 0 (default 1e-4)                  */
  float chi2;      /* Eq. 12 bound on d^2, > 0, may be +inf (default 7.815)      */
  float bg_alpha;  /* Eq. 5 background coefficient, > 0 (default 1e-2)           */
  float bg_color;  /* Eq. 6 background colour (default 0)                         */
  int32_t tile_w;  /* tile width in pixels (default 16); (tile_w, tile_h) is one
                      of 8x8, 16x8, 8x16, 16x16, 32x8, 32x16, 16x32, 32x32      */
  int32_t tile_h;  /* tile height in pixels (default 16)                          */
  int32_t px_per_lane; /* forward pixels per lane: tile_w / 8 (or 0 = that)        */
  int32_t lds_batch; /* records each forward wave stages in LDS per round: 32, 64,
                        128 or 256 (default 64)                                   */
  int32_t box_mode;  /* UG_BOX_* (default UG_BOX_PAPER)                           */
  int32_t flags;     /* UG_FLAG_* bits (default 0)                                */
} ug_params;

/* Fills *out with the defaults listed above. */
void ug_params_default(ug_params *out);

/* Creates a plan for n Gaussians and p planes whose sizes are
 * wh_host[p][2] = (W, H) (host memory, copied).  record_capacity bounds the
 * accepted (Gaussian, plane) pairs, key_capacity the (pair, tile) keys of one
 * render; ug_plan_measure returns the exact numbers for given inputs.
 * Allocates the plan's small device tables on the current device.
 * Errors: UG_ERR_INVALID_ARG (n < 0, p < 1, W or H outside [1, 32767],
 * more than 2^(32 - Q) tiles in the launch, Q = (tile_w / 8) (tile_h / 8)
 * (a key word carries the tile id and the tile's Q-bit sub-block mask),
 * bad params, capacities < 0 or >= 2^31, null out), UG_ERR_HIP. */
int ug_plan_create(int32_t n, int32_t p, const int32_t *wh_host, const ug_params *params,
                   int64_t record_capacity, int64_t key_capacity, ug_plan **out);

/* Changes the capacities (the workspace size changes with them). */
int ug_plan_reserve(ug_plan *plan, int64_t record_capacity, int64_t key_capacity);

/* Bytes of device workspace a render/backward pair needs (256-byte aligned
 * base required). */
size_t ug_plan_workspace_bytes(const ug_plan *plan);

/* Total pixels of the plan (sum of W*H): the length of image buffers. */
int64_t ug_plan_num_pixels(const ug_plan *plan);

/* Number of tiles of the plan's tile grid over all planes. */
int64_t ug_plan_num_tiles(const ug_plan *plan);

/* Runs the culling and record passes (no key emission) and returns,
 * synchronously, out_host[0] = the accepted (Gaussian, plane) records and
 * out_host[1] = the (record, tile) keys that ug_render_planes would produce
 * for these inputs; out_host[1] is -1 when the records exceed the plan's
 * record capacity (reserve, then measure again).  The workspace must hold
 * ug_plan_workspace_bytes(plan) bytes. */
int ug_plan_measure(const ug_plan *plan, const ug_gaussians *g, const ug_planes *planes,
                    void *workspace, int64_t *out_host, void *stream);

/* Forward render (Section 4.1-4.4).  image: [num_pixels] float32, packed
 * plane after plane, row-major (index v*W + u).  Fills the workspace with the
 * state the backward needs (records, sorted keys, per-pixel denominators).
 * With UG_FLAG_SCATTER the accumulation is the atomic scatter of Phase 2. */
int ug_render_planes(const ug_plan *plan, const ug_gaussians *g, const ug_planes *planes,
                     float *image, void *workspace, void *stream);

/* Forward render that allocates nothing, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same operation, arguments, image layout
 * and launches as ug_render_planes, with the workspace taken from a static
 * device array of UG_NOALLOC_WORKSPACE_BYTES (64 MiB) that the library holds
 * on every device it runs on until the process ends; its address is looked up
 * once per device when a plan is created there (or at this call's first use
 * on the device).  Nothing is allocated or freed and no library routine that
 * allocates is called.  The render leaves nothing in the workspace that a
 * later call reads, so nothing has to start at zero.
 * Limits and caveats:
 *   - the plan's ug_plan_workspace_bytes must be at most
 *     UG_NOALLOC_WORKSPACE_BYTES, else UG_ERR_SCRATCH_SIZE (nothing enqueued);
 *   - every call on one device shares that device's array, which keeps the
 *     last call's contents: calls that overlap on one device (other streams,
 *     other host threads, other plans) race and give wrong images;
 *   - the workspace is not the caller's, so the render's device-side status
 *     (capacity overflow, non-finite inputs) cannot be read with
 *     ug_plan_status and there is no backward for this forward: on a
 *     capacity overflow the image is background only, as with
 *     ug_render_planes; size the plan with ug_plan_measure beforehand;
 *   - the current device must be the one the plan was created on
 *     (UG_ERR_INVALID_ARG otherwise).
 * Other errors as ug_render_planes. */
#define UG_NOALLOC_WORKSPACE_BYTES (64u << 20)
int ug_render_planes_noalloc(const ug_plan *plan, const ug_gaussians *g, const ug_planes *planes,
                             float *image, void *stream);

/* Adjoint of ug_render_planes for an upstream gradient d_image (same layout
 * as image).  image and workspace must be those the matching forward wrote,
 * unchanged.  Gradients are with respect to the raw parameters:
 * d_means [n][3], d_lraw [n][6], d_intensity [n], d_opacity [n] (logits).
 * accumulate = 0 overwrites them, 1 adds to them.  The cut-off set of Eq. 12
 * is held fixed (the map is piecewise smooth).  Deterministic: no atomics. */
/* Plans with UG_FLAG_SCATTER have no backward (UG_ERR_INVALID_ARG). */
int ug_render_planes_backward(const ug_plan *plan, const ug_gaussians *g,
                              const ug_planes *planes, const float *image,
                              const float *d_image, void *workspace, float *d_means,
                              float *d_lraw, float *d_intensity, float *d_opacity,
                              int32_t accumulate, void *stream);

/* The same adjoint for the training loss of Sec. 4.5, the mean squared
 * error against target ([num_pixels] float32, the image's layout), fused:
 * dL/dc_hat = 2 (image - target) / num_pixels is formed inside the first
 * adjoint kernel with the float operations ug_mse_grad uses, so the
 * gradients equal ug_mse_grad followed by ug_render_planes_backward bit for
 * bit, with one launch and one pixel array less.  loss_dev (device float32,
 * may be NULL) receives the mean squared error, written by the last adjoint
 * kernel from per-block sums added in a fixed order (FP64).  Other
 * arguments, errors and determinism as ug_render_planes_backward. */
int ug_render_planes_backward_mse(const ug_plan *plan, const ug_gaussians *g,
                                  const ug_planes *planes, const float *image,
                                  const float *target, void *workspace, float *d_means,
                                  float *d_lraw, float *d_intensity, float *d_opacity,
                                  int32_t accumulate, float *loss_dev, void *stream);

/* Reads the device-side status the last render left in the workspace
 * (synchronises the stream): UG_OK, UG_ERR_CAPACITY, UG_ERR_NONFINITE or
 * UG_ERR_INTERNAL.  counts_host (may be NULL) receives [records, keys,
 * in-support pairs, evaluated pairs] of that render; the last two are 0
 * unless the plan was created with UG_FLAG_COUNT_EVALS. */
int ug_plan_status(const ug_plan *plan, const void *workspace, int64_t *counts_host,
                   void *stream);

/* Measurement hooks (not for use under graph capture).  ug_profile_begin
 * makes the plan record a pair of HIP events on the launch stream around
 * each kernel launch of the stages whose bit is set in stage_mask
 * (bit UG_STAGE_*), for at most max_launches launches; the events are
 * created here.  ug_profile_read synchronises on the last event, writes the
 * summed milliseconds and launch counts per stage (arrays of UG_NUM_STAGES,
 * either may be NULL), and turns recording off. */
int ug_profile_begin(ug_plan *plan, uint32_t stage_mask, int32_t max_launches);
int ug_profile_read(ug_plan *plan, float *ms_host, int32_t *launches_host);

/* Mean squared error over m pixels: loss_dev[0] = mean((image - target)^2)
 * and d_image = 2 (image - target) / m (the training loss; the paper trains
 * the Gaussians by gradient descent on rendered slices, Section 4.5).
 * loss_dev must hold UG_MSE_SCRATCH_FLOATS floats: [0] receives the loss,
 * the rest is scratch for the deterministic one-launch reduction and must
 * be zero-filled before the first call (every call leaves it usable: its
 * completion counter returns to zero).  Calls sharing one loss_dev must
 * not overlap. */
#define UG_MSE_SCRATCH_FLOATS 1026
int ug_mse_grad(const float *image, const float *target, int64_t m, float *d_image,
                float *loss_dev, void *stream);

/* One Adam step over `count` parameters (Section 4.5 trains with Adam):
 *   mo = b1 mo + (1-b1) g;  ve = b2 ve + (1-b2) g^2;
 *   p -= lr * (mo / (1 - b1^t)) / (sqrt(ve / (1 - b2^t)) + eps).
 * step_t >= 1 is the 1-based step number. */
int ug_adam_step(float *param, const float *grad, float *mo, float *ve, int64_t count,
                 float lr, float beta1, float beta2, float eps, int32_t step_t, void *stream);

/* Mutable Gaussian tensors (device, float32), same layout as ug_gaussians. */
typedef struct {
  float *means;     /* [n][3] */
  float *lraw;      /* [n][6] */
  float *intensity; /* [n]    */
  float *opacity;   /* [n]    */
  int32_t n;
} ug_gaussians_mut;

/* Adam hyper-parameters for the Gaussian tensors (Section 4.5: Adam, learning
 * rate 0.05 for every parameter except the means, which start at 1.6e-4 with
 * an exponential decay; the final value is not given in the paper). */
typedef struct {
  float lr_means;       /* learning rate of the means at step 1             */
  float lr_means_final; /* reached after decay_steps steps, then held        */
  int32_t decay_steps;  /* >= 1                                             */
  float lr;             /* learning rate of lraw, intensity and opacity      */
  float beta1, beta2, eps;
} ug_adam_params;

/* One Adam step over all four Gaussian tensors in one launch:
 *   m1 = b1 m1 + (1-b1) g;  m2 = b2 m2 + (1-b2) g^2;
 *   p -= lr_t * (m1 / (1 - b1^t)) / (sqrt(m2 / (1 - b2^t)) + eps),
 * with t = 1 + *step_dev read from DEVICE memory and incremented on the
 * device after the update, so a captured hipGraph advances the schedule on
 * every replay.  lr_t for the means decays exponentially from lr_means to
 * lr_means_final over decay_steps.  If plan and workspace are given and the
 * render that filled the workspace overflowed its capacity, the update and
 * the step increment are skipped on the device (the gradients were not
 * computed).  Moments must start at zero and *step_dev at 0. */
int ug_adam_gaussians(const ug_plan *plan, const void *workspace, const ug_gaussians_mut *params,
                      const ug_gaussians_mut *grads, const ug_gaussians_mut *m1,
                      const ug_gaussians_mut *m2, const ug_adam_params *hp, int32_t *step_dev,
                      void *stream);

/* ---- the training step as one HIP graph -------------------------------- */

/* Captures one training step of Sec. 4.5 into a HIP graph held by the plan:
 * ug_render_planes into image, ug_render_planes_backward_mse against target
 * into grads (overwritten) and *loss_dev (may be NULL), optionally
 * ug_accumulate_grad_norm into grad_acc / grad_cnt (both NULL or both
 * given), and ug_adam_gaussians on params with m1, m2, adam and step_dev.
 * Nothing runs at capture: the library captures on a stream of its own
 * (default priority) and instantiates the graph; every pointer passed is
 * baked into it, so the buffers must stay allocated and in place, and new
 * contents (poses, targets) may be copied into them between replays.  The
 * graph holds no memset or copy nodes (only kernels) and nothing in it
 * allocates or synchronises.  A new capture replaces the previous one;
 * ug_plan_reserve and ug_plan_destroy drop it.  Errors: UG_ERR_INVALID_ARG
 * for NULL or inconsistent arguments, a plan with UG_FLAG_SCATTER (no
 * backward) or stage profiling active (its events would be captured);
 * UG_ERR_HIP if capture or instantiation fails. */
int ug_step_capture(ug_plan *plan, const ug_gaussians_mut *params, const ug_planes *planes,
                    const float *target, float *image, void *workspace, const ug_gaussians_mut *grads,
                    const ug_gaussians_mut *m1, const ug_gaussians_mut *m2, const ug_adam_params *adam,
                    int32_t *step_dev, float *loss_dev, float *grad_acc, int32_t *grad_cnt);

/* Launches the captured step on stream (asynchronous; the device-side step
 * counter advances the learning-rate schedule on every replay).
 * UG_ERR_INVALID_ARG if nothing is captured. */
int ug_step_replay(ug_plan *plan, void *stream);

/* ---- test hook: the records of the last render -------------------------- */

/* One accepted (Gaussian, plane) pair as the accumulate kernels see it: in
 * pixel units, with du = u - ub - fu and dv = v - vb - fv,
 *   t1 = t11 du + t12 dv,  t2 = t22 dv,  e = e0 - t1^2 - t2^2,
 * and the pair adds weight 2^e (intensity c) to pixel (u, v) iff e >= emin
 * (Eq. 8 restricted to the plane, base 2: e0 = log2 alpha - r^2 log2(e) / 2,
 * emin = log2 alpha - chi^2 log2(e) / 2).  [tx0, tx1] x [ty0, ty1] is its
 * tile rectangle (pixel rectangle under UG_FLAG_BOX_SUPPORT). */
typedef struct {
  int32_t gaussian, plane;
  float t11, t12, t22, fu, fv, e0, emin, c;
  int32_t ub, vb;
  uint16_t tx0, tx1, ty0, ty1;
} ug_record;

/* Copies up to cap records of the last render (Gaussian-major, planes
 * ascending) to host_out and returns their number (which may exceed cap),
 * or a negative status.  Synchronises the stream.  For tests; not for use
 * under graph capture. */
int64_t ug_debug_records(const ug_plan *plan, const void *workspace, ug_record *host_out, int64_t cap,
                         void *stream);

/* ---- test hook: the tile binning of the last render ---------------------- */

/* Copies the keys of the last gather render as the radix sort left them
 * (Section 4.4 binning: one key per (record, touched tile), sorted by tile
 * id, stably, so a tile's keys keep the order in which they were emitted)
 * and the tile ranges derived from them:
 *   key_out[j]   key word: the tile id in its low 32 - Q bits, the tile's
 *                8 x 8 sub-block coverage mask in its top Q bits
 *                (Q = (tile_w / 8) (tile_h / 8); bit b = sub-block
 *                (b % (tile_w / 8), b / (tile_w / 8)));
 *   eidx_out[j]  position of key j in the emitted (unsorted) order;
 *   rec_out[j]   record index (as ug_debug_records numbers them);
 *   ranges_out   num_tiles + 1 entries: tile t's keys are [ranges_out[t],
 *                ranges_out[t + 1]).
 * Any of the four host pointers may be null (not copied); at most cap keys
 * are copied.  Returns the number of keys (which may exceed cap), or a
 * negative status (UG_ERR_INVALID_ARG for a scatter plan, which has no
 * keys).  Synchronises the stream.  For tests; not for use under graph
 * capture. */
int64_t ug_debug_keys(const ug_plan *plan, const void *workspace, uint32_t *key_out, uint32_t *eidx_out,
                      uint32_t *rec_out, uint32_t *ranges_out, int64_t cap, void *stream);

/* ---- Densification and pruning between training steps.  Section 4.2
 * draws new means from a Gaussian through its triangular factor,
 * y = mu + L^-T z (back substitution with L^T, no general inverse); the
 * clone / split / prune rule is only referenced by the paper (to 3D
 * Gaussian splatting), so the one below is a stated choice.  Random numbers
 * are inputs (z), so results are reproducible. */

/* out[j] = means[idx[j]] + L^-T z[j], j < k, with L from lraw[idx[j]] by
 * Eq. 11 (shift beta).  idx [k] int32, z [k][3] (standard normals for a
 * draw from the Gaussian), out [k][3]: device, float32.  An idx entry
 * outside [0, g->n) yields NaN for that sample.  No synchronisation. */
int ug_sample_gaussians(const ug_gaussians *g, float beta, const int32_t *idx, const float *z, int64_t k,
                        float *out, void *stream);

/* acc[i] += |d_means[i]| (Euclidean norm) and cnt[i] += 1 for i < n: the
 * per-Gaussian statistic ug_densify reads (device arrays; start at zero).
 * If plan and workspace are given and the render that filled the workspace
 * overflowed its capacity, the update is skipped on the device (as in
 * ug_adam_gaussians: the gradients were not computed). */
int ug_accumulate_grad_norm(const ug_plan *plan, const void *workspace, const float *d_means, int32_t n,
                            float *acc, int32_t *cnt, void *stream);

typedef struct {
  float beta;         /* Eq. 11 shift, as in the render (default 1e-4)                  */
  float min_opacity;  /* prune when sigmoid(a) < this (default 0.005)                   */
  float grad_thresh;  /* clone or split when acc >= grad_thresh * cnt, cnt > 0
                         (default 2e-4, in loss units per world unit)                  */
  float split_size;   /* split (else clone) when size > this, world units (default 1)  */
  float max_size;     /* prune when size > this; 0 = no limit (default 0)              */
  float split_factor; /* a split child has every std divided by this, > 1 (default 1.6) */
} ug_densify_params;

/* Fills *out with the defaults listed above. */
void ug_densify_params_default(ug_densify_params *out);

/* Bytes of device workspace ug_densify needs for n Gaussians. */
size_t ug_densify_workspace_bytes(int32_t n);

/* The rule, per Gaussian i, decided in float32 with the operations in a fixed
 * order (size^2 = trace of the covariance = sum of squares of the entries of
 * L^-1, written out; the opacity floor compared in logit space):
 *   prune if sigmoid(a) < min_opacity, or max_size > 0 and size > max_size;
 *   else if cnt[i] > 0 and acc[i] >= grad_thresh * cnt[i]:
 *     split if size > split_size: two children, means mu + L^-T z[i][c]
 *       (c = 0, 1) and factor split_factor * L (every std divided by
 *       split_factor), intensity and opacity copied;
 *     else clone: two copies;
 *   else keep one copy.
 * out (device, capacity out_capacity Gaussians; its n is ignored) receives
 * the outputs in Gaussian order (i ascending, a Gaussian's outputs
 * together): deterministic.  z [n][2][3] standard normals, read for split
 * Gaussians only.  The number of outputs goes to *count_dev (device int64);
 * when it exceeds out_capacity nothing past the capacity is written.
 * workspace: ug_densify_workspace_bytes(n) bytes of device memory, 256-byte
 * aligned, caller-owned.  Arrays must not overlap g's.  No synchronisation. */
int ug_densify(const ug_gaussians *g, const float *acc, const int32_t *cnt, const float *z,
               const ug_densify_params *dp, const ug_gaussians_mut *out, int64_t out_capacity,
               int64_t *count_dev, void *workspace, void *stream);

/* ---- scoring reconstructions ------------------------------------------ */

/* Bytes of device workspace ug_image_quality needs for this plan's planes. */
size_t ug_quality_workspace_bytes(const ug_plan *plan);

/* Image-quality scores of packed planes against references, for the SSIM
 * and PSNR evaluation of Section 5.2.  image, ref: device float32 [M_px],
 * packed like ug_render_planes images (the plan's planes and sizes).  Per
 * plane p: ssim[p] = the mean SSIM (Wang et al. 2004: 11 x 11 Gaussian
 * window, standard deviation 1.5, weights summing to one, weighted
 * population moments, C1 = (0.01 L)^2, C2 = (0.03 L)^2, L = data_range)
 * over the window positions that lie wholly inside the image (NaN for a
 * plane under 11 pixels in either direction); mse[p] = the mean squared
 * difference over all its pixels, so PSNR = 10 log10(L^2 / mse[p]).
 * ssim, mse: device float64 [P].  Moments are summed in FP64 and every sum
 * is taken in a fixed order, so the scores are deterministic.  workspace:
 * ug_quality_workspace_bytes(plan) bytes of device memory, 256-byte aligned,
 * caller-owned (independent of the render workspace).  Errors:
 * UG_ERR_INVALID_ARG for a NULL pointer, misaligned workspace or a
 * data_range that is not positive and finite.  No synchronisation. */
int ug_image_quality(const ug_plan *plan, const float *image, const float *ref, float data_range,
                     double *ssim, double *mse, void *workspace, void *stream);

/* ---- covariance parameterisation study -------------------------------- */

#define UG_PARAM_TRI 0  /* Eq. 11: (l11, l21, l31, l22, l32, l33), Sigma^-1 = L L^T,
                           diagonal l^2 + beta                                    */
#define UG_PARAM_SYM 1  /* Eq. 10: (M11, M12, M13, M22, M23, M33), M symmetric,
                           Sigma^-1 = M M^T + beta I                               */
#define UG_PARAM_QUAT 2 /* (qw, qx, qy, qz, s1, s2, s3): Sigma = R diag(s^2) R^T,
                           R of the normalised quaternion                          */

/* Sec. 4.2's comparison of covariance parameterisations: per Gaussian, one
 * route's covariance, a draw and a distance, in float32 (fp64 = 0) or
 * float64 (fp64 = 1; the reference for the float32 rounding, which for SYM
 * inverts the precision through its Cholesky factor instead of the
 * adjugate, whose error grows with the squared condition number).
 *   raw   [n][8] float32, the kind's layout (unused entries ignored);
 *   z     [n][3] float32 standard normals; delta [n][3] float32 offsets;
 *   sigma [n][6] out: Sigma (11, 12, 13, 22, 23, 33) -- from L^-1 written out
 *         (TRI), the adjugate inverse of the precision (SYM), the product
 *         (QUAT);
 *   draw  [n][3] out: F z with F F^T = Sigma -- back substitution with L^T
 *         (TRI), the lower Cholesky factor of that Sigma (SYM; NaN when a
 *         pivot is not positive), R diag(s) (QUAT);
 *   d2    [n] out: delta^T Sigma^-1 delta.
 * Outputs are float32 or float64 as fp64 says; all pointers are device
 * memory owned by the caller.  Errors: UG_ERR_INVALID_ARG for an unknown
 * kind, n < 0 or a NULL pointer with n > 0.  No synchronisation. */
int ug_param_eval(int32_t kind, int32_t fp64, const float *raw, const float *z, const float *delta, int64_t n,
                  float beta, void *sigma, void *draw, void *d2, void *stream);

/* ---- Throughput probes (measurement only) --------------------------------
 * The rates behind the roofline fractions the benchmark reports, measured
 * on the device the library runs on:
 *   UG_PROBE_FMA    8 independent FMA chains per thread, iters steps each
 *                   (2 flop per FMA: 16 x iters x 256 x blocks flop);
 *   UG_PROBE_EXP    8 chains of v_exp_f32 per thread (8 x iters x 256 x
 *                   blocks transcendentals);
 *   UG_PROBE_PAIRS  the forward accumulate's evaluation of one (record,
 *                   pixel) pair (two FMAs, the cut-off compare, exp2, two
 *                   sums) on registers only, 8 pairs per thread and step;
 *   UG_PROBE_COPY   dst = src over n floats (n a multiple of 4, both 16-byte
 *                   aligned), a grid-stride loop of blocks x 256 threads.
 * For the first three, dst receives one float per thread (n >= blocks x
 * 256) and src is unused.  Device pointers, caller-owned.  Times the launch
 * with two events on stream, synchronises, and stores its milliseconds in
 * *ms_host.  UG_ERR_INVALID_ARG for an unknown kind, blocks outside
 * [1, 2^20], iters < 1 or a buffer too small or misaligned. */
#define UG_PROBE_FMA 0
#define UG_PROBE_EXP 1
#define UG_PROBE_PAIRS 2
#define UG_PROBE_COPY 3
int ug_probe(int32_t kind, int32_t blocks, int32_t iters, const float *src, float *dst, int64_t n, float *ms_host,
             void *stream);

/* Human-readable text for a status code (static storage). */
const char *ug_status_string(int status);

/* Frees the plan and its device tables.  NULL is ignored. */
void ug_plan_destroy(ug_plan *plan);

#ifdef __cplusplus
}
#endif

#endif /* UG_H */
