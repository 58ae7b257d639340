// Host side of the C ABI (include/ug.h): plans, workspace layout, argument
// validation and the enqueue order of the render and backward passes.
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <utility>
#include <vector>

#include "ug_kernels.h"

using namespace ug;

// Workspace of ug_render_planes_noalloc: one array per device, allocated by
// the loader with the code object and held until the process ends.  Host code
// uses only the address hipGetSymbolAddress returns for the current device
// (the array's name on the host is a stand-in, not a device address).
static __device__ __align__(256) unsigned char scratch[UG_NOALLOC_WORKSPACE_BYTES];

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
  size_t ctrl, pconst, pcull, pgroups, cnt_rec, accbits, off_rec, blk_g, blk_r;
  size_t rec_pair, recs, rec_nkey, rec_koff, side;
  size_t tile_start, dsave, gq, hist;
  size_t key_tile0, key_tile1, key_val0, key_val1, rec_of_key, srec, partial;
  size_t loss_part;
  size_t total;
};

}  // namespace

struct ug_plan {
  int32_t n = 0, p = 0;
  ug_params prm{};
  int ppl = 1;
  uint32_t num_tiles = 0;
  uint64_t num_pixels = 0;
  int bits = 1;
  int final_buf = 0;
  uint32_t rec_cap = 0, key_cap = 0;
  uint32_t sort_blocks = 1;
  int device = 0;
  PlaneInt* d_pint = nullptr;
  uint32_t* d_tile_plane = nullptr;
  uint32_t* d_tile_org = nullptr;  // pixel origin of each tile, x0 | y0 << 16 (W, H < 2^15)
  Layout lay{};
  // Measurement hooks: event pairs around the launches of selected stages.
  struct Prof {
    bool on = false;
    uint32_t mask = 0;
    int cap = 0, used = 0;
    std::vector<hipEvent_t> ev;  // 2 * cap
    std::vector<int> stage;      // cap
  };
  mutable Prof prof;
  hipGraphExec_t step_exec = nullptr;  // the captured training step, if any
  int32_t max_w = 0;                   // widest plane (pixels)
};

namespace {

// Workspace regions for the current capacities; also the sort's set that
// holds the result (the passes alternate between two sets).
void compute_layout(ug_plan* pl) {
  pl->final_buf = sort_passes(pl->bits, pl->sort_blocks) % 2;
  Layout& L = pl->lay;
  size_t o = 0;
  auto take = [&o](size_t bytes) {
    const size_t at = o;
    o = align_up(o + (bytes ? bytes : 1));
    return at;
  };
  const size_t n = (size_t)pl->n, P = (size_t)pl->p;
  const size_t T = pl->num_tiles, R = pl->rec_cap, K = pl->key_cap;
  const size_t tpx = (size_t)pl->prm.tile_w * pl->prm.tile_h;
  L.ctrl = take(sizeof(Ctrl));
  L.pconst = take(P * sizeof(PlaneConst));
  L.pcull = take(P * sizeof(PlaneCull));
  L.pgroups = take(sizeof(PlaneGroups));
  L.cnt_rec = take(n * 4);
  L.accbits = take(accbits_words(pl->n, pl->p) * 8);
  L.off_rec = take(n * 8);
  L.blk_g = take((size_t)cull_blocks(pl->n, pl->p) * 4);
  L.blk_r = take((size_t)record_blocks(pl->rec_cap) * 4);
  L.rec_pair = take(R * 8);
  L.recs = take(R * sizeof(Rec));
  L.rec_nkey = take(R * 4);
  L.rec_koff = take((R + 1) * 4);
  L.side = take(adjoint_side_floats(pl->rec_cap) * 4);
  L.tile_start = take((T + 1) * 4);
  L.dsave = take(pl->num_pixels * 4);
  L.gq = take(T * tpx * 8);
  L.hist = take((size_t)sort_digit_slots(pl->bits, pl->sort_blocks) * (pl->sort_blocks + 1) * 4);
  L.key_tile0 = take(K * 4);
  L.key_tile1 = take(K * 4);
  L.key_val0 = take(K * 4);
  L.key_val1 = take(K * 4);
  L.rec_of_key = take(K * 4);
  L.srec = take(K * 4);
  L.partial = take(K * 32);
  L.loss_part = take((size_t)bwd_prep_blocks(pl->prm.tile_w, pl->prm.tile_h, pl->num_tiles) * 4);
  L.total = o;
}

template <typename T>
inline T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

bool valid_params(const ug_params& p) {
  if (!(p.beta > 0.f) || !std::isfinite(p.beta)) return false;
  if (!(p.chi2 > 0.f)) return false;  // +inf allowed, NaN rejected
  if (!(p.bg_alpha > 0.f) || !std::isfinite(p.bg_alpha)) return false;
  if (!std::isfinite(p.bg_color)) return false;
  if (p.box_mode != UG_BOX_PAPER && p.box_mode != UG_BOX_CONIC && p.box_mode != UG_BOX_ROWS) return false;
  if ((p.flags & ~(UG_FLAG_COUNT_EVALS | UG_FLAG_SCATTER | UG_FLAG_BOX_SUPPORT | UG_FLAG_SPLIT_FORWARD |
                   UG_FLAG_CULL_EACH_PLANE)) != 0)
    return false;
  if ((p.flags & UG_FLAG_BOX_SUPPORT) && !(p.flags & UG_FLAG_SCATTER)) return false;
  const int ppl = p.px_per_lane ? p.px_per_lane : accum_default_ppl(p.tile_w, p.tile_h);
  // the split forward doubles the staging LDS: (TH / 8) bands x 2 waves x
  // max(batch, 64) records x 80 B, kept within 128 KB
  if ((p.flags & UG_FLAG_SPLIT_FORWARD) &&
      (size_t)(p.tile_h / 8) * 2 * (size_t)(p.lds_batch > 64 ? p.lds_batch : 64) * 80 > (size_t)128 * 1024)
    return false;
  return accum_config_supported(p.tile_w, p.tile_h, ppl, p.lds_batch);
}

int hip_status(hipError_t e) { return e == hipSuccess ? UG_OK : UG_ERR_HIP; }

// Records a begin/end event pair around one launch when the stage is profiled.
class StageScope {
 public:
  StageScope(const ug_plan* pl, int stage, hipStream_t s) : pl_(pl), s_(s) {
    ug_plan::Prof& P = pl->prof;
    if (P.on && ((P.mask >> stage) & 1u) && P.used < P.cap) {
      slot_ = P.used++;
      P.stage[(size_t)slot_] = stage;
      (void)hipEventRecord(P.ev[2 * (size_t)slot_], s_);
    }
  }
  ~StageScope() {
    if (slot_ >= 0) (void)hipEventRecord(pl_->prof.ev[2 * (size_t)slot_ + 1], s_);
  }
  StageScope(const StageScope&) = delete;
  StageScope& operator=(const StageScope&) = delete;

 private:
  const ug_plan* pl_;
  hipStream_t s_;
  int slot_ = -1;
};

void prof_release(ug_plan* pl) {
  for (hipEvent_t e : pl->prof.ev) (void)hipEventDestroy(e);
  pl->prof.ev.clear();
  pl->prof.stage.clear();
  pl->prof.cap = pl->prof.used = 0;
  pl->prof.on = false;
}

RenderParams make_rp(const ug_plan* pl) {
  RenderParams rp;
  rp.beta = pl->prm.beta;
  rp.chi2 = pl->prm.chi2;
  rp.bg_alpha = pl->prm.bg_alpha;
  rp.bg_color = pl->prm.bg_color;
  rp.tile_w = pl->prm.tile_w;
  rp.tile_h = pl->prm.tile_h;
  rp.box_mode = pl->prm.box_mode;
  rp.box_support = (pl->prm.flags & UG_FLAG_BOX_SUPPORT) ? 1 : 0;
  rp.n = pl->n;
  rp.p = pl->p;
  rp.num_tiles = pl->num_tiles;
  rp.rec_cap = pl->rec_cap;
  rp.key_cap = pl->key_cap;
  return rp;
}

int check_inputs(const ug_plan* plan, const ug_gaussians* g, const ug_planes* pl, const void* ws) {
  if (!plan || !g || !pl || !ws) return UG_ERR_INVALID_ARG;
  if (reinterpret_cast<uintptr_t>(ws) % kAlign) return UG_ERR_INVALID_ARG;
  if (g->n != plan->n || pl->p != plan->p) return UG_ERR_INVALID_ARG;
  if (g->n > 0 && (!g->means || !g->lraw || !g->intensity || !g->opacity)) return UG_ERR_INVALID_ARG;
  if (!pl->rot || !pl->origin || !pl->spacing) return UG_ERR_INVALID_ARG;
  return UG_OK;
}

// Culling and record passes shared by measure and render.
hipError_t enqueue_preprocess(const ug_plan* plan, const ug_gaussians& g, const ug_planes& pl, void* ws,
                              const RenderParams& rp, hipStream_t s, bool emit = true) {
  const Layout& L = plan->lay;
  Ctrl* ctrl = at<Ctrl>(ws, L.ctrl);
  hipError_t e;
  {
    StageScope sc(plan, UG_STAGE_SETUP, s);
    e = launch_init(pl, plan->d_pint, at<PlaneConst>(ws, L.pconst), at<PlaneCull>(ws, L.pcull),
                    at<PlaneGroups>(ws, L.pgroups), (plan->prm.flags & UG_FLAG_CULL_EACH_PLANE) == 0, ctrl, s);
  }
  if (e != hipSuccess) return e;
  {
    StageScope sc(plan, UG_STAGE_CULL_COUNT, s);
    e = launch_cull_count(g, at<PlaneCull>(ws, L.pcull), at<PlaneGroups>(ws, L.pgroups), rp, at<uint32_t>(ws, L.cnt_rec),
                          at<unsigned long long>(ws, L.accbits), at<uint32_t>(ws, L.blk_g), ctrl, s);
  }
  if (e != hipSuccess) return e;
  {
    StageScope sc(plan, UG_STAGE_CULL_WRITE, s);
    e = launch_cull_write(rp, at<uint32_t>(ws, L.cnt_rec), at<unsigned long long>(ws, L.accbits),
                          at<uint32_t>(ws, L.blk_g), at<unsigned long long>(ws, L.off_rec), at<uint2>(ws, L.rec_pair),
                          ctrl, s);
  }
  if (e != hipSuccess) return e;
  {
    StageScope sc(plan, UG_STAGE_RECORD, s);
    e = launch_record(g, at<PlaneConst>(ws, L.pconst), plan->d_pint, rp, at<uint2>(ws, L.rec_pair),
                      at<Rec>(ws, L.recs), at<uint32_t>(ws, L.rec_nkey),
                      at<uint32_t>(ws, L.blk_r), ctrl, s);
  }
  if (e != hipSuccess || !emit) return e;
  StageScope sc(plan, UG_STAGE_EMIT, s);
  return launch_emit(plan->d_pint, rp, at<uint2>(ws, L.rec_pair), at<Rec>(ws, L.recs),
                     at<uint32_t>(ws, L.rec_nkey), at<uint32_t>(ws, L.blk_r), at<uint32_t>(ws, L.rec_koff), ctrl,
                     at<uint32_t>(ws, L.key_tile0), at<uint32_t>(ws, L.rec_of_key), s);
}

// The radix sort of the emitted keys, one launch per kernel and pass.  Set 0
// = (key_tile0, key_val0, rec_of_key) holds the emitted keys; passes
// alternate between set 0 and set 1 = (key_tile1, key_val1, srec).
hipError_t enqueue_sort(const ug_plan* plan, void* ws, hipStream_t s) {
  const Layout& L = plan->lay;
  const Ctrl* ctrl = at<Ctrl>(ws, L.ctrl);
  uint32_t* set[2][3] = {{at<uint32_t>(ws, L.key_tile0), at<uint32_t>(ws, L.key_val0), at<uint32_t>(ws, L.rec_of_key)},
                         {at<uint32_t>(ws, L.key_tile1), at<uint32_t>(ws, L.key_val1), at<uint32_t>(ws, L.srec)}};
  uint32_t* hist = at<uint32_t>(ws, L.hist);
  const uint32_t G = plan->sort_blocks;
  const int passes = sort_passes(plan->bits, G);
  hipError_t e = hipSuccess;
  for (int pass = 0, cur = 0; pass < passes && e == hipSuccess; ++pass, cur ^= 1) {
    {
      StageScope sc(plan, UG_STAGE_SORT_HIST, s);
      e = launch_radix_hist(ctrl, set[cur][0], hist, G, plan->bits, pass, s);
    }
    if (e != hipSuccess) break;
    {
      StageScope sc(plan, UG_STAGE_SORT_SCAN, s);
      e = launch_radix_colscan(hist, G, plan->bits, s);
    }
    if (e != hipSuccess) break;
    StageScope sc(plan, UG_STAGE_SORT_SCATTER, s);
    const uint32_t* in[3] = {set[cur][0], set[cur][1], set[cur][2]};
    e = launch_radix_scatter(ctrl, in, set[cur ^ 1], hist, G, plan->bits, pass,
                             passes == 1 ? at<uint32_t>(ws, L.tile_start) : nullptr, plan->num_tiles, s);
  }
  return e;
}

// Sorted arrays {key word, emission index, record id} left by the sort.
struct Sorted {
  const uint32_t *key, *val, *rec;
};
Sorted sorted_set(const ug_plan* plan, void* ws) {
  const Layout& L = plan->lay;
  if (plan->final_buf) return {at<uint32_t>(ws, L.key_tile1), at<uint32_t>(ws, L.key_val1), at<uint32_t>(ws, L.srec)};
  return {at<uint32_t>(ws, L.key_tile0), at<uint32_t>(ws, L.key_val0), at<uint32_t>(ws, L.rec_of_key)};
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Looks up (once per device, with that device current) the device address of
// the static workspace; nullptr if the runtime call fails.
void* scratch_for_current_device() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

int render_impl(const ug_plan* plan, const ug_gaussians* g, const ug_planes* planes, float* image, void* workspace,
                void* stream);

}  // namespace

extern "C" {

void ug_params_default(ug_params* out) {
  if (!out) return;
  out->beta = 1e-4f;
  out->chi2 = 7.815f;
  out->bg_alpha = 1e-2f;
  out->bg_color = 0.f;
  out->tile_w = 16;
  out->tile_h = 16;
  out->px_per_lane = 0;
  out->lds_batch = 64;
  out->box_mode = UG_BOX_PAPER;
  out->flags = 0;
}

int ug_plan_create(int32_t n, int32_t p, const int32_t* wh_host, const ug_params* params, int64_t record_capacity,
                   int64_t key_capacity, ug_plan** out) {
  if (!out) return UG_ERR_INVALID_ARG;
  *out = nullptr;
  if (n < 0 || p < 1 || !wh_host || !params) return UG_ERR_INVALID_ARG;
  if (record_capacity < 0 || key_capacity < 0 || record_capacity >= (int64_t(1) << 31) ||
      key_capacity >= (int64_t(1) << 31))
    return UG_ERR_INVALID_ARG;
  if (!valid_params(*params)) return UG_ERR_INVALID_ARG;
  const int TW = params->tile_w, TH = params->tile_h;
  std::vector<PlaneInt> pint((size_t)p);
  uint64_t tiles = 0, pix = 0;
  int32_t max_w = 0;
  for (int32_t i = 0; i < p; ++i) {
    const int32_t W = wh_host[2 * i], H = wh_host[2 * i + 1];
    if (W < 1 || H < 1 || W > 32767 || H > 32767) return UG_ERR_INVALID_ARG;
    PlaneInt& q = pint[(size_t)i];
    max_w = W > max_w ? W : max_w;
    q.W = W;
    q.H = H;
    q.ntx = (W + TW - 1) / TW;
    q.nty = (H + TH - 1) / TH;
    q.tile_off = (uint32_t)tiles;
    q.pix_off_lo = (uint32_t)(pix & 0xffffffffu);
    q.pix_off_hi = (uint32_t)(pix >> 32);
    q.pad = 0;
    tiles += (uint64_t)q.ntx * q.nty;
    pix += (uint64_t)W * H;
    // tile ids share the key word with the tile's sub-block mask
    if (tiles > (uint64_t(1) << key_mask_shift(TW, TH))) return UG_ERR_INVALID_ARG;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return UG_ERR_NO_DEVICE;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return UG_ERR_NO_DEVICE;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return UG_ERR_NO_DEVICE;
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return UG_ERR_NO_DEVICE;

  ug_plan* pl = new (std::nothrow) ug_plan();
  if (!pl) return UG_ERR_HIP;
  pl->n = n;
  pl->p = p;
  pl->max_w = max_w;
  pl->prm = *params;
  pl->ppl = params->px_per_lane ? params->px_per_lane : accum_default_ppl(TW, TH);
  pl->num_tiles = (uint32_t)tiles;
  pl->num_pixels = pix;
  int bits = 1;
  while (bits < 32 && (uint64_t(1) << bits) < tiles) ++bits;
  pl->bits = bits;
  pl->device = dev;
  pl->rec_cap = (uint32_t)record_capacity;
  pl->key_cap = (uint32_t)key_capacity;
  pl->sort_blocks = sort_blocks_for(pl->key_cap);
  std::vector<uint32_t> tile_plane((size_t)tiles), tile_org((size_t)tiles);
  for (int32_t i = 0; i < p; ++i) {
    const PlaneInt& q = pint[(size_t)i];
    const uint32_t nt = (uint32_t)(q.ntx * q.nty);
    for (uint32_t t = 0; t < nt; ++t) {
      tile_plane[q.tile_off + t] = (uint32_t)i;
      tile_org[q.tile_off + t] = (t % (uint32_t)q.ntx) * (uint32_t)TW | ((t / (uint32_t)q.ntx) * (uint32_t)TH) << 16;
    }
  }
  if (hipMalloc(&pl->d_pint, sizeof(PlaneInt) * (size_t)p) != hipSuccess ||
      hipMalloc(&pl->d_tile_plane, sizeof(uint32_t) * (size_t)tiles) != hipSuccess ||
      hipMalloc(&pl->d_tile_org, sizeof(uint32_t) * (size_t)tiles) != hipSuccess ||
      hipMemcpy(pl->d_pint, pint.data(), sizeof(PlaneInt) * (size_t)p, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(pl->d_tile_plane, tile_plane.data(), sizeof(uint32_t) * (size_t)tiles, hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(pl->d_tile_org, tile_org.data(), sizeof(uint32_t) * (size_t)tiles, hipMemcpyHostToDevice) !=
          hipSuccess) {
    ug_plan_destroy(pl);
    return UG_ERR_HIP;
  }
  compute_layout(pl);
  // set-up of the no-allocation forward's workspace on this device; a failure
  // here is reported by that entry point, which tries again
  (void)scratch_for_current_device();
  *out = pl;
  return UG_OK;
}

int ug_plan_reserve(ug_plan* plan, int64_t record_capacity, int64_t key_capacity) {
  if (!plan || record_capacity < 0 || key_capacity < 0 || record_capacity >= (int64_t(1) << 31) ||
      key_capacity >= (int64_t(1) << 31))
    return UG_ERR_INVALID_ARG;
  plan->rec_cap = (uint32_t)record_capacity;
  plan->key_cap = (uint32_t)key_capacity;
  plan->sort_blocks = sort_blocks_for(plan->key_cap);
  compute_layout(plan);
  if (plan->step_exec) {  // its kernels were captured with the old layout
    (void)hipGraphExecDestroy(plan->step_exec);
    plan->step_exec = nullptr;
  }
  return UG_OK;
}

size_t ug_plan_workspace_bytes(const ug_plan* plan) { return plan ? plan->lay.total : 0; }

int64_t ug_plan_num_pixels(const ug_plan* plan) { return plan ? (int64_t)plan->num_pixels : -1; }

int64_t ug_plan_num_tiles(const ug_plan* plan) { return plan ? (int64_t)plan->num_tiles : -1; }

int ug_plan_measure(const ug_plan* plan, const ug_gaussians* g, const ug_planes* planes, void* workspace,
                    int64_t* out_host, void* stream) {
  const int st = check_inputs(plan, g, planes, workspace);
  if (st != UG_OK) return st;
  if (!out_host) return UG_ERR_INVALID_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  RenderParams rp = make_rp(plan);
  rp.key_cap = 0;  // count keys, emit none
  hipError_t e = enqueue_preprocess(plan, *g, *planes, workspace, rp, s);
  if (e != hipSuccess) return UG_ERR_HIP;
  Ctrl c;
  if (hipMemcpyAsync(&c, at<Ctrl>(workspace, plan->lay.ctrl), sizeof(Ctrl), hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return UG_ERR_HIP;
  out_host[0] = (int64_t)c.n_rec;
  out_host[1] = (c.flags & kFlagRecCap) ? -1 : (int64_t)c.n_key;
  if (c.flags & kFlagInternal) return UG_ERR_INTERNAL;
  return (c.flags & kFlagNonfinite) ? UG_ERR_NONFINITE : UG_OK;
}

int ug_render_planes(const ug_plan* plan, const ug_gaussians* g, const ug_planes* planes, float* image,
                     void* workspace, void* stream) {
  return render_impl(plan, g, planes, image, workspace, stream);
}

int ug_render_planes_noalloc(const ug_plan* plan, const ug_gaussians* g, const ug_planes* planes, float* image,
                             void* stream) {
  if (!plan) return UG_ERR_INVALID_ARG;
  if (plan->lay.total > (size_t)UG_NOALLOC_WORKSPACE_BYTES) return UG_ERR_SCRATCH_SIZE;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return UG_ERR_HIP;
  if (dev != plan->device) return UG_ERR_INVALID_ARG;  // the plan's tables live on its own device
  void* ws = scratch_for_current_device();
  if (!ws) return UG_ERR_HIP;
  return render_impl(plan, g, planes, image, ws, stream);
}

}  // extern "C"

namespace {

int render_impl(const ug_plan* plan, const ug_gaussians* g, const ug_planes* planes, float* image, void* workspace,
                void* stream) {
  const int st = check_inputs(plan, g, planes, workspace);
  if (st != UG_OK) return st;
  if (!image) return UG_ERR_INVALID_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const Layout& L = plan->lay;
  void* ws = workspace;
  const RenderParams rp = make_rp(plan);
  Ctrl* ctrl = at<Ctrl>(ws, L.ctrl);
  if (plan->prm.flags & UG_FLAG_SCATTER) {
    // Phase 2: records only, then the atomic scatter into image (numerator)
    // and the saved denominators
    hipError_t e = enqueue_preprocess(plan, *g, *planes, ws, rp, s, false);
    if (e != hipSuccess) return UG_ERR_HIP;
    float* den = at<float>(ws, L.dsave);
    {
      StageScope sc(plan, UG_STAGE_SCATTER, s);
      e = launch_scatter_zero(image, den, plan->num_pixels, s);
    }
    if (e != hipSuccess) return UG_ERR_HIP;
    {
      // box-support records carry their rectangle in pixels, others in tiles
      const bool px = rp.box_support != 0;
      StageScope sc(plan, UG_STAGE_SCATTER, s);
      e = launch_scatter(ctrl, at<uint2>(ws, L.rec_pair), plan->d_pint, at<Rec>(ws, L.recs),
                         px ? 1 : plan->prm.tile_w, px ? 1 : plan->prm.tile_h,
                         plan->rec_cap, image, den, s);
    }
    if (e != hipSuccess) return UG_ERR_HIP;
    StageScope sc(plan, UG_STAGE_SCATTER, s);
    return hip_status(launch_scatter_norm(image, den, plan->num_pixels, plan->prm.bg_alpha, plan->prm.bg_color, s));
  }
  hipError_t e = enqueue_preprocess(plan, *g, *planes, ws, rp, s);
  if (e != hipSuccess) return UG_ERR_HIP;
  e = enqueue_sort(plan, ws, s);
  if (e != hipSuccess) return UG_ERR_HIP;
  const Sorted so = sorted_set(plan, ws);
  if (sort_passes(plan->bits, plan->sort_blocks) > 1) {  // one pass wrote the ranges itself
    StageScope sc(plan, UG_STAGE_RANGES, s);
    e = launch_tile_ranges(ctrl, so.key, plan->num_tiles, plan->key_cap,
                           key_mask_shift(plan->prm.tile_w, plan->prm.tile_h), at<uint32_t>(ws, L.tile_start), s);
  }
  if (e != hipSuccess) return UG_ERR_HIP;
  unsigned long long* n_eval = (plan->prm.flags & UG_FLAG_COUNT_EVALS) ? &ctrl->n_eval : nullptr;
  StageScope sc(plan, UG_STAGE_ACCUM, s);
  e = launch_accum_fwd(plan->prm.tile_w, plan->prm.tile_h, plan->prm.lds_batch,
                       (plan->prm.flags & UG_FLAG_SPLIT_FORWARD) ? 2 : 1, plan->d_pint, plan->d_tile_plane,
                       at<uint32_t>(ws, L.tile_start), so.key, so.rec, at<Rec>(ws, L.recs), image, at<float>(ws, L.dsave),
                       plan->prm.bg_alpha, plan->prm.bg_color, std::isfinite(plan->prm.chi2), plan->num_tiles,
                       n_eval, s);
  return hip_status(e);
}

// The backward passes; with target (mse), dL/dc_hat is formed from it in the
// first kernel and the loss goes to loss_dev (if not null).
int backward_impl(const ug_plan* plan, const ug_gaussians* g, const ug_planes* planes, const float* image,
                  const float* second, bool mse, float* loss_dev, void* workspace, float* d_means, float* d_lraw,
                  float* d_intensity, float* d_opacity, int32_t accumulate, void* stream) {
  const int st = check_inputs(plan, g, planes, workspace);
  if (st != UG_OK) return st;
  if (!image || !second) return UG_ERR_INVALID_ARG;
  if (plan->n > 0 && (!d_means || !d_lraw || !d_intensity || !d_opacity)) return UG_ERR_INVALID_ARG;
  if (accumulate != 0 && accumulate != 1) return UG_ERR_INVALID_ARG;
  if (plan->prm.flags & UG_FLAG_SCATTER) return UG_ERR_INVALID_ARG;  // no keys to walk
  hipStream_t s = static_cast<hipStream_t>(stream);
  const Layout& L = plan->lay;
  void* ws = workspace;
  const RenderParams rp = make_rp(plan);
  const Ctrl* ctrl = at<Ctrl>(ws, L.ctrl);
  const Sorted so = sorted_set(plan, ws);
  hipError_t e;
  {
    StageScope sc(plan, UG_STAGE_BWD_PREP, s);
    const float scale = 2.0f / (float)(plan->num_pixels > 0 ? plan->num_pixels : 1);
    e = launch_bwd_prep(plan->prm.tile_w, plan->prm.tile_h, plan->d_pint, plan->d_tile_plane, image, second, mse,
                        scale, at<float>(ws, L.loss_part), at<float>(ws, L.dsave), at<float>(ws, L.gq),
                        plan->num_tiles, s);
  }
  if (e != hipSuccess) return UG_ERR_HIP;
  {
    StageScope sc(plan, UG_STAGE_ACCUM_BWD, s);
    e = launch_accum_bwd(plan->prm.tile_w, plan->prm.tile_h, ctrl, plan->d_tile_org, so.key, so.val, so.rec, at<Rec>(ws, L.recs),
                         at<float>(ws, L.gq),
                         at<float>(ws, L.partial), std::isfinite(plan->prm.chi2), plan->key_cap, s);
  }
  if (e != hipSuccess) return UG_ERR_HIP;
  {
    StageScope sc(plan, UG_STAGE_RECORD_ADJ, s);
    e = launch_record_adjoint(*g, at<PlaneConst>(ws, L.pconst), rp, ctrl, at<uint2>(ws, L.rec_pair),
                              at<uint32_t>(ws, L.rec_koff), at<float>(ws, L.partial), at<uint32_t>(ws, L.cnt_rec),
                              at<unsigned long long>(ws, L.off_rec), at<float>(ws, L.side), d_means, d_lraw,
                              d_intensity, d_opacity, accumulate, s);
  }
  if (e != hipSuccess) return UG_ERR_HIP;
  StageScope sc(plan, UG_STAGE_GAUSS_GRAD, s);
  const uint32_t nparts = bwd_prep_blocks(plan->prm.tile_w, plan->prm.tile_h, plan->num_tiles);
  e = launch_gauss_grad(*g, rp, ctrl, at<uint32_t>(ws, L.cnt_rec), at<unsigned long long>(ws, L.off_rec),
                        at<float>(ws, L.side), d_means, d_lraw, d_intensity, d_opacity, accumulate,
                        at<float>(ws, L.loss_part), nparts,
                        1.0 / (double)(plan->num_pixels > 0 ? plan->num_pixels : 1), mse ? loss_dev : nullptr, s);
  return hip_status(e);
}

}  // namespace

extern "C" {

int ug_render_planes_backward(const ug_plan* plan, const ug_gaussians* g, const ug_planes* planes,
                              const float* image, const float* d_image, void* workspace, float* d_means,
                              float* d_lraw, float* d_intensity, float* d_opacity, int32_t accumulate,
                              void* stream) {
  return backward_impl(plan, g, planes, image, d_image, false, nullptr, workspace, d_means, d_lraw, d_intensity,
                       d_opacity, accumulate, stream);
}

int ug_render_planes_backward_mse(const ug_plan* plan, const ug_gaussians* g, const ug_planes* planes,
                                  const float* image, const float* target, void* workspace, float* d_means,
                                  float* d_lraw, float* d_intensity, float* d_opacity, int32_t accumulate,
                                  float* loss_dev, void* stream) {
  return backward_impl(plan, g, planes, image, target, true, loss_dev, workspace, d_means, d_lraw, d_intensity,
                       d_opacity, accumulate, stream);
}

int ug_plan_status(const ug_plan* plan, const void* workspace, int64_t* counts_host, void* stream) {
  if (!plan || !workspace) return UG_ERR_INVALID_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Ctrl c;
  if (hipMemcpyAsync(&c, static_cast<const char*>(workspace) + plan->lay.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost,
                     s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return UG_ERR_HIP;
  if (counts_host) {
    counts_host[0] = (int64_t)c.n_rec;
    counts_host[1] = (int64_t)c.n_key;
    counts_host[2] = (int64_t)c.n_eval;
    counts_host[3] = (int64_t)c.n_exec;
  }
  if (c.flags & kFlagInternal) return UG_ERR_INTERNAL;
  if (c.flags & (kFlagRecCap | kFlagKeyCap)) return UG_ERR_CAPACITY;
  if (c.flags & kFlagNonfinite) return UG_ERR_NONFINITE;
  return UG_OK;
}

int ug_mse_grad(const float* image, const float* target, int64_t m, float* d_image, float* loss_dev, void* stream) {
  if (!image || !target || !d_image || !loss_dev || m < 1) return UG_ERR_INVALID_ARG;
  return hip_status(launch_mse(image, target, m, d_image, loss_dev, static_cast<hipStream_t>(stream)));
}

int ug_adam_step(float* param, const float* grad, float* mo, float* ve, int64_t count, float lr, float beta1,
                 float beta2, float eps, int32_t step_t, void* stream) {
  if (!param || !grad || !mo || !ve || count < 0 || step_t < 1) return UG_ERR_INVALID_ARG;
  if (!(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f) || !std::isfinite(lr))
    return UG_ERR_INVALID_ARG;
  if (count == 0) return UG_OK;
  return hip_status(
      launch_adam(param, grad, mo, ve, count, lr, beta1, beta2, eps, step_t, static_cast<hipStream_t>(stream)));
}

int ug_adam_gaussians(const ug_plan* plan, const void* workspace, const ug_gaussians_mut* params,
                      const ug_gaussians_mut* grads, const ug_gaussians_mut* m1, const ug_gaussians_mut* m2,
                      const ug_adam_params* hp, int32_t* step_dev, void* stream) {
  if (!params || !grads || !m1 || !m2 || !hp || !step_dev) return UG_ERR_INVALID_ARG;
  const int32_t n = params->n;
  if (n < 0 || grads->n != n || m1->n != n || m2->n != n) return UG_ERR_INVALID_ARG;
  if ((plan == nullptr) != (workspace == nullptr)) return UG_ERR_INVALID_ARG;
  if (plan && plan->n != n) return UG_ERR_INVALID_ARG;
  const ug_gaussians_mut* all[4] = {params, grads, m1, m2};
  for (const ug_gaussians_mut* x : all)
    if (n > 0 && (!x->means || !x->lraw || !x->intensity || !x->opacity)) return UG_ERR_INVALID_ARG;
  if (!(hp->beta1 >= 0.f && hp->beta1 < 1.f) || !(hp->beta2 >= 0.f && hp->beta2 < 1.f) || !(hp->eps > 0.f) ||
      !(hp->lr_means > 0.f) || !(hp->lr_means_final > 0.f) || !std::isfinite(hp->lr) || hp->decay_steps < 1)
    return UG_ERR_INVALID_ARG;
  if (n == 0) return UG_OK;
  float* const p[4] = {params->means, params->lraw, params->intensity, params->opacity};
  const float* const g[4] = {grads->means, grads->lraw, grads->intensity, grads->opacity};
  float* const m[4] = {m1->means, m1->lraw, m1->intensity, m1->opacity};
  float* const v[4] = {m2->means, m2->lraw, m2->intensity, m2->opacity};
  const Ctrl* ctrl = plan ? reinterpret_cast<const Ctrl*>(static_cast<const char*>(workspace) + plan->lay.ctrl)
                          : nullptr;
  return hip_status(launch_adam_gaussians(p, g, m, v, n, *hp, step_dev, ctrl, static_cast<hipStream_t>(stream)));
}

int ug_sample_gaussians(const ug_gaussians* g, float beta, const int32_t* idx, const float* z, int64_t k,
                        float* out, void* stream) {
  if (!g || k < 0 || g->n < 0 || !(beta > 0.f) || !std::isfinite(beta)) return UG_ERR_INVALID_ARG;
  if (k == 0) return UG_OK;
  if (!idx || !z || !out || !g->means || !g->lraw) return UG_ERR_INVALID_ARG;
  return hip_status(launch_sample(*g, beta, idx, z, k, out, static_cast<hipStream_t>(stream)));
}

int ug_accumulate_grad_norm(const ug_plan* plan, const void* workspace, const float* d_means, int32_t n, float* acc,
                            int32_t* cnt, void* stream) {
  if (n < 0 || (plan == nullptr) != (workspace == nullptr)) return UG_ERR_INVALID_ARG;
  if (plan && plan->n != n) return UG_ERR_INVALID_ARG;
  if (n == 0) return UG_OK;
  if (!d_means || !acc || !cnt) return UG_ERR_INVALID_ARG;
  const Ctrl* ctrl = plan ? reinterpret_cast<const Ctrl*>(static_cast<const char*>(workspace) + plan->lay.ctrl)
                          : nullptr;
  return hip_status(launch_grad_norm(ctrl, d_means, n, acc, cnt, static_cast<hipStream_t>(stream)));
}

void ug_densify_params_default(ug_densify_params* out) {
  if (!out) return;
  out->beta = 1e-4f;
  out->min_opacity = 0.005f;
  out->grad_thresh = 2e-4f;
  out->split_size = 1.0f;
  out->max_size = 0.0f;
  out->split_factor = 1.6f;
}

size_t ug_densify_workspace_bytes(int32_t n) {
  return n < 0 ? 0 : align_up((size_t)densify_blocks(n) * 4 + 4);
}

int ug_densify(const ug_gaussians* g, const float* acc, const int32_t* cnt, const float* z,
               const ug_densify_params* dp, const ug_gaussians_mut* out, int64_t out_capacity, int64_t* count_dev,
               void* workspace, void* stream) {
  if (!g || !dp || !out || !count_dev || !workspace || g->n < 0 || out_capacity < 0) return UG_ERR_INVALID_ARG;
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return UG_ERR_INVALID_ARG;
  if (!(dp->beta > 0.f) || !std::isfinite(dp->beta) || !(dp->min_opacity >= 0.f && dp->min_opacity <= 1.f) ||
      !std::isfinite(dp->grad_thresh) || !(dp->split_size >= 0.f) || !std::isfinite(dp->split_size) ||
      !(dp->max_size >= 0.f) || !std::isfinite(dp->max_size) || !(dp->split_factor > 1.f) ||
      !std::isfinite(dp->split_factor))
    return UG_ERR_INVALID_ARG;
  if (g->n > 0 && (!g->means || !g->lraw || !g->intensity || !g->opacity || !acc || !cnt || !z))
    return UG_ERR_INVALID_ARG;
  if (out_capacity > 0 && (!out->means || !out->lraw || !out->intensity || !out->opacity)) return UG_ERR_INVALID_ARG;
  return hip_status(launch_densify(*g, acc, cnt, z, *dp, *out, out_capacity, count_dev,
                                   static_cast<uint32_t*>(workspace), static_cast<hipStream_t>(stream)));
}

size_t ug_quality_workspace_bytes(const ug_plan* plan) {
  return plan ? align_up((size_t)plan->p * quality_strips(plan->max_w) * sizeof(double2)) : 0;
}

int ug_image_quality(const ug_plan* plan, const float* image, const float* ref, float data_range, double* ssim,
                     double* mse, void* workspace, void* stream) {
  if (!plan || !image || !ref || !ssim || !mse || !workspace) return UG_ERR_INVALID_ARG;
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return UG_ERR_INVALID_ARG;
  if (!(data_range > 0.f) || !std::isfinite(data_range)) return UG_ERR_INVALID_ARG;
  QualityConst q;
  double sum = 0.0;
  for (int k = 0; k < 11; ++k) {
    const double d = (double)(k - 5);
    q.taps[k] = std::exp(-d * d / (2.0 * 1.5 * 1.5));
    sum += q.taps[k];
  }
  for (int k = 0; k < 11; ++k) q.taps[k] /= sum;
  const double L = (double)data_range;
  q.c1 = (0.01 * L) * (0.01 * L);
  q.c2 = (0.03 * L) * (0.03 * L);
  return hip_status(launch_quality(plan->d_pint, plan->p, quality_strips(plan->max_w), image, ref, q,
                                   static_cast<double2*>(workspace), ssim, mse, static_cast<hipStream_t>(stream)));
}

int ug_param_eval(int32_t kind, int32_t fp64, const float* raw, const float* z, const float* delta, int64_t n,
                  float beta, void* sigma, void* draw, void* d2, void* stream) {
  if (kind != UG_PARAM_TRI && kind != UG_PARAM_SYM && kind != UG_PARAM_QUAT) return UG_ERR_INVALID_ARG;
  if (n < 0 || (fp64 != 0 && fp64 != 1)) return UG_ERR_INVALID_ARG;
  if (n > 0 && (!raw || !z || !delta || !sigma || !draw || !d2)) return UG_ERR_INVALID_ARG;
  if (n > (int64_t)0x7fffffff * 256) return UG_ERR_INVALID_ARG;  // grid limit
  return hip_status(launch_param_eval(kind, fp64 != 0, raw, z, delta, n, beta, sigma, draw, d2,
                                      static_cast<hipStream_t>(stream)));
}

int ug_probe(int32_t kind, int32_t blocks, int32_t iters, const float* src, float* dst, int64_t n, float* ms_host,
             void* stream) {
  if (kind < UG_PROBE_FMA || kind > UG_PROBE_COPY || blocks < 1 || blocks > (1 << 20) || iters < 1 || !dst ||
      !ms_host || n < 0)
    return UG_ERR_INVALID_ARG;
  if (kind == UG_PROBE_COPY) {
    if (!src || n % 4 || reinterpret_cast<uintptr_t>(src) % 16 || reinterpret_cast<uintptr_t>(dst) % 16)
      return UG_ERR_INVALID_ARG;
  } else if (n < (int64_t)blocks * 256) {
    return UG_ERR_INVALID_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int st = UG_OK;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) st = UG_ERR_HIP;
  if (st == UG_OK && (hipEventRecord(e0, s) != hipSuccess || launch_probe(kind, blocks, iters, src, dst, n, s) !=
                                                                   hipSuccess ||
                      hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                      hipEventElapsedTime(ms_host, e0, e1) != hipSuccess))
    st = UG_ERR_HIP;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return st;
}

const char* ug_status_string(int status) {
  switch (status) {
    case UG_OK: return "ok";
    case UG_ERR_INVALID_ARG: return "invalid argument";
    case UG_ERR_CAPACITY: return "record or key capacity exceeded; re-plan with larger capacities";
    case UG_ERR_NONFINITE: return "non-finite Gaussian or plane input (skipped)";
    case UG_ERR_HIP: return "HIP runtime error";
    case UG_ERR_NO_DEVICE: return "no gfx950 device available";
    case UG_ERR_INTERNAL: return "internal consistency check failed (please report)";
    case UG_ERR_SCRATCH_SIZE:
      return "the plan needs more workspace than the no-allocation forward holds (UG_NOALLOC_WORKSPACE_BYTES)";
    default: return "unknown status";
  }
}

int ug_profile_begin(ug_plan* plan, uint32_t stage_mask, int32_t max_launches) {
  if (!plan || max_launches < 1 || max_launches > (1 << 20)) return UG_ERR_INVALID_ARG;
  prof_release(plan);
  ug_plan::Prof& P = plan->prof;
  P.ev.resize(2 * (size_t)max_launches, nullptr);
  P.stage.assign((size_t)max_launches, -1);
  for (auto& e : P.ev) {
    if (hipEventCreate(&e) != hipSuccess) {
      e = nullptr;
      prof_release(plan);
      return UG_ERR_HIP;
    }
  }
  P.cap = max_launches;
  P.used = 0;
  P.mask = stage_mask;
  P.on = true;
  return UG_OK;
}

int ug_profile_read(ug_plan* plan, float* ms_host, int32_t* launches_host) {
  if (!plan) return UG_ERR_INVALID_ARG;
  ug_plan::Prof& P = plan->prof;
  float ms[UG_NUM_STAGES] = {0};
  int32_t cnt[UG_NUM_STAGES] = {0};
  int st = UG_OK;
  if (P.used > 0) {
    if (hipEventSynchronize(P.ev[2 * (size_t)(P.used - 1) + 1]) != hipSuccess) st = UG_ERR_HIP;
    for (int i = 0; i < P.used && st == UG_OK; ++i) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, P.ev[2 * (size_t)i], P.ev[2 * (size_t)i + 1]) != hipSuccess) {
        st = UG_ERR_HIP;
        break;
      }
      const int sg = P.stage[(size_t)i];
      if (sg >= 0 && sg < UG_NUM_STAGES) {
        ms[sg] += t;
        cnt[sg] += 1;
      }
    }
  }
  if (ms_host)
    for (int i = 0; i < UG_NUM_STAGES; ++i) ms_host[i] = ms[i];
  if (launches_host)
    for (int i = 0; i < UG_NUM_STAGES; ++i) launches_host[i] = cnt[i];
  prof_release(plan);
  return st;
}

static_assert(sizeof(ug_record) == 56, "ug_record layout");

int64_t ug_debug_records(const ug_plan* plan, const void* workspace, ug_record* host_out, int64_t cap,
                         void* stream) {
  if (!plan || !workspace || cap < 0 || (cap > 0 && !host_out)) return UG_ERR_INVALID_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const Layout& L = plan->lay;
  const char* ws = static_cast<const char*>(workspace);
  Ctrl c;
  if (hipMemcpyAsync(&c, ws + L.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return UG_ERR_HIP;
  const int64_t n = (int64_t)c.n_rec_eff;
  const int64_t m = n < cap ? n : cap;
  if (m > 0) {
    std::vector<uint2> pair((size_t)m);
    std::vector<Rec> rec((size_t)m);
    if (hipMemcpyAsync(pair.data(), ws + L.rec_pair, (size_t)m * sizeof(uint2), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipMemcpyAsync(rec.data(), ws + L.recs, (size_t)m * sizeof(Rec), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return UG_ERR_HIP;
    for (int64_t i = 0; i < m; ++i) {
      ug_record& r = host_out[i];
      r.gaussian = (int32_t)pair[(size_t)i].x;
      r.plane = (int32_t)pair[(size_t)i].y;
      const RecAcc& a = rec[(size_t)i].acc;
      r.t11 = a.t11;
      r.t12 = a.t12;
      r.t22 = a.t22;
      r.fu = a.fu;
      r.fv = a.fv;
      r.e0 = a.e0;
      r.emin = a.emin;
      r.c = a.c;
      const RecGeo& gg = rec[(size_t)i].geo;
      r.ub = gg.ub;
      r.vb = gg.vb;
      r.tx0 = gg.tx0;
      r.tx1 = gg.tx1;
      r.ty0 = gg.ty0;
      r.ty1 = gg.ty1;
    }
  }
  return n;
}

int64_t ug_debug_keys(const ug_plan* plan, const void* workspace, uint32_t* key_out, uint32_t* eidx_out,
                      uint32_t* rec_out, uint32_t* ranges_out, int64_t cap, void* stream) {
  if (!plan || !workspace || cap < 0) return UG_ERR_INVALID_ARG;
  if (plan->prm.flags & UG_FLAG_SCATTER) return UG_ERR_INVALID_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const Layout& L = plan->lay;
  void* ws = const_cast<void*>(workspace);
  Ctrl c;
  if (hipMemcpyAsync(&c, at<Ctrl>(ws, L.ctrl), sizeof(Ctrl), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return UG_ERR_HIP;
  const int64_t n = (int64_t)c.n_key_eff;
  const int64_t m = n < cap ? n : cap;
  const Sorted so = sorted_set(plan, ws);
  const std::pair<uint32_t*, const uint32_t*> arrays[3] = {{key_out, so.key}, {eidx_out, so.val}, {rec_out, so.rec}};
  for (const auto& a : arrays) {
    if (a.first && m > 0 &&
        hipMemcpyAsync(a.first, a.second, (size_t)m * 4, hipMemcpyDeviceToHost, s) != hipSuccess)
      return UG_ERR_HIP;
  }
  if (ranges_out && hipMemcpyAsync(ranges_out, at<uint32_t>(ws, L.tile_start), ((size_t)plan->num_tiles + 1) * 4,
                                   hipMemcpyDeviceToHost, s) != hipSuccess)
    return UG_ERR_HIP;
  if (hipStreamSynchronize(s) != hipSuccess) return UG_ERR_HIP;
  return n;
}

int ug_step_capture(ug_plan* plan, const ug_gaussians_mut* params, const ug_planes* planes, const float* target,
                    float* image, void* workspace, const ug_gaussians_mut* grads, const ug_gaussians_mut* m1,
                    const ug_gaussians_mut* m2, const ug_adam_params* adam, int32_t* step_dev, float* loss_dev,
                    float* grad_acc, int32_t* grad_cnt) {
  if (!plan || !params || !planes || !target || !image || !workspace || !grads || !m1 || !m2 || !adam ||
      !step_dev)
    return UG_ERR_INVALID_ARG;
  if ((grad_acc == nullptr) != (grad_cnt == nullptr)) return UG_ERR_INVALID_ARG;
  if (plan->prof.on) return UG_ERR_INVALID_ARG;  // the hooks' events would be captured
  if (plan->prm.flags & UG_FLAG_SCATTER) return UG_ERR_INVALID_ARG;
  const ug_gaussians g{params->means, params->lraw, params->intensity, params->opacity, params->n};
  int st = check_inputs(plan, &g, planes, workspace);
  if (st != UG_OK) return st;
  int prev = 0;
  if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(plan->device) != hipSuccess) return UG_ERR_HIP;
  hipStream_t cs = nullptr;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
    (void)hipSetDevice(prev);
    return UG_ERR_HIP;
  }
  st = UG_OK;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) st = UG_ERR_HIP;
  if (st == UG_OK) {
    st = ug_render_planes(plan, &g, planes, image, workspace, cs);
    if (st == UG_OK)
      st = ug_render_planes_backward_mse(plan, &g, planes, image, target, workspace, grads->means, grads->lraw,
                                         grads->intensity, grads->opacity, 0, loss_dev, cs);
    if (st == UG_OK && grad_acc)
      st = ug_accumulate_grad_norm(plan, workspace, grads->means, g.n, grad_acc, grad_cnt, cs);
    if (st == UG_OK) st = ug_adam_gaussians(plan, workspace, params, grads, m1, m2, adam, step_dev, cs);
    hipGraph_t graph = nullptr;
    const hipError_t ee = hipStreamEndCapture(cs, &graph);  // always ends the capture
    hipGraphExec_t exec = nullptr;
    if (st == UG_OK && (ee != hipSuccess || !graph || hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) !=
                                                           hipSuccess))
      st = UG_ERR_HIP;
    if (graph) (void)hipGraphDestroy(graph);
    if (st == UG_OK) {
      if (plan->step_exec) (void)hipGraphExecDestroy(plan->step_exec);
      plan->step_exec = exec;
    } else if (exec) {
      (void)hipGraphExecDestroy(exec);
    }
  }
  (void)hipStreamDestroy(cs);
  (void)hipSetDevice(prev);
  return st;
}

int ug_step_replay(ug_plan* plan, void* stream) {
  if (!plan || !plan->step_exec) return UG_ERR_INVALID_ARG;
  return hip_status(hipGraphLaunch(plan->step_exec, static_cast<hipStream_t>(stream)));
}

void ug_plan_destroy(ug_plan* plan) {
  if (!plan) return;
  prof_release(plan);
  if (plan->step_exec) (void)hipGraphExecDestroy(plan->step_exec);
  if (plan->d_pint) (void)hipFree(plan->d_pint);
  if (plan->d_tile_plane) (void)hipFree(plan->d_tile_plane);
  if (plan->d_tile_org) (void)hipFree(plan->d_tile_org);
  delete plan;
}

}  // extern "C"
