// C ABI of the rasterizer (include/psm.h): argument validation, workspace
// layout and the ordered enqueue of the kernels on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "../../include/psm.h"
#include "internal.h"

using namespace psm;

namespace {

const char* const kStageNames[kNumStages] = {"preprocess", "depth_sort", "count_scan", "emit",
                                             "pair_sort",  "ranges",     "walk",       "feature_blend",
                                             "bwd_feature", "bwd_walk",  "bwd_reduce", "fill"};

// HIP-event stage timer: an event pair per stage and call, on the call's stream.
struct Profiler {
  std::vector<hipEvent_t> pool;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[kNumStages];
  hipEvent_t open[kNumStages] = {};
  double total_ms[kNumStages] = {};
  int64_t calls[kNumStages] = {};

  hipEvent_t take() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
  }
  static void mark(void* self, int stage, int is_end, hipStream_t st) {
    Profiler* p = static_cast<Profiler*>(self);
    hipEvent_t e = p->take();
    (void)hipEventRecord(e, st);
    if (!is_end) p->open[stage] = e;
    else p->pending[stage].push_back({p->open[stage], e});
  }
  bool collect() {
    bool ok = true;
    for (int s = 0; s < kNumStages; ++s) {
      for (auto& pr : pending[s]) {
        float ms = 0.0f;
        if (hipEventSynchronize(pr.second) != hipSuccess || hipEventElapsedTime(&ms, pr.first, pr.second) != hipSuccess)
          ok = false;
        total_ms[s] += ms;
        calls[s] += 1;
        pool.push_back(pr.first);
        pool.push_back(pr.second);
      }
      pending[s].clear();
    }
    return ok;
  }
  ~Profiler() {
    for (auto& v : pending)
      for (auto& pr : v) pool.push_back(pr.first), pool.push_back(pr.second);
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};

}  // namespace

struct TuneKey {
  std::string key;
  psm::Tuning tu;
  int tile_w;
  double ms;
};

struct psm_ctx {
  int device;
  int cu_count;
  void* scratch;  // device address of the static workspace on `device`
  Profiler prof;
  std::vector<TuneKey> tuned;
};

namespace psm {

// Persistent grids: as many blocks as fit on the device at once.
int tile_grid(const Layout& L, int sched, const void* kernel, size_t dyn_lds) {
  if (sched != kSchedPersistent) return xcd_grid(L.tiles);
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, dyn_lds) != hipSuccess || per_cu < 1)
    per_cu = 1;
  const int64_t g = (int64_t)cus * per_cu;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, L.tiles));
}

}  // namespace psm

// ----------------------------------------------------- static workspace
// For callers that cannot allocate device memory: a file-scope device array
// used as the workspace of psm_forward_static.  Each device holds its own
// copy from the library's load until the process ends.  In host code the
// array's name is only a stand-in; its device address is fetched once per
// device (psm_create, with that device current) and kept per device.
static __device__ __align__(256) char scratch[PSM_STATIC_WORKSPACE_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device` (the current device).
hipError_t fetch_scratch(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = ptr;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

}  // namespace

namespace {

ProfHook hook_for(psm_ctx* ctx, const psm_config* cfg) {
  ProfHook h;
  if (cfg->flags & PSM_FLAG_PROFILE) {
    h.self = &ctx->prof;
    h.mark = &Profiler::mark;
  }
  return h;
}

thread_local std::string g_err;

psm_status fail(psm_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

// Keeps the caller's current device and restores it on exit.
struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

psm_status check_hip(const char* where) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(PSM_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
  return PSM_OK;
}

psm_status validate_camera(const psm_camera* cam) {
  if (cam->width < 1 || cam->height < 1 || cam->width > 16384 || cam->height > 16384)
    return fail(PSM_ERR_INVALID_ARG, "image size must be in [1, 16384]");
  if (!(cam->near_plane > 0.0f) || !std::isfinite(cam->near_plane))
    return fail(PSM_ERR_INVALID_ARG, "near_plane must be finite and > 0");
  if (!std::isfinite(cam->fx) || !std::isfinite(cam->fy) || cam->fx == 0.0f || cam->fy == 0.0f)
    return fail(PSM_ERR_INVALID_ARG, "focal lengths must be finite and non-zero");
  return PSM_OK;
}

psm_status validate_common(const psm_camera* cams, int32_t n_cams, const psm_config* cfg, int64_t n, int32_t c,
                           int64_t pair_capacity) {
  if (!cams || !cfg) return fail(PSM_ERR_INVALID_ARG, "camera and config are required");
  if (n_cams < 1 || n_cams > kMaxCams) return fail(PSM_ERR_INVALID_ARG, "n_cams must be in [1, 8]");
  if (n < 0 || n * n_cams > 0x7FFFFFFFLL) return fail(PSM_ERR_INVALID_ARG, "n * n_cams must be in [0, 2^31)");
  const int tw = cfg->tile_w;
  if (tw != 0 && tw != 8 && tw != 16 && tw != 32 && tw != 64)
    return fail(PSM_ERR_INVALID_ARG, "tile_w must be 0, 8, 16, 32 or 64");
  const int tw1 = tw == 0 ? kTileDefault : tw, th1 = kTilePix / tw1;
  int64_t tiles = 0;
  for (int b = 0; b < n_cams; ++b) {
    psm_status r = validate_camera(cams + b);
    if (r != PSM_OK) return r;
    tiles += cdiv(cams[b].width, tw1) * cdiv(cams[b].height, th1);
  }
  if (tiles * kTilePix > 0x7FFFFFFFLL) return fail(PSM_ERR_INVALID_ARG, "too many pixels in one call");
  if (cfg->k < 1 || cfg->k > kMaxK) return fail(PSM_ERR_INVALID_ARG, "k must be in [1, 32]");
  if (cfg->tile_mode < 0 || cfg->tile_mode > 2) return fail(PSM_ERR_INVALID_ARG, "bad tile_mode");
  if (cfg->blend < 0 || cfg->blend > 1) return fail(PSM_ERR_INVALID_ARG, "bad blend mode");
  if (cfg->schedule < 0 || cfg->schedule > 1) return fail(PSM_ERR_INVALID_ARG, "bad schedule");
  if (cfg->bwd_schedule < 0 || cfg->bwd_schedule > 1) return fail(PSM_ERR_INVALID_ARG, "bad bwd_schedule");
  if (cfg->blend_pass != 0 && cfg->blend_pass != 16 && cfg->blend_pass != 32)
    return fail(PSM_ERR_INVALID_ARG, "blend_pass must be 0, 16 or 32");
  if (cfg->bwd_pass != 0 && cfg->bwd_pass != 16 && cfg->bwd_pass != 32)
    return fail(PSM_ERR_INVALID_ARG, "bwd_pass must be 0, 16 or 32");
  if (cfg->flags & ~(PSM_FLAG_NO_SYNC | PSM_FLAG_PROFILE | PSM_FLAG_OPACITY_FOOTPRINT | PSM_FLAG_FEATURE_ONLY |
                     PSM_FLAG_TOPK_RENORM | PSM_FLAG_LOWPASS))
    return fail(PSM_ERR_INVALID_ARG, "unknown flag bits");
  if ((cfg->flags & PSM_FLAG_TOPK_RENORM) && (cfg->blend != PSM_BLEND_TOPK || c == 0))
    return fail(PSM_ERR_INVALID_ARG, "PSM_FLAG_TOPK_RENORM needs the Top-K blend and c > 0");
  if ((cfg->flags & PSM_FLAG_FEATURE_ONLY) && (cfg->blend != PSM_BLEND_TOPK || c == 0))
    return fail(PSM_ERR_INVALID_ARG, "PSM_FLAG_FEATURE_ONLY needs the Top-K blend and c > 0");
  if (c < 0 || c > 1024) return fail(PSM_ERR_INVALID_ARG, "c must be in [0, 1024]");
  if (c % 8 != 0) return fail(PSM_ERR_UNSUPPORTED, "c must be a multiple of 8");
  if (pair_capacity < 0 || pair_capacity > 0x7FFFFFFFLL)
    return fail(PSM_ERR_INVALID_ARG, "pair_capacity must be in [0, 2^31)");
  return PSM_OK;
}

psm_status validate_surfels(const psm_surfels* s) {
  if (!s) return fail(PSM_ERR_INVALID_ARG, "surfels are required");
  if (s->feat_dtype < 0 || s->feat_dtype > 2) return fail(PSM_ERR_INVALID_ARG, "bad feat_dtype");
  if (s->n > 0 && (!s->means || !s->scales || !s->quats || !s->opacity || !s->rgb))
    return fail(PSM_ERR_INVALID_ARG, "null surfel parameter array");
  if (s->c < 0 || s->c > 1024 || s->c_ext < 0 || s->c_ext > 1024)
    return fail(PSM_ERR_INVALID_ARG, "c and c_ext must be in [0, 1024]");
  if (s->c_ext % 8 != 0) return fail(PSM_ERR_UNSUPPORTED, "c_ext must be a multiple of 8");
  if (s->n > 0 && s->c > 0) {
    if (!s->feat) return fail(PSM_ERR_INVALID_ARG, "null feature array");
    if (reinterpret_cast<uintptr_t>(s->feat) % 16 != 0)
      return fail(PSM_ERR_INVALID_ARG, "feature array must be 16-byte aligned");
  }
  if (s->n > 0 && s->c_ext > 0) {
    if (!s->feat_ext) return fail(PSM_ERR_INVALID_ARG, "null second feature array");
    if (reinterpret_cast<uintptr_t>(s->feat_ext) % 16 != 0)
      return fail(PSM_ERR_INVALID_ARG, "second feature array must be 16-byte aligned");
  }
  return PSM_OK;
}

// Rendered feature channels: both sources (validate_surfels bounds each part,
// validate_common the sum).
int feat_channels(const psm_surfels* s) { return s->c + s->c_ext; }

int tile_width(const psm_config* cfg) { return !cfg || cfg->tile_w == 0 ? kTileDefault : cfg->tile_w; }

CamTable cam_table(const psm_camera* cams, int32_t n_cams, int64_t n, const psm_config* cfg) {
  CamTable t;
  std::memset(&t, 0, sizeof(t));
  t.n = n_cams;
  t.nsurf = n;
  t.tw = tile_width(cfg);
  t.th = kTilePix / t.tw;
  t.tsh = 0;
  while ((1 << t.tsh) < t.tw) ++t.tsh;
  int tile = 0;
  int64_t pix = 0;
  for (int b = 0; b < n_cams; ++b) {
    const psm_camera* cam = cams + b;
    CamArgs& a = t.cam[b];
    std::memcpy(a.R, cam->R, sizeof(a.R));
    std::memcpy(a.t, cam->t, sizeof(a.t));
    a.fx = cam->fx; a.fy = cam->fy; a.cx = cam->cx; a.cy = cam->cy; a.near_plane = cam->near_plane;
    a.W = cam->width; a.H = cam->height;
    t.ntx[b] = (int)cdiv(cam->width, t.tw);
    t.nty[b] = (int)cdiv(cam->height, t.th);
    t.tile0[b] = tile;
    t.pix0[b] = pix;
    tile += t.ntx[b] * t.nty[b];
    pix += (int64_t)cam->width * cam->height;
  }
  for (int b = n_cams; b <= kMaxCams; ++b) {
    t.tile0[b] = tile;
    t.pix0[b] = pix;
  }
  for (int b = n_cams; b < kMaxCams; ++b) t.ntx[b] = t.nty[b] = 1;
  return t;
}

Tuning tuning_of(const psm_config* cfg) {
  Tuning t;
  t.sched = cfg->schedule;
  t.sched_bwd = cfg->bwd_schedule;
  t.blend_pass = cfg->blend_pass == 0 ? 32 : cfg->blend_pass;
  t.bwd_pass = cfg->bwd_pass == 0 ? 16 : cfg->bwd_pass;
  return t;
}

SurfelArgs surfel_args(const psm_surfels* s) {
  return SurfelArgs{s->n,      s->means,           s->scales,     s->quats,   s->opacity,
                    s->rgb,    s->feat,            feat_channels(s), s->feat_dtype,
                    s->c_ext > 0 ? s->feat_ext : nullptr, s->c};
}

int bits_for(int64_t tiles) {
  int b = 0;
  while ((1LL << b) < tiles) ++b;
  return b;
}

psm_status check_workspace(const Layout& L, const void* ws, size_t bytes) {
  if (!ws) return fail(PSM_ERR_INVALID_ARG, "workspace is required");
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(PSM_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  if (bytes < L.total)
    return fail(PSM_ERR_INVALID_ARG, "workspace too small: need " + std::to_string(L.total) + " bytes");
  return PSM_OK;
}

psm_status read_status(const Layout& L, const void* ws, uint32_t* st_host, hipStream_t st) {
  if (hipMemcpyAsync(st_host, (const char*)ws + L.status, kStWords * 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return fail(PSM_ERR_HIP, std::string("status read-back: ") + hipGetErrorString(hipGetLastError()));
  return PSM_OK;
}

// Checks the layout the forward recorded against the one the read-back
// computed from its arguments (so no read-back addresses past the workspace).
psm_status check_signature(const Layout& L, const uint32_t* h) {
  const uint64_t total = (uint64_t)h[kStSigLo] | ((uint64_t)h[kStSigHi] << 32);
  if (total != (uint64_t)L.total || h[kStSigCap] != (uint32_t)L.cap || h[kStSigTiles] != (uint32_t)L.tiles)
    return fail(PSM_ERR_INVALID_ARG, "the workspace was laid out by a forward with other arguments (n, cameras, "
                                     "k, c or pair capacity) or holds no forward");
  return PSM_OK;
}

inline int64_t word64(const uint32_t* h, int i) { return (int64_t)((uint64_t)h[i] | ((uint64_t)h[i + 1] << 32)); }

psm_status capacity_error(const Layout& L, const uint32_t* h) {
  const uint64_t req = (uint64_t)h[kStReqLo] | ((uint64_t)h[kStReqHi] << 32);
  return fail(PSM_ERR_CAPACITY, "pair capacity " + std::to_string(L.cap) + " < required " + std::to_string(req));
}

// Enqueues the forward on `st` (no host synchronisation).
void enqueue_forward(const SurfelArgs& sa, const CamTable& ct, const psm_config* cfg, const Layout& L, char* ws,
                     const psm_images* out, hipStream_t st, const ProfHook& prof) {
  const Tuning tu = tuning_of(cfg);
  int64_t big = std::max<int64_t>(std::max<int64_t>(L.n, L.cap), L.tiles);
  const int64_t nb_max = cdiv(std::max<int64_t>(big, 1), kSortTile);
  uint32_t* status = (uint32_t*)(ws + L.status);
  uint32_t* hist = (uint32_t*)(ws + L.hist);
  prof.begin(kStageFill, st);
  launch_init_status(status, L, st);
  launch_fill_u32(ws + L.ranges, 0u, L.tiles * 2, st);
  prof.end(kStageFill, st);
  prof.begin(kStagePreprocess, st);
  const bool lp = (cfg->flags & PSM_FLAG_LOWPASS) != 0;
  launch_preprocess(sa, ct, cfg->tile_mode, (cfg->flags & PSM_FLAG_OPACITY_FOOTPRINT) != 0, lp, L, ws, st);
  prof.end(kStagePreprocess, st);
  prof.begin(kStageDepthSort, st);
  radix_sort_pairs((uint32_t*)(ws + L.key0), (uint32_t*)(ws + L.id0), (uint32_t*)(ws + L.key1),
                   (uint32_t*)(ws + L.id1), status + kStN, L.n, 32, hist, nb_max, st);
  prof.end(kStageDepthSort, st);
  prof.begin(kStageScan, st);
  launch_scan_counts(L, ws, st);
  prof.end(kStageScan, st);
  prof.begin(kStageEmit, st);
  launch_emit(ct, cfg->tile_mode, L, ws, st);
  prof.end(kStageEmit, st);
  prof.begin(kStagePairSort, st);
  radix_sort_pairs((uint32_t*)(ws + L.ptile0), (uint32_t*)(ws + L.eid0), (uint32_t*)(ws + L.ptile1),
                   (uint32_t*)(ws + L.eid1), status + kStP, L.cap, bits_for(L.tiles), hist, nb_max, st);
  prof.end(kStagePairSort, st);
  prof.begin(kStageRanges, st);
  launch_ranges(L, ws, st);
  if (tu.sched == kSchedPersistent || tu.sched_bwd == kSchedPersistent) launch_tile_order(L, ws, st);
  prof.end(kStageRanges, st);
  ImageArgs ia{out->rgb, out->depth, out->normal, out->alpha, out->feat};
  prof.begin(kStageWalk, st);
  launch_walk(L, ct, cfg->blend, tu, ia, (cfg->flags & PSM_FLAG_FEATURE_ONLY) != 0, lp, ws, st);
  prof.end(kStageWalk, st);
  prof.begin(kStageBlend, st);
  launch_feature_blend(sa, L, ct, cfg->blend, tu, out->feat, (cfg->flags & PSM_FLAG_TOPK_RENORM) != 0, lp, ws, st);
  prof.end(kStageBlend, st);
}

psm_status forward_impl(psm_ctx* ctx, const psm_surfels* s, const psm_camera* cams, int32_t n_cams,
                        const psm_config* cfg, void* workspace, size_t workspace_bytes, int64_t pair_capacity,
                        psm_images* out, void* stream) {
  if (!ctx) return fail(PSM_ERR_INVALID_ARG, "ctx is null");
  if (!out) return fail(PSM_ERR_INVALID_ARG, "out is null");
  psm_status r = validate_surfels(s);
  if (r != PSM_OK) return r;
  r = validate_common(cams, n_cams, cfg, s->n, feat_channels(s), pair_capacity);
  if (r != PSM_OK) return r;
  const CamTable ct = cam_table(cams, n_cams, s->n, cfg);
  const Layout L = make_layout(ct, cfg->k, feat_channels(s), pair_capacity);
  r = check_workspace(L, workspace, workspace_bytes);
  if (r != PSM_OK) return r;
  if (feat_channels(s) > 0 && !out->feat) return fail(PSM_ERR_INVALID_ARG, "out->feat is required when c > 0");
  if ((cfg->flags & PSM_FLAG_FEATURE_ONLY) && (out->rgb || out->depth || out->normal || out->alpha))
    return fail(PSM_ERR_INVALID_ARG, "PSM_FLAG_FEATURE_ONLY renders only the feature map: pass null rgb, depth, "
                                     "normal and alpha");
  DeviceGuard dg(ctx->device);
  if (!dg.ok) return fail(PSM_ERR_HIP, "hipSetDevice failed");
  hipStream_t st = (hipStream_t)stream;
  enqueue_forward(surfel_args(s), ct, cfg, L, (char*)workspace, out, st, hook_for(ctx, cfg));
  r = check_hip("psm_forward launch");
  if (r != PSM_OK) return r;
  if (!(cfg->flags & PSM_FLAG_NO_SYNC)) {
    uint32_t h[kStWords];
    r = read_status(L, workspace, h, st);
    if (r != PSM_OK) return r;
    if (h[kStOverflow]) return capacity_error(L, h);
  }
  g_err.clear();
  return PSM_OK;
}

psm_status backward_impl(psm_ctx* ctx, const psm_surfels* s, const psm_camera* cams, int32_t n_cams,
                         const psm_config* cfg, void* workspace, size_t workspace_bytes, int64_t pair_capacity,
                         const psm_image_grads* grad_out, psm_grads* grads, void* stream) {
  if (!ctx) return fail(PSM_ERR_INVALID_ARG, "ctx is null");
  if (!grad_out || !grads) return fail(PSM_ERR_INVALID_ARG, "grad_out and grads are required");
  psm_status r = validate_surfels(s);
  if (r != PSM_OK) return r;
  r = validate_common(cams, n_cams, cfg, s->n, feat_channels(s), pair_capacity);
  if (r != PSM_OK) return r;
  if (s->n > 0 && (!grads->means || !grads->scales || !grads->quats || !grads->opacity || !grads->rgb ||
                   (s->c > 0 && !grads->feat) || (s->c_ext > 0 && !grads->feat_ext)))
    return fail(PSM_ERR_INVALID_ARG, "every gradient array is required");
  if ((cfg->flags & PSM_FLAG_FEATURE_ONLY) && (grad_out->rgb || grad_out->depth || grad_out->normal || grad_out->alpha))
    return fail(PSM_ERR_INVALID_ARG, "PSM_FLAG_FEATURE_ONLY takes only the feature map's upstream gradient");
  const CamTable ct = cam_table(cams, n_cams, s->n, cfg);
  const Layout L = make_layout(ct, cfg->k, feat_channels(s), pair_capacity);
  r = check_workspace(L, workspace, workspace_bytes);
  if (r != PSM_OK) return r;
  DeviceGuard dg(ctx->device);
  if (!dg.ok) return fail(PSM_ERR_HIP, "hipSetDevice failed");
  hipStream_t st = (hipStream_t)stream;
  ImageGradArgs g{grad_out->rgb, grad_out->depth, grad_out->normal, grad_out->alpha, grad_out->feat};
  GradArgs ga{grads->means, grads->scales, grads->quats, grads->opacity, grads->rgb, grads->feat,
              s->c_ext > 0 ? grads->feat_ext : nullptr};
  launch_backward(surfel_args(s), ct, cfg->blend, tuning_of(cfg), L, g, ga, (cfg->flags & PSM_FLAG_TOPK_RENORM) != 0,
                  (cfg->flags & PSM_FLAG_LOWPASS) != 0, (char*)workspace, st,
                  hook_for(ctx, cfg));
  r = check_hip("psm_backward launch");
  if (r != PSM_OK) return r;
  g_err.clear();
  return PSM_OK;
}

psm_status read_stats_impl(psm_ctx* ctx, const void* workspace, int64_t n, const psm_camera* cams, int32_t n_cams,
                           const psm_config* cfg, int32_t c, int64_t pair_capacity, psm_stats* out, void* stream) {
  if (!ctx || !out) return fail(PSM_ERR_INVALID_ARG, "ctx and out are required");
  psm_status r = validate_common(cams, n_cams, cfg, n, c, pair_capacity);
  if (r != PSM_OK) return r;
  const Layout L = make_layout(cam_table(cams, n_cams, n, cfg), cfg->k, c, pair_capacity);
  if (!workspace) return fail(PSM_ERR_INVALID_ARG, "workspace is required");
  DeviceGuard dg(ctx->device);
  hipStream_t st = (hipStream_t)stream;
  uint32_t h[kStWords];
  r = read_status(L, workspace, h, st);
  if (r != PSM_OK) return r;
  r = check_signature(L, h);
  if (r != PSM_OK) return r;
  const bool topk = cfg->blend == PSM_BLEND_TOPK;
  if (topk) {
    launch_count_selected(L, (char*)workspace, st);
    r = check_hip("psm_read_stats selection count");
    if (r != PSM_OK) return r;
    r = read_status(L, workspace, h, st);
    if (r != PSM_OK) return r;
  }
  std::memset(out, 0, sizeof(*out));
  out->n = n;
  out->visible = h[kStVisible];
  for (int i = 0; i < 5; ++i) out->culled[i] = i == 0 ? 0 : h[kStCull + i];
  out->pairs = h[kStP];
  out->pairs_required = (int64_t)((uint64_t)h[kStReqLo] | ((uint64_t)h[kStReqHi] << 32));
  out->pair_capacity = pair_capacity;
  out->tiles = L.tiles;
  out->pairs_walked = word64(h, kStWalked);
  out->contributors = word64(h, kStBlended);
  out->bwd_entries = word64(h, kStBwdEntries);
  out->selected_unique = topk ? word64(h, kStUnique) : -1;
  out->selections = topk ? word64(h, kStSelected) : -1;
  out->selected_pairs = topk ? word64(h, kStSelPairs) : -1;
  return PSM_OK;
}

psm_status read_pairs_impl(psm_ctx* ctx, const void* workspace, int64_t n, const psm_camera* cams, int32_t n_cams,
                           const psm_config* cfg, int32_t c, int64_t pair_capacity, int32_t* tile_out,
                           int32_t* id_out, int64_t cap, int32_t* cull_out, uint32_t* depth_bits_out,
                           int32_t* count_out, int64_t* pairs_out, void* stream) {
  if (!ctx) return fail(PSM_ERR_INVALID_ARG, "ctx is null");
  psm_status r = validate_common(cams, n_cams, cfg, n, c, pair_capacity);
  if (r != PSM_OK) return r;
  if (!workspace) return fail(PSM_ERR_INVALID_ARG, "workspace is required");
  const Layout L = make_layout(cam_table(cams, n_cams, n, cfg), cfg->k, c, pair_capacity);
  DeviceGuard dg(ctx->device);
  hipStream_t st = (hipStream_t)stream;
  const char* ws = (const char*)workspace;
  uint32_t h[kStWords];
  r = read_status(L, workspace, h, st);
  if (r != PSM_OK) return r;
  r = check_signature(L, h);
  if (r != PSM_OK) return r;
  const int64_t P = h[kStP];
  if (pairs_out) *pairs_out = P;
  const int64_t m = std::min<int64_t>(P, cap);
  if (m > 0 && tile_out) (void)hipMemcpyAsync(tile_out, ws + L.ptile0, m * 4, hipMemcpyDeviceToDevice, st);
  if (m > 0 && id_out) (void)hipMemcpyAsync(id_out, ws + L.pid, m * 4, hipMemcpyDeviceToDevice, st);
  launch_export_keys(L, (char*)workspace, cull_out, depth_bits_out, count_out, st);
  r = check_hip("psm_read_pairs");
  if (r != PSM_OK) return r;
  if (hipStreamSynchronize(st) != hipSuccess) return fail(PSM_ERR_HIP, "psm_read_pairs sync");
  return PSM_OK;
}

psm_status read_selection_impl(psm_ctx* ctx, const void* workspace, int64_t n, const psm_camera* cams,
                               int32_t n_cams, const psm_config* cfg, int32_t c, int64_t pair_capacity,
                               int32_t* sel_id_out, float* sel_w_out, int32_t* n_last_out, float* t_final_out,
                               void* stream) {
  if (!ctx) return fail(PSM_ERR_INVALID_ARG, "ctx is null");
  psm_status r = validate_common(cams, n_cams, cfg, n, c, pair_capacity);
  if (r != PSM_OK) return r;
  if (!workspace) return fail(PSM_ERR_INVALID_ARG, "workspace is required");
  const CamTable ct = cam_table(cams, n_cams, n, cfg);
  const Layout L = make_layout(ct, cfg->k, c, pair_capacity);
  DeviceGuard dg(ctx->device);
  uint32_t h[kStWords];
  r = read_status(L, workspace, h, (hipStream_t)stream);
  if (r != PSM_OK) return r;
  r = check_signature(L, h);
  if (r != PSM_OK) return r;
  launch_export_selection(L, ct, (char*)workspace, cfg->blend == PSM_BLEND_TOPK ? sel_id_out : nullptr,
                          cfg->blend == PSM_BLEND_TOPK ? sel_w_out : nullptr, n_last_out, t_final_out,
                          (hipStream_t)stream);
  return check_hip("psm_read_selection");
}

std::string tune_key(const psm_surfels* s, const psm_camera* cams, int32_t n_cams, const psm_config* cfg,
                     bool bwd) {
  std::string k = std::to_string(s->n) + "|" + std::to_string(s->c) + "+" + std::to_string(s->c_ext) + "|" + std::to_string(s->feat_dtype) + "|" +
                  std::to_string(cfg->k) + "|" + std::to_string(cfg->tile_mode) + "|" + std::to_string(cfg->blend) +
                  "|" + (bwd ? "b" : "f");
  for (int b = 0; b < n_cams; ++b) k += "|" + std::to_string(cams[b].width) + "x" + std::to_string(cams[b].height);
  return k;
}

// No C++ exception crosses the C ABI: a host allocation failure or any other
// exception inside an entry point becomes an error status and message.
psm_status fail_noexcept(psm_status s, const char* where, const char* msg) noexcept {
  try {
    g_err = std::string(where) + ": " + msg;
  } catch (...) {
    g_err.clear();
  }
  return s;
}

template <class F>
psm_status guarded(const char* where, F&& body) noexcept {
  try {
    return body();
  } catch (const std::bad_alloc&) {
    return fail_noexcept(PSM_ERR_HIP, where, "host memory allocation failed");
  } catch (...) {
    return fail_noexcept(PSM_ERR_HIP, where, "unexpected internal exception");
  }
}

}  // namespace

extern "C" {

const char* psm_last_error(void) { return g_err.c_str(); }

const char* psm_version(void) { return "psm 0.3 (gfx950)"; }

psm_status psm_create(psm_ctx** ctx_out, int device) {
  return guarded("psm_create", [&]() -> psm_status {
    if (!ctx_out) return fail(PSM_ERR_INVALID_ARG, "ctx_out is null");
    *ctx_out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
      return fail(PSM_ERR_HIP, "no usable HIP device " + std::to_string(device));
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return fail(PSM_ERR_HIP, "hipGetDeviceProperties failed");
    void* scr = nullptr;
    {
      DeviceGuard dg(device);
      if (!dg.ok) return fail(PSM_ERR_HIP, "hipSetDevice failed");
      const hipError_t e = fetch_scratch(device, &scr);
      if (e != hipSuccess)
        return fail(PSM_ERR_HIP, std::string("static workspace address: ") + hipGetErrorString(e));
    }
    psm_ctx* c = new psm_ctx;
    c->device = device;
    c->cu_count = prop.multiProcessorCount;
    c->scratch = scr;
    *ctx_out = c;
    g_err.clear();
    return PSM_OK;
  });
}

void psm_destroy(psm_ctx* ctx) { delete ctx; }

psm_status psm_workspace_size_batch(int64_t n, const psm_camera* cams, int32_t n_cams, const psm_config* cfg,
                                    int32_t c, int64_t pair_capacity, size_t* bytes_out) {
  return guarded("psm_workspace_size_batch", [&]() -> psm_status {
    if (!bytes_out) return fail(PSM_ERR_INVALID_ARG, "bytes_out is null");
    psm_status s = validate_common(cams, n_cams, cfg, n, c, pair_capacity);
    if (s != PSM_OK) return s;
    *bytes_out = make_layout(cam_table(cams, n_cams, n, cfg), cfg->k, c, pair_capacity).total;
    return PSM_OK;
  });
}

psm_status psm_workspace_size(int64_t n, const psm_camera* cam, const psm_config* cfg, int32_t c,
                              int64_t pair_capacity, size_t* bytes_out) {
  return guarded("psm_workspace_size", [&]() -> psm_status {
    return psm_workspace_size_batch(n, cam, 1, cfg, c, pair_capacity, bytes_out);
  });
}

psm_status psm_forward_batch(psm_ctx* ctx, const psm_surfels* s, const psm_camera* cams, int32_t n_cams,
                             const psm_config* cfg, void* workspace, size_t workspace_bytes, int64_t pair_capacity,
                             psm_images* out, void* stream) {
  return guarded("psm_forward_batch", [&]() -> psm_status {
    return forward_impl(ctx, s, cams, n_cams, cfg, workspace, workspace_bytes, pair_capacity, out, stream);
  });
}

psm_status psm_forward(psm_ctx* ctx, const psm_surfels* s, const psm_camera* cam, const psm_config* cfg,
                       void* workspace, size_t workspace_bytes, int64_t pair_capacity, psm_images* out,
                       void* stream) {
  return guarded("psm_forward", [&]() -> psm_status {
    return forward_impl(ctx, s, cam, 1, cfg, workspace, workspace_bytes, pair_capacity, out, stream);
  });
}

psm_status psm_backward_batch(psm_ctx* ctx, const psm_surfels* s, const psm_camera* cams, int32_t n_cams,
                              const psm_config* cfg, void* workspace, size_t workspace_bytes, int64_t pair_capacity,
                              const psm_image_grads* grad_out, psm_grads* grads, void* stream) {
  return guarded("psm_backward_batch", [&]() -> psm_status {
    return backward_impl(ctx, s, cams, n_cams, cfg, workspace, workspace_bytes, pair_capacity, grad_out, grads,
                         stream);
  });
}

psm_status psm_backward(psm_ctx* ctx, const psm_surfels* s, const psm_camera* cam, const psm_config* cfg,
                        void* workspace, size_t workspace_bytes, int64_t pair_capacity,
                        const psm_image_grads* grad_out, psm_grads* grads, void* stream) {
  return guarded("psm_backward", [&]() -> psm_status {
    return backward_impl(ctx, s, cam, 1, cfg, workspace, workspace_bytes, pair_capacity, grad_out, grads, stream);
  });
}

psm_status psm_read_stats_batch(psm_ctx* ctx, const void* workspace, int64_t n, const psm_camera* cams,
                                int32_t n_cams, const psm_config* cfg, int32_t c, int64_t pair_capacity,
                                psm_stats* out, void* stream) {
  return guarded("psm_read_stats_batch", [&]() -> psm_status {
    return read_stats_impl(ctx, workspace, n, cams, n_cams, cfg, c, pair_capacity, out, stream);
  });
}

psm_status psm_read_stats(psm_ctx* ctx, const void* workspace, int64_t n, const psm_camera* cam,
                          const psm_config* cfg, int32_t c, int64_t pair_capacity, psm_stats* out, void* stream) {
  return guarded("psm_read_stats", [&]() -> psm_status {
    return read_stats_impl(ctx, workspace, n, cam, 1, cfg, c, pair_capacity, out, stream);
  });
}

psm_status psm_read_pairs_batch(psm_ctx* ctx, const void* workspace, int64_t n, const psm_camera* cams,
                                int32_t n_cams, const psm_config* cfg, int32_t c, int64_t pair_capacity,
                                int32_t* tile_out, int32_t* id_out, int64_t cap, int32_t* cull_out,
                                uint32_t* depth_bits_out, int32_t* count_out, int64_t* pairs_out, void* stream) {
  return guarded("psm_read_pairs_batch", [&]() -> psm_status {
    return read_pairs_impl(ctx, workspace, n, cams, n_cams, cfg, c, pair_capacity, tile_out, id_out, cap, cull_out,
                           depth_bits_out, count_out, pairs_out, stream);
  });
}

psm_status psm_read_pairs(psm_ctx* ctx, const void* workspace, int64_t n, const psm_camera* cam,
                          const psm_config* cfg, int32_t c, int64_t pair_capacity, int32_t* tile_out,
                          int32_t* id_out, int64_t cap, int32_t* cull_out, uint32_t* depth_bits_out,
                          int32_t* count_out, int64_t* pairs_out, void* stream) {
  return guarded("psm_read_pairs", [&]() -> psm_status {
    return read_pairs_impl(ctx, workspace, n, cam, 1, cfg, c, pair_capacity, tile_out, id_out, cap, cull_out,
                           depth_bits_out, count_out, pairs_out, stream);
  });
}

psm_status psm_read_selection_batch(psm_ctx* ctx, const void* workspace, int64_t n, const psm_camera* cams,
                                    int32_t n_cams, const psm_config* cfg, int32_t c, int64_t pair_capacity,
                                    int32_t* sel_id_out, float* sel_w_out, int32_t* n_last_out, float* t_final_out,
                                    void* stream) {
  return guarded("psm_read_selection_batch", [&]() -> psm_status {
    return read_selection_impl(ctx, workspace, n, cams, n_cams, cfg, c, pair_capacity, sel_id_out, sel_w_out,
                               n_last_out, t_final_out, stream);
  });
}

psm_status psm_read_selection(psm_ctx* ctx, const void* workspace, int64_t n, const psm_camera* cam,
                              const psm_config* cfg, int32_t c, int64_t pair_capacity, int32_t* sel_id_out,
                              float* sel_w_out, int32_t* n_last_out, float* t_final_out, void* stream) {
  return guarded("psm_read_selection", [&]() -> psm_status {
    return read_selection_impl(ctx, workspace, n, cam, 1, cfg, c, pair_capacity, sel_id_out, sel_w_out, n_last_out,
                               t_final_out, stream);
  });
}

psm_status psm_autotune(psm_ctx* ctx, const psm_surfels* s, const psm_camera* cams, int32_t n_cams,
                        psm_config* cfg, void* workspace, size_t workspace_bytes, int64_t pair_capacity,
                        psm_images* out, const psm_image_grads* grad_out, psm_grads* grads, int32_t reps,
                        double* best_ms_out, void* stream) {
  return guarded("psm_autotune", [&]() -> psm_status {
    if (!ctx || !cfg || !out) return fail(PSM_ERR_INVALID_ARG, "ctx, cfg and out are required");
    if (reps < 1 || reps > 1000) return fail(PSM_ERR_INVALID_ARG, "reps must be in [1, 1000]");
    psm_status r = validate_surfels(s);
    if (r != PSM_OK) return r;
    r = validate_common(cams, n_cams, cfg, s->n, feat_channels(s), pair_capacity);
    if (r != PSM_OK) return r;
    const bool bwd = grads != nullptr;
    if (bwd && !grad_out) return fail(PSM_ERR_INVALID_ARG, "grad_out is required with grads");
    const std::string key = tune_key(s, cams, n_cams, cfg, bwd);
    auto apply = [&](const Tuning& tu, int tw) {
      cfg->schedule = tu.sched;
      cfg->bwd_schedule = tu.sched_bwd;
      cfg->blend_pass = tu.blend_pass;
      cfg->bwd_pass = tu.bwd_pass;
      cfg->tile_w = tw;
    };
    for (const TuneKey& t : ctx->tuned) {
      if (t.key == key) {
        apply(t.tu, t.tile_w);
        if (best_ms_out) *best_ms_out = t.ms;
        return PSM_OK;
      }
    }
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return fail(PSM_ERR_HIP, "hipSetDevice failed");
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
      return fail(PSM_ERR_HIP, "hipEventCreate failed");
    // Median time of one candidate; usable = false when its layout does not
    // fit the workspace or its pairs overflow the capacity (the candidate is
    // then left out, the error is not the caller's).
    auto time_cand = [&](const Tuning& tu, int tw, double& med, bool& usable) -> psm_status {
      psm_config c2 = *cfg;
      c2.schedule = tu.sched;
      c2.bwd_schedule = tu.sched_bwd;
      c2.blend_pass = tu.blend_pass;
      c2.bwd_pass = tu.bwd_pass;
      c2.tile_w = tw;
      c2.flags = (cfg->flags | PSM_FLAG_NO_SYNC) & ~PSM_FLAG_PROFILE;
      const Layout L = make_layout(cam_table(cams, n_cams, s->n, &c2), c2.k, feat_channels(s), pair_capacity);
      usable = L.total <= workspace_bytes;
      if (!usable) return PSM_OK;
      std::vector<double> ts;
      for (int it = 0; it <= reps; ++it) {
        (void)hipEventRecord(e0, st);
        psm_status res = forward_impl(ctx, s, cams, n_cams, &c2, workspace, workspace_bytes, pair_capacity, out, stream);
        if (res == PSM_OK && bwd)
          res = backward_impl(ctx, s, cams, n_cams, &c2, workspace, workspace_bytes, pair_capacity, grad_out, grads,
                              stream);
        if (res != PSM_OK) return res;
        (void)hipEventRecord(e1, st);
        float ms = 0.0f;
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
          return fail(PSM_ERR_HIP, "autotune timing failed");
        if (it > 0) ts.push_back(ms);
      }
      uint32_t h[kStWords];
      psm_status res = read_status(L, workspace, h, st);
      if (res != PSM_OK) return res;
      usable = h[kStOverflow] == 0;
      std::sort(ts.begin(), ts.end());
      med = ts[ts.size() / 2];
      return PSM_OK;
    };
    const bool feat = feat_channels(s) > 0 && cfg->blend == PSM_BLEND_TOPK;
    // dense blend with a backward: the pass width picks the feature contraction's unit
    const bool dense_bwd = bwd && feat_channels(s) > 0 && cfg->blend == PSM_BLEND_FULL;
    Tuning best{kSchedPersistent, bwd ? kSchedPersistent : 0, 32, 16};
    int best_tw = cfg->tile_w == 0 ? kTileDefault : cfg->tile_w;
    double best_ms = 1e300;
    psm_status res = PSM_OK;
    // stage 1: the tile shape, with persistent schedules and the default passes
    for (int tw : {16, 8, 32, 64}) {
      double med = 0.0;
      bool usable = false;
      res = time_cand(best, tw, med, usable);
      if (res != PSM_OK) break;
      if (usable && med < best_ms) {
        best_ms = med;
        best_tw = tw;
      }
    }
    // stage 2: schedules and pass widths at that shape
    if (res == PSM_OK) {
      const Tuning base = best;
      best_ms = 1e300;
      for (int sched = 0; sched < 2 && res == PSM_OK; ++sched)
        for (int sched_bwd = 0; sched_bwd < 2 && res == PSM_OK; ++sched_bwd)
          for (int bp : {16, 32})
            for (int gp : {16, 32}) {
              if (res != PSM_OK) break;
              if (!bwd && sched_bwd != 0) continue;
              if (!feat && bp != 32) continue;
              if (!feat && !dense_bwd && gp != 16) continue;
              if (feat && !bwd && gp != 16) continue;
              const Tuning tu{sched, sched_bwd, bp, gp};
              double med = 0.0;
              bool usable = false;
              res = time_cand(tu, best_tw, med, usable);
              if (res == PSM_OK && usable && med < best_ms) {
                best_ms = med;
                best = tu;
              }
            }
      if (res == PSM_OK && best_ms == 1e300) best = base;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (res != PSM_OK) return res;
    if (best_ms == 1e300)
      return fail(PSM_ERR_CAPACITY, "psm_autotune: no candidate fits the workspace and its pair capacity");
    ctx->tuned.push_back(TuneKey{key, best, best_tw, best_ms});
    apply(best, best_tw);
    if (best_ms_out) *best_ms_out = best_ms;
    g_err.clear();
    return PSM_OK;
  });
}

}  // extern "C"

namespace {

psm_status validate_queries(int64_t n, const psm_queries* q, int32_t f_dtype) {
  if (!q) return fail(PSM_ERR_INVALID_ARG, "queries are required");
  if (n < 0 || n > 0x7FFFFFFFLL) return fail(PSM_ERR_INVALID_ARG, "n must be in [0, 2^31)");
  if (q->n_q < 1 || q->n_q > 256) return fail(PSM_ERR_INVALID_ARG, "n_q must be in [1, 256]");
  if (q->c < 4 || q->c > 512 || q->c % 4 != 0) return fail(PSM_ERR_INVALID_ARG, "c must be in [4, 512], c % 4 == 0");
  if (f_dtype < 0 || f_dtype > 2) return fail(PSM_ERR_INVALID_ARG, "bad f_dtype");
  if (!q->feat || !q->mean || !q->prec) return fail(PSM_ERR_INVALID_ARG, "null query array");
  return PSM_OK;
}

LabelQueries label_queries(const psm_queries* q) { return LabelQueries{q->n_q, q->c, q->feat, q->mean, q->prec}; }

}  // namespace

extern "C" {

psm_status psm_instance_labels(psm_ctx* ctx, int64_t n, const float* means, const void* f_ins, int32_t f_dtype,
                               const psm_queries* q, float* labels, int32_t ld, void* stream) {
  return guarded("psm_instance_labels", [&]() -> psm_status {
    if (!ctx) return fail(PSM_ERR_INVALID_ARG, "ctx is null");
    psm_status r = validate_queries(n, q, f_dtype);
    if (r != PSM_OK) return r;
    if (ld < ((q->n_q + 7) & ~7)) return fail(PSM_ERR_INVALID_ARG, "ld must be >= round_up(n_q, 8)");
    if (n > 0 && (!means || !f_ins || !labels)) return fail(PSM_ERR_INVALID_ARG, "null surfel or label array");
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return fail(PSM_ERR_HIP, "hipSetDevice failed");
    launch_labels(n, means, f_ins, f_dtype, label_queries(q), labels, ld, (hipStream_t)stream);
    r = check_hip("psm_instance_labels launch");
    if (r != PSM_OK) return r;
    g_err.clear();
    return PSM_OK;
  });
}

psm_status psm_instance_labels_workspace_size(int64_t n, const psm_queries* q, size_t* bytes_out) {
  return guarded("psm_instance_labels_workspace_size", [&]() -> psm_status {
    if (!bytes_out) return fail(PSM_ERR_INVALID_ARG, "bytes_out is null");
    psm_status r = validate_queries(n, q, 0);
    if (r != PSM_OK) return r;
    *bytes_out = label_workspace_bytes(n, q->n_q, q->c);
    return PSM_OK;
  });
}

psm_status psm_instance_labels_backward(psm_ctx* ctx, int64_t n, const float* means, const void* f_ins,
                                        int32_t f_dtype, const psm_queries* q, const float* d_labels, int32_t ld,
                                        void* workspace, size_t workspace_bytes, float* d_means, float* d_f_ins,
                                        float* d_qfeat, float* d_qmean, float* d_qprec, void* stream) {
  return guarded("psm_instance_labels_backward", [&]() -> psm_status {
    if (!ctx) return fail(PSM_ERR_INVALID_ARG, "ctx is null");
    psm_status r = validate_queries(n, q, f_dtype);
    if (r != PSM_OK) return r;
    if (ld < ((q->n_q + 7) & ~7)) return fail(PSM_ERR_INVALID_ARG, "ld must be >= round_up(n_q, 8)");
    if (n > 0 && (!means || !f_ins || !d_labels || !d_means || !d_f_ins))
      return fail(PSM_ERR_INVALID_ARG, "null surfel-side array");
    if (!d_qfeat || !d_qmean || !d_qprec) return fail(PSM_ERR_INVALID_ARG, "null query gradient array");
    if (!workspace || reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
      return fail(PSM_ERR_INVALID_ARG, "workspace must be non-null and 256-byte aligned");
    if (workspace_bytes < label_workspace_bytes(n, q->n_q, q->c))
      return fail(PSM_ERR_INVALID_ARG, "workspace too small");
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return fail(PSM_ERR_HIP, "hipSetDevice failed");
    launch_labels_backward(n, means, f_ins, f_dtype, label_queries(q), d_labels, ld, (char*)workspace, d_means,
                           d_f_ins, d_qfeat, d_qmean, d_qprec, (hipStream_t)stream);
    r = check_hip("psm_instance_labels_backward launch");
    if (r != PSM_OK) return r;
    g_err.clear();
    return PSM_OK;
  });
}

// ------------------------------------------------------ frustum attention
static psm_status validate_attention(int64_t n, const psm_attention* a) {
  if (!a) return fail(PSM_ERR_INVALID_ARG, "attention description is null");
  if (n < 0 || n > 0x7FFFFFFFLL) return fail(PSM_ERR_INVALID_ARG, "n must be in [0, 2^31)");
  if (a->n_q < 1 || a->n_q > 256) return fail(PSM_ERR_INVALID_ARG, "n_q must be in [1, 256]");
  if (!attention_supported(a->c, a->d))
    return fail(PSM_ERR_UNSUPPORTED, "(c, d) must be (16,16), (32,32), (64,32) or (64,64)");
  if (a->feat_dtype < 0 || a->feat_dtype > 2) return fail(PSM_ERR_INVALID_ARG, "bad feat_dtype");
  if (!a->q || !a->wq || !a->wk || !a->wv) return fail(PSM_ERR_INVALID_ARG, "null query or projection array");
  if (n > 0 && !a->feat) return fail(PSM_ERR_INVALID_ARG, "null feature array");
  if (!(a->pos_length > 0.0f)) return fail(PSM_ERR_INVALID_ARG, "pos_length must be > 0");
  return PSM_OK;
}

static int attention_blocks(const psm_ctx* ctx) { return std::max(64, 4 * ctx->cu_count); }

psm_status psm_frustum_attention_workspace_size(psm_ctx* ctx, int64_t n, const psm_attention* a, size_t* bytes_out) {
  return guarded("psm_frustum_attention_workspace_size", [&]() -> psm_status {
    if (!ctx || !bytes_out) return fail(PSM_ERR_INVALID_ARG, "ctx and bytes_out are required");
    psm_status r = validate_attention(n, a);
    if (r != PSM_OK) return r;
    *bytes_out = attention_workspace_bytes(n, a->n_q, a->d, attention_blocks(ctx));
    return PSM_OK;
  });
}

psm_status psm_frustum_attention(psm_ctx* ctx, int64_t n, const float* means, const float* scales,
                                 const psm_camera* cam, const psm_attention* a, void* workspace,
                                 size_t workspace_bytes, float* out, uint8_t* active, void* stream) {
  return guarded("psm_frustum_attention", [&]() -> psm_status {
    if (!ctx) return fail(PSM_ERR_INVALID_ARG, "ctx is null");
    psm_status r = validate_attention(n, a);
    if (r != PSM_OK) return r;
    if (!cam) return fail(PSM_ERR_INVALID_ARG, "camera is null");
    r = validate_camera(cam);
    if (r != PSM_OK) return r;
    if (n > 0 && (!means || !scales)) return fail(PSM_ERR_INVALID_ARG, "null surfel array");
    if (!out) return fail(PSM_ERR_INVALID_ARG, "out is null");
    const int nblk = attention_blocks(ctx);
    if (!workspace || reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
      return fail(PSM_ERR_INVALID_ARG, "workspace must be non-null and 256-byte aligned");
    if (workspace_bytes < attention_workspace_bytes(n, a->n_q, a->d, nblk))
      return fail(PSM_ERR_INVALID_ARG, "workspace too small");
    if (n > 0 && reinterpret_cast<uintptr_t>(a->feat) % 16 != 0)
      return fail(PSM_ERR_INVALID_ARG, "feature array must be 16-byte aligned");
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return fail(PSM_ERR_HIP, "hipSetDevice failed");
    AttentionArgs aa{};
    aa.n = n;
    aa.means = means;
    aa.scales = scales;
    const CamTable ct = cam_table(cam, 1, n, nullptr);  // only the camera parameters are used
    aa.cam = ct.cam[0];
    aa.nq = a->n_q;
    aa.c = a->c;
    aa.d = a->d;
    aa.feat = a->feat;
    aa.feat_dtype = a->feat_dtype;
    aa.q = a->q;
    aa.wq = a->wq;
    aa.wk = a->wk;
    aa.wv = a->wv;
    aa.pos_length = a->pos_length;
    aa.nblk = nblk;
    launch_attention(aa, (char*)workspace, out, active, (hipStream_t)stream);
    r = check_hip("psm_frustum_attention launch");
    if (r != PSM_OK) return r;
    g_err.clear();
    return PSM_OK;
  });
}

// ------------------------------------------------------- geometric loss
static psm_status validate_gmm(int64_t n, const psm_gmm* g) {
  if (!g) return fail(PSM_ERR_INVALID_ARG, "gmm is null");
  if (n < 0 || n > 0x7FFFFFFFLL) return fail(PSM_ERR_INVALID_ARG, "n must be in [0, 2^31)");
  if (g->k < 1 || g->k > (1 << 20)) return fail(PSM_ERR_INVALID_ARG, "k must be in [1, 2^20]");
  if (!g->mean || !g->cov || !g->weight) return fail(PSM_ERR_INVALID_ARG, "null gmm array");
  return PSM_OK;
}

psm_status psm_geometry_loss_workspace_size(int64_t n, const psm_gmm* g, size_t* bytes_out) {
  return guarded("psm_geometry_loss_workspace_size", [&]() -> psm_status {
    if (!bytes_out) return fail(PSM_ERR_INVALID_ARG, "bytes_out is null");
    psm_status r = validate_gmm(n, g);
    if (r != PSM_OK) return r;
    *bytes_out = geometry_workspace_bytes(n, g->k);
    return PSM_OK;
  });
}

psm_status psm_geometry_loss(psm_ctx* ctx, int64_t n, const float* means, const float* scales, const float* quats,
                             const psm_gmm* g, float lambda_n, void* workspace, size_t workspace_bytes,
                             double* losses, int32_t* assign, float* d_means, float* d_scales, float* d_quats,
                             void* stream) {
  return guarded("psm_geometry_loss", [&]() -> psm_status {
    if (!ctx) return fail(PSM_ERR_INVALID_ARG, "ctx is null");
    psm_status r = validate_gmm(n, g);
    if (r != PSM_OK) return r;
    if (!losses) return fail(PSM_ERR_INVALID_ARG, "losses is null");
    if (n > 0 && (!means || !scales || !quats || !d_means || !d_scales || !d_quats))
      return fail(PSM_ERR_INVALID_ARG, "null surfel or gradient array");
    if (!workspace || reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
      return fail(PSM_ERR_INVALID_ARG, "workspace must be non-null and 256-byte aligned");
    if (workspace_bytes < geometry_workspace_bytes(n, g->k)) return fail(PSM_ERR_INVALID_ARG, "workspace too small");
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return fail(PSM_ERR_HIP, "hipSetDevice failed");
    GeometryArgs a{n, means, scales, quats, g->k, g->mean, g->cov, g->weight, lambda_n, losses, assign,
                   d_means, d_scales, d_quats};
    launch_geometry_loss(a, (char*)workspace, (hipStream_t)stream);
    r = check_hip("psm_geometry_loss launch");
    if (r != PSM_OK) return r;
    g_err.clear();
    return PSM_OK;
  });
}

psm_status psm_forward_static(psm_ctx* ctx, const psm_surfels* s, const psm_camera* cam, const psm_config* cfg,
                              int64_t pair_capacity, psm_images* out, void* stream) {
  return guarded("psm_forward_static", [&]() -> psm_status {
    if (!ctx || !ctx->scratch) return fail(PSM_ERR_INVALID_ARG, "ctx is null or has no static workspace");
    if (!cam || !cfg) return fail(PSM_ERR_INVALID_ARG, "camera and config are required");
    if (pair_capacity < -1) return fail(PSM_ERR_INVALID_ARG, "pair_capacity must be -1 or >= 0");
    psm_status r = validate_surfels(s);
    if (r != PSM_OK) return r;
    r = validate_common(cam, 1, cfg, s->n, feat_channels(s), pair_capacity < 0 ? 0 : pair_capacity);
    if (r != PSM_OK) return r;
    const CamTable ct = cam_table(cam, 1, s->n, cfg);
    const size_t limit = PSM_STATIC_WORKSPACE_BYTES;
    const size_t base = make_layout(ct, cfg->k, feat_channels(s), 0).total;
    if (base > limit)
      return fail(PSM_ERR_INVALID_ARG, "psm_forward_static: n, image size, k and c need " + std::to_string(base) +
                                           " bytes of workspace before any pair; the static workspace holds " +
                                           std::to_string(limit));
    int64_t cap = pair_capacity;
    if (cap < 0) {  // the largest capacity that fits (the layout grows with it)
      int64_t lo = 0, hi = (int64_t)1 << 31;
      while (hi - lo > 1) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (make_layout(ct, cfg->k, feat_channels(s), mid).total <= limit) lo = mid;
        else hi = mid;
      }
      cap = lo;
    } else if (make_layout(ct, cfg->k, feat_channels(s), cap).total > limit) {
      return fail(PSM_ERR_INVALID_ARG, "psm_forward_static: pair capacity " + std::to_string(cap) + " needs " +
                                           std::to_string(make_layout(ct, cfg->k, feat_channels(s), cap).total) +
                                           " bytes of workspace; the static workspace holds " + std::to_string(limit));
    }
    psm_config c2 = *cfg;
    c2.flags &= ~PSM_FLAG_PROFILE;  // stage timing creates events
    return forward_impl(ctx, s, cam, 1, &c2, ctx->scratch, limit, cap, out, stream);
  });
}

psm_status psm_profile_read(psm_ctx* ctx, int32_t stage, const char** name_out, double* total_ms_out,
                            int64_t* calls_out) {
  return guarded("psm_profile_read", [&]() -> psm_status {
    if (!ctx) return fail(PSM_ERR_INVALID_ARG, "ctx is null");
    if (stage < 0 || stage >= kNumStages) return fail(PSM_ERR_INVALID_ARG, "stage out of range");
    DeviceGuard dg(ctx->device);
    if (!ctx->prof.collect()) return fail(PSM_ERR_HIP, "profile events could not be read");
    if (name_out) *name_out = kStageNames[stage];
    if (total_ms_out) *total_ms_out = ctx->prof.total_ms[stage];
    if (calls_out) *calls_out = ctx->prof.calls[stage];
    return PSM_OK;
  });
}

psm_status psm_profile_reset(psm_ctx* ctx) {
  return guarded("psm_profile_reset", [&]() -> psm_status {
    if (!ctx) return fail(PSM_ERR_INVALID_ARG, "ctx is null");
    DeviceGuard dg(ctx->device);
    const bool ok = ctx->prof.collect();
    for (int s = 0; s < kNumStages; ++s) {
      ctx->prof.total_ms[s] = 0.0;
      ctx->prof.calls[s] = 0;
    }
    return ok ? PSM_OK : fail(PSM_ERR_HIP, "profile events could not be read");
  });
}

}  // extern "C"
