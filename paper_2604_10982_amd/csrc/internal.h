// Host-side launch wrappers shared between the kernel translation units and
// the C ABI (api.cpp).  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "common.h"

namespace psm {

// feat holds channels [0, ca) in the storage dtype, feat_ext (FP32, may be
// null) channels [ca, c); c is the rendered feature width.
struct SurfelArgs {
  int64_t n;
  const float *means, *scales, *quats, *opacity, *rgb;
  const void* feat;
  int c, dtype;
  const float* feat_ext;
  int ca;
};

template <typename FT>
inline FeatSrc<FT> feat_src(const SurfelArgs& s) {
  return FeatSrc<FT>{(const FT*)s.feat, s.feat_ext, s.ca, s.c - s.ca};
}

struct ImageArgs {
  float *rgb, *depth, *normal, *alpha, *feat;
};

struct ImageGradArgs {
  const float *rgb, *depth, *normal, *alpha, *feat;
};

// feat: [n][ca] FP32, feat_ext: [n][c - ca] FP32 (the split of SurfelArgs)
struct GradArgs {
  float *means, *scales, *quats, *opacity, *rgb, *feat, *feat_ext;
};

// Stage timing hook (events are recorded by the C ABI layer).
enum Stage : int {
  kStagePreprocess = 0, kStageDepthSort, kStageScan, kStageEmit, kStagePairSort, kStageRanges, kStageWalk,
  kStageBlend, kStageBwdFeature, kStageBwdWalk, kStageBwdPreprocess, kStageFill, kNumStages
};
struct ProfHook {
  void* self = nullptr;
  void (*mark)(void* self, int stage, int is_end, hipStream_t st) = nullptr;
  void begin(int s, hipStream_t st) const { if (mark) mark(self, s, 0, st); }
  void end(int s, hipStream_t st) const { if (mark) mark(self, s, 1, st); }
};

// Launch choices the autotuner searches (all give identical results).
struct Tuning {
  int sched;       // forward tile kernels: kSchedGrid or kSchedPersistent
  int sched_bwd;   // backward tile kernels
  int blend_pass;  // feature channels per Top-K blend pass: 16 or 32
  int bwd_pass;    // feature channels per feature-backward pass: 8 or 16
};
enum : int { kSchedGrid = 0, kSchedPersistent = 1 };

// keystage.hip
void launch_fill_u32(void* p, uint32_t v, int64_t count, hipStream_t st);
void launch_init_status(uint32_t* status, const Layout& L, hipStream_t st);
void launch_preprocess(const SurfelArgs& s, const CamTable& ct, int mode, bool opacity_foot, bool lowpass,
                       const Layout& L,
                       char* ws, hipStream_t st);
void launch_scan_counts(const Layout& L, char* ws, hipStream_t st);
void launch_emit(const CamTable& ct, int mode, const Layout& L, char* ws, hipStream_t st);
void launch_ranges(const Layout& L, char* ws, hipStream_t st);
void launch_tile_order(const Layout& L, char* ws, hipStream_t st);
void launch_export_keys(const Layout& L, char* ws, int32_t* cull, uint32_t* depth, int32_t* count, hipStream_t st);

// sort.hip: stable LSD radix sort of (key, value) pairs on bits [0, bits) of
// the key, n read from *n_dev, at most cap_n elements.  Uses an even number of
// passes, so the result ends in (k0, v0); (k1, v1) is scratch.
void radix_sort_pairs(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, const uint32_t* n_dev,
                      int64_t cap_n, int bits, uint32_t* hist, int64_t nb_max, hipStream_t st);

// Grid of a per-tile kernel: one block per tile, or (persistent) enough
// blocks to fill the device once.
int tile_grid(const Layout& L, int sched, const void* kernel, size_t dyn_lds);

// Work queue of a per-tile kernel (work order sorted by the forward; queue
// heads zeroed before each use).
inline TileQueue tile_queue(const Layout& L, int sched, char* ws, int q) {
  TileQueue t;
  t.tiles = (int)L.tiles;
  t.order = sched == kSchedPersistent ? (const uint32_t*)(ws + L.torder0) : nullptr;
  t.head = (uint32_t*)(ws + L.status) + kStQueue + q;
  return t;
}

// raster_fwd.hip
void launch_walk(const Layout& L, const CamTable& ct, int blend, const Tuning& tu, const ImageArgs& out,
                 bool feat_only, bool lowpass, char* ws, hipStream_t st);
void launch_feature_blend(const SurfelArgs& s, const Layout& L, const CamTable& ct, int blend, const Tuning& tu,
                          float* out_feat, bool renorm, bool lowpass, char* ws, hipStream_t st);
void launch_export_selection(const Layout& L, const CamTable& ct, char* ws, int32_t* sel_id, float* sel_w,
                             int32_t* n_last, float* t_final, hipStream_t st);
// Counts the distinct selected virtual surfels and the (pixel, slot)
// selections of the last Top-K forward into the status words.
void launch_count_selected(const Layout& L, char* ws, hipStream_t st);

// labels.hip: instance labels of surfels from localized queries
struct LabelQueries {
  int nq, c;
  const float *feat, *mean, *prec;  // [nq][c], [nq][3], [nq][6]
};
inline int pow2_ge_host(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}
int label_blocks16(int nq);
int64_t label_segments(int64_t n);
size_t label_workspace_bytes(int64_t n, int nq, int c);
void launch_labels(int64_t n, const float* means, const void* fg, int dtype, const LabelQueries& q, float* out,
                   int ld, hipStream_t st);
void launch_labels_backward(int64_t n, const float* means, const void* fg, int dtype, const LabelQueries& q,
                            const float* dl, int ld, char* ws, float* d_means, float* d_fg, float* d_qfeat,
                            float* d_qmean, float* d_qprec, hipStream_t st);

// raster_bwd.hip
void launch_backward(const SurfelArgs& s, const CamTable& ct, int blend, const Tuning& tu, const Layout& L,
                     const ImageGradArgs& g, const GradArgs& grads, bool renorm, bool lowpass, char* ws, hipStream_t st,
                     const ProfHook& prof);

// Frustum-local cross-attention (attention.hip).
struct AttentionArgs {
  int64_t n;
  const float* means;
  const float* scales;
  CamArgs cam;
  int nq, c, d;
  const void* feat;
  int feat_dtype;
  const float *q, *wq, *wk, *wv;
  float pos_length;
  int nblk;    // attention blocks (key ranges)
  int64_t nb;  // cull blocks (set by the launcher)
};
bool attention_supported(int c, int d);
size_t attention_workspace_bytes(int64_t n, int nq, int d, int nblk);
void launch_attention(const AttentionArgs& a, char* ws, float* out, uint8_t* active_out, hipStream_t st);

// SOGMM geometric loss (geometry.hip).
struct GeometryArgs {
  int64_t n;
  const float *means, *scales, *quats;
  int k;
  const float *gmean, *gcov, *gweight;
  float lambda_n;
  double* losses;   // [2] device
  int32_t* assign;  // optional [n]
  float *d_means, *d_scales, *d_quats;
};
size_t geometry_workspace_bytes(int64_t n, int k);
void launch_geometry_loss(const GeometryArgs& a, char* ws, hipStream_t st);

}  // namespace psm
