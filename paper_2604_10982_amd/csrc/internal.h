// Host-side launch wrappers shared between the kernel translation units and
// the C ABI (api.cpp).  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "common.h"

namespace psm {

struct SurfelArgs {
  int64_t n;
  const float *means, *scales, *quats, *opacity, *rgb;
  const void* feat;
  int c, dtype;
};

struct CamArgs {
  float R[9], t[3], fx, fy, cx, cy, near_plane;
  int W, H;
};

struct ImageArgs {
  float *rgb, *depth, *normal, *alpha, *feat;
};

struct ImageGradArgs {
  const float *rgb, *depth, *normal, *alpha, *feat;
};

struct GradArgs {
  float *means, *scales, *quats, *opacity, *rgb, *feat;
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

// keystage.hip
void launch_fill_u32(void* p, uint32_t v, int64_t count, hipStream_t st);
void launch_init_status(uint32_t* status, int64_t n, hipStream_t st);
void launch_preprocess(const SurfelArgs& s, const CamArgs& c, int mode, const Layout& L, char* ws, hipStream_t st);
void launch_scan_counts(const Layout& L, char* ws, hipStream_t st);
void launch_emit(const CamArgs& c, int mode, const Layout& L, char* ws, hipStream_t st);
void launch_ranges(const Layout& L, char* ws, hipStream_t st);
void launch_export_keys(const Layout& L, char* ws, int32_t* cull, uint32_t* depth, int32_t* count, hipStream_t st);

// sort.hip: stable LSD radix sort of (key, value) pairs on bits [0, bits) of
// the key, n read from *n_dev, at most cap_n elements.  Uses an even number of
// passes, so the result ends in (k0, v0); (k1, v1) is scratch.
void radix_sort_pairs(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, const uint32_t* n_dev,
                      int64_t cap_n, int bits, uint32_t* hist, int64_t nb_max, hipStream_t st);

// raster_fwd.hip
void launch_walk(const Layout& L, const CamArgs& c, int blend, const ImageArgs& out, char* ws, hipStream_t st);
void launch_feature_blend(const SurfelArgs& s, const Layout& L, const CamArgs& c, int blend, float* out_feat,
                          char* ws, hipStream_t st);
void launch_export_selection(const Layout& L, const CamArgs& c, char* ws, int32_t* sel_id, float* sel_w,
                             int32_t* n_last, float* t_final, hipStream_t st);

// raster_bwd.hip
void launch_backward(const SurfelArgs& s, const CamArgs& c, int blend, const Layout& L, const ImageGradArgs& g,
                     const GradArgs& grads, char* ws, hipStream_t st, const ProfHook& prof);

}  // namespace psm
