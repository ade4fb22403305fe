/*
 * psm.h -- C ABI of the MI355X (gfx950) rasterizer for Psi-Map panoptic
 * surfel maps (arXiv 2604.10982).
 *
 * The library renders 2D Gaussian surfels (Sec. 3.1 of the paper: tangent
 * plane disks with kernel exp(-(u^2+v^2)/2) and alpha = o * kernel) by
 * tile-based front-to-back alpha blending (eq. (1)), with the two
 * optimisations of Sec. 5: Precise Tile Intersection (surfel->tile pairs from
 * the exact projected ellipse, eq. (17) and its exact-ellipse refinement) and
 * Top-K Hard Selection (eq. (18): only the K largest blend weights of a pixel
 * accumulate the feature channels).  A hand-written backward returns the
 * gradients of a loss with respect to every surfel parameter.
 *
 * Conventions
 *   - All pointers passed to psm_forward/psm_backward/psm_read_* are DEVICE
 *     pointers on the context's device unless stated otherwise; all work is
 *     enqueued asynchronously on `stream` (a hipStream_t passed as void*;
 *     NULL = the default stream).  The caller owns every buffer: inputs,
 *     outputs, gradients and the workspace.
 *   - Camera: OpenCV axes (x right, y down, z forward), world->camera
 *     rotation R (row-major) and translation t; pinhole intrinsics; pixel
 *     (i, j) samples the image point (i + 0.5, j + 0.5).
 *   - Surfel parameters are *activated* values: opacity in (0, 1], scales > 0;
 *     quaternions are (w, x, y, z) and are normalised inside.
 *   - Images are row-major: rgb/normal [H][W][3], depth/alpha [H][W],
 *     feat [H][W][C], all FP32.
 *   - Errors: every entry point returns a psm_status; negative values are
 *     errors and psm_last_error() returns a thread-local message.  No entry
 *     point aborts or throws: a failed host allocation or any other C++
 *     exception inside the library is caught at the entry point and returned
 *     as PSM_ERR_HIP.  NaN/Inf inputs are not checked; they propagate.
 */
#ifndef PSM_H
#define PSM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PSM_OK = 0,
  PSM_ERR_INVALID_ARG = -1,  /* null pointer, bad size, bad enum value */
  PSM_ERR_UNSUPPORTED = -2,  /* valid but not implemented (e.g. C % 8 != 0) */
  PSM_ERR_CAPACITY = -3,     /* workspace pair capacity too small; see stats.pairs_required */
  PSM_ERR_HIP = -4           /* a HIP runtime call failed; message in psm_last_error() */
} psm_status;

typedef enum { PSM_F32 = 0, PSM_F16 = 1, PSM_BF16 = 2 } psm_dtype;

/* Footprint used to build surfel->tile pairs (Sec. 5, "Precise Tile
 * Intersection").  SPHERE is the isotropic bound the paper improves on, AABB
 * is eq. (17), ELLIPSE is the exact projected-ellipse/tile test.  All three
 * are conservative for the per-pixel cutoff, so images do not depend on it. */
typedef enum { PSM_TILE_SPHERE = 0, PSM_TILE_AABB = 1, PSM_TILE_ELLIPSE = 2 } psm_tile_mode;

/* Feature blending: FULL = eq. (1) with c_i = f_i over every contributor;
 * TOPK = eq. (18), the K largest weights only.  RGB, depth, normal and alpha
 * always use the dense blend. */
typedef enum { PSM_BLEND_FULL = 0, PSM_BLEND_TOPK = 1 } psm_blend_mode;

typedef struct {
  int64_t n;            /* number of surfels, >= 0 */
  const float* means;   /* [n][3] world-space centres */
  const float* scales;  /* [n][2] tangent-plane scales (s_u, s_v) > 0 */
  const float* quats;   /* [n][4] (w, x, y, z) */
  const float* opacity; /* [n] in (0, 1] */
  const float* rgb;     /* [n][3] */
  const void* feat;     /* [n][c] row-major in feat_dtype, 16-byte aligned */
  int32_t c;            /* feature channels from feat: 0 <= c <= 1024, c % 8 == 0 */
  int32_t feat_dtype;   /* psm_dtype */
  /* Optional second feature source, FP32 [n][c_ext] row-major, 16-byte
   * aligned: channels c .. c + c_ext - 1 of every blended feature row.  Both
   * sources are gathered by the same walk and selection, so one render yields
   * e.g. the semantic map and the instance map of eq. (8) (Sec. 4.1) side by
   * side without a concatenated copy of the surfel features.  The rendered
   * feature map, and every `c` argument that sizes a workspace for these
   * surfels, has c + c_ext <= 1024 channels.  NULL and 0 for none. */
  const float* feat_ext;
  int32_t c_ext;        /* 0 <= c_ext, c_ext % 8 == 0 */
} psm_surfels;

typedef struct {
  float R[9];         /* world -> camera rotation, row-major */
  float t[3];         /* world -> camera translation */
  float fx, fy, cx, cy;
  float near_plane;   /* > 0; surfels whose cutoff disk reaches it are culled */
  int32_t width, height; /* 1..16384 */
} psm_camera;

typedef struct {
  int32_t k;          /* Top-K size, 1..32 (also sizes the saved selection) */
  int32_t tile_mode;  /* psm_tile_mode */
  int32_t blend;      /* psm_blend_mode */
  int32_t flags;      /* PSM_FLAG_* */
  /* Launch choices (results do not depend on them; psm_autotune picks them).
   * A backward must use the values of its forward. */
  int32_t schedule;   /* psm_schedule */
  int32_t blend_pass; /* feature channels per Top-K blend pass: 0 (= 32), 16 or 32 */
  int32_t bwd_pass;   /* feature channels per feature-backward pass: 0 (= 16), 16 or 32; with the dense
                       * blend it selects the backward's feature contractions: 16 vector FMAs,
                       * 32 matrix cores (the same sums in another order) */
  int32_t bwd_schedule; /* psm_schedule of the backward's tile kernels */
  /* Tile shape: tile_w x (256 / tile_w) pixels, tile_w in {8, 16, 32, 64};
   * 0 = 16 (16 x 16 tiles, Sec. 5's tile-based rasterisation).  One 256-thread
   * block owns one tile, a wave 64 / tile_w of its rows.  The pair lists
   * follow the tiles; images and the Top-K selection do not depend on the
   * shape (gradients only through the order of their sums).  The read-backs
   * and the backward must use the forward's value. */
  int32_t tile_w;
} psm_config;

/* Tile scheduling of the per-tile kernels (forward: schedule, backward:
 * bwd_schedule).  GRID: one workgroup per tile, tiles of neighbouring
 * ids kept on one XCD.  PERSISTENT: a grid that fills the device once takes
 * tiles from a work queue ordered longest lists first (the forward orders the
 * tiles when either schedule is persistent). */
typedef enum { PSM_SCHED_GRID = 0, PSM_SCHED_PERSISTENT = 1 } psm_schedule;

/* Skip the end-of-call status read-back (graph-safe; the caller checks
 * psm_read_stats later). */
#define PSM_FLAG_NO_SYNC 1
/* Record a HIP event pair around every stage on the call's stream; read the
 * accumulated stage times with psm_profile_read. */
#define PSM_FLAG_PROFILE 2
/* Opacity-aware footprint (an exact work reduction of the key stage): a pixel
 * is skipped when alpha = o exp(-rho/2) < 1/255 (Sec. 3.1), so a surfel's tile
 * footprint is the ellipse of rho <= min(9, 2 ln(255 o)) (plus a 2^-10 margin,
 * rounded up to a multiple of 2^-12) instead of rho <= 9.  Cull decisions,
 * images, selections and gradients are unchanged bit for bit; faint surfels
 * emit fewer (tile, surfel) pairs. */
#define PSM_FLAG_OPACITY_FOOTPRINT 4
/* Feature-only rendering (an exact work reduction of the forward walk): with
 * the Top-K blend and c > 0, a pixel stops walking once it holds K weights
 * and fl(0.99 T) is at most the smallest of them, since no later weight
 * alpha T' (alpha <= 0.99, T' <= T) can enter the K largest (a tie goes to
 * the earlier surfel).  The selection and the feature map equal those of the
 * full walk bit for bit; only the feature map is rendered (rgb, depth, normal
 * and alpha outputs, and their upstream gradients, must be null), and the
 * backward gives the gradients of the feature loss. */
#define PSM_FLAG_FEATURE_ONLY 8
/* Renormalised Top-K (a variant of eq. (18)): the feature map is
 * sum_sel w_k f_k / sum_sel w_k, the selected weights rescaled to sum 1 (zero
 * where nothing is selected); the backward differentiates the quotient.
 * Needs the Top-K blend and c > 0. */
#define PSM_FLAG_TOPK_RENORM 16
/* Screen-space low-pass filter (the 2D surfel splatting variant of the
 * surfel kernel, Sec. 3.1): rho = min(u^2 + v^2, 2 |x - c|^2) with c the
 * projected surfel centre in pixels; where the filter term is the smaller the
 * depth is the centre's camera depth.  The listed footprint is the union with
 * the filter's disk (radius^2 = footprint radius^2 / 2 + 1/16 px^2 about the
 * FP32 centre).  Any blend and tile mode. */
#define PSM_FLAG_LOWPASS 32

typedef struct { float *rgb, *depth, *normal, *alpha, *feat; } psm_images;
typedef struct { const float *rgb, *depth, *normal, *alpha, *feat; } psm_image_grads;
/* Gradients, FP32, shapes of the inputs (feat: [n][c] FP32 for every storage
 * dtype; feat_ext: [n][c_ext], needed only when c_ext > 0).  psm_backward
 * overwrites them (no accumulation). */
typedef struct { float *means, *scales, *quats, *opacity, *rgb, *feat, *feat_ext; } psm_grads;

typedef struct {
  int64_t n;              /* surfels */
  int64_t visible;        /* surfels surviving the cull (summed over cameras) */
  int64_t culled[5];      /* by code: 0 unused, 1 zero quaternion, 2 centre behind near,
                             3 disk reaches near plane, 4 degenerate projection */
  int64_t pairs;          /* surfel->tile pairs emitted (the sorted list length) */
  int64_t pairs_required; /* pairs the footprint asked for (> capacity on PSM_ERR_CAPACITY) */
  int64_t pair_capacity;  /* capacity the workspace was laid out for */
  int64_t tiles;          /* number of tiles of the config's shape (all cameras) */
  int64_t pairs_walked;   /* pixel x list-entry evaluations of the forward walk */
  int64_t contributors;   /* (pixel, surfel) pairs blended by the forward walk */
  int64_t bwd_entries;    /* sum over pixels of the list position one past the last contributor: the
                             list entries the backward walk must evaluate (Sec. 3.1 eq. (1) adjoint) */
  int64_t selected_unique;  /* Top-K blend: distinct (camera, surfel) pairs selected by at least one pixel
                               (the feature rows eq. (18) reads); -1 for the dense blend */
  int64_t selections;     /* Top-K blend: (pixel, slot) selections held, sum over pixels of min(K,
                             contributors); -1 for the dense blend */
  int64_t selected_pairs; /* Top-K blend: (tile, surfel) pairs selected by at least one pixel of the
                             tile (the per-tile feature rows of eq. (18) and of its adjoint); -1 for
                             the dense blend */
} psm_stats;

typedef struct psm_ctx psm_ctx;

/* Create a context bound to HIP device `device` (host memory; holds device
 * properties and the last error).  Returns PSM_ERR_HIP if the device is not
 * usable. */
psm_status psm_create(psm_ctx** ctx_out, int device);
void psm_destroy(psm_ctx* ctx);

/* Size in bytes of the workspace for n surfels, this camera and config,
 * c feature channels and room for `pair_capacity` surfel->tile pairs.  The
 * workspace holds the per-surfel records, the pair lists and sort scratch,
 * the tile ranges and the per-pixel state saved for the backward (last
 * contributor, final transmittance, Top-K positions and weights).  Pure host
 * computation; ctx may be NULL. */
psm_status psm_workspace_size(int64_t n, const psm_camera* cam, const psm_config* cfg, int32_t c,
                              int64_t pair_capacity, size_t* bytes_out);

/* Forward render (Sec. 3.1 eq. (1); Sec. 5 eqs. (17), (18)).
 * workspace: device buffer of at least psm_workspace_size(...) bytes, 256-byte
 * aligned, that must stay untouched until the matching psm_backward.
 * out: device pointers; any member may be NULL to skip that map (feat must be
 * non-NULL when c > 0 and blend is used).  Unless PSM_FLAG_NO_SYNC is set the
 * call synchronises `stream` once at the end to read the pair count and
 * returns PSM_ERR_CAPACITY when the pairs did not fit (images are then
 * invalid; re-run with a larger capacity). */
psm_status psm_forward(psm_ctx* ctx, const psm_surfels* s, const psm_camera* cam,
                       const psm_config* cfg, void* workspace, size_t workspace_bytes,
                       int64_t pair_capacity, psm_images* out, void* stream);

/* Backward of L = sum over all maps of <grad_out, image>: writes dL/d(every
 * surfel parameter) into `grads` (all members required, FP32 device arrays).
 * Uses the workspace state of the last psm_forward with the same inputs,
 * camera and config; grad_out members may be NULL (treated as zero).
 * Gradients hold the Top-K set, the contributor set and the alpha clamp
 * fixed (their a.e. derivative). */
psm_status psm_backward(psm_ctx* ctx, const psm_surfels* s, const psm_camera* cam,
                        const psm_config* cfg, void* workspace, size_t workspace_bytes,
                        int64_t pair_capacity, const psm_image_grads* grad_out, psm_grads* grads,
                        void* stream);

/* Reads the counters of the last psm_forward in this workspace into *out
 * (host memory).  For the Top-K blend it first counts the selections on
 * `stream` (two small kernels over the saved selection; a bitmap region of
 * the workspace is overwritten, nothing the backward reads), then
 * synchronises `stream`.  n, cam, cfg, c and pair_capacity must be those of
 * that forward: the forward records its workspace layout (total bytes, pair
 * capacity, tiles) in the workspace, and this call and the other read-backs
 * return PSM_ERR_INVALID_ARG, before touching anything else in the
 * workspace, when the layout they compute differs (the workspace must hold
 * at least the 256-byte status block that starts it). */
psm_status psm_read_stats(psm_ctx* ctx, const void* workspace, int64_t n, const psm_camera* cam,
                          const psm_config* cfg, int32_t c, int64_t pair_capacity, psm_stats* out,
                          void* stream);

/* Inspection of the key stage, for testing: copies (device to device, on
 * `stream`) the sorted pair list -- tile ids and surfel ids, `cap` entries at
 * most -- and per surfel the cull code, the FP32 depth-key bits and the pair
 * count.  Any output may be NULL.  *pairs_out (host) receives the list
 * length (this call synchronises `stream`). */
psm_status psm_read_pairs(psm_ctx* ctx, const void* workspace, int64_t n, const psm_camera* cam,
                          const psm_config* cfg, int32_t c, int64_t pair_capacity,
                          int32_t* tile_out, int32_t* id_out, int64_t cap, int32_t* cull_out,
                          uint32_t* depth_bits_out, int32_t* count_out, int64_t* pairs_out,
                          void* stream);

/* Inspection of the Top-K selection saved by the last forward: for every
 * pixel (row-major), K surfel ids in front-to-back order (-1 padded) and
 * their blend weights, plus the number of list entries walked and T_final.
 * Device outputs, any may be NULL. */
psm_status psm_read_selection(psm_ctx* ctx, const void* workspace, int64_t n, const psm_camera* cam,
                              const psm_config* cfg, int32_t c, int64_t pair_capacity,
                              int32_t* sel_id_out, float* sel_w_out, int32_t* n_last_out,
                              float* t_final_out, void* stream);

/* Stage timing (PSM_FLAG_PROFILE).  Stages are numbered 0 .. PSM_NUM_STAGES-1
 * (preprocess, depth_sort, count_scan, emit, pair_sort, ranges, walk,
 * feature_blend, bwd_feature, bwd_walk, bwd_reduce, fill).  psm_profile_read
 * synchronises the recorded events and returns, for `stage`, its name (static
 * string), the summed duration in ms and the number of recorded calls since
 * the last psm_profile_reset.  Events are recorded on the stream each call was
 * given. */
#define PSM_NUM_STAGES 12
psm_status psm_profile_read(psm_ctx* ctx, int32_t stage, const char** name_out, double* total_ms_out,
                            int64_t* calls_out);
psm_status psm_profile_reset(psm_ctx* ctx);

/* ------------------------------------------------------------------------
 * Forward without a caller workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments and results as psm_forward, but the
 * workspace is the library's static device array of
 * PSM_STATIC_WORKSPACE_BYTES (one per device, held from the library's load
 * until the process ends; psm_create fetches its address).  The call makes no
 * device allocation and no allocating library call.
 *   pair_capacity: -1 = the largest capacity the static workspace holds for
 *     these sizes; >= 0 = that capacity (it must fit).
 *   Sizes (n, image size, k, c, capacity) whose workspace exceeds the static
 *   array return PSM_ERR_INVALID_ARG (nothing is enqueued); more pairs than
 *   the capacity return PSM_ERR_CAPACITY as in psm_forward (unless
 *   PSM_FLAG_NO_SYNC).  PSM_FLAG_PROFILE is ignored.
 *   Every call on a device shares that device's array and leaves its state
 *   there (the forward initialises everything it reads): calls that overlap
 *   on one device (other streams, other host threads) race, and there is no
 *   backward of a static forward.
 * ------------------------------------------------------------------------ */
#define PSM_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)
psm_status psm_forward_static(psm_ctx* ctx, const psm_surfels* s, const psm_camera* cam, const psm_config* cfg,
                              int64_t pair_capacity, psm_images* out, void* stream);

/* ------------------------------------------------------------------------
 * Several cameras in one call (one launch per stage for all of them).
 * Surfel i seen by camera b is the virtual surfel v = b * n + i; every
 * camera gets its own tiles and images, and the gradients are summed over
 * the cameras (in camera order, deterministically).  Output and upstream
 * maps are the cameras' maps concatenated in camera order: camera b's map
 * starts at pixel sum_{b' < b} width_b' * height_b' (times the map's
 * channels).  1 <= n_cams <= PSM_MAX_CAMERAS and n * n_cams < 2^31.
 * Rendering camera b alone gives bit-identical images.  psm_read_pairs_batch
 * reports global tile ids (camera b's tiles follow those of the cameras
 * before it) and virtual surfel ids; its per-surfel outputs have n_cams * n
 * entries.  The single-camera entry points above are the n_cams = 1 case.
 * ------------------------------------------------------------------------ */
#define PSM_MAX_CAMERAS 8

psm_status psm_workspace_size_batch(int64_t n, const psm_camera* cams, int32_t n_cams, const psm_config* cfg,
                                    int32_t c, int64_t pair_capacity, size_t* bytes_out);
psm_status psm_forward_batch(psm_ctx* ctx, const psm_surfels* s, const psm_camera* cams, int32_t n_cams,
                             const psm_config* cfg, void* workspace, size_t workspace_bytes,
                             int64_t pair_capacity, psm_images* out, void* stream);
psm_status psm_backward_batch(psm_ctx* ctx, const psm_surfels* s, const psm_camera* cams, int32_t n_cams,
                              const psm_config* cfg, void* workspace, size_t workspace_bytes,
                              int64_t pair_capacity, const psm_image_grads* grad_out, psm_grads* grads,
                              void* stream);
psm_status psm_read_stats_batch(psm_ctx* ctx, const void* workspace, int64_t n, const psm_camera* cams,
                                int32_t n_cams, const psm_config* cfg, int32_t c, int64_t pair_capacity,
                                psm_stats* out, void* stream);
psm_status psm_read_pairs_batch(psm_ctx* ctx, const void* workspace, int64_t n, const psm_camera* cams,
                                int32_t n_cams, const psm_config* cfg, int32_t c, int64_t pair_capacity,
                                int32_t* tile_out, int32_t* id_out, int64_t cap, int32_t* cull_out,
                                uint32_t* depth_bits_out, int32_t* count_out, int64_t* pairs_out, void* stream);
psm_status psm_read_selection_batch(psm_ctx* ctx, const void* workspace, int64_t n, const psm_camera* cams,
                                    int32_t n_cams, const psm_config* cfg, int32_t c, int64_t pair_capacity,
                                    int32_t* sel_id_out, float* sel_w_out, int32_t* n_last_out,
                                    float* t_final_out, void* stream);

/* Autotuner: picks the tile shape (tile_w) and the launch choices (schedule,
 * bwd_schedule, blend_pass, bwd_pass) on these inputs by timing them --
 * forward, plus backward when grads is non-NULL -- `reps` times each after
 * one warm-up: first the four tile shapes with persistent schedules and the
 * default pass widths, then every schedule and pass width at the fastest
 * shape.  Writes the fastest into *cfg (and its median time in ms into
 * *best_ms_out when non-NULL).  A shape whose workspace layout exceeds
 * workspace_bytes, or whose pairs exceed pair_capacity, is left out (size the
 * workspace for the largest shape to have every shape timed).  The choice is
 * cached in the context per (cameras' sizes, n, c, k, dtype, modes, backward)
 * and returned without timing on later calls.  Overwrites the outputs, the
 * gradients and the workspace; synchronises `stream` (not for use under
 * stream capture).  Returns PSM_ERR_CAPACITY if no shape fits. */
psm_status psm_autotune(psm_ctx* ctx, const psm_surfels* s, const psm_camera* cams, int32_t n_cams,
                        psm_config* cfg, void* workspace, size_t workspace_bytes, int64_t pair_capacity,
                        psm_images* out, const psm_image_grads* grad_out, psm_grads* grads, int32_t reps,
                        double* best_ms_out, void* stream);

/* ------------------------------------------------------------------------
 * Instance labels of surfels from localized queries (Sec. 4.1, eqs. (4)-(7)).
 * For surfel g (centre p_g = means[g], instance feature f_g) and query q
 * (feature f_q, Gaussian with mean mu_q and precision P_q = Sigma_q^-1):
 *   A(q, g) = sigmoid(f_q . f_g) * exp(-(p_g - mu_q)^T P_q (p_g - mu_q) / 2)
 *   labels(g) = softmax over the queries of A(., g).
 * The rendered instance map, eq. (8), is the feature blend of the labels: write
 * them into columns of the feature array passed to psm_forward (e.g. after the
 * semantic channels) and one walk with one Top-K selection renders both.
 * ------------------------------------------------------------------------ */
typedef struct {
  int32_t n_q;         /* queries, 1..256 */
  int32_t c;           /* instance feature dim, 4..512, multiple of 4 */
  const float* feat;   /* [n_q][c] query features f_q */
  const float* mean;   /* [n_q][3] query centres mu_q */
  const float* prec;   /* [n_q][6] query precisions (xx, xy, xz, yy, yz, zz) */
} psm_queries;

/* labels: FP32 [n][ld] (device); columns 0 .. n_q-1 receive the labels,
 * columns n_q .. round_up(n_q, 8)-1 zeros, other columns are untouched.
 * ld >= round_up(n_q, 8).  f_ins: [n][c] in f_dtype (psm_dtype). */
psm_status psm_instance_labels(psm_ctx* ctx, int64_t n, const float* means, const void* f_ins, int32_t f_dtype,
                               const psm_queries* q, float* labels, int32_t ld, void* stream);

/* Device workspace (bytes, 256-aligned) of psm_instance_labels_backward. */
psm_status psm_instance_labels_workspace_size(int64_t n, const psm_queries* q, size_t* bytes_out);

/* Gradients of L = sum(d_labels * labels) (d_labels FP32 [n][ld], columns
 * 0 .. n_q-1 read).  Writes (overwrites) d_means [n][3], d_f_ins [n][c] (FP32
 * for every storage dtype), d_qfeat [n_q][c], d_qmean [n_q][3], d_qprec
 * [n_q][6] (with respect to the 6 numbers: an off-diagonal number appears twice
 * in the matrix).  Deterministic. */
psm_status psm_instance_labels_backward(psm_ctx* ctx, int64_t n, const float* means, const void* f_ins,
                                        int32_t f_dtype, const psm_queries* q, const float* d_labels, int32_t ld,
                                        void* workspace, size_t workspace_bytes, float* d_means, float* d_f_ins,
                                        float* d_qfeat, float* d_qmean, float* d_qprec, void* stream);

/* ------------------------------------------------------------------------
 * Frustum-local cross-attention of instance queries over surfels (Sec. 4.1,
 * eqs. (9)-(11)):
 *   active set V: surfels whose 99% confidence disk (rho <= -2 ln 0.01 in its
 *     plane) has a bounding sphere (radius 3.0349 max(s_u, s_v)) meeting the
 *     view frustum: not wholly behind the near plane or outside one of the
 *     planes through the camera centre and the image borders (FP32);
 *   K_j = f_j + psi(mu_j), V_j = f_j,  psi_c(mu) = sin or cos (for c / 3 even
 *     or odd) of 2^(c / 6) pi mu_(c mod 3) / pos_length;
 *   e_ij = (Q_i W_Q) . (K_j W_K) / sqrt(d),
 *   out_i = sum over j in V of softmax_j(e_ij) (V_j W_V)   (zero if V is empty).
 * FP32 matrix-core products; deterministic (fixed split of the active list,
 * merged in order).
 * ------------------------------------------------------------------------ */
typedef struct {
  int32_t n_q;          /* queries, 1..256 */
  int32_t c;            /* feature width C; (c, d) in (16,16) (32,32) (64,32) (64,64) */
  int32_t d;            /* projection width d */
  int32_t feat_dtype;   /* psm_dtype of feat */
  const void* feat;     /* [n][c] instance features f_j (device, 16-byte aligned) */
  const float* q;       /* [n_q][c] query tokens Q_i (device) */
  const float* wq;      /* [c][d] W_Q (device) */
  const float* wk;      /* [c][d] W_K (device) */
  const float* wv;      /* [c][d] W_V (device) */
  float pos_length;     /* length scale L of psi, > 0 */
} psm_attention;

/* Device workspace (bytes, 256-aligned) of psm_frustum_attention. */
psm_status psm_frustum_attention_workspace_size(psm_ctx* ctx, int64_t n, const psm_attention* a, size_t* bytes_out);

/* out: FP32 [n_q][d] (device).  active: optional uint8 [n] (device), 1 for the
 * surfels of V.  means [n][3], scales [n][2] (device).  Enqueued on stream. */
psm_status psm_frustum_attention(psm_ctx* ctx, int64_t n, const float* means, const float* scales,
                                 const psm_camera* cam, const psm_attention* a, void* workspace,
                                 size_t workspace_bytes, float* out, uint8_t* active, void* stream);

/* ------------------------------------------------------------------------
 * SOGMM geometric loss of surfels (Sec. 3.2 eq. (3), Sec. 4.2 eq. (13) and the
 * anisotropy term).  Plane prior component k: weight pi_k, mean mu_k,
 * covariance Sigma_k; reference normal n_k = eigenvector of Sigma_k's smallest
 * eigenvalue.  Surfel i takes the component of largest posterior
 * pi_k N(mu_i; mu_k, Sigma_k) (smallest FP32 score
 * (x - mu_k)^T Sigma_k^-1 (x - mu_k) + ln det Sigma_k - 2 ln pi_k, ties to the
 * lower index), and
 *   L_geo = sum_i |(mu_i - mu_k) . n_k| + lambda_n (1 - |n_i . n_k|),
 *   L_iso = sum_i (s_i1 - s_i2)^2
 * with n_i the third column of the rotation of the normalised quaternion.
 * Gradients hold the assignment fixed (sign subgradient 0 at zero).
 * ------------------------------------------------------------------------ */
typedef struct {
  int32_t k;            /* components, 1..2^20 */
  const float* mean;    /* [k][3] (device) */
  const float* cov;     /* [k][6] (xx, xy, xz, yy, yz, zz), positive definite (device) */
  const float* weight;  /* [k] mixing weights > 0 (device) */
} psm_gmm;

/* Device workspace (bytes, 256-aligned) of psm_geometry_loss. */
psm_status psm_geometry_loss_workspace_size(int64_t n, const psm_gmm* g, size_t* bytes_out);

/* losses: FP64 [2] (device) = (L_geo, L_iso); assign: optional int32 [n]
 * (device); d_means [n][3], d_scales [n][2], d_quats [n][4] (device) are
 * overwritten with dL_geo/dmu, dL_iso/ds and dL_geo/dq.  Deterministic. */
psm_status psm_geometry_loss(psm_ctx* ctx, int64_t n, const float* means, const float* scales, const float* quats,
                             const psm_gmm* g, float lambda_n, void* workspace, size_t workspace_bytes,
                             double* losses, int32_t* assign, float* d_means, float* d_scales, float* d_quats,
                             void* stream);

/* Thread-local description of the last error on this thread ("" if none). */
const char* psm_last_error(void);

/* Library version string (host memory, static). */
const char* psm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PSM_H */
