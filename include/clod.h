/*
 * clod.h -- C ABI of libclod, the MI355X (gfx950) render path of CLoD-GS
 * (continuous level of detail for 3D Gaussian splatting, arXiv 2510.09997).
 *
 * Conventions for every call
 *   - Pointers are DEVICE pointers owned by the caller unless a comment says "host".  The
 *     library never allocates, frees or retains device memory; it carves the two caller
 *     workspaces described by clod_batch.
 *   - Work is enqueued on `stream` (a hipStream_t passed as void*, NULL = default stream) and
 *     returns before it completes.  Only clod_bin_sort with a non-NULL `n_dup_host` and
 *     clod_read_info synchronise the stream.
 *   - Argument errors are detected on the host before anything is launched and return
 *     CLOD_E_ARG; clod_last_error() then names the argument.  A HIP launch failure returns
 *     CLOD_E_HIP.  Duplicate-buffer overflow is detected on the device; see clod_bin_sort.
 *   - Every floating-point step follows the binary32 arithmetic contract (operation order,
 *     fused multiply-adds only where specified, correctly rounded division and square root,
 *     a fixed polynomial exponential), so integer results (keys, order, ranges, counts,
 *     last-contributor indices) are reproducible bit for bit.
 *   - One clod_batch (and its workspaces) per stream at a time; the library keeps no other
 *     state, except the thread-local error message.
 *
 * Layouts ("plane-major" structure of arrays, n = number of Gaussians):
 *   mean [3][n], log_scale [3][n], quat [4][n] (w, x, y, z), opacity [n] (logit),
 *   decay [n] (sigma_d), sh [(deg+1)^2][3][n].  Gradients use the same layout.
 *   Images of a batch of views are concatenated: view v starts at pixel offset
 *   P_v = sum_{u<v} H_u W_u; rgb holds [3][H_v][W_v] at 3 P_v, T and last hold [H_v][W_v] at P_v.
 */
#ifndef CLOD_H
#define CLOD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CLOD_ABI_VERSION 13
#define CLOD_MAX_VIEWS 1024

typedef enum {
  CLOD_OK = 0,
  CLOD_E_ARG = -1,       /* invalid argument (host check, nothing launched)           */
  CLOD_E_CAPACITY = -2,  /* more tile duplicates than the duplicate buffer holds       */
  CLOD_E_HIP = -3,       /* a HIP runtime call or kernel launch failed                  */
  CLOD_E_UNSUPPORTED = -4,
  CLOD_E_BUSY = -5       /* every slot of the persistent server holds an unfinished job    */
} clod_status;

/* A scene: n Gaussians (Sec. 3.1: mean, covariance from scale and rotation, opacity, SH
   colour coefficients) plus the one extra learnable decay factor sigma_d of Sec. 3.2. */
typedef struct clod_scene {
  int64_t n;              /* >= 0 */
  int32_t sh_degree;      /* 0..3 */
  int32_t reserved;
  const float *mean, *log_scale, *quat, *opacity, *decay, *sh;
  const float *sh_packed; /* NULL, or the same SH coefficients laid out per Gaussian,
                             [n][(sh_degree+1)^2][3]; when set, clod_project reads colours from
                             it (one contiguous block per Gaussian instead of 3 (deg+1)^2 planes:
                             far fewer memory lines for the sparse set of rendered Gaussians).
                             For static scenes (serving); the caller keeps it equal to sh. */
} clod_scene;

/* Gradient planes, same layout as clod_scene; all must be non-NULL. */
typedef struct clod_scene_grad {
  float *mean, *log_scale, *quat, *opacity, *decay, *sh;
} clod_scene_grad;

/* One view: a pinhole camera (OpenCV axes: x right, y down, z forward; pixel (i, j) covers
   [i, i+1) x [j, j+1) and is sampled at its centre) and the virtual distance scale s_v >= 1
   of Sec. 3.2 (it strengthens the decay and the mask threshold; it does not move the camera).
   112 bytes. */
typedef struct clod_view {
  float W[9];             /* world-to-camera rotation, row-major */
  float t[3];             /* world-to-camera translation */
  float c[3];             /* camera centre (the c of d_i = |mu_i - c|, Sec. 3.2); must equal -W^T t to 1e-4 relative */
  float fx, fy, cx, cy;   /* intrinsics in pixels */
  int32_t width, height;  /* 1..16384 */
  float s_v;              /* virtual distance scale, finite, >= 1 */
  int64_t budget;         /* LoD selection: 0 keeps alpha'' > tau * s_v (Sec. 3.2); K > 0 keeps the
                             K Gaussians of largest alpha'' (lower index first among equal values),
                             the primitive-budget selection of the Sec. 4 comparisons */
  int32_t frame_width;    /* 0: the view is its own frame.  > 0: the view renders the viewport */
  int32_t frame_height;   /*   [vx, vx + width) x [vy, vy + height) of a frame_width x frame_height */
  int32_t vx, vy;         /*   image (vx, vy multiples of 16): frustum, frustum maximum and pixel
                               coordinates are the frame's, tile rectangles the frame's clipped to
                               the viewport -- spatially varying s_v renders a frame as viewports
                               with their own s_v (the strips of the Sec. 4 DLoD comparison) */
} clod_view;

/* Constants the paper leaves open (readings; defaults in parentheses). */
typedef struct clod_params {
  float tau;              /* base threshold of the mask alpha'' > tau s_v (1/255), >= 0 */
  float eps;              /* epsilon of Eq. (2) (1e-6), > 0 */
  float near_z;           /* frustum near plane (0.2), > 0 */
  float guard;            /* frustum widening of the half field-of-view tangents (1.3), > 0 */
  float dilation;         /* EWA screen-space dilation in px^2 (0.3), >= 0 */
  float bg[3];            /* background colour (0) */
} clod_params;

/* A batch of views rendered together (continuous batching and multi-view training use
   n_views > 1; resolutions may differ).  All fields are host values except the device
   pointers marked so. */
typedef struct clod_batch {
  int64_t n;                       /* Gaussians of the scene this batch renders (= scene->n) */
  int32_t n_views;                 /* 1..CLOD_MAX_VIEWS */
  int32_t reserved;
  const clod_view *views_host;     /* host: n_views entries (validation, launch geometry) */
  const clod_view *views_dev;      /* device: the same n_views entries, read by the kernels;
                                      poses and s_v may be rewritten between graph replays,
                                      width/height must stay equal to views_host */
  clod_params params;
  void *ws;  size_t ws_bytes;      /* device workspace, >= clod_ws_bytes(), 256-byte aligned */
  void *dup; size_t dup_bytes;     /* device duplicate buffer, clod_dup_bytes(capacity) */
} clod_batch;

/* Bytes of the per-Gaussian / per-view / per-tile workspace for n Gaussians and these views. */
size_t clod_ws_bytes(int64_t n, int32_t n_views, const clod_view *views_host);

/* Bytes of a duplicate buffer holding `capacity` (tile, Gaussian) pairs (keys, values,
   ping-pong copies and radix histograms). */
size_t clod_dup_bytes(int64_t capacity);

/* Largest capacity that fits in dup_bytes. */
int64_t clod_dup_capacity(size_t dup_bytes);

/* Sec. 3.2 and Sec. 3.1 (projection): for every view and Gaussian, camera distance d_i, the
   frustum set N_view and its maximum distance (argmax = lowest index among equals; an empty
   frustum uses 1), normalised distance d'_i, attenuated opacity of Eq. (2), LoD mask
   M_i = alpha''_i > tau s_v, and for M_i and in-frustum Gaussians the EWA projection, cull,
   16x16-tile rectangle and SH colour.  counts_dev (nullable, device int64 [n_views][3])
   receives {n_frustum, n_mask, n_rendered}; eta_dev (nullable, device float [n_views]) receives
   the kept ratio eta_actual = n_mask / n of Sec. 3.3, Eq. (4) (binary32 quotient of the two
   counts rounded to binary32; 0 when n = 0).  The results stay in batch->ws for the calls
   below.  Consecutive views with the same camera (pose, intrinsics, size, frame and viewport,
   bit for bit), such as the LoD frames of one pose at several s_v, share the camera-dependent
   work (frustum maximum, distances, projection, colour); the results are the same as for
   separate batches. */
clod_status clod_project(const clod_scene *scene, const clod_batch *batch, int64_t *counts_dev,
                         float *eta_dev, void *stream);

/* Sec. 3.1 (splats sorted by depth per tile): the (rendered Gaussian, covered tile) pairs in
   the stable order of the keys (tile_base[view] + tile) << 32 | bits(depth) emitted per
   rendered Gaussian in index order and per covered tile in row-major order -- i.e. ordered by
   (view, tile, depth, Gaussian index) -- and per-tile [start, end) ranges of the sorted list.
   Built as a radix sort of the rendered records by depth followed by a stable radix sort of
   the pairs, emitted in that depth order, by tile id.  If more pairs exist than the duplicate buffer holds, nothing is written beyond
   it, the overflow is recorded in ws and later calls on this batch are no-ops; with
   n_dup_host != NULL the call synchronises `stream`, stores the pair count D (also on
   overflow) and returns CLOD_E_CAPACITY on overflow (enlarge batch->dup and call again; the
   clod_project results stay valid). */
clod_status clod_bin_sort(const clod_batch *batch, int64_t *n_dup_host, void *stream);

/* Sec. 3.1, Eq. (1): per pixel, front-to-back blending of its tile's sorted list with
   alpha'_i = alpha''_i G2D_i (clamped to 0.99, skipped below 1/255), stopping before the
   entry that would bring transmittance below 1e-4.  Writes rgb (colour + T * bg), the final
   transmittance T and last = 1 + position (within the tile's list) of the last blended entry
   (0 if none).  pairs_dev (nullable, device int64 [3]) is incremented by the work of the
   per-pixel loop: {pairs evaluated (entries visited up to and including the terminating one),
   exponentials evaluated (pairs that are not provably skipped before it), pairs blended}.
   The first and last are properties of the contract; the middle one of this implementation. */
clod_status clod_render_fwd(const clod_batch *batch, float *rgb, float *T, uint32_t *last,
                            int64_t *pairs_dev, void *stream);

/* Adjoint of clod_project + clod_render_fwd (the method is end-to-end differentiable,
   Sec. 1 and Sec. 3.2).  Given dL/drgb (same layout as rgb) and optionally dL/deta
   (device float [n_views]: the straight-through gradient of the point-count term, applied
   as d eta / d alpha''_i = 1 / n for every Gaussian), recomputes each pixel's blend
   back-to-front from its stored last index and T, and writes (accumulate = 0) or adds
   (accumulate != 0) the gradients of all parameter planes, including the decay factor and the
   normalised distance through the virtual distance scale and the frustum maximum.
   Requires the same scene and batch as the preceding clod_project / clod_bin_sort /
   clod_render_fwd.  pairs_dev (nullable, device int64 [3]) receives, added to its contents
   (zero it first), the work of the per-pixel adjoint loop: (pixel, entry) lanes walked, pairs
   whose exponential was evaluated (blended in the forward, power in range) and pairs that
   contribute to the gradients; counting costs an extra pass over the per-tile partials. */
clod_status clod_render_bwd(const clod_scene *scene, const clod_batch *batch, const float *T,
                            const uint32_t *last, const float *dL_drgb, const float *dL_deta,
                            int32_t accumulate, const clod_scene_grad *grad, int64_t *pairs_dev, void *stream);

/* Sec. 3.2 mask and Sec. 3.3 eta_actual for many views without rendering: counts_dev
   (device int64 [n_views][3]) receives {n_frustum, n_mask, n_rendered} per view, with the
   same decisions as clod_project.  Uses the leading part of batch->ws (per-view data and a
   work list of n entries; a workspace of clod_ws_bytes(n, ...) bytes always suffices, and a
   shorter one is rejected with CLOD_E_ARG); batch->dup is not used. */
clod_status clod_lod_count(const clod_scene *scene, const clod_batch *batch, int64_t *counts_dev,
                           void *stream);

/* Scene preparation, not an operation of the method: reorders a scene's Gaussians along a
   Morton (Z-order) curve of their means, so that Gaussians close in space are close in memory
   (the per-(view, Gaussian) records that the blend gathers are indexed by Gaussian, and
   neighbours in memory then tend to serve the same tiles).  Every result of the library is
   defined on the scene as stored, so a reordered scene renders the Gaussians of the original
   one (ties in depth fall to the lower index of the new order).
   The order: 10 bits per axis over the bounding box of the finite mean coordinates (coordinates
   outside it or not finite clamp to its faces, an axis without extent gives zero bits), bits
   interleaved x lowest, then a stable sort by the 30-bit code (equal codes keep index order).
   perm (device uint32 [n]) receives perm[j] = the original index of the Gaussian placed at j;
   dst (device planes in clod_scene's layout, sh with src's degree) receives src's planes
   gathered by perm; sh_packed is not read or written (build it from dst's sh).  workspace:
   device, 256-byte aligned, >= clod_scene_reorder_ws_bytes(n) bytes.  dst must not overlap
   src; n <= 2^31 - 1.  CLOD_E_ARG on invalid arguments (nothing launched); n = 0 is a no-op. */
size_t clod_scene_reorder_ws_bytes(int64_t n);
clod_status clod_scene_reorder(const clod_scene *src, const clod_scene_grad *dst, uint32_t *perm,
                               void *workspace, size_t workspace_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, serving loops
   that must not call hipMalloc, harnesses that forbid it): the counts of clod_lod_count, with
   the same decisions, for n Gaussians and n_views views (views_host: host array for validation
   and launch geometry; views_dev: the same views in device memory; params: host), without a
   caller workspace.  The per-view constants, per-block partials and the work list live in a
   library-owned device array of CLOD_LOD_SCRATCH_BYTES per GPU (held by each GPU the library
   runs on until the process ends); the call allocates nothing.  Inputs whose workspace exceeds
   it (about 4 bytes per Gaussian plus about 24 KiB per view, plus 128 KiB per budgeted view)
   are rejected with CLOD_E_ARG before anything is launched.  Every call on one GPU shares that
   array and leaves its contents behind (nothing in it needs to start cleared): calls that
   overlap on one GPU (other streams or threads) race and must be serialised by the caller. */
#define CLOD_LOD_SCRATCH_BYTES (64u << 20)
clod_status clod_lod_count_noalloc(const clod_scene *scene, int32_t n_views, const clod_view *views_host,
                                   const clod_view *views_dev, const clod_params *params,
                                   int64_t *counts_dev, void *stream);

/* Sec. 3.3, Eq. (3)-(5), with L_render the 3DGS rendering loss, a weighted sum of L1 and
   D-SSIM: per view v,
     L1_v = mean |rgb - target| over 3 H W,
     SSIM_v = mean over pixels and channels of the SSIM map (11 x 11 Gaussian window, sigma 1.5,
              zero padding, C1 = 0.01^2, C2 = 0.03^2),
     L_render = (1 - lambda_dssim) L1_v + lambda_dssim (1 - SSIM_v),
     eta_v = n_mask / batch->n (from the last clod_project), eta_target = s_v^-1.5,
     L_reg = (s_v - 1)^2 ReLU(eta_v - eta_target)^2, w_s = (1 - 0.5 s_v / s_max)^2,
     L_v = w_s (L_render + lambda_reg L_reg).
   Writes loss_dev (device float [n_views]), dL_drgb (the gradient of L_v with respect to the
   view's rgb; sign(0) = 0) and dL_deta_dev (device float [n_views], nullable) = w_s lambda_reg
   dL_reg/deta.  lambda_dssim in [0, 1]; when it is > 0, ssim_scratch is a device buffer of at
   least 36 bytes per pixel of the batch (per-pixel SSIM derivatives); with 0 it may be NULL and
   L_render = L1. */
clod_status clod_loss(const clod_batch *batch, const float *rgb, const float *target,
                      float s_max, float lambda_reg, float lambda_dssim, float *ssim_scratch,
                      size_t ssim_scratch_bytes, float *loss_dev, float *dL_drgb,
                      float *dL_deta_dev, void *stream);

/* Hyperparameters of one Adam step (binary32). */
typedef struct clod_adam {
  float lr[7];            /* learning rates of the groups mean, log_scale, quat, opacity, decay,
                             SH degree 0 (sh[0 .. 3n)), SH degree >= 1 (sh[3n ..)); >= 0 */
  float beta1, beta2;     /* in [0, 1) */
  float eps;              /* > 0 */
  int32_t reserved;
  int64_t step;           /* t >= 1: the library forms the bias corrections bias1 = 1 - beta1^t and
                             bias2 = 1 - beta2^t in double precision from the binary32 betas and
                             rounds each once to binary32 */
} clod_adam;

/* Sec. 4.1 (training follows the 3DGS recipe, with sigma_d as one more per-Gaussian parameter
   and its own learning rate): one fused Adam step over every parameter plane of a scene of n
   Gaussians of SH degree sh_degree.  param, grad, m and v are device planes in the clod_scene
   layout (grad is only read; param, m and v are updated in place; all non-NULL when n > 0).
   Per element, in binary32 and this order: m = beta1*m + (1-beta1)*g;
   v = beta2*v + (1-beta2)*(g*g); p = p - lr*((m/bias1) / (sqrt(v/bias2) + eps)).
   Asynchronous on `stream`. */
clod_status clod_adam_step(int64_t n, int32_t sh_degree, const clod_scene_grad *param,
                           const clod_scene_grad *grad, const clod_scene_grad *m,
                           const clod_scene_grad *v, const clod_adam *hp, void *stream);

/* Synchronises `stream` and copies to host info[4] = {D (tile pairs of the last
   clod_bin_sort), overflow flag, duplicate capacity, radix passes}. */
clod_status clod_read_info(const clod_batch *batch, int64_t *info_host, void *stream);

/* Read-only views of intermediate results (for inspection and tests).  Stores the device
   address of the section and its element count; nothing is launched or copied.
     CLOD_SEC_KEYS     uint32 tile ids of the sorted pairs (count = duplicate capacity; the
                       first D are valid, D from clod_bin_sort or clod_read_info)
     CLOD_SEC_VALUES   uint32 sorted record indices v*n + i (count as above)
     CLOD_SEC_RANGES   uint32 pairs [start, end) per tile of the batch (count = tiles)
     CLOD_SEC_REC      64-byte records per (view, Gaussian), four 16-byte quads: float (u, v,
                       alpha'', radius), float (conic A, B, C, 0), float (r, g, b, 0), then
                       (float camera depth, uint32 x0 | x1 << 16, uint32 y0 | y1 << 16, uint32
                       tiles touched) -- the tile rectangle [x0, x1) x [y0, y1) in the view's
                       tiles; written whole for rendered Gaussians only (count = n_views * n)
     CLOD_SEC_ALPHA    float per (view, Gaussian): alpha'' of Eq. (2), every Gaussian
     CLOD_SEC_FLAGS    uint8 per (view, Gaussian): bit0 frustum, bit1 mask, bit2 rendered,
                       bits 3..5 colour clamped
     CLOD_SEC_DMAX     uint64 per view: bits(d_max) << 32 | (2^32 - 1 - argmax), 0 if empty
     CLOD_SEC_GSCREEN  float [n_views * n][9] screen-space partials of the last backward
                       (u, v, conic A, B, C, alpha'', r, g, b), nine per (view, Gaussian);
                       only rendered records are cleared and accumulated, others unspecified
     CLOD_SEC_HEADER   uint64 [2] = {D of the last clod_bin_sort, overflow flag} (count = 2);
                       an asynchronous copy of it avoids the synchronisation of clod_read_info */
enum {
  CLOD_SEC_KEYS = 0, CLOD_SEC_VALUES = 1, CLOD_SEC_RANGES = 2, CLOD_SEC_REC = 3, CLOD_SEC_ALPHA = 4,
  CLOD_SEC_FLAGS = 6, CLOD_SEC_DMAX = 7, CLOD_SEC_GSCREEN = 9, CLOD_SEC_HEADER = 10
  /* 5 and 8 are not used (depth and rectangle live in the fourth quad of a record) */
};
clod_status clod_inspect(const clod_batch *batch, int32_t section, const void **dev_ptr,
                         int64_t *count);

/* Persistent serving launch (Sec. 4.2: real-time rendering of a resident scene at any viewing
   distance; requests are batched continuously).  One kernel stays resident on the stream given
   to clod_server_start until clod_server_stop.  A job is one batch of views: the stages that
   clod_project, clod_bin_sort and clod_render_fwd launch one kernel at a time, run instead by
   the resident workgroups, which take blocks of the open stage of the oldest unfinished job;
   stages of different jobs overlap.  Results are bit-identical to those three calls.

   Threading: one host thread drives a server.  Jobs complete in any order; up to
   CLOD_SERVER_SLOTS are in flight.  Each job's scene, workspace, duplicate buffer and outputs
   must stay valid and untouched until clod_server_poll reports the job done.  While the server
   runs, work of other streams still gets the device capacity the server leaves free (one
   workgroup slot per compute unit by default); never synchronise the whole device, free device
   memory (which synchronises it) or wait on the server's stream before clod_server_stop. */
#define CLOD_SERVER_SLOTS 16
#define CLOD_SERVER_MAX_VIEWS 16
typedef struct clod_server clod_server;

/* Allocates the server's queue state (device memory, and coherent pinned host memory for the
   job ring and completion records) and launches the resident kernel on `stream`.  workers: 0
   fills the device's resident capacity but one workgroup per compute unit, else that many
   worker workgroups.  max_seconds in (0, 3600]: the kernel ends by itself after this long (a
   bound on every wait; jobs still open then never complete).  *server receives the handle,
   *workers_used (nullable) the worker count. */
clod_status clod_server_start(int32_t workers, double max_seconds, void *stream, clod_server **server,
                              int32_t *workers_used);

/* Publishes one job: the views of `batch` rendered as clod_project + clod_bin_sort +
   clod_render_fwd would (no counters), into rgb / T / last with their layouts.  Same checks as
   those calls, plus: batch->n_views <= CLOD_SERVER_MAX_VIEWS, scene->sh_packed set (the
   server's projection reads the packed coefficients); batch->views_dev is not read (the job
   carries its own copy of views_host).  Never blocks: CLOD_E_BUSY when the next slot's job has
   not completed yet (poll, then retry).  *seq receives the job's sequence number (0, 1, ...). */
clod_status clod_server_submit(clod_server *server, const clod_scene *scene, const clod_batch *batch, float *rgb,
                               float *T, uint32_t *last, int64_t *seq);

/* *done = 1 once job seq is complete (its outputs are then visible to later work on any
   stream), else 0.  info (nullable) receives {overflow flag, tile pairs D, completion time in ns
   of the device clock since the server started}.  A job whose duplicate buffer overflowed
   completes with the flag set and its outputs unwritten; submit it again with a larger buffer.
   CLOD_E_ARG if seq was never published or its slot already holds a later job. */
clod_status clod_server_poll(clod_server *server, int64_t seq, int32_t *done, int64_t *info);

/* Device clock in ns since the server started, as of the server's last poll of the host (it
   polls continuously while idle); -1 before the kernel runs. */
clod_status clod_server_clock(clod_server *server, int64_t *ns);

/* Timeline of completed job seq (for profiling the resident kernel): ns[k] = device clock in ns
   since the server started when stage k opened (stage 0: when the job was activated) and
   kinds[k] (nullable) its stage kind (an internal enumeration), for the job's stages, then
   its completion time with kind 0; *count receives the entries written (at most max).  Valid
   until the slot takes a later job; CLOD_E_ARG if the job is not complete. */
clod_status clod_server_stage_times(clod_server *server, int64_t seq, int64_t *ns, int32_t *kinds, int32_t max,
                                    int32_t *count);

/* Raises the stop flag, waits for the kernel to end and frees the server.  *status (nullable):
   1 stopped on request, 2 deadline reached, 3 protocol error, 4 unsupported stage; anything
   but 1 also returns CLOD_E_HIP.  Jobs not complete by then are abandoned. */
clod_status clod_server_stop(clod_server *server, int32_t *status);

/* Message of the last error on this thread ("" if none). */
const char *clod_last_error(void);

int32_t clod_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CLOD_H */
