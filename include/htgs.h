/*
 * htgs.h - C ABI of the MI355X perspective-correct hybrid-transparency
 * Gaussian-splatting renderer (Hahlbohm et al., arXiv 2410.08129).
 *
 * The library renders 3D Gaussians by evaluating each one exactly along every
 * pixel ray (Sec. 3.2: Pluecker coordinates of the ray in normalised splat
 * space, Eq. rho-pluecker, no matrix inversion) and blends the fragments of a
 * pixel with hybrid transparency (Sec. 3.3, Eq. pixel_color_computation: the
 * K front-most fragments with alpha >= tau_K in exact depth order, every other
 * fragment in an order-independent tail). Tile lists use plain tile-id keys
 * with no depth sort (Sec. 4.3). The backward pass gives the gradient with
 * respect to every Gaussian parameter.
 *
 * Conventions shared by every entry point
 *  - Every array argument is a DEVICE pointer to float32 (unless stated),
 *    C-contiguous, owned by the caller. The library never allocates device
 *    memory; the caller provides a workspace sized by htgs_workspace_bytes().
 *  - All device work is enqueued on `stream` (a hipStream_t, NULL = the null
 *    stream) and is asynchronous, except where a function says it
 *    synchronises.
 *  - Return value: HTGS_OK (0) or a negative HTGS_E_* code; argument checks
 *    run before any device work, so an error return means nothing was
 *    enqueued. No C++ exception crosses this boundary.
 *  - Calls that share one workspace on one device must not overlap.
 */
#ifndef HTGS_H
#define HTGS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  HTGS_OK = 0,
  HTGS_E_INVAL = -1,      /* null pointer, bad size, K out of [0,32], bad tile shape */
  HTGS_E_WORKSPACE = -2,  /* workspace smaller than htgs_workspace_bytes() with 0 instances */
  HTGS_E_KEYWIDTH = -3,   /* total tile count exceeds the 32-bit key range */
  HTGS_E_HIP = -4,        /* a HIP call or kernel launch failed */
  HTGS_E_OVERFLOW = -5,   /* (status) more instances than the workspace holds */
  HTGS_E_TOO_MANY_VIEWS = -6,
  HTGS_E_TOO_LARGE = -7   /* htgs_render_forward_noalloc: beyond its fixed workspace */
};

/* Status flags reported by htgs_read_status(). */
enum {
  HTGS_STATUS_OVERFLOW = 1u       /* instance count exceeded the capacity; outputs invalid */
};

#define HTGS_MAX_VIEWS 16

/* Gaussian parameters (Sec. 3.1). 0 <= n < 2^27. Every array pointer (and
 * every gradient pointer of htgs_grads) must be 16-byte aligned; rows are
 * read and written with 16-byte accesses where their size allows.
 *  means          [n,3]  world-space centres
 *  log_scales     [n,3]  s = exp(log_scale); -INFINITY gives an exact zero axis
 *  quats          [n,4]  (w,x,y,z), normalised internally, must be non-zero
 *  opacity_logits [n]    o = sigmoid(logit)
 *  sh             [n,(sh_degree+1)^2,3]  real SH coefficients, index l*l+l+m,
 *                 orthonormal basis without the Condon-Shortley phase;
 *                 colour = max(0, sum k_lm Y_lm(dir) + 0.5), dir = unit vector
 *                 from the camera centre to the mean.
 *  filter_var     [n] or NULL (4-byte aligned): variance f >= 0 of the 3D
 *                 smoothing filter (Mip-Splatting, which the paper uses in
 *                 place of a screen-space filter, Sec. 4.2), normally
 *                 derived by the caller from the training cameras' sampling
 *                 rates. Each covariance R diag(s^2) R^T becomes
 *                 R diag(s^2 + f) R^T and the opacity o prod_k s_k /
 *                 sqrt(s_k^2 + f) (the peak of the density convolved with
 *                 an isotropic unit-mass Gaussian of variance f); gradients
 *                 flow through both to log_scales and opacity_logits.
 * With HTGS_FLAG_BAKED ("baked" inputs, frame-rate appendix) log_scales
 * holds the scales themselves, quats unit quaternions and opacity_logits
 * the opacities: the activations are skipped; filter_var must then be NULL
 * (bake the filter into the scales and opacities), and there is no
 * backward. */
typedef struct htgs_gaussians {
  int64_t n;
  int32_t sh_degree; /* 0..3 */
  int32_t reserved;
  const float *means;
  const float *log_scales;
  const float *quats;
  const float *opacity_logits;
  const float *sh;
  const float *filter_var;
} htgs_gaussians;

/* Pinhole camera. world_to_cam is the row-major 3x4 [R|t] (host memory, part
 * of this struct); camera axes x right, y down, z forward. A view point
 * (X,Y,Z) lands at window x = fx X/Z + cx, y = fy Y/Z + cy; pixel (i,j) has
 * its centre at (i+0.5, j+0.5). Gaussians whose view depth is <= z_near are
 * culled. */
typedef struct htgs_camera {
  float world_to_cam[12];
  float fx, fy, cx, cy;
  int32_t width, height;
  float z_near;
  int32_t reserved;
} htgs_camera;

/* Renderer settings.
 *  K          core size, 0..32 (Sec. 3.3; the paper uses 16)
 *  tau_alpha  minimum alpha of a fragment; gives rho_c = 2 ln(o/tau_alpha) (Sec. 3.2)
 *  tau_core   minimum alpha for core membership, tau_K (Sec. 4.2, 0.05)
 *  alpha_max  alpha clamp, alpha = min(alpha_max, o exp(-rho^2/2)), in (0,1)
 *  bg         background colour c_bg of Eq. pixel_color_computation
 *  tile_w/h   8x8, 16x8, 16x16 or 32x8 pixels (one 64-lane wave per 8x8
 *             block); K <= 16 for the 256-pixel shapes. There is no
 *             "0 = choose for me" value: the schedule (tile shape, LDS
 *             batch, order, culling, queue) is picked by timing candidates
 *             on the workload, which the Python package's autotuner does
 *             above this boundary, and passed in here
 *  lds_batch  records staged per batch in the forward: 0 or the tile's pixel
 *             count (one per thread), or, with 8x8 tiles, twice that
 *  flags      HTGS_FLAG_COST_ORDER: rasterize tiles in descending order of
 *             their instance count (better load balance on uneven scenes);
 *             HTGS_FLAG_GRAD_OVERWRITE: the backward writes the gradients
 *             instead of adding to them (zeros for Gaussians that no view
 *             covers), so the caller need not clear them first;
 *             HTGS_FLAG_TILE_CULL: for screen boxes of at most 64 tiles,
 *             drop the tiles of the box that the splat's rho_c-ellipse does
 *             not reach (exact float64 test against the tile's pixel
 *             centres, with 0.1% slack on rho_c). Images, state and
 *             gradients are the same as without it; the tile lists are then
 *             a subset of Sec. 3.2's box lists (forward and backward of one
 *             frame must use the same flag);
 *             HTGS_FLAG_PERSISTENT: the raster launches hold as many
 *             workgroups as fit on the device at once, each pulling tiles
 *             from an atomic queue (in descending-cost order with
 *             HTGS_FLAG_COST_ORDER) until it runs out;
 *             HTGS_FLAG_NO_TAIL: inference without the tail (Sec. 4.3,
 *             "Hybrid Transparency Ablations"): C = sum over the core of
 *             alpha_i T_i c_i + T_{n+1} c_bg, every non-core fragment left
 *             out; the state then holds an empty tail. Forward only: the
 *             backward rejects it with HTGS_E_INVAL;
 *             HTGS_FLAG_BAKED: the parameter arrays hold activated values
 *             (see htgs_gaussians). Forward only;
 *             HTGS_FLAG_SORTED: sorted alpha blending instead of hybrid
 *             transparency, the paper's "w/o per-pixel HT" configuration
 *             (Sec. 4.3, Table splat_eval): every tile's list holds its
 *             Gaussians front to back by the view depth of their means
 *             (the means' view z in float64, rounded to float32; ties by
 *             ascending index), and each pixel alpha-blends its fragments
 *             in that order (Eq. alpha_blending), C = sum alpha_i T_i c_i +
 *             T c_bg, leaving out the first fragment that would take T
 *             below tau_T and everything after it (the early stop plain
 *             alpha blending allows, Sec. 5). K and tau_core are unused.
 *             One view per call; forward only */
typedef struct htgs_config {
  int32_t K;
  float tau_alpha;
  float tau_core;
  float alpha_max;
  float bg[3];
  int32_t tile_w;
  int32_t tile_h;
  int32_t lds_batch;
  uint32_t flags;
  float tau_T;       /* HTGS_FLAG_SORTED: transmittance threshold of the early stop, [0,1) */
} htgs_config;

#define HTGS_FLAG_COST_ORDER 1u
#define HTGS_FLAG_GRAD_OVERWRITE 2u
#define HTGS_FLAG_TILE_CULL 4u
#define HTGS_FLAG_PERSISTENT 8u
#define HTGS_FLAG_NO_TAIL 16u
#define HTGS_FLAG_BAKED 32u
#define HTGS_FLAG_SORTED 64u

/* Gradient outputs, same shapes as htgs_gaussians. The backward ADDS into
 * them (+=), or overwrites them with HTGS_FLAG_GRAD_OVERWRITE; any pointer
 * may be NULL to skip that parameter.
 * Densification sums (Sec. 4.2; [n] each, 4-byte aligned, or NULL), always
 * ADDED to, whatever the flags, so that they gather over training steps:
 *  mean_grad_stat  per view v of the call, |dL_v/dmu| * |mu - c_v| / 2: the
 *                  gradient of the mean scaled by half the distance of the
 *                  mean from the camera centre (the paper's replacement for
 *                  the screen-space mean gradient of 3DGS)
 *  visible_count   per view, 1 where the Gaussian survives culling and its
 *                  screen box (Sec. 3.2) holds a pixel centre */
typedef struct htgs_grads {
  float *means;
  float *log_scales;
  float *quats;
  float *opacity_logits;
  float *sh;
  float *mean_grad_stat;
  float *visible_count;
} htgs_grads;

/* Bytes of workspace for n Gaussians, the given views and settings, and room
 * for max_instances (Gaussian, tile) instances. The workspace carries the
 * per-splat records, tile lists and backward partials from a forward call to
 * the matching backward call; its capacity is derived from the byte size
 * passed to every call. */
int htgs_workspace_bytes(int64_t n, const htgs_camera *cams, int32_t n_views,
                         const htgs_config *cfg, int64_t max_instances,
                         int64_t *bytes_out);

/* Bytes of the per-pixel forward state of ALL views (caller-owned, kept from
 * forward to backward). With HTGS_FLAG_SORTED: 7 values per pixel, T after
 * the last blended fragment, the blended colour sum (3 float32), the list
 * position after the last blended fragment, the number of blended
 * fragments and the index of the Gaussian the early stop left out (-1:
 * none) (int32 each), in the tile-major layout below. Otherwise per pixel
 * 24K+24 bytes, 6K+6 float32 values: K core
 * Gaussian ids (int32, -1 = empty, front to back), K core alphas, K core
 * positions in the pixel's tile list (int32, used by the backward), K core
 * colours (r, g, b each), T_{n+1}, tail sum of alpha, tail sum of
 * alpha*rgb (3 values), tail product of (1-alpha). Layout, per view in
 * order: tile by tile (row-major
 * over the view's tiles, each tile padded to full size at the image edge);
 * inside a tile, value by value; inside a value, the tile's 8x8 pixel
 * blocks row-major, inside a block its pixels row-major. (A tile's values
 * are contiguous, so the forward writes and the backward reads them with
 * whole cache lines.) */
int htgs_state_bytes(const htgs_camera *cams, int32_t n_views, const htgs_config *cfg,
                     int64_t *bytes_out);

/* Runs the preprocessing of every view and returns the number of
 * (Gaussian, tile) instances the forward will need. SYNCHRONISES the stream.
 * ws may be sized for 0 instances. */
int htgs_count_instances(const htgs_gaussians *g, const htgs_camera *cams, int32_t n_views,
                         const htgs_config *cfg, void *ws, int64_t ws_bytes,
                         int64_t *instances_out, void *stream);

/* Forward render of one view (Sec. 3.2-3.3). out_rgb is [3,H,W]. state may be
 * NULL (inference); otherwise it receives the per-pixel state described at
 * htgs_state_bytes() that htgs_render_backward() needs. If more instances
 * arise than the workspace holds, the status word reports
 * HTGS_STATUS_OVERFLOW and the image is invalid. */
int htgs_render_forward(const htgs_gaussians *g, const htgs_camera *cam,
                        const htgs_config *cfg, void *ws, int64_t ws_bytes, void *state,
                        float *out_rgb, void *stream);

/* Bytes of the library-owned device workspace of htgs_render_forward_noalloc
 * (one copy per GPU, held from the library's load until the process ends). */
#define HTGS_NOALLOC_WS_BYTES (64ll << 20)

/* Allocation-free forward render of one view, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc). Same image as htgs_render_forward() with
 * state = NULL (inference; no backward), but with no caller workspace: the
 * library uses its own device array of HTGS_NOALLOC_WS_BYTES on the current
 * device (which must be the stream's device), and this call allocates
 * nothing (no hipMalloc, no events). The device address of that array is
 * looked up on the first call on each device.
 *  out_rgb     [3,H,W] DEVICE float32, caller-owned
 *  status_out  DEVICE uint32 or NULL (4-byte aligned): receives the
 *              HTGS_STATUS_* flags of this call (asynchronously, on stream);
 *              HTGS_STATUS_OVERFLOW means the instances did not fit in the
 *              array and the image is invalid
 * Returns HTGS_E_TOO_LARGE when the per-splat data (about 160 bytes per
 * Gaussian) and the image's tiles alone exceed the array (so at most about
 * 400,000 Gaussians, fewer as instances need room too). Every call on one GPU shares that GPU's
 * array: calls that overlap on one GPU (two streams, two threads) race and
 * give wrong images; serialise them. Each call clears the array's headers
 * itself, so no call depends on the one before. */
int htgs_render_forward_noalloc(const htgs_gaussians *g, const htgs_camera *cam,
                                const htgs_config *cfg, float *out_rgb, uint32_t *status_out,
                                void *stream);

/* Backward of the last htgs_render_forward() on this workspace and state
 * (Sec. 3.3, last paragraph: the core's fragments are re-evaluated from the
 * stored per-pixel core and differentiated back to front; every tail
 * fragment's derivative uses per-pixel factors precomputed from the stored
 * tail sums). grad_rgb is dL/dC [3,H,W]; gradients w.r.t. every parameter
 * are ADDED to `grads` (or written, with HTGS_FLAG_GRAD_OVERWRITE).
 * Deterministic (no floating-point atomics). The backward evaluates each
 * pixel's fragments with the forward's own float32 forms, so it
 * differentiates exactly the fragments the forward blended. Same g, cam, cfg
 * as the forward. After a forward whose status reports a flag, the
 * gradients are zero (added: unchanged). */
int htgs_render_backward(const htgs_gaussians *g, const htgs_camera *cam,
                         const htgs_config *cfg, void *ws, int64_t ws_bytes,
                         const void *state, const float *grad_rgb, const htgs_grads *grads,
                         void *stream);

/* Several views of one scene in one pass per stage (1 <= n_views <=
 * HTGS_MAX_VIEWS). out_rgb[v] is [3,H_v,W_v]; state holds all views in order
 * (htgs_state_bytes). The backward sums the gradients of all views. */
int htgs_render_forward_batched(const htgs_gaussians *g, const htgs_camera *cams,
                                int32_t n_views, const htgs_config *cfg, void *ws,
                                int64_t ws_bytes, void *state, float *const *out_rgb,
                                void *stream);
int htgs_render_backward_batched(const htgs_gaussians *g, const htgs_camera *cams,
                                 int32_t n_views, const htgs_config *cfg, void *ws,
                                 int64_t ws_bytes, const void *state,
                                 const float *const *grad_rgb, const htgs_grads *grads,
                                 void *stream);

/* Reads the status flags (HTGS_STATUS_*), the instance count and the number
 * of fragments (pixel-Gaussian pairs with rho^2 <= rho_c) of the last call on
 * ws; instances_out and fragments_out may be NULL. SYNCHRONISES the stream. */
int htgs_read_status(const void *ws, int64_t ws_bytes, uint32_t *flags_out,
                     int64_t *instances_out, int64_t *fragments_out, void *stream);

/* Stage timing for benchmarking. While enabled, every later call records a
 * pair of HIP events on its stream around each stage it launches;
 * htgs_profile_read() waits for those events and returns, per stage, the
 * summed milliseconds and the number of kernel launches, then clears them.
 * Host-side state, not thread-safe; keep it disabled during graph capture. */
enum {
  HTGS_STAGE_FILL = 0, HTGS_STAGE_PREPROCESS = 1, HTGS_STAGE_SORT = 2, HTGS_STAGE_RANGES = 3,
  HTGS_STAGE_RASTER_FWD = 4, HTGS_STAGE_RASTER_BWD = 5,
  HTGS_STAGE_REDUCE = 6, /* kept for numbering; no separate reduction pass is launched */
  HTGS_STAGE_PREPROCESS_BWD = 7,
  HTGS_STAGE_DEPTH_SORT = 8, /* sorted blending: depth keys and their four sort passes */
  HTGS_NUM_STAGES = 9
};
int htgs_profile_enable(int on);
int htgs_profile_read(double *ms_out, int64_t *launches_out, int32_t n_stages);

/* Copies the sorted tile lists of the last forward to HOST memory: keys
 * (global tile id, converted to uint32) and values (Gaussian index), up to
 * max_out entries each, plus the per-Gaussian tile rectangles of view 0
 * (int32 [n,4]: tx0, ty0, tx1, ty1, empty when tx0 > tx1; rects_out may be
 * NULL). Same n, cams, cfg as the forward. SYNCHRONISES the stream. */
int htgs_debug_export_bins(const htgs_gaussians *g, const htgs_camera *cams, int32_t n_views,
                           const htgs_config *cfg, const void *ws, int64_t ws_bytes,
                           uint32_t *keys_out, uint32_t *values_out, int64_t max_out,
                           int32_t *rects_out, int64_t *instances_out, void *stream);

/* Opacity decay of the densification phase (Sec. 4.2: opacities are
 * multiplied by lambda_o = 0.9995 every 50 iterations instead of being
 * reset): opacity_logits[i] <- logit(lambda * sigmoid(opacity_logits[i])),
 * in place, DEVICE pointer, n entries, 0 < lambda <= 1; computed in float64
 * and finite for every finite input. Asynchronous on stream. */
int htgs_opacity_decay(float *opacity_logits, int64_t n, double lambda, void *stream);

/* Debugging and testing.
 * htgs_debug_fragment_counts: fragments (pixel-Gaussian pairs with
 *   rho^2 <= rho_c) counted by the last forward raster on ws and by the
 *   backward rasters since that forward. SYNCHRONISES the stream. */
int htgs_debug_fragment_counts(const void *ws, int64_t ws_bytes, int64_t *forward_out,
                               int64_t *backward_out, void *stream);

/* Static description of an error code. */
const char *htgs_strerror(int code);

/* ABI version, currently 4 (htgs_debug_set_spin_limit removed: no launch
 * waits across workgroups any more). */
int htgs_version(void);

#ifdef __cplusplus
}
#endif

#endif /* HTGS_H */
