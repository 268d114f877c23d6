/*
 * ddgs.h -- C ABI of libddgs.so, the MI355X (gfx950) DRR splatting renderer
 * of DDGS-CT (arXiv 2406.02518).
 *
 * The library renders digitally reconstructed radiographs from two disjoint
 * sets of 3D Gaussians (isotropic and direction-dependent, Sec. 3.2) through
 * a cone-beam geometry, and differentiates the images with respect to every
 * Gaussian parameter, the two shared bases and the 6-DoF source pose of
 * every view.
 *
 *   image (Sec. 3.1, Eq. 1):  C(p) = sum_j c_j s_j prod_{l<j} (1 - s_l),
 *       s_j = min(sigma_max, alpha_j exp(-d2_j / 2)),
 *       d2_j = (p - mu^_j)^T A_j (p - mu^_j), A_j = (J Sigma_c J^T + dI)^-1,
 *       Gaussians with d2_j > kappa^2 are not considered at p, and the
 *       order is ascending depth (source-frame z of the mean, ties by index);
 *       both sets are composited together (App. A.2).
 *   radiosity (Sec. 3.2, Eq. 3):  iso c = sigmoid(b_iso . f),
 *       dir c = sigmoid(Y_{1..L}(d) . (B_dir f)), d the unit direction from
 *       the source to the Gaussian mean in the world frame, Y the real
 *       orthonormal spherical basis of degrees 1..L (k_L = L(L+2)
 *       functions, order l = 1..L, m = -l..l, no Condon-Shortley phase).
 *   loss (Sec. 3.1, Eq. 2):  (1 - lambda) mean|I - I*| + lambda (1 - SSIM),
 *       or 1 - NCC for pose scoring.
 *
 * Conventions shared by every entry point:
 *   - All array pointers in ddgs_model, ddgs_grads, images, targets and
 *     gradients are DEVICE pointers on the context's device, float32,
 *     structure-of-arrays, at least 4-byte aligned (ddgs_set_model rejects
 *     others with DDGS_ERR_INVALID_ARG), owned by the caller.  The library
 *     never frees them.  ddgs_view arrays are host memory and are copied.
 *   - All device work is enqueued on the context's stream (settable, e.g.
 *     torch's current stream).  Entry points do not synchronise the stream
 *     except where stated (ddgs_render reads the number of tile entries back;
 *     ddgs_check and the debug getters synchronise).
 *   - Every function returns a ddgs_status; on failure nothing is written to
 *     the outputs that the status code does not mention, and the message is
 *     kept in ddgs_last_error(ctx).  No C++ exception crosses the ABI.
 *   - The library's internal workspace (records, tile lists, sort
 *     temporaries, gradient slots, ...) comes from the caller's allocator
 *     (ddgs_set_allocator; the Python binding hands it torch's caching
 *     allocator), from a caller-owned region (ddgs_set_workspace), or, when
 *     neither is set, from hipMalloc.  It grows on demand, never inside a
 *     captured step, and is released by ddgs_destroy.
 *   - Every result is deterministic: no floating-point atomics are used and
 *     every reduction runs in a fixed order, so repeated calls on the same
 *     inputs give bit-identical images and gradients.  There is therefore no
 *     "deterministic" option.  Every call renders all views set with
 *     ddgs_set_views in one batch (one launch per kernel for all views);
 *     there is no separate batch-size option -- a caller wanting smaller
 *     batches sets fewer views per call.
 *   - A context is not thread-safe; use one per host thread.
 */
#ifndef DDGS_H
#define DDGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DDGS_OK = 0,
    DDGS_ERR_INVALID_ARG = 1, /* bad pointer, size, alignment or option        */
    DDGS_ERR_OOM = 2,         /* device allocation failed or workspace too small */
    DDGS_ERR_HIP = 3,         /* a HIP runtime call failed (message kept)      */
    DDGS_ERR_CAPACITY = 4,    /* tile entries exceeded the captured capacity   */
    DDGS_ERR_NONFINITE = 5,   /* non-finite value met in an input              */
    DDGS_ERR_STATE = 6,       /* call out of order (e.g. backward before render)*/
    DDGS_ERR_UNSUPPORTED = 7  /* valid request this build does not implement   */
} ddgs_status;

typedef struct ddgs_ctx ddgs_ctx;

/* Gaussian model, device SoA arrays (borrowed until the next ddgs_set_model
 * or ddgs_destroy; the caller may change their contents between calls).
 * Gaussians [0, n_iso) are isotropic, [n_iso, n) direction-dependent.
 * Activations: Sigma = R(q/|q|) diag(exp(2 log_scale)) R^T,
 * alpha = sigmoid(opacity_logit).
 * Radiosity (Sec. 3.2, Eq. 3): DDGS_RADIOSITY_DISENTANGLED gives
 * c = sigmoid(b_iso . f) to the isotropic set and
 * c = sigmoid(Y_{1..L}(dir) . (B_dir f)) to the directional one, dir being
 * the unit ray from the source to the mean.  DDGS_RADIOSITY_ENTANGLED is
 * the co-located ablation of Sec. 4 ("direct-entangled"): every Gaussian
 * carries both terms under one sigmoid, c = sigmoid(b_iso . f +
 * Y_{1..L}(dir) . (B_dir f)), and n_iso must be 0.  Iso-only and dir-only
 * models are n_iso = n and n_iso = 0 of the disentangled form. */
enum { DDGS_RADIOSITY_DISENTANGLED = 0, DDGS_RADIOSITY_ENTANGLED = 1 };
typedef struct {
    int64_t n, n_iso;            /* 0 <= n_iso <= n < 2^31 / n_views          */
    int32_t k;                   /* feature size, 1..32                       */
    int32_t L;                   /* directional degree, 1..3                  */
    const float *mean;           /* [3][n] world mm                           */
    const float *quat;           /* [4][n] (w, x, y, z), non-zero             */
    const float *log_scale;      /* [3][n]                                    */
    const float *opacity_logit;  /* [n]                                       */
    const float *feat;           /* [k][n]                                    */
    const float *b_iso;          /* [k]                                       */
    const float *B_dir;          /* [L(L+2)][k] row-major                     */
    int32_t radiosity;           /* DDGS_RADIOSITY_*, 0 = Eq. 3 as printed     */
    int32_t reserved;            /* must be 0                                 */
} ddgs_model;

/* One cone-beam view.  pose = [R | t] row-major 3x4, world -> source frame:
 * +z along the principal ray towards the detector, +x along detector
 * columns, +y along detector rows; R must be a rotation.  Focal length
 * f = sdd_mm / pitch_mm pixels, principal point (W/2, H/2), pixel (u, v)
 * has centre (u + 0.5, v + 0.5).  Images of all views are concatenated
 * view-major, each H rows of W floats. */
typedef struct {
    int32_t W, H;                /* 1..16384                                  */
    float pitch_mm, sdd_mm;      /* > 0                                       */
    float pose[12];
} ddgs_view;

/* Options; ddgs_default_options fills the defaults shown. */
typedef struct {
    int32_t tile_w, tile_h;      /* 16, 16; supported: 8x8, 16x8, 16x16, 32x8 */
    float kappa;                 /* 3: Mahalanobis cut-off radius             */
    float dilation;              /* 0.3: added to the projected covariance    */
    float t_min;                 /* 0: early stop when T(1-s) < t_min (off)  */
    float z_near;                /* 1 mm: depth at or below which a Gaussian is culled */
    float sigma_max;             /* 0.99: clamp of s                          */
    int32_t persistent;          /* 0: one workgroup per work item; m in
                                    1..8: persistent workgroups (m x 4 per CU
                                    in the forward, m x 2 in the backward)
                                    taking work items from a counter (longest
                                    tiles first when split is 0)              */
    int32_t split;               /* 256: entries per work item -- a tile's
                                    depth-ordered list is cut into chunks of
                                    this many entries, composited in parallel
                                    and merged exactly with the over operator
                                    (images then differ from split 0 only by
                                    rounding); 0: one work item per tile (the
                                    image is bit-identical for every tile
                                    shape).  Forced to 0 when t_min > 0.      */
    int64_t capacity;            /* tile-entry capacity of a captured step;
                                    0 = chosen by ddgs_step_capture          */
} ddgs_options;

/* Gradient outputs, device arrays with the shapes of the inputs; every
 * non-NULL array is OVERWRITTEN (not accumulated).  NULL skips the group;
 * if only dpose is non-NULL the per-Gaussian chain is skipped. */
typedef struct {
    float *dmean;            /* [3][n] */
    float *dquat;            /* [4][n] */
    float *dlog_scale;       /* [3][n] */
    float *dopacity_logit;   /* [n]    */
    float *dfeat;            /* [k][n] */
    float *db_iso;           /* [k]    */
    float *dB_dir;           /* [L(L+2)][k] */
    float *dpose;            /* [n_views][6]: (rho, omega), the left tangent
                                delta of pose' = Exp(delta) pose at delta = 0,
                                i.e. R' = Exp(omega) R, t' = Exp(omega) t + rho;
                                mm and rad                                   */
} ddgs_grads;

enum { DDGS_LOSS_L1_DSSIM = 0, DDGS_LOSS_NCC = 1, DDGS_LOSS_LINEAR = 2 };

/* ---------------------------------------------------------------- context */
ddgs_status ddgs_create(ddgs_ctx **out, int device, void *hip_stream);
void ddgs_destroy(ddgs_ctx *ctx);
ddgs_status ddgs_set_stream(ddgs_ctx *ctx, void *hip_stream);
const char *ddgs_status_str(ddgs_status s);
const char *ddgs_last_error(const ddgs_ctx *ctx);
void ddgs_default_options(ddgs_options *opt);
ddgs_status ddgs_set_options(ddgs_ctx *ctx, const ddgs_options *opt);
ddgs_status ddgs_get_options(const ddgs_ctx *ctx, ddgs_options *opt);

/* Eq. 1/3 inputs. */
ddgs_status ddgs_set_model(ddgs_ctx *ctx, const ddgs_model *model);
ddgs_status ddgs_set_views(ddgs_ctx *ctx, const ddgs_view *views, int n_views);
/* Pose registration (Sec. 4.3).  With an optimiser set, ddgs_step_capture
 * appends one Adam step per view on the pose-tangent gradient the step just
 * computed (grads->dpose must be non-NULL; up to 256 views) and re-bases the
 * device view table with it: (rho, omega) = -lr * mhat / (sqrt(vhat) + eps)
 * per component (lr_trans for rho in mm, lr_rot for omega in rad), then the
 * view is re-based, so every replay is one registration iteration.
 *   pivot_mode DDGS_PIVOT_SOURCE: the left tangent the backward
 *     differentiates, R <- Exp(omega) R, t <- Exp(omega) t + rho (rotation
 *     about the source point).
 *   pivot_mode DDGS_PIVOT_POINT: rotation about the world point pivot[3]
 *     (mm; the isocentre is the world origin), with p = R pivot + t its
 *     source-frame position: R <- Exp(omega) R, t <- Exp(omega)(t - p) + p
 *     + rho.  The tangent gradient is mapped first, g_omega += g_rho x p,
 *     and Adam runs on the mapped gradient.  Rotating about the source moves
 *     the image almost as a sideways shift does, which makes the two nearly
 *     interchangeable for the optimiser; a pivot inside the object avoids it.
 * The moments restart from zero at the first replay after
 * ddgs_set_pose_optimizer or ddgs_set_views.  NULL turns the optimiser off.
 * Either call drops a captured step (a new capture keeps the moments).
 * ddgs_get_views synchronises and
 * returns the current views, with the poses the optimiser has reached (they
 * also replace the host copy the library keeps).  The dpose output keeps the
 * left-tangent gradient in both modes. */
enum { DDGS_PIVOT_SOURCE = 0, DDGS_PIVOT_POINT = 1 };
typedef struct ddgs_adam {
    float lr_trans, lr_rot, beta1, beta2, eps;
    int32_t pivot_mode;
    float pivot[3];
} ddgs_adam;
ddgs_status ddgs_set_pose_optimizer(ddgs_ctx *ctx, const ddgs_adam *adam);
ddgs_status ddgs_get_views(ddgs_ctx *ctx, ddgs_view *views, int n_views);

/* Fitting (Sec. 4.1, implementation paragraph; App., Gaussians that move,
 * split and drop).
 *
 * ddgs_set_fit_optimizer: with options set, ddgs_step_capture appends one
 * Adam step over every parameter group (grads must hold all seven
 * parameter gradients) that updates the model arrays IN PLACE -- the caller
 * enables it only for writable device memory.  Per element:
 * m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * p -= lr m / (1 - b1^t) / (sqrt(v / (1 - b2^t)) + eps), t = 1, 2, ... the
 * step count kept on the device.  The position rate decays log-linearly from
 * lr_mean_init to lr_mean_final over lr_mean_steps steps and is held after.
 * Defaults (ddgs_default_fit_options): the paper's 1.25e-4 for both bases
 * and 2.5e-3 for the features; 3D Gaussian splatting's 5e-3 log-scales,
 * 1e-3 rotations, 5e-2 opacity logits, beta (0.9, 0.999), eps 1e-15 and
 * position 1.6e-4 -> 1.6e-6 times the scene extent over 30000 steps (the
 * extent argument, mm).  Moments and step count restart at the next replay
 * after this call and after ddgs_set_model, except that a model set with the
 * shape a ddgs_densify_apply produced keeps the moments it re-laid out.
 * NULL turns the optimiser off.  Either call drops a captured step. */
typedef struct ddgs_fit_opts {
    float lr_mean_init, lr_mean_final;   /* mm per step                       */
    int32_t lr_mean_steps;               /* >= 1                              */
    float lr_quat, lr_log_scale, lr_opacity, lr_feat, lr_b_iso, lr_B_dir;
    float beta1, beta2, eps;
} ddgs_fit_opts;
void ddgs_default_fit_options(ddgs_fit_opts *opts, float scene_extent_mm);
ddgs_status ddgs_set_fit_optimizer(ddgs_ctx *ctx, const ddgs_fit_opts *opts);

/* Densification statistics: device [n] floats owned by the caller
 * (borrowed; zero them to start).  Every backward, plain or captured, adds
 * for each Gaussian visible in a view (non-empty tile rectangle) the norm of
 * its 2D-mean gradient in normalised device units (pixel gradient times W/2
 * and H/2) to grad_accum and 1 to count, and raises max_radius to its
 * projected radius kappa sqrt(lambda_max(Sigma^)) in pixels.  NULL arrays
 * turn the accumulation off.  Drops a captured step. */
ddgs_status ddgs_set_densify_stats(ddgs_ctx *ctx, float *grad_accum, float *count, float *max_radius);

/* Densification of the current model from the statistics, in two calls.
 * ddgs_densify_plan decides on the device, for every Gaussian: mean
 * gradient a = grad_accum / count (0 if count is 0), s = largest log-scale;
 * a >= grad_threshold and s <= log(dense_scale): clone (exact copy added);
 * a >= grad_threshold and s > log(dense_scale): split (the parent is replaced
 * by two children at mu + R(q) diag(exp(log_scale)) eps_c, eps_c = noise[i][c]
 * (device [n][2][3], N(0, 1) draws supplied by the caller, read by
 * ddgs_densify_apply), log-scales lowered by log(split_factor)).  Then every
 * resulting Gaussian is dropped if sigmoid(opacity_logit) < min_opacity, or
 * if max_world_scale > 0 and its largest scale exceeds it, or -- originals
 * only -- if max_screen_radius > 0 and max_radius exceeds it.  Thresholds
 * are compared in float32 against float32 images of log(dense_scale),
 * logit(min_opacity), log(max_world_scale) and log(split_factor) formed in
 * double.  It synchronises and returns the new counts.
 * ddgs_densify_apply writes the new model into caller-allocated device
 * arrays of n_new Gaussians (out; b_iso and B_dir are copied), ordered per
 * set -- isotropic then directional -- as kept originals, clones, children,
 * each in parent order, and re-lays out the optimiser moments (zero for new
 * Gaussians).  The caller then sets the new model with ddgs_set_model. */
typedef struct ddgs_densify_opts {
    float grad_threshold;      /* 2e-4 (normalised device units)             */
    float dense_scale;         /* mm; 3DGS: 0.01 x scene extent              */
    float min_opacity;         /* 0.005                                      */
    float max_world_scale;     /* mm; 3DGS: 0.1 x scene extent; <= 0: off    */
    float max_screen_radius;   /* px; 3DGS: 20 after the first opacity reset */
    float split_factor;        /* 1.6                                        */
} ddgs_densify_opts;
typedef struct ddgs_params {
    float *mean, *quat, *log_scale, *opacity_logit, *feat, *b_iso, *B_dir;
} ddgs_params;
ddgs_status ddgs_densify_plan(ddgs_ctx *ctx, const ddgs_densify_opts *opts, const float *noise,
                              int64_t *n_new, int64_t *n_iso_new);
ddgs_status ddgs_densify_apply(ddgs_ctx *ctx, const ddgs_params *out);

/* Opacity reset: opacity_logit = min(opacity_logit, logit(max_alpha)) in
 * place, and the opacity moments are zeroed. */
ddgs_status ddgs_fit_reset_opacity(ddgs_ctx *ctx, float max_alpha);

/* Initialisation by radiodensity-aware dual sampling (Sec. 3.3; level and
 * set sizes of Sec. 4.1), in two calls.
 * ddgs_rads_prepare reads a CT volume and finds (synchronising):
 *   - the interface level (min + max) / 2 of the volume (*level);
 *   - every point where that level crosses an edge between neighbouring
 *     voxel centres, linearly interpolated -- the vertex set marching cubes
 *     places -- in edge order ((z ny + y) nx + x) 3 + axis, axes x, y, z
 *     (*n_crossings = M); an edge crosses when exactly one end is below the
 *     level;
 *   - the voxel weights floor((hu - min) / (max - min) * 65535) (float32
 *     arithmetic) and their total (*total_weight = W).
 * The volume may be freed after it returns.
 * ddgs_rads_sample writes N = min(n1, M) + n2 points, device [3][N]:
 *   - P^mc: the min(n1, M) crossings with the smallest mc_keys (device [M]
 *     u32, random keys supplied by the caller; ties by edge order), in key
 *     order;
 *   - P^dw: n2 voxel centres, draw j picking the first voxel whose inclusive
 *     weight sum exceeds dw_draws[j] (device [n2] u64, uniform in [0, W)
 *     supplied by the caller; a draw >= W picks the last voxel).
 * P^mc and the first n2 / 2 draws form the isotropic set, the rest the
 * directional one: *n_iso = min(n1, M) + n2 / 2.  log_scale (device [3][N],
 * may be NULL) receives log sqrt(mean squared distance to the three nearest
 * other points) on every axis, the mean clamped below at 1e-7 mm^2 (the
 * initial scales of 3D Gaussian splatting). */
typedef struct ddgs_volume {
    int32_t nx, ny, nz;          /* voxels; nx ny nz < 2^30                   */
    float spacing[3];            /* voxel size along x, y, z, mm (> 0)         */
    float origin[3];             /* world position of the centre of voxel
                                    (0, 0, 0), mm                             */
    const float *hu;             /* device [nz][ny][nx] radiodensity, HU      */
} ddgs_volume;
ddgs_status ddgs_rads_prepare(ddgs_ctx *ctx, const ddgs_volume *vol, float *level, int64_t *n_crossings,
                              uint64_t *total_weight);
ddgs_status ddgs_rads_sample(ddgs_ctx *ctx, int64_t n1, const uint32_t *mc_keys, int64_t n2, const uint64_t *dw_draws,
                             float *points, float *log_scale, int64_t *n_iso);

/* Test hook: radiosity c per (view, Gaussian), device [n_views][n] floats,
 * used instead of Eq. 3 (NULL restores Eq. 3).  With it the image is linear
 * in c (Eq. 1), and the backward leaves the features and bases out of the
 * chain (their gradients are zero).  Borrowed like the model arrays; the
 * caller keeps it sized for the current views.  Drops a captured step. */
ddgs_status ddgs_set_radiosity_override(ddgs_ctx *ctx, const float *c);
/* Pose composition used for a non-zero pose tangent: out = Exp(delta) pose,
 * i.e. R' = Exp(omega) R and t' = Exp(omega) t + rho for delta = (rho,
 * omega) (mm, rad; the left tangent the backward differentiates), evaluated
 * in float64 from the float32 pose and rounded once to float32.  Exp is the
 * rotation-vector exponential (Rodrigues' formula).  Host arrays; out may
 * alias pose.  Needs no context. */
ddgs_status ddgs_compose_pose(const float pose[12], const double delta[6], float out[12]);
/* Number of floats of the concatenated images of the current views. */
ddgs_status ddgs_image_size(const ddgs_ctx *ctx, int64_t *n_floats);

/* Device workspace.  By default the library allocates its workspace (tile
 * lists, records, sort temporaries, gradient slots, ...) with hipMalloc and
 * grows it on demand.  ddgs_set_workspace hands it a caller-owned device
 * region instead (e.g. a torch byte tensor; 256-byte aligned; the caller
 * keeps it alive and unchanged until the next ddgs_set_workspace or
 * ddgs_destroy): every workspace buffer is then carved from that region, and
 * a call that needs more than is left fails with DDGS_ERR_OOM and leaves the
 * device untouched.  NULL returns to library-owned allocation.  Either way
 * the previous workspace, any captured step and the last render are
 * dropped.  ddgs_workspace_size reports the bytes needed for the current
 * model, views and options with room for `capacity` tile entries (<= 0: the
 * option's capacity, else the last render's count); ddgs_autotune and the
 * debug getters need more for their own trial buffers. */
ddgs_status ddgs_set_workspace(ddgs_ctx *ctx, void *dev, size_t bytes);
ddgs_status ddgs_workspace_size(ddgs_ctx *ctx, int64_t capacity, size_t *bytes);

/* Caller allocator for the workspace buffers.  alloc(user, bytes) returns a
 * device pointer on the context's device, at least 256-byte aligned, valid
 * until free(user, ptr) (NULL: out of memory -> DDGS_ERR_OOM); it is called
 * only from inside the library's entry points on the calling host thread,
 * never while a stream capture is open.  A buffer is freed when it grows
 * (after the context's stream has been synchronised), by
 * ddgs_set_allocator / ddgs_set_workspace and by ddgs_destroy.  The caller's
 * allocator may hand the memory of a freed buffer to later work on the same
 * stream (a stream-ordered caching allocator such as torch's).  alloc NULL
 * returns to hipMalloc.  Like ddgs_set_workspace, the call drops the previous
 * workspace, any captured step and the last render; it takes precedence over
 * a caller region set earlier (which it drops). */
typedef void *(*ddgs_alloc_fn)(void *user, size_t bytes);
typedef void (*ddgs_free_fn)(void *user, void *ptr);
ddgs_status ddgs_set_allocator(ddgs_ctx *ctx, ddgs_alloc_fn alloc, ddgs_free_fn free_fn, void *user);

/* ---------------------------------------------------------------- compute */

/* Renders every view (Eq. 1 with Eq. 3) into images (device,
 * ddgs_image_size floats).  Reads the number of tile entries back to size
 * the sort (one stream synchronisation).  Keeps what the backward needs
 * (the sorted tile lists, per-pixel final value and last contributor). */
ddgs_status ddgs_render(ddgs_ctx *ctx, float *images);

/* Gradient of L = sum_p dL_dimages[p] I(p) with respect to the model and the
 * view poses; the transmittance is recomputed from the saved tile lists.
 * Requires a preceding ddgs_render with the same model, views and options
 * (DDGS_ERR_STATE otherwise). */
ddgs_status ddgs_backward(ddgs_ctx *ctx, const float *dL_dimages, const ddgs_grads *grads);

/* Eq. 2 losses of the current images against target (same layout):
 *   DDGS_LOSS_L1_DSSIM: per view (1-lambda) mean|I-I*| + lambda (1 - SSIM),
 *     SSIM with an 11x11 Gaussian window of std 1.5, K1 = 0.01, K2 = 0.03,
 *     dynamic range 1, zero padding;
 *   DDGS_LOSS_NCC: per view 1 - NCC over all pixels (population statistics,
 *     1e-12 added to each variance);
 *   DDGS_LOSS_LINEAR: sum_p target[p] I(p) (target holds the weights).
 * loss_out: device [n_views] floats (may be NULL); dL_dimages: device, image
 * layout, overwritten with the gradient (may be NULL). */
ddgs_status ddgs_loss(ddgs_ctx *ctx, int kind, const float *images, const float *target,
                      float lambda, float *loss_out, float *dL_dimages);

/* ------------------------------------------------------- batched step */

/* Records render -> loss -> backward of all views as one HIP graph with a
 * fixed tile-entry capacity (options.capacity, or twice the current need)
 * and no host synchronisation inside.  The pointers passed here are baked
 * into the graph and must stay valid.  ddgs_step_launch replays it;
 * ddgs_check synchronises and reports DDGS_ERR_CAPACITY if any replay (or
 * render) since the previous ddgs_check overflowed, and clears that flag.
 * The images, loss values and gradients of an overflowed replay are invalid,
 * and from the first overflowed replay until that ddgs_check every replay
 * leaves the optimiser state alone: the appended pose and fitting Adam steps
 * and the densification statistics are skipped (parameters, poses, moments
 * and step counts unchanged), so an overflowed replay can be run again.
 * The model and views may change contents between replays but not shapes
 * (n, views' W/H); ddgs_set_model / ddgs_set_views with a different shape
 * drop the graph.
 *
 * Retry after DDGS_ERR_CAPACITY: ddgs_step_report returns what the last
 * ddgs_check found -- the number of replays whose updates were skipped
 * (always the last ones launched before that check) and the largest number
 * of tile entries any replay since the previous check needed.  The caller
 * raises options.capacity above that need (ddgs_set_options), captures the
 * step again (the optimiser moments and step counts are kept) and replays the
 * skipped iterations again, in the same order. */
ddgs_status ddgs_step_capture(ddgs_ctx *ctx, int loss_kind, const float *target, float lambda,
                              float *images, float *dL_dimages, float *loss_out,
                              const ddgs_grads *grads);
ddgs_status ddgs_step_launch(ddgs_ctx *ctx);
/* Sets the target image the captured step's loss reads from the next replay
 * on (Eq. 2 fitting target, NCC reference or linear-loss weights; device
 * memory in the image layout of the current views, caller-owned, 4-byte
 * aligned, and left unchanged until the replays that read it have run).  A
 * fitting loop over many poses keeps every target resident and passes the
 * current one here instead of copying it into the captured buffer; the
 * pointer travels with the view table's upload (no copy of the image).
 * DDGS_ERR_STATE without a captured step, DDGS_ERR_INVALID_ARG for NULL or
 * misaligned pointers. */
ddgs_status ddgs_step_set_target(ddgs_ctx *ctx, const float *target);
ddgs_status ddgs_check(ddgs_ctx *ctx, uint32_t *flags);
ddgs_status ddgs_step_report(const ddgs_ctx *ctx, int64_t *skipped_replays, int64_t *entries_needed);

/* Times forward + backward (median of `repeats` after one warm-up call) on
 * the current model and views and selects the fastest raster options.  Each
 * candidate's kernels (projection to projection backward, as a captured step
 * runs them) are captured into a graph of the tuner's own and replayed, so
 * that the plain render's host round trip is not timed (on the default
 * stream, which cannot be captured, plain render + backward calls are timed
 * instead).  Like any ddgs_set_options call it drops a captured step;
 * the step counters that ddgs_check reads are kept.  First
 * every tile shape (16x16, 8x8, 16x8, 32x8; the waves per tile and the LDS
 * batch follow from the shape: one pixel per lane, one staged record per
 * pixel) with split 128, 256, 1024 and 0, one workgroup per item; then, at
 * the best shape, split 64, 128, 256, 512, 1024, 2048, 4096 and 0 with
 * persistent 0, 1, 2 and 4.  Images of candidates with split 0 are bit-identical; chunked ones
 * differ only by rounding.  If cache_path is not NULL, a JSON cache keyed by
 * the workload signature (device architecture, Gaussian-count bucket, k, L,
 * footprint bucket -- tile entries per (view, Gaussian) at 16x16 tiles, in
 * half octaves -- and the detector mix) is read first and written after.
 * best_ms (may be NULL) receives the chosen candidate's median time. */
ddgs_status ddgs_autotune(ddgs_ctx *ctx, const char *cache_path, int repeats, float *best_ms);

/* ------------------------------------------------------------- inspection */

/* Per-Gaussian float count (position 3, rotation 4, scale 3, opacity 1,
 * features k) and shared float count (k + k_L k); Sec. 4.2 counts 19 and 32
 * at k = 8, L = 1. */
ddgs_status ddgs_param_count(int k, int L, int64_t n, int64_t *per_gaussian, int64_t *shared);

/* Number of (tile, Gaussian) entries of the last render. */
ddgs_status ddgs_num_rendered(const ddgs_ctx *ctx, int64_t *n);

enum {
    DDGS_DBG_RECORDS = 0,     /* [n_views*n][8] f32: mu^x, mu^y, A00, A01, A11, alpha, c, 0 */
    DDGS_DBG_DEPTH_KEYS = 1,  /* [n_views*n] u32: float bits of z, 0xFFFFFFFF if culled */
    DDGS_DBG_COUNTS = 2,      /* [n_views*n] u32: tiles kept (see TILE_MASKS)    */
    DDGS_DBG_RECTS = 3,       /* [n_views*n][4] u16: tile x0, y0, x1, y1 (incl.)   */
    DDGS_DBG_TILE_KEYS_UNSORTED = 4, /* [M] u32 global tile id, emission order  */
    DDGS_DBG_TILE_VALS_UNSORTED = 5, /* [M] u32 Gaussian index, emission order  */
    DDGS_DBG_TILE_KEYS = 6,   /* [M] u32 sorted                                  */
    DDGS_DBG_TILE_VALS = 7,   /* [M] u32 sorted                                  */
    DDGS_DBG_RANGES = 8,      /* [n_tiles][2] u32 [start, end)                   */
    DDGS_DBG_NLAST = 9,       /* [pixels] u32: end of the contributing prefix    */
    DDGS_DBG_TILE_BASE = 10,  /* [n_views+1] i32: first global tile id per view  */
    DDGS_DBG_FIT_MOMENTS = 11, /* [2][n(11+k) + k + k_L k] f32: Adam first, then
                                  second moments, groups in model order      */
    DDGS_DBG_TILE_MASKS = 12  /* [n_views*n] u32: tiles of the rectangle the
                                 cut-off ellipse reaches, bit b = row-major
                                 place b, for rectangles of at most 32 tiles
                                 (larger ones keep every tile: 0xFFFFFFFF);
                                 a tile is kept when the least d^T A d over
                                 its pixel centres (the centres' box) is at
                                 most 1.001 kappa^2 */
};
/* Copies an internal array of the last render to host memory (synchronises).
 * The *_UNSORTED arrays are kept only when options are set with
 * ddgs_debug_keep_unsorted(ctx, 1) before the render. */
ddgs_status ddgs_debug_copy(ddgs_ctx *ctx, int what, void *host, size_t bytes);
ddgs_status ddgs_debug_keep_unsorted(ddgs_ctx *ctx, int keep);

/* Stable LSD radix sort of n (key, value) u32 pairs in place on the device,
 * by key bits [0, bits) (bits 1..32).  Exposes the sort that orders the
 * tile lists. */
ddgs_status ddgs_debug_sort_pairs(ddgs_ctx *ctx, uint32_t *keys, uint32_t *vals, int64_t n, int bits);

/* The radix sort of ddgs_debug_sort_pairs without any allocation, for callers
 * that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid it): its temporaries (the ping-pong
 * halves and the digit counts) live in a static device array of 12 MiB that
 * each GPU holds for the life of the process, so n is limited to 2^20 pairs
 * (larger n: DDGS_ERR_INVALID_ARG, nothing enqueued).  Same result as
 * ddgs_debug_sort_pairs (stable by key bits [0, bits), in place); the work is
 * enqueued on the context's stream without synchronising.  Every call on one
 * GPU shares that array, so calls that overlap on a GPU (other streams, other
 * threads or contexts) race; the array holds the last call's temporaries and
 * needs no clearing between calls. */
ddgs_status ddgs_sort_pairs_noalloc(ddgs_ctx *ctx, uint32_t *keys, uint32_t *vals, int64_t n, int bits);

/* Exclusive prefix sum of n u32 values on the device; *total receives the
 * 64-bit sum (host).  Exposes the scan that places the tile entries. */
ddgs_status ddgs_debug_exclusive_scan(ddgs_ctx *ctx, const uint32_t *in, uint32_t *out, int64_t n,
                                      uint64_t *total);

/* Pair statistics of the forward raster: once enabled, every render counts
 * the (pixel, tile entry) pairs it evaluated and the pairs that contributed
 * to Eq. 1 (inside the cut-off radius, before any early stop).  The counts
 * of the last render are returned by ddgs_debug_pair_counts. */
ddgs_status ddgs_debug_count_pairs(ddgs_ctx *ctx, int enable);
ddgs_status ddgs_debug_pair_counts(ddgs_ctx *ctx, int64_t *evaluated, int64_t *contributing);

/* Device time of the last render/backward per stage, ms (filled when timing
 * is enabled with ddgs_enable_timing; captured steps are not timed).  The
 * sort stage is the sum of its two parts: between them a render reads the
 * entry total back to the host, which is not device work. */
enum { DDGS_T_PROJECT = 0, DDGS_T_SORT = 1, DDGS_T_RASTER_FWD = 2, DDGS_T_LOSS = 3,
       DDGS_T_RASTER_BWD = 4, DDGS_T_PROJECT_BWD = 5, DDGS_T_COUNT = 6 };
ddgs_status ddgs_enable_timing(ddgs_ctx *ctx, int enable);
ddgs_status ddgs_stage_times(const ddgs_ctx *ctx, float *ms /* [DDGS_T_COUNT] */);

#ifdef __cplusplus
}
#endif
#endif
