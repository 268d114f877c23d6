/*
 * ddgs_oracle.h -- plain CPU FP64 reference of the DDGS-CT DRR splatting
 * renderer (arXiv 2406.02518).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU path; it
 * shares no code, header, table or constant with it.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it.  The
 * product path never calls it and has no CPU fallback.
 *
 * What it computes (every pixel against every Gaussian, no tiling, FP64):
 *   - Sec. 3.1, Eq. 1: front-to-back alpha compositing
 *       C(p) = sum_j c_j s_j prod_{l<j} (1 - s_l),
 *       s_j = alpha_j exp(-1/2 (p - mu^_j)^T Sigma^_j^-1 (p - mu^_j))
 *     where mu^, Sigma^ are the image-plane projections of the 3D mean and
 *     covariance (the local-affine projection of 3D Gaussian splatting,
 *     which the paper inherits rather than restates).
 *   - Sec. 3.2, Eq. 3: radiosity c = sigmoid(b_iso . f) for the isotropic
 *     set and c = sigmoid(Y_{1..L}(dir) . (B_dir f)) for the
 *     direction-dependent set, with k_L = L(L+2) basis functions and no
 *     degree-0 term; or, for the co-located ablation, the sigmoid of the sum
 *     of both logits on every Gaussian.
 *   - App. A.2: both sets are composited jointly in one depth order.
 *   - App. A.1: transmittance is the running product of (1 - s).
 *   - Sec. 3.1, Eq. 2: the (1-lambda) L1 + lambda D-SSIM fitting loss, and a
 *     global normalised cross-correlation loss for pose scoring.
 * Readings of points the paper leaves open (cut-off radius, sigma clamp,
 * low-pass dilation, pixel-centre convention, depth key, spherical basis
 * sign convention) are fixed by the fields of orc_opts and documented at
 * each function below.
 *
 * All arrays are host memory owned by the caller.  Functions return 0 on
 * success and a negative number on invalid arguments; they never allocate
 * caller-visible memory.
 */
#ifndef DDGS_ORACLE_H
#define DDGS_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Gaussian set, structure of arrays.  Values are float32 numbers widened to
 * double (the depth key re-reads them as float, which is exact then).
 * Gaussians [0, n_iso) are isotropic, [n_iso, n) direction-dependent.
 * entangled = 1 is the co-located ablation of Sec. 4 ("direct-entangled"):
 * every Gaussian carries both terms under one sigmoid,
 * c = sigmoid(b_iso . f + Y_{1..L}(dir) . (B_dir f)); it needs n_iso = 0. */
typedef struct {
    int64_t n, n_iso;
    int32_t k, L;
    const double *mean;          /* [3][n] world mm                          */
    const double *quat;          /* [4][n] (w,x,y,z), any non-zero norm      */
    const double *log_scale;     /* [3][n] log of per-axis std, mm           */
    const double *opacity_logit; /* [n]    alpha = sigmoid(.)                */
    const double *feat;          /* [k][n]                                   */
    const double *b_iso;         /* [k]                                      */
    const double *B_dir;         /* [k_L][k] row-major                       */
    int32_t entangled;           /* 0: Eq. 3 as printed; 1: co-located        */
} orc_model;

/* Cone-beam view.  pose = [R | t] row-major 3x4, world -> source frame:
 * +z along the principal ray towards the detector, +x along detector
 * columns, +y along detector rows.  Focal length f = sdd/pitch pixels,
 * principal point at (W/2, H/2), pixel (u, v) has centre (u+.5, v+.5). */
typedef struct {
    int32_t W, H;
    double pitch_mm, sdd_mm;
    double pose[12];
} orc_view;

typedef struct {
    double kappa;      /* Mahalanobis cut-off radius (3)                      */
    double dilation;   /* added to the projected covariance diagonal (0.3)   */
    double t_min;      /* stop when T(1-s) < t_min; 0 disables (0)           */
    double z_near;     /* cull when depth key <= z_near, mm (1)              */
    double sigma_max;  /* s = min(sigma_max, alpha G) (0.99)                 */
    const double *c_override; /* [V][n] radiosity replacing Eq. 3, or NULL  */
} orc_opts;

typedef struct {
    double *dmean;          /* [3][n] */
    double *dquat;          /* [4][n] */
    double *dlog_scale;     /* [3][n] */
    double *dopacity_logit; /* [n]    */
    double *dfeat;          /* [k][n] */
    double *db_iso;         /* [k]    */
    double *dB_dir;         /* [k_L][k] */
    double *dpose;          /* [V][6]: (rho, omega), left tangent at 0      */
    double *dc;             /* [V][n] gradient w.r.t. the radiosity c (opt) */
    double *g2d;            /* [V][n][7] image-plane gradients (optional):
                               d mu^x, d mu^y, d A00, d A01, d A11,
                               d alpha, d c                                 */
} orc_grads;

int orc_kl(int L);
void orc_param_count(int k, int L, int64_t n, int64_t *per_gaussian,
                     int64_t *shared, int64_t *total);

/* Real orthonormal spherical basis of degrees 1..L (L <= 3), Cartesian,
 * order l = 1..L, m = -l..l, no Condon-Shortley phase.  dY (k_L x 3, may be
 * NULL) is the gradient of each polynomial with respect to d. */
int orc_sh(int L, const double d[3], double *Y, double *dY);

/* Rotation matrix of q / |q|, row-major. */
void orc_quat_to_rot(const double q[4], double R[9]);

/* Per-Gaussian projection for one view.  out is [n][ORC_PROJ_COLS]:
 * valid, mu^x, mu^y, A00, A01, A11, alpha, c, zkey, S00, S01, S11, z */
#define ORC_PROJ_COLS 13
int orc_project(const orc_model *m, const orc_view *v, int view_index,
                const orc_opts *o, double *out);

/* Full images, view-major concatenation of H*W rows.  contrib_hash[v] is an
 * order-independent hash of the set of contributing (pixel, Gaussian)
 * pairs and n_contrib[v] their count (both optional). */
int orc_render(const orc_model *m, const orc_view *views, int V,
               const orc_opts *o, double *img, uint64_t *contrib_hash,
               int64_t *n_contrib, int threads);

/* Selected pixels: pix is [npix][3] = (view, u, v). */
int orc_render_pixels(const orc_model *m, const orc_view *views, int V,
                      const orc_opts *o, int64_t npix, const int32_t *pix,
                      double *out, int threads);

/* Distance of each listed pixel from the decisions Eq. 1 takes there, as
 * the smallest relative gap over its Gaussians of: |d2 - kappa^2| / kappa^2
 * (the cutoff), |alpha G - sigma_max| / sigma_max for considered Gaussians
 * (the clamp) and, with t_min > 0, |T (1 - s) - t_min| / t_min (the early
 * stop).  A pixel whose margin is within rounding of 0 has more than one
 * correct set of contributors at a given working precision. */
int orc_pixel_margins(const orc_model *m, const orc_view *views, int V,
                      const orc_opts *o, int64_t npix, const int32_t *pix,
                      double *margin, int threads);

/* Analytic gradient of L = sum_p g_p I(p) over the listed pixels
 * (pix [npix][3] = (view, u, v), g [npix]).  Every non-NULL output is
 * overwritten. */
int orc_backward(const orc_model *m, const orc_view *views, int V,
                 const orc_opts *o, int64_t npix, const int32_t *pix,
                 const double *g, const orc_grads *out, int threads);

/* Eq. 2 with the D-SSIM reading: L = (1-lambda) mean|x-y| +
 * lambda (1 - mean SSIM(x, y)); 11x11 Gaussian window, std 1.5, K1 = 0.01,
 * K2 = 0.03, dynamic range 1, zero padding.  grad = dL/dx (may be NULL). */
int orc_loss_l1ssim(const double *x, const double *y, int W, int H,
                    double lambda, double *loss, double *ssim_mean,
                    double *grad);

/* L = 1 - NCC(x, y), NCC over all P pixels with population statistics and
 * eps added to both variances.  grad = dL/dx (may be NULL). */
int orc_loss_ncc(const double *x, const double *y, int64_t P, double eps,
                 double *loss, double *grad);

#ifdef __cplusplus
}
#endif
#endif
