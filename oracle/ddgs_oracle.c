/*
 * ddgs_oracle.c -- plain CPU FP64 reference of the DDGS-CT DRR renderer.
 *
 * TEST INFRASTRUCTURE ONLY (see ddgs_oracle.h).  Slow and direct on purpose:
 * every pixel is tested against every projected Gaussian in depth order,
 * with no tiling, binning or early culling beyond the definition itself.
 *
 * Paper passages followed (arXiv 2406.02518):
 *   Sec. 3.1 Eq. 1  compositing and the per-pixel opacity s_j
 *   Sec. 3.1 Eq. 2  fitting loss (read with D-SSIM, lambda = 0.2)
 *   Sec. 3.2 Eq. 3  dual radiosity, k_L = L(L+2), no degree-0 term
 *   App. A.1 Eq. S2 transmittance as a product of (1 - s)
 *   App. A.2        joint compositing of the isotropic and directional sets
 *   Sec. 4 (registration) gradients with respect to the source pose
 * The projection of mean and covariance to the detector is the local-affine
 * (EWA) projection of 3D Gaussian splatting, which Eq. 1 refers to as the
 * image-plane projections of mu and Sigma.
 */
#include "ddgs_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXKL 15

static double sigmoid(double x) { return 1.0 / (1.0 + exp(-x)); }

int orc_kl(int L) { return L * (L + 2); }

/* Sec. 4.2 / Table 1 discussion: 19 floats per Gaussian at k = 8 (position 3,
 * rotation 4, scale 3, opacity 1, features k) and a shared basis of
 * k + k_L k floats (32 at k = 8, L = 1). */
void orc_param_count(int k, int L, int64_t n, int64_t *per_gaussian,
                     int64_t *shared, int64_t *total)
{
    int64_t per = 3 + 4 + 3 + 1 + (int64_t)k;
    int64_t sh = (int64_t)k + (int64_t)orc_kl(L) * k;
    if (per_gaussian) *per_gaussian = per;
    if (shared) *shared = sh;
    if (total) *total = per * n + sh;
}

/* Real orthonormal spherical harmonics without Condon-Shortley phase, written
 * as polynomials in the unit direction d = (x, y, z).  Degree 0 is absent
 * (Sec. 3.2: "without constant term"). */
int orc_sh(int L, const double d[3], double *Y, double *dY)
{
    if (L < 1 || L > 3) return -1;
    const double x = d[0], y = d[1], z = d[2];
    const double pi = M_PI;
    const double c1 = sqrt(3.0 / (4.0 * pi));
    double v[ORC_MAXKL], g[ORC_MAXKL][3];
    memset(g, 0, sizeof(g));
    /* l = 1: m = -1, 0, 1 */
    v[0] = c1 * y;  g[0][1] = c1;
    v[1] = c1 * z;  g[1][2] = c1;
    v[2] = c1 * x;  g[2][0] = c1;
    if (L >= 2) {
        const double a = 0.5 * sqrt(15.0 / pi);
        const double b = 0.25 * sqrt(5.0 / pi);
        const double c = 0.25 * sqrt(15.0 / pi);
        v[3] = a * x * y;                 g[3][0] = a * y; g[3][1] = a * x;
        v[4] = a * y * z;                 g[4][1] = a * z; g[4][2] = a * y;
        v[5] = b * (3.0 * z * z - 1.0);   g[5][2] = 6.0 * b * z;
        v[6] = a * x * z;                 g[6][0] = a * z; g[6][2] = a * x;
        v[7] = c * (x * x - y * y);       g[7][0] = 2.0 * c * x; g[7][1] = -2.0 * c * y;
    }
    if (L >= 3) {
        const double a = 0.25 * sqrt(35.0 / (2.0 * pi));
        const double b = 0.5 * sqrt(105.0 / pi);
        const double c = 0.25 * sqrt(21.0 / (2.0 * pi));
        const double e = 0.25 * sqrt(7.0 / pi);
        const double h = 0.25 * sqrt(105.0 / pi);
        v[8] = a * y * (3.0 * x * x - y * y);
        g[8][0] = 6.0 * a * x * y; g[8][1] = 3.0 * a * (x * x - y * y);
        v[9] = b * x * y * z;
        g[9][0] = b * y * z; g[9][1] = b * x * z; g[9][2] = b * x * y;
        v[10] = c * y * (5.0 * z * z - 1.0);
        g[10][1] = c * (5.0 * z * z - 1.0); g[10][2] = 10.0 * c * y * z;
        v[11] = e * z * (5.0 * z * z - 3.0);
        g[11][2] = e * (15.0 * z * z - 3.0);
        v[12] = c * x * (5.0 * z * z - 1.0);
        g[12][0] = c * (5.0 * z * z - 1.0); g[12][2] = 10.0 * c * x * z;
        v[13] = h * z * (x * x - y * y);
        g[13][0] = 2.0 * h * x * z; g[13][1] = -2.0 * h * y * z; g[13][2] = h * (x * x - y * y);
        v[14] = a * x * (x * x - 3.0 * y * y);
        g[14][0] = 3.0 * a * (x * x - y * y); g[14][1] = -6.0 * a * x * y;
    }
    const int kl = orc_kl(L);
    for (int m = 0; m < kl; ++m) {
        Y[m] = v[m];
        if (dY) { dY[3 * m] = g[m][0]; dY[3 * m + 1] = g[m][1]; dY[3 * m + 2] = g[m][2]; }
    }
    return 0;
}

void orc_quat_to_rot(const double q[4], double R[9])
{
    const double nq = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    const double w = q[0] / nq, x = q[1] / nq, y = q[2] / nq, z = q[3] / nq;
    R[0] = 1.0 - 2.0 * (y * y + z * z); R[1] = 2.0 * (x * y - w * z);       R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);       R[4] = 1.0 - 2.0 * (x * x + z * z); R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);       R[7] = 2.0 * (y * z + w * x);       R[8] = 1.0 - 2.0 * (x * x + y * y);
}

/* ---------------------------------------------------------------- projection */

typedef struct {
    int valid;
    float zkey;
    double muc[3];           /* source-frame mean                             */
    double Rq[9], sc[3];     /* rotation of the unit quaternion, std per axis */
    double qn[4], qnorm;     /* unit quaternion and the norm of the raw one   */
    double Sw[9], Sc[9];     /* world and source-frame covariance             */
    double J[6];             /* 2x3 Jacobian of the pinhole map at muc        */
    double S2[3];            /* projected covariance + dilation (00, 01, 11)  */
    double A[3];             /* conic = inverse of S2 (00, 01, 11)            */
    double m2[2];            /* projected mean, pixels                        */
    double alpha, c, zl;     /* opacity, radiosity, radiosity logit           */
    double dir[3], rlen;     /* unit direction source -> mean, distance       */
    double Y[ORC_MAXKL], h[ORC_MAXKL];
} gproj;

typedef struct { double mx, my, A0, A1, A2, alpha, c; } gfast;

static void mat3_mul(const double *a, const double *b, double *o)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += a[3 * i + k] * b[3 * k + j];
            o[3 * i + j] = s;
        }
}
static void mat3_transpose(const double *a, double *o)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) o[3 * j + i] = a[3 * i + j];
}

/* The depth key: the source-frame z of the mean evaluated in float32 as a
 * chain of fused multiply-adds, z = R20 x + (R21 y + (R22 z + t2)).  The
 * ordering of Gaussians along each ray (Eq. 1: "the j-th Gaussian on the
 * ray") is an integer decision, so it is taken in the GPU kernel's precision;
 * ties are broken by the Gaussian index. */
static float depth_key(const double *pose, double mx, double my, double mz)
{
    float t = fmaf((float)pose[10], (float)mz, (float)pose[11]);
    t = fmaf((float)pose[9], (float)my, t);
    t = fmaf((float)pose[8], (float)mx, t);
    return t;
}

static void project_one(const orc_model *m, const orc_view *v, int vi,
                        const orc_opts *o, int64_t i, gproj *g)
{
    const int64_t n = m->n;
    const double *P = v->pose;
    const double R[9] = {P[0], P[1], P[2], P[4], P[5], P[6], P[8], P[9], P[10]};
    const double t[3] = {P[3], P[7], P[11]};
    const double mu[3] = {m->mean[i], m->mean[n + i], m->mean[2 * n + i]};
    memset(g, 0, sizeof(*g));
    g->zkey = depth_key(P, mu[0], mu[1], mu[2]);
    if (!(g->zkey > (float)o->z_near)) { g->valid = 0; return; }

    for (int r = 0; r < 3; ++r)
        g->muc[r] = R[3 * r] * mu[0] + R[3 * r + 1] * mu[1] + R[3 * r + 2] * mu[2] + t[r];

    /* Sigma = Rq diag(s^2) Rq^T with s = exp(log_scale) */
    const double q[4] = {m->quat[i], m->quat[n + i], m->quat[2 * n + i], m->quat[3 * n + i]};
    g->qnorm = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int r = 0; r < 4; ++r) g->qn[r] = q[r] / g->qnorm;
    orc_quat_to_rot(q, g->Rq);
    for (int r = 0; r < 3; ++r) g->sc[r] = exp(m->log_scale[r * n + i]);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += g->Rq[3 * a + k] * g->sc[k] * g->sc[k] * g->Rq[3 * b + k];
            g->Sw[3 * a + b] = s;
        }
    /* Sigma_c = R Sigma R^T */
    double tmp[9], Rt[9];
    mat3_transpose(R, Rt);
    mat3_mul(R, g->Sw, tmp);
    mat3_mul(tmp, Rt, g->Sc);

    /* local-affine projection */
    const double f = v->sdd_mm / v->pitch_mm;
    const double x = g->muc[0], y = g->muc[1], z = g->muc[2];
    g->J[0] = f / z; g->J[1] = 0.0;   g->J[2] = -f * x / (z * z);
    g->J[3] = 0.0;   g->J[4] = f / z; g->J[5] = -f * y / (z * z);
    double JS[6];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 3; ++b) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += g->J[3 * a + k] * g->Sc[3 * k + b];
            JS[3 * a + b] = s;
        }
    double S2f[4];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += JS[3 * a + k] * g->J[3 * b + k];
            S2f[2 * a + b] = s;
        }
    g->S2[0] = S2f[0] + o->dilation;
    g->S2[1] = 0.5 * (S2f[1] + S2f[2]);
    g->S2[2] = S2f[3] + o->dilation;
    const double det = g->S2[0] * g->S2[2] - g->S2[1] * g->S2[1];
    if (!(det > 0.0)) { g->valid = 0; return; }
    g->A[0] = g->S2[2] / det;
    g->A[1] = -g->S2[1] / det;
    g->A[2] = g->S2[0] / det;
    g->m2[0] = f * x / z + 0.5 * v->W;
    g->m2[1] = f * y / z + 0.5 * v->H;
    g->alpha = sigmoid(m->opacity_logit[i]);

    /* Eq. 3 radiosity: the isotropic logit b_iso . f, the directional logit
     * Y(dir) . (B_dir f), or (co-located ablation) their sum */
    const int k = m->k, kl = orc_kl(m->L);
    if (o->c_override) {
        g->c = o->c_override[(int64_t)vi * n + i];
    } else {
        double s = 0.0;
        if (m->entangled || i < m->n_iso)
            for (int j = 0; j < k; ++j) s += m->b_iso[j] * m->feat[(int64_t)j * n + i];
        if (m->entangled || i >= m->n_iso) {
            /* source position s_o = -R^T t; ray direction source -> mean, world frame */
            double so[3];
            for (int r = 0; r < 3; ++r) so[r] = -(R[r] * t[0] + R[3 + r] * t[1] + R[6 + r] * t[2]);
            double rv[3] = {mu[0] - so[0], mu[1] - so[1], mu[2] - so[2]};
            g->rlen = sqrt(rv[0] * rv[0] + rv[1] * rv[1] + rv[2] * rv[2]);
            for (int r = 0; r < 3; ++r) g->dir[r] = rv[r] / g->rlen;
            orc_sh(m->L, g->dir, g->Y, NULL);
            for (int a = 0; a < kl; ++a) {
                double hv = 0.0;
                for (int j = 0; j < k; ++j) hv += m->B_dir[a * k + j] * m->feat[(int64_t)j * n + i];
                g->h[a] = hv;
                s += g->Y[a] * hv;
            }
        }
        g->zl = s;
        g->c = sigmoid(s);
    }
    g->valid = 1;
}

int orc_project(const orc_model *m, const orc_view *v, int view_index,
                const orc_opts *o, double *out)
{
    if (!m || !v || !o || !out || m->n < 0 || m->L < 1 || m->L > 3) return -1;
    for (int64_t i = 0; i < m->n; ++i) {
        gproj g;
        project_one(m, v, view_index, o, i, &g);
        double *r = out + i * ORC_PROJ_COLS;
        memset(r, 0, sizeof(double) * ORC_PROJ_COLS);
        r[0] = g.valid;
        r[8] = (double)g.zkey;
        if (!g.valid) continue;
        r[1] = g.m2[0]; r[2] = g.m2[1];
        r[3] = g.A[0]; r[4] = g.A[1]; r[5] = g.A[2];
        r[6] = g.alpha; r[7] = g.c;
        r[9] = g.S2[0]; r[10] = g.S2[1]; r[11] = g.S2[2];
        r[12] = g.muc[2];
    }
    return 0;
}

/* ------------------------------------------------------------ depth ordering */

typedef struct { float key; int64_t idx; } korder;

static int korder_cmp(const void *a, const void *b)
{
    const korder *x = (const korder *)a, *y = (const korder *)b;
    if (x->key < y->key) return -1;
    if (x->key > y->key) return 1;
    return (x->idx > y->idx) - (x->idx < y->idx);
}

/* Projects every Gaussian for one view and returns the valid ones sorted by
 * (depth key, index).  Caller frees *order_out, *gp_out, *fast_out. */
static int64_t prepare_view(const orc_model *m, const orc_view *v, int vi,
                            const orc_opts *o, gproj **gp_out, int64_t **order_out,
                            gfast **fast_out)
{
    const int64_t n = m->n;
    gproj *gp = (gproj *)malloc(sizeof(gproj) * (size_t)(n > 0 ? n : 1));
    korder *ko = (korder *)malloc(sizeof(korder) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) project_one(m, v, vi, o, i, &gp[i]);
    int64_t nv = 0;
    for (int64_t i = 0; i < n; ++i)
        if (gp[i].valid) { ko[nv].key = gp[i].zkey; ko[nv].idx = i; ++nv; }
    qsort(ko, (size_t)nv, sizeof(korder), korder_cmp);
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nv > 0 ? nv : 1));
    gfast *fast = (gfast *)malloc(sizeof(gfast) * (size_t)(nv > 0 ? nv : 1));
    for (int64_t j = 0; j < nv; ++j) {
        const gproj *g = &gp[ko[j].idx];
        order[j] = ko[j].idx;
        fast[j].mx = g->m2[0]; fast[j].my = g->m2[1];
        fast[j].A0 = g->A[0]; fast[j].A1 = g->A[1]; fast[j].A2 = g->A[2];
        fast[j].alpha = g->alpha; fast[j].c = g->c;
    }
    free(ko);
    *gp_out = gp; *order_out = order; *fast_out = fast;
    return nv;
}

/* ----------------------------------------------------------------- one pixel */

typedef struct { int64_t j; double s, T, G, dx, dy; int clamped; } contrib;

static uint64_t mix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Eq. 1 at pixel centre (px, py): Gaussians in depth order; a Gaussian
 * whose Mahalanobis distance exceeds kappa is not considered (leaves the
 * state untouched); s = min(sigma_max, alpha exp(-d2/2)); optional early
 * stop before a Gaussian that would push T below t_min. */
static double render_pixel(const gfast *fast, int64_t nv, double px, double py,
                           const orc_opts *o, contrib *list, int64_t *nlist,
                           const int64_t *order, uint64_t pixel_id, int64_t n,
                           uint64_t *hash, int64_t *count, double *margin)
{
    const double k2 = o->kappa * o->kappa;
    double T = 1.0, C = 0.0, mg = HUGE_VAL;
    int64_t nl = 0;
    for (int64_t j = 0; j < nv; ++j) {
        const gfast *g = &fast[j];
        const double dx = px - g->mx, dy = py - g->my;
        const double d2 = g->A0 * dx * dx + 2.0 * g->A1 * dx * dy + g->A2 * dy * dy;
        if (margin) mg = fmin(mg, fabs(d2 - k2) / k2);
        if (d2 > k2) continue;
        const double G = exp(-0.5 * d2);
        double s = g->alpha * G;
        if (margin) mg = fmin(mg, fabs(s - o->sigma_max) / o->sigma_max);
        int clamped = 0;
        if (s > o->sigma_max) { s = o->sigma_max; clamped = 1; }
        if (o->t_min > 0.0) {
            if (margin) mg = fmin(mg, fabs(T * (1.0 - s) - o->t_min) / o->t_min);
            if (T * (1.0 - s) < o->t_min) break;
        }
        if (list) {
            list[nl].j = j; list[nl].s = s; list[nl].T = T; list[nl].G = G;
            list[nl].dx = dx; list[nl].dy = dy; list[nl].clamped = clamped;
        }
        ++nl;
        if (hash) *hash += mix64(pixel_id * (uint64_t)(n + 1) + (uint64_t)order[j]);
        C += g->c * s * T;
        T *= (1.0 - s);
    }
    if (nlist) *nlist = nl;
    if (count) *count += nl;
    if (margin) *margin = mg;
    return C;
}

static int check_args(const orc_model *m, const orc_view *views, int V, const orc_opts *o)
{
    if (!m || !views || !o || V < 0 || m->n < 0) return -1;
    if (m->n_iso < 0 || m->n_iso > m->n) return -1;
    if (m->entangled != 0 && (m->entangled != 1 || m->n_iso != 0)) return -1;
    if (m->L < 1 || m->L > 3 || m->k < 1) return -1;
    for (int v = 0; v < V; ++v)
        if (views[v].W <= 0 || views[v].H <= 0 || !(views[v].pitch_mm > 0.0) || !(views[v].sdd_mm > 0.0))
            return -1;
    return 0;
}

int orc_render(const orc_model *m, const orc_view *views, int V,
               const orc_opts *o, double *img, uint64_t *contrib_hash,
               int64_t *n_contrib, int threads)
{
    if (check_args(m, views, V, o) || !img) return -1;
    if (threads < 1) threads = 1;
    int64_t base = 0;
    for (int v = 0; v < V; ++v) {
        gproj *gp; int64_t *order; gfast *fast;
        const int64_t nv = prepare_view(m, &views[v], v, o, &gp, &order, &fast);
        const int W = views[v].W, H = views[v].H;
        uint64_t hsum = 0; int64_t csum = 0;
#pragma omp parallel for schedule(dynamic, 1) num_threads(threads) reduction(+ : hsum, csum)
        for (int row = 0; row < H; ++row) {
            for (int col = 0; col < W; ++col) {
                uint64_t h = 0; int64_t c = 0;
                img[base + (int64_t)row * W + col] =
                    render_pixel(fast, nv, col + 0.5, row + 0.5, o, NULL, NULL, order,
                                 (uint64_t)row * W + col, m->n, &h, &c, NULL);
                hsum += h; csum += c;
            }
        }
        if (contrib_hash) contrib_hash[v] = hsum;
        if (n_contrib) n_contrib[v] = csum;
        base += (int64_t)W * H;
        free(gp); free(order); free(fast);
    }
    return 0;
}

static int render_pixels_impl(const orc_model *m, const orc_view *views, int V,
                              const orc_opts *o, int64_t npix, const int32_t *pix,
                              double *out, double *margin, int threads)
{
    if (check_args(m, views, V, o) || (npix > 0 && (!pix || (!out && !margin)))) return -1;
    for (int64_t p = 0; p < npix; ++p) {
        const int32_t v = pix[3 * p];
        if (v < 0 || v >= V || pix[3 * p + 1] < 0 || pix[3 * p + 1] >= views[v].W ||
            pix[3 * p + 2] < 0 || pix[3 * p + 2] >= views[v].H) return -1;
    }
    if (threads < 1) threads = 1;
    for (int v = 0; v < V; ++v) {
        int any = 0;
        for (int64_t p = 0; p < npix && !any; ++p) any = (pix[3 * p] == v);
        if (!any) continue;
        gproj *gp; int64_t *order; gfast *fast;
        const int64_t nv = prepare_view(m, &views[v], v, o, &gp, &order, &fast);
#pragma omp parallel for schedule(dynamic, 16) num_threads(threads)
        for (int64_t p = 0; p < npix; ++p) {
            if (pix[3 * p] != v) continue;
            const double c = render_pixel(fast, nv, pix[3 * p + 1] + 0.5, pix[3 * p + 2] + 0.5, o,
                                          NULL, NULL, order, 0, m->n, NULL, NULL,
                                          margin ? &margin[p] : NULL);
            if (out) out[p] = c;
        }
        free(gp); free(order); free(fast);
    }
    return 0;
}

int orc_render_pixels(const orc_model *m, const orc_view *views, int V,
                      const orc_opts *o, int64_t npix, const int32_t *pix,
                      double *out, int threads)
{
    return render_pixels_impl(m, views, V, o, npix, pix, out, NULL, threads);
}

int orc_pixel_margins(const orc_model *m, const orc_view *views, int V,
                      const orc_opts *o, int64_t npix, const int32_t *pix,
                      double *margin, int threads)
{
    return render_pixels_impl(m, views, V, o, npix, pix, NULL, margin, threads);
}

/* ------------------------------------------------------------------ backward */

/* cross-product matrix [a]x */
static void skew(const double a[3], double S[9])
{
    S[0] = 0.0;   S[1] = -a[2]; S[2] = a[1];
    S[3] = a[2];  S[4] = 0.0;   S[5] = -a[0];
    S[6] = -a[1]; S[7] = a[0];  S[8] = 0.0;
}

/* Chain rule from the image-plane gradient of one (view, Gaussian) pair to
 * the Gaussian's parameters, the shared bases and the view's pose tangent.
 * g7 = (d mu^x, d mu^y, d A00, d A01, d A11, d alpha, d c), where d A01 is
 * the derivative with respect to the single off-diagonal conic value. */
static void chain_one(const orc_model *m, const orc_view *v, const orc_opts *o,
                      int64_t i, const gproj *g, const double g7[7],
                      double gmu[3], double gq[4], double gls[3], double *gop,
                      double *gf /* [k] */, double *gb /* [k] */, double *gB /* [kl*k] */,
                      double gpose[6], double *gc_out)
{
    const int64_t n = m->n;
    const double *P = v->pose;
    const double R[9] = {P[0], P[1], P[2], P[4], P[5], P[6], P[8], P[9], P[10]};
    const double f = v->sdd_mm / v->pitch_mm;
    const double x = g->muc[0], y = g->muc[1], z = g->muc[2];

    /* conic A = S2^-1: dL/dS2 = -A Gbar A with Gbar the symmetric gradient */
    const double Gb[4] = {g7[2], 0.5 * g7[3], 0.5 * g7[3], g7[4]};
    const double A[4] = {g->A[0], g->A[1], g->A[1], g->A[2]};
    double AG[4], GS2[4];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) AG[2 * a + b] = A[2 * a] * Gb[b] + A[2 * a + 1] * Gb[2 + b];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) GS2[2 * a + b] = -(AG[2 * a] * A[b] + AG[2 * a + 1] * A[2 + b]);

    /* S2 = J Sc J^T + dilation I */
    double GSc[9], GJ[6], tmp[6];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double s = 0.0;
            for (int p = 0; p < 2; ++p)
                for (int q = 0; q < 2; ++q) s += g->J[3 * p + a] * GS2[2 * p + q] * g->J[3 * q + b];
            GSc[3 * a + b] = s;
        }
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 3; ++b) {
            double s = 0.0;
            for (int q = 0; q < 2; ++q) s += GS2[2 * a + q] * g->J[3 * q + b];
            tmp[3 * a + b] = s;
        }
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 3; ++b) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += tmp[3 * a + k] * g->Sc[3 * k + b];
            GJ[3 * a + b] = 2.0 * s;
        }

    /* mean through mu^ and J */
    double gmc[3];
    gmc[0] = g7[0] * f / z + GJ[2] * (-f / (z * z));
    gmc[1] = g7[1] * f / z + GJ[5] * (-f / (z * z));
    gmc[2] = -(g7[0] * f * x + g7[1] * f * y) / (z * z)
             + (GJ[0] + GJ[4]) * (-f / (z * z))
             + GJ[2] * (2.0 * f * x / (z * z * z)) + GJ[5] * (2.0 * f * y / (z * z * z));

    /* pose tangent: mu_c' = Exp(w) mu_c + rho, Sigma_c' = Exp(w) Sigma_c Exp(w)^T */
    for (int r = 0; r < 3; ++r) gpose[r] += gmc[r];
    gpose[3] += g->muc[1] * gmc[2] - g->muc[2] * gmc[1];
    gpose[4] += g->muc[2] * gmc[0] - g->muc[0] * gmc[2];
    gpose[5] += g->muc[0] * gmc[1] - g->muc[1] * gmc[0];
    for (int kk = 0; kk < 3; ++kk) {
        double e[3] = {0.0, 0.0, 0.0}, E[9], ES[9], SE[9];
        e[kk] = 1.0;
        skew(e, E);
        mat3_mul(E, g->Sc, ES);
        mat3_mul(g->Sc, E, SE);
        double s = 0.0;
        for (int q = 0; q < 9; ++q) s += GSc[q] * (ES[q] - SE[q]);
        gpose[3 + kk] += s;
    }

    /* world frame: mu_c = R mu + t, Sigma_c = R Sigma R^T */
    for (int a = 0; a < 3; ++a) gmu[a] += R[a] * gmc[0] + R[3 + a] * gmc[1] + R[6 + a] * gmc[2];
    double Rt[9], t1[9], GSw[9];
    mat3_transpose(R, Rt);
    mat3_mul(Rt, GSc, t1);
    mat3_mul(t1, R, GSw);

    /* Sigma = M M^T, M = Rq diag(s): dL/dM = 2 GSw M */
    double M[9], GM[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) M[3 * a + b] = g->Rq[3 * a + b] * g->sc[b];
    mat3_mul(GSw, M, GM);
    for (int q = 0; q < 9; ++q) GM[q] *= 2.0;
    double GR[9];
    for (int b = 0; b < 3; ++b) {
        double s = 0.0;
        for (int a = 0; a < 3; ++a) s += GM[3 * a + b] * g->Rq[3 * a + b];
        gls[b] += s * g->sc[b];
        for (int a = 0; a < 3; ++a) GR[3 * a + b] = GM[3 * a + b] * g->sc[b];
    }
    /* rotation matrix of the unit quaternion (w, x, y, z) */
    const double qw = g->qn[0], qx = g->qn[1], qy = g->qn[2], qz = g->qn[3];
    double gqn[4];
    gqn[0] = 2.0 * (-qz * GR[1] + qy * GR[2] + qz * GR[3] - qx * GR[5] - qy * GR[6] + qx * GR[7]);
    gqn[1] = 2.0 * (qy * GR[1] + qz * GR[2] + qy * GR[3] - qw * GR[5] + qz * GR[6] + qw * GR[7])
             - 4.0 * qx * (GR[4] + GR[8]);
    gqn[2] = 2.0 * (qx * GR[1] + qw * GR[2] + qx * GR[3] + qz * GR[5] - qw * GR[6] + qz * GR[7])
             - 4.0 * qy * (GR[0] + GR[8]);
    gqn[3] = 2.0 * (-qw * GR[1] + qx * GR[2] + qw * GR[3] + qy * GR[5] + qx * GR[6] + qy * GR[7])
             - 4.0 * qz * (GR[0] + GR[4]);
    const double dotq = gqn[0] * qw + gqn[1] * qx + gqn[2] * qy + gqn[3] * qz;
    for (int a = 0; a < 4; ++a) gq[a] += (gqn[a] - g->qn[a] * dotq) / g->qnorm;

    /* opacity */
    *gop += g7[5] * g->alpha * (1.0 - g->alpha);

    /* radiosity */
    if (gc_out) *gc_out += g7[6];
    if (o->c_override) return;
    const int k = m->k, kl = orc_kl(m->L);
    const double gz = g7[6] * g->c * (1.0 - g->c);
    if (m->entangled || i < m->n_iso) {
        for (int j = 0; j < k; ++j) {
            gf[j] += gz * m->b_iso[j];
            gb[j] += gz * m->feat[(int64_t)j * n + i];
        }
    }
    if (m->entangled || i >= m->n_iso) {
        double Y[ORC_MAXKL], dY[3 * ORC_MAXKL];
        orc_sh(m->L, g->dir, Y, dY);
        double gd[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < kl; ++a) {
            const double gh = gz * Y[a];
            for (int j = 0; j < k; ++j) {
                gf[j] += m->B_dir[a * k + j] * gh;
                gB[a * k + j] += gh * m->feat[(int64_t)j * n + i];
            }
            const double gY = gz * g->h[a];
            gd[0] += gY * dY[3 * a]; gd[1] += gY * dY[3 * a + 1]; gd[2] += gY * dY[3 * a + 2];
        }
        /* d = r/|r|, r = mu - s_o, s_o = -R^T t: dr/drho = R^T at zero tangent */
        const double dd = gd[0] * g->dir[0] + gd[1] * g->dir[1] + gd[2] * g->dir[2];
        double gr[3];
        for (int a = 0; a < 3; ++a) gr[a] = (gd[a] - g->dir[a] * dd) / g->rlen;
        for (int a = 0; a < 3; ++a) gmu[a] += gr[a];
        for (int a = 0; a < 3; ++a) gpose[a] += R[3 * a] * gr[0] + R[3 * a + 1] * gr[1] + R[3 * a + 2] * gr[2];
    }
}

int orc_backward(const orc_model *m, const orc_view *views, int V,
                 const orc_opts *o, int64_t npix, const int32_t *pix,
                 const double *gpix, const orc_grads *out, int threads)
{
    if (check_args(m, views, V, o) || !out || (npix > 0 && (!pix || !gpix))) return -1;
    for (int64_t p = 0; p < npix; ++p) {
        const int32_t v = pix[3 * p];
        if (v < 0 || v >= V || pix[3 * p + 1] < 0 || pix[3 * p + 1] >= views[v].W ||
            pix[3 * p + 2] < 0 || pix[3 * p + 2] >= views[v].H) return -1;
    }
    if (threads < 1) threads = 1;
    const int64_t n = m->n;
    const int k = m->k, kl = orc_kl(m->L);
    if (out->dmean) memset(out->dmean, 0, sizeof(double) * 3 * n);
    if (out->dquat) memset(out->dquat, 0, sizeof(double) * 4 * n);
    if (out->dlog_scale) memset(out->dlog_scale, 0, sizeof(double) * 3 * n);
    if (out->dopacity_logit) memset(out->dopacity_logit, 0, sizeof(double) * n);
    if (out->dfeat) memset(out->dfeat, 0, sizeof(double) * k * n);
    if (out->db_iso) memset(out->db_iso, 0, sizeof(double) * k);
    if (out->dB_dir) memset(out->dB_dir, 0, sizeof(double) * kl * k);
    if (out->dpose) memset(out->dpose, 0, sizeof(double) * 6 * V);
    if (out->dc) memset(out->dc, 0, sizeof(double) * V * n);
    if (out->g2d) memset(out->g2d, 0, sizeof(double) * 7 * V * n);

    double *gb_all = (double *)calloc((size_t)threads * (k + kl * k), sizeof(double));
    double *acc = (double *)malloc(sizeof(double) * 7 * (size_t)(n > 0 ? n : 1) * threads);
    double *g2d = (double *)malloc(sizeof(double) * 7 * (size_t)(n > 0 ? n : 1));

    for (int v = 0; v < V; ++v) {
        int any = 0;
        for (int64_t p = 0; p < npix && !any; ++p) any = (pix[3 * p] == v);
        if (!any) continue;
        gproj *gp; int64_t *order; gfast *fast;
        const int64_t nv = prepare_view(m, &views[v], v, o, &gp, &order, &fast);
        memset(acc, 0, sizeof(double) * 7 * (size_t)n * threads);

        /* per pixel: list the contributing Gaussians, then walk it back to
         * front so that S_j = sum_{m>j} c_m s_m T_m is available */
#pragma omp parallel num_threads(threads)
        {
#ifdef _OPENMP
            const int tid = omp_get_thread_num();
#else
            const int tid = 0;
#endif
            double *a = acc + (size_t)tid * 7 * n;
            contrib *list = (contrib *)malloc(sizeof(contrib) * (size_t)(nv > 0 ? nv : 1));
#pragma omp for schedule(static, 1)
            for (int64_t p = 0; p < npix; ++p) {
                if (pix[3 * p] != v) continue;
                const double gp_ = gpix[p];
                if (gp_ == 0.0) continue;
                int64_t nl = 0;
                render_pixel(fast, nv, pix[3 * p + 1] + 0.5, pix[3 * p + 2] + 0.5, o, list, &nl,
                             order, 0, n, NULL, NULL, NULL);
                double S = 0.0;
                for (int64_t q = nl - 1; q >= 0; --q) {
                    const contrib *e = &list[q];
                    const gfast *g = &fast[e->j];
                    double *ai = a + 7 * order[e->j];
                    const double ds = gp_ * (g->c * e->T - S / (1.0 - e->s));
                    ai[6] += gp_ * e->s * e->T;
                    S += g->c * e->s * e->T;
                    if (e->clamped) continue;
                    ai[5] += ds * e->G;
                    const double dd2 = -0.5 * e->G * g->alpha * ds;
                    ai[0] += dd2 * (-2.0) * (g->A0 * e->dx + g->A1 * e->dy);
                    ai[1] += dd2 * (-2.0) * (g->A1 * e->dx + g->A2 * e->dy);
                    ai[2] += dd2 * e->dx * e->dx;
                    ai[3] += dd2 * 2.0 * e->dx * e->dy;
                    ai[4] += dd2 * e->dy * e->dy;
                }
            }
            free(list);
        }
        /* fixed-order reduction over threads */
        for (int64_t q = 0; q < 7 * n; ++q) {
            double s = 0.0;
            for (int t = 0; t < threads; ++t) s += acc[(size_t)t * 7 * n + q];
            g2d[q] = s;
        }
        if (out->g2d) memcpy(out->g2d + (size_t)v * 7 * n, g2d, sizeof(double) * 7 * n);

        /* chain rule per Gaussian; globals accumulated per thread */
        double *pose_t = (double *)calloc((size_t)threads * 6, sizeof(double));
        memset(gb_all, 0, sizeof(double) * threads * (k + kl * k));
#pragma omp parallel for schedule(static) num_threads(threads)
        for (int64_t i = 0; i < n; ++i) {
            if (!gp[i].valid) continue;
            const double *g7 = g2d + 7 * i;
            if (g7[0] == 0.0 && g7[1] == 0.0 && g7[2] == 0.0 && g7[3] == 0.0 && g7[4] == 0.0 &&
                g7[5] == 0.0 && g7[6] == 0.0) continue;
#ifdef _OPENMP
            const int tid = omp_get_thread_num();
#else
            const int tid = 0;
#endif
            double gmu[3] = {0, 0, 0}, gq[4] = {0, 0, 0, 0}, gls[3] = {0, 0, 0}, gop = 0.0, gcv = 0.0;
            double gf[64];
            memset(gf, 0, sizeof(gf));
            double *gbt = gb_all + (size_t)tid * (k + kl * k);
            chain_one(m, &views[v], o, i, &gp[i], g7, gmu, gq, gls, &gop, gf, gbt, gbt + k,
                      pose_t + 6 * tid, &gcv);
            if (out->dmean) for (int a = 0; a < 3; ++a) out->dmean[a * n + i] += gmu[a];
            if (out->dquat) for (int a = 0; a < 4; ++a) out->dquat[a * n + i] += gq[a];
            if (out->dlog_scale) for (int a = 0; a < 3; ++a) out->dlog_scale[a * n + i] += gls[a];
            if (out->dopacity_logit) out->dopacity_logit[i] += gop;
            if (out->dfeat) for (int j = 0; j < k; ++j) out->dfeat[(int64_t)j * n + i] += gf[j];
            if (out->dc) out->dc[(int64_t)v * n + i] += gcv;
        }
        for (int t = 0; t < threads; ++t) {
            if (out->dpose) for (int a = 0; a < 6; ++a) out->dpose[6 * v + a] += pose_t[6 * t + a];
            const double *gbt = gb_all + (size_t)t * (k + kl * k);
            if (out->db_iso) for (int j = 0; j < k; ++j) out->db_iso[j] += gbt[j];
            if (out->dB_dir) for (int j = 0; j < kl * k; ++j) out->dB_dir[j] += gbt[k + j];
        }
        free(pose_t);
        free(gp); free(order); free(fast);
    }
    free(acc); free(g2d); free(gb_all);
    return 0;
}

/* -------------------------------------------------------------------- losses */

/* 11x11 Gaussian window of std 1.5, normalised to unit sum (Wang et al.
 * defaults, the SSIM that Eq. 2 cites). */
static void ssim_window(double w[121])
{
    double g[11], s = 0.0;
    for (int i = 0; i < 11; ++i) { g[i] = exp(-((i - 5) * (i - 5)) / (2.0 * 1.5 * 1.5)); s += g[i]; }
    for (int i = 0; i < 11; ++i) g[i] /= s;
    for (int a = 0; a < 11; ++a)
        for (int b = 0; b < 11; ++b) w[11 * a + b] = g[a] * g[b];
}

/* o(p) = sum over the window of w(q) in(p + q - 5), zero outside the image */
static void window_sum(const double *in, int W, int H, const double *w, double *o)
{
    for (int r = 0; r < H; ++r)
        for (int c = 0; c < W; ++c) {
            double s = 0.0;
            for (int a = 0; a < 11; ++a) {
                const int rr = r + a - 5;
                if (rr < 0 || rr >= H) continue;
                for (int b = 0; b < 11; ++b) {
                    const int cc = c + b - 5;
                    if (cc < 0 || cc >= W) continue;
                    s += w[11 * a + b] * in[(int64_t)rr * W + cc];
                }
            }
            o[(int64_t)r * W + c] = s;
        }
}

int orc_loss_l1ssim(const double *x, const double *y, int W, int H,
                    double lambda, double *loss, double *ssim_mean, double *grad)
{
    if (!x || !y || W <= 0 || H <= 0) return -1;
    const int64_t P = (int64_t)W * H;
    const double C1 = 0.01 * 0.01, C2 = 0.03 * 0.03;
    double w[121];
    ssim_window(w);
    double *buf = (double *)malloc(sizeof(double) * P * 13);
    double *xx = buf, *yy = buf + P, *xy = buf + 2 * P;
    double *mx = buf + 3 * P, *my = buf + 4 * P, *sxx = buf + 5 * P, *syy = buf + 6 * P, *sxy = buf + 7 * P;
    double *da = buf + 8 * P, *db = buf + 9 * P, *dc = buf + 10 * P, *fa = buf + 11 * P, *fb = buf + 12 * P;
    for (int64_t p = 0; p < P; ++p) { xx[p] = x[p] * x[p]; yy[p] = y[p] * y[p]; xy[p] = x[p] * y[p]; }
    window_sum(x, W, H, w, mx);
    window_sum(y, W, H, w, my);
    window_sum(xx, W, H, w, sxx);
    window_sum(yy, W, H, w, syy);
    window_sum(xy, W, H, w, sxy);
    double ssum = 0.0, l1 = 0.0;
    for (int64_t p = 0; p < P; ++p) {
        const double ux = mx[p], uy = my[p];
        const double vx = sxx[p] - ux * ux, vy = syy[p] - uy * uy, cxy = sxy[p] - ux * uy;
        const double A1 = 2.0 * ux * uy + C1, A2 = 2.0 * cxy + C2;
        const double B1 = ux * ux + uy * uy + C1, B2 = vx + vy + C2;
        const double D = B1 * B2, s = A1 * A2 / D;
        ssum += s;
        l1 += fabs(x[p] - y[p]);
        /* partial derivatives of s w.r.t. the windowed mean of x, the
         * windowed mean of x^2 and the windowed mean of x y */
        da[p] = (2.0 * uy * A2 + A1 * (-2.0 * uy) - s * (2.0 * ux * B2 + B1 * (-2.0 * ux))) / D;
        db[p] = -s * B1 / D;
        dc[p] = 2.0 * A1 / D;
    }
    const double sm = ssum / (double)P;
    if (ssim_mean) *ssim_mean = sm;
    if (loss) *loss = (1.0 - lambda) * l1 / (double)P + lambda * (1.0 - sm);
    if (grad) {
        /* the window is symmetric, so the adjoint of the windowed sum is the
         * same windowed sum (zero padding on both sides) */
        window_sum(da, W, H, w, fa);
        window_sum(db, W, H, w, fb);
        window_sum(dc, W, H, w, xx);
        for (int64_t p = 0; p < P; ++p) {
            const double d = x[p] - y[p];
            const double sg = (d > 0.0) - (d < 0.0);
            const double dssim = fa[p] + 2.0 * x[p] * fb[p] + y[p] * xx[p];
            grad[p] = (1.0 - lambda) * sg / (double)P - lambda * dssim / (double)P;
        }
    }
    free(buf);
    return 0;
}

int orc_loss_ncc(const double *x, const double *y, int64_t P, double eps,
                 double *loss, double *grad)
{
    if (!x || !y || P <= 0) return -1;
    double sx = 0.0, sy = 0.0;
    for (int64_t p = 0; p < P; ++p) { sx += x[p]; sy += y[p]; }
    const double mxv = sx / (double)P, myv = sy / (double)P;
    double vx = 0.0, vy = 0.0, cv = 0.0;
    for (int64_t p = 0; p < P; ++p) {
        const double a = x[p] - mxv, b = y[p] - myv;
        vx += a * a; vy += b * b; cv += a * b;
    }
    vx /= (double)P; vy /= (double)P; cv /= (double)P;
    const double sdx = sqrt(vx + eps), sdy = sqrt(vy + eps);
    const double ncc = cv / (sdx * sdy);
    if (loss) *loss = 1.0 - ncc;
    if (grad)
        for (int64_t p = 0; p < P; ++p) {
            const double xh = (x[p] - mxv) / sdx, yh = (y[p] - myv) / sdy;
            grad[p] = -(yh - ncc * xh) / ((double)P * sdx);
        }
    return 0;
}
