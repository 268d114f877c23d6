// project.hip -- per-Gaussian and per-(view, Gaussian) kernels of the DDGS
// DRR splatting path on gfx950: view-independent preparation, cone-beam
// projection with the Eq. 3 radiosity and tile footprint, and the backward
// chain rule to the Gaussian parameters, the shared bases and the source pose.
//
// Layout: every model array is structure-of-arrays ([component][n]) so that
// consecutive lanes of a wave read consecutive floats (coalesced 256-byte
// wave loads).  One thread handles one Gaussian (x) of one view (y).
#include "internal.h"

namespace ddgs {

namespace {

constexpr int kBlock = 256;
static_assert(kBlock == kSlotBlock, "one projection block per block of the slot numbering");

// Real orthonormal spherical basis of degrees 1..L at the unit direction
// (x, y, z): order l = 1..L, m = -l..l, no Condon-Shortley phase.  The
// normalisations are sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!) times the factor
// sqrt(2) for m != 0, folded into the Cartesian polynomials.
template <int L>
__device__ __forceinline__ void sh_basis(float x, float y, float z, float *Y)
{
    const float c1 = 0.48860251190291992f;
    Y[0] = c1 * y;
    Y[1] = c1 * z;
    Y[2] = c1 * x;
    if constexpr (L >= 2) {
        const float a2 = 1.0925484305920792f, b2 = 0.31539156525252005f, c2 = 0.54627421529603959f;
        Y[3] = a2 * x * y;
        Y[4] = a2 * y * z;
        Y[5] = b2 * (3.0f * z * z - 1.0f);
        Y[6] = a2 * x * z;
        Y[7] = c2 * (x * x - y * y);
    }
    if constexpr (L >= 3) {
        const float a3 = 0.59004358992664352f, b3 = 2.8906114426405538f, c3 = 0.45704579946446572f;
        const float e3 = 0.37317633259011540f, h3 = 1.4453057213202769f;
        Y[8] = a3 * y * (3.0f * x * x - y * y);
        Y[9] = b3 * x * y * z;
        Y[10] = c3 * y * (5.0f * z * z - 1.0f);
        Y[11] = e3 * z * (5.0f * z * z - 3.0f);
        Y[12] = c3 * x * (5.0f * z * z - 1.0f);
        Y[13] = h3 * z * (x * x - y * y);
        Y[14] = a3 * x * (x * x - 3.0f * y * y);
    }
}

// sum_m w[m] * grad Y_m(x, y, z) (gradient of the polynomials above)
template <int L>
__device__ __forceinline__ void sh_basis_grad(float x, float y, float z, const float *w, float &gx,
                                              float &gy, float &gz)
{
    const float c1 = 0.48860251190291992f;
    gx = c1 * w[2];
    gy = c1 * w[0];
    gz = c1 * w[1];
    if constexpr (L >= 2) {
        const float a2 = 1.0925484305920792f, b2 = 0.31539156525252005f, c2 = 0.54627421529603959f;
        gx += a2 * (y * w[3] + z * w[6]) + 2.0f * c2 * x * w[7];
        gy += a2 * (x * w[3] + z * w[4]) - 2.0f * c2 * y * w[7];
        gz += a2 * (y * w[4] + x * w[6]) + 6.0f * b2 * z * w[5];
    }
    if constexpr (L >= 3) {
        const float a3 = 0.59004358992664352f, b3 = 2.8906114426405538f, c3 = 0.45704579946446572f;
        const float e3 = 0.37317633259011540f, h3 = 1.4453057213202769f;
        const float q = 5.0f * z * z - 1.0f;
        gx += 6.0f * a3 * x * y * w[8] + b3 * y * z * w[9] + c3 * q * w[12] +
              2.0f * h3 * x * z * w[13] + 3.0f * a3 * (x * x - y * y) * w[14];
        gy += 3.0f * a3 * (x * x - y * y) * w[8] + b3 * x * z * w[9] + c3 * q * w[10] -
              2.0f * h3 * y * z * w[13] - 6.0f * a3 * x * y * w[14];
        gz += b3 * x * y * w[9] + 10.0f * c3 * y * z * w[10] + e3 * (15.0f * z * z - 3.0f) * w[11] +
              10.0f * c3 * x * z * w[12] + h3 * (x * x - y * y) * w[13];
    }
}

__device__ __forceinline__ float sigmoidf(float x) { return 1.0f / (1.0f + expf(-x)); }

// Geometry of one (view, Gaussian) pair: source-frame mean and covariance,
// the Jacobian of the pinhole map at the mean, the projected covariance with
// the low-pass dilation, its inverse (the conic) and the projected mean.
struct Geom {
    float xc, yc, zc, iz;
    float Sc[6];                 // 00 01 02 11 12 22
    float J00, J02, J11, J12;
    float a, b, c;               // projected covariance 00 01 11
    float A00, A01, A11;         // conic
    float mux, muy;
    uint32_t zbits;
};

// Source-frame depth of the mean as a chain of fused multiply-adds in the
// order R20 x + (R21 y + (R22 z + t2)); it doubles as the sort key.
__device__ __forceinline__ float depth_of(const ViewDev &V, float mx, float my, float mz)
{
    return __builtin_fmaf(V.R[6], mx, __builtin_fmaf(V.R[7], my, __builtin_fmaf(V.R[8], mz, V.t[2])));
}

__device__ __forceinline__ bool project_geom(const ViewDev &V, float mx, float my, float mz,
                                             const float *cw, const RenderOpts &o, Geom &g)
{
    const float z = depth_of(V, mx, my, mz);
    g.zbits = __float_as_uint(z);
    if (!(z > o.z_near)) return false;
    g.xc = V.R[0] * mx + V.R[1] * my + V.R[2] * mz + V.t[0];
    g.yc = V.R[3] * mx + V.R[4] * my + V.R[5] * mz + V.t[1];
    g.zc = z;
    g.iz = 1.0f / z;
    // T = R Sigma (Sigma symmetric: xx xy xz yy yz zz)
    const float *R = V.R;
    float T[9];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        T[3 * r + 0] = R[3 * r] * cw[0] + R[3 * r + 1] * cw[1] + R[3 * r + 2] * cw[2];
        T[3 * r + 1] = R[3 * r] * cw[1] + R[3 * r + 1] * cw[3] + R[3 * r + 2] * cw[4];
        T[3 * r + 2] = R[3 * r] * cw[2] + R[3 * r + 1] * cw[4] + R[3 * r + 2] * cw[5];
    }
    // Sigma_c = T R^T
    g.Sc[0] = T[0] * R[0] + T[1] * R[1] + T[2] * R[2];
    g.Sc[1] = T[0] * R[3] + T[1] * R[4] + T[2] * R[5];
    g.Sc[2] = T[0] * R[6] + T[1] * R[7] + T[2] * R[8];
    g.Sc[3] = T[3] * R[3] + T[4] * R[4] + T[5] * R[5];
    g.Sc[4] = T[3] * R[6] + T[4] * R[7] + T[5] * R[8];
    g.Sc[5] = T[6] * R[6] + T[7] * R[7] + T[8] * R[8];
    const float f = V.f, iz = g.iz;
    g.J00 = f * iz;
    g.J11 = f * iz;
    g.J02 = -f * g.xc * iz * iz;
    g.J12 = -f * g.yc * iz * iz;
    const float *S = g.Sc;
    g.a = g.J00 * g.J00 * S[0] + 2.0f * g.J00 * g.J02 * S[2] + g.J02 * g.J02 * S[5] + o.dilation;
    g.b = g.J00 * g.J11 * S[1] + g.J00 * g.J12 * S[2] + g.J02 * g.J11 * S[4] + g.J02 * g.J12 * S[5];
    g.c = g.J11 * g.J11 * S[3] + 2.0f * g.J11 * g.J12 * S[4] + g.J12 * g.J12 * S[5] + o.dilation;
    const float det = g.a * g.c - g.b * g.b;
    if (!(det > 0.0f)) return false;
    const float idet = 1.0f / det;
    g.A00 = g.c * idet;
    g.A01 = -g.b * idet;
    g.A11 = g.a * idet;
    g.mux = f * g.xc * iz + V.cx;
    g.muy = f * g.yc * iz + V.cy;
    return isfinite(g.mux) && isfinite(g.muy) && isfinite(g.A00) && isfinite(g.A11);
}

// ------------------------------------------------------------------ prepare

// Bases staged in LDS by every block of the preparing kernels.
template <int KMAX, int L>
__device__ __forceinline__ void stage_bases(const ModelDev &m, float *sb, float *sB)
{
    constexpr int KL = L * (L + 2);
    const int k = m.k;
    for (int q = threadIdx.x; q < KMAX; q += kBlock) sb[q] = q < k ? m.b_iso[q] : 0.0f;
    for (int q = threadIdx.x; q < KL * KMAX; q += kBlock) {
        const int r = q / KMAX, j = q % KMAX;
        sB[q] = j < k ? m.B_dir[r * k + j] : 0.0f;
    }
}

// The view-independent cache of Gaussian i: world covariance, opacity, the
// isotropic radiosity (its logit for entangled models) and the directional
// h = B f; written to gc and returned in registers (h only for directional
// Gaussians).
template <int KMAX, int L>
__device__ __forceinline__ void prep_one(const ModelDev &m, const GaussCache &gc, int i, const float *sb,
                                         const float *sB, float (&cw)[6], float &alpha, float &ciso,
                                         float (&h)[L * (L + 2)])
{
    constexpr int KL = L * (L + 2);
    const int n = m.n, k = m.k;
    float qw = m.quat[i], qx = m.quat[n + i], qy = m.quat[2 * n + i], qz = m.quat[3 * n + i];
    const float inv = 1.0f / sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
    qw *= inv; qx *= inv; qy *= inv; qz *= inv;
    float Rq[9];
    quat_rot(qw, qx, qy, qz, Rq);
    float s2[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float s = expf(m.log_scale[a * n + i]);
        s2[a] = s * s;
    }
    // Sigma = Rq diag(s^2) Rq^T
    cw[0] = Rq[0] * Rq[0] * s2[0] + Rq[1] * Rq[1] * s2[1] + Rq[2] * Rq[2] * s2[2];
    cw[1] = Rq[0] * Rq[3] * s2[0] + Rq[1] * Rq[4] * s2[1] + Rq[2] * Rq[5] * s2[2];
    cw[2] = Rq[0] * Rq[6] * s2[0] + Rq[1] * Rq[7] * s2[1] + Rq[2] * Rq[8] * s2[2];
    cw[3] = Rq[3] * Rq[3] * s2[0] + Rq[4] * Rq[4] * s2[1] + Rq[5] * Rq[5] * s2[2];
    cw[4] = Rq[3] * Rq[6] * s2[0] + Rq[4] * Rq[7] * s2[1] + Rq[5] * Rq[8] * s2[2];
    cw[5] = Rq[6] * Rq[6] * s2[0] + Rq[7] * Rq[7] * s2[1] + Rq[8] * Rq[8] * s2[2];
#pragma unroll
    for (int a = 0; a < 6; ++a) gc.cov[a * n + i] = cw[a];
    alpha = sigmoidf(m.opacity_logit[i]);
    gc.alpha[i] = alpha;
    float f[KMAX];
#pragma unroll
    for (int j = 0; j < KMAX; ++j) f[j] = j < k ? m.feat[(size_t)j * n + i] : 0.0f;
    ciso = 0.0f;
    if (i < m.n_iso || m.entangled) {
        float zl = 0.0f;
#pragma unroll
        for (int j = 0; j < KMAX; ++j) zl += sb[j] * f[j];
        ciso = m.entangled ? zl : sigmoidf(zl);
        gc.ciso[i] = ciso;
    }
#pragma unroll
    for (int r = 0; r < KL; ++r) h[r] = 0.0f;
    if (i >= m.n_iso) {
        const int nd = n - m.n_iso, id = i - m.n_iso;
#pragma unroll
        for (int r = 0; r < KL; ++r) {
            float hr = 0.0f;
#pragma unroll
            for (int j = 0; j < KMAX; ++j) hr += sB[r * KMAX + j] * f[j];
            h[r] = hr;
            gc.hdir[(size_t)r * nd + id] = hr;
        }
    }
}

template <int KMAX, int L>
__global__ __launch_bounds__(kBlock) void prep_kernel(ModelDev m, GaussCache gc)
{
    constexpr int KL = L * (L + 2);
    __shared__ float sb[KMAX];
    __shared__ float sB[KL * KMAX];
    stage_bases<KMAX, L>(m, sb, sB);
    __syncthreads();
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= m.n) return;
    float cw[6], alpha, ciso, h[KL];
    prep_one<KMAX, L>(m, gc, i, sb, sB, cw, alpha, ciso, h);
}

// ------------------------------------------------------------------ project

// Minimum of d^T A d over the box [xl, xh] x [yl, yh] of offsets from the
// mean (A positive definite, iA00 = 1 / A00, iA11 = 1 / A11): zero when the
// mean lies in the box, else the least of the four edges' minima (on an edge
// the quadratic is a parabola in the free coordinate, minimised at
// -A01 x / A11 or -A01 y / A00 and clamped to the edge).
__device__ __forceinline__ float box_min_d2(float A00, float A01, float A11, float iA00, float iA11, float xl,
                                            float xh, float yl, float yh)
{
    if (xl <= 0.0f && 0.0f <= xh && yl <= 0.0f && 0.0f <= yh) return 0.0f;
    auto q = [&](float x, float y) { return x * (A00 * x + 2.0f * A01 * y) + A11 * y * y; };
    auto on_x = [&](float x) { return q(x, fminf(fmaxf(-A01 * x * iA11, yl), yh)); };
    auto on_y = [&](float y) { return q(fminf(fmaxf(-A01 * y * iA00, xl), xh), y); };
    return fminf(fminf(on_x(xl), on_x(xh)), fminf(on_y(yl), on_y(yh)));
}

// Tiles of the rectangle [tx0, tx1] x [ty0, ty1] (at most 32, bit b =
// row-major place in the rectangle) whose pixel centres come within the
// cut-off ellipse d^T A d <= kappa^2, widened by 0.1 % (far above the
// rounding of these FP32 evaluations and of the per-pixel test) so that no
// pixel the exact definition puts inside is dropped.  The rectangle is the
// ellipse's bounding box, so its corner tiles are often outside.
__device__ __forceinline__ uint32_t tile_mask(const Geom &g, const RenderOpts &o, const ViewDev &V, int tx0, int ty0,
                                              int tx1, int ty1)
{
    const float lim = o.kappa * o.kappa * 1.001f;
    const float iA00 = 1.0f / g.A00, iA11 = 1.0f / g.A11;
    uint32_t m = 0u;
    int b = 0;
    for (int ty = ty0; ty <= ty1; ++ty) {
        const float yl = (float)(ty * o.tile_h) + 0.5f - g.muy;
        const float yh = (float)min((ty + 1) * o.tile_h, V.H) - 0.5f - g.muy;
        for (int tx = tx0; tx <= tx1; ++tx, ++b) {
            const float xl = (float)(tx * o.tile_w) + 0.5f - g.mux;
            const float xh = (float)min((tx + 1) * o.tile_w, V.W) - 0.5f - g.mux;
            if (box_min_d2(g.A00, g.A01, g.A11, iA00, iA11, xl, xh, yl, yh) <= lim) m |= 1u << b;
        }
    }
    return m;
}

// Projection of Gaussian i into view v from its cache values (cw, alpha,
// ciso; hd(r) gives h_r of a directional Gaussian), then this block's scan of
// the tile counts for the slot numbering (every thread of the block calls it).
template <int L, class HD>
__device__ __forceinline__ void project_one(const ModelDev &m, const ViewDev *views, const RenderOpts &o,
                                            const ProjOut &po, int v, int i, const float (&cw)[6], float alpha,
                                            float ciso, HD hd)
{
    static_assert(kBlock == kSlotBlock, "one projection block per block of the slot numbering");
    constexpr int KL = L * (L + 2);
    const int n = m.n;
    const size_t vi = (size_t)v * n + i;
    uint32_t count = 0;
    float4 r1 = make_float4(0.f, 0.f, 0.f, 0.f);
    if (i < n) {
        const ViewDev V = views[v];
        const float mx = m.mean[i], my = m.mean[n + i], mz = m.mean[2 * n + i];
        Geom g;
        const bool ok = project_geom(V, mx, my, mz, cw, o, g);
        if (!ok) {
            po.zkey[vi] = 0xFFFFFFFFu;
            po.cnt[vi] = 0;
            po.rect[vi] = make_uint2(0, 0);
            po.tmask[vi] = 0u;
            po.rec[4 * vi] = make_float4(0.f, 0.f, 0.f, 0.f);
            po.rec[4 * vi + 2] = make_float4(0.f, 0.f, 0.f, 0.f);
        } else {
            float c;
            if (m.c_override) {
                c = m.c_override[vi];
            } else if (i < m.n_iso) {
                c = ciso;
            } else {
                float rx = mx - V.so[0], ry = my - V.so[1], rz = mz - V.so[2];
                const float il = 1.0f / sqrtf(rx * rx + ry * ry + rz * rz);
                float Y[KL];
                sh_basis<L>(rx * il, ry * il, rz * il, Y);
                float zl = m.entangled ? ciso : 0.0f;
#pragma unroll
                for (int r = 0; r < KL; ++r) zl += Y[r] * hd(r);
                c = sigmoidf(zl);
            }
            // conservative pixel box of the kappa ellipse: half-widths kappa sqrt(S00),
            // kappa sqrt(S11), widened for float rounding of the per-pixel test
            const float rxp = o.kappa * sqrtf(g.a) * 1.0005f + 0.01f;
            const float ryp = o.kappa * sqrtf(g.c) * 1.0005f + 0.01f;
            const float fu0 = fmaxf(ceilf(g.mux - rxp - 0.5f), 0.0f);
            const float fu1 = fminf(floorf(g.mux + rxp - 0.5f), (float)(V.W - 1));
            const float fv0 = fmaxf(ceilf(g.muy - ryp - 0.5f), 0.0f);
            const float fv1 = fminf(floorf(g.muy + ryp - 0.5f), (float)(V.H - 1));
            uint2 rc = make_uint2(0, 0);
            uint32_t mask = kAllTiles;
            if (fu0 <= fu1 && fv0 <= fv1) {
                const int tx0 = (int)fu0 / o.tile_w, tx1 = (int)fu1 / o.tile_w;
                const int ty0 = (int)fv0 / o.tile_h, ty1 = (int)fv1 / o.tile_h;
                count = (uint32_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1));
                // rectangles of up to 32 tiles keep only the tiles the
                // ellipse reaches (larger ones keep every tile)
                if (count <= kMaskTiles) {
                    mask = tile_mask(g, o, V, tx0, ty0, tx1, ty1);
                    count = (uint32_t)__popc(mask);
                }
                rc = make_uint2((uint32_t)tx0 | ((uint32_t)ty0 << 16), (uint32_t)tx1 | ((uint32_t)ty1 << 16));
            }
            po.zkey[vi] = g.zbits;
            po.cnt[vi] = count;
            po.rect[vi] = rc;
            po.tmask[vi] = mask;
            po.rec[4 * vi] = make_float4(g.mux, g.muy, g.A00, g.A01);
            r1 = make_float4(g.A11, alpha, c, 0.0f);
            po.rec[4 * vi + 2] = make_float4(__uint_as_float(rc.x), __uint_as_float(rc.y), __uint_as_float(mask), 0.0f);
        }
    }
    // the pair's place in its block's slot numbering (exclusive scan of the
    // counts over the block's Gaussians, in index order) and the block total
    __shared__ uint32_t wsum[kBlock / kWave];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const uint32_t inc = wave_incl_scan(count);
    if (lane == kWave - 1) wsum[w] = inc;
    __syncthreads();
    uint32_t before = 0, total = 0;
#pragma unroll
    for (int q = 0; q < kBlock / kWave; ++q) {
        const uint32_t t = wsum[q];
        if (q < w) before += t;
        total += t;
    }
    const uint32_t lp = before + inc - count;
    if (i < n) {
        r1.w = __uint_as_float(lp);
        po.rec[4 * vi + 1] = r1;
        po.slot_lp[vi] = lp;
    }
    if (threadIdx.x == 0) po.slot_btot[(size_t)v * gridDim.x + blockIdx.x] = total;
    __syncthreads();  // (wsum is reused by the next call)
}

// One block per kSlotBlock Gaussians and view (grid.y): the cache is read
// back from gc.
template <int L>
__global__ __launch_bounds__(kBlock) void project_kernel(ModelDev m, GaussCache gc, const ViewDev *views,
                                                         RenderOpts o, ProjOut po)
{
    const int n = m.n;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const int ii = i < n ? i : 0;
    float cw[6];
#pragma unroll
    for (int a = 0; a < 6; ++a) cw[a] = i < n ? gc.cov[a * n + ii] : 0.0f;
    const float alpha = i < n ? gc.alpha[ii] : 0.0f;
    const bool iso_c = i < m.n_iso || m.entangled;
    const float ciso = (i < n && iso_c) ? gc.ciso[ii] : 0.0f;
    const int nd = n - m.n_iso, id = ii - m.n_iso;
    project_one<L>(m, views, o, po, blockIdx.y, i, cw, alpha, ciso,
                   [&](int r) { return gc.hdir[(size_t)r * nd + id]; });
}

// One view: the cache is computed, written for the backward, and used for
// the projection straight from registers (one launch, no read-back).
template <int KMAX, int L>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8))) void prep_project_kernel(ModelDev m, GaussCache gc, const ViewDev *views,
                                                              RenderOpts o, ProjOut po)
{
    constexpr int KL = L * (L + 2);
    __shared__ float sb[KMAX];
    __shared__ float sB[KL * KMAX];
    stage_bases<KMAX, L>(m, sb, sB);
    __syncthreads();
    const int i = blockIdx.x * kBlock + threadIdx.x;
    float cw[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, alpha = 0.0f, ciso = 0.0f, h[KL];
    if (i < m.n) prep_one<KMAX, L>(m, gc, i, sb, sB, cw, alpha, ciso, h);
    project_one<L>(m, views, o, po, 0, i, cw, alpha, ciso, [&](int r) { return h[r]; });
}

// ------------------------------------------------------------ backward chain

template <int KMAX, int L>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3))) void project_bwd_kernel(ProjBwdArgs a)
{
    constexpr int KL = L * (L + 2);
    const int n = a.m.n;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const bool valid = i < n;
    const int ii = valid ? i : 0;
    const int lane = threadIdx.x & (kWave - 1);
    const bool is_dir = ii >= a.m.n_iso;
    const int nd = n - a.m.n_iso, id = ii - a.m.n_iso;
    // the next view's slot count and first slot, read one view ahead (the
    // first view's before the parameters, since its slot reads wait on them)
    uint32_t c_next = 0, off_next = 0;
    if (valid && a.V > 0) {
        c_next = a.cnt[ii];
        off_next = first_slot(a.slot_bofs, a.slot_nblk, 0, ii, a.slot_lp[ii]);
    }
    // isotropic radiosity, or for entangled models the isotropic logit (read
    // early too: values derived from it are computed before the view loop)
    const float ciso = (is_dir && !a.m.entangled) ? 0.0f : a.gc.ciso[ii];
    const float zl0 = a.m.entangled ? ciso : 0.0f;

    const float mx = a.m.mean[ii], my = a.m.mean[n + ii], mz = a.m.mean[2 * n + ii];
    float cw[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) cw[q] = a.gc.cov[q * n + ii];
    // values used after the view loop, read here so that their latency
    // overlaps the slot reads (stores in the loop keep the compiler from
    // moving them up)
    const float al = a.gc.alpha[ii];
    float quat0[4] = {1.f, 0.f, 0.f, 0.f}, lsc0[3] = {0.f, 0.f, 0.f}, st0[3] = {0.f, 0.f, 0.f};
    if (a.per_gaussian) {
#pragma unroll
        for (int q = 0; q < 4; ++q) quat0[q] = a.m.quat[q * n + ii];
#pragma unroll
        for (int q = 0; q < 3; ++q) lsc0[q] = a.m.log_scale[q * n + ii];
    }
    if (a.st_grad) {
        st0[0] = a.st_grad[ii];
        st0[1] = a.st_cnt[ii];
        st0[2] = a.st_rad[ii];
    }
    constexpr int NW = kBlock / kWave;
    __shared__ float sP[2][NW][9];
    const int w = threadIdx.x / kWave;
    float h[KL];
#pragma unroll
    for (int r = 0; r < KL; ++r) h[r] = 0.0f;
    if (nd > 0) {
        // read by every lane so that the loads are not split by per-lane
        // branches: isotropic lanes read a clamped index and never use it
        const int idc = min(max(id, 0), nd - 1);
#pragma unroll
        for (int r = 0; r < KL; ++r) h[r] = a.gc.hdir[(size_t)r * nd + idc];
    }

    float gmu[3] = {0.f, 0.f, 0.f};
    float GSw[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float galpha = 0.0f, zsum = 0.0f;
    float st_grad = 0.0f, st_cnt = 0.0f, st_rad = 0.0f;  // densification statistics
    float u[KL];
#pragma unroll
    for (int r = 0; r < KL; ++r) u[r] = 0.0f;

    for (int v = 0; v < a.V; ++v) {
        const ViewDev &V = a.views[v];
        float pose[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        // (the offset is only used when the count is non-zero)
        uint32_t c = c_next, off = off_next;
        if (valid && v + 1 < a.V) {
            c_next = a.cnt[(size_t)(v + 1) * n + ii];
            off_next = first_slot(a.slot_bofs, a.slot_nblk, v + 1, ii, a.slot_lp[(size_t)(v + 1) * n + ii]);
        }
        // slots past the capacity do not exist (overflowed step)
        if (c > 0) {
            if (off >= a.slot_cap) c = 0;
            else if ((uint64_t)off + c > a.slot_cap) c = a.slot_cap - off;
        }
        float g7[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        // the pair's slots in rectangle order; four entries' loads in flight
        // at once (the sums keep the same order)
        uint32_t e = 0;
        for (; e + 4u <= c; e += 4u) {
            float4 s0[4], s1[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                s0[t] = a.slot[2 * ((size_t)off + e + t)];
                s1[t] = a.slot[2 * ((size_t)off + e + t) + 1];
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                g7[0] += s0[t].x; g7[1] += s0[t].y; g7[2] += s0[t].z; g7[3] += s0[t].w;
                g7[4] += s1[t].x; g7[5] += s1[t].y; g7[6] += s1[t].z;
            }
        }
        if (e < c) {
            // the last one to three entries, loaded together (addresses past
            // the pair's last slot repeat it and are not added)
            const uint32_t rem = c - e;
            float4 s0[3], s1[3];
#pragma unroll
            for (int t = 0; t < 3; ++t) {
                const size_t q = (size_t)off + e + min((uint32_t)t, rem - 1u);
                s0[t] = a.slot[2 * q];
                s1[t] = a.slot[2 * q + 1];
            }
#pragma unroll
            for (int t = 0; t < 3; ++t) {
                if ((uint32_t)t < rem) {
                    g7[0] += s0[t].x; g7[1] += s0[t].y; g7[2] += s0[t].z; g7[3] += s0[t].w;
                    g7[4] += s1[t].x; g7[5] += s1[t].y; g7[6] += s1[t].z;
                }
            }
        }
        Geom g;
        if (c > 0 && project_geom(V, mx, my, mz, cw, a.o, g)) {
            // the slots hold moments of q = dL/ds G over the pixels, with
            // (dx, dy) = pixel - mean: (sum q dx, sum q dy, sum q dx^2,
            // sum q dx dy, sum q dy^2, sum q, dL/dc).  With s = alpha G,
            // G = exp(-d2 / 2), d2 = d^T A d: dL/dmu = alpha A sum q d,
            // dL/dA00 = -alpha/2 sum q dx^2, dL/dA01 (both off-diagonal
            // entries together) = -alpha sum q dx dy, dL/dA11 = -alpha/2 sum q dy^2.
            {
                const float m1x = g7[0], m1y = g7[1];
                g7[0] = al * (g.A00 * m1x + g.A01 * m1y);
                g7[1] = al * (g.A01 * m1x + g.A11 * m1y);
                g7[2] = -0.5f * al * g7[2];
                g7[3] = -al * g7[3];
                g7[4] = -0.5f * al * g7[4];
            }
            if (a.st_grad) {
                // visible in this view: 2D-mean gradient in normalised device
                // units and the projected radius kappa sqrt(lambda_max)
                const float gx = g7[0] * (0.5f * (float)V.W), gy = g7[1] * (0.5f * (float)V.H);
                st_grad += sqrtf(gx * gx + gy * gy);
                st_cnt += 1.0f;
                const float mid = 0.5f * (g.a + g.c);
                const float lam = mid + sqrtf(fmaxf(mid * mid - (g.a * g.c - g.b * g.b), 0.0f));
                st_rad = fmaxf(st_rad, a.o.kappa * sqrtf(lam));
            }
            // conic = inverse of the projected covariance: dL/dS2 = -A Gbar A
            const float gb00 = g7[2], gb01 = 0.5f * g7[3], gb11 = g7[4];
            const float t00 = g.A00 * gb00 + g.A01 * gb01, t01 = g.A00 * gb01 + g.A01 * gb11;
            const float t10 = g.A01 * gb00 + g.A11 * gb01, t11 = g.A01 * gb01 + g.A11 * gb11;
            const float G00 = -(t00 * g.A00 + t01 * g.A01);
            const float G01 = -(t00 * g.A01 + t01 * g.A11);
            const float G11 = -(t10 * g.A01 + t11 * g.A11);
            // S2 = J Sc J^T + dI
            float GSc[6];
            GSc[0] = g.J00 * g.J00 * G00;
            GSc[1] = g.J00 * g.J11 * G01;
            GSc[2] = g.J00 * (g.J02 * G00 + g.J12 * G01);
            GSc[3] = g.J11 * g.J11 * G11;
            GSc[4] = g.J11 * (g.J02 * G01 + g.J12 * G11);
            GSc[5] = g.J02 * g.J02 * G00 + 2.0f * g.J02 * g.J12 * G01 + g.J12 * g.J12 * G11;
            const float *S = g.Sc;
            const float p0x = G00 * g.J00, p0y = G01 * g.J11, p0z = G00 * g.J02 + G01 * g.J12;
            const float p1x = G01 * g.J00, p1y = G11 * g.J11, p1z = G01 * g.J02 + G11 * g.J12;
            const float GJ00 = 2.0f * (p0x * S[0] + p0y * S[1] + p0z * S[2]);
            const float GJ02 = 2.0f * (p0x * S[2] + p0y * S[4] + p0z * S[5]);
            const float GJ11 = 2.0f * (p1x * S[1] + p1y * S[3] + p1z * S[4]);
            const float GJ12 = 2.0f * (p1x * S[2] + p1y * S[4] + p1z * S[5]);
            // source-frame mean through mu^ and J
            const float f = V.f, fiz = f * g.iz, fz2 = fiz * g.iz;
            const float gxc = g7[0] * fiz - GJ02 * fz2;
            const float gyc = g7[1] * fiz - GJ12 * fz2;
            const float gzc = -(g7[0] * g.xc + g7[1] * g.yc) * fz2 - (GJ00 + GJ11) * fz2 +
                              2.0f * fz2 * g.iz * (GJ02 * g.xc + GJ12 * g.yc);
            // pose tangent (source frame moved by Exp(w), rho)
            const float *R = V.R;
            const float rmx = R[0] * mx + R[1] * my + R[2] * mz;
            const float rmy = R[3] * mx + R[4] * my + R[5] * mz;
            const float rmz = R[6] * mx + R[7] * my + R[8] * mz;
            pose[0] = gxc; pose[1] = gyc; pose[2] = gzc;
            // N = Sc GSc; the covariance term of d/dw_k is 2 (N12-N21, N20-N02, N01-N10)
            const float N01 = S[0] * GSc[1] + S[1] * GSc[3] + S[2] * GSc[4];
            const float N02 = S[0] * GSc[2] + S[1] * GSc[4] + S[2] * GSc[5];
            const float N10 = S[1] * GSc[0] + S[3] * GSc[1] + S[4] * GSc[2];
            const float N12 = S[1] * GSc[2] + S[3] * GSc[4] + S[4] * GSc[5];
            const float N20 = S[2] * GSc[0] + S[4] * GSc[1] + S[5] * GSc[2];
            const float N21 = S[2] * GSc[1] + S[4] * GSc[3] + S[5] * GSc[4];
            pose[3] = rmy * gzc - rmz * gyc + 2.0f * (N12 - N21);
            pose[4] = rmz * gxc - rmx * gzc + 2.0f * (N20 - N02);
            pose[5] = rmx * gyc - rmy * gxc + 2.0f * (N01 - N10);
            // world frame
            gmu[0] += R[0] * gxc + R[3] * gyc + R[6] * gzc;
            gmu[1] += R[1] * gxc + R[4] * gyc + R[7] * gzc;
            gmu[2] += R[2] * gxc + R[5] * gyc + R[8] * gzc;
            // GSw = R^T GSc R
            float Gf[9] = {GSc[0], GSc[1], GSc[2], GSc[1], GSc[3], GSc[4], GSc[2], GSc[4], GSc[5]};
            float U[9];  // GSc R
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int q = 0; q < 3; ++q)
                    U[3 * r + q] = Gf[3 * r] * R[q] + Gf[3 * r + 1] * R[3 + q] + Gf[3 * r + 2] * R[6 + q];
            GSw[0] += R[0] * U[0] + R[3] * U[3] + R[6] * U[6];
            GSw[1] += R[0] * U[1] + R[3] * U[4] + R[6] * U[7];
            GSw[2] += R[0] * U[2] + R[3] * U[5] + R[6] * U[8];
            GSw[3] += R[1] * U[1] + R[4] * U[4] + R[7] * U[7];
            GSw[4] += R[1] * U[2] + R[4] * U[5] + R[7] * U[8];
            GSw[5] += R[2] * U[2] + R[5] * U[5] + R[8] * U[8];
            galpha += g7[5];
            // radiosity (none when it is overridden)
            if (a.m.c_override) {
            } else if (!is_dir) {
                zsum += g7[6] * ciso * (1.0f - ciso);
            } else {
                const float rx = mx - V.so[0], ry = my - V.so[1], rz = mz - V.so[2];
                const float il = 1.0f / sqrtf(rx * rx + ry * ry + rz * rz);
                const float dx = rx * il, dy = ry * il, dz = rz * il;
                float Y[KL];
                sh_basis<L>(dx, dy, dz, Y);
                float zl = zl0;
#pragma unroll
                for (int r = 0; r < KL; ++r) zl += Y[r] * h[r];
                const float cd = 1.0f / (1.0f + expf(-zl));
                const float gz = g7[6] * cd * (1.0f - cd);
                if (a.m.entangled) zsum += gz;
                float wy[KL];
#pragma unroll
                for (int r = 0; r < KL; ++r) {
                    u[r] += gz * Y[r];
                    wy[r] = gz * h[r];
                }
                float gdx, gdy, gdz;
                sh_basis_grad<L>(dx, dy, dz, wy, gdx, gdy, gdz);
                const float dd = gdx * dx + gdy * dy + gdz * dz;
                const float grx = (gdx - dx * dd) * il, gry = (gdy - dy * dd) * il, grz = (gdz - dz * dd) * il;
                gmu[0] += grx; gmu[1] += gry; gmu[2] += grz;
                pose[6] = R[0] * grx + R[1] * gry + R[2] * grz;
                pose[7] = R[3] * grx + R[4] * gry + R[5] * grz;
                pose[8] = R[6] * grx + R[7] * gry + R[8] * grz;
            }
        }
        // per-block pose partials, component-major (deterministic: the
        // waves' sums added in a fixed order; reduced in FP64 later).  Two
        // buffers: no wave gets two views ahead of the barrier.
#pragma unroll
        for (int q = 0; q < 9; ++q) pose[q] = wave_sum_to_lane63(pose[q]);
        if (lane == kWave - 1) {
#pragma unroll
            for (int q = 0; q < 9; ++q) sP[v & 1][w][q] = pose[q];
        }
        __syncthreads();
        if (threadIdx.x < 9) {
            const int q = threadIdx.x;
            float t = sP[v & 1][0][q];
#pragma unroll
            for (int wv = 1; wv < NW; ++wv) t += sP[v & 1][wv][q];
            a.pose_part[((size_t)v * 9 + q) * gridDim.x + blockIdx.x] = t;
        }
    }
    if (valid && a.st_grad && !(a.skip && (*a.skip & 1u))) {
        a.st_grad[i] = st0[0] + st_grad;
        a.st_cnt[i] = st0[1] + st_cnt;
        a.st_rad[i] = fmaxf(st0[2], st_rad);
    }
    if (valid && a.per_gaussian) {
        // Sigma = M M^T, M = Rq diag(s): dL/dM = 2 GSw M
        float qw = quat0[0], qx = quat0[1], qy = quat0[2], qz = quat0[3];
        const float qnorm = sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
        const float iq = 1.0f / qnorm;
        qw *= iq; qx *= iq; qy *= iq; qz *= iq;
        float Rq[9];
        quat_rot(qw, qx, qy, qz, Rq);
        float s[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) s[q] = expf(lsc0[q]);
        const float Gs[9] = {GSw[0], GSw[1], GSw[2], GSw[1], GSw[3], GSw[4], GSw[2], GSw[4], GSw[5]};
        float GR[9];
        float gls[3];
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            float acc = 0.0f;
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                // GM[r][b] = 2 sum_q Gs[r][q] M[q][b], M[q][b] = Rq[q][b] s[b]
                const float gm =
                    2.0f * (Gs[3 * r] * Rq[b] + Gs[3 * r + 1] * Rq[3 + b] + Gs[3 * r + 2] * Rq[6 + b]) * s[b];
                acc += gm * Rq[3 * r + b];
                GR[3 * r + b] = gm * s[b];
            }
            gls[b] = acc * s[b];
        }
        float gq[4];
        gq[0] = 2.0f * (-qz * GR[1] + qy * GR[2] + qz * GR[3] - qx * GR[5] - qy * GR[6] + qx * GR[7]);
        gq[1] = 2.0f * (qy * GR[1] + qz * GR[2] + qy * GR[3] - qw * GR[5] + qz * GR[6] + qw * GR[7]) -
                4.0f * qx * (GR[4] + GR[8]);
        gq[2] = 2.0f * (qx * GR[1] + qw * GR[2] + qx * GR[3] + qz * GR[5] - qw * GR[6] + qz * GR[7]) -
                4.0f * qy * (GR[0] + GR[8]);
        gq[3] = 2.0f * (-qw * GR[1] + qx * GR[2] + qw * GR[3] + qy * GR[5] + qx * GR[6] + qy * GR[7]) -
                4.0f * qz * (GR[0] + GR[4]);
        const float dq = gq[0] * qw + gq[1] * qx + gq[2] * qy + gq[3] * qz;
        const float qh[4] = {qw, qx, qy, qz};
        if (a.dmean) {
#pragma unroll
            for (int q = 0; q < 3; ++q) a.dmean[q * n + i] = gmu[q];
        }
        if (a.dquat) {
#pragma unroll
            for (int q = 0; q < 4; ++q) a.dquat[q * n + i] = (gq[q] - qh[q] * dq) * iq;
        }
        if (a.dlog_scale) {
#pragma unroll
            for (int q = 0; q < 3; ++q) a.dlog_scale[q * n + i] = gls[q];
        }
        if (a.dopacity) {
            a.dopacity[i] = galpha * al * (1.0f - al);
        }
        // the radiosity logits' gradients, for the feature and basis
        // gradients of the second launch: z (isotropic term) and u (the
        // directional coefficients)
        if (a.zbuf) {
            a.zbuf[i] = zsum;
            if (is_dir) {
#pragma unroll
                for (int r = 0; r < KL; ++r) a.ubuf[(size_t)r * nd + id] = u[r];
            }
        }
    }
}

// Feature and basis gradients from the radiosity logits' gradients the
// projection backward leaves (z = dL/dc_iso c (1 - c) in zbuf, the
// directional coefficients' u = dL/dc c (1 - c) Y(d) in ubuf), one thread per
// Gaussian: d f = z b_iso (isotropic term) + B_dir^T u (directional term),
// and this block's share of the shared bases' gradients (Eq. 3), d B_dir[r][j]
// = sum over directional Gaussians of u_r f_j, d b_iso[j] = sum over
// isotropic ones (and every Gaussian of an entangled model) of z f_j.  Kept
// apart from the projection backward so that the features are not held
// through its chain rule.
//
// The contraction U F^T, a wave's 64 Gaussians at a time: row r of the
// wave's tile is sum u_r f over the wave, the sixteen products per lane and
// 16 columns summed by a transposing butterfly (lane 4 j ends with column
// j); a wave of isotropic Gaussians only has row 15 (z f).  The contraction
// is small beside the feature traffic (k_L + 1 rows of 16 products per
// Gaussian), so it stays on the vector ALU without operand staging.  Each
// wave leaves its tile in LDS; the block's last wave to finish adds the four
// tiles in a fixed order (no workgroup barrier: waves do not wait for each
// other).
template <int KMAX, int L>
__global__ __launch_bounds__(kBlock) void feat_grad_kernel(ProjBwdArgs a)
{
    constexpr int KL = L * (L + 2);
    constexpr int NTILE = (KMAX + 15) / 16, NCOL = NTILE * 16;
    constexpr int NW = kBlock / kWave;
    __shared__ float sT[NW][16 * NCOL];
    __shared__ float sbi[KMAX], sBd[KL * KMAX];
    __shared__ uint32_t s_done;
    const int n = a.m.n, k = a.m.k;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const bool valid = i < n;
    const int ii = valid ? i : 0;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const bool is_dir = ii >= a.m.n_iso;
    const int nd = n - a.m.n_iso, id = ii - a.m.n_iso;
    if (threadIdx.x == 0) s_done = 0;
    stage_bases<KMAX, L>(a.m, sbi, sBd);
    const float z = valid ? a.zbuf[ii] : 0.0f;
    float u[KL];
#pragma unroll
    for (int r = 0; r < KL; ++r) u[r] = 0.0f;
    if (valid && is_dir) {
#pragma unroll
        for (int r = 0; r < KL; ++r) u[r] = a.ubuf[(size_t)r * nd + id];
    }
    float fc[NCOL];
#pragma unroll
    for (int j = 0; j < NCOL; ++j) {
        // (a clamped row past k; masked)
        const float x = a.bpart ? a.m.feat[(size_t)min(j, k - 1) * n + ii] : 0.0f;
        fc[j] = (valid && j < k) ? x : 0.0f;
    }
    __syncthreads();
    const bool iso_term = !is_dir || a.m.entangled;
    if (a.dfeat && valid) {
        // (bases from LDS: sbi[j] = b_iso[j], sBd[r KMAX + j] = B_dir[r][j])
#pragma unroll
        for (int j = 0; j < KMAX; ++j) {
            if (j < k) {
                float acc = iso_term ? z * sbi[j] : 0.0f;
                if (is_dir) {
#pragma unroll
                    for (int r = 0; r < KL; ++r) acc += sBd[r * KMAX + j] * u[r];
                }
                a.dfeat[(size_t)j * n + i] = acc;
            }
        }
    }
    if (!a.bpart) return;
    float *tile = &sT[w][0];
    // row r of the tile: sum over the wave of wr f
    auto tile_row = [&](int r, float wr) {
#pragma unroll
        for (int t = 0; t < NTILE; ++t) {
            float v[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) v[j] = wr * fc[t * 16 + j];
            const float sum = wave_transpose_sum16(v);
            if ((lane & 3) == 0) tile[r * NCOL + t * 16 + (lane >> 2)] = sum;
        }
    };
    const bool dir_wave = __builtin_amdgcn_ballot_w64(valid && is_dir) != 0ull;
    for (int e = lane; e < 15 * NCOL; e += kWave)
        if (!dir_wave || e >= KL * NCOL) tile[e] = 0.0f;
    if (dir_wave) {
#pragma unroll
        for (int r = 0; r < KL; ++r) tile_row(r, u[r]);
    }
    tile_row(15, iso_term ? z : 0.0f);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    uint32_t before = 0;
    if (lane == 0) before = atomicAdd(&s_done, 1u);
    before = (uint32_t)__shfl((int)before, 0, kWave);
    if (before == NW - 1) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        for (int e = lane; e < 16 * NCOL; e += kWave)
            a.bpart[(size_t)blockIdx.x * 16 * NCOL + e] = ((sT[0][e] + sT[1][e]) + sT[2][e]) + sT[3][e];
    }
}

// FP64 reductions after the projection backward, in one launch of
// kFinalBlock-thread blocks: blocks [0, 16 NCOL) each sum one element of the
// per-wave basis tiles (when basis gradients are wanted), the next V blocks
// each turn one view's per-wave pose partials into (rho, omega).
constexpr int kFinalBlock = 256;

template <int N>
__device__ __forceinline__ void block_sum_f64(double (&x)[N], double (*red)[N])
{
#pragma unroll
    for (int q = 0; q < N; ++q) {
        double y = x[q];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) y += __shfl_xor(y, o, kWave);
        x[q] = y;
    }
    if ((threadIdx.x & (kWave - 1)) == 0)
#pragma unroll
        for (int q = 0; q < N; ++q) red[threadIdx.x / kWave][q] = x[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < N; ++q) {
        double t = 0.0;
        for (int w = 0; w < kFinalBlock / kWave; ++w) t += red[w][q];
        x[q] = t;
    }
}

template <int KMAX, int L>
__device__ void basis_final_block(int o, int k, const float *part, int nwaves, float *db, float *dB)
{
    constexpr int KL = L * (L + 2);
    constexpr int NCOL = ((KMAX + 15) / 16) * 16;
    const int i = o / NCOL, j = o % NCOL;  // (row, column) of the 16 x NCOL tile
    double s[1] = {0.0};
    for (int w = threadIdx.x; w < nwaves; w += kFinalBlock) s[0] += (double)part[((size_t)w * 16 + i) * NCOL + j];
    __shared__ double red[kFinalBlock / kWave][1];
    block_sum_f64<1>(s, red);
    if (threadIdx.x != 0 || j >= k) return;
    if (i == 15) {
        if (db) db[j] = (float)s[0];
    } else if (i < KL) {
        if (dB) dB[i * k + j] = (float)s[0];
    }
}

// dpose[v] = (rho, omega) from the per-wave partials: rho = sum d mu_c +
// sum R d r; omega = sum (R mu) x d mu_c + covariance term + t x sum d mu_c.
__device__ void pose_final_block(int v, const ViewDev *views, int n_parts, const float *part, float *dpose)
{
    double s[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) s[q] = 0.0;
    // component-major partials ([9][n_parts] per view): coalesced rows, the
    // loads of two partials in flight per thread
    const float *p = part + (size_t)v * 9 * n_parts;
    int w = threadIdx.x;
    for (; w + kFinalBlock < n_parts; w += 2 * kFinalBlock) {
        float x[2][9];
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int q = 0; q < 9; ++q) x[u][q] = p[(size_t)q * n_parts + w + u * kFinalBlock];
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int q = 0; q < 9; ++q) s[q] += (double)x[u][q];
    }
    if (w < n_parts) {
#pragma unroll
        for (int q = 0; q < 9; ++q) s[q] += (double)p[(size_t)q * n_parts + w];
    }
    __shared__ double red[kFinalBlock / kWave][9];
    block_sum_f64<9>(s, red);
    if (threadIdx.x == 0) {
        const ViewDev &V = views[v];
        const double tx = V.t[0], ty = V.t[1], tz = V.t[2];
        float *o = dpose + 6 * v;
        o[0] = (float)(s[0] + s[6]);
        o[1] = (float)(s[1] + s[7]);
        o[2] = (float)(s[2] + s[8]);
        o[3] = (float)(s[3] + ty * s[2] - tz * s[1]);
        o[4] = (float)(s[4] + tz * s[0] - tx * s[2]);
        o[5] = (float)(s[5] + tx * s[1] - ty * s[0]);
    }
}

template <int KMAX, int L>
__global__ __launch_bounds__(kFinalBlock) void grad_final_kernel(int k, const float *bpart, int bwaves, int nbasis,
                                                                 float *db, float *dB, const ViewDev *views,
                                                                 int n_parts, const float *ppart, float *dpose)
{
    const int o = blockIdx.x;
    if (o < nbasis) basis_final_block<KMAX, L>(o, k, bpart, bwaves, db, dB);
    else pose_final_block(o - nbasis, views, n_parts, ppart, dpose);
}

template <typename F>
hipError_t dispatch_kl(int k, int L, F &&f)
{
    // feature sizes 8 and 16 get exact instances; anything else <= 32 runs in
    // the 32-wide instance with the tail masked
    auto byL = [&](auto kc) -> hipError_t {
        constexpr int K = decltype(kc)::value;
        switch (L) {
        case 1: return f(std::integral_constant<int, K>{}, std::integral_constant<int, 1>{});
        case 2: return f(std::integral_constant<int, K>{}, std::integral_constant<int, 2>{});
        case 3: return f(std::integral_constant<int, K>{}, std::integral_constant<int, 3>{});
        default: return hipErrorInvalidValue;
        }
    };
    if (k == 8) return byL(std::integral_constant<int, 8>{});
    if (k == 16) return byL(std::integral_constant<int, 16>{});
    if (k >= 1 && k <= 32) return byL(std::integral_constant<int, 32>{});
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_prep_project(const ModelDev &m, const GaussCache &gc, const ViewDev *views, int V,
                               const RenderOpts &o, const ProjOut &po, hipStream_t s)
{
    if (m.n == 0 || V == 0) return hipSuccess;
    const int nb = (m.n + kBlock - 1) / kBlock;
    return dispatch_kl(m.k, m.L, [&](auto K, auto L) {
        constexpr int KK = decltype(K)::value, LL = decltype(L)::value;
        if (V == 1) {
            prep_project_kernel<KK, LL><<<nb, kBlock, 0, s>>>(m, gc, views, o, po);
        } else {
            prep_kernel<KK, LL><<<nb, kBlock, 0, s>>>(m, gc);
            project_kernel<LL><<<dim3(nb, V), kBlock, 0, s>>>(m, gc, views, o, po);
        }
        return hipGetLastError();
    });
}

hipError_t launch_project_bwd(const ProjBwdArgs &a, hipStream_t s)
{
    if (a.m.n == 0 || a.V == 0) return hipSuccess;
    return dispatch_kl(a.m.k, a.m.L, [&](auto K, auto L) {
        constexpr int KK = decltype(K)::value, LL = decltype(L)::value;
        const int nb = (a.m.n + kBlock - 1) / kBlock;
        project_bwd_kernel<KK, LL><<<nb, kBlock, 0, s>>>(a);
        if (a.zbuf && (a.dfeat || a.bpart)) feat_grad_kernel<KK, LL><<<nb, kBlock, 0, s>>>(a);
        return hipGetLastError();
    });
}

size_t basis_part_floats(int n) { return (size_t)std::max<int64_t>(1, slot_blocks(n)) * 16 * 32; }

hipError_t launch_grad_final(const ModelDev &m, const float *bpart, float *db, float *dB, const ViewDev *views,
                             int V, int n_parts, const float *ppart, float *dpose, hipStream_t s)
{
    const bool basis = (db || dB) && m.n > 0;
    const int nview = dpose ? V : 0;
    const int bwaves = (int)slot_blocks(m.n);  // one basis tile per projection-backward block
    return dispatch_kl(m.k, m.L, [&](auto K, auto L) {
        constexpr int KK = decltype(K)::value, LL = decltype(L)::value;
        constexpr int NCOL = ((KK + 15) / 16) * 16;
        const int nbasis = basis ? 16 * NCOL : 0;
        if (nbasis + nview > 0)
            grad_final_kernel<KK, LL><<<nbasis + nview, kFinalBlock, 0, s>>>(m.k, bpart, bwaves, nbasis, db, dB,
                                                                            views, n_parts, ppart, dpose);
        return hipGetLastError();
    });
}

}  // namespace ddgs
