// fit.hip -- device work of the fitting loop (Sec. 4.1 training with Adam;
// App.: Gaussians move, split and drop during optimisation): one fused Adam
// step over every parameter group, the densification that clones, splits and
// drops Gaussians while keeping the isotropic and directional sets apart, and
// the opacity reset.
#include "internal.h"

#include <math.h>

#include <algorithm>

namespace ddgs {

int64_t fit_param_count(int64_t n, int k, int kl) { return n * (11 + k) + k + (int64_t)kl * k; }

void fit_offsets(int64_t n, int k, int kl, int64_t *off)
{
    const int64_t rows[kGroups] = {3 * n, 4 * n, 3 * n, n, (int64_t)k * n, k, (int64_t)kl * k};
    off[0] = 0;
    for (int g = 0; g < kGroups; ++g) off[g + 1] = off[g] + rows[g];
}

namespace {

constexpr int kFitBlock = 256;

// Adam on the flat parameter index (groups in model order).  The step count
// t and the schedule are read once per thread; every element is independent,
// so the kernel streams parameters, gradients and both moments once.
__global__ __launch_bounds__(kFitBlock) void fit_adam_kernel(FitArgs a)
{
    // an overflowed step leaves parameters and moments alone
    if (a.skip && (*a.skip & 1u)) return;
    const uint32_t t = *a.step + 1u;
    const double bc1 = 1.0 - pow((double)a.cfg.beta1, (double)t);
    const double bc2 = 1.0 - pow((double)a.cfg.beta2, (double)t);
    const double sfrac = fmin((double)t / (double)a.cfg.lr_steps, 1.0);
    const float lr_mean =
        (float)exp((1.0 - sfrac) * log((double)a.cfg.lr_mean0) + sfrac * log((double)a.cfg.lr_mean1));
    const float ib1 = (float)(1.0 / bc1), ib2 = (float)(1.0 / bc2);
    const float b1 = a.cfg.beta1, b2 = a.cfg.beta2, eps = a.cfg.eps;
    const int64_t total = a.off[kGroups];
    const int64_t stride = (int64_t)gridDim.x * kFitBlock;
    for (int64_t e = (int64_t)blockIdx.x * kFitBlock + threadIdx.x; e < total; e += stride) {
        int g = 0;
#pragma unroll
        for (int q = 1; q < kGroups; ++q) g += e >= a.off[q] ? 1 : 0;
        const int64_t j = e - a.off[g];
        const float grad = a.g[g][j];
        const float m = b1 * a.m[e] + (1.0f - b1) * grad;
        const float v = b2 * a.v[e] + (1.0f - b2) * grad * grad;
        a.m[e] = m;
        a.v[e] = v;
        const float lr = g == 0 ? lr_mean : a.cfg.lr[g];
        a.p[g][j] -= lr * (m * ib1) / (sqrtf(v * ib2) + eps);
    }
}

__global__ void fit_step_kernel(uint32_t *step, const uint32_t *skip)
{
    if (threadIdx.x == 0 && !(skip && (*skip & 1u))) *step = *step + 1u;
}

__global__ __launch_bounds__(kFitBlock) void densify_plan_kernel(int n, const float *ls, const float *op,
                                                                 const float *acc, const float *cnt,
                                                                 const float *rad, DensifyTh th, uint32_t *keep,
                                                                 uint32_t *clone, uint32_t *child)
{
    const int i = blockIdx.x * kFitBlock + threadIdx.x;
    if (i >= n) return;
    const float c = cnt[i];
    const float avg = c > 0.0f ? acc[i] / c : 0.0f;
    const float lmax = fmaxf(fmaxf(ls[i], ls[n + i]), ls[2 * n + i]);
    const bool big_grad = avg >= th.grad;
    const bool is_clone = big_grad && lmax <= th.log_dense;
    const bool is_split = big_grad && lmax > th.log_dense;
    const bool low_op = op[i] < th.logit_min_op;
    const bool too_big = lmax > th.log_world;
    const bool on_screen_big = rad[i] > th.screen;
    const float child_lmax = lmax - th.log_split;
    keep[i] = (!is_split && !(low_op || too_big || on_screen_big)) ? 1u : 0u;
    clone[i] = (is_clone && !(low_op || too_big)) ? 1u : 0u;
    child[i] = (is_split && !(low_op || child_lmax > th.log_world)) ? 2u : 0u;
}

// Writes source Gaussian i to the new arrays at position p; moments are
// copied for a kept original, zeroed for a new Gaussian.
__device__ __forceinline__ void put(const DensifyApplyArgs &a, int i, int64_t p, bool keep_moments)
{
    const int64_t n = a.n, nn = a.n_new;
    const int rows[5] = {3, 4, 3, 1, a.k};
    int64_t off_old = 0, off_new = 0;
    for (int g = 0; g < 5; ++g) {
        for (int r = 0; r < rows[g]; ++r) {
            a.dst[g][r * nn + p] = a.src[g][r * n + i];
            if (a.m_new) {
                a.m_new[off_new + r * nn + p] = keep_moments ? a.m_old[off_old + r * n + i] : 0.0f;
                a.v_new[off_new + r * nn + p] = keep_moments ? a.v_old[off_old + r * n + i] : 0.0f;
            }
        }
        off_old += rows[g] * n;
        off_new += rows[g] * nn;
    }
}

__global__ __launch_bounds__(kFitBlock) void densify_apply_kernel(DensifyApplyArgs a)
{
    const int i = blockIdx.x * kFitBlock + threadIdx.x;
    // moments of the shared bases follow the per-Gaussian groups
    const int nshared = a.k + a.kl * a.k;
    if (a.m_new && i < nshared) {
        const int64_t so = (int64_t)a.n * (11 + a.k), sn = a.n_new * (11 + a.k);
        a.m_new[sn + i] = a.m_old[so + i];
        a.v_new[sn + i] = a.v_old[so + i];
    }
    if (i >= a.n) return;
    const bool iso = i < a.n_iso;
    const uint32_t base = iso ? 0u : a.k_iso + a.c_iso + a.h_iso;
    const uint32_t k_set = iso ? a.k_iso : a.k_tot - a.k_iso;
    const uint32_t c_set = iso ? a.c_iso : a.c_tot - a.c_iso;
    const uint32_t pk = a.keep_ex[i] - (iso ? 0u : a.k_iso);
    const uint32_t pc = a.clone_ex[i] - (iso ? 0u : a.c_iso);
    const uint32_t ph = a.child_ex[i] - (iso ? 0u : a.h_iso);
    if (a.keep[i]) put(a, i, base + pk, true);
    if (a.clone[i]) put(a, i, base + k_set + pc, false);
    if (a.child[i]) {
        const int64_t n = a.n, nn = a.n_new;
        float qw = a.src[1][i], qx = a.src[1][n + i], qy = a.src[1][2 * n + i], qz = a.src[1][3 * n + i];
        const float iq = 1.0f / sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
        qw *= iq; qx *= iq; qy *= iq; qz *= iq;
        float R[9];
        quat_rot(qw, qx, qy, qz, R);
        float s[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) s[r] = expf(a.src[2][r * n + i]);
        for (int c = 0; c < 2; ++c) {
            const int64_t p = base + k_set + c_set + ph + c;
            put(a, i, p, false);
            const float *e = a.noise + ((int64_t)i * 2 + c) * 3;
            const float d0 = s[0] * e[0], d1 = s[1] * e[1], d2 = s[2] * e[2];
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                a.dst[0][r * nn + p] = a.src[0][r * n + i] + (R[3 * r] * d0 + R[3 * r + 1] * d1 + R[3 * r + 2] * d2);
                a.dst[2][r * nn + p] = a.src[2][r * n + i] - a.log_split;
            }
        }
    }
}

__global__ __launch_bounds__(kFitBlock) void opacity_reset_kernel(float *op, int n, float cap, float *m, float *v)
{
    const int i = blockIdx.x * kFitBlock + threadIdx.x;
    if (i >= n) return;
    op[i] = fminf(op[i], cap);
    if (m) {
        m[i] = 0.0f;
        v[i] = 0.0f;
    }
}

}  // namespace

hipError_t launch_fit_adam(const FitArgs &a, int num_cu, hipStream_t s)
{
    const int64_t total = a.off[kGroups];
    if (total == 0) return hipSuccess;
    const int64_t want = (total + kFitBlock - 1) / kFitBlock;
    const int grid = (int)std::min<int64_t>(want, (int64_t)num_cu * 16);
    fit_adam_kernel<<<grid, kFitBlock, 0, s>>>(a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    fit_step_kernel<<<1, 64, 0, s>>>(a.step, a.skip);
    return hipGetLastError();
}

hipError_t launch_densify_plan(int n, const float *log_scale, const float *opacity, const float *acc,
                               const float *cnt, const float *rad, const DensifyTh &th, uint32_t *keep,
                               uint32_t *clone, uint32_t *child, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    densify_plan_kernel<<<(n + kFitBlock - 1) / kFitBlock, kFitBlock, 0, s>>>(n, log_scale, opacity, acc, cnt, rad,
                                                                            th, keep, clone, child);
    return hipGetLastError();
}

hipError_t launch_densify_apply(const DensifyApplyArgs &a, hipStream_t s)
{
    const int work = std::max(a.n, a.k + a.kl * a.k);
    if (work <= 0) return hipSuccess;
    densify_apply_kernel<<<(work + kFitBlock - 1) / kFitBlock, kFitBlock, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_opacity_reset(float *opacity, int n, float cap, float *m, float *v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    opacity_reset_kernel<<<(n + kFitBlock - 1) / kFitBlock, kFitBlock, 0, s>>>(opacity, n, cap, m, v);
    return hipGetLastError();
}

}  // namespace ddgs
