// pose.hip -- on-device pose optimisation for registration (Sec. 4.3): one
// Adam step on every view's pose tangent (rho, omega) from the gradient of
// the step just computed, then the view is re-based so that the next replay
// of a captured step renders from the new poses.  The rotation turns about
// the source (R <- Exp(omega) R, t <- Exp(omega) t + rho: the left tangent at
// 0 the backward differentiates) or about a world pivot with source-frame
// position p = R pivot + t (t <- Exp(omega)(t - p) + p + rho).  The second
// moves every camera-frame point x by omega x (x - p) + rho to first order,
// i.e. the left tangent (rho - omega x p, omega), so its gradient is
// (g_rho, g_omega + g_rho x p).
#include "internal.h"

#include <math.h>

namespace ddgs {

namespace {

// Rodrigues: Exp(w) for a rotation vector w (FP64, series near 0).
__device__ void exp_so3(const double w[3], double E[9])
{
    const double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    const double th = sqrt(th2);
    double a, b;  // sin(th)/th, (1 - cos(th))/th^2
    if (th < 1e-4) {
        a = 1.0 - th2 / 6.0;
        b = 0.5 - th2 / 24.0;
    } else {
        a = sin(th) / th;
        b = (1.0 - cos(th)) / th2;
    }
    const double x = w[0], y = w[1], z = w[2];
    E[0] = 1.0 - b * (y * y + z * z); E[1] = -a * z + b * x * y;      E[2] = a * y + b * x * z;
    E[3] = a * z + b * x * y;         E[4] = 1.0 - b * (x * x + z * z); E[5] = -a * x + b * y * z;
    E[6] = -a * y + b * x * z;        E[7] = a * x + b * y * z;        E[8] = 1.0 - b * (x * x + y * y);
}

// One thread per view.  state: [V][12] (first moments of (rho, omega), then
// second moments); *step: completed Adam steps (shared by all views).
__global__ __launch_bounds__(256) void pose_adam_kernel(ViewDev *views, int V, const float *dpose, float *state,
                                                        uint32_t *step, AdamCfg cfg, const uint32_t *skip)
{
    // an overflowed step leaves poses, moments and the step count alone
    if (skip && (*skip & 1u)) return;
    const int v = threadIdx.x;
    const uint32_t t = *step + 1u;
    __syncthreads();  // every thread has read the step count
    if (v < V) {
        float *m = state + 12 * v, *s = m + 6;
        ViewDev &V0 = views[v];
        // pivot in the source frame (zero: rotation about the source)
        double p[3] = {0.0, 0.0, 0.0};
        if (cfg.pivot_mode == 1)
            for (int r = 0; r < 3; ++r)
                p[r] = (double)V0.R[3 * r] * cfg.pivot[0] + (double)V0.R[3 * r + 1] * cfg.pivot[1] +
                       (double)V0.R[3 * r + 2] * cfg.pivot[2] + (double)V0.t[r];
        double gv[6];
        for (int q = 0; q < 6; ++q) gv[q] = dpose[6 * v + q];
        gv[3] += gv[1] * p[2] - gv[2] * p[1];
        gv[4] += gv[2] * p[0] - gv[0] * p[2];
        gv[5] += gv[0] * p[1] - gv[1] * p[0];
        const double bc1 = 1.0 - pow((double)cfg.beta1, (double)t), bc2 = 1.0 - pow((double)cfg.beta2, (double)t);
        double d[6];
        for (int q = 0; q < 6; ++q) {
            const double g = gv[q];
            const double mq = cfg.beta1 * (double)m[q] + (1.0 - cfg.beta1) * g;
            const double sq = cfg.beta2 * (double)s[q] + (1.0 - cfg.beta2) * g * g;
            m[q] = (float)mq;
            s[q] = (float)sq;
            const double lr = q < 3 ? cfg.lr_trans : cfg.lr_rot;
            d[q] = -lr * (mq / bc1) / (sqrt(sq / bc2) + cfg.eps);
        }
        double E[9];
        exp_so3(d + 3, E);
        double R[9], tt[3];
        for (int r = 0; r < 3; ++r) {
            for (int c = 0; c < 3; ++c)
                R[3 * r + c] = E[3 * r] * V0.R[c] + E[3 * r + 1] * V0.R[3 + c] + E[3 * r + 2] * V0.R[6 + c];
            tt[r] = E[3 * r] * (V0.t[0] - p[0]) + E[3 * r + 1] * (V0.t[1] - p[1]) + E[3 * r + 2] * (V0.t[2] - p[2]) +
                    p[r] + d[r];
        }
        // keep R orthonormal in FP32 storage over many steps (Gram-Schmidt on rows)
        double n0 = sqrt(R[0] * R[0] + R[1] * R[1] + R[2] * R[2]);
        for (int c = 0; c < 3; ++c) R[c] /= n0;
        const double pr = R[0] * R[3] + R[1] * R[4] + R[2] * R[5];
        for (int c = 0; c < 3; ++c) R[3 + c] -= pr * R[c];
        const double n1 = sqrt(R[3] * R[3] + R[4] * R[4] + R[5] * R[5]);
        for (int c = 0; c < 3; ++c) R[3 + c] /= n1;
        R[6] = R[1] * R[5] - R[2] * R[4];
        R[7] = R[2] * R[3] - R[0] * R[5];
        R[8] = R[0] * R[4] - R[1] * R[3];
        for (int q = 0; q < 9; ++q) V0.R[q] = (float)R[q];
        for (int q = 0; q < 3; ++q) V0.t[q] = (float)tt[q];
        for (int q = 0; q < 3; ++q)
            V0.so[q] = (float)(-(R[q] * tt[0] + R[3 + q] * tt[1] + R[6 + q] * tt[2]));
    }
    __syncthreads();
    if (v == 0) *step = t;
}

}  // namespace

hipError_t launch_pose_adam(ViewDev *views, int V, const float *dpose, float *state, uint32_t *step,
                            const AdamCfg &cfg, const uint32_t *skip, hipStream_t s)
{
    if (V <= 0) return hipSuccess;
    if (V > 256) return hipErrorInvalidValue;
    pose_adam_kernel<<<1, 256, 0, s>>>(views, V, dpose, state, step, cfg, skip);
    return hipGetLastError();
}

}  // namespace ddgs
