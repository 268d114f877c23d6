// loss.hip -- image losses of the DRR fitting and registration steps on
// gfx950: the Eq. 2 fitting loss read as (1 - lambda) L1 + lambda D-SSIM
// (11x11 Gaussian window of std 1.5, K1 = 0.01, K2 = 0.03, dynamic range 1,
// zero padding), 1 - NCC for pose scoring, and a linear loss whose gradient
// is a fixed weight image.  Scalar reductions accumulate in FP64.
//
// SSIM: each output tile (kLossTileW x kLossTileH) stages its input halo
// (5 pixels wider on every side) in LDS and filters separably (rows, then
// columns).  The gradient needs the adjoint of
// the windowed means, which for a symmetric window with zero padding is the
// same windowed sum applied to the per-pixel partial derivatives; a second
// kernel filters those three maps the same way.
#include "internal.h"

namespace ddgs {

namespace {

constexpr int kTW = kLossTileW, kTH = kLossTileH;  // output tile
constexpr int kR = 5;                               // window radius
constexpr int kHaloW = kTW + 2 * kR, kHaloH = kTH + 2 * kR;
constexpr int kBlock = kTW * kTH;
constexpr int kBlockWaves = kBlock / kWave;

struct Window { float w[11]; };

__device__ __forceinline__ int tile_view(const int32_t *base, int V, int t)
{
    int lo = 0, hi = V - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (base[mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// the target image: through the captured step's device slot when set
__device__ __forceinline__ const float *loss_target(const LossArgs &a) { return a.target_ref ? *a.target_ref : a.target; }

// (NW waves; red holds NW x NQ doubles)
template <int NQ, int NW>
__device__ __forceinline__ void block_sum_d(double (&x)[NQ], double *red)
{
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double v = x[q];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
        x[q] = v;
    }
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < NQ; ++q) red[w * NQ + q] = x[q];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            double t = red[q];
#pragma unroll
            for (int u = 1; u < NW; ++u) t += red[u * NQ + q];
            x[q] = t;
        }
}

// 5 windowed moments per pixel: mean x, mean y, mean x^2, mean y^2, mean xy
__global__ __launch_bounds__(kBlock) void ssim_fwd_kernel(LossArgs a, Window win)
{
    __shared__ float sx[kHaloH][kHaloW + 1], sy[kHaloH][kHaloW + 1];
    __shared__ float hs[5][kHaloH][kTW + 1];
    __shared__ double red[kBlockWaves * 2];
    const int t = blockIdx.x;
    const int v = tile_view(a.loss_tile_base, a.V, t);
    const ViewDev &V = a.views[v];
    const int ntx = (V.W + kTW - 1) / kTW;
    const int lt = t - a.loss_tile_base[v];
    const int ty = lt / ntx, tx = lt - ty * ntx;
    const int ox = tx * kTW - kR, oy = ty * kTH - kR;
    const float *x = a.img + V.pix_base, *y = loss_target(a) + V.pix_base;
    for (int q = threadIdx.x; q < kHaloH * kHaloW; q += kBlock) {
        const int r = q / kHaloW, c = q % kHaloW;
        const int gx = ox + c, gy = oy + r;
        const bool in = gx >= 0 && gx < V.W && gy >= 0 && gy < V.H;
        sx[r][c] = in ? x[(size_t)gy * V.W + gx] : 0.0f;
        sy[r][c] = in ? y[(size_t)gy * V.W + gx] : 0.0f;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < kHaloH * kTW; q += kBlock) {
        const int r = q / kTW, c = q % kTW;
        float m0 = 0.f, m1 = 0.f, m2 = 0.f, m3 = 0.f, m4 = 0.f;
#pragma unroll
        for (int d = 0; d < 11; ++d) {
            const float xv = sx[r][c + d], yv = sy[r][c + d], wd = win.w[d];
            m0 += wd * xv; m1 += wd * yv; m2 += wd * xv * xv; m3 += wd * yv * yv; m4 += wd * xv * yv;
        }
        hs[0][r][c] = m0; hs[1][r][c] = m1; hs[2][r][c] = m2; hs[3][r][c] = m3; hs[4][r][c] = m4;
    }
    __syncthreads();
    const int lx = threadIdx.x % kTW, ly = threadIdx.x / kTW;
    const int gx = tx * kTW + lx, gy = ty * kTH + ly;
    double part[2] = {0.0, 0.0};
    if (gx < V.W && gy < V.H) {
        float mo[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int d = 0; d < 11; ++d)
#pragma unroll
            for (int q = 0; q < 5; ++q) mo[q] += win.w[d] * hs[q][ly + d][lx];
        const float C1 = 0.01f * 0.01f, C2 = 0.03f * 0.03f;
        const float ux = mo[0], uy = mo[1];
        const float vx = mo[2] - ux * ux, vy = mo[3] - uy * uy, cxy = mo[4] - ux * uy;
        const float A1 = 2.0f * ux * uy + C1, A2 = 2.0f * cxy + C2;
        const float B1 = ux * ux + uy * uy + C1, B2 = vx + vy + C2;
        const float D = B1 * B2, iD = 1.0f / D;
        const float s = A1 * A2 * iD;
        const float xv = sx[ly + kR][lx + kR], yv = sy[ly + kR][lx + kR];
        part[0] = s;
        part[1] = fabsf(xv - yv);
        const size_t p = (size_t)V.pix_base + (size_t)gy * V.W + gx;
        a.maps[p] = (2.0f * uy * (A2 - A1) - s * 2.0f * ux * (B2 - B1)) * iD;   // d s / d mean x
        a.maps[a.total_pix + p] = -s * B1 * iD;                                 // d s / d mean x^2
        a.maps[2 * a.total_pix + p] = 2.0f * A1 * iD;                           // d s / d mean xy
    }
    block_sum_d<2, kBlockWaves>(part, red);
    if (threadIdx.x == 0) {
        a.part[2 * (size_t)t] = part[0];
        a.part[2 * (size_t)t + 1] = part[1];
    }
}

// Loss of view v from the per-tile partial sums of the forward (one block of
// kBlock threads; FP64 sums in a fixed order).
__device__ void ssim_final_view(const LossArgs &a, int v)
{
    const int t0 = a.loss_tile_base[v], t1 = a.loss_tile_base[v + 1];
    double x[2] = {0.0, 0.0};
    for (int t = t0 + threadIdx.x; t < t1; t += kBlock) {
        x[0] += a.part[2 * (size_t)t];
        x[1] += a.part[2 * (size_t)t + 1];
    }
    __shared__ double red[kBlockWaves * 2];
    block_sum_d<2, kBlockWaves>(x, red);
    if (threadIdx.x == 0 && a.loss_out) {
        const ViewDev &V = a.views[v];
        const double P = (double)V.W * (double)V.H;
        a.loss_out[v] = (float)((1.0 - a.lambda) * x[1] / P + a.lambda * (1.0 - x[0] / P));
    }
}

__global__ __launch_bounds__(kBlock) void ssim_bwd_kernel(LossArgs a, Window win)
{
    __shared__ float sm[3][kHaloH][kHaloW + 1];
    __shared__ float hs[3][kHaloH][kTW + 1];
    const int t = blockIdx.x;
    // the forward's partial sums are complete: the first V blocks also
    // finish the views' loss values (every view has at least one tile)
    if (t < a.V) ssim_final_view(a, t);
    const int v = tile_view(a.loss_tile_base, a.V, t);
    const ViewDev &V = a.views[v];
    const int ntx = (V.W + kTW - 1) / kTW;
    const int lt = t - a.loss_tile_base[v];
    const int ty = lt / ntx, tx = lt - ty * ntx;
    const int ox = tx * kTW - kR, oy = ty * kTH - kR;
    for (int q = threadIdx.x; q < kHaloH * kHaloW; q += kBlock) {
        const int r = q / kHaloW, c = q % kHaloW;
        const int gx = ox + c, gy = oy + r;
        const bool in = gx >= 0 && gx < V.W && gy >= 0 && gy < V.H;
        const size_t p = (size_t)V.pix_base + (size_t)gy * V.W + gx;
#pragma unroll
        for (int m = 0; m < 3; ++m) sm[m][r][c] = in ? a.maps[m * a.total_pix + p] : 0.0f;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < kHaloH * kTW; q += kBlock) {
        const int r = q / kTW, c = q % kTW;
        float m0 = 0.f, m1 = 0.f, m2 = 0.f;
#pragma unroll
        for (int d = 0; d < 11; ++d) {
            m0 += win.w[d] * sm[0][r][c + d];
            m1 += win.w[d] * sm[1][r][c + d];
            m2 += win.w[d] * sm[2][r][c + d];
        }
        hs[0][r][c] = m0; hs[1][r][c] = m1; hs[2][r][c] = m2;
    }
    __syncthreads();
    const int lx = threadIdx.x % kTW, ly = threadIdx.x / kTW;
    const int gx = tx * kTW + lx, gy = ty * kTH + ly;
    if (gx >= V.W || gy >= V.H) return;
    float f0 = 0.f, f1 = 0.f, f2 = 0.f;
#pragma unroll
    for (int d = 0; d < 11; ++d) {
        f0 += win.w[d] * hs[0][ly + d][lx];
        f1 += win.w[d] * hs[1][ly + d][lx];
        f2 += win.w[d] * hs[2][ly + d][lx];
    }
    const size_t p = (size_t)V.pix_base + (size_t)gy * V.W + gx;
    const float xv = a.img[p], yv = loss_target(a)[p];
    const float P = (float)V.W * (float)V.H;
    const float d = xv - yv;
    const float sg = (d > 0.0f) ? 1.0f : ((d < 0.0f) ? -1.0f : 0.0f);
    a.grad[p] = ((1.0f - a.lambda) * sg - a.lambda * (f0 + 2.0f * xv * f1 + yv * f2)) / P;
}

__global__ __launch_bounds__(kBlock) void ssim_final_kernel(LossArgs a) { ssim_final_view(a, blockIdx.x); }

// ------------------------------------------------------------------- NCC

constexpr int kChunk = 4096;

__global__ __launch_bounds__(256) void ncc_stats_kernel(LossArgs a, int nchunks)
{
    const int v = blockIdx.y;
    const ViewDev &V = a.views[v];
    const int64_t P = (int64_t)V.W * V.H;
    const int64_t p0 = (int64_t)blockIdx.x * kChunk;
    const float *tg = loss_target(a);
    double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t p = p0 + threadIdx.x; p < min(P, p0 + kChunk); p += 256) {
        const double x = a.img[V.pix_base + p], y = tg[V.pix_base + p];
        s[0] += x; s[1] += y; s[2] += x * x; s[3] += y * y; s[4] += x * y;
    }
    __shared__ double red[4 * 5];
    block_sum_d<5, 4>(s, red);
    if (threadIdx.x == 0)
#pragma unroll
        for (int q = 0; q < 5; ++q) a.part[((size_t)v * nchunks + blockIdx.x) * 5 + q] = s[q];
}

// per view: means, standard deviations (eps added to the variances) and NCC
__global__ __launch_bounds__(256) void ncc_final_kernel(LossArgs a, int nchunks, double *stats)
{
    const int v = blockIdx.x;
    const ViewDev &V = a.views[v];
    const double P = (double)V.W * (double)V.H;
    double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int c = threadIdx.x; c < nchunks; c += 256)
#pragma unroll
        for (int q = 0; q < 5; ++q) s[q] += a.part[((size_t)v * nchunks + c) * 5 + q];
    __shared__ double red[4 * 5];
    block_sum_d<5, 4>(s, red);
    if (threadIdx.x == 0) {
        const double mx = s[0] / P, my = s[1] / P;
        const double vx = fmax(s[2] / P - mx * mx, 0.0), vy = fmax(s[3] / P - my * my, 0.0);
        const double cv = s[4] / P - mx * my;
        const double sx = sqrt(vx + 1e-12), sy = sqrt(vy + 1e-12);
        const double ncc = cv / (sx * sy);
        stats[4 * v] = mx; stats[4 * v + 1] = my; stats[4 * v + 2] = sx; stats[4 * v + 3] = ncc;
        if (a.loss_out) a.loss_out[v] = (float)(1.0 - ncc);
        stats[4 * (size_t)a.V + v] = sy;
    }
}

__global__ __launch_bounds__(256) void ncc_grad_kernel(LossArgs a, const double *stats)
{
    const int v = blockIdx.y;
    const ViewDev &V = a.views[v];
    const int64_t P = (int64_t)V.W * V.H;
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= P) return;
    const float mx = (float)stats[4 * v], my = (float)stats[4 * v + 1], sx = (float)stats[4 * v + 2];
    const float ncc = (float)stats[4 * v + 3], sy = (float)stats[4 * (size_t)a.V + v];
    const float xh = (a.img[V.pix_base + p] - mx) / sx;
    const float yh = (loss_target(a)[V.pix_base + p] - my) / sy;
    a.grad[V.pix_base + p] = -(yh - ncc * xh) / ((float)P * sx);
}

// ---------------------------------------------------------------- linear

__global__ __launch_bounds__(256) void linear_kernel(LossArgs a, int nchunks)
{
    const int v = blockIdx.y;
    const ViewDev &V = a.views[v];
    const int64_t P = (int64_t)V.W * V.H;
    const int64_t p0 = (int64_t)blockIdx.x * kChunk;
    const float *tg = loss_target(a);
    double s[1] = {0.0};
    for (int64_t p = p0 + threadIdx.x; p < min(P, p0 + kChunk); p += 256) {
        const float w = tg[V.pix_base + p];
        s[0] += (double)w * a.img[V.pix_base + p];
        if (a.grad) a.grad[V.pix_base + p] = w;
    }
    __shared__ double red[4];
    block_sum_d<1, 4>(s, red);
    if (threadIdx.x == 0) a.part[(size_t)v * nchunks + blockIdx.x] = s[0];
}

__global__ __launch_bounds__(256) void linear_final_kernel(LossArgs a, int nchunks)
{
    const int v = blockIdx.x;
    double s[1] = {0.0};
    for (int c = threadIdx.x; c < nchunks; c += 256) s[0] += a.part[(size_t)v * nchunks + c];
    __shared__ double red[4];
    block_sum_d<1, 4>(s, red);
    if (threadIdx.x == 0 && a.loss_out) a.loss_out[v] = (float)s[0];
}

Window make_window()
{
    Window w;
    double g[11], s = 0.0;
    for (int i = 0; i < 11; ++i) {
        g[i] = std::exp(-double((i - 5) * (i - 5)) / (2.0 * 1.5 * 1.5));
        s += g[i];
    }
    for (int i = 0; i < 11; ++i) w.w[i] = (float)(g[i] / s);
    return w;
}

}  // namespace

size_t loss_part_doubles(int V, int64_t max_view_pix, int loss_tiles)
{
    const int64_t nchunks = (max_view_pix + kChunk - 1) / kChunk + 1;
    return (size_t)std::max<int64_t>(2 * (int64_t)loss_tiles, 5 * (int64_t)V * nchunks) + 8 * (size_t)V + 16;
}

hipError_t launch_loss(int kind, const LossArgs &a, hipStream_t s)
{
    if (a.V == 0) return hipSuccess;
    // the largest view decides the chunk grid; blocks past a smaller view exit
    const int64_t maxP = a.max_view_pix;
    if (kind == 0) {
        const Window w = make_window();
        ssim_fwd_kernel<<<a.loss_tiles, kBlock, 0, s>>>(a, w);
        if (a.grad) ssim_bwd_kernel<<<a.loss_tiles, kBlock, 0, s>>>(a, w);
        else ssim_final_kernel<<<a.V, kBlock, 0, s>>>(a);
        return hipGetLastError();
    }
    const int nchunks = (int)((maxP + kChunk - 1) / kChunk);
    if (kind == 1) {
        double *stats = a.part + (size_t)5 * a.V * nchunks;
        ncc_stats_kernel<<<dim3(nchunks, a.V), 256, 0, s>>>(a, nchunks);
        ncc_final_kernel<<<a.V, 256, 0, s>>>(a, nchunks, stats);
        if (a.grad) ncc_grad_kernel<<<dim3((unsigned)((maxP + 255) / 256), a.V), 256, 0, s>>>(a, stats);
        return hipGetLastError();
    }
    if (kind == 2) {
        linear_kernel<<<dim3(nchunks, a.V), 256, 0, s>>>(a, nchunks);
        linear_final_kernel<<<a.V, 256, 0, s>>>(a, nchunks);
        return hipGetLastError();
    }
    return hipErrorInvalidValue;
}

}  // namespace ddgs
