// rads.hip -- radiodensity-aware dual sampling (Sec. 3.3) on the device: the
// interface points of the CT volume at the (min + max) / 2 level (Sec. 4.1),
// i.e. the vertices marching cubes places on voxel edges, and voxel centres
// drawn in proportion to radiodensity, plus the nearest-neighbour scales the
// Gaussians start from.
#include "internal.h"

#include <math.h>

#include <algorithm>

namespace ddgs {

namespace {

constexpr int kRadsBlock = 256;
constexpr int kScan64IPT = 16;
constexpr int kScan64Tile = kRadsBlock * kScan64IPT;

__device__ __forceinline__ bool below(float v, float iso) { return v < iso; }

__global__ __launch_bounds__(kRadsBlock) void minmax_kernel(const float *hu, int64_t n, float2 *part)
{
    __shared__ float smin[kRadsBlock], smax[kRadsBlock];
    float mn = INFINITY, mx = -INFINITY;
    for (int64_t i = (int64_t)blockIdx.x * kRadsBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kRadsBlock) {
        const float v = hu[i];
        mn = fminf(mn, v);
        mx = fmaxf(mx, v);
    }
    smin[threadIdx.x] = mn;
    smax[threadIdx.x] = mx;
    __syncthreads();
    for (int o = kRadsBlock / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            smin[threadIdx.x] = fminf(smin[threadIdx.x], smin[threadIdx.x + o]);
            smax[threadIdx.x] = fmaxf(smax[threadIdx.x], smax[threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = make_float2(smin[0], smax[0]);
}

// mm = (min, max, level = (min + max) / 2)
__global__ __launch_bounds__(kRadsBlock) void minmax_final_kernel(const float2 *part, int nb, float *mm)
{
    __shared__ float smin[kRadsBlock], smax[kRadsBlock];
    float mn = INFINITY, mx = -INFINITY;
    for (int b = threadIdx.x; b < nb; b += kRadsBlock) {
        mn = fminf(mn, part[b].x);
        mx = fmaxf(mx, part[b].y);
    }
    smin[threadIdx.x] = mn;
    smax[threadIdx.x] = mx;
    __syncthreads();
    for (int o = kRadsBlock / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            smin[threadIdx.x] = fminf(smin[threadIdx.x], smin[threadIdx.x + o]);
            smax[threadIdx.x] = fmaxf(smax[threadIdx.x], smax[threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        mm[0] = smin[0];
        mm[1] = smax[0];
        mm[2] = (smin[0] + smax[0]) * 0.5f;
    }
}

// crossings of the +x, +y, +z edges leaving each voxel centre
__global__ __launch_bounds__(kRadsBlock) void mc_count_kernel(RadsVol v, const float *mm, uint32_t *cnt)
{
    const int64_t nxy = (int64_t)v.nx * v.ny, n = nxy * v.nz;
    const int64_t i = (int64_t)blockIdx.x * kRadsBlock + threadIdx.x;
    if (i >= n) return;
    const float iso = mm[2];
    const int x = (int)(i % v.nx), y = (int)((i / v.nx) % v.ny), z = (int)(i / nxy);
    const bool a = below(v.hu[i], iso);
    uint32_t c = 0;
    if (x + 1 < v.nx) c += a != below(v.hu[i + 1], iso) ? 1u : 0u;
    if (y + 1 < v.ny) c += a != below(v.hu[i + v.nx], iso) ? 1u : 0u;
    if (z + 1 < v.nz) c += a != below(v.hu[i + nxy], iso) ? 1u : 0u;
    cnt[i] = c;
}

// the crossing points, [3][M], in edge order (voxel, then axis)
__global__ __launch_bounds__(kRadsBlock) void mc_emit_kernel(RadsVol v, const float *mm, const uint32_t *off,
                                                             float *pts, int64_t M)
{
    const int64_t nxy = (int64_t)v.nx * v.ny, n = nxy * v.nz;
    const int64_t i = (int64_t)blockIdx.x * kRadsBlock + threadIdx.x;
    if (i >= n) return;
    const float iso = mm[2];
    const int x = (int)(i % v.nx), y = (int)((i / v.nx) % v.ny), z = (int)(i / nxy);
    const float a = v.hu[i];
    const bool ba = below(a, iso);
    uint32_t o = off[i];
    const int64_t step[3] = {1, v.nx, nxy};
    const bool inside[3] = {x + 1 < v.nx, y + 1 < v.ny, z + 1 < v.nz};
    for (int ax = 0; ax < 3; ++ax) {
        if (!inside[ax]) continue;
        const float b = v.hu[i + step[ax]];
        if (ba == below(b, iso)) continue;
        const float t = (iso - a) / (b - a);
        const float gx = (float)x + (ax == 0 ? t : 0.0f);
        const float gy = (float)y + (ax == 1 ? t : 0.0f);
        const float gz = (float)z + (ax == 2 ? t : 0.0f);
        pts[o] = v.ox + gx * v.sx;
        pts[M + o] = v.oy + gy * v.sy;
        pts[2 * M + o] = v.oz + gz * v.sz;
        ++o;
    }
}

// 16-bit radiodensity weight: floor((hu - min) / (max - min) * 65535)
__device__ __forceinline__ uint32_t weight_of(float hu, const float *mm)
{
    const float mn = mm[0], mx = mm[1];
    if (!(mx > mn)) return 0u;
    return (uint32_t)floorf(((hu - mn) / (mx - mn)) * 65535.0f);
}

__device__ __forceinline__ uint64_t block_excl_scan_u64(uint64_t x, uint64_t *sh, uint64_t *total)
{
    // inclusive scan over the block's threads in LDS (Hillis-Steele), then shift
    sh[threadIdx.x] = x;
    __syncthreads();
    for (int o = 1; o < kRadsBlock; o <<= 1) {
        const uint64_t add = threadIdx.x >= (unsigned)o ? sh[threadIdx.x - o] : 0ull;
        __syncthreads();
        sh[threadIdx.x] += add;
        __syncthreads();
    }
    const uint64_t incl = sh[threadIdx.x];
    *total = sh[kRadsBlock - 1];
    __syncthreads();
    return incl - x;
}

__global__ __launch_bounds__(kRadsBlock) void scan64_reduce_kernel(const float *hu, int64_t n, const float *mm,
                                                                   uint64_t *bsum)
{
    __shared__ uint64_t sh[kRadsBlock];
    const int64_t base = (int64_t)blockIdx.x * kScan64Tile;
    uint64_t s = 0;
#pragma unroll
    for (int r = 0; r < kScan64IPT; ++r) {
        const int64_t i = base + (int64_t)r * kRadsBlock + threadIdx.x;
        if (i < n) s += weight_of(hu[i], mm);
    }
    uint64_t tot;
    (void)block_excl_scan_u64(s, sh, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// exclusive scan of the block sums in place (one block); bsum[nb] = total
__global__ __launch_bounds__(kRadsBlock) void scan64_top_kernel(uint64_t *bsum, int64_t nb)
{
    __shared__ uint64_t sh[kRadsBlock];
    uint64_t carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += kRadsBlock) {
        const int64_t b = b0 + threadIdx.x;
        const uint64_t x = b < nb ? bsum[b] : 0ull;
        uint64_t tot;
        const uint64_t ex = block_excl_scan_u64(x, sh, &tot);
        if (b < nb) bsum[b] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) bsum[nb] = carry;
}

// cdf[i] = inclusive running weight sum; each thread owns kScan64IPT
// consecutive voxels of its block's tile
__global__ __launch_bounds__(kRadsBlock) void scan64_apply_kernel(const float *hu, int64_t n, const float *mm,
                                                                  const uint64_t *bsum, uint64_t *cdf)
{
    __shared__ uint64_t sh[kRadsBlock];
    const int64_t base = (int64_t)blockIdx.x * kScan64Tile + (int64_t)threadIdx.x * kScan64IPT;
    uint32_t w[kScan64IPT];
    uint64_t s = 0;
#pragma unroll
    for (int r = 0; r < kScan64IPT; ++r) {
        const int64_t i = base + r;
        w[r] = i < n ? weight_of(hu[i], mm) : 0u;
        s += w[r];
    }
    uint64_t tot;
    uint64_t run = bsum[blockIdx.x] + block_excl_scan_u64(s, sh, &tot);
#pragma unroll
    for (int r = 0; r < kScan64IPT; ++r) {
        const int64_t i = base + r;
        run += w[r];
        if (i < n) cdf[i] = run;
    }
}

__global__ __launch_bounds__(kRadsBlock) void iota_kernel(uint32_t *p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * kRadsBlock + threadIdx.x;
    if (i < n) p[i] = (uint32_t)i;
}

// out[:, j] = src[:, idx[j]] for the first n1 sorted crossings
__global__ __launch_bounds__(kRadsBlock) void gather_kernel(const float *src, int64_t M, const uint32_t *idx,
                                                            int64_t n1, float *out, int64_t N)
{
    const int64_t j = (int64_t)blockIdx.x * kRadsBlock + threadIdx.x;
    if (j >= n1) return;
    const uint32_t i = idx[j];
    out[j] = src[i];
    out[N + j] = src[M + i];
    out[2 * N + j] = src[2 * M + i];
}

// draw j: the first voxel whose inclusive weight sum exceeds draws[j]
__global__ __launch_bounds__(kRadsBlock) void draw_kernel(RadsVol v, const uint64_t *cdf, const uint64_t *draws,
                                                          int64_t n2, float *out, int64_t N, int64_t first)
{
    const int64_t j = (int64_t)blockIdx.x * kRadsBlock + threadIdx.x;
    if (j >= n2) return;
    const uint64_t r = draws[j];
    const int64_t n = (int64_t)v.nx * v.ny * v.nz;
    int64_t lo = 0, hi = n - 1;  // answer in [lo, hi]; the last voxel if r is past the total
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (cdf[mid] > r) hi = mid;
        else lo = mid + 1;
    }
    const int64_t nxy = (int64_t)v.nx * v.ny;
    const int x = (int)(lo % v.nx), y = (int)((lo / v.nx) % v.ny), z = (int)(lo / nxy);
    out[first + j] = v.ox + (float)x * v.sx;
    out[N + first + j] = v.oy + (float)y * v.sy;
    out[2 * N + first + j] = v.oz + (float)z * v.sz;
}

// log sqrt(mean squared distance to the 3 nearest other points), by brute
// force over LDS tiles of the point set
constexpr int kKnnBlock = 128;
__global__ __launch_bounds__(kKnnBlock) void knn3_kernel(const float *pts, int64_t N, float *ls)
{
    __shared__ float tx[kKnnBlock], ty[kKnnBlock], tz[kKnnBlock];
    const int64_t i = (int64_t)blockIdx.x * kKnnBlock + threadIdx.x;
    const bool valid = i < N;
    const float px = valid ? pts[i] : 0.0f, py = valid ? pts[N + i] : 0.0f, pz = valid ? pts[2 * N + i] : 0.0f;
    float d0 = INFINITY, d1 = INFINITY, d2 = INFINITY;
    for (int64_t b = 0; b < N; b += kKnnBlock) {
        const int64_t j = b + threadIdx.x;
        if (j < N) {
            tx[threadIdx.x] = pts[j];
            ty[threadIdx.x] = pts[N + j];
            tz[threadIdx.x] = pts[2 * N + j];
        }
        __syncthreads();
        const int cnt = N - b < kKnnBlock ? (int)(N - b) : kKnnBlock;
        for (int q = 0; q < cnt; ++q) {
            const float dx = tx[q] - px, dy = ty[q] - py, dz = tz[q] - pz;
            float d = dx * dx + dy * dy + dz * dz;
            if (b + q == i) d = INFINITY;
            if (d < d2) {
                if (d < d1) {
                    d2 = d1;
                    if (d < d0) {
                        d1 = d0;
                        d0 = d;
                    } else {
                        d1 = d;
                    }
                } else {
                    d2 = d;
                }
            }
        }
        __syncthreads();
    }
    if (!valid) return;
    const int64_t kk = N - 1 < 3 ? N - 1 : 3;
    float mean = 0.0f;
    if (kk == 3) mean = (d0 + d1 + d2) / 3.0f;
    else if (kk == 2) mean = (d0 + d1) * 0.5f;
    else if (kk == 1) mean = d0;
    const float l = 0.5f * logf(fmaxf(mean, 1e-7f));
    ls[i] = l;
    ls[N + i] = l;
    ls[2 * N + i] = l;
}

int64_t blocks(int64_t n, int per) { return (n + per - 1) / per; }

}  // namespace

int64_t rads_minmax_blocks(int64_t n, int num_cu) { return std::max<int64_t>(1, std::min<int64_t>(blocks(n, kRadsBlock), (int64_t)num_cu * 8)); }
int64_t rads_scan64_blocks(int64_t n) { return std::max<int64_t>(1, blocks(n, kScan64Tile)); }

hipError_t launch_rads_level(const RadsVol &v, float2 *part, int64_t nb, float *mm, hipStream_t s)
{
    const int64_t n = (int64_t)v.nx * v.ny * v.nz;
    minmax_kernel<<<(unsigned)nb, kRadsBlock, 0, s>>>(v.hu, n, part);
    minmax_final_kernel<<<1, kRadsBlock, 0, s>>>(part, (int)nb, mm);
    return hipGetLastError();
}

hipError_t launch_mc_count(const RadsVol &v, const float *mm, uint32_t *cnt, hipStream_t s)
{
    const int64_t n = (int64_t)v.nx * v.ny * v.nz;
    mc_count_kernel<<<(unsigned)blocks(n, kRadsBlock), kRadsBlock, 0, s>>>(v, mm, cnt);
    return hipGetLastError();
}

hipError_t launch_mc_emit(const RadsVol &v, const float *mm, const uint32_t *off, float *pts, int64_t M, hipStream_t s)
{
    const int64_t n = (int64_t)v.nx * v.ny * v.nz;
    if (M == 0) return hipSuccess;
    mc_emit_kernel<<<(unsigned)blocks(n, kRadsBlock), kRadsBlock, 0, s>>>(v, mm, off, pts, M);
    return hipGetLastError();
}

hipError_t launch_rads_cdf(const RadsVol &v, const float *mm, uint64_t *bsum, uint64_t *cdf, hipStream_t s)
{
    const int64_t n = (int64_t)v.nx * v.ny * v.nz;
    const int64_t nb = rads_scan64_blocks(n);
    scan64_reduce_kernel<<<(unsigned)nb, kRadsBlock, 0, s>>>(v.hu, n, mm, bsum);
    scan64_top_kernel<<<1, kRadsBlock, 0, s>>>(bsum, nb);
    scan64_apply_kernel<<<(unsigned)nb, kRadsBlock, 0, s>>>(v.hu, n, mm, bsum, cdf);
    return hipGetLastError();
}

hipError_t launch_iota(uint32_t *p, int64_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    iota_kernel<<<(unsigned)blocks(n, kRadsBlock), kRadsBlock, 0, s>>>(p, n);
    return hipGetLastError();
}

hipError_t launch_rads_gather(const float *src, int64_t M, const uint32_t *idx, int64_t n1, float *out, int64_t N,
                              hipStream_t s)
{
    if (n1 == 0) return hipSuccess;
    gather_kernel<<<(unsigned)blocks(n1, kRadsBlock), kRadsBlock, 0, s>>>(src, M, idx, n1, out, N);
    return hipGetLastError();
}

hipError_t launch_rads_draws(const RadsVol &v, const uint64_t *cdf, const uint64_t *draws, int64_t n2, float *out,
                             int64_t N, int64_t first, hipStream_t s)
{
    if (n2 == 0) return hipSuccess;
    draw_kernel<<<(unsigned)blocks(n2, kRadsBlock), kRadsBlock, 0, s>>>(v, cdf, draws, n2, out, N, first);
    return hipGetLastError();
}

hipError_t launch_knn3(const float *pts, int64_t N, float *ls, hipStream_t s)
{
    if (N == 0) return hipSuccess;
    knn3_kernel<<<(unsigned)blocks(N, kKnnBlock), kKnnBlock, 0, s>>>(pts, N, ls);
    return hipGetLastError();
}

}  // namespace ddgs
