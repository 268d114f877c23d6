// raster.hip -- per-tile compositing of Eq. 1 on gfx950 and its backward.
//
// Work items.  A work item is a (tile, depth chunk) pair: the tile's
// depth-ordered list is cut into chunks of `split` entries (split = 0: one
// item per tile).  Chunking bounds the serial walk of any one workgroup, so
// tiles with very long lists no longer set the kernel's critical path, and
// the 256 CUs get thousands of similar-sized items.  Eq. 1 is a left fold
// of the "over" operator (C, T) o (C', T') = (C + T C', T T'), which is
// associative, so chunk results are merged exactly in depth order by a
// small merge kernel (which also stores, for every chunk, the (C, T) in
// front of it for the backward).  With split = 0 the image is bit-identical
// for every tile shape; with chunks it differs only by rounding.
//
// Inside an item one workgroup owns the tile and one lane owns one pixel.
// The item's entries are staged in LDS in batches (one 32-byte record per
// entry) and read back as wave-wide broadcasts.  The per-pair arithmetic is
// written with explicit round-to-nearest intrinsics so that the forward and
// the backward (which recomputes the transmittance instead of storing it)
// take bit-identical decisions.
//
// Backward: the tail S_j = sum_{m>j} c_m s_m T_m is the saved pixel value
// minus the running sum.  Per-pair image-plane gradients are summed over the
// wave with DPP row operations (VALU only, no LDS round trip), over the
// waves of the workgroup in LDS in a fixed order, and written once per tile
// entry into its own slot (the pair's first slot plus the tile's row-major
// place in the pair's rectangle) -- no float atomics, so the gradients are
// run-to-run deterministic.
#include "internal.h"

namespace ddgs {

namespace {

// The falloff exponent.  The conic is staged in LDS pre-multiplied by
// kExpScale = -log2(e) / 2 (A00 k, 2 A01 k, A11 k), so that
// e = dx (A00' dx + B' dy) + A11' dy dy -- five rounded operations, the same
// in the forward and the backward -- is -d2 / 2 in base-2 units: the falloff
// exp(-d2 / 2) is v_exp_f32(e), and the cut-off d2 <= kappa^2 becomes
// e >= kappa^2 k (both sides scaled by the same negative factor).
constexpr float kExpScale = -0.7213475108146667f;  // 0xBF38AA3B, -log2(e) / 2
__device__ __forceinline__ float falloff_exponent(float dx, float dy, float A00, float B, float A11)
{
    const float u = __fmaf_rn(B, dy, __fmul_rn(A00, dx));
    return __fmaf_rn(dx, u, __fmul_rn(__fmul_rn(A11, dy), dy));
}
// The staged conic of a record: (mx, my, A00 k, 2 A01 k) and (A11 k, alpha, c, .)
__device__ __forceinline__ void scale_conic(float4 &r0, float4 &r1)
{
    r0.z = __fmul_rn(r0.z, kExpScale);
    r0.w = __fmul_rn(2.0f * r0.w, kExpScale);
    r1.x = __fmul_rn(r1.x, kExpScale);
}
// Cut-off value of a lane: kappa^2 k (< 0) while it composites, +infinity
// (which no exponent of a finite record reaches) once it has stopped or lies
// outside the image.
constexpr float kLaneOff = __builtin_huge_valf();

// min(s, sigma_max) for s = alpha G >= 0 as one v_med3_f32 (median of s,
// 0 and sigma_max), without the NaN canonicalisation fminf brings.
__device__ __forceinline__ float clamp_opacity(float s, float smax) { return __builtin_amdgcn_fmed3f(s, 0.0f, smax); }
// 1 - s for an unclamped s = alpha G, in one rounding (the same in the
// forward and every backward)
__device__ __forceinline__ float one_minus_alpha_g(float alpha, float G) { return __fmaf_rn(-alpha, G, 1.0f); }

// Wave-wide OR of a predicate as a lane mask (the compare mask itself).
__device__ __forceinline__ uint64_t wave_any_mask(bool p) { return __builtin_amdgcn_ballot_w64(p); }


__device__ __forceinline__ int view_of_tile(const ViewDev *views, int V, int tile)
{
    int lo = 0, hi = V - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (views[mid].tile_base <= tile) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

struct Item {
    int tile;
    uint32_t b, e;    // entry range [b, e) of the item
    int chunk;
};

// Resolves work item `it`; tile < 0 when `it` is past the last item.  The
// item is built in registers and returned whole (field-wise stores through
// a reference were kept in scratch memory by the compiler).
__device__ __forceinline__ Item resolve_item(const RasterArgs &a, int it)
{
    int tile = -1, chunk = 0;
    uint32_t b = 0, e = 0;
    if (it != 0x7FFFFFFF) {
        if (a.split == 0) {
            if (it < a.n_tiles) {
                const uint2 rg = a.ranges[it];
                tile = it;
                b = rg.x;
                e = rg.y;
            }
        } else if (it < (int)*a.n_items) {
            const uint2 q = a.items[it];
            const uint2 rg = a.ranges[q.x];
            tile = (int)q.x;
            chunk = (int)q.y;
            b = rg.x + q.y * (uint32_t)a.split;
            e = min(rg.y, b + (uint32_t)a.split);
        }
    }
    return Item{__builtin_amdgcn_readfirstlane(tile), (uint32_t)__builtin_amdgcn_readfirstlane((int)b),
                (uint32_t)__builtin_amdgcn_readfirstlane((int)e), __builtin_amdgcn_readfirstlane(chunk)};
}

// Item of block b when blocks map to items directly.  Workgroups are dealt
// to the eight XCDs in turn (block b to XCD b mod 8), and each XCD has its
// own L2: XCD x gets the x-th contiguous eighth of the n items, so that
// neighbouring tiles, which share most of their Gaussians, read those
// records through the same L2.  The grid is a multiple of 8 and at least n.
__device__ __forceinline__ int xcd_item(int b, int n)
{
    const int per = (n + 7) >> 3;
    const int k = b >> 3;
    return k < per ? (b & 7) * per + k : 0x7FFFFFFF;
}

// Next work item of this workgroup: the item of its block once, or
// (persistent mode) items taken from a shared counter until none are left.
__device__ __forceinline__ int next_item(const RasterArgs &a, int &iter, int *sh)
{
    if (!a.queue_counter) {
        const int n = a.split ? (int)*a.n_items : a.n_tiles;
        const int t = iter == 0 ? xcd_item((int)blockIdx.x, n) : 0x7FFFFFFF;
        ++iter;
        return t;
    }
    __syncthreads();
    if (threadIdx.x == 0) *sh = (int)atomicAdd(a.queue_counter, 1u);
    __syncthreads();
    const int k = *sh;
    ++iter;
    const int limit = a.split ? (int)*a.n_items : a.n_tiles;
    if (k >= limit) return 0x7FFFFFFF;
    return a.queue ? (int)a.queue[k] : k;
}

// SPLIT: work items are chunks (a.split > 0), so no per-pixel last index is
// kept; COUNT: pair counters on.
template <int TW, int TH, bool SPLIT, bool COUNT>
__global__ __launch_bounds__(TW *TH) void raster_fwd_kernel(RasterArgs a)
{
    constexpr int NT = TW * TH;
    __shared__ float4 s0[NT];
    __shared__ float4 s1[NT];
    __shared__ int sh_item;
    const int tid = threadIdx.x;
    const float k2s = __fmul_rn(a.o.kappa2, kExpScale), tmin = a.o.t_min;
    const float smax = a.o.sigma_max;
    int iter = 0;
    for (;;) {
        const int it = next_item(a, iter, &sh_item);
        const Item I = resolve_item(a, it);
        if (I.tile < 0) break;
        const int v = view_of_tile(a.views, a.V, I.tile);
        const ViewDev &V = a.views[v];
        const int lt = I.tile - V.tile_base;
        const int ty = lt / V.ntx, tx = lt - ty * V.ntx;
        const int px = tx * TW + tid % TW, py = ty * TH + tid / TW;
        const bool inside = px < V.W && py < V.H;
        const float fpx = (float)px + 0.5f, fpy = (float)py + 0.5f;
        const size_t vbase = (size_t)v * a.n;
        float T = 1.0f, C = 0.0f;
        uint32_t last = I.b;
        uint32_t n_eval = 0, n_contrib = 0;
        // the cut-off test with the lane's state folded in (kLaneOff once the
        // lane has stopped or lies outside the image), so that a hit is one
        // compare and its wave ballot costs no vector instruction
        float k2e = inside ? k2s : kLaneOff;
        // one entry: when any lane hits, the whole wave runs it without
        // branches; lanes that miss keep their state.  CLAMP: some entry of
        // the batch has alpha > sigma_max / 2.  Otherwise alpha G stays below
        // sigma_max with a factor-two margin (G <= 1, up to the rounding of
        // its exponent) and the clamp min(alpha G, sigma_max) is the identity
        auto entry = [&](const float4 r0, const float4 r1, uint32_t pos, auto clamp_c) {
            constexpr bool CLAMP = decltype(clamp_c)::value;
            const float dx = __fsub_rn(fpx, r0.x), dy = __fsub_rn(fpy, r0.y);
            const float ex = falloff_exponent(dx, dy, r0.z, r0.w, r1.x);
            bool hit = ex >= k2e;
            if (wave_any_mask(hit) != 0ull) {
                // (an empty volatile asm keeps this a branch: the compiler would
                // otherwise turn the entry into selects, which run it, and
                // two more selects, even when no lane hits)
                asm volatile("");
                // lanes that miss run the same arithmetic with G = 0: s = 0,
                // 1 - s = 1, so C and T stay exactly as they are
                float G = hit ? __builtin_amdgcn_exp2f(ex) : 0.0f;
                float s = __fmul_rn(r1.y, G), om;
                if constexpr (CLAMP) {
                    s = clamp_opacity(s, smax);
                    om = __fsub_rn(1.0f, s);
                } else {
                    om = one_minus_alpha_g(r1.y, G);
                }
                if constexpr (!SPLIT) {
                    // early termination (t_min > 0 runs unsplit): the lane
                    // stops before this entry
                    if (tmin > 0.0f) {
                        const bool stop = hit & (__fmul_rn(T, om) < tmin);
                        k2e = stop ? kLaneOff : k2e;
                        hit = hit & !stop;
                        s = stop ? 0.0f : s;
                        om = stop ? 1.0f : om;
                    }
                }
                // C += c (s T); T *= 1 - s exactly as the backward recomputes it
                C = __fmaf_rn(r1.z, __fmul_rn(s, T), C);
                T = __fmul_rn(T, om);
                if constexpr (!SPLIT) last = hit ? pos + 1u : last;
                if constexpr (COUNT) n_contrib += hit ? 1u : 0u;
            }
        };
        // the batch's entries in order, four records read together (one LDS
        // address, immediate offsets)
        auto run_batch = [&](uint32_t b0, int cnt, auto clamp_c) {
            int q = 0;
            for (; q + 4 <= cnt; q += 4) {
                float4 r0[4], r1[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    r0[u] = s0[q + u];
                    r1[u] = s1[q + u];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) entry(r0[u], r1[u], b0 + (uint32_t)(q + u), clamp_c);
            }
            for (; q < cnt; ++q) entry(s0[q], s1[q], b0 + (uint32_t)q, clamp_c);
        };
        for (uint32_t b0 = I.b; b0 < I.e; b0 += NT) {
            __syncthreads();
            const uint32_t j = b0 + tid;
            bool over = false;  // an opacity above sigma_max / 2 in this batch
            if (j < I.e) {
                const uint32_t gid = min(a.tval[j], (uint32_t)a.n - 1u);
                const size_t idx = vbase + gid;
                float4 r0 = a.rec[4 * idx], r1 = a.rec[4 * idx + 1];
                over = r1.y > 0.5f * smax;
                scale_conic(r0, r1);
                s0[tid] = r0;
                s1[tid] = r1;
            }
            const bool clamp = __syncthreads_or(over);
            const int cnt = (int)min((uint32_t)NT, I.e - b0);
            if (COUNT && k2e < 0.0f) n_eval += (uint32_t)cnt;
            if (clamp) run_batch(b0, cnt, std::true_type{});
            else run_batch(b0, cnt, std::false_type{});
            if (tmin > 0.0f && __syncthreads_and(k2e == kLaneOff)) break;
        }
        if constexpr (COUNT) {
            unsigned long long e = n_eval, c = n_contrib;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                e += __shfl_xor(e, o, kWave);
                c += __shfl_xor(c, o, kWave);
            }
            if ((tid & (kWave - 1)) == 0) {
                // 64 counter pairs, chosen by block, keep the atomics uncontended
                const int slot = (int)(blockIdx.x & 63u);
                atomicAdd(&a.pair_counts[2 * slot], e);
                atomicAdd(&a.pair_counts[2 * slot + 1], c);
            }
        }
        if constexpr (SPLIT) {
            a.part[(size_t)it * NT + tid] = make_float2(C, T);
        } else if (inside) {
            const size_t p = (size_t)V.pix_base + (size_t)py * V.W + px;
            a.img[p] = C;
            a.img_saved[p] = C;
            a.nlast[p] = last;
        }
    }
}

// Forward of 8 x 8 tiles in chunks (the tuned shape) with an entry list per
// 4 x 4 quadrant.  An entry's cut-off ellipse usually covers a part of the
// tile, and a wave that runs it on all 64 pixels spends most lanes on misses.
// Here lane l covers pixel (4 (q % 2) + r % 4, 4 (q / 2) + r / 4) of the tile
// (q = l / 16, r = l % 16); each batch of entries is listed per quadrant
// whose pixel centres the ellipse's bounding box reaches (half-widths
// kappa sqrt(Sigma_xx), kappa sqrt(Sigma_yy) of Sigma = A^-1, widened by
// 0.1 %, far above the rounding of the per-pixel test), and the wave runs the
// longest list, the lanes of each quadrant taking their own list's entries
// in depth order (shorter lists are padded with a record that no pixel
// reaches).  An entry left out of a quadrant's list misses all its pixels,
// where the update is an exact no-op, so the images and chunk results equal
// the unculled kernel's bit for bit.  The chunk results are stored by pixel
// (row-major in the tile), as the other kernels index them.
__global__ __launch_bounds__(kWave) void raster_fwd_quad_kernel(RasterArgs a)
{
    constexpr int TW = 8, TH = 8, NT = TW * TH, NUL = NT;
    static_assert(NT == kWave, "one wave per tile");
    // records by entry, s1 first: entry e's pair sits at byte 16 e (s1) and
    // 16 e + S0OFF (s0), so that one register with two immediate offsets
    // reads it; the lists hold these byte places
    constexpr uint32_t S0OFF = 16u * (NT + 1);
    __shared__ float4 s10[2 * (NT + 1)];
    float4 *const s1 = s10;
    float4 *const s0 = s10 + (NT + 1);
    // per quadrant: the byte places of its entries (rows four words apart in
    // bank, so that the four quadrants' reads of one step do not collide)
    __shared__ __align__(16) uint32_t ql[4][NT + 4];
    __shared__ int sh_item;
    const int tid = threadIdx.x;
    const int qd = tid >> 4, qr = tid & 15;
    const int lx = 4 * (qd & 1) + (qr & 3), ly = 4 * (qd >> 1) + (qr >> 2);
    const float k2s = __fmul_rn(a.o.kappa2, kExpScale);
    const float smax = a.o.sigma_max;
    const float kw = a.o.kappa * 1.001f;
    if (tid == 0) {
        // the padding record: d^T A d = -(dx^2 + dy^2) ~ -2e36 < any cut-off
        s0[NUL] = make_float4(1e18f, 1e18f, -1.0f, 0.0f);
        s1[NUL] = make_float4(-1.0f, 0.0f, 0.0f, 0.0f);
    }
    const char *const srec = reinterpret_cast<const char *>(s10);
    int iter = 0;
    for (;;) {
        const int it = next_item(a, iter, &sh_item);
        const Item I = resolve_item(a, it);
        if (I.tile < 0) break;
        const int v = view_of_tile(a.views, a.V, I.tile);
        const ViewDev &V = a.views[v];
        const int lt = I.tile - V.tile_base;
        const int ty = lt / V.ntx, tx = lt - ty * V.ntx;
        const int px = tx * TW + lx, py = ty * TH + ly;
        const bool inside = px < V.W && py < V.H;
        const float fpx = (float)px + 0.5f, fpy = (float)py + 0.5f;
        const float tx0 = (float)(tx * TW), ty0 = (float)(ty * TH);
        const size_t vbase = (size_t)v * a.n;
        float T = 1.0f, C = 0.0f;
        const float k2e = inside ? k2s : kLaneOff;
        auto entry = [&](const float4 r0, const float4 r1, auto clamp_c) {
            constexpr bool CLAMP = decltype(clamp_c)::value;
            const float dx = __fsub_rn(fpx, r0.x), dy = __fsub_rn(fpy, r0.y);
            const float ex = falloff_exponent(dx, dy, r0.z, r0.w, r1.x);
            const bool hit = ex >= k2e;
            if (wave_any_mask(hit) != 0ull) {
                asm volatile("");
                const float G = hit ? __builtin_amdgcn_exp2f(ex) : 0.0f;
                float s = __fmul_rn(r1.y, G), om;
                if constexpr (CLAMP) {
                    s = clamp_opacity(s, smax);
                    om = __fsub_rn(1.0f, s);
                } else {
                    om = one_minus_alpha_g(r1.y, G);
                }
                C = __fmaf_rn(r1.z, __fmul_rn(s, T), C);
                T = __fmul_rn(T, om);
            }
        };
        // the longest list in steps of four: four places of the lane's list,
        // then their records
        const uint32_t *const myl = &ql[qd][0];
        auto run_lists = [&](int nmax, auto clamp_c) {
            for (int i0 = 0; i0 < nmax; i0 += 4) {
                const uint4 ev = *reinterpret_cast<const uint4 *>(myl + i0);
                const uint32_t e[4] = {ev.x, ev.y, ev.z, ev.w};
                float4 r0[4], r1[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    r1[u] = *reinterpret_cast<const float4 *>(srec + e[u]);
                    r0[u] = *reinterpret_cast<const float4 *>(srec + e[u] + S0OFF);
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) entry(r0[u], r1[u], clamp_c);
            }
        };
        for (uint32_t b0 = I.b; b0 < I.e; b0 += NT) {
            __syncthreads();
            const uint32_t j = b0 + tid;
            bool over = false;  // an opacity above sigma_max / 2 in this batch
            uint32_t qm = 0u;   // quadrants this lane's entry reaches
            if (j < I.e) {
                const uint32_t gid = min(a.tval[j], (uint32_t)a.n - 1u);
                const size_t idx = vbase + gid;
                float4 r0 = a.rec[4 * idx], r1 = a.rec[4 * idx + 1];
                over = r1.y > 0.5f * smax;
                // bounding box of the cut-off ellipse against the quadrants'
                // pixel-centre ranges [0.5, 3.5] and [4.5, 7.5] of the tile
                const float idet = 1.0f / (r0.z * r1.x - r0.w * r0.w);
                const float hx = kw * sqrtf(r1.x * idet), hy = kw * sqrtf(r0.z * idet);
                const float ux = r0.x - tx0, uy = r0.y - ty0;
                const bool xa = ux - hx <= 3.5f && ux + hx >= 0.5f, xb = ux - hx <= 7.5f && ux + hx >= 4.5f;
                const bool ya = uy - hy <= 3.5f && uy + hy >= 0.5f, yb = uy - hy <= 7.5f && uy + hy >= 4.5f;
                qm = (xa && ya ? 1u : 0u) | (xb && ya ? 2u : 0u) | (xa && yb ? 4u : 0u) | (xb && yb ? 8u : 0u);
                scale_conic(r0, r1);
                s0[tid] = r0;
                s1[tid] = r1;
            }
            // lists: every place first holds the padding record, then each
            // quadrant's entries in batch order
            reinterpret_cast<uint4 *>(&ql[qd][4 * qr])[0] = make_uint4(16u * NUL, 16u * NUL, 16u * NUL, 16u * NUL);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            int nmax = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const bool in = (qm >> q) & 1u;
                const uint64_t b = wave_any_mask(in);
                if (in) {
                    const uint32_t pos = __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32),
                                                                   __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
                    ql[q][pos] = 16u * (uint32_t)tid;
                }
                nmax = max(nmax, (int)__popcll(b));
            }
            const bool clamp = __syncthreads_or(over);
            if (clamp) run_lists(nmax, std::true_type{});
            else run_lists(nmax, std::false_type{});
        }
        a.part[(size_t)it * NT + ly * TW + lx] = make_float2(C, T);
    }
}

// Split mode: folds each tile's chunk results in depth order with the over
// operator, writes the images, and replaces every chunk's (C, T) by the
// (C, T) accumulated in front of it (what the chunk's backward starts from).
// (several tiles per workgroup for the one-wave tiles, one per wave:
// fewer, larger workgroups)
template <int TW, int TH>
constexpr int merge_tiles_per_block() { return TW * TH >= 256 ? 1 : 256 / (TW * TH); }

template <int TW, int TH>
__global__ __launch_bounds__((TW * TH * merge_tiles_per_block<TW, TH>())) void merge_kernel(RasterArgs a)
{
    constexpr int NT = TW * TH;
    const int tile = blockIdx.x * merge_tiles_per_block<TW, TH>() + (int)threadIdx.x / NT;
    if (tile >= a.n_tiles) return;
    const int tid = threadIdx.x % NT;
    const int v = view_of_tile(a.views, a.V, tile);
    const ViewDev &V = a.views[v];
    const int lt = tile - V.tile_base;
    const int ty = lt / V.ntx, tx = lt - ty * V.ntx;
    const int px = tx * TW + tid % TW, py = ty * TH + tid / TW;
    const uint32_t base = a.item_base[tile], cnt = a.item_cnt[tile];
    const uint32_t last = a.ranges[tile].y;
    // items past the item capacity do not exist (overflowed step)
    const uint32_t mi = (uint32_t)a.max_items;
    const uint32_t kend = base < mi ? min(cnt, mi - base) : 0u;
    float2 *const pp = a.part + (size_t)base * NT + tid;
    float C = 0.0f, T = 1.0f;
    // four items' partials read together (each item's place then receives
    // the (C, T) in front of it)
    uint32_t k = 0;
    for (; k + 4u <= kend; k += 4u) {
        float2 ck[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) ck[u] = pp[(size_t)(k + u) * NT];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            pp[(size_t)(k + u) * NT] = make_float2(C, T);
            C = __fmaf_rn(T, ck[u].x, C);
            T = __fmul_rn(T, ck[u].y);
        }
    }
    for (; k < kend; ++k) {
        const float2 ck = pp[(size_t)k * NT];
        pp[(size_t)k * NT] = make_float2(C, T);
        C = __fmaf_rn(T, ck.x, C);
        T = __fmul_rn(T, ck.y);
    }
    if (px < V.W && py < V.H) {
        const size_t p = (size_t)V.pix_base + (size_t)py * V.W + px;
        a.img[p] = C;
        a.img_saved[p] = C;
        a.nlast[p] = last;
    }
}

// SPLIT: work items are chunks (every entry of an item lies before the
// pixel's last contribution).
template <int TW, int TH, bool SPLIT>
__global__ __launch_bounds__(TW *TH) void raster_bwd_kernel(RasterArgs a)
{
    constexpr int NT = TW * TH;
    constexpr int NW = NT / kWave;
    constexpr int NA = NW > 1 ? NW : 1, NTA = NW > 1 ? NT : 1;
    // one array, s1 first: the paired 4-byte reads of alpha and c then reach
    // it with in-range immediate offsets from the same register as the
    // 16-byte reads of s0
    __shared__ float4 s10[2 * NT];
    float4 *const s1 = s10;
    float4 *const s0 = s10 + NT;
    __shared__ uint32_t se[NT];
    __shared__ __align__(16) float acc[NA][NTA][8];  // several waves: per-wave entry sums
    __shared__ uint32_t wmax[NW];
    __shared__ int sh_item;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
    // entries per transposing sum, gradient terms per entry, entries staged
    // per batch (a whole number of groups), and this lane's (entry, term)
    // after the sum (lane 63 holds the pad)
    constexpr int kTerms = 7, EPG = kWave / kTerms;
    constexpr int BATCH = (NT / EPG) * EPG;
    static_assert(EPG * kTerms < kWave, "one pad value");
    const int l_entry = lane / kTerms, l_term = lane - l_entry * kTerms;
    const float k2s = __fmul_rn(a.o.kappa2, kExpScale), tmin = a.o.t_min;
    const float smax = a.o.sigma_max;
    float *slotf = reinterpret_cast<float *>(a.slot);
    int iter = 0;
    for (;;) {
        const int it = next_item(a, iter, &sh_item);
        const Item I = resolve_item(a, it);
        if (I.tile < 0) break;
        const int v = view_of_tile(a.views, a.V, I.tile);
        const ViewDev &V = a.views[v];
        const int lt = I.tile - V.tile_base;
        const int ty = lt / V.ntx, tx = lt - ty * V.ntx;
        const int px = tx * TW + tid % TW, py = ty * TH + tid / TW;
        const bool inside = px < V.W && py < V.H;
        const float fpx = (float)px + 0.5f, fpy = (float)py + 0.5f;
        const size_t vbase = (size_t)v * a.n;
        float g = 0.0f, Cf = 0.0f, T = 1.0f, Cacc = 0.0f;
        uint32_t lastp = I.b;
        if (inside) {
            const size_t p = (size_t)V.pix_base + (size_t)py * V.W + px;
            g = a.dL_dimg[p];
            Cf = a.img_saved[p];
            lastp = a.split ? I.e : a.nlast[p];
        }
        if (a.split) {
            const float2 pre = a.part[(size_t)it * NT + tid];
            Cacc = pre.x;
            T = pre.y;
        }
        // g times the tail S (the saved pixel value minus the colour
        // composited so far), kept up to date entry by entry
        float Sg = g * (Cf - Cacc);
        // end of the longest contributing prefix in the item
        uint32_t m = lastp;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, o, kWave));
        __syncthreads();
        if (lane == 0) wmax[w] = m;
        __syncthreads();
        uint32_t end = wmax[0];
#pragma unroll
        for (int q = 1; q < NW; ++q) end = max(end, wmax[q]);

        // the cut-off test with the lane's state folded in (kLaneOff once
        // stopped or outside the image): a hit is one compare, its ballot is free
        float k2e = inside ? k2s : kLaneOff;
        // the staged batch's entries in groups of EPG, CLAMP as in the forward
        // (without it every alpha of the batch is at most sigma_max / 2: s =
        // alpha G and no step is clamped)
        auto run_groups = [&](uint32_t b0, int cnt, auto clamp_c) {
            constexpr bool CLAMP = decltype(clamp_c)::value;
            // groups of EPG = 9 entries: their 7 gradient terms fill 63 of
            // the 64 values of one transposing wave sum (the last is a
            // zero pad); lane l ends with term l % 7 of entry l / 7
            for (int q0 = 0; q0 < cnt; q0 += EPG) {
                float gb[64];
                bool any = false;
                // the group's first entry index, held in one vector
                // register (an empty asm makes it opaque) so that the
                // entries' LDS reads use it with immediate offsets instead
                // of rebuilding an address for each entry
                int qv = q0;
                asm volatile("" : "+v"(qv));
#pragma unroll
                for (int qq = 0; qq < EPG; ++qq) {
                    float gv[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                    const int q = q0 + qq;
                    if (q < cnt) {
                        const float4 r0 = s0[qv + qq];
                        const float4 r1 = s1[qv + qq];
                        const float dx = __fsub_rn(fpx, r0.x), dy = __fsub_rn(fpy, r0.y);
                        const float ex = falloff_exponent(dx, dy, r0.z, r0.w, r1.x);
                        bool hit = ex >= k2e;
                        if constexpr (!SPLIT) hit = hit && (b0 + (uint32_t)q) < lastp;
                        // when any lane hits, the whole wave runs the entry:
                        // computed without branches, lanes that miss keep
                        // their state and contribute zeros
                        if (wave_any_mask(hit) != 0ull) {
                            // lanes that miss run the same arithmetic with
                            // G = 0: s = 0, 1 - s = 1, so the running colour
                            // and T stay exactly as they are and every term
                            // below is zero
                            float G = hit ? __builtin_amdgcn_exp2f(ex) : 0.0f;
                            float sraw = __fmul_rn(r1.y, G);
                            float s = sraw, om;
                            if constexpr (CLAMP) {
                                s = clamp_opacity(sraw, smax);
                                om = __fsub_rn(1.0f, s);
                            } else {
                                om = one_minus_alpha_g(r1.y, G);
                            }
                            if constexpr (!SPLIT) {
                                // t_min > 0 runs unsplit
                                if (tmin > 0.0f) {
                                    const bool stop = hit & (__fmul_rn(T, om) < tmin);
                                    k2e = stop ? kLaneOff : k2e;
                                    hit = hit & !stop;
                                    G = stop ? 0.0f : G;
                                    sraw = stop ? 0.0f : sraw;
                                    s = stop ? 0.0f : s;
                                    om = stop ? 1.0f : om;
                                }
                            }
                            // dL/ds = g (c T - S / (1 - s)) with S the tail
                            // after this entry: g S is updated by -g c s T
                            const float c = r1.z;
                            const float sT = __fmul_rn(s, T);
                            const float gc = g * c;
                            Sg = __fmaf_rn(-gc, sT, Sg);
                            const float ds = __fmaf_rn(gc, T, -(Sg * __builtin_amdgcn_rcpf(om)));
                            // moments of dL/ds G about the mean; the conic and
                            // alpha factors are applied once per (view,
                            // Gaussian) in the projection backward
                            float gds = ds * G;
                            if constexpr (CLAMP) gds = (sraw > smax) ? 0.0f : gds;
                            const float m1x = gds * dx, m1y = gds * dy;
                            gv[0] = m1x;
                            gv[1] = m1y;
                            gv[2] = m1x * dx;
                            gv[3] = m1x * dy;
                            gv[4] = m1y * dy;
                            gv[5] = gds;
                            gv[6] = g * sT;
                            T = __fmul_rn(T, om);
                            any = true;
                        }
                    }
#pragma unroll
                    for (int c = 0; c < kTerms; ++c) gb[qq * kTerms + c] = gv[c];
                }
                gb[63] = 0.0f;
                float res = 0.0f;
                if (wave_any_mask(any) != 0ull) {
                    wave_transpose_sum64(gb);
                    res = gb[0];
                }
                const int q = q0 + l_entry;
                if (l_entry < EPG && q < cnt) {
                    if constexpr (NW == 1) {
                        const size_t e = se[q];
                        if (e < a.slot_cap) slotf[8 * e + l_term] = res;
                    } else {
                        acc[w][q][l_term] = res;
                    }
                }
            }
        };
        for (uint32_t b0 = I.b; b0 < I.e; b0 += BATCH) {
            const int cnt = (int)min((uint32_t)BATCH, I.e - b0);
            __syncthreads();
            const uint32_t j = b0 + tid;
            bool over = false;  // an opacity above sigma_max / 2 in this batch
            if (tid < BATCH && j < I.e) {
                const uint32_t gid = min(a.tval[j], (uint32_t)a.n - 1u);
                const size_t idx = vbase + gid;
                // one 64-byte line per pair: record, place in the slot
                // numbering, rectangle and tile mask
                float4 r0 = a.rec[4 * idx], r1 = a.rec[4 * idx + 1];
                const float4 r2 = a.rec[4 * idx + 2];
                const uint32_t place = __float_as_uint(r1.w);
                over = r1.y > 0.5f * smax;
                scale_conic(r0, r1);
                s0[tid] = r0;
                s1[tid] = r1;
                // the slot: the pair's first slot plus this tile's rank among
                // the pair's kept tiles (row-major in its rectangle)
                const uint32_t rx = __float_as_uint(r2.x), ry = __float_as_uint(r2.y);
                const int tx0 = rx & 0xFFFF, ty0 = rx >> 16, tx1 = ry & 0xFFFF, ty1 = ry >> 16;
                const uint32_t area = (uint32_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1));
                const uint32_t at = (uint32_t)((ty - ty0) * (tx1 - tx0 + 1) + (tx - tx0));
                se[tid] = first_slot(a.slot_bofs, a.slot_nblk, v, (int)gid, place) +
                          kept_rank(__float_as_uint(r2.z), area, at);
            }
            const bool clamp = __syncthreads_or(over);
            if (b0 < end && clamp) run_groups(b0, cnt, std::true_type{});
            else if (b0 < end) run_groups(b0, cnt, std::false_type{});
            if constexpr (NW > 1) {
                __syncthreads();
                if (tid < cnt) {
                    float4 r0 = make_float4(0.f, 0.f, 0.f, 0.f), r1 = r0;
                    if (b0 < end) {
#pragma unroll
                        for (int q = 0; q < NW; ++q) {
                            const float4 x0 = *reinterpret_cast<const float4 *>(&acc[q][tid][0]);
                            const float4 x1 = *reinterpret_cast<const float4 *>(&acc[q][tid][4]);
                            r0.x += x0.x; r0.y += x0.y; r0.z += x0.z; r0.w += x0.w;
                            r1.x += x1.x; r1.y += x1.y; r1.z += x1.z;
                        }
                    }
                    const size_t e = se[tid];
                    if (e < a.slot_cap) {
                        a.slot[2 * e] = r0;
                        a.slot[2 * e + 1] = r1;
                    }
                }
            } else {
                if (b0 >= end && tid < cnt) {
                    const size_t e = se[tid];
                    if (e < a.slot_cap) {
                        a.slot[2 * e] = make_float4(0.f, 0.f, 0.f, 0.f);
                        a.slot[2 * e + 1] = make_float4(0.f, 0.f, 0.f, 0.f);
                    }
                }
            }
        }
    }
}

typedef float floatx4 __attribute__((ext_vector_type(4)));

// Backward of 8 x 8 tiles in chunks (the tuned shape).  The seven per-entry
// sums are formed in two parts instead of by a seven-term butterfly per
// entry.  The per-pair factor q = dL/ds G (zero where a pixel misses the
// entry) goes to LDS for sixteen entries at a time, and its moments about the
// mean come from one dense contraction over the 64 pixels on the matrix
// cores: raw moments M_n = sum_p q(p) P_n(p) of the pixel monomials
// P = (1, x, y, x^2, x y, y^2) about the tile centre, sixteen steps of
// v_mfma_f32_16x16x4_f32 with the entries as rows and the monomials as
// columns, then shifted to each entry's mean.  The colour term g s T is
// summed by a transposing butterfly over the wave.  The vector ALU keeps the
// per-pair compositing arithmetic; the matrix cores, which run beside it,
// take the reductions.
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(5))) void raster_bwd_mm_kernel(RasterArgs a)
{
    // entries per contraction, and entries whose records are read together
    // (two: 0.2235 ms against 0.2242 for one and 0.2242 for four, at 500k /
    // 512^2; reading the next batch's records during the current one was
    // slower, 0.2443 ms, through the registers it holds)
    constexpr int TW = 8, TH = 8, NT = TW * TH, GRP = 16, PF = 2;
    static_assert(NT == kWave, "one wave per tile");
    // s1 first, as in the general kernel (paired reads of alpha and c)
    __shared__ float4 s10[2 * NT];
    float4 *const s1 = s10;
    float4 *const s0 = s10 + NT;
    __shared__ uint32_t se[NT];
    // q by (entry, pixel), the rows padded so that the operand reads of one
    // step fall in distinct banks
    __shared__ float aq[GRP][NT + 1];
    __shared__ float dm[GRP][8];  // raw moments by (entry, monomial)
    __shared__ float tsm[GRP];    // the colour term by entry
    __shared__ int sh_item;
    const int tid = threadIdx.x;
    const float k2s = __fmul_rn(a.o.kappa2, kExpScale);
    const float smax = a.o.sigma_max;
    // matrix operands: lane l supplies A[l % 16][l / 16] = q of entry l % 16 at
    // pixel p = st + 16 (l / 16) in step st, and B[l / 16][l % 16] = monomial
    // l % 16 of that pixel (zero past the sixth); D[r][j] comes back in lane
    // j + 16 (r / 4), item r % 4
    float bm[GRP];
    {
        const int nn = tid & 15, kq = tid >> 4;
#pragma unroll
        for (int st = 0; st < GRP; ++st) {
            const int p = st + 16 * kq;
            const float x = (float)(p & 7) - 3.5f, y = (float)(p >> 3) - 3.5f;
            float b = 0.0f;
            b = nn == 0 ? 1.0f : b;
            b = nn == 1 ? x : b;
            b = nn == 2 ? y : b;
            b = nn == 3 ? x * x : b;
            b = nn == 4 ? x * y : b;
            b = nn == 5 ? y * y : b;
            bm[st] = b;
        }
    }
    int iter = 0;
    for (;;) {
        const int it = next_item(a, iter, &sh_item);
        const Item I = resolve_item(a, it);
        if (I.tile < 0) break;
        const int v = view_of_tile(a.views, a.V, I.tile);
        const ViewDev &V = a.views[v];
        const int lt = I.tile - V.tile_base;
        const int ty = lt / V.ntx, tx = lt - ty * V.ntx;
        const int px = tx * TW + tid % TW, py = ty * TH + tid / TW;
        const bool inside = px < V.W && py < V.H;
        const float fpx = (float)px + 0.5f, fpy = (float)py + 0.5f;
        // the monomials' origin
        const float cx = (float)(tx * TW) + 0.5f * TW, cy = (float)(ty * TH) + 0.5f * TH;
        const size_t vbase = (size_t)v * a.n;
        float g = 0.0f, Cf = 0.0f;
        if (inside) {
            const size_t p = (size_t)V.pix_base + (size_t)py * V.W + px;
            g = a.dL_dimg[p];
            Cf = a.img_saved[p];
        }
        // (C, T) in front of the chunk, and g times the tail S
        const float2 pre = a.part[(size_t)it * NT + tid];
        float T = pre.y;
        float Sg = g * (Cf - pre.x);
        float k2e = inside ? k2s : kLaneOff;
        // slots of group qp (its raw moments in acc, its colour terms in tsm):
        // the moments go through LDS by (entry, monomial), then lane e < 16
        // shifts entry qp + e's moments to the mean and stores its slot
        auto finalize = [&](int qp, int cnt, const floatx4 &acc) {
            if ((tid & 15) < 6) {
#pragma unroll
                for (int i = 0; i < 4; ++i) dm[4 * (tid >> 4) + i][tid & 15] = acc[i];
            }
            __syncthreads();
            if (tid < GRP && qp + tid < cnt) {
                // moments about the mean: with x = u + (x - u), u the mean's
                // offset from the tile centre
                const float M0 = dm[tid][0], M1 = dm[tid][1], M2 = dm[tid][2];
                const float M3 = dm[tid][3], M4 = dm[tid][4], M5 = dm[tid][5];
                const float4 r0 = s0[qp + tid];
                const float ux = r0.x - cx, uy = r0.y - cy;
                const float m1x = M1 - ux * M0, m1y = M2 - uy * M0;
                const float mxx = M3 - ux * (2.0f * M1 - ux * M0);
                const float mxy = M4 - ux * M2 - uy * M1 + ux * uy * M0;
                const float myy = M5 - uy * (2.0f * M2 - uy * M0);
                const size_t e = se[qp + tid];
                if (e < a.slot_cap) {
                    a.slot[2 * e] = make_float4(m1x, m1y, mxx, mxy);
                    a.slot[2 * e + 1] = make_float4(myy, M0, tsm[tid], 0.0f);
                }
            }
            __syncthreads();
        };
        // The batch's groups of 16 entries.  Software-pipelined: group k's
        // contraction is issued after its entries, and its slots are
        // finalised after group k + 1's entries, so the matrix cores' latency
        // is covered by the next group's arithmetic.
        auto run_groups = [&](int cnt, auto clamp_c) {
            constexpr bool CLAMP = decltype(clamp_c)::value;
            floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
            for (int q0 = 0; q0 < cnt; q0 += GRP) {
                float tv[GRP];
                // the group's first entry in one vector register (opaque to
                // the compiler), so that the record reads take immediate offsets
                int qv = q0;
                asm volatile("" : "+v"(qv));
                // PF entries' records read together, then run in order
#pragma unroll
                for (int e4 = 0; e4 < GRP; e4 += PF) {
                    float4 R0[PF], R1[PF];
#pragma unroll
                    for (int u = 0; u < PF; ++u) {
                        R0[u] = s0[qv + e4 + u];
                        R1[u] = s1[qv + e4 + u];
                    }
#pragma unroll
                    for (int u = 0; u < PF; ++u) {
                        const int e = e4 + u;
                        const float4 r0 = R0[u], r1 = R1[u];
                        // branch-free: lanes that miss (and the padding record)
                        // run the same arithmetic with G = 0, which leaves T and
                        // the tail as they are and makes q and g s T zero, so
                        // the compiler may interleave the entries of the group
                        const float dx = __fsub_rn(fpx, r0.x), dy = __fsub_rn(fpy, r0.y);
                        const float ex = falloff_exponent(dx, dy, r0.z, r0.w, r1.x);
                        const bool hit = ex >= k2e;
                        const float G = hit ? __builtin_amdgcn_exp2f(ex) : 0.0f;
                        const float sraw = __fmul_rn(r1.y, G);
                        float s = sraw, om;
                        if constexpr (CLAMP) {
                            s = clamp_opacity(sraw, smax);
                            om = __fsub_rn(1.0f, s);
                        } else {
                            om = one_minus_alpha_g(r1.y, G);
                        }
                        // dL/ds = g (c T - S / (1 - s)), S the tail after this entry
                        const float gc = g * r1.z;
                        const float sT = __fmul_rn(s, T);
                        Sg = __fmaf_rn(-gc, sT, Sg);
                        const float ds = __fmaf_rn(gc, T, -(Sg * __builtin_amdgcn_rcpf(om)));
                        float qq = ds * G;
                        if constexpr (CLAMP) qq = (sraw > smax) ? 0.0f : qq;
                        T = __fmul_rn(T, om);
                        aq[e][tid] = qq;
                        tv[e] = g * sT;
                    }
                }
                const float tsum = wave_transpose_sum16(tv);
                if (q0 > 0) finalize(q0 - GRP, cnt, acc);
                if ((tid & 3) == 0) tsm[tid >> 2] = tsum;
                __syncthreads();
                acc = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int st = 0; st < GRP; ++st)
                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(aq[tid & 15][st + 16 * (tid >> 4)], bm[st], acc, 0, 0, 0);
            }
            finalize((cnt - 1) / GRP * GRP, cnt, acc);
        };
        for (uint32_t b0 = I.b; b0 < I.e; b0 += NT) {
            const int cnt = (int)min((uint32_t)NT, I.e - b0);
            __syncthreads();
            const uint32_t j = b0 + tid;
            bool over = false;  // an opacity above sigma_max / 2 in this batch
            if (j < I.e) {
                const uint32_t gid = min(a.tval[j], (uint32_t)a.n - 1u);
                const size_t idx = vbase + gid;
                float4 r0 = a.rec[4 * idx], r1 = a.rec[4 * idx + 1];
                const float4 r2 = a.rec[4 * idx + 2];
                const uint32_t place = __float_as_uint(r1.w);
                over = r1.y > 0.5f * smax;
                scale_conic(r0, r1);
                s0[tid] = r0;
                s1[tid] = r1;
                // the slot: the pair's first slot plus this tile's rank among
                // the pair's kept tiles (row-major in its rectangle)
                const uint32_t rx = __float_as_uint(r2.x), ry = __float_as_uint(r2.y);
                const int tx0 = rx & 0xFFFF, ty0 = rx >> 16, tx1 = ry & 0xFFFF, ty1 = ry >> 16;
                const uint32_t area = (uint32_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1));
                const uint32_t at = (uint32_t)((ty - ty0) * (tx1 - tx0 + 1) + (tx - tx0));
                se[tid] = first_slot(a.slot_bofs, a.slot_nblk, v, (int)gid, place) +
                          kept_rank(__float_as_uint(r2.z), area, at);
            } else {
                // places past the batch's entries hold a record that no pixel
                // reaches (d^T A d = -(dx^2 + dy^2) ~ -2e36, alpha = c = 0):
                // every group runs all its entries without a bound check, and
                // these contribute exact zeros
                s0[tid] = make_float4(1e18f, 1e18f, -1.0f, 0.0f);
                s1[tid] = make_float4(-1.0f, 0.0f, 0.0f, 0.0f);
            }
            const bool clamp = __syncthreads_or(over);
            if (clamp) run_groups(cnt, std::true_type{});
            else run_groups(cnt, std::false_type{});
        }
    }
}

__global__ __launch_bounds__(256) void tile_cost_kernel(const uint2 *ranges, int n_tiles, uint32_t *keys,
                                                        uint32_t *vals, uint32_t *counter)
{
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t == 0) *counter = 0;
    if (t >= n_tiles) return;
    const uint2 r = ranges[t];
    const uint32_t len = min(r.y - r.x, 0xFFFFFFu);
    keys[t] = 0xFFFFFFu - len;  // ascending sort -> longest first
    vals[t] = (uint32_t)t;
}

// grids of blocks mapped by xcd_item
inline int round_up8(int n) { return (n + 7) / 8 * 8; }

template <int TW, int TH>
hipError_t fwd_inst(const RasterArgs &a, int pb, hipStream_t s)
{
    const int grid = a.queue_counter ? pb : round_up8(a.split ? a.max_items : a.n_tiles);
    if (grid > 0) {
        const bool cnt = a.pair_counts != nullptr;
        if (a.split && cnt) raster_fwd_kernel<TW, TH, true, true><<<grid, TW * TH, 0, s>>>(a);
        else if (a.split && TW == 8 && TH == 8) raster_fwd_quad_kernel<<<grid, TW * TH, 0, s>>>(a);
        else if (a.split) raster_fwd_kernel<TW, TH, true, false><<<grid, TW * TH, 0, s>>>(a);
        else if (cnt) raster_fwd_kernel<TW, TH, false, true><<<grid, TW * TH, 0, s>>>(a);
        else raster_fwd_kernel<TW, TH, false, false><<<grid, TW * TH, 0, s>>>(a);
    }
    if (a.split && a.n_tiles > 0) {
        constexpr int MTB = merge_tiles_per_block<TW, TH>();
        merge_kernel<TW, TH><<<(a.n_tiles + MTB - 1) / MTB, TW * TH * MTB, 0, s>>>(a);
    }
    return hipGetLastError();
}

template <int TW, int TH>
hipError_t bwd_inst(const RasterArgs &a, int pb, hipStream_t s)
{
    const int grid = a.queue_counter ? pb : round_up8(a.split ? a.max_items : a.n_tiles);
    if (grid > 0) {
        if (a.split && TW == 8 && TH == 8)
            raster_bwd_mm_kernel<<<grid, TW * TH, 0, s>>>(a);
        else if (a.split)
            raster_bwd_kernel<TW, TH, true><<<grid, TW * TH, 0, s>>>(a);
        else
            raster_bwd_kernel<TW, TH, false><<<grid, TW * TH, 0, s>>>(a);
    }
    return hipGetLastError();
}

}  // namespace

bool raster_tile_supported(int tw, int th)
{
    return (tw == 16 && th == 16) || (tw == 8 && th == 8) || (tw == 16 && th == 8) || (tw == 32 && th == 8);
}

hipError_t launch_raster_fwd(const RasterArgs &a, int pb, hipStream_t s)
{
    const int tw = a.o.tile_w, th = a.o.tile_h;
    if (tw == 16 && th == 16) return fwd_inst<16, 16>(a, pb, s);
    if (tw == 8 && th == 8) return fwd_inst<8, 8>(a, pb, s);
    if (tw == 16 && th == 8) return fwd_inst<16, 8>(a, pb, s);
    if (tw == 32 && th == 8) return fwd_inst<32, 8>(a, pb, s);
    return hipErrorInvalidValue;
}

hipError_t launch_raster_bwd(const RasterArgs &a, int pb, hipStream_t s)
{
    const int tw = a.o.tile_w, th = a.o.tile_h;
    if (tw == 16 && th == 16) return bwd_inst<16, 16>(a, pb, s);
    if (tw == 8 && th == 8) return bwd_inst<8, 8>(a, pb, s);
    if (tw == 16 && th == 8) return bwd_inst<16, 8>(a, pb, s);
    if (tw == 32 && th == 8) return bwd_inst<32, 8>(a, pb, s);
    return hipErrorInvalidValue;
}

hipError_t launch_tile_cost_keys(const uint2 *ranges, int n_tiles, uint32_t *keys, uint32_t *vals,
                                 uint32_t *counter, hipStream_t s)
{
    tile_cost_kernel<<<(n_tiles + 255) / 256 + (n_tiles == 0), 256, 0, s>>>(ranges, n_tiles, keys, vals, counter);
    return hipGetLastError();
}

}  // namespace ddgs
