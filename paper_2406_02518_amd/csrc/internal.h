// internal.h -- device-side structures and launch wrappers of libddgs.so
// (gfx950, wave64).  Not part of the public ABI (include/ddgs.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ddgs {

constexpr int kWave = 64;
constexpr int kMaxK = 32;   // feature size supported (Eq. 3: f in R^k)
constexpr int kMaxKL = 15;  // L(L+2) at L = 3

// One view as the kernels see it (host prepares it from ddgs_view).
struct ViewDev {
    float R[9];      // world -> source rotation, row-major
    float t[3];
    float so[3];     // source position in the world frame, -R^T t
    float f;         // focal length in pixels, sdd / pitch
    float cx, cy;    // principal point, (W/2, H/2)
    int32_t W, H;
    int32_t ntx, nty;      // tiles per row / column
    int32_t tile_base;     // first global tile id of this view
    int32_t pad;
    int64_t pix_base;      // first pixel of this view in the concatenated image
};

// Rotation matrix of the unit quaternion (w, x, y, z), row-major.
__device__ __forceinline__ void quat_rot(float w, float x, float y, float z, float *R)
{
    R[0] = 1.0f - 2.0f * (y * y + z * z); R[1] = 2.0f * (x * y - w * z); R[2] = 2.0f * (x * z + w * y);
    R[3] = 2.0f * (x * y + w * z); R[4] = 1.0f - 2.0f * (x * x + z * z); R[5] = 2.0f * (y * z - w * x);
    R[6] = 2.0f * (x * z - w * y); R[7] = 2.0f * (y * z + w * x); R[8] = 1.0f - 2.0f * (x * x + y * y);
}

struct RenderOpts {
    float kappa, kappa2, dilation, t_min, z_near, sigma_max;
    int32_t tile_w, tile_h;
};

// Device pointers of the model (SoA, caller-owned).
struct ModelDev {
    int32_t n, n_iso, k, L;
    int32_t entangled;  // 1: both radiosity terms under one sigmoid on every Gaussian (n_iso = 0)
    const float *mean, *quat, *log_scale, *opacity_logit, *feat, *b_iso, *B_dir;
    const float *c_override;  // [V][n] radiosity used instead of Eq. 3 (NULL: Eq. 3)
};

// View-independent per-Gaussian values, computed once per step.
struct GaussCache {
    float *cov;    // [6][n]: world covariance xx, xy, xz, yy, yz, zz
    float *alpha;  // [n]
    float *ciso;   // [n]: isotropic radiosity (only [0, n_iso) meaningful); entangled
                   // models hold the isotropic logit b_iso . f of every Gaussian
    float *hdir;   // [k_L][n - n_iso]: B_dir f for directional Gaussians
};

// Gaussians per block of the projection (and of the slot numbering).
constexpr int kSlotBlock = 256;
inline int64_t slot_blocks(int64_t n) { return (n + kSlotBlock - 1) / kSlotBlock; }

// Tile selection of a pair: its rectangle [tx0, tx1] x [ty0, ty1] and, when
// the rectangle has at most kMaskTiles tiles, a mask of the tiles the cut-off
// ellipse reaches (bit b = row-major place b in the rectangle); larger
// rectangles keep every tile (mask kAllTiles).
constexpr uint32_t kMaskTiles = 32;
constexpr uint32_t kAllTiles = 0xFFFFFFFFu;
__device__ __forceinline__ bool tile_kept(uint32_t mask, uint32_t area, uint32_t place)
{
    return area > kMaskTiles || ((mask >> place) & 1u);
}
// place of a kept tile among the pair's kept tiles (its gradient slot)
__device__ __forceinline__ uint32_t kept_rank(uint32_t mask, uint32_t area, uint32_t place)
{
    return area > kMaskTiles ? place : (uint32_t)__popc(mask & ((1u << place) - 1u));
}

// Per (view, Gaussian) projection output.
struct ProjOut {
    float4 *rec;     // [V*n][4], 64 B (one cache line) per pair: (mx, my, A00, A01),
                     // (A11, alpha, c, bits of the pair's place in its block's
                     // slot numbering), (bits of rect.x, rect.y, tile mask, 0), unused
    uint2 *rect;     // [V*n]: (tx0 | ty0 << 16, tx1 | ty1 << 16), inclusive
    uint32_t *tmask; // [V*n]: kept tiles of the rectangle (tile_kept)
    uint32_t *zkey;  // [V*n]: float bits of the source-frame depth, ~0u if culled
    uint32_t *cnt;   // [V*n]: number of tiles kept
    // gradient-slot numbering in (view, Gaussian) order: each block of
    // kSlotBlock Gaussians of a view stores its exclusive scan of the tile
    // counts (slot_lp, [V*n]) and its total (slot_btot, [V * slot_blocks(n)]),
    // which the emission turns into the blocks' first slots
    uint32_t *slot_lp, *slot_btot;
};

// First gradient slot of pair (v, i): its block's first slot (bofs, from
// the emission) plus its place in the block (lp, the projection's
// block scan).  The slots of one Gaussian are consecutive, row-major over
// its tile rectangle, and the pairs' slot ranges follow (view, Gaussian)
// order, so the projection backward reads them with neighbouring lanes on
// neighbouring ranges.
__device__ __forceinline__ uint32_t first_slot(const uint32_t *bofs, int nblk, int v, int i, uint32_t lp)
{
    return bofs[(size_t)v * nblk + i / kSlotBlock] + lp;
}

// Per-(view, Gaussian) image-plane gradient terms accumulated by the raster
// backward, one 8-float slot per tile entry (numbered by first_slot): with
// q = dL/ds G at each hit pixel (0 where sigma_max clamps) and (dx, dy) =
// pixel - mean, the sums over the tile's pixels of q dx, q dy, q dx^2,
// q dx dy, q dy^2, q, and dL/dc, then 0.
struct GradSlots { float4 *slot; };

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ float wave_sum(float x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
    return x;
}

// DPP move with identity fill (rows outside ROW_MASK read 0)
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ float dpp_move(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xF, false));
}

// Sum over the 64 lanes of a wave using only VALU data-parallel moves; the
// total lands in lane 63.  Butterflies inside quads and rows of 16
// (quad_perm, row_half_mirror, row_mirror), then row_bcast:15 and
// row_bcast:31 fold the four rows into the last one.
__device__ __forceinline__ float wave_sum_to_lane63(float x)
{
    x += dpp_move<0xB1>(x);        // quad_perm [1,0,3,2]
    x += dpp_move<0x4E>(x);        // quad_perm [2,3,0,1]
    x += dpp_move<0x141>(x);       // row_half_mirror
    x += dpp_move<0x140>(x);       // row_mirror
    x += dpp_move<0x142, 0xA>(x);  // row_bcast:15 into rows 1 and 3
    x += dpp_move<0x143, 0xC>(x);  // row_bcast:31 into rows 2 and 3
    return x;
}

// One in-row step of the transposing sum for lane bit 3 (row_mirror pairs
// lane l of a row with 15 - l) or bit 2 (row_half_mirror: l with 7 - l):
// lanes whose bit is 0 get x + x[partner], the others y + y[partner].  Two
// DPP additions with complementary bank masks write the same register (a
// lane outside the bank mask is not written), instead of two selects and an
// addition.  The leading s_nop 1 gives the two wait states a DPP read needs
// after a VALU write of its source; r is early-clobber so that it never
// shares a register with y, which the second addition still reads.
__device__ __forceinline__ float pair_sum_bit3(float x, float y)
{
    float r;
    asm volatile("s_nop 1\n\t"
                 "v_add_f32_dpp %0, %1, %1 row_mirror row_mask:0xf bank_mask:0x3\n\t"
                 "v_add_f32_dpp %0, %2, %2 row_mirror row_mask:0xf bank_mask:0xc"
                 : "=&v"(r)
                 : "v"(x), "v"(y));
    return r;
}
__device__ __forceinline__ float pair_sum_bit2(float x, float y)
{
    float r;
    asm volatile("s_nop 1\n\t"
                 "v_add_f32_dpp %0, %1, %1 row_half_mirror row_mask:0xf bank_mask:0x5\n\t"
                 "v_add_f32_dpp %0, %2, %2 row_half_mirror row_mask:0xf bank_mask:0xa"
                 : "=&v"(r)
                 : "v"(x), "v"(y));
    return r;
}

// Sums 64 per-lane values over the wave at once: afterwards v[0] of lane l
// holds the wave total of v[l].  Transposing butterfly: every step pairs
// values i and i + h, each half of the lane pairs keeps one of them and adds
// the partner's copy, so the per-lane work halves every step (63 additions
// in all, instead of 6 per value).  The cross-row steps swap register
// halves with v_permlane32_swap / v_permlane16_swap; the in-row steps pair
// lane bits 3, 2, 1, 0 through row_mirror, row_half_mirror and the two quad
// permutations, each of which maps a lane to one whose bit differs.
__device__ __forceinline__ void wave_transpose_sum64(float (&v)[64])
{
    const uint32_t lane = __lane_id();
#pragma unroll
    for (int i = 0; i < 32; ++i) {
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[i]), __float_as_uint(v[i + 32]),
                                                        false, false);
        v[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v[i]), __float_as_uint(v[i + 16]),
                                                        false, false);
        v[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
    const bool b1 = lane & 2, b0 = lane & 1;
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = pair_sum_bit3(v[i], v[i + 8]);
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = pair_sum_bit2(v[i], v[i + 4]);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const float keep = b1 ? v[i + 2] : v[i], send = b1 ? v[i] : v[i + 2];
        v[i] = keep + dpp_move<0x4E>(send);   // quad_perm [2,3,0,1]: l <-> l ^ 2
    }
    {
        const float keep = b0 ? v[1] : v[0], send = b0 ? v[0] : v[1];
        v[0] = keep + dpp_move<0xB1>(send);   // quad_perm [1,0,3,2]: l <-> l ^ 1
    }
}

// Sums 16 per-lane values over the wave at once: afterwards every lane l
// holds the wave total of v[(l >> 2) & 15].  The transposing butterfly of
// wave_transpose_sum64 over lane bits 5, 4, 3 and 2 (value index bits 3..0),
// then plain butterflies over bits 1 and 0, which leave the four lanes of a
// quad with the same total.
__device__ __forceinline__ float wave_transpose_sum16(float (&v)[16])
{
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[i]), __float_as_uint(v[i + 8]),
                                                        false, false);
        v[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v[i]), __float_as_uint(v[i + 4]),
                                                        false, false);
        v[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) v[i] = pair_sum_bit3(v[i], v[i + 2]);
    float x = pair_sum_bit2(v[0], v[1]);
    x += dpp_move<0xB1>(x);   // quad_perm [1,0,3,2]
    x += dpp_move<0x4E>(x);   // quad_perm [2,3,0,1]
    return x;
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x)
{
    const int lane = (int)__lane_id();
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        uint32_t y = __shfl_up(x, o, kWave);
        if (lane >= o) x += y;
    }
    return x;
}

// ---------------------------------------------------------------- launches
// (each returns hipGetLastError() of its launches)

// project.hip
// The view-independent cache (gc) and the projection into V views (po); one
// launch when V == 1, else the cache then one block row per view.
hipError_t launch_prep_project(const ModelDev &m, const GaussCache &gc, const ViewDev *views, int V,
                               const RenderOpts &o, const ProjOut &po, hipStream_t s);

// Backward of the projection: sums each (view, Gaussian)'s gradient slots,
// applies the chain rule to the parameters, and writes, per block of
// kSlotBlock Gaussians, pose partials [V][9][blocks] and its share of the
// basis gradients: the 16 x NCOL tile U F^T over the block's Gaussians, with
// row r < k_L of U the direction terms of a directional Gaussian and row 15
// the isotropic logit's gradient (NCOL = 16 or 32 columns of features).
struct ProjBwdArgs {
    ModelDev m;
    GaussCache gc;
    const ViewDev *views;
    int V;
    RenderOpts o;
    const uint32_t *cnt;
    const uint32_t *slot_lp, *slot_bofs;  // slot numbering (first_slot)
    int slot_nblk;
    const float4 *slot;
    float *dmean, *dquat, *dlog_scale, *dopacity, *dfeat;  // NULL: skip
    float *bpart;       // [blocks][16][NCOL] basis tiles (NULL: skip)
    float *pose_part;   // [V][9][blocks]
    int per_gaussian;   // 0: pose only
    uint32_t slot_cap;  // number of gradient slots (entries beyond are ignored)
    // densification statistics, [n] each (NULL: off): norm of the 2D-mean
    // gradient in normalised device units, visible views, largest radius (px)
    float *st_grad, *st_cnt, *st_rad;
    // step flags of a captured step (NULL: plain call): while bit 0 (a tile
    // list overflowed its capacity) is set the statistics are not updated
    const uint32_t *skip;
    // the radiosity logits' gradients handed to the feature-gradient launch
    // (NULL: neither feature nor basis gradients are wanted): zbuf [n], the
    // isotropic term's z = dL/dc c (1 - c) (every Gaussian of an entangled
    // model; 0 for the directional ones of a disentangled one), ubuf
    // [k_L][n - n_iso], the directional coefficients' u = z Y(d)
    float *zbuf, *ubuf;
};
// The projection backward, then (zbuf set and dfeat or bpart wanted) the
// feature gradients and the basis tiles from zbuf and ubuf.
hipError_t launch_project_bwd(const ProjBwdArgs &a, hipStream_t s);
// floats of the basis tiles of the projection backward (one per block)
size_t basis_part_floats(int n);
// FP64 sums of the basis tiles (when db or dB) and of the pose partials (when
// dpose), in one launch
hipError_t launch_grad_final(const ModelDev &m, const float *bpart, float *db, float *dB, const ViewDev *views,
                             int V, int n_parts, const float *ppart, float *dpose, hipStream_t s);

// sort.hip
constexpr int kScanTile = 4096;

// Temporaries of the scans and radix sorts (device memory).
constexpr int kSortTotWords = 512;  // digit totals of the widest radix pass (9-bit digits)
struct SortWs {
    uint32_t *counts;      // [counts_words]: per-block digit counts, then offsets
    uint32_t *tot;         // [kSortTotWords]: digit totals of the current pass
    uint64_t *blocksum;    // [blocksum_words]: scan block sums
    size_t counts_words, blocksum_words;
};
// words of SortWs::counts / ::blocksum for sorts and scans of up to n elements
size_t sort_counts_words(int64_t n);
size_t sort_blocksum_words(int64_t n);
// out[i] = sum_{j<i} in[g(j)] with g = gather ? gather[j] : j; *total (device u64) = sum.
hipError_t launch_exclusive_scan(const uint32_t *in, const uint32_t *gather, uint32_t *out, int64_t n,
                                 const SortWs &ws, uint64_t *total, hipStream_t s);
// Sorts (keys, vals) by key bits [0, bits) (stable).  n_dev (may be NULL)
// limits the count at run time to min(*n_dev, n_cap).  Ping-pongs between
// (k0, v0) and (k1, v1); *in_k1 tells where the result ended.
// gsrc / gdst (optional): the last pass also writes gdst[i] = gsrc[value i].
hipError_t radix_sort_pairs(uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1, int64_t n_cap,
                            const uint32_t *n_dev, int bits, const SortWs &ws, bool *in_k1, hipStream_t s,
                            const uint32_t *gsrc = nullptr, uint32_t *gdst = nullptr);
// (also clears the n_tiles tile ranges and turns the slot_nb block totals of
// the slot numbering into the blocks' first slots, in place; cnt_sorted: tile
// counts in depth order)
// zero: clear the ranges first (else they must already be clear)
hipError_t launch_ranges(const uint32_t *keys, const uint32_t *m_dev, int64_t m_cap, uint2 *ranges,
                         int n_tiles, bool zero, hipStream_t s);

// bin.hip -- tile binning and the per-tile sort of the tile lists.
// Exclusive scan of the per-tile entry counts: ranges[t] = [start, end)
// clamped to capacity ([0, 0) if empty), cursor[t] = start clamped to
// capacity; *total (u64) = all entries,
// *m_out = min(total, capacity), flags bit 0 set when total > capacity
// (captured steps also pass skipped / need: the count of replays whose
// optimiser updates are skipped -- every replay from the first overflow on,
// until the flags are cleared -- and the largest entry total; NULL: plain
// call).  Also turns the slot numbering's block totals (slot_btot, slot_nb
// of them) into the blocks' first slots.  One launch up to kTileScanSelfMax
// tiles, else three (bsum: [tiles / 256] u64 scratch).
// With `items` (only where tile_scan_makes_items: the one-launch scan), the
// same launch also writes the work items of `split` entries per tile (what
// launch_items writes).
constexpr int kTileScanSelfMax = 16384;
struct TileItems {
    int split;
    uint32_t *cnt, *base;
    uint2 *items;
    uint32_t max_items;
    uint32_t *n_items, *counter;
};
// The tiles too long for the per-tile sort's first launch, listed by the
// tile scan for its second: list [n_tiles], n (one word: the list's length),
// bsum [bsum_words >= ceil(n_tiles / 256)] per-block counts of the
// three-launch scan.
struct LongTiles {
    uint32_t *list, *n, *bsum;
    size_t bsum_words;
};
bool tile_scan_makes_items(int n_tiles);
hipError_t launch_tile_scan(const uint32_t *tile_cnt, int n_tiles, uint2 *ranges, uint32_t *cursor,
                            uint32_t capacity, uint64_t *total, uint32_t *m_out, uint32_t *flags,
                            uint32_t *skipped, unsigned long long *need, uint32_t *slot_btot, int64_t slot_nb,
                            uint64_t *bsum, size_t bsum_words, const TileItems *items, const LongTiles &lt,
                            hipStream_t s);
// Per-tile entry counts without global atomics: groups of Gaussians of each
// view count their entries per tile in LDS into a count matrix mat
// ([bin_matrix_words] u32), whose columns are then scanned into every
// group's offset inside its tile; tile_cnt[t] receives the tile's total.
// max_view_tiles: the largest tile count of one view.
size_t bin_matrix_words(int64_t n, int64_t n_tiles);
hipError_t launch_bin_count(int n, int V, const uint32_t *cnt, const uint2 *rect, const uint32_t *tmask,
                            const ViewDev *views, int n_tiles, int max_view_tiles, uint32_t *mat, uint32_t *tile_cnt,
                            hipStream_t s);
// Every (pair, tile) entry goes to start[tile] + its group's offset + a place
// claimed inside the group, as (depth key, Gaussian index); places at or
// beyond capacity are dropped.
hipError_t launch_bin_scatter(int n, int V, const uint32_t *cnt, const uint2 *rect, const uint32_t *tmask,
                              const uint32_t *zkey, const ViewDev *views, int n_tiles, int max_view_tiles,
                              const uint32_t *mat, const uint32_t *start, uint32_t capacity, uint2 *out,
                              hipStream_t s);
// Sorts every tile's range of ent by (depth key, index) and writes the
// indices to tval; tmp (same layout as ent) is scratch for ranges longer than
// the LDS holds.  tile_cnt and lt are those the tile scan of the same step
// used (the long tiles go to a second launch of at most long_grid
// workgroups, each taking the listed tiles round-robin; with long_grid 0
// there is no second launch and the first one sorts the long tiles too,
// through global memory: meant for steps that rarely or never have any).
hipError_t launch_tile_sort(const uint2 *ranges, const uint32_t *tile_cnt, int n_tiles, const uint2 *ent, uint2 *tmp,
                            uint32_t *tval, const LongTiles &lt, int long_grid, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);
hipError_t launch_zero_u64(uint64_t *p, hipStream_t s);
hipError_t launch_copy_u32(uint32_t *dst, const uint32_t *src, const uint32_t *n_dev, int64_t n_cap,
                           hipStream_t s);

// raster.hip
struct RasterArgs {
    const ViewDev *views;
    int V, n;
    RenderOpts o;
    const uint2 *ranges;
    const uint32_t *tval;
    const float4 *rec;
    int n_tiles;
    const uint32_t *queue;     // persistent mode, split 0: tile order (NULL: natural order)
    uint32_t *queue_counter;   // persistent mode work counter (NULL: one item per block)
    // work items: split = entries per item (0: one item per tile)
    int split;
    const uint2 *items;        // [max_items] (tile, chunk)
    const uint32_t *n_items;   // device count of items
    int max_items;
    const uint32_t *item_base, *item_cnt;  // [n_tiles] first item and item count per tile
    float2 *part;              // [max_items][tile pixels] chunk (C, T), then (C, T) in front of it
    // forward
    float *img, *img_saved;
    uint32_t *nlast;
    unsigned long long *pair_counts;  // [64][2]: evaluated, contributing per slot (NULL: off)
    // backward
    const float *dL_dimg;
    const uint2 *rect;
    const uint32_t *slot_bofs;  // slot numbering (first_slot; the place in the block is in the record)
    int slot_nblk;
    float4 *slot;
    uint32_t slot_cap;
};
hipError_t launch_raster_fwd(const RasterArgs &a, int persistent_blocks, hipStream_t s);
hipError_t launch_raster_bwd(const RasterArgs &a, int persistent_blocks, hipStream_t s);
// persistent queue: order tiles by descending list length
hipError_t launch_tile_cost_keys(const uint2 *ranges, int n_tiles, uint32_t *keys, uint32_t *vals,
                                 uint32_t *counter, hipStream_t s);
// work items of `split` entries (sort.hip): per-tile counts and bases, the
// item list, the device item count; also clears the two work-queue counters
hipError_t launch_items(const uint2 *ranges, int n_tiles, int split, uint32_t *cnt, uint32_t *base, uint2 *items,
                        uint32_t max_items, const SortWs &ws, uint64_t *scan_total, uint32_t *n_items,
                        uint32_t *counter, hipStream_t s);
bool raster_tile_supported(int tw, int th);

// pose.hip: one Adam step per view on its pose tangent gradient, then the
// device view table is re-based (R <- Exp(w) R, t <- Exp(w) t + rho).
struct AdamCfg {
    float lr_trans, lr_rot, beta1, beta2, eps;
    int pivot_mode;  // 0: rotate about the source, 1: about the world point pivot
    float pivot[3];
};
// (skip: step flags; nothing changes while bit 0, a capacity overflow, is set)
hipError_t launch_pose_adam(ViewDev *views, int V, const float *dpose, float *state, uint32_t *step,
                            const AdamCfg &cfg, const uint32_t *skip, hipStream_t s);

// fit.hip -- the fitting loop: fused Adam over every parameter group,
// densification and the opacity reset.  The flat parameter index runs over
// the groups in model order: mean [3][n], quat [4][n], log_scale [3][n],
// opacity_logit [n], feat [k][n], b_iso [k], B_dir [k_L][k].
constexpr int kGroups = 7;
struct FitCfg {
    float lr_mean0, lr_mean1;  // position rate, log-linear decay over lr_steps steps
    int lr_steps;
    float lr[kGroups];         // rates of the other groups (lr[0] unused)
    float beta1, beta2, eps;
};
struct FitArgs {
    float *p[kGroups];
    const float *g[kGroups];
    int64_t off[kGroups + 1];  // flat offsets of the groups
    float *m, *v;              // moments [off[7]] each
    uint32_t *step;            // completed steps
    const uint32_t *skip;      // step flags: no update while bit 0 (overflow) is set
    FitCfg cfg;
};
int64_t fit_param_count(int64_t n, int k, int kl);
void fit_offsets(int64_t n, int k, int kl, int64_t *off);
// one Adam step, then the step count is raised (two launches)
hipError_t launch_fit_adam(const FitArgs &a, int num_cu, hipStream_t s);

struct DensifyTh {
    float grad, log_dense, logit_min_op, log_world, screen, log_split;  // +inf: bound off
};
// per Gaussian: keep (0/1), kept clone (0/1), kept children (0/2)
hipError_t launch_densify_plan(int n, const float *log_scale, const float *opacity, const float *acc,
                               const float *cnt, const float *rad, const DensifyTh &th, uint32_t *keep,
                               uint32_t *clone, uint32_t *child, hipStream_t s);
struct DensifyApplyArgs {
    int n, n_iso, k, kl;
    int64_t n_new;
    const float *src[5];   // mean, quat, log_scale, opacity_logit, feat of the current model
    float *dst[5];         // the same groups of the new model
    const uint32_t *keep, *clone, *child;           // plan
    const uint32_t *keep_ex, *clone_ex, *child_ex;  // their exclusive prefix sums
    uint32_t k_iso, c_iso, h_iso, k_tot, c_tot;     // prefixes at n_iso and totals
    const float *noise;    // [n][2][3]
    float log_split;
    const float *m_old, *v_old;  // moments of the current model (NULL: none)
    float *m_new, *v_new;
};
hipError_t launch_densify_apply(const DensifyApplyArgs &a, hipStream_t s);
// opacity_logit = min(opacity_logit, cap), opacity moments zeroed (m, v may be NULL)
hipError_t launch_opacity_reset(float *opacity, int n, float cap, float *m, float *v, hipStream_t s);

// rads.hip -- radiodensity-aware dual sampling
struct RadsVol {
    int nx, ny, nz;
    float sx, sy, sz;  // voxel size, mm
    float ox, oy, oz;  // centre of voxel (0, 0, 0), mm
    const float *hu;   // [nz][ny][nx]
};
int64_t rads_minmax_blocks(int64_t n, int num_cu);
int64_t rads_scan64_blocks(int64_t n);
// mm[0..2] = min, max, level (min + max) / 2
hipError_t launch_rads_level(const RadsVol &v, float2 *part, int64_t nb, float *mm, hipStream_t s);
hipError_t launch_mc_count(const RadsVol &v, const float *mm, uint32_t *cnt, hipStream_t s);
hipError_t launch_mc_emit(const RadsVol &v, const float *mm, const uint32_t *off, float *pts, int64_t M, hipStream_t s);
// cdf[i]: inclusive sum of the 16-bit weights; bsum [blocks + 1], bsum[blocks] = total
hipError_t launch_rads_cdf(const RadsVol &v, const float *mm, uint64_t *bsum, uint64_t *cdf, hipStream_t s);
hipError_t launch_iota(uint32_t *p, int64_t n, hipStream_t s);
hipError_t launch_rads_gather(const float *src, int64_t M, const uint32_t *idx, int64_t n1, float *out, int64_t N,
                              hipStream_t s);
hipError_t launch_rads_draws(const RadsVol &v, const uint64_t *cdf, const uint64_t *draws, int64_t n2, float *out,
                             int64_t N, int64_t first, hipStream_t s);
hipError_t launch_knn3(const float *pts, int64_t N, float *ls, hipStream_t s);

// loss.hip
// SSIM output tile (pixels): one workgroup of kLossTileW x kLossTileH threads
constexpr int kLossTileW = 32, kLossTileH = 32;
struct LossArgs {
    const ViewDev *views;
    int V;
    int64_t total_pix;
    const float *img, *target;
    // (captured steps) the target is read from this device slot, so that a
    // replay can take another target image without a copy; NULL: target
    const float *const *target_ref;
    float lambda;
    float *loss_out;   // [V] (may be NULL)
    float *grad;       // image layout (may be NULL)
    double *part;      // scratch
    float *maps;       // scratch, 3 * total_pix floats (SSIM)
    int loss_tiles;    // SSIM: total output tiles
    const int32_t *loss_tile_base; // [V+1]
    int64_t max_view_pix;          // largest W*H among the views
};
size_t loss_part_doubles(int V, int64_t max_view_pix, int loss_tiles);
hipError_t launch_loss(int kind, const LossArgs &a, hipStream_t s);

}  // namespace ddgs
