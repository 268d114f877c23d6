// ddgs_api.hip -- host runtime behind the C ABI of include/ddgs.h: context
// and error state, workspace planning, the plain single-call render and
// backward, the losses, the captured batched step (one HIP graph per shape,
// fixed tile-entry capacity with an overflow flag), the autotuner and the
// debug getters.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <limits>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/ddgs.h"
#include "internal.h"

using namespace ddgs;

// The static scratch of ddgs_sort_pairs_noalloc (the one entry point that
// allocates nothing): one copy per GPU, alive until the process ends.
constexpr int64_t kNoallocSortMax = (int64_t)1 << 20;         // pairs
constexpr size_t kNoallocScratchBytes = (size_t)12 << 20;    // 12 MiB
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace {

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

struct Status {
    ddgs_status code;
};

}  // namespace

struct ddgs_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int num_cu = 256;
    std::string err;

    ddgs_options opt{};
    bool has_model = false;
    ddgs_model model{};
    const float *c_override = nullptr;  // test hook: [V][n] radiosity instead of Eq. 3

    // pose optimiser appended to captured steps (registration)
    bool adam_on = false;
    AdamCfg adam{};
    bool adam_reset = true;   // zero the moments before the next replay

    // fitting optimiser appended to captured steps; densification
    bool fit_on = false;
    FitCfg fit{};
    bool fit_reset = true;          // zero moments and step count before the next replay
    bool fit_live = false;          // "fit_mv" holds moments of the current model
    int64_t fit_pending_n = -1, fit_pending_iso = -1;  // shape the last densify re-laid them out for
    float *st_grad = nullptr, *st_cnt = nullptr, *st_rad = nullptr;
    bool plan_ok = false;
    uint64_t plan_model_gen = 0;
    int64_t plan_n_new = 0, plan_iso_new = 0;
    uint32_t plan_pref[5] = {};     // keep, clone, child prefixes at n_iso; keep, clone totals
    const float *plan_noise = nullptr;
    float plan_log_split = 0.0f;

    // radiodensity-aware dual sampling between prepare and sample
    bool rads_ok = false;
    RadsVol rads_vol{};
    int64_t rads_m = 0;
    uint64_t rads_w = 0;
    std::vector<ddgs_view> views_h;

    // derived view table for the current options
    std::vector<ViewDev> vdev_h;
    std::vector<int32_t> loss_tile_base_h;
    int n_tiles = 0, loss_tiles = 0, max_view_tiles = 0;
    int64_t total_pix = 0, max_view_pix = 0;
    bool views_dirty = true;

    // workspace: buffers from the caller's allocator, carved from a caller
    // region, or (neither set) from hipMalloc
    std::map<std::string, DevBuf> bufs;
    char *ws_base = nullptr;      // caller workspace (NULL: an allocator per buffer)
    size_t ws_size = 0, ws_used = 0;
    ddgs_alloc_fn alloc_fn = nullptr;  // caller allocator (NULL: hipMalloc)
    ddgs_free_fn free_fn = nullptr;
    void *alloc_user = nullptr;
    bool dry_run = false;         // ensure() only adds up sizes (ddgs_workspace_size)
    size_t dry_total = 0;

    // state of the last render
    bool rendered = false;
    uint64_t model_gen = 0, views_gen = 0, opt_gen = 0;
    uint64_t r_model_gen = ~0ull, r_views_gen = ~0ull, r_opt_gen = ~0ull;
    int64_t M = 0;             // entries of the last render
    uint32_t *queue = nullptr;
    int64_t entry_cap = 0;     // capacity of the entry buffers
    bool keep_unsorted = false;
    bool count_pairs = false;

    // captured step
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    int64_t step_cap = 0;
    int64_t last_skipped = 0, last_need = 0;  // found by the last ddgs_check
    int max_items = 0;         // work items the raster grids are sized for
    bool items_folded = false; // the tile scan wrote the work items (captured step)
    // workgroups of the long-range tile sort: a plain render reads the number
    // of long tiles with the entry total and launches one per long tile (no
    // launch if there are none); a captured step takes twice the most that
    // plain renders of the same Gaussian count and tile layout saw (at least
    // 16), the full grid when none has been seen, and no second launch when
    // they saw none (the first launch then sorts any long tile a replay
    // has, through global memory).  Fewer workgroups than long tiles only
    // take several each; the lists are the same either way.
    int long_grid = 0;
    int64_t long_seen = -1, long_seen_n = -1;
    int long_seen_tiles = -1;

    // target image of the captured step's loss (uploaded with the view table)
    const float *step_target = nullptr;

    // pinned staging of the view table uploads
    void *stage_host = nullptr;
    size_t stage_bytes = 0;
    hipEvent_t stage_event = nullptr;
    bool stage_pending = false;

    // timing: a start and an end event per stage
    bool timing = false;
    hipEvent_t ev_s[DDGS_T_COUNT] = {};
    hipEvent_t ev_e[DDGS_T_COUNT] = {};
    // second part of the sort stage (enqueue_back)
    hipEvent_t ev_sort_tail_s = nullptr, ev_sort_tail_e = nullptr;
    bool ev_sort_tail_valid = false;
    bool ev_valid[DDGS_T_COUNT] = {};
};

namespace {

ddgs_status fail(ddgs_ctx *c, ddgs_status s, const std::string &msg)
{
    if (c) c->err = msg;
    return s;
}

#define HIP_TRY(ctx, expr)                                                                       \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return fail((ctx), e_ == hipErrorOutOfMemory ? DDGS_ERR_OOM : DDGS_ERR_HIP,          \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                       \
    } while (0)

#define DDGS_TRY(expr)                  \
    do {                                \
        ddgs_status s_ = (expr);        \
        if (s_ != DDGS_OK) return s_;   \
    } while (0)

constexpr size_t kWsAlign = 256;
size_t ws_round(size_t x) { return (x + kWsAlign - 1) / kWsAlign * kWsAlign; }

// (Re)allocates a workspace buffer of at least `bytes` (contents undefined),
// with room to grow by a quarter.  With a caller workspace the buffer is
// carved from it (a grown buffer takes new space; the region is never
// reused before ddgs_set_workspace is called again).  In a dry run only the
// sizes of fresh buffers are added up.  Never called while a stream capture
// is open.
ddgs_status ensure(ddgs_ctx *c, const char *name, size_t bytes, void **out)
{
    if (bytes == 0) bytes = 16;
    const size_t nb = ws_round(bytes + bytes / 4 + 256);
    if (c->dry_run) {
        c->dry_total += nb;
        *out = nullptr;
        return DDGS_OK;
    }
    DevBuf &b = c->bufs[name];
    if (b.bytes < bytes) {
        if (c->ws_base) {
            if (c->ws_used + nb > c->ws_size)
                return fail(c, DDGS_ERR_OOM, std::string("workspace too small: ") + name + " needs " +
                                                 std::to_string(nb) + " more bytes beyond " +
                                                 std::to_string(c->ws_used) + " of " + std::to_string(c->ws_size) +
                                                 " (see ddgs_workspace_size)");
            b.p = c->ws_base + c->ws_used;
            c->ws_used += nb;
        } else {
            if (b.p) {
                HIP_TRY(c, hipStreamSynchronize(c->stream));
                if (c->alloc_fn) c->free_fn(c->alloc_user, b.p);
                else HIP_TRY(c, hipFree(b.p));
                b.p = nullptr;
                b.bytes = 0;
            }
            if (c->alloc_fn) {
                b.p = c->alloc_fn(c->alloc_user, nb);
                if (!b.p)
                    return fail(c, DDGS_ERR_OOM, std::string("the caller's allocator returned NULL for ") + name +
                                                     " (" + std::to_string(nb) + " bytes)");
                if (((uintptr_t)b.p) % kWsAlign != 0) {
                    c->free_fn(c->alloc_user, b.p);
                    b.p = nullptr;
                    return fail(c, DDGS_ERR_INVALID_ARG, "the caller's allocator returned memory not 256-byte aligned");
                }
            } else {
                hipError_t e = hipMalloc(&b.p, nb);
                if (e != hipSuccess) {
                    b.p = nullptr;
                    return fail(c, DDGS_ERR_OOM, std::string("hipMalloc of ") + name + " (" + std::to_string(nb) +
                                                     " bytes) failed: " + hipGetErrorString(e));
                }
            }
        }
        b.bytes = nb;
    }
    *out = b.p;
    return DDGS_OK;
}

// Releases every workspace buffer (library-owned ones are freed).
void release_buffers(ddgs_ctx *c)
{
    (void)hipStreamSynchronize(c->stream);
    if (!c->ws_base)
        for (auto &kv : c->bufs) {
            if (!kv.second.p) continue;
            if (c->alloc_fn) c->free_fn(c->alloc_user, kv.second.p);
            else (void)hipFree(kv.second.p);
        }
    c->bufs.clear();
    c->ws_used = 0;
}

template <typename T>
ddgs_status ensure_t(ddgs_ctx *c, const char *name, size_t count, T **out)
{
    void *p = nullptr;
    DDGS_TRY(ensure(c, name, count * sizeof(T), &p));
    *out = (T *)p;
    return DDGS_OK;
}

template <typename T>
T *buf(ddgs_ctx *c, const char *name)
{
    auto it = c->bufs.find(name);
    return it == c->bufs.end() ? nullptr : (T *)it->second.p;
}

int kl_of(int L) { return L * (L + 2); }

RenderOpts render_opts(const ddgs_options &o)
{
    RenderOpts r;
    r.kappa = o.kappa;
    r.kappa2 = o.kappa * o.kappa;
    r.dilation = o.dilation;
    r.t_min = o.t_min;
    r.z_near = o.z_near;
    r.sigma_max = o.sigma_max;
    r.tile_w = o.tile_w;
    r.tile_h = o.tile_h;
    return r;
}

ModelDev model_dev(const ddgs_model &m, const float *c_override)
{
    ModelDev d;
    d.c_override = c_override;
    d.n = (int32_t)m.n;
    d.n_iso = (int32_t)m.n_iso;
    d.k = m.k;
    d.L = m.L;
    d.entangled = m.radiosity == DDGS_RADIOSITY_ENTANGLED ? 1 : 0;
    d.mean = m.mean;
    d.quat = m.quat;
    d.log_scale = m.log_scale;
    d.opacity_logit = m.opacity_logit;
    d.feat = m.feat;
    d.b_iso = m.b_iso;
    d.B_dir = m.B_dir;
    return d;
}

int bits_for(int64_t n)
{
    int b = 1;
    while (b < 32 && ((int64_t)1 << b) < n) ++b;
    return b;
}

// The "views" buffer holds the device views (at least one slot), the V + 1
// first loss tiles per view, and the captured step's target image pointer.
size_t loss_base_offset(int V) { return sizeof(ViewDev) * (size_t)std::max(1, V); }
size_t target_slot_offset(int V) { return (loss_base_offset(V) + sizeof(int32_t) * (size_t)(V + 1) + 7) & ~(size_t)7; }
size_t views_bytes(int V) { return target_slot_offset(V) + sizeof(void *); }
const float *const *target_slot_ptr(ddgs_ctx *c)
{
    char *p = buf<char>(c, "views");
    return p ? reinterpret_cast<const float *const *>(p + target_slot_offset((int)c->views_h.size())) : nullptr;
}
int32_t *loss_tile_base_ptr(ddgs_ctx *c)
{
    char *p = buf<char>(c, "views");
    return p ? reinterpret_cast<int32_t *>(p + loss_base_offset((int)c->views_h.size())) : nullptr;
}

// Builds the device view table (tile grid depends on the tile size).
ddgs_status prepare_views(ddgs_ctx *c)
{
    if (!c->views_dirty) return DDGS_OK;
    const int V = (int)c->views_h.size();
    c->vdev_h.assign(V, ViewDev{});
    c->loss_tile_base_h.assign(V + 1, 0);
    int64_t tiles = 0, pix = 0, ltiles = 0, maxp = 0;
    c->max_view_tiles = 0;
    for (int v = 0; v < V; ++v) {
        const ddgs_view &h = c->views_h[v];
        ViewDev &d = c->vdev_h[v];
        for (int r = 0; r < 3; ++r) {
            for (int q = 0; q < 3; ++q) d.R[3 * r + q] = h.pose[4 * r + q];
            d.t[r] = h.pose[4 * r + 3];
        }
        for (int q = 0; q < 3; ++q) {
            const double s = -((double)h.pose[q] * h.pose[3] + (double)h.pose[4 + q] * h.pose[7] +
                               (double)h.pose[8 + q] * h.pose[11]);
            d.so[q] = (float)s;
        }
        d.f = (float)((double)h.sdd_mm / (double)h.pitch_mm);
        d.cx = 0.5f * (float)h.W;
        d.cy = 0.5f * (float)h.H;
        d.W = h.W;
        d.H = h.H;
        d.ntx = (h.W + c->opt.tile_w - 1) / c->opt.tile_w;
        d.nty = (h.H + c->opt.tile_h - 1) / c->opt.tile_h;
        d.tile_base = (int32_t)tiles;
        d.pix_base = pix;
        tiles += (int64_t)d.ntx * d.nty;
        c->max_view_tiles = std::max(c->max_view_tiles, d.ntx * d.nty);
        pix += (int64_t)h.W * h.H;
        maxp = std::max<int64_t>(maxp, (int64_t)h.W * h.H);
        c->loss_tile_base_h[v] = (int32_t)ltiles;
        ltiles += (int64_t)((h.W + kLossTileW - 1) / kLossTileW) * ((h.H + kLossTileH - 1) / kLossTileH);
    }
    c->loss_tile_base_h[V] = (int32_t)ltiles;
    if (tiles >= (int64_t)1 << 30 || ltiles >= (int64_t)1 << 30)
        return fail(c, DDGS_ERR_INVALID_ARG, "too many tiles");
    c->n_tiles = (int)tiles;
    c->loss_tiles = (int)ltiles;
    c->total_pix = pix;
    c->max_view_pix = maxp;
    // one buffer, one upload: the views, then the loss tiles' bases
    void *vp;
    DDGS_TRY(ensure(c, "views", views_bytes(V), &vp));
    // stage through pinned host memory so the copy stays asynchronous; the
    // staging area is reused only after the previous upload has completed
    const size_t need = views_bytes(V);
    if (c->stage_pending) {
        HIP_TRY(c, hipEventSynchronize(c->stage_event));
        c->stage_pending = false;
    }
    if (c->stage_bytes < need) {
        if (c->stage_host) HIP_TRY(c, hipHostFree(c->stage_host));
        c->stage_host = nullptr;
        c->stage_bytes = 0;
        HIP_TRY(c, hipHostMalloc(&c->stage_host, need + 1024, hipHostMallocDefault));
        c->stage_bytes = need + 1024;
    }
    char *h = (char *)c->stage_host;
    if (V > 0) std::memcpy(h, c->vdev_h.data(), sizeof(ViewDev) * V);
    std::memcpy(h + loss_base_offset(V), c->loss_tile_base_h.data(), sizeof(int32_t) * (V + 1));
    std::memcpy(h + target_slot_offset(V), &c->step_target, sizeof(void *));
    HIP_TRY(c, hipMemcpyAsync(vp, h, need, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipEventRecord(c->stage_event, c->stream));
    c->stage_pending = true;
    c->views_dirty = false;
    return DDGS_OK;
}

ddgs_status check_ready(ddgs_ctx *c)
{
    if (!c->has_model) return fail(c, DDGS_ERR_STATE, "no model set");
    if (c->views_h.empty()) return fail(c, DDGS_ERR_STATE, "no views set");
    return prepare_views(c);
}

// Buffers whose size depends on n and the views only.
ddgs_status ensure_static(ddgs_ctx *c)
{
    const int64_t n = c->model.n, V = (int64_t)c->views_h.size(), VN = n * V;
    const int KL = kl_of(c->model.L);
    float *f;
    uint32_t *u;
    DDGS_TRY(ensure_t(c, "cov", 6 * n, &f));
    DDGS_TRY(ensure_t(c, "alpha", n, &f));
    DDGS_TRY(ensure_t(c, "ciso", n, &f));
    DDGS_TRY(ensure_t(c, "hdir", (size_t)KL * std::max<int64_t>(1, n - c->model.n_iso), &f));
    float4 *f4;
    DDGS_TRY(ensure_t(c, "rec", 4 * VN, &f4));
    uint2 *u2;
    DDGS_TRY(ensure_t(c, "rect", VN, &u2));
    const char *u32s[] = {"zkey", "cnt", "slot_lp", "tmask"};
    for (const char *nm : u32s) DDGS_TRY(ensure_t(c, nm, VN, &u));
    DDGS_TRY(ensure_t(c, "tile_cnt", std::max(1, c->n_tiles), &u));
    DDGS_TRY(ensure_t(c, "bin_mat", bin_matrix_words(n, c->n_tiles), &u));
    DDGS_TRY(ensure_t(c, "cursor", std::max(1, c->n_tiles), &u));
    uint64_t *tb;
    DDGS_TRY(ensure_t(c, "tile_bsum", std::max(1, (c->n_tiles + 255) / 256), &tb));
    DDGS_TRY(ensure_t(c, "slot_btot", std::max<int64_t>(1, (int64_t)c->views_h.size() * slot_blocks(n)), &u));
    DDGS_TRY(ensure_t(c, "ranges", std::max(1, c->n_tiles), &u2));
    DDGS_TRY(ensure_t(c, "long_tiles", std::max(1, c->n_tiles), &u));
    DDGS_TRY(ensure_t(c, "long_bsum", std::max(1, (c->n_tiles + 255) / 256), &u));
    DDGS_TRY(ensure_t(c, "qkey", std::max(1, c->n_tiles), &u));
    DDGS_TRY(ensure_t(c, "qval", std::max(1, c->n_tiles), &u));
    DDGS_TRY(ensure_t(c, "qkey2", std::max(1, c->n_tiles), &u));
    DDGS_TRY(ensure_t(c, "qval2", std::max(1, c->n_tiles), &u));
    DDGS_TRY(ensure_t(c, "img_saved", c->total_pix, &f));
    DDGS_TRY(ensure_t(c, "nlast", c->total_pix, &u));
    {
        // the flags word is sticky (cleared by ddgs_check), so a new buffer
        // starts cleared
        uint32_t *prev = buf<uint32_t>(c, "scalars");
        DDGS_TRY(ensure_t(c, "scalars", 16, &u));
        if (u && u != prev) HIP_TRY(c, hipMemsetAsync(u, 0, sizeof(uint32_t) * 16, c->stream));
    }
    DDGS_TRY(ensure_t(c, "pose_part", (size_t)std::max<int64_t>(1, V * slot_blocks(n) * 9), &f));
    DDGS_TRY(ensure_t(c, "basis_part", basis_part_floats((int)std::max<int64_t>(1, n)), &f));
    DDGS_TRY(ensure_t(c, "zbuf", (size_t)std::max<int64_t>(1, n), &f));
    DDGS_TRY(ensure_t(c, "ubuf", (size_t)KL * std::max<int64_t>(1, n - c->model.n_iso), &f));
    double *d;
    DDGS_TRY(ensure_t(c, "loss_part", loss_part_doubles((int)V, c->max_view_pix, c->loss_tiles), &d));
    DDGS_TRY(ensure_t(c, "loss_maps", (size_t)3 * c->total_pix, &f));
    return DDGS_OK;
}

// Chunked work items are exact for Eq. 1 without early termination; with
// t_min > 0 each tile is walked by one workgroup.
int effective_split(const ddgs_ctx *c) { return c->opt.t_min > 0.0f ? 0 : std::max(0, (int)c->opt.split); }

// long-range sort grid of a captured step (see ddgs_ctx::long_grid)
int captured_long_grid(const ddgs_ctx *c)
{
    const bool seen = c->long_seen >= 0 && c->long_seen_n == c->model.n && c->long_seen_tiles == c->n_tiles;
    if (!seen) return 1 << 30;
    if (c->long_seen == 0) return 0;
    return (int)std::max<int64_t>(16, std::min<int64_t>(2 * c->long_seen, 1 << 30));
}

int64_t max_items_for(const ddgs_ctx *c, int64_t cap)
{
    const int split = effective_split(c);
    return split > 0 ? cap / split + c->n_tiles + 1 : c->n_tiles;
}

// Entry-level buffers (tile entries) and the radix / scan temporaries.
ddgs_status ensure_entries(ddgs_ctx *c, int64_t cap)
{
    const int64_t VN = c->model.n * (int64_t)c->views_h.size();
    uint32_t *u;
    float4 *f4;
    uint2 *e2;
    DDGS_TRY(ensure_t(c, "bin_ent", cap, &e2));
    DDGS_TRY(ensure_t(c, "bin_tmp", cap, &e2));
    DDGS_TRY(ensure_t(c, "tval", cap, &u));
    DDGS_TRY(ensure_t(c, "slot", 2 * cap, &f4));
    if (c->keep_unsorted) DDGS_TRY(ensure_t(c, "ubin", cap, &e2));
    // work items of the chunked raster and their per-pixel (C, T) partials
    const int split = effective_split(c);
    const int64_t max_items = split > 0 ? cap / split + c->n_tiles + 1 : 1;
    uint2 *u2;
    float2 *f2;
    DDGS_TRY(ensure_t(c, "items", max_items, &u2));
    DDGS_TRY(ensure_t(c, "item_cnt", std::max(1, c->n_tiles), &u));
    DDGS_TRY(ensure_t(c, "item_base", std::max(1, c->n_tiles), &u));
    DDGS_TRY(ensure_t(c, "part", (size_t)(split > 0 ? max_items : 1) * c->opt.tile_w * c->opt.tile_h, &f2));
    const int64_t big = std::max<int64_t>({VN, (int64_t)c->n_tiles, 1});
    DDGS_TRY(ensure_t(c, "sort_counts", sort_counts_words(big), &u));
    DDGS_TRY(ensure_t(c, "sort_tot", kSortTotWords, &u));
    uint64_t *bs;
    DDGS_TRY(ensure_t(c, "sort_bsum", sort_blocksum_words(big), &bs));
    if (!c->dry_run) c->entry_cap = std::max(c->entry_cap, cap);
    return DDGS_OK;
}

void stage_begin(ddgs_ctx *c, int i)
{
    if (c->timing) (void)hipEventRecord(c->ev_s[i], c->stream);
    if (i == DDGS_T_SORT) c->ev_sort_tail_valid = false;
}
void stage_end(ddgs_ctx *c, int i)
{
    if (c->timing) {
        (void)hipEventRecord(c->ev_e[i], c->stream);
        c->ev_valid[i] = true;
    }
}

// device scalars: [0..1] u64 entry total, [2] entries kept (min(total, cap)),
// [3] flags (bit 0: capacity overflow in some step since the last
// ddgs_check, which clears them), [4], [5] work-queue counters,
// [6] work items, [7] captured replays whose updates were skipped since the
// last ddgs_check, [8..9] u64 scratch total, [10..11] u64 largest entry total
// of a captured replay since the last ddgs_check, [12] the number of tiles
// the tile scan listed for the tile sort's long-range launch
uint64_t *total_ptr(ddgs_ctx *c) { return (uint64_t *)buf<uint32_t>(c, "scalars"); }
uint32_t *mdev_ptr(ddgs_ctx *c) { return buf<uint32_t>(c, "scalars") + 2; }
uint32_t *flags_ptr(ddgs_ctx *c) { return buf<uint32_t>(c, "scalars") + 3; }
uint32_t *skipped_ptr(ddgs_ctx *c) { return buf<uint32_t>(c, "scalars") + 7; }
unsigned long long *need_ptr(ddgs_ctx *c) { return (unsigned long long *)(buf<uint32_t>(c, "scalars") + 10); }
uint32_t *counter_ptr(ddgs_ctx *c) { return buf<uint32_t>(c, "scalars") + 4; }
uint64_t *sort_total_ptr(ddgs_ctx *c) { return (uint64_t *)(buf<uint32_t>(c, "scalars") + 8); }
uint32_t *n_items_ptr(ddgs_ctx *c) { return buf<uint32_t>(c, "scalars") + 6; }
LongTiles long_tiles(ddgs_ctx *c)
{
    return LongTiles{buf<uint32_t>(c, "long_tiles"), buf<uint32_t>(c, "scalars") + 12, buf<uint32_t>(c, "long_bsum"),
                     c->bufs["long_bsum"].bytes / sizeof(uint32_t)};
}
SortWs sort_ws(ddgs_ctx *c)
{
    return SortWs{buf<uint32_t>(c, "sort_counts"), buf<uint32_t>(c, "sort_tot"), buf<uint64_t>(c, "sort_bsum"),
                  c->bufs["sort_counts"].bytes / sizeof(uint32_t), c->bufs["sort_bsum"].bytes / sizeof(uint64_t)};
}

// Sort / scan temporaries of the calls outside the render path (the debug
// entry points, densification, dual sampling): buffers of their own, so such a
// call leaves the render state alone.
ddgs_status aux_sort_ws(ddgs_ctx *c, int64_t n, SortWs *ws)
{
    uint32_t *u;
    uint64_t *bs;
    DDGS_TRY(ensure_t(c, "aux_counts", sort_counts_words(std::max<int64_t>(n, 1)), &u));
    DDGS_TRY(ensure_t(c, "aux_tot", kSortTotWords, &u));
    DDGS_TRY(ensure_t(c, "aux_bsum", sort_blocksum_words(std::max<int64_t>(n, 1)), &bs));
    *ws = SortWs{buf<uint32_t>(c, "aux_counts"), buf<uint32_t>(c, "aux_tot"), buf<uint64_t>(c, "aux_bsum"),
                 c->bufs["aux_counts"].bytes / sizeof(uint32_t), c->bufs["aux_bsum"].bytes / sizeof(uint64_t)};
    return DDGS_OK;
}

// Work-item fields shared by the forward and backward raster launches.
void set_items(ddgs_ctx *c, RasterArgs &ra, bool backward)
{
    ra.split = effective_split(c);
    ra.items = buf<uint2>(c, "items");
    ra.n_items = n_items_ptr(c);
    ra.max_items = c->max_items;
    ra.item_base = buf<uint32_t>(c, "item_base");
    ra.item_cnt = buf<uint32_t>(c, "item_cnt");
    ra.part = buf<float2>(c, "part");
    ra.queue = c->queue;
    ra.queue_counter = c->opt.persistent ? counter_ptr(c) + (backward ? 1 : 0) : nullptr;
}

// Projection (which also counts every tile's entries) and the scan of the
// tile counts into the tile ranges (stages shared by the plain and the
// captured paths).  capacity: entries the tile lists may hold (the plain path
// passes 2^32 - 1 and sizes its buffers from the total afterwards); captured:
// the step counters (skipped replays, largest need) are kept.
ddgs_status enqueue_front(ddgs_ctx *c, uint32_t capacity, bool captured)
{
    hipStream_t s = c->stream;
    const ModelDev m = model_dev(c->model, c->c_override);
    const int V = (int)c->views_h.size();
    GaussCache gc{buf<float>(c, "cov"), buf<float>(c, "alpha"), buf<float>(c, "ciso"), buf<float>(c, "hdir")};
    ProjOut po{buf<float4>(c, "rec"),   buf<uint2>(c, "rect"),        buf<uint32_t>(c, "tmask"),
               buf<uint32_t>(c, "zkey"), buf<uint32_t>(c, "cnt"),       buf<uint32_t>(c, "slot_lp"),
               buf<uint32_t>(c, "slot_btot")};
    const RenderOpts ro = render_opts(c->opt);
    stage_begin(c, DDGS_T_PROJECT);
    HIP_TRY(c, launch_prep_project(m, gc, buf<ViewDev>(c, "views"), V, ro, po, s));
    stage_end(c, DDGS_T_PROJECT);
    stage_begin(c, DDGS_T_SORT);
    HIP_TRY(c, launch_bin_count(m.n, V, buf<uint32_t>(c, "cnt"), buf<uint2>(c, "rect"), buf<uint32_t>(c, "tmask"),
                                buf<ViewDev>(c, "views"), c->n_tiles, c->max_view_tiles, buf<uint32_t>(c, "bin_mat"),
                                buf<uint32_t>(c, "tile_cnt"), s));
    // a captured step (its buffers are sized already) has the scan write the
    // chunked raster's work items too
    TileItems ti{};
    const bool fold = captured && effective_split(c) > 0 && tile_scan_makes_items(c->n_tiles);
    if (fold) {
        c->max_items = (int)max_items_for(c, capacity);
        ti = TileItems{effective_split(c), buf<uint32_t>(c, "item_cnt"), buf<uint32_t>(c, "item_base"),
                       buf<uint2>(c, "items"), (uint32_t)c->max_items, n_items_ptr(c), counter_ptr(c)};
    }
    c->items_folded = fold;
    HIP_TRY(c, launch_tile_scan(buf<uint32_t>(c, "tile_cnt"), c->n_tiles, buf<uint2>(c, "ranges"),
                                buf<uint32_t>(c, "cursor"), capacity, total_ptr(c), mdev_ptr(c), flags_ptr(c),
                                captured ? skipped_ptr(c) : nullptr, captured ? need_ptr(c) : nullptr,
                                buf<uint32_t>(c, "slot_btot"), (int64_t)V * slot_blocks(m.n), buf<uint64_t>(c, "tile_bsum"),
                                c->bufs["tile_bsum"].bytes / sizeof(uint64_t), fold ? &ti : nullptr, long_tiles(c), s));
    // the sort stage is timed in two parts: a plain render reads the entry
    // total back to the host between them, and that round trip is not device work
    stage_end(c, DDGS_T_SORT);
    return DDGS_OK;
}

// Scatter of the entries into their tile ranges, the per-tile sort, the
// optional work items or queue, and the forward raster.
ddgs_status enqueue_back(ddgs_ctx *c, int64_t cap, float *images)
{
    hipStream_t s = c->stream;
    const int V = (int)c->views_h.size();
    const int n = (int)c->model.n;
    uint2 *ent = buf<uint2>(c, "bin_ent");
    if (c->timing) (void)hipEventRecord(c->ev_sort_tail_s, c->stream);
    HIP_TRY(c, launch_bin_scatter(n, V, buf<uint32_t>(c, "cnt"), buf<uint2>(c, "rect"), buf<uint32_t>(c, "tmask"),
                                  buf<uint32_t>(c, "zkey"), buf<ViewDev>(c, "views"), c->n_tiles, c->max_view_tiles,
                                  buf<uint32_t>(c, "bin_mat"), buf<uint32_t>(c, "cursor"), (uint32_t)cap, ent, s));
    if (c->keep_unsorted)
        HIP_TRY(c, launch_copy_u32((uint32_t *)buf<uint2>(c, "ubin"), (const uint32_t *)ent, nullptr, 2 * cap, s));
    HIP_TRY(c, launch_tile_sort(buf<uint2>(c, "ranges"), buf<uint32_t>(c, "tile_cnt"), c->n_tiles, ent,
                                buf<uint2>(c, "bin_tmp"), buf<uint32_t>(c, "tval"), long_tiles(c), c->long_grid, s));
    c->queue = nullptr;
    const int split = effective_split(c);
    c->max_items = (int)max_items_for(c, cap);
    if (split > 0 && c->items_folded) {
        // (written by the tile scan)
    } else if (split > 0) {
        HIP_TRY(c, launch_items(buf<uint2>(c, "ranges"), c->n_tiles, split, buf<uint32_t>(c, "item_cnt"),
                                buf<uint32_t>(c, "item_base"), buf<uint2>(c, "items"), (uint32_t)c->max_items,
                                sort_ws(c), sort_total_ptr(c), n_items_ptr(c), counter_ptr(c), s));
    } else if (c->opt.persistent) {
        bool qk1 = false;
        HIP_TRY(c, launch_tile_cost_keys(buf<uint2>(c, "ranges"), c->n_tiles, buf<uint32_t>(c, "qkey"),
                                         buf<uint32_t>(c, "qval"), counter_ptr(c), s));
        HIP_TRY(c, radix_sort_pairs(buf<uint32_t>(c, "qkey"), buf<uint32_t>(c, "qval"), buf<uint32_t>(c, "qkey2"),
                                    buf<uint32_t>(c, "qval2"), c->n_tiles, nullptr, 24, sort_ws(c), &qk1, s));
        c->queue = qk1 ? buf<uint32_t>(c, "qval2") : buf<uint32_t>(c, "qval");
    }
    if (c->timing) {
        (void)hipEventRecord(c->ev_sort_tail_e, c->stream);
        c->ev_sort_tail_valid = true;
    }
    stage_begin(c, DDGS_T_RASTER_FWD);
    RasterArgs ra{};
    ra.views = buf<ViewDev>(c, "views");
    ra.V = V;
    ra.n = n;
    ra.o = render_opts(c->opt);
    ra.ranges = buf<uint2>(c, "ranges");
    ra.tval = buf<uint32_t>(c, "tval");
    ra.rec = buf<float4>(c, "rec");
    ra.n_tiles = c->n_tiles;
    set_items(c, ra, false);
    ra.img = images;
    ra.img_saved = buf<float>(c, "img_saved");
    ra.nlast = buf<uint32_t>(c, "nlast");
    ra.pair_counts = nullptr;
    if (c->count_pairs) {
        unsigned long long *pc;
        DDGS_TRY(ensure_t(c, "pair_counts", 128, &pc));
        ra.pair_counts = pc;
        HIP_TRY(c, launch_fill_u32((uint32_t *)pc, 0u, 256, s));
    }
    HIP_TRY(c, launch_raster_fwd(ra, c->num_cu * 4 * std::max(1, (int)c->opt.persistent), s));
    stage_end(c, DDGS_T_RASTER_FWD);
    return DDGS_OK;
}

// Writable pointers of the model groups in flat order: the fitting optimiser
// and the opacity reset update the caller's arrays in place (the caller
// enables them only for writable memory).
void fit_groups(ddgs_ctx *c, float **p)
{
    const ddgs_model &m = c->model;
    const float *q[kGroups] = {m.mean, m.quat, m.log_scale, m.opacity_logit, m.feat, m.b_iso, m.B_dir};
    for (int g = 0; g < kGroups; ++g) p[g] = const_cast<float *>(q[g]);
}

bool any_param_grad(const ddgs_grads *g)
{
    return g->dmean || g->dquat || g->dlog_scale || g->dopacity_logit || g->dfeat || g->db_iso || g->dB_dir;
}

// captured: the densification statistics skip overflowed replays
ddgs_status enqueue_backward(ddgs_ctx *c, const float *dL, const ddgs_grads *g, int64_t slot_cap, bool captured)
{
    hipStream_t s = c->stream;
    const int V = (int)c->views_h.size();
    const int n = (int)c->model.n;
    RasterArgs ra{};
    ra.views = buf<ViewDev>(c, "views");
    ra.V = V;
    ra.n = n;
    ra.o = render_opts(c->opt);
    ra.ranges = buf<uint2>(c, "ranges");
    ra.tval = buf<uint32_t>(c, "tval");
    ra.rec = buf<float4>(c, "rec");
    ra.n_tiles = c->n_tiles;
    set_items(c, ra, true);
    ra.img_saved = buf<float>(c, "img_saved");
    ra.nlast = buf<uint32_t>(c, "nlast");
    ra.dL_dimg = dL;
    ra.rect = buf<uint2>(c, "rect");
    ra.slot_bofs = buf<uint32_t>(c, "slot_btot");
    ra.slot_nblk = (int)slot_blocks(n);
    ra.slot = buf<float4>(c, "slot");
    ra.slot_cap = (uint32_t)std::min<int64_t>(slot_cap, 0xFFFFFFFFll);
    stage_begin(c, DDGS_T_RASTER_BWD);
    if (c->opt.persistent) HIP_TRY(c, launch_fill_u32(counter_ptr(c) + 1, 0u, 1, s));
    HIP_TRY(c, launch_raster_bwd(ra, c->num_cu * 2 * std::max(1, (int)c->opt.persistent), s));
    stage_end(c, DDGS_T_RASTER_BWD);
    stage_begin(c, DDGS_T_PROJECT_BWD);

    const bool per_g = any_param_grad(g);
    ProjBwdArgs pa{};
    pa.m = model_dev(c->model, c->c_override);
    pa.gc = GaussCache{buf<float>(c, "cov"), buf<float>(c, "alpha"), buf<float>(c, "ciso"), buf<float>(c, "hdir")};
    pa.views = buf<ViewDev>(c, "views");
    pa.V = V;
    pa.o = render_opts(c->opt);
    pa.cnt = buf<uint32_t>(c, "cnt");
    pa.slot_lp = buf<uint32_t>(c, "slot_lp");
    pa.slot_bofs = buf<uint32_t>(c, "slot_btot");
    pa.slot_nblk = (int)slot_blocks(n);
    pa.slot = buf<float4>(c, "slot");
    pa.dmean = g->dmean;
    pa.dquat = g->dquat;
    pa.dlog_scale = g->dlog_scale;
    pa.dopacity = g->dopacity_logit;
    pa.dfeat = g->dfeat;
    pa.bpart = (g->db_iso || g->dB_dir) ? buf<float>(c, "basis_part") : nullptr;
    pa.pose_part = buf<float>(c, "pose_part");
    pa.per_gaussian = per_g ? 1 : 0;
    pa.slot_cap = ra.slot_cap;
    pa.st_grad = c->st_grad;
    pa.st_cnt = c->st_cnt;
    pa.st_rad = c->st_rad;
    pa.skip = captured ? flags_ptr(c) : nullptr;
    // feature and basis gradients in a second launch, from the radiosity
    // logits' gradients
    const bool feat_g = per_g && (pa.dfeat || pa.bpart);
    pa.zbuf = feat_g ? buf<float>(c, "zbuf") : nullptr;
    pa.ubuf = feat_g ? buf<float>(c, "ubuf") : nullptr;
    HIP_TRY(c, launch_project_bwd(pa, s));
    // (one pose partial per projection block)
    HIP_TRY(c, launch_grad_final(pa.m, buf<float>(c, "basis_part"), g->db_iso, g->dB_dir, buf<ViewDev>(c, "views"), V,
                                 (int)slot_blocks(n), buf<float>(c, "pose_part"), g->dpose, s));
    stage_end(c, DDGS_T_PROJECT_BWD);
    return DDGS_OK;
}

// (captured: the target is read from the view table's target slot)
ddgs_status enqueue_loss(ddgs_ctx *c, int kind, const float *images, const float *target, float lambda,
                         float *loss_out, float *dL, bool captured = false)
{
    LossArgs la{};
    la.views = buf<ViewDev>(c, "views");
    la.V = (int)c->views_h.size();
    la.total_pix = c->total_pix;
    la.img = images;
    la.target = target;
    la.target_ref = captured ? target_slot_ptr(c) : nullptr;
    la.lambda = lambda;
    la.loss_out = loss_out;
    la.grad = dL;
    la.part = buf<double>(c, "loss_part");
    la.maps = buf<float>(c, "loss_maps");
    la.loss_tiles = c->loss_tiles;
    la.loss_tile_base = loss_tile_base_ptr(c);
    la.max_view_pix = c->max_view_pix;
    stage_begin(c, DDGS_T_LOSS);
    HIP_TRY(c, launch_loss(kind, la, c->stream));
    stage_end(c, DDGS_T_LOSS);
    return DDGS_OK;
}

void drop_graph(ddgs_ctx *c)
{
    if (c->exec) (void)hipGraphExecDestroy(c->exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->exec = nullptr;
    c->graph = nullptr;
}

ddgs_status validate_options(ddgs_ctx *c, const ddgs_options &o)
{
    if (!raster_tile_supported(o.tile_w, o.tile_h))
        return fail(c, DDGS_ERR_UNSUPPORTED, "tile shape not supported (8x8, 16x8, 16x16, 32x8)");
    if (!(o.kappa > 0.0f) || !std::isfinite(o.kappa)) return fail(c, DDGS_ERR_INVALID_ARG, "kappa must be > 0");
    if (!(o.dilation >= 0.0f) || !std::isfinite(o.dilation)) return fail(c, DDGS_ERR_INVALID_ARG, "dilation must be >= 0");
    if (!(o.t_min >= 0.0f) || !(o.t_min < 1.0f)) return fail(c, DDGS_ERR_INVALID_ARG, "t_min must be in [0, 1)");
    if (!(o.z_near > 0.0f) || !std::isfinite(o.z_near)) return fail(c, DDGS_ERR_INVALID_ARG, "z_near must be > 0");
    if (!(o.sigma_max > 0.0f) || !(o.sigma_max < 1.0f)) return fail(c, DDGS_ERR_INVALID_ARG, "sigma_max must be in (0, 1)");
    if (o.capacity < 0 || o.capacity > 0xFFFFFFFFll) return fail(c, DDGS_ERR_INVALID_ARG, "capacity out of range");
    if (o.split < 0 || o.split > (1 << 24)) return fail(c, DDGS_ERR_INVALID_ARG, "split must be in 0..2^24");
    if (o.persistent < 0 || o.persistent > 8) return fail(c, DDGS_ERR_INVALID_ARG, "persistent must be in 0..8");
    return DDGS_OK;
}

bool is_state_current(const ddgs_ctx *c)
{
    return c->rendered && c->r_model_gen == c->model_gen && c->r_views_gen == c->views_gen &&
           c->r_opt_gen == c->opt_gen;
}

// ----------------------------------------------- static scratch (no allocation)
// ddgs_sort_pairs_noalloc takes its temporaries from this file-scope device
// array instead of the workspace: every GPU the library runs on holds its own
// copy until the process ends.  Host code never passes the array's name to
// a kernel (on the host it is only a stand-in for the symbol); it uses the
// device address hipGetSymbolAddress returns, looked up once per device (at
// ddgs_create, or at the entry point's first call on a device) and kept.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Looks up the scratch address of the current device (c->device) once.
ddgs_status scratch_lookup(ddgs_ctx *c)
{
    if (c->device < 0 || c->device >= kMaxDevices) return fail(c, DDGS_ERR_UNSUPPORTED, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[c->device]) return DDGS_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return fail(c, DDGS_ERR_HIP, std::string("hipGetSymbolAddress of the static scratch: ") + hipGetErrorString(e));
    g_scratch_ptr[c->device] = p;
    return DDGS_OK;
}

ddgs_status scratch_base(ddgs_ctx *c, char **out)
{
    DDGS_TRY(scratch_lookup(c));
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    *out = (char *)g_scratch_ptr[c->device];
    return DDGS_OK;
}

}  // namespace

// ======================================================================= ABI

extern "C" {

const char *ddgs_status_str(ddgs_status s)
{
    switch (s) {
    case DDGS_OK: return "ok";
    case DDGS_ERR_INVALID_ARG: return "invalid argument";
    case DDGS_ERR_OOM: return "out of device memory";
    case DDGS_ERR_HIP: return "HIP runtime error";
    case DDGS_ERR_CAPACITY: return "tile-entry capacity exceeded";
    case DDGS_ERR_NONFINITE: return "non-finite input";
    case DDGS_ERR_STATE: return "call out of order";
    case DDGS_ERR_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char *ddgs_last_error(const ddgs_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

void ddgs_default_options(ddgs_options *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->tile_w = 16;
    o->tile_h = 16;
    o->kappa = 3.0f;
    o->dilation = 0.3f;
    o->t_min = 0.0f;
    o->z_near = 1.0f;
    o->sigma_max = 0.99f;
    o->persistent = 0;
    o->split = 256;
    o->capacity = 0;
}

ddgs_status ddgs_create(ddgs_ctx **out, int device, void *hip_stream)
{
    if (!out) return DDGS_ERR_INVALID_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return DDGS_ERR_HIP;
    if (device < 0 || device >= ndev) return DDGS_ERR_INVALID_ARG;
    if (hipSetDevice(device) != hipSuccess) return DDGS_ERR_HIP;
    ddgs_ctx *c = new (std::nothrow) ddgs_ctx();
    if (!c) return DDGS_ERR_OOM;
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    ddgs_default_options(&c->opt);
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && ncu > 0)
        c->num_cu = ncu;
    for (int i = 0; i < DDGS_T_COUNT; ++i) {
        if (hipEventCreate(&c->ev_s[i]) != hipSuccess || hipEventCreate(&c->ev_e[i]) != hipSuccess) {
            ddgs_destroy(c);
            return DDGS_ERR_HIP;
        }
    }
    if (hipEventCreate(&c->ev_sort_tail_s) != hipSuccess || hipEventCreate(&c->ev_sort_tail_e) != hipSuccess) {
        ddgs_destroy(c);
        return DDGS_ERR_HIP;
    }
    if (hipEventCreateWithFlags(&c->stage_event, hipEventDisableTiming) != hipSuccess) {
        ddgs_destroy(c);
        return DDGS_ERR_HIP;
    }
    // the static scratch of ddgs_sort_pairs_noalloc: looked up once per device
    // (a failure is reported by that entry point, which tries again)
    (void)scratch_lookup(c);
    *out = c;
    return DDGS_OK;
}

void ddgs_destroy(ddgs_ctx *c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    drop_graph(c);
    release_buffers(c);
    for (int i = 0; i < DDGS_T_COUNT; ++i) {
        if (c->ev_s[i]) (void)hipEventDestroy(c->ev_s[i]);
        if (c->ev_e[i]) (void)hipEventDestroy(c->ev_e[i]);
    }
    if (c->ev_sort_tail_s) (void)hipEventDestroy(c->ev_sort_tail_s);
    if (c->ev_sort_tail_e) (void)hipEventDestroy(c->ev_sort_tail_e);
    if (c->stage_event) (void)hipEventDestroy(c->stage_event);
    if (c->stage_host) (void)hipHostFree(c->stage_host);
    delete c;
}

ddgs_status ddgs_set_stream(ddgs_ctx *c, void *s)
{
    if (!c) return DDGS_ERR_INVALID_ARG;
    c->stream = (hipStream_t)s;
    drop_graph(c);
    return DDGS_OK;
}

ddgs_status ddgs_set_options(ddgs_ctx *c, const ddgs_options *o)
{
    if (!c || !o) return fail(c, DDGS_ERR_INVALID_ARG, "null argument");
    DDGS_TRY(validate_options(c, *o));
    const bool tiles_changed = o->tile_w != c->opt.tile_w || o->tile_h != c->opt.tile_h;
    c->opt = *o;
    if (tiles_changed) c->views_dirty = true;
    ++c->opt_gen;
    drop_graph(c);
    return DDGS_OK;
}

ddgs_status ddgs_get_options(const ddgs_ctx *c, ddgs_options *o)
{
    if (!c || !o) return DDGS_ERR_INVALID_ARG;
    *o = c->opt;
    return DDGS_OK;
}

ddgs_status ddgs_set_model(ddgs_ctx *c, const ddgs_model *m)
{
    if (!c || !m) return fail(c, DDGS_ERR_INVALID_ARG, "null argument");
    if (m->n < 0 || m->n_iso < 0 || m->n_iso > m->n) return fail(c, DDGS_ERR_INVALID_ARG, "need 0 <= n_iso <= n");
    if (m->n >= ((int64_t)1 << 31)) return fail(c, DDGS_ERR_INVALID_ARG, "n too large");
    if (m->k < 1 || m->k > kMaxK) return fail(c, DDGS_ERR_INVALID_ARG, "k must be in 1..32");
    if (m->L < 1 || m->L > 3) return fail(c, DDGS_ERR_UNSUPPORTED, "L must be in 1..3");
    if (m->reserved != 0) return fail(c, DDGS_ERR_INVALID_ARG, "reserved must be 0");
    if (m->radiosity != DDGS_RADIOSITY_DISENTANGLED && m->radiosity != DDGS_RADIOSITY_ENTANGLED)
        return fail(c, DDGS_ERR_INVALID_ARG, "unknown radiosity form");
    if (m->radiosity == DDGS_RADIOSITY_ENTANGLED && m->n_iso != 0)
        return fail(c, DDGS_ERR_INVALID_ARG, "an entangled model has no separate isotropic set (n_iso must be 0)");
    if (m->n > 0 && (!m->mean || !m->quat || !m->log_scale || !m->opacity_logit || !m->feat))
        return fail(c, DDGS_ERR_INVALID_ARG, "null Gaussian array");
    if (!m->b_iso || !m->B_dir) return fail(c, DDGS_ERR_INVALID_ARG, "null basis array");
    const void *ptrs[] = {m->mean, m->quat, m->log_scale, m->opacity_logit, m->feat, m->b_iso, m->B_dir};
    for (const void *p : ptrs)
        if (((uintptr_t)p) % 4 != 0) return fail(c, DDGS_ERR_INVALID_ARG, "arrays must be 4-byte aligned");
    const bool shape_changed = !c->has_model || c->model.n != m->n || c->model.n_iso != m->n_iso ||
                               c->model.k != m->k || c->model.L != m->L || c->model.radiosity != m->radiosity;
    const bool ptr_changed = !c->has_model || std::memcmp(&c->model, m, sizeof(*m)) != 0;
    // the fitting moments survive only the model a densification produced
    const bool adopt = c->fit_live && c->fit_pending_n == m->n && c->fit_pending_iso == m->n_iso &&
                       c->has_model && c->model.k == m->k && c->model.L == m->L;
    if (!adopt) {
        c->fit_reset = true;
        c->fit_live = false;
    }
    c->fit_pending_n = c->fit_pending_iso = -1;
    c->plan_ok = false;
    c->model = *m;
    c->has_model = true;
    ++c->model_gen;
    if (shape_changed || ptr_changed) drop_graph(c);
    return DDGS_OK;
}

ddgs_status ddgs_set_workspace(ddgs_ctx *c, void *dev, size_t bytes)
{
    if (!c) return DDGS_ERR_INVALID_ARG;
    if (dev && (((uintptr_t)dev) % kWsAlign != 0 || bytes == 0))
        return fail(c, DDGS_ERR_INVALID_ARG, "workspace must be non-empty and 256-byte aligned");
    HIP_TRY(c, hipSetDevice(c->device));
    drop_graph(c);
    release_buffers(c);
    c->ws_base = (char *)dev;
    c->ws_size = dev ? bytes : 0;
    c->ws_used = 0;
    // everything lived in the released buffers
    c->views_dirty = true;
    c->entry_cap = 0;
    c->rendered = false;
    c->queue = nullptr;
    return DDGS_OK;
}

ddgs_status ddgs_workspace_size(ddgs_ctx *c, int64_t capacity, size_t *bytes)
{
    if (!c || !bytes) return DDGS_ERR_INVALID_ARG;
    DDGS_TRY(check_ready(c));
    int64_t cap = capacity > 0 ? capacity : (c->opt.capacity > 0 ? c->opt.capacity : std::max<int64_t>(c->entry_cap, c->M));
    if (cap <= 0) return fail(c, DDGS_ERR_STATE, "no entry capacity known: pass one, set options.capacity or render once");
    c->dry_run = true;
    c->dry_total = 0;
    const int V = (int)c->views_h.size();
    void *p;
    ddgs_status st = ensure(c, "views", views_bytes(V), &p);
    if (st == DDGS_OK) st = ensure_static(c);
    if (st == DDGS_OK) st = ensure_entries(c, cap);
    c->dry_run = false;
    if (st != DDGS_OK) return st;
    *bytes = c->dry_total;
    return DDGS_OK;
}

ddgs_status ddgs_set_pose_optimizer(ddgs_ctx *c, const ddgs_adam *a)
{
    if (!c) return DDGS_ERR_INVALID_ARG;
    if (a) {
        const bool ok = a->lr_trans >= 0.0f && a->lr_rot >= 0.0f && a->beta1 >= 0.0f && a->beta1 < 1.0f &&
                        a->beta2 >= 0.0f && a->beta2 < 1.0f && a->eps > 0.0f && std::isfinite(a->lr_trans) &&
                        std::isfinite(a->lr_rot) && std::isfinite(a->eps) &&
                        (a->pivot_mode == DDGS_PIVOT_SOURCE || a->pivot_mode == DDGS_PIVOT_POINT) &&
                        std::isfinite(a->pivot[0]) && std::isfinite(a->pivot[1]) && std::isfinite(a->pivot[2]);
        if (!ok)
            return fail(c, DDGS_ERR_INVALID_ARG,
                        "need lr >= 0, 0 <= beta < 1, eps > 0, a known pivot mode and a finite pivot");
        c->adam = AdamCfg{a->lr_trans, a->lr_rot, a->beta1, a->beta2, a->eps, a->pivot_mode,
                          {a->pivot[0], a->pivot[1], a->pivot[2]}};
    }
    c->adam_on = a != nullptr;
    c->adam_reset = true;
    drop_graph(c);
    return DDGS_OK;
}

ddgs_status ddgs_get_views(ddgs_ctx *c, ddgs_view *out, int nv)
{
    if (!c || (nv > 0 && !out)) return DDGS_ERR_INVALID_ARG;
    if (nv != (int)c->views_h.size()) return fail(c, DDGS_ERR_INVALID_ARG, "n_views differs from the views set");
    HIP_TRY(c, hipSetDevice(c->device));
    if (nv == 0) return DDGS_OK;
    if (!c->views_dirty && buf<ViewDev>(c, "views")) {
        std::vector<ViewDev> d(nv);
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        HIP_TRY(c, hipMemcpy(d.data(), buf<ViewDev>(c, "views"), sizeof(ViewDev) * nv, hipMemcpyDeviceToHost));
        for (int v = 0; v < nv; ++v) {
            ddgs_view &h = c->views_h[v];
            for (int r = 0; r < 3; ++r) {
                for (int q = 0; q < 3; ++q) h.pose[4 * r + q] = d[v].R[3 * r + q];
                h.pose[4 * r + 3] = d[v].t[r];
            }
            c->vdev_h[v] = d[v];
        }
    }
    std::copy(c->views_h.begin(), c->views_h.end(), out);
    return DDGS_OK;
}

void ddgs_default_fit_options(ddgs_fit_opts *o, float extent)
{
    if (!o) return;
    *o = ddgs_fit_opts{};
    o->lr_mean_init = 1.6e-4f * extent;
    o->lr_mean_final = 1.6e-6f * extent;
    o->lr_mean_steps = 30000;
    o->lr_quat = 1e-3f;
    o->lr_log_scale = 5e-3f;
    o->lr_opacity = 5e-2f;
    o->lr_feat = 2.5e-3f;
    o->lr_b_iso = 1.25e-4f;
    o->lr_B_dir = 1.25e-4f;
    o->beta1 = 0.9f;
    o->beta2 = 0.999f;
    o->eps = 1e-15f;
}

ddgs_status ddgs_set_fit_optimizer(ddgs_ctx *c, const ddgs_fit_opts *o)
{
    if (!c) return DDGS_ERR_INVALID_ARG;
    if (o) {
        const float rates[] = {o->lr_mean_init, o->lr_mean_final, o->lr_quat, o->lr_log_scale, o->lr_opacity,
                               o->lr_feat, o->lr_b_iso, o->lr_B_dir};
        bool ok = o->lr_mean_steps >= 1 && o->beta1 >= 0.0f && o->beta1 < 1.0f && o->beta2 >= 0.0f &&
                  o->beta2 < 1.0f && o->eps > 0.0f && std::isfinite(o->eps) && o->lr_mean_init > 0.0f &&
                  o->lr_mean_final > 0.0f;
        for (float r : rates) ok = ok && r >= 0.0f && std::isfinite(r);
        if (!ok)
            return fail(c, DDGS_ERR_INVALID_ARG,
                        "need finite rates >= 0 (position rates > 0), steps >= 1, 0 <= beta < 1, eps > 0");
        FitCfg f{};
        f.lr_mean0 = o->lr_mean_init;
        f.lr_mean1 = o->lr_mean_final;
        f.lr_steps = o->lr_mean_steps;
        const float lr[kGroups] = {0.0f, o->lr_quat, o->lr_log_scale, o->lr_opacity, o->lr_feat, o->lr_b_iso, o->lr_B_dir};
        for (int g = 0; g < kGroups; ++g) f.lr[g] = lr[g];
        f.beta1 = o->beta1;
        f.beta2 = o->beta2;
        f.eps = o->eps;
        c->fit = f;
    }
    c->fit_on = o != nullptr;
    c->fit_reset = true;
    c->fit_live = false;
    drop_graph(c);
    return DDGS_OK;
}

ddgs_status ddgs_set_densify_stats(ddgs_ctx *c, float *grad_accum, float *count, float *max_radius)
{
    if (!c) return DDGS_ERR_INVALID_ARG;
    const bool any = grad_accum || count || max_radius;
    if (any && !(grad_accum && count && max_radius))
        return fail(c, DDGS_ERR_INVALID_ARG, "pass all three statistics arrays or none");
    c->st_grad = grad_accum;
    c->st_cnt = count;
    c->st_rad = max_radius;
    c->plan_ok = false;
    drop_graph(c);
    return DDGS_OK;
}

ddgs_status ddgs_densify_plan(ddgs_ctx *c, const ddgs_densify_opts *o, const float *noise, int64_t *n_new,
                              int64_t *n_iso_new)
{
    if (!c || !o || !n_new || !n_iso_new) return DDGS_ERR_INVALID_ARG;
    if (!c->has_model) return fail(c, DDGS_ERR_STATE, "no model");
    if (!c->st_grad) return fail(c, DDGS_ERR_STATE, "no densification statistics (ddgs_set_densify_stats)");
    const int n = (int)c->model.n, n_iso = (int)c->model.n_iso;
    if (n > 0 && !noise) return fail(c, DDGS_ERR_INVALID_ARG, "null noise");
    if (!(o->grad_threshold >= 0.0f && std::isfinite(o->grad_threshold) && o->dense_scale > 0.0f &&
          std::isfinite(o->dense_scale) && o->min_opacity > 0.0f && o->min_opacity < 1.0f &&
          std::isfinite(o->max_world_scale) && std::isfinite(o->max_screen_radius) && o->split_factor > 1.0f &&
          std::isfinite(o->split_factor)))
        return fail(c, DDGS_ERR_INVALID_ARG,
                    "need grad_threshold >= 0, dense_scale > 0, 0 < min_opacity < 1, split_factor > 1, finite bounds");
    if (c->model.radiosity == DDGS_RADIOSITY_ENTANGLED && n_iso != 0)
        return fail(c, DDGS_ERR_STATE, "entangled model with an isotropic set");
    HIP_TRY(c, hipSetDevice(c->device));
    const float inf = std::numeric_limits<float>::infinity();
    DensifyTh th;
    th.grad = o->grad_threshold;
    th.log_dense = (float)std::log((double)o->dense_scale);
    th.logit_min_op = (float)(std::log((double)o->min_opacity) - std::log1p(-(double)o->min_opacity));
    th.log_world = o->max_world_scale > 0.0f ? (float)std::log((double)o->max_world_scale) : inf;
    th.screen = o->max_screen_radius > 0.0f ? o->max_screen_radius : inf;
    th.log_split = (float)std::log((double)o->split_factor);
    uint32_t *keep, *clone, *child, *keep_ex, *clone_ex, *child_ex;
    uint64_t *tot;
    const size_t nn = (size_t)std::max(n, 1);
    DDGS_TRY(ensure_t(c, "dn_keep", nn, &keep));
    DDGS_TRY(ensure_t(c, "dn_clone", nn, &clone));
    DDGS_TRY(ensure_t(c, "dn_child", nn, &child));
    DDGS_TRY(ensure_t(c, "dn_keep_ex", nn, &keep_ex));
    DDGS_TRY(ensure_t(c, "dn_clone_ex", nn, &clone_ex));
    DDGS_TRY(ensure_t(c, "dn_child_ex", nn, &child_ex));
    DDGS_TRY(ensure_t(c, "dn_tot", 4, &tot));
    SortWs ws;
    DDGS_TRY(aux_sort_ws(c, n, &ws));
    hipStream_t s = c->stream;
    HIP_TRY(c, launch_densify_plan(n, c->model.log_scale, c->model.opacity_logit, c->st_grad, c->st_cnt, c->st_rad,
                                   th, keep, clone, child, s));
    HIP_TRY(c, launch_exclusive_scan(keep, nullptr, keep_ex, n, ws, tot, s));
    HIP_TRY(c, launch_exclusive_scan(clone, nullptr, clone_ex, n, ws, tot + 1, s));
    HIP_TRY(c, launch_exclusive_scan(child, nullptr, child_ex, n, ws, tot + 2, s));
    uint64_t t_h[3] = {0, 0, 0};
    uint32_t at_iso[3] = {0, 0, 0};
    HIP_TRY(c, hipMemcpyAsync(t_h, tot, sizeof(t_h), hipMemcpyDeviceToHost, s));
    if (n_iso < n) {
        HIP_TRY(c, hipMemcpyAsync(&at_iso[0], keep_ex + n_iso, 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(c, hipMemcpyAsync(&at_iso[1], clone_ex + n_iso, 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(c, hipMemcpyAsync(&at_iso[2], child_ex + n_iso, 4, hipMemcpyDeviceToHost, s));
    }
    HIP_TRY(c, hipStreamSynchronize(s));
    if (n_iso == n)
        for (int q = 0; q < 3; ++q) at_iso[q] = (uint32_t)t_h[q];
    const int64_t total = (int64_t)(t_h[0] + t_h[1] + t_h[2]);
    if (total >= ((int64_t)1 << 31)) return fail(c, DDGS_ERR_UNSUPPORTED, "densified model too large");
    c->plan_pref[0] = at_iso[0];
    c->plan_pref[1] = at_iso[1];
    c->plan_pref[2] = at_iso[2];
    c->plan_pref[3] = (uint32_t)t_h[0];
    c->plan_pref[4] = (uint32_t)t_h[1];
    c->plan_n_new = total;
    c->plan_iso_new = (int64_t)at_iso[0] + at_iso[1] + at_iso[2];
    c->plan_noise = noise;
    c->plan_log_split = th.log_split;
    c->plan_model_gen = c->model_gen;
    c->plan_ok = true;
    *n_new = c->plan_n_new;
    *n_iso_new = c->plan_iso_new;
    return DDGS_OK;
}

ddgs_status ddgs_densify_apply(ddgs_ctx *c, const ddgs_params *out)
{
    if (!c || !out) return DDGS_ERR_INVALID_ARG;
    if (!c->plan_ok || c->plan_model_gen != c->model_gen)
        return fail(c, DDGS_ERR_STATE, "ddgs_densify_apply needs a ddgs_densify_plan of the current model");
    float *dst[kGroups] = {out->mean, out->quat, out->log_scale, out->opacity_logit, out->feat, out->b_iso, out->B_dir};
    for (int g = 0; g < kGroups; ++g) {
        if (!dst[g] && (g >= 5 || c->plan_n_new > 0)) return fail(c, DDGS_ERR_INVALID_ARG, "null output array");
        if (((uintptr_t)dst[g]) % 4 != 0) return fail(c, DDGS_ERR_INVALID_ARG, "arrays must be 4-byte aligned");
    }
    HIP_TRY(c, hipSetDevice(c->device));
    drop_graph(c);
    const ddgs_model &m = c->model;
    const int kl = kl_of(m.L);
    DensifyApplyArgs a{};
    a.n = (int)m.n;
    a.n_iso = (int)m.n_iso;
    a.k = m.k;
    a.kl = kl;
    a.n_new = c->plan_n_new;
    const float *src[5] = {m.mean, m.quat, m.log_scale, m.opacity_logit, m.feat};
    for (int g = 0; g < 5; ++g) {
        a.src[g] = src[g];
        a.dst[g] = dst[g];
    }
    a.keep = buf<uint32_t>(c, "dn_keep");
    a.clone = buf<uint32_t>(c, "dn_clone");
    a.child = buf<uint32_t>(c, "dn_child");
    a.keep_ex = buf<uint32_t>(c, "dn_keep_ex");
    a.clone_ex = buf<uint32_t>(c, "dn_clone_ex");
    a.child_ex = buf<uint32_t>(c, "dn_child_ex");
    a.k_iso = c->plan_pref[0];
    a.c_iso = c->plan_pref[1];
    a.h_iso = c->plan_pref[2];
    a.k_tot = c->plan_pref[3];
    a.c_tot = c->plan_pref[4];
    a.noise = c->plan_noise;
    a.log_split = c->plan_log_split;
    const bool moments = c->fit_live && buf<float>(c, "fit_mv") != nullptr;
    if (moments) {
        const int64_t P_old = fit_param_count(m.n, m.k, kl), P_new = fit_param_count(c->plan_n_new, m.k, kl);
        float *mv2;
        DDGS_TRY(ensure_t(c, "fit_mv_next", (size_t)2 * P_new, &mv2));
        a.m_old = buf<float>(c, "fit_mv");
        a.v_old = a.m_old + P_old;
        a.m_new = mv2;
        a.v_new = mv2 + P_new;
    }
    HIP_TRY(c, launch_densify_apply(a, c->stream));
    const size_t nb = sizeof(float) * m.k, nB = sizeof(float) * kl * m.k;
    if (out->b_iso != m.b_iso) HIP_TRY(c, hipMemcpyAsync(out->b_iso, m.b_iso, nb, hipMemcpyDeviceToDevice, c->stream));
    if (out->B_dir != m.B_dir) HIP_TRY(c, hipMemcpyAsync(out->B_dir, m.B_dir, nB, hipMemcpyDeviceToDevice, c->stream));
    if (moments) {
        std::swap(c->bufs["fit_mv"], c->bufs["fit_mv_next"]);
        c->fit_pending_n = c->plan_n_new;
        c->fit_pending_iso = c->plan_iso_new;
    }
    c->plan_ok = false;
    return DDGS_OK;
}

ddgs_status ddgs_fit_reset_opacity(ddgs_ctx *c, float max_alpha)
{
    if (!c) return DDGS_ERR_INVALID_ARG;
    if (!c->has_model) return fail(c, DDGS_ERR_STATE, "no model");
    if (!(max_alpha > 0.0f && max_alpha < 1.0f)) return fail(c, DDGS_ERR_INVALID_ARG, "need 0 < max_alpha < 1");
    HIP_TRY(c, hipSetDevice(c->device));
    const float cap = (float)(std::log((double)max_alpha) - std::log1p(-(double)max_alpha));
    float *p[kGroups];
    fit_groups(c, p);
    float *mm = nullptr, *vv = nullptr;
    if (c->fit_live && buf<float>(c, "fit_mv")) {
        int64_t off[kGroups + 1];
        fit_offsets(c->model.n, c->model.k, kl_of(c->model.L), off);
        mm = buf<float>(c, "fit_mv") + off[3];
        vv = buf<float>(c, "fit_mv") + off[kGroups] + off[3];
    }
    HIP_TRY(c, launch_opacity_reset(p[3], (int)c->model.n, cap, mm, vv, c->stream));
    return DDGS_OK;
}

ddgs_status ddgs_rads_prepare(ddgs_ctx *c, const ddgs_volume *vol, float *level, int64_t *n_crossings,
                              uint64_t *total_weight)
{
    if (!c || !vol || !level || !n_crossings || !total_weight) return DDGS_ERR_INVALID_ARG;
    c->rads_ok = false;
    const int64_t n = (int64_t)vol->nx * vol->ny * vol->nz;
    if (vol->nx < 1 || vol->ny < 1 || vol->nz < 1 || n >= ((int64_t)1 << 30))
        return fail(c, DDGS_ERR_INVALID_ARG, "need 1 <= nx, ny, nz and nx ny nz < 2^30");
    for (int a = 0; a < 3; ++a)
        if (!(vol->spacing[a] > 0.0f) || !std::isfinite(vol->spacing[a]) || !std::isfinite(vol->origin[a]))
            return fail(c, DDGS_ERR_INVALID_ARG, "need finite spacing > 0 and a finite origin");
    if (!vol->hu || ((uintptr_t)vol->hu) % 4 != 0) return fail(c, DDGS_ERR_INVALID_ARG, "null or unaligned volume");
    HIP_TRY(c, hipSetDevice(c->device));
    hipStream_t s = c->stream;
    RadsVol v{vol->nx, vol->ny, vol->nz, vol->spacing[0], vol->spacing[1], vol->spacing[2],
              vol->origin[0], vol->origin[1], vol->origin[2], vol->hu};
    const int64_t nb = rads_minmax_blocks(n, c->num_cu), nb64 = rads_scan64_blocks(n);
    float2 *part;
    float *mm;
    uint32_t *cnt, *off;
    uint64_t *tot, *bsum, *cdf;
    DDGS_TRY(ensure_t(c, "rads_part", (size_t)nb, &part));
    DDGS_TRY(ensure_t(c, "rads_mm", 4, &mm));
    DDGS_TRY(ensure_t(c, "rads_cnt", (size_t)n, &cnt));
    DDGS_TRY(ensure_t(c, "rads_off", (size_t)n, &off));
    DDGS_TRY(ensure_t(c, "rads_tot", 1, &tot));
    DDGS_TRY(ensure_t(c, "rads_bsum", (size_t)nb64 + 1, &bsum));
    DDGS_TRY(ensure_t(c, "rads_cdf", (size_t)n, &cdf));
    SortWs ws;
    DDGS_TRY(aux_sort_ws(c, n, &ws));
    HIP_TRY(c, launch_rads_level(v, part, nb, mm, s));
    HIP_TRY(c, launch_mc_count(v, mm, cnt, s));
    HIP_TRY(c, launch_exclusive_scan(cnt, nullptr, off, n, ws, tot, s));
    HIP_TRY(c, launch_rads_cdf(v, mm, bsum, cdf, s));
    uint64_t m_h = 0, w_h = 0;
    float mm_h[3] = {0.0f, 0.0f, 0.0f};
    HIP_TRY(c, hipMemcpyAsync(&m_h, tot, 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipMemcpyAsync(&w_h, bsum + nb64, 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipMemcpyAsync(mm_h, mm, sizeof(mm_h), hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    float *pts;
    DDGS_TRY(ensure_t(c, "rads_pts", (size_t)std::max<uint64_t>(3 * m_h, 1), &pts));
    HIP_TRY(c, launch_mc_emit(v, mm, off, pts, (int64_t)m_h, s));
    v.hu = nullptr;  // not read after this call
    c->rads_vol = v;
    c->rads_m = (int64_t)m_h;
    c->rads_w = w_h;
    c->rads_ok = true;
    *level = mm_h[2];
    *n_crossings = (int64_t)m_h;
    *total_weight = w_h;
    return DDGS_OK;
}

ddgs_status ddgs_rads_sample(ddgs_ctx *c, int64_t n1, const uint32_t *mc_keys, int64_t n2, const uint64_t *dw_draws,
                             float *points, float *log_scale, int64_t *n_iso)
{
    if (!c || !n_iso) return DDGS_ERR_INVALID_ARG;
    if (!c->rads_ok) return fail(c, DDGS_ERR_STATE, "ddgs_rads_sample needs ddgs_rads_prepare");
    if (n1 < 0 || n2 < 0) return fail(c, DDGS_ERR_INVALID_ARG, "need n1, n2 >= 0");
    const int64_t M = c->rads_m, n1e = std::min(n1, M), N = n1e + n2;
    if (N >= ((int64_t)1 << 31)) return fail(c, DDGS_ERR_INVALID_ARG, "too many points");
    if (N > 0 && !points) return fail(c, DDGS_ERR_INVALID_ARG, "null points");
    if (n1e > 0 && !mc_keys) return fail(c, DDGS_ERR_INVALID_ARG, "null mc_keys");
    if (n2 > 0 && !dw_draws) return fail(c, DDGS_ERR_INVALID_ARG, "null dw_draws");
    if (n2 > 0 && c->rads_w == 0) return fail(c, DDGS_ERR_STATE, "the volume has no weight (constant radiodensity)");
    HIP_TRY(c, hipSetDevice(c->device));
    hipStream_t s = c->stream;
    if (n1e > 0) {
        uint32_t *k0, *k1, *v0, *v1;
        DDGS_TRY(ensure_t(c, "rads_k0", (size_t)M, &k0));
        DDGS_TRY(ensure_t(c, "rads_k1", (size_t)M, &k1));
        DDGS_TRY(ensure_t(c, "rads_v0", (size_t)M, &v0));
        DDGS_TRY(ensure_t(c, "rads_v1", (size_t)M, &v1));
        SortWs ws;
        DDGS_TRY(aux_sort_ws(c, M, &ws));
        HIP_TRY(c, hipMemcpyAsync(k0, mc_keys, sizeof(uint32_t) * M, hipMemcpyDeviceToDevice, s));
        HIP_TRY(c, launch_iota(v0, M, s));
        bool in_k1 = false;
        HIP_TRY(c, radix_sort_pairs(k0, v0, k1, v1, M, nullptr, 32, ws, &in_k1, s));
        HIP_TRY(c, launch_rads_gather(buf<float>(c, "rads_pts"), M, in_k1 ? v1 : v0, n1e, points, N, s));
    }
    HIP_TRY(c, launch_rads_draws(c->rads_vol, buf<uint64_t>(c, "rads_cdf"), dw_draws, n2, points, N, n1e, s));
    if (log_scale) HIP_TRY(c, launch_knn3(points, N, log_scale, s));
    *n_iso = n1e + n2 / 2;
    return DDGS_OK;
}

ddgs_status ddgs_set_radiosity_override(ddgs_ctx *c, const float *cv)
{
    if (!c) return DDGS_ERR_INVALID_ARG;
    if (((uintptr_t)cv) % 4 != 0) return fail(c, DDGS_ERR_INVALID_ARG, "arrays must be 4-byte aligned");
    if (cv != c->c_override) {
        c->c_override = cv;
        ++c->model_gen;
        drop_graph(c);
    }
    return DDGS_OK;
}

ddgs_status ddgs_set_views(ddgs_ctx *c, const ddgs_view *v, int nv)
{
    if (!c || (nv > 0 && !v) || nv < 0) return fail(c, DDGS_ERR_INVALID_ARG, "bad views");
    for (int i = 0; i < nv; ++i) {
        if (v[i].W < 1 || v[i].H < 1 || v[i].W > 16384 || v[i].H > 16384)
            return fail(c, DDGS_ERR_INVALID_ARG, "detector size must be in 1..16384");
        if (!(v[i].pitch_mm > 0.0f) || !(v[i].sdd_mm > 0.0f))
            return fail(c, DDGS_ERR_INVALID_ARG, "pitch and sdd must be > 0");
        for (int q = 0; q < 12; ++q)
            if (!std::isfinite(v[i].pose[q])) return fail(c, DDGS_ERR_NONFINITE, "non-finite pose");
        if (!std::isfinite(v[i].pitch_mm) || !std::isfinite(v[i].sdd_mm))
            return fail(c, DDGS_ERR_NONFINITE, "non-finite intrinsics");
    }
    bool same_shape = (int)c->views_h.size() == nv;
    for (int i = 0; same_shape && i < nv; ++i)
        same_shape = c->views_h[i].W == v[i].W && c->views_h[i].H == v[i].H;
    c->views_h.assign(v, v + nv);
    c->views_dirty = true;
    c->adam_reset = true;
    ++c->views_gen;
    if (!same_shape) drop_graph(c);
    if (c->exec) {
        // same shapes: refresh the device table in place for the captured graph
        DDGS_TRY(prepare_views(c));
    }
    return DDGS_OK;
}

ddgs_status ddgs_image_size(const ddgs_ctx *c, int64_t *nf)
{
    if (!c || !nf) return DDGS_ERR_INVALID_ARG;
    int64_t s = 0;
    for (const auto &v : c->views_h) s += (int64_t)v.W * v.H;
    *nf = s;
    return DDGS_OK;
}

ddgs_status ddgs_render(ddgs_ctx *c, float *images)
{
    if (!c) return DDGS_ERR_INVALID_ARG;
    if (!images) return fail(c, DDGS_ERR_INVALID_ARG, "null images");
    HIP_TRY(c, hipSetDevice(c->device));
    DDGS_TRY(check_ready(c));
    c->rendered = false;
    DDGS_TRY(ensure_static(c));
    DDGS_TRY(ensure_entries(c, std::max<int64_t>(c->entry_cap, 1)));
    const int64_t VN = c->model.n * (int64_t)c->views_h.size();
    if (VN > 0) {
        DDGS_TRY(enqueue_front(c, 0xFFFFFFFFu, false));
        // entry total ([0..1]) and number of long tiles ([12])
        uint32_t sc[13] = {};
        HIP_TRY(c, hipMemcpyAsync(sc, total_ptr(c), sizeof(sc), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        const uint64_t total = (uint64_t)sc[0] | ((uint64_t)sc[1] << 32);
        const int64_t n_long = sc[12];
        if (c->long_seen_n != c->model.n || c->long_seen_tiles != c->n_tiles) c->long_seen = -1;
        c->long_seen = std::max(c->long_seen, n_long);
        c->long_seen_n = c->model.n;
        c->long_seen_tiles = c->n_tiles;
        c->long_grid = (int)std::min<int64_t>(n_long, 1 << 30);
        ddgs_status st = DDGS_OK;
        if (total >= 0xFFFFFFFFull) st = fail(c, DDGS_ERR_CAPACITY, "more than 2^32-1 tile entries");
        c->M = (int64_t)total;
        if (st == DDGS_OK && c->M > c->entry_cap) st = ensure_entries(c, c->M);
        if (st != DDGS_OK) return st;
        // (the exact total bounds the work items, so the raster grids take
        // no more workgroups than this render can fill; the buffers keep
        // entry_cap)
        DDGS_TRY(enqueue_back(c, std::max<int64_t>(c->M, 1), images));
    } else {
        // no Gaussians: empty lists everywhere
        c->M = 0;
        HIP_TRY(c, launch_zero_u64(total_ptr(c), c->stream));
        HIP_TRY(c, launch_fill_u32(mdev_ptr(c), 0u, 1, c->stream));
        HIP_TRY(c, launch_ranges(nullptr, mdev_ptr(c), 0, buf<uint2>(c, "ranges"), c->n_tiles, true, c->stream));
        c->queue = nullptr;
        RasterArgs ra{};
        ra.views = buf<ViewDev>(c, "views");
        ra.V = (int)c->views_h.size();
        ra.n = 1;
        ra.o = render_opts(c->opt);
        ra.ranges = buf<uint2>(c, "ranges");
        ra.tval = buf<uint32_t>(c, "tval");
        ra.rec = buf<float4>(c, "rec");
        ra.n_tiles = c->n_tiles;
        ra.img = images;
        ra.img_saved = buf<float>(c, "img_saved");
        ra.nlast = buf<uint32_t>(c, "nlast");
        HIP_TRY(c, launch_raster_fwd(ra, c->num_cu, c->stream));
    }
    c->rendered = true;
    c->r_model_gen = c->model_gen;
    c->r_views_gen = c->views_gen;
    c->r_opt_gen = c->opt_gen;
    return DDGS_OK;
}

ddgs_status ddgs_backward(ddgs_ctx *c, const float *dL, const ddgs_grads *g)
{
    if (!c) return DDGS_ERR_INVALID_ARG;
    if (!dL || !g) return fail(c, DDGS_ERR_INVALID_ARG, "null argument");
    if (!is_state_current(c)) return fail(c, DDGS_ERR_STATE, "backward needs a render with the current model, views and options");
    HIP_TRY(c, hipSetDevice(c->device));
    if (c->model.n == 0) {
        // nothing depends on any parameter: zero outputs
        if (g->db_iso) HIP_TRY(c, launch_fill_u32((uint32_t *)g->db_iso, 0u, c->model.k, c->stream));
        if (g->dB_dir) HIP_TRY(c, launch_fill_u32((uint32_t *)g->dB_dir, 0u, (int64_t)kl_of(c->model.L) * c->model.k, c->stream));
        if (g->dpose) HIP_TRY(c, launch_fill_u32((uint32_t *)g->dpose, 0u, 6 * (int64_t)c->views_h.size(), c->stream));
        return DDGS_OK;
    }
    DDGS_TRY(enqueue_backward(c, dL, g, c->entry_cap, false));
    return DDGS_OK;
}

ddgs_status ddgs_loss(ddgs_ctx *c, int kind, const float *images, const float *target, float lambda,
                      float *loss_out, float *dL)
{
    if (!c) return DDGS_ERR_INVALID_ARG;
    if (!images || !target) return fail(c, DDGS_ERR_INVALID_ARG, "null images or target");
    if (kind < 0 || kind > 2) return fail(c, DDGS_ERR_INVALID_ARG, "unknown loss kind");
    if (!(lambda >= 0.0f && lambda <= 1.0f)) return fail(c, DDGS_ERR_INVALID_ARG, "lambda must be in [0, 1]");
    HIP_TRY(c, hipSetDevice(c->device));
    DDGS_TRY(check_ready(c));
    DDGS_TRY(ensure_static(c));
    DDGS_TRY(enqueue_loss(c, kind, images, target, lambda, loss_out, dL));
    return DDGS_OK;
}

ddgs_status ddgs_step_capture(ddgs_ctx *c, int kind, const float *target, float lambda, float *images, float *dL,
                              float *loss_out, const ddgs_grads *g)
{
    if (!c) return DDGS_ERR_INVALID_ARG;
    if (!images || !dL || !g || !target) return fail(c, DDGS_ERR_INVALID_ARG, "null argument");
    if (kind < 0 || kind > 2) return fail(c, DDGS_ERR_INVALID_ARG, "unknown loss kind");
    HIP_TRY(c, hipSetDevice(c->device));
    DDGS_TRY(check_ready(c));
    if (c->model.n == 0) return fail(c, DDGS_ERR_UNSUPPORTED, "a captured step needs n > 0");
    if (!c->stream) return fail(c, DDGS_ERR_INVALID_ARG, "capture needs a non-default stream");
    if (c->adam_on && !g->dpose) return fail(c, DDGS_ERR_INVALID_ARG, "the pose optimiser needs grads->dpose");
    if (c->adam_on && c->views_h.size() > 256) return fail(c, DDGS_ERR_UNSUPPORTED, "the pose optimiser takes up to 256 views");
    if (c->fit_on && !(g->dmean && g->dquat && g->dlog_scale && g->dopacity_logit && g->dfeat && g->db_iso && g->dB_dir))
        return fail(c, DDGS_ERR_INVALID_ARG, "the fitting optimiser needs every parameter gradient");
    drop_graph(c);
    DDGS_TRY(ensure_static(c));
    c->step_target = target;
    c->views_dirty = true;
    DDGS_TRY(prepare_views(c));
    if (c->adam_on) {
        float *st_;
        uint32_t *sp_;
        // (moments restart only after ddgs_set_pose_optimizer / ddgs_set_views,
        // so a capture repeated with a larger capacity continues the run)
        const float *prev = buf<float>(c, "adam_state");
        DDGS_TRY(ensure_t(c, "adam_state", (size_t)12 * c->views_h.size(), &st_));
        DDGS_TRY(ensure_t(c, "adam_step", 1, &sp_));
        if (st_ != prev) c->adam_reset = true;
    }
    if (c->fit_on) {
        float *mv_;
        uint32_t *fs_;
        const int64_t P = fit_param_count(c->model.n, c->model.k, kl_of(c->model.L));
        const bool had = buf<float>(c, "fit_mv") != nullptr;
        DDGS_TRY(ensure_t(c, "fit_mv", (size_t)2 * P, &mv_));
        DDGS_TRY(ensure_t(c, "fit_step", 1, &fs_));
        if (!had || !c->fit_live) c->fit_reset = true;
    }
    int64_t cap = c->opt.capacity;
    if (cap <= 0) {
        // one plain render sizes the capacity: twice the current need
        float *tmp_img;
        DDGS_TRY(ensure_t(c, "capture_probe_img", c->total_pix, &tmp_img));
        DDGS_TRY(ddgs_render(c, tmp_img));
        cap = std::max<int64_t>(2 * c->M, 1024);
    }
    cap = std::min<int64_t>(cap, 0xFFFFFFF0ll);
    DDGS_TRY(ensure_entries(c, cap));
    c->step_cap = cap;
    const bool saved_timing = c->timing;
    c->timing = false;
    HIP_TRY(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    c->long_grid = captured_long_grid(c);
    ddgs_status st = enqueue_front(c, (uint32_t)c->step_cap, true);
    if (st == DDGS_OK) st = enqueue_back(c, c->step_cap, images);
    if (st == DDGS_OK) st = enqueue_loss(c, kind, images, target, lambda, loss_out, dL, true);
    if (st == DDGS_OK) st = enqueue_backward(c, dL, g, c->step_cap, true);
    if (st == DDGS_OK && c->adam_on) {
        hipError_t ea = launch_pose_adam(buf<ViewDev>(c, "views"), (int)c->views_h.size(), g->dpose,
                                         buf<float>(c, "adam_state"), buf<uint32_t>(c, "adam_step"), c->adam,
                                         flags_ptr(c), c->stream);
        if (ea != hipSuccess) st = fail(c, DDGS_ERR_HIP, std::string("pose optimiser: ") + hipGetErrorString(ea));
    }
    if (st == DDGS_OK && c->fit_on) {
        FitArgs fa{};
        const float *gs[kGroups] = {g->dmean, g->dquat, g->dlog_scale, g->dopacity_logit, g->dfeat, g->db_iso, g->dB_dir};
        fit_groups(c, fa.p);
        for (int q = 0; q < kGroups; ++q) fa.g[q] = gs[q];
        fit_offsets(c->model.n, c->model.k, kl_of(c->model.L), fa.off);
        fa.m = buf<float>(c, "fit_mv");
        fa.v = fa.m + fa.off[kGroups];
        fa.step = buf<uint32_t>(c, "fit_step");
        fa.skip = flags_ptr(c);
        fa.cfg = c->fit;
        hipError_t ea = launch_fit_adam(fa, c->num_cu, c->stream);
        if (ea != hipSuccess) st = fail(c, DDGS_ERR_HIP, std::string("fitting optimiser: ") + hipGetErrorString(ea));
    }
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(c->stream, &graph);
    c->timing = saved_timing;
    if (st != DDGS_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (e != hipSuccess) return fail(c, DDGS_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    c->graph = graph;
    e = hipGraphInstantiate(&c->exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        drop_graph(c);
        return fail(c, DDGS_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    c->rendered = false;
    return DDGS_OK;
}

ddgs_status ddgs_step_launch(ddgs_ctx *c)
{
    if (!c) return DDGS_ERR_INVALID_ARG;
    if (!c->exec) return fail(c, DDGS_ERR_STATE, "no captured step");
    HIP_TRY(c, hipSetDevice(c->device));
    if (c->adam_on && c->adam_reset) {
        // fresh moments (outside the graph: no memset nodes are captured)
        HIP_TRY(c, hipMemsetAsync(buf<float>(c, "adam_state"), 0, sizeof(float) * 12 * c->views_h.size(), c->stream));
        HIP_TRY(c, hipMemsetAsync(buf<uint32_t>(c, "adam_step"), 0, sizeof(uint32_t), c->stream));
        c->adam_reset = false;
    }
    if (c->fit_on && c->fit_reset) {
        const int64_t P = fit_param_count(c->model.n, c->model.k, kl_of(c->model.L));
        HIP_TRY(c, hipMemsetAsync(buf<float>(c, "fit_mv"), 0, sizeof(float) * 2 * P, c->stream));
        HIP_TRY(c, hipMemsetAsync(buf<uint32_t>(c, "fit_step"), 0, sizeof(uint32_t), c->stream));
        c->fit_reset = false;
        c->fit_live = true;
    }
    // (a target set by ddgs_step_set_target since the last upload)
    DDGS_TRY(prepare_views(c));
    HIP_TRY(c, hipGraphLaunch(c->exec, c->stream));
    c->M = -1;  // unknown until ddgs_check
    c->rendered = true;
    c->r_model_gen = c->model_gen;
    c->r_views_gen = c->views_gen;
    c->r_opt_gen = c->opt_gen;
    return DDGS_OK;
}

ddgs_status ddgs_step_set_target(ddgs_ctx *c, const float *target)
{
    if (!c) return DDGS_ERR_INVALID_ARG;
    if (!target) return fail(c, DDGS_ERR_INVALID_ARG, "null target");
    if (((uintptr_t)target) % 4 != 0) return fail(c, DDGS_ERR_INVALID_ARG, "arrays must be 4-byte aligned");
    if (!c->exec) return fail(c, DDGS_ERR_STATE, "no captured step");
    if (target != c->step_target) {
        c->step_target = target;
        c->views_dirty = true;  // uploaded with the view table, at the latest by the next launch
    }
    return DDGS_OK;
}

ddgs_status ddgs_check(ddgs_ctx *c, uint32_t *flags)
{
    if (!c) return DDGS_ERR_INVALID_ARG;
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    uint32_t sc[12] = {};
    if (buf<uint32_t>(c, "scalars"))
        HIP_TRY(c, hipMemcpy(sc, buf<uint32_t>(c, "scalars"), sizeof(sc), hipMemcpyDeviceToHost));
    if (flags) *flags = sc[3];
    const uint64_t total = (uint64_t)sc[0] | ((uint64_t)sc[1] << 32);
    const uint64_t need = (uint64_t)sc[10] | ((uint64_t)sc[11] << 32);
    c->last_skipped = (int64_t)sc[7];
    c->last_need = (int64_t)std::max(need, total);
    // the flags and step counters accumulate over replays until read here
    if (sc[3] || sc[7] || need) {
        HIP_TRY(c, hipMemsetAsync(flags_ptr(c), 0, sizeof(uint32_t), c->stream));
        HIP_TRY(c, hipMemsetAsync(skipped_ptr(c), 0, sizeof(uint32_t), c->stream));
        HIP_TRY(c, hipMemsetAsync(need_ptr(c), 0, sizeof(uint64_t), c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
    }
    if (c->M < 0) c->M = (int64_t)std::min<uint64_t>(total, (uint64_t)c->step_cap);
    if (sc[3] & 1u)
        return fail(c, DDGS_ERR_CAPACITY, "tile entries (" + std::to_string(total) + ") exceeded the capacity (" +
                                              std::to_string(c->step_cap) + ")");
    return DDGS_OK;
}

ddgs_status ddgs_step_report(const ddgs_ctx *c, int64_t *skipped, int64_t *need)
{
    if (!c) return DDGS_ERR_INVALID_ARG;
    if (skipped) *skipped = c->last_skipped;
    if (need) *need = c->last_need;
    return DDGS_OK;
}

ddgs_status ddgs_set_allocator(ddgs_ctx *c, ddgs_alloc_fn alloc, ddgs_free_fn free_fn, void *user)
{
    if (!c) return DDGS_ERR_INVALID_ARG;
    if ((alloc == nullptr) != (free_fn == nullptr))
        return fail(c, DDGS_ERR_INVALID_ARG, "pass both allocator functions or neither");
    HIP_TRY(c, hipSetDevice(c->device));
    drop_graph(c);
    release_buffers(c);  // with the functions they came from
    c->alloc_fn = alloc;
    c->free_fn = free_fn;
    c->alloc_user = alloc ? user : nullptr;
    c->ws_base = nullptr;
    c->ws_size = c->ws_used = 0;
    c->views_dirty = true;
    c->entry_cap = 0;
    c->rendered = false;
    c->queue = nullptr;
    return DDGS_OK;
}

ddgs_status ddgs_compose_pose(const float pose[12], const double delta[6], float out[12])
{
    if (!pose || !delta || !out) return DDGS_ERR_INVALID_ARG;
    for (int q = 0; q < 6; ++q)
        if (!std::isfinite(delta[q])) return DDGS_ERR_NONFINITE;
    // Exp(omega) by Rodrigues' formula, E = I + a [w]x + b [w]x^2 with
    // a = sin(th) / th, b = (1 - cos(th)) / th^2 (series below th = 1e-4)
    const double x = delta[3], y = delta[4], z = delta[5];
    const double th2 = x * x + y * y + z * z, th = std::sqrt(th2);
    double a, b;
    if (th < 1e-4) {
        a = 1.0 - th2 / 6.0;
        b = 0.5 - th2 / 24.0;
    } else {
        a = std::sin(th) / th;
        b = (1.0 - std::cos(th)) / th2;
    }
    const double E[9] = {1.0 - b * (y * y + z * z), -a * z + b * x * y, a * y + b * x * z,
                         a * z + b * x * y, 1.0 - b * (x * x + z * z), -a * x + b * y * z,
                         -a * y + b * x * z, a * x + b * y * z, 1.0 - b * (x * x + y * y)};
    double P[12];
    for (int q = 0; q < 12; ++q) P[q] = (double)pose[q];
    for (int r = 0; r < 3; ++r) {
        double row[4];
        for (int col = 0; col < 4; ++col)
            row[col] = E[3 * r] * P[col] + E[3 * r + 1] * P[4 + col] + E[3 * r + 2] * P[8 + col];
        row[3] += delta[r];
        for (int col = 0; col < 4; ++col) out[4 * r + col] = (float)row[col];
    }
    return DDGS_OK;
}

ddgs_status ddgs_param_count(int k, int L, int64_t n, int64_t *per, int64_t *shared)
{
    if (k < 1 || L < 1 || L > 3 || n < 0) return DDGS_ERR_INVALID_ARG;
    if (per) *per = 3 + 4 + 3 + 1 + (int64_t)k;
    if (shared) *shared = (int64_t)k + (int64_t)kl_of(L) * k;
    return DDGS_OK;
}

ddgs_status ddgs_num_rendered(const ddgs_ctx *c, int64_t *n)
{
    if (!c || !n) return DDGS_ERR_INVALID_ARG;
    *n = c->M;
    return DDGS_OK;
}

ddgs_status ddgs_debug_count_pairs(ddgs_ctx *c, int enable)
{
    if (!c) return DDGS_ERR_INVALID_ARG;
    c->count_pairs = enable != 0;
    drop_graph(c);
    return DDGS_OK;
}

ddgs_status ddgs_debug_pair_counts(ddgs_ctx *c, int64_t *evaluated, int64_t *contributing)
{
    if (!c) return DDGS_ERR_INVALID_ARG;
    if (!c->count_pairs || !c->rendered) return fail(c, DDGS_ERR_STATE, "pair counting was off for the last render");
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    unsigned long long h[128];
    HIP_TRY(c, hipMemcpy(h, buf<unsigned long long>(c, "pair_counts"), sizeof(h), hipMemcpyDeviceToHost));
    int64_t e = 0, k = 0;
    for (int i = 0; i < 64; ++i) {
        e += (int64_t)h[2 * i];
        k += (int64_t)h[2 * i + 1];
    }
    if (evaluated) *evaluated = e;
    if (contributing) *contributing = k;
    return DDGS_OK;
}

ddgs_status ddgs_debug_keep_unsorted(ddgs_ctx *c, int keep)
{
    if (!c) return DDGS_ERR_INVALID_ARG;
    c->keep_unsorted = keep != 0;
    if (keep && c->entry_cap > 0) DDGS_TRY(ensure_entries(c, c->entry_cap));
    drop_graph(c);
    return DDGS_OK;
}

ddgs_status ddgs_debug_copy(ddgs_ctx *c, int what, void *host, size_t bytes)
{
    if (!c || !host) return DDGS_ERR_INVALID_ARG;
    if (what == DDGS_DBG_FIT_MOMENTS) {
        if (!c->fit_live) return fail(c, DDGS_ERR_STATE, "no fitting moments for the current model");
        const size_t need = sizeof(float) * 2 * fit_param_count(c->model.n, c->model.k, kl_of(c->model.L));
        if (bytes < need) return fail(c, DDGS_ERR_INVALID_ARG, "buffer too small: need " + std::to_string(need));
        HIP_TRY(c, hipSetDevice(c->device));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        HIP_TRY(c, hipMemcpy(host, buf<void>(c, "fit_mv"), need, hipMemcpyDeviceToHost));
        return DDGS_OK;
    }
    if (!c->rendered) return fail(c, DDGS_ERR_STATE, "nothing rendered");
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const int64_t VN = c->model.n * (int64_t)c->views_h.size();
    if (c->M < 0) {
        uint32_t fl = 0;
        ddgs_check(c, &fl);
    }
    const int64_t M = std::max<int64_t>(c->M, 0);
    const void *src = nullptr;
    size_t need = 0;
    std::vector<uint16_t> rect16;
    switch (what) {
    case DDGS_DBG_RECORDS: {
        // the first 32 bytes of every 64-byte pair record
        need = (size_t)VN * 32;
        if (bytes < need) return fail(c, DDGS_ERR_INVALID_ARG, "buffer too small: need " + std::to_string(need));
        if (VN > 0)
            HIP_TRY(c, hipMemcpy2D(host, 32, buf<void>(c, "rec"), 64, 32, (size_t)VN, hipMemcpyDeviceToHost));
        return DDGS_OK;
    }
    case DDGS_DBG_DEPTH_KEYS: src = buf<void>(c, "zkey"); need = (size_t)VN * 4; break;
    case DDGS_DBG_COUNTS: src = buf<void>(c, "cnt"); need = (size_t)VN * 4; break;
    case DDGS_DBG_RECTS: src = buf<void>(c, "rect"); need = (size_t)VN * 8; break;
    case DDGS_DBG_TILE_MASKS: src = buf<void>(c, "tmask"); need = (size_t)VN * 4; break;
    case DDGS_DBG_TILE_KEYS:
    case DDGS_DBG_TILE_KEYS_UNSORTED: {
        // the entries are binned by tile: every place of tile t's range holds t
        if (what == DDGS_DBG_TILE_KEYS_UNSORTED && !c->keep_unsorted)
            return fail(c, DDGS_ERR_STATE, "unsorted entries were not kept");
        need = (size_t)M * 4;
        if (bytes < need) return fail(c, DDGS_ERR_INVALID_ARG, "buffer too small: need " + std::to_string(need));
        std::vector<uint2> rg(std::max(1, c->n_tiles));
        if (c->n_tiles > 0)
            HIP_TRY(c, hipMemcpy(rg.data(), buf<void>(c, "ranges"), sizeof(uint2) * c->n_tiles, hipMemcpyDeviceToHost));
        uint32_t *o = (uint32_t *)host;
        for (int t = 0; t < c->n_tiles; ++t)
            for (uint32_t j = rg[t].x; j < rg[t].y && j < (uint32_t)M; ++j) o[j] = (uint32_t)t;
        return DDGS_OK;
    }
    case DDGS_DBG_TILE_VALS_UNSORTED: {
        if (!c->keep_unsorted) return fail(c, DDGS_ERR_STATE, "unsorted entries were not kept");
        need = (size_t)M * 4;
        if (bytes < need) return fail(c, DDGS_ERR_INVALID_ARG, "buffer too small: need " + std::to_string(need));
        if (M > 0)
            HIP_TRY(c, hipMemcpy2D(host, 4, (const char *)buf<void>(c, "ubin") + 4, 8, 4, (size_t)M, hipMemcpyDeviceToHost));
        return DDGS_OK;
    }
    case DDGS_DBG_TILE_VALS: src = buf<void>(c, "tval"); need = (size_t)M * 4; break;
    case DDGS_DBG_RANGES: src = buf<void>(c, "ranges"); need = (size_t)c->n_tiles * 8; break;
    case DDGS_DBG_NLAST: src = buf<void>(c, "nlast"); need = (size_t)c->total_pix * 4; break;
    case DDGS_DBG_TILE_BASE: {
        const size_t V = c->views_h.size();
        if (bytes < (V + 1) * 4) return fail(c, DDGS_ERR_INVALID_ARG, "buffer too small");
        int32_t *o = (int32_t *)host;
        for (size_t v = 0; v < V; ++v) o[v] = c->vdev_h[v].tile_base;
        o[V] = c->n_tiles;
        return DDGS_OK;
    }
    default: return fail(c, DDGS_ERR_INVALID_ARG, "unknown debug array");
    }
    if (bytes < need) return fail(c, DDGS_ERR_INVALID_ARG, "buffer too small: need " + std::to_string(need));
    if (need > 0 && src) HIP_TRY(c, hipMemcpy(host, src, need, hipMemcpyDeviceToHost));
    return DDGS_OK;
}

ddgs_status ddgs_debug_sort_pairs(ddgs_ctx *c, uint32_t *keys, uint32_t *vals, int64_t n, int bits)
{
    if (!c || n < 0 || bits < 1 || bits > 32 || (n > 0 && (!keys || !vals))) return fail(c, DDGS_ERR_INVALID_ARG, "bad sort arguments");
    if (n > 0xFFFFFFFFll) return fail(c, DDGS_ERR_INVALID_ARG, "n too large");
    if (n == 0) return DDGS_OK;
    HIP_TRY(c, hipSetDevice(c->device));
    uint32_t *k1, *v1;
    DDGS_TRY(ensure_t(c, "dbg_k1", n, &k1));
    DDGS_TRY(ensure_t(c, "dbg_v1", n, &v1));
    SortWs ws{};
    DDGS_TRY(aux_sort_ws(c, n, &ws));
    bool in_k1 = false;
    HIP_TRY(c, radix_sort_pairs(keys, vals, k1, v1, n, nullptr, bits, ws, &in_k1, c->stream));
    if (in_k1) {
        HIP_TRY(c, launch_copy_u32(keys, k1, nullptr, n, c->stream));
        HIP_TRY(c, launch_copy_u32(vals, v1, nullptr, n, c->stream));
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return DDGS_OK;
}

ddgs_status ddgs_sort_pairs_noalloc(ddgs_ctx *c, uint32_t *keys, uint32_t *vals, int64_t n, int bits)
{
    if (!c || n < 0 || bits < 1 || bits > 32 || (n > 0 && (!keys || !vals)))
        return fail(c, DDGS_ERR_INVALID_ARG, "bad sort arguments");
    if (n > kNoallocSortMax)
        return fail(c, DDGS_ERR_INVALID_ARG,
                    "n = " + std::to_string(n) + " exceeds the static scratch limit of " +
                        std::to_string(kNoallocSortMax) + " pairs of ddgs_sort_pairs_noalloc");
    if (n == 0) return DDGS_OK;
    HIP_TRY(c, hipSetDevice(c->device));
    char *base = nullptr;
    DDGS_TRY(scratch_base(c, &base));
    // carve the ping-pong halves and the radix temporaries for this n
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base + off;
        off += ws_round(bytes);
        return p;
    };
    uint32_t *k1 = (uint32_t *)take(sizeof(uint32_t) * (size_t)n);
    uint32_t *v1 = (uint32_t *)take(sizeof(uint32_t) * (size_t)n);
    const size_t cw = sort_counts_words(n), bw = sort_blocksum_words(n);
    uint32_t *counts = (uint32_t *)take(sizeof(uint32_t) * cw);
    uint32_t *tot = (uint32_t *)take(sizeof(uint32_t) * kSortTotWords);
    uint64_t *bsum = (uint64_t *)take(sizeof(uint64_t) * bw);
    if (off > kNoallocScratchBytes) return fail(c, DDGS_ERR_INVALID_ARG, "static scratch too small for this sort");
    const SortWs ws{counts, tot, bsum, cw, bw};
    bool in_k1 = false;
    HIP_TRY(c, radix_sort_pairs(keys, vals, k1, v1, n, nullptr, bits, ws, &in_k1, c->stream));
    if (in_k1) {
        HIP_TRY(c, launch_copy_u32(keys, k1, nullptr, n, c->stream));
        HIP_TRY(c, launch_copy_u32(vals, v1, nullptr, n, c->stream));
    }
    return DDGS_OK;
}

ddgs_status ddgs_debug_exclusive_scan(ddgs_ctx *c, const uint32_t *in, uint32_t *out, int64_t n, uint64_t *total)
{
    if (!c || n < 0 || (n > 0 && (!in || !out))) return fail(c, DDGS_ERR_INVALID_ARG, "bad scan arguments");
    HIP_TRY(c, hipSetDevice(c->device));
    SortWs ws{};
    DDGS_TRY(aux_sort_ws(c, n, &ws));
    uint64_t *tot;
    DDGS_TRY(ensure_t(c, "dbg_total", 1, &tot));
    HIP_TRY(c, launch_exclusive_scan(in, nullptr, out, n, ws, tot, c->stream));
    uint64_t h = 0;
    HIP_TRY(c, hipMemcpyAsync(&h, tot, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (total) *total = h;
    return DDGS_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ autotune

namespace {

struct TuneEntry {
    int tile_w = 16, tile_h = 16, persistent = 0, split = 256;
    double ms = 0.0;
};

std::string device_arch(const ddgs_ctx *c)
{
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, c->device) != hipSuccess) return "unknown";
    std::string a = p.gcnArchName;
    const size_t colon = a.find(':');  // drop the target features (e.g. ":sramecc+:xnack-")
    return colon == std::string::npos ? a : a.substr(0, colon);
}

std::string tune_signature(const ddgs_ctx *c, double entries_per_pair)
{
    // workload signature: device architecture, Gaussian-count bucket (power
    // of two), the feature size and the degree, the footprint bucket (tile
    // entries per (view, Gaussian) pair at 16x16 tiles, in half octaves) and
    // the detector mix (sizes with multiplicity)
    std::map<std::pair<int, int>, int> mix;
    for (const auto &v : c->views_h) mix[{v.W, v.H}]++;
    int b = 0;
    while (((int64_t)1 << b) < c->model.n) ++b;
    const int fb = entries_per_pair > 0.0 ? (int)std::floor(2.0 * std::log2(entries_per_pair)) : -99;
    std::ostringstream s;
    s << device_arch(c) << "|n2^" << b << "|k" << c->model.k << "|L" << c->model.L << "|fp" << fb << "|";
    for (const auto &kv : mix) s << kv.first.first << "x" << kv.first.second << "*" << kv.second << ";";
    return s.str();
}

bool parse_num(const std::string &obj, const char *key, double *out)
{
    const std::string k = std::string("\"") + key + "\"";
    const size_t p = obj.find(k);
    if (p == std::string::npos) return false;
    const size_t colon = obj.find(':', p + k.size());
    if (colon == std::string::npos) return false;
    char *end = nullptr;
    const double v = std::strtod(obj.c_str() + colon + 1, &end);
    if (end == obj.c_str() + colon + 1 || !std::isfinite(v)) return false;
    *out = v;
    return true;
}

// Reads {"sig": {"tile_w": .., "tile_h": .., "persistent": .., "ms": ..}, ...};
// anything unreadable is skipped (an unusable cache just means re-tuning).
std::map<std::string, TuneEntry> read_cache(const char *path)
{
    std::map<std::string, TuneEntry> out;
    std::ifstream f(path);
    if (!f) return out;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string s = ss.str();
    size_t pos = 0;
    while (true) {
        const size_t q0 = s.find('"', pos);
        if (q0 == std::string::npos) break;
        const size_t q1 = s.find('"', q0 + 1);
        if (q1 == std::string::npos) break;
        const size_t ob = s.find('{', q1);
        const size_t cb = s.find('}', q1);
        if (ob == std::string::npos || cb == std::string::npos || cb < ob) break;
        const std::string key = s.substr(q0 + 1, q1 - q0 - 1);
        const std::string obj = s.substr(ob, cb - ob + 1);
        double tw, th, pe, sp, ms;
        if (parse_num(obj, "tile_w", &tw) && parse_num(obj, "tile_h", &th) && parse_num(obj, "persistent", &pe) &&
            parse_num(obj, "split", &sp) && parse_num(obj, "ms", &ms) && raster_tile_supported((int)tw, (int)th) &&
            pe >= 0.0 && pe <= 8.0 && pe == std::floor(pe) && sp >= 0.0 && sp <= (double)(1 << 24)) {
            TuneEntry e;
            e.tile_w = (int)tw;
            e.tile_h = (int)th;
            e.persistent = (int)pe;
            e.split = (int)sp;
            e.ms = ms;
            out[key] = e;
        }
        pos = cb + 1;
    }
    return out;
}

bool write_cache(const char *path, const std::map<std::string, TuneEntry> &m)
{
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream f(tmp);
        if (!f) return false;
        f << "{\n";
        size_t i = 0;
        for (const auto &kv : m) {
            f << "  \"" << kv.first << "\": {\"tile_w\": " << kv.second.tile_w << ", \"tile_h\": " << kv.second.tile_h
              << ", \"persistent\": " << kv.second.persistent << ", \"split\": " << kv.second.split
              << ", \"ms\": " << kv.second.ms << "}"
              << (++i < m.size() ? ",\n" : "\n");
        }
        f << "}\n";
        if (!f) return false;
    }
    return std::rename(tmp.c_str(), path) == 0;
}

}  // namespace

extern "C" {

ddgs_status ddgs_autotune(ddgs_ctx *c, const char *cache_path, int repeats, float *best_ms)
{
    if (!c) return DDGS_ERR_INVALID_ARG;
    if (repeats < 1) repeats = 5;
    HIP_TRY(c, hipSetDevice(c->device));
    DDGS_TRY(check_ready(c));
    const int64_t n = c->model.n, k = c->model.k, KL = kl_of(c->model.L), V = (int64_t)c->views_h.size();
    const ddgs_options base = c->opt;
    float *img, *dL, *gm, *gq, *gs, *go, *gf, *gb, *gB, *gp;
    DDGS_TRY(prepare_views(c));
    DDGS_TRY(ensure_t(c, "tune_img", c->total_pix, &img));
    // the footprint bucket of the cache key: entries per pair at 16x16 tiles
    double epp = 0.0;
    {
        ddgs_options o = base;
        o.tile_w = o.tile_h = 16;
        DDGS_TRY(ddgs_set_options(c, &o));
        const ddgs_status st0 = ddgs_render(c, img);
        const ddgs_status st1 = ddgs_set_options(c, &base);
        if (st0 != DDGS_OK) return st0;
        if (st1 != DDGS_OK) return st1;
        if (n > 0 && V > 0) epp = (double)c->M / (double)(n * V);
    }
    const std::string sig = tune_signature(c, epp);
    std::map<std::string, TuneEntry> cache;
    if (cache_path) {
        cache = read_cache(cache_path);
        auto it = cache.find(sig);
        if (it != cache.end()) {
            ddgs_options o = c->opt;
            o.tile_w = it->second.tile_w;
            o.tile_h = it->second.tile_h;
            o.persistent = it->second.persistent;
            o.split = it->second.split;
            DDGS_TRY(ddgs_set_options(c, &o));
            if (best_ms) *best_ms = (float)it->second.ms;
            return DDGS_OK;
        }
    }
    DDGS_TRY(prepare_views(c));
    DDGS_TRY(ensure_t(c, "tune_dl", c->total_pix, &dL));
    DDGS_TRY(ensure_t(c, "tune_gm", 3 * n, &gm));
    DDGS_TRY(ensure_t(c, "tune_gq", 4 * n, &gq));
    DDGS_TRY(ensure_t(c, "tune_gs", 3 * n, &gs));
    DDGS_TRY(ensure_t(c, "tune_go", n, &go));
    DDGS_TRY(ensure_t(c, "tune_gf", k * n, &gf));
    DDGS_TRY(ensure_t(c, "tune_gb", k, &gb));
    DDGS_TRY(ensure_t(c, "tune_gB", KL * k, &gB));
    DDGS_TRY(ensure_t(c, "tune_gp", 6 * V, &gp));
    HIP_TRY(c, launch_fill_u32((uint32_t *)dL, 0x3f800000u, c->total_pix, c->stream));  // 1.0f
    ddgs_grads g{gm, gq, gs, go, gf, gb, gB, gp};
    hipEvent_t e0, e1;
    HIP_TRY(c, hipEventCreate(&e0));
    HIP_TRY(c, hipEventCreate(&e1));
    TuneEntry best;
    double best_t = 1e300;
    ddgs_status st = DDGS_OK;
    // median forward + backward time of one candidate: the kernels a captured
    // step of these options runs (projection, binning, sort, raster, merge,
    // backward), captured into a graph of the tuner's own and replayed, so
    // that the host round trip of a plain render (which reads the entry total
    // back between the scan and the scatter) does not enter the timing.  One
    // plain render sizes the graph's capacity (twice its entries) and the
    // long-range sort grid; one replay warms up.
    const bool saved_timing = c->timing;
    ddgs_options cand = base;
    auto record = [&](std::vector<float> &ts) {
        std::sort(ts.begin(), ts.end());
        const double med = ts[ts.size() / 2];
        if (med < best_t) {
            best_t = med;
            best.tile_w = cand.tile_w;
            best.tile_h = cand.tile_h;
            best.persistent = cand.persistent;
            best.split = cand.split;
            best.ms = med;
        }
    };
    // the trial graphs update the step counters of the scalars block (flags,
    // skipped replays, largest need) as a captured step does; what the
    // caller's replays left there for ddgs_check is restored afterwards
    uint32_t saved_sc[16] = {};
    HIP_TRY(c, hipMemcpyAsync(saved_sc, buf<uint32_t>(c, "scalars"), sizeof(saved_sc), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    auto trial = [&](int tw, int th, int pe, int sp) {
        ddgs_options o = base;
        o.tile_w = tw;
        o.tile_h = th;
        o.persistent = pe;
        o.split = sp;
        cand = o;
        st = ddgs_set_options(c, &o);
        if (st == DDGS_OK) st = ddgs_render(c, img);
        if (st != DDGS_OK) return;
        std::vector<float> ts;
        if (!c->stream) {
            // (the default stream cannot be captured: plain render + backward)
            st = ddgs_backward(c, dL, &g);
            for (int r = 0; r < repeats && st == DDGS_OK; ++r) {
                (void)hipEventRecord(e0, c->stream);
                st = ddgs_render(c, img);
                if (st == DDGS_OK) st = ddgs_backward(c, dL, &g);
                (void)hipEventRecord(e1, c->stream);
                if (hipEventSynchronize(e1) != hipSuccess) st = fail(c, DDGS_ERR_HIP, "event sync failed");
                float t = 0.0f;
                (void)hipEventElapsedTime(&t, e0, e1);
                ts.push_back(t);
            }
        }
        const int64_t cap = std::min<int64_t>(std::max<int64_t>(2 * c->M, 1024), 0xFFFFFFF0ll);
        if (c->stream) st = ensure_entries(c, cap);
        if (st != DDGS_OK || !c->stream) {
            if (st == DDGS_OK) record(ts);
            return;
        }
        c->long_grid = captured_long_grid(c);
        c->timing = false;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        if (hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            c->timing = saved_timing;
            st = fail(c, DDGS_ERR_HIP, "tuner: hipStreamBeginCapture failed");
            return;
        }
        st = enqueue_front(c, (uint32_t)cap, true);
        if (st == DDGS_OK) st = enqueue_back(c, cap, img);
        if (st == DDGS_OK) st = enqueue_backward(c, dL, &g, cap, true);
        const hipError_t ec = hipStreamEndCapture(c->stream, &graph);
        c->timing = saved_timing;
        if (st == DDGS_OK && ec != hipSuccess)
            st = fail(c, DDGS_ERR_HIP, std::string("tuner: hipStreamEndCapture: ") + hipGetErrorString(ec));
        if (st == DDGS_OK && hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess)
            st = fail(c, DDGS_ERR_HIP, "tuner: hipGraphInstantiate failed");
        if (st == DDGS_OK && hipGraphLaunch(exec, c->stream) != hipSuccess)
            st = fail(c, DDGS_ERR_HIP, "tuner: hipGraphLaunch failed");
        for (int r = 0; r < repeats && st == DDGS_OK; ++r) {
            (void)hipEventRecord(e0, c->stream);
            if (hipGraphLaunch(exec, c->stream) != hipSuccess) st = fail(c, DDGS_ERR_HIP, "tuner: hipGraphLaunch failed");
            (void)hipEventRecord(e1, c->stream);
            if (hipEventSynchronize(e1) != hipSuccess) st = fail(c, DDGS_ERR_HIP, "event sync failed");
            float t = 0.0f;
            (void)hipEventElapsedTime(&t, e0, e1);
            ts.push_back(t);
        }
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (st == DDGS_OK) record(ts);
    };
    // stage 1: tile shape x a coarse chunking, one workgroup per item; stage
    // 2: at the best shape, every chunk size x the persistent grid (0: off,
    // else m x 4 (forward) and m x 2 (backward) workgroups per CU)
    const int shapes[4][2] = {{16, 16}, {8, 8}, {16, 8}, {32, 8}};
    // (at 500k Gaussians, 512^2 and 8x8 tiles the captured step took 0.457,
    // 0.453, 0.471, 0.520 ms at chunks of 64, 128, 256, 512; the 64-view
    // 256^2 batch is fastest at 512 and above, the uneven batch at 256)
    const int coarse[4] = {128, 256, 1024, 0};
    for (int si = 0; si < 4 && st == DDGS_OK; ++si)
        for (int ci = 0; ci < 4 && st == DDGS_OK; ++ci) trial(shapes[si][0], shapes[si][1], 0, coarse[ci]);
    const int splits[8] = {64, 128, 256, 512, 1024, 2048, 4096, 0};
    const int mults[4] = {0, 1, 2, 4};
    const int tw = best.tile_w, th = best.tile_h;
    for (int sj = 0; sj < 8 && st == DDGS_OK; ++sj)
        for (int mj = 0; mj < 4 && st == DDGS_OK; ++mj) {
            bool done = false;
            for (int ci = 0; ci < 4; ++ci) done = done || (mults[mj] == 0 && splits[sj] == coarse[ci]);
            if (!done) trial(tw, th, mults[mj], splits[sj]);
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    {
        uint32_t sc[16] = {};
        HIP_TRY(c, hipMemcpyAsync(sc, buf<uint32_t>(c, "scalars"), sizeof(sc), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        for (int w : {3, 7, 10, 11}) sc[w] = saved_sc[w];
        HIP_TRY(c, hipMemcpyAsync(buf<uint32_t>(c, "scalars"), sc, sizeof(sc), hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
    }
    ddgs_options o = base;
    if (st == DDGS_OK) {
        o.tile_w = best.tile_w;
        o.tile_h = best.tile_h;
        o.persistent = best.persistent;
        o.split = best.split;
    }
    const ddgs_status st2 = ddgs_set_options(c, &o);
    if (st != DDGS_OK) return st;
    if (st2 != DDGS_OK) return st2;
    if (best_ms) *best_ms = (float)best.ms;
    if (cache_path) {
        cache[sig] = best;
        if (!write_cache(cache_path, cache)) return fail(c, DDGS_ERR_INVALID_ARG, "cannot write the tuning cache");
    }
    return DDGS_OK;
}

ddgs_status ddgs_enable_timing(ddgs_ctx *c, int enable)
{
    if (!c) return DDGS_ERR_INVALID_ARG;
    c->timing = enable != 0;
    for (int i = 0; i < DDGS_T_COUNT; ++i) c->ev_valid[i] = false;
    c->ev_sort_tail_valid = false;
    return DDGS_OK;
}

ddgs_status ddgs_stage_times(const ddgs_ctx *cc, float *ms)
{
    ddgs_ctx *c = const_cast<ddgs_ctx *>(cc);
    if (!c || !ms) return DDGS_ERR_INVALID_ARG;
    if (!c->timing) return fail(c, DDGS_ERR_STATE, "timing is not enabled");
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (int i = 0; i < DDGS_T_COUNT; ++i) {
        ms[i] = 0.0f;
        if (!c->ev_valid[i]) continue;
        float t = 0.0f;
        if (hipEventElapsedTime(&t, c->ev_s[i], c->ev_e[i]) == hipSuccess) ms[i] = t;
        if (i == DDGS_T_SORT && c->ev_sort_tail_valid &&
            hipEventElapsedTime(&t, c->ev_sort_tail_s, c->ev_sort_tail_e) == hipSuccess)
            ms[i] += t;
    }
    return DDGS_OK;
}

}  // extern "C"
