// bin.hip -- tile binning of the projected footprints on gfx950: the per-tile
// entry counts (accumulated by the projection), their scan into the tile
// ranges, the scatter of every (tile, Gaussian) entry into its tile's range,
// and the per-tile sort that puts each list in compositing order.
//
// Ordering scheme.  Eq. 1 composites a pixel's Gaussians front to back, so
// each tile's list must be ordered by (depth key, Gaussian index).  Instead of
// sorting every entry globally, the entries are binned by tile first: per-
// tile counts from LDS histograms of groups of Gaussians, one scan of the
// counts into the tile ranges, and a scatter that places each entry inside
// its tile's range (the order inside a range is arbitrary).  One workgroup
// per tile then orders its range: entries are bucketed by the leading bits
// of their (depth, index) code relative to the tile's smallest depth and
// index, and ranked inside their bucket.  The result is bit-identical to a
// global stable sort on (tile, depth, index), since that order is total.
// The stage takes five launches after the projection (count, column scan,
// tile scan, scatter, sort), against the dozen of a global multi-pass radix
// sort, which on this path ran at the launch floor.
#include "internal.h"

namespace ddgs {

namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / kWave;

// exclusive scan over a block of 256 threads; returns the block total
__device__ __forceinline__ uint32_t block_scan(uint32_t x, uint32_t *lds /* >= 4 */, uint32_t &total)
{
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const uint32_t inc = wave_incl_scan(x);
    if (lane == kWave - 1) lds[w] = inc;
    __syncthreads();
    uint32_t before = 0;
    total = 0;
#pragma unroll
    for (int q = 0; q < kWaves; ++q) {
        const uint32_t t = lds[q];
        if (q < w) before += t;
        total += t;
    }
    __syncthreads();
    return before + inc - x;
}

// ------------------------------------------------------------- tile scan
// One launch: block b (256 tiles) first sums the counts of the tiles before
// its own, then scans its own.  Writes the ranges (clamped to the capacity)
// and the scatter cursors (= range starts); the last block stores the total,
// the kept count and the step flags.  Block 0 also turns the slot
// numbering's block totals into the blocks' first slots (in place).  The
// same scan lists, in tile order, the tiles of more than kSortShort entries
// for the tile sort's long-range launch (a list built with a global atomic
// per tile would serialise on its counter).
constexpr int kSortShort = 2560;  // longest range the per-tile sort's first launch takes
struct ScanArgs {
    const uint32_t *tile_cnt;
    int n_tiles;
    uint2 *ranges;
    uint32_t *cursor;
    uint32_t capacity;
    uint64_t *total;
    uint32_t *m_out, *flags, *skipped;
    unsigned long long *need;
    uint32_t *slot_btot;
    int64_t slot_nb;
    // work items of `split` entries (split > 0, one-launch scan only): per
    // tile the item count and first item, the (tile, chunk) list, the item
    // count (clamped to max_items) and the two work-queue counters cleared
    uint32_t split;
    uint32_t *item_cnt, *item_base;
    uint2 *items;
    uint32_t max_items;
    uint32_t *n_items, *counter;
    // long tiles (count > kSortShort): the list, its length, and per-block
    // counts of the three-launch scan
    uint32_t *long_list, *long_n, *long_bsum;
};

__device__ __forceinline__ uint32_t is_long(uint32_t cnt) { return cnt > (uint32_t)kSortShort ? 1u : 0u; }

__device__ void slot_block_scan(uint32_t *slot_btot, int64_t slot_nb, uint32_t *wl)
{
    // exclusive scan in place, wrapping at 2^32 like the slot indices
    uint32_t carry = 0;
    for (int64_t c0 = 0; c0 < slot_nb; c0 += 4 * kBlock) {
        const int64_t b = c0 + 4 * (int64_t)threadIdx.x;
        uint32_t x[4], s = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            x[q] = b + q < slot_nb ? slot_btot[b + q] : 0u;
            s += x[q];
        }
        uint32_t tot;
        uint32_t pre = carry + block_scan(s, wl, tot);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (b + q < slot_nb) slot_btot[b + q] = pre;
            pre += x[q];
        }
        carry += tot;
    }
}

__device__ void finish_scan(const ScanArgs &a, uint64_t t)
{
    const bool over = t > (uint64_t)a.capacity;
    *a.total = t;
    *a.m_out = over ? a.capacity : (uint32_t)t;
    const uint32_t f = *a.flags | (over ? 1u : 0u);
    *a.flags = f;
    if (a.skipped) {
        // captured step: from the first overflow on, every replay until the
        // flags are cleared skips its optimiser updates
        if (f & 1u) *a.skipped = *a.skipped + 1u;
        if ((unsigned long long)t > *a.need) *a.need = (unsigned long long)t;
    }
}

__device__ __forceinline__ void write_range(const ScanArgs &a, int t, uint64_t start, uint32_t c)
{
    const uint64_t end = start + c, cap = a.capacity;
    const uint32_t s = (uint32_t)(start < cap ? start : cap), e = (uint32_t)(end < cap ? end : cap);
    a.ranges[t] = e > s ? make_uint2(s, e) : make_uint2(0u, 0u);  // empty tiles: [0, 0)
    a.cursor[t] = s;
}

__global__ __launch_bounds__(kBlock) void tile_scan_self_kernel(ScanArgs a)
{
    __shared__ uint32_t wl[kWaves];
    __shared__ uint64_t red[kWaves];
    __shared__ uint32_t ired[kWaves], lred[kWaves];
    if (blockIdx.x == 0) slot_block_scan(a.slot_btot, a.slot_nb, wl);
    const int base = blockIdx.x * kBlock;
    const uint32_t sp = a.split;
    // entries, long tiles and (with chunks) work items of the tiles before
    // this block's
    uint64_t c = 0;
    uint32_t ci = 0, cl = 0;
    // (unrolled so that the loads of up to 16 rounds are in flight together)
#pragma unroll 16
    for (int t = threadIdx.x; t < base; t += kBlock) {
        const uint32_t x = a.tile_cnt[t];
        c += x;
        cl += is_long(x);
        if (sp) ci += (x + sp - 1u) / sp;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        c += __shfl_xor(c, o, kWave);
        ci += __shfl_xor(ci, o, kWave);
        cl += __shfl_xor(cl, o, kWave);
    }
    if ((threadIdx.x & (kWave - 1)) == 0) {
        red[threadIdx.x / kWave] = c;
        ired[threadIdx.x / kWave] = ci;
        lred[threadIdx.x / kWave] = cl;
    }
    __syncthreads();
    uint64_t carry = 0;
    uint32_t icarry = 0, lcarry = 0;
#pragma unroll
    for (int q = 0; q < kWaves; ++q) {
        carry += red[q];
        icarry += ired[q];
        lcarry += lred[q];
    }
    const int t = base + threadIdx.x;
    const uint32_t v = t < a.n_tiles ? a.tile_cnt[t] : 0u;
    uint32_t tot;
    const uint32_t pre = block_scan(v, wl, tot);
    if (t < a.n_tiles) write_range(a, t, carry + pre, v);
    uint32_t ltot;
    const uint32_t lf = is_long(v);
    const uint32_t lpre = lcarry + block_scan(lf, wl, ltot);
    if (lf) a.long_list[lpre] = (uint32_t)t;
    uint32_t itot = 0;
    if (sp) {
        // (chunks of the unclamped count: past a clamped range end an item is
        // empty, and only an overflowed step, whose results are discarded,
        // clamps)
        const uint32_t nv = (v + sp - 1u) / sp;
        const uint32_t ipre = icarry + block_scan(nv, wl, itot);
        if (t < a.n_tiles) {
            a.item_cnt[t] = nv;
            a.item_base[t] = ipre;
            for (uint32_t k = 0; k < nv && ipre + k < a.max_items; ++k) a.items[ipre + k] = make_uint2((uint32_t)t, k);
        }
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
        finish_scan(a, carry + tot);
        *a.long_n = lcarry + ltot;
        if (sp) {
            const uint32_t ni = icarry + itot;
            *a.n_items = ni > a.max_items ? a.max_items : ni;
            a.counter[0] = 0u;
            a.counter[1] = 0u;
        }
    }
}

// More tiles: block sums, one block scanning them, then the blocks' scans.
__global__ __launch_bounds__(kBlock) void tile_sum_kernel(const uint32_t *cnt, int n, uint64_t *bsum, uint32_t *lsum)
{
    const int t = blockIdx.x * kBlock + threadIdx.x;
    const uint32_t x = t < n ? cnt[t] : 0u;
    uint64_t c = x;
    uint32_t l = is_long(x);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        c += __shfl_xor(c, o, kWave);
        l += __shfl_xor(l, o, kWave);
    }
    __shared__ uint64_t red[kWaves];
    __shared__ uint32_t lred[kWaves];
    if ((threadIdx.x & (kWave - 1)) == 0) {
        red[threadIdx.x / kWave] = c;
        lred[threadIdx.x / kWave] = l;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        bsum[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
        lsum[blockIdx.x] = lred[0] + lred[1] + lred[2] + lred[3];
    }
}

__global__ __launch_bounds__(1024) void tile_top_kernel(uint64_t *bsum, uint32_t *lsum, int nb, ScanArgs a)
{
    __shared__ uint64_t wt[16];
    __shared__ uint32_t lwt[16];
    __shared__ uint64_t carry_s;
    __shared__ uint32_t lcarry_s;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    if (threadIdx.x == 0) {
        carry_s = 0;
        lcarry_s = 0;
    }
    __syncthreads();
    for (int c0 = 0; c0 < nb; c0 += 1024) {
        const int idx = c0 + threadIdx.x;
        const uint64_t x = idx < nb ? bsum[idx] : 0;
        const uint32_t lx = idx < nb ? lsum[idx] : 0u;
        uint64_t inc = x;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const uint64_t y = __shfl_up(inc, o, kWave);
            if (lane >= o) inc += y;
        }
        const uint32_t linc = wave_incl_scan(lx);
        if (lane == kWave - 1) {
            wt[w] = inc;
            lwt[w] = linc;
        }
        __syncthreads();
        uint64_t before = carry_s, tot = 0;
        uint32_t lbefore = lcarry_s, ltot = 0;
        for (int q = 0; q < 16; ++q) {
            if (q < w) {
                before += wt[q];
                lbefore += lwt[q];
            }
            tot += wt[q];
            ltot += lwt[q];
        }
        if (idx < nb) {
            bsum[idx] = before + inc - x;
            lsum[idx] = lbefore + linc - lx;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            carry_s += tot;
            lcarry_s += ltot;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        finish_scan(a, carry_s);
        *a.long_n = lcarry_s;
    }
}

__global__ __launch_bounds__(kBlock) void tile_apply_kernel(const uint64_t *bsum, const uint32_t *lsum, ScanArgs a)
{
    __shared__ uint32_t wl[kWaves];
    if (blockIdx.x == gridDim.x - 1) slot_block_scan(a.slot_btot, a.slot_nb, wl);
    const int t = blockIdx.x * kBlock + threadIdx.x;
    const uint32_t v = t < a.n_tiles ? a.tile_cnt[t] : 0u;
    uint32_t tot;
    const uint32_t pre = block_scan(v, wl, tot);
    if (t < a.n_tiles) write_range(a, t, bsum[blockIdx.x] + pre, v);
    const uint32_t lf = is_long(v);
    const uint32_t lpre = lsum[blockIdx.x] + block_scan(lf, wl, tot);
    if (lf) a.long_list[lpre] = (uint32_t)t;
}

// ------------------------------------------------------- count and scatter
// Global atomics on a few thousand tile counters serialise per address on
// this part (a probe measured ~0.3 us per increment of one counter, 0.23 ms
// for 3.3M entries over 4096 tiles), so no global atomic is used.  Instead
// the pairs of each view are cut into groups of `per` Gaussians, and one
// workgroup per (group, view, window of kWin tiles) counts its group's
// entries per tile in LDS and writes the counts as one row of a count matrix
// (per view: [groups][tiles of the view]).  A column scan turns every
// column into the group's offset inside its tile and yields the tile
// totals, the tile scan turns the totals into ranges, and the scatter
// re-walks the same groups: an entry's place is its tile's start + its
// group's offset + a place claimed from an LDS cursor (the order inside a
// group is arbitrary; the per-tile sort fixes it).
constexpr int kWin = 16384;  // tiles of one view held in LDS at a time

struct BinArgs {
    int n, V, groups, per;        // per: Gaussians per group
    const uint32_t *cnt;          // [V*n] tiles kept per pair
    const uint2 *rect;            // [V*n] tile rectangles
    const uint32_t *tmask;        // [V*n] kept tiles of the rectangles (tile_kept)
    const uint32_t *zkey;         // [V*n]
    const ViewDev *views;
    uint32_t *mat;                // [groups * n_tiles]: view v at groups * tile_base[v]
};

// Calls f(local tile) for every kept tile of pair r's rectangle inside [t0, t1).
template <class F>
__device__ __forceinline__ void for_tiles(const BinArgs &a, int64_t r, int ntx, int t0, int t1, F f)
{
    const uint2 rc = a.rect[r];
    const int tx0 = rc.x & 0xFFFF, ty0 = rc.x >> 16, tx1 = rc.y & 0xFFFF, ty1 = rc.y >> 16;
    if ((ty1 + 1) * ntx <= t0 || ty0 * ntx >= t1) return;  // no row of the rectangle in the window
    const uint32_t mask = a.tmask[r], area = (uint32_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1));
    uint32_t place = 0;
    for (int ty = ty0; ty <= ty1; ++ty)
        for (int tx = tx0; tx <= tx1; ++tx, ++place) {
            const int lt = ty * ntx + tx;
            if (lt >= t0 && lt < t1 && tile_kept(mask, area, place)) f(lt);
        }
}

// (1024 threads per workgroup: the groups are few, so each needs many waves
// in flight to hide the latency of its reads and LDS atomics)
constexpr int kBinBlock = 1024;

__global__ __launch_bounds__(kBinBlock) void bin_count_kernel(BinArgs a)
{
    extern __shared__ uint32_t hist[];
    const int g = blockIdx.x, v = blockIdx.y, w = blockIdx.z;
    const ViewDev &V = a.views[v];
    const int Tv = V.ntx * V.nty, t0 = w * kWin;
    if (t0 >= Tv) return;
    const int t1 = min(Tv, t0 + kWin), nt = t1 - t0;
    for (int j = threadIdx.x; j < nt; j += kBinBlock) hist[j] = 0u;
    __syncthreads();
    const int i0 = g * a.per, i1 = min(a.n, i0 + a.per);
    for (int i = i0 + (int)threadIdx.x; i < i1; i += kBinBlock) {
        const int64_t r = (int64_t)v * a.n + i;
        if (a.cnt[r] == 0u) continue;
        for_tiles(a, r, V.ntx, t0, t1, [&](int lt) { atomicAdd(&hist[lt - t0], 1u); });
    }
    __syncthreads();
    uint32_t *row = a.mat + (size_t)a.groups * V.tile_base + (size_t)g * Tv + t0;
    for (int j = threadIdx.x; j < nt; j += kBinBlock) row[j] = hist[j];
}

// 16 tiles per workgroup (256 workgroups at 4096 tiles), the groups cut into
// kColBlocks contiguous blocks: thread (b, c) sums column c over row block b
// (16 consecutive tiles of a row are one 64-byte read), the block sums are
// combined in LDS, and every thread writes its rows' exclusive offsets.
// tile_cnt[t] receives the column total.
constexpr int kColTiles = 16, kColBlocks = 32;
__global__ __launch_bounds__(kColTiles *kColBlocks) void bin_colscan_kernel(BinArgs a, int n_tiles,
                                                                          uint32_t *tile_cnt)
{
    __shared__ uint32_t part[kColBlocks][kColTiles];
    const int c = threadIdx.x % kColTiles, rb = threadIdx.x / kColTiles;
    const int t = blockIdx.x * kColTiles + c;
    const bool ok = t < n_tiles;
    int v = 0;
    if (ok) {
        int lo = 0, hi = a.V - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.views[mid].tile_base <= t) lo = mid;
            else hi = mid - 1;
        }
        v = lo;
    }
    const ViewDev &V = a.views[v];
    const int Tv = V.ntx * V.nty, lt = t - V.tile_base;
    uint32_t *col = a.mat + (size_t)a.groups * V.tile_base + lt;
    const int rows = (a.groups + kColBlocks - 1) / kColBlocks;
    const int g0 = rb * rows, g1 = min(a.groups, g0 + rows);
    // the block's rows, sixteen loads in flight
    uint32_t sum = 0;
    for (int g = g0; g < g1; g += 16) {
        uint32_t x[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) x[q] = (ok && g + q < g1) ? col[(size_t)(g + q) * Tv] : 0u;
#pragma unroll
        for (int q = 0; q < 16; ++q) sum += x[q];
    }
    part[rb][c] = sum;
    __syncthreads();
    uint32_t run = 0, tot = 0;
#pragma unroll
    for (int q = 0; q < kColBlocks; ++q) {
        const uint32_t x = part[q][c];
        if (q < rb) run += x;
        tot += x;
    }
    if (ok && rb == 0) tile_cnt[t] = tot;
    for (int g = g0; g < g1; g += 16) {
        uint32_t x[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) x[q] = (ok && g + q < g1) ? col[(size_t)(g + q) * Tv] : 0u;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            if (ok && g + q < g1) col[(size_t)(g + q) * Tv] = run;
            run += x[q];
        }
    }
}

// Places: every tile's cursor starts at the tile's range start (clamped to
// the capacity) + the group's offset, and each entry claims the next place
// from it (an LDS atomic); places at or beyond the capacity are dropped (an
// overflowed step, which the flags report).
//
// Workgroups go to the eight XCDs in turn (block b to XCD b mod 8), each
// with its own L2.  Group g's places in a tile's range follow those of group
// g - 1, so XCD x takes the x-th contiguous eighth of the groups: the
// partial cache lines that consecutive groups write into one range are then
// completed in one L2 instead of across XCDs.  gridDim.x is a multiple of 8.
__global__ __launch_bounds__(kBinBlock) void bin_scatter_kernel(BinArgs a, const uint32_t *start, uint32_t capacity,
                                                                uint2 *out)
{
    extern __shared__ uint32_t cur[];
    const int per_x = (a.groups + 7) >> 3;
    const int g = (int)(blockIdx.x & 7u) * per_x + (int)(blockIdx.x >> 3);
    if ((int)(blockIdx.x >> 3) >= per_x || g >= a.groups) return;
    const int v = blockIdx.y, w = blockIdx.z;
    const ViewDev &V = a.views[v];
    const int Tv = V.ntx * V.nty, t0 = w * kWin;
    if (t0 >= Tv) return;
    const int t1 = min(Tv, t0 + kWin), nt = t1 - t0;
    const uint32_t *row = a.mat + (size_t)a.groups * V.tile_base + (size_t)g * Tv + t0;
    const uint32_t *st = start + V.tile_base + t0;
    for (int j = threadIdx.x; j < nt; j += kBinBlock) cur[j] = st[j] + row[j];
    __syncthreads();
    const int i0 = g * a.per, i1 = min(a.n, i0 + a.per);
    for (int i = i0 + (int)threadIdx.x; i < i1; i += kBinBlock) {
        const int64_t r = (int64_t)v * a.n + i;
        if (a.cnt[r] == 0u) continue;
        const uint32_t key = a.zkey[r];
        for_tiles(a, r, V.ntx, t0, t1, [&](int lt) {
            const uint32_t p = atomicAdd(&cur[lt - t0], 1u);
            if (p < capacity) out[p] = make_uint2(key, (uint32_t)i);
        });
    }
}

// ------------------------------------------------------------ tile sort
// One workgroup per tile puts its range in (depth key, index) order.  With
// k = key - (smallest key of the tile) and i = index - (smallest index), the
// order is that of the integer C = k 2^bi + i (bi = bits of the index span),
// which is unique per entry.  The entries are bucketed by the top kBinBits
// bits of C (a counting pass with LDS atomics; the order inside a bucket
// does not matter), and each entry's final place is its bucket's start plus
// the number of entries of its bucket with a smaller C.  Buckets hold a few
// entries on average, so the ranking costs a few comparisons per entry (and
// stays correct, if quadratic, for any distribution).  Ranges that fit the
// LDS capacity CAP are bucketed in LDS, longer ones in the same range of a
// second global buffer.
// Two instances: ranges of up to 2560 entries with 512 threads per tile (the
// per-tile phases are latency-bound: 512 measured 0.037 ms at 500k / 8x8
// tiles, 256 0.045, 1024 0.053; four workgroups of 37 KB LDS per CU), and
// longer ranges, up to 7168 in LDS (two workgroups of 74 KB per CU), with
// 1024 threads in a second launch.  Each launch leaves the other's tiles.
constexpr int kSortShortBlock = 512;
constexpr int kSortLong = 7168, kSortLongBlock = 1024;
constexpr int kSortLongGrid = 512;  // two workgroups per CU
constexpr int kBinBits = 11;
constexpr int kBins = 1 << kBinBits;

template <int CAP, int BLOCK>
struct SortLds {
    uint2 e[CAP];               // (key, index) in bucket order
    uint32_t start[kBins];      // bucket starts
    uint32_t cur[kBins];        // counts, then cursors (bucket ends at the last step)
    uint32_t wl[BLOCK / kWave];
    uint32_t red[4 * (BLOCK / kWave)];
};

// exclusive scan over a block of BLOCK threads; returns the block total
template <int BLOCK>
__device__ __forceinline__ uint32_t sort_block_scan(uint32_t x, uint32_t *lds, uint32_t &total)
{
    constexpr int kSortWaves = BLOCK / kWave;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const uint32_t inc = wave_incl_scan(x);
    if (lane == kWave - 1) lds[w] = inc;
    __syncthreads();
    uint32_t before = 0;
    total = 0;
#pragma unroll
    for (int q = 0; q < kSortWaves; ++q) {
        const uint32_t t = lds[q];
        if (q < w) before += t;
        total += t;
    }
    __syncthreads();
    return before + inc - x;
}

__device__ __forceinline__ int bit_length(uint32_t x) { return x ? 32 - __clz((int)x) : 0; }

// Sorts one tile's range rg (len >= 1) with the whole block; entry j of the
// range sits in a thread's slot q, j = tid + q * BLOCK.  Writes S from its
// first steps on: a caller that sorts several tiles puts a barrier between
// them.
template <int CAP, int BLOCK>
__device__ __forceinline__ void sort_tile(SortLds<CAP, BLOCK> &S, uint2 rg, const uint2 *ent, uint2 *tmp,
                                          uint32_t *tval)
{
    constexpr int kSortLds = CAP, kSortBlock = BLOCK, kSortWaves = BLOCK / kWave;
    constexpr int kSortRegs = CAP / BLOCK;  // entries per thread held in registers
    const int len = (int)(rg.y - rg.x);
    const uint2 *g = ent + rg.x;
    const int tid = threadIdx.x;
    if (len == 1) {
        if (tid == 0) tval[rg.x] = g[0].y;
        return;
    }
    const bool in_regs = len <= kSortLds;  // uniform over the block
    // the range (in registers when it fits), and the key and index spans
    uint2 x[kSortRegs];
    uint32_t kmin = 0xFFFFFFFFu, kmax = 0u, imin = 0xFFFFFFFFu, imax = 0u;
    if (in_regs) {
#pragma unroll
        for (int q = 0; q < kSortRegs; ++q) {
            const int j = tid + q * kSortBlock;
            x[q] = j < len ? g[j] : make_uint2(0xFFFFFFFFu, 0xFFFFFFFFu);
        }
#pragma unroll
        for (int q = 0; q < kSortRegs; ++q) {
            if (tid + q * kSortBlock < len) {
                kmin = min(kmin, x[q].x);
                kmax = max(kmax, x[q].x);
                imin = min(imin, x[q].y);
                imax = max(imax, x[q].y);
            }
        }
    } else {
        for (int j = tid; j < len; j += kSortBlock) {
            const uint2 y = g[j];
            kmin = min(kmin, y.x);
            kmax = max(kmax, y.x);
            imin = min(imin, y.y);
            imax = max(imax, y.y);
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        kmin = min(kmin, (uint32_t)__shfl_xor((int)kmin, o, kWave));
        kmax = max(kmax, (uint32_t)__shfl_xor((int)kmax, o, kWave));
        imin = min(imin, (uint32_t)__shfl_xor((int)imin, o, kWave));
        imax = max(imax, (uint32_t)__shfl_xor((int)imax, o, kWave));
    }
    const int lane = tid & (kWave - 1), w = tid / kWave;
    if (lane == 0) {
        S.red[w] = kmin;
        S.red[kSortWaves + w] = kmax;
        S.red[2 * kSortWaves + w] = imin;
        S.red[3 * kSortWaves + w] = imax;
    }
    for (int b = tid; b < kBins; b += kSortBlock) S.cur[b] = 0u;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kSortWaves; ++q) {
        kmin = min(kmin, S.red[q]);
        kmax = max(kmax, S.red[kSortWaves + q]);
        imin = min(imin, S.red[2 * kSortWaves + q]);
        imax = max(imax, S.red[3 * kSortWaves + q]);
    }
    const int bi = bit_length(imax - imin);
    const int total_bits = bit_length(kmax - kmin) + bi;
    const int sh = total_bits > kBinBits ? total_bits - kBinBits : 0;
    auto code = [&](uint2 y) -> uint64_t {
        return ((uint64_t)(y.x - kmin) << bi) | (uint64_t)(y.y - imin);
    };
    // bucket counts
    if (in_regs) {
#pragma unroll
        for (int q = 0; q < kSortRegs; ++q)
            if (tid + q * kSortBlock < len) atomicAdd(&S.cur[(uint32_t)(code(x[q]) >> sh)], 1u);
    } else {
        for (int j = tid; j < len; j += kSortBlock) atomicAdd(&S.cur[(uint32_t)(code(g[j]) >> sh)], 1u);
    }
    __syncthreads();
    // bucket starts: thread t owns buckets t B .. t B + B - 1
    {
        constexpr int B = kBins / kSortBlock;
        uint32_t c[B], sum = 0;
#pragma unroll
        for (int q = 0; q < B; ++q) {
            c[q] = S.cur[tid * B + q];
            sum += c[q];
        }
        uint32_t tot;
        uint32_t pre = sort_block_scan<BLOCK>(sum, S.wl, tot);
#pragma unroll
        for (int q = 0; q < B; ++q) {
            S.start[tid * B + q] = pre;
            S.cur[tid * B + q] = pre;
            pre += c[q];
        }
    }
    __syncthreads();
    if (in_regs) {
        // bucketing in LDS, then each entry (still in registers) is ranked
        // against the other entries of its bucket
#pragma unroll
        for (int q = 0; q < kSortRegs; ++q)
            if (tid + q * kSortBlock < len) S.e[atomicAdd(&S.cur[(uint32_t)(code(x[q]) >> sh)], 1u)] = x[q];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kSortRegs; ++q) {
            if (tid + q * kSortBlock >= len) continue;
            const uint64_t cx = code(x[q]);
            const uint32_t b = (uint32_t)(cx >> sh);
            const uint32_t s0 = S.start[b], e0 = S.cur[b];
            uint32_t r = s0;
            for (uint32_t p = s0; p < e0; ++p) r += code(S.e[p]) < cx ? 1u : 0u;
            tval[rg.x + r] = x[q].y;
        }
    } else {
        // long range: bucketed in the range's place in tmp
        uint2 *buf = tmp + rg.x;
        for (int j = tid; j < len; j += kSortBlock) {
            const uint2 y = g[j];
            buf[atomicAdd(&S.cur[(uint32_t)(code(y) >> sh)], 1u)] = y;
        }
        __syncthreads();
        for (int p = tid; p < len; p += kSortBlock) {
            const uint2 y = buf[p];
            const uint64_t cy = code(y);
            const uint32_t b = (uint32_t)(cy >> sh);
            const uint32_t s0 = S.start[b], e0 = S.cur[b];
            uint32_t r = s0;
            for (uint32_t q = s0; q < e0; ++q) r += code(buf[q]) < cy ? 1u : 0u;
            tval[rg.x + r] = y.y;
        }
    }
}

// One workgroup per tile, leaving the long tiles (is_long of the tile's
// count, the tile scan's rule for its list) to the second launch unless
// take_long is set (then there is no second launch, and a long tile is
// bucketed in global memory by this launch's workgroup).
template <int CAP, int BLOCK>
__global__ __launch_bounds__(BLOCK) void tile_sort_kernel(const uint2 *ranges, const uint32_t *tile_cnt, int n_tiles,
                                                          const uint2 *ent, uint2 *tmp, uint32_t *tval, int take_long)
{
    static_assert(CAP >= kSortShort, "short ranges are sorted in LDS");
    __shared__ SortLds<CAP, BLOCK> S;
    const int tile = blockIdx.x;
    if (tile >= n_tiles) return;
    const uint32_t cnt = tile_cnt[tile];  // (both loads in flight together)
    const uint2 rg = ranges[tile];
    if ((is_long(cnt) && !take_long) || rg.y <= rg.x) return;
    sort_tile<CAP, BLOCK>(S, rg, ent, tmp, tval);
}

// The tile scan's list of long tiles.  Few tiles are that long and they
// cluster in the image, so a fixed grid takes them round-robin from the list
// (a workgroup per tile, with this much LDS each, would spend more on being
// dispatched for every short or empty tile than on the long ones).
template <int CAP, int BLOCK>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(8, 8))) void tile_sort_long_kernel(
    const uint2 *ranges, const uint2 *ent, uint2 *tmp, uint32_t *tval, const uint32_t *list, const uint32_t *n_list)
{
    __shared__ SortLds<CAP, BLOCK> S;
    const uint32_t n_long = *n_list;
    for (uint32_t i = blockIdx.x; i < n_long; i += gridDim.x) {
        const uint2 rg = ranges[list[i]];
        if (rg.y <= rg.x) continue;  // (a range clamped away by an overflowed step)
        sort_tile<CAP, BLOCK>(S, rg, ent, tmp, tval);
        __syncthreads();
    }
}

}  // namespace

bool tile_scan_makes_items(int n_tiles) { return n_tiles <= kTileScanSelfMax; }

hipError_t launch_tile_scan(const uint32_t *tile_cnt, int n_tiles, uint2 *ranges, uint32_t *cursor,
                            uint32_t capacity, uint64_t *total, uint32_t *m_out, uint32_t *flags,
                            uint32_t *skipped, unsigned long long *need, uint32_t *slot_btot, int64_t slot_nb,
                            uint64_t *bsum, size_t bsum_words, const TileItems *it, const LongTiles &lt,
                            hipStream_t s)
{
    ScanArgs a{tile_cnt, n_tiles, ranges, cursor, capacity, total, m_out, flags, skipped, need, slot_btot, slot_nb,
               0u, nullptr, nullptr, nullptr, 0u, nullptr, nullptr, lt.list, lt.n, lt.bsum};
    if (!lt.list || !lt.n) return hipErrorInvalidValue;
    const int nb = (n_tiles + kBlock - 1) / kBlock;
    if (n_tiles <= kTileScanSelfMax) {
        if (it && it->split > 0) {
            a.split = (uint32_t)it->split;
            a.item_cnt = it->cnt;
            a.item_base = it->base;
            a.items = it->items;
            a.max_items = it->max_items;
            a.n_items = it->n_items;
            a.counter = it->counter;
        }
        tile_scan_self_kernel<<<std::max(1, nb), kBlock, 0, s>>>(a);
        return hipGetLastError();
    }
    if (it) return hipErrorInvalidValue;  // the three-launch scan makes no items
    if (!bsum || (size_t)nb > bsum_words || !lt.bsum || (size_t)nb > lt.bsum_words) return hipErrorInvalidValue;
    tile_sum_kernel<<<nb, kBlock, 0, s>>>(tile_cnt, n_tiles, bsum, lt.bsum);
    tile_top_kernel<<<1, 1024, 0, s>>>(bsum, lt.bsum, nb, a);
    tile_apply_kernel<<<nb, kBlock, 0, s>>>(bsum, lt.bsum, a);
    return hipGetLastError();
}

// Gaussians per group: at least 1024 (one per thread of the count and
// scatter workgroups; with the XCD-ordered groups 1024 measured 0.024 ms for
// the scatter at 500k Gaussians / 8x8 tiles against 0.036 ms for 2048), and
// few enough groups that the count matrix stays within kMatWords words
// (256 MB; with many views the cap sets the group size: at 1M Gaussians and
// 96256 tiles a cap of 8M words made groups of 16k and the scatter took
// 1.21 ms, 64M words 0.96 ms, the 64-pose batch 8.33 -> 8.10 ms per step).
constexpr int64_t kMatWords = (int64_t)64 << 20;
int bin_per_group(int64_t n, int64_t n_tiles)
{
    int64_t per = 1024;
    while (per < n && ((n + per - 1) / per) * std::max<int64_t>(n_tiles, 1) > kMatWords) per *= 2;
    return (int)per;
}

size_t bin_matrix_words(int64_t n, int64_t n_tiles)
{
    const int64_t per = bin_per_group(n, n_tiles);
    return (size_t)std::max<int64_t>(1, ((n + per - 1) / per) * std::max<int64_t>(n_tiles, 1));
}

hipError_t launch_bin_count(int n, int V, const uint32_t *cnt, const uint2 *rect, const uint32_t *tmask,
                            const ViewDev *views, int n_tiles, int max_view_tiles, uint32_t *mat, uint32_t *tile_cnt,
                            hipStream_t s)
{
    if (n <= 0 || V <= 0 || n_tiles <= 0) return hipSuccess;
    if (V > 65535 || max_view_tiles <= 0) return hipErrorInvalidValue;
    const int per = bin_per_group(n, n_tiles);
    BinArgs a{n, V, (n + per - 1) / per, per, cnt, rect, tmask, nullptr, views, mat};
    const int wins = (max_view_tiles + kWin - 1) / kWin;
    const size_t lds = sizeof(uint32_t) * std::min(max_view_tiles, kWin);
    bin_count_kernel<<<dim3(a.groups, V, wins), kBinBlock, lds, s>>>(a);
    bin_colscan_kernel<<<(n_tiles + kColTiles - 1) / kColTiles, kColTiles * kColBlocks, 0, s>>>(a, n_tiles, tile_cnt);
    return hipGetLastError();
}

hipError_t launch_bin_scatter(int n, int V, const uint32_t *cnt, const uint2 *rect, const uint32_t *tmask,
                              const uint32_t *zkey, const ViewDev *views, int n_tiles, int max_view_tiles,
                              const uint32_t *mat,
                              const uint32_t *start, uint32_t capacity, uint2 *out, hipStream_t s)
{
    if (n <= 0 || V <= 0 || n_tiles <= 0) return hipSuccess;
    if (V > 65535 || max_view_tiles <= 0) return hipErrorInvalidValue;
    const int per = bin_per_group(n, n_tiles);
    BinArgs a{n, V, (n + per - 1) / per, per, cnt, rect, tmask, zkey, views, const_cast<uint32_t *>(mat)};
    const int wins = (max_view_tiles + kWin - 1) / kWin;
    const size_t lds = sizeof(uint32_t) * std::min(max_view_tiles, kWin);
    bin_scatter_kernel<<<dim3((a.groups + 7) / 8 * 8, V, wins), kBinBlock, lds, s>>>(a, start, capacity, out);
    return hipGetLastError();
}

hipError_t launch_tile_sort(const uint2 *ranges, const uint32_t *tile_cnt, int n_tiles, const uint2 *ent, uint2 *tmp,
                            uint32_t *tval, const LongTiles &lt, int long_grid, hipStream_t s)
{
    if (n_tiles <= 0) return hipSuccess;
    const int g = std::min(std::min(n_tiles, kSortLongGrid), long_grid);
    tile_sort_kernel<kSortShort, kSortShortBlock><<<n_tiles, kSortShortBlock, 0, s>>>(ranges, tile_cnt, n_tiles, ent,
                                                                                       tmp, tval, g <= 0 ? 1 : 0);
    if (g <= 0) return hipGetLastError();
    tile_sort_long_kernel<kSortLong, kSortLongBlock><<<g, kSortLongBlock, 0, s>>>(ranges, ent, tmp, tval, lt.list,
                                                                                   lt.n);
    return hipGetLastError();
}

}  // namespace ddgs
