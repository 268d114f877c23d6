// bin.hip -- tile binning of the projected footprints on gfx950: the per-tile
// entry counts (accumulated by the projection), their scan into the tile
// ranges, the scatter of every (tile, Gaussian) entry into its tile's range,
// and the per-tile sort that puts each list in compositing order.
//
// Ordering scheme.  Eq. 1 composites a pixel's Gaussians front to back, so
// each tile's list must be ordered by (depth key, Gaussian index).  Instead of
// sorting every entry globally, the entries are binned by tile first: the
// projection counts the entries of every tile with one atomic increment per
// entry, one scan turns the counts into the tile ranges, and the scatter
// claims a place inside its tile's range with an atomic cursor (so the order
// inside a range is arbitrary).  One workgroup per tile then sorts its range
// in LDS: a stable LSD radix sort on the depth key relative to the tile's
// smallest key (only the bits that differ inside the tile), after which runs
// of equal keys -- rare, FP32 depths of different Gaussians -- are put in
// index order.  The result is bit-identical to a global stable sort on
// (tile, depth, index), since that order is total.  The whole stage is three
// launches (scan, scatter, sort) after the projection, against the dozen
// of a global multi-pass radix sort, which on this path ran at the launch
// floor.
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
// numbering's block totals into the blocks' first slots (in place).
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
};

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
    if (blockIdx.x == 0) slot_block_scan(a.slot_btot, a.slot_nb, wl);
    const int base = blockIdx.x * kBlock;
    uint64_t c = 0;
#pragma unroll 4
    for (int t = threadIdx.x; t < base; t += kBlock) c += a.tile_cnt[t];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = c;
    __syncthreads();
    uint64_t carry = 0;
#pragma unroll
    for (int q = 0; q < kWaves; ++q) carry += red[q];
    const int t = base + threadIdx.x;
    const uint32_t v = t < a.n_tiles ? a.tile_cnt[t] : 0u;
    uint32_t tot;
    const uint32_t pre = block_scan(v, wl, tot);
    if (t < a.n_tiles) write_range(a, t, carry + pre, v);
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) finish_scan(a, carry + tot);
}

// More tiles: block sums, one block scanning them, then the blocks' scans.
__global__ __launch_bounds__(kBlock) void tile_sum_kernel(const uint32_t *cnt, int n, uint64_t *bsum)
{
    const int t = blockIdx.x * kBlock + threadIdx.x;
    uint64_t c = t < n ? cnt[t] : 0u;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, kWave);
    __shared__ uint64_t red[kWaves];
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = c;
    __syncthreads();
    if (threadIdx.x == 0) bsum[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ __launch_bounds__(1024) void tile_top_kernel(uint64_t *bsum, int nb, ScanArgs a)
{
    __shared__ uint64_t wt[16];
    __shared__ uint64_t carry_s;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    if (threadIdx.x == 0) carry_s = 0;
    __syncthreads();
    for (int c0 = 0; c0 < nb; c0 += 1024) {
        const int idx = c0 + threadIdx.x;
        const uint64_t x = idx < nb ? bsum[idx] : 0;
        uint64_t inc = x;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const uint64_t y = __shfl_up(inc, o, kWave);
            if (lane >= o) inc += y;
        }
        if (lane == kWave - 1) wt[w] = inc;
        __syncthreads();
        uint64_t before = carry_s, tot = 0;
        for (int q = 0; q < 16; ++q) {
            if (q < w) before += wt[q];
            tot += wt[q];
        }
        if (idx < nb) bsum[idx] = before + inc - x;
        __syncthreads();
        if (threadIdx.x == 0) carry_s += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) finish_scan(a, carry_s);
}

__global__ __launch_bounds__(kBlock) void tile_apply_kernel(const uint64_t *bsum, ScanArgs a)
{
    __shared__ uint32_t wl[kWaves];
    if (blockIdx.x == gridDim.x - 1) slot_block_scan(a.slot_btot, a.slot_nb, wl);
    const int t = blockIdx.x * kBlock + threadIdx.x;
    const uint32_t v = t < a.n_tiles ? a.tile_cnt[t] : 0u;
    uint32_t tot;
    const uint32_t pre = block_scan(v, wl, tot);
    if (t < a.n_tiles) write_range(a, t, bsum[blockIdx.x] + pre, v);
}

// ---------------------------------------------------------------- scatter
// One thread per (view, Gaussian) pair: every tile of its rectangle claims
// the next free place of that tile's range and stores (depth key, index).
// Places at or beyond the capacity are dropped (an overflowed step, which the
// flags report).  The grid also clears the tile counters for the next
// projection.
__global__ __launch_bounds__(kBlock) void bin_scatter_kernel(int64_t VN, int n, const uint32_t *cnt,
                                                             const uint2 *rect, const uint32_t *zkey,
                                                             const ViewDev *views, uint32_t *cursor,
                                                             uint32_t capacity, uint2 *out, uint32_t *tile_cnt,
                                                             int n_tiles)
{
    const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    for (int64_t t = r; t < n_tiles; t += (int64_t)gridDim.x * kBlock) tile_cnt[t] = 0u;
    if (r >= VN) return;
    if (cnt[r] == 0u) return;
    const uint32_t v = (uint32_t)(r / n), i = (uint32_t)(r - (int64_t)v * n);
    const uint2 rc = rect[r];
    const uint32_t key = zkey[r];
    const int tx0 = rc.x & 0xFFFF, ty0 = rc.x >> 16, tx1 = rc.y & 0xFFFF, ty1 = rc.y >> 16;
    const int base = views[v].tile_base, ntx = views[v].ntx;
    for (int ty = ty0; ty <= ty1; ++ty)
        for (int tx = tx0; tx <= tx1; ++tx) {
            const uint32_t p = atomicAdd(&cursor[base + ty * ntx + tx], 1u);
            if (p < capacity) out[p] = make_uint2(key, i);
        }
}

// ------------------------------------------------------------ tile sort
// One workgroup per tile.  Entries (depth key, index) of the tile's range
// are sorted by key - (smallest key of the tile), 8 bits per pass, with a
// stable ranking: each wave ranks its rounds of 64 consecutive entries with
// ballots (the lanes sharing the digit), the block adds the four waves'
// histograms, and entries move to digit start + earlier waves + rank.  A
// range of up to kSortLds entries stays in LDS across the passes; a longer
// one is processed kSortLds entries at a time from global memory (each chunk
// ranked in LDS, placed after the earlier chunks' entries of its digit), in
// the range itself and a second buffer of the same layout.  Finally every
// run of equal keys is put in index order and the indices are written out.
constexpr int kSortLds = 4096;                       // entries held in LDS
constexpr int kSortRounds = kSortLds / kBlock;       // rounds of 64 per wave
constexpr int kDigits = 256;

struct SortLds {
    uint2 a[kSortLds];        // (relative key, index)
    uint2 b[kSortLds];
    uint32_t wh[kWaves][kDigits];  // per-wave digit counts, then offsets
    uint32_t dstart[kDigits];      // digit start inside the chunk
    uint32_t dcount[kDigits];      // entries of each digit in the chunk
    uint32_t run[kDigits];         // global path: next place of each digit in the range
    uint32_t wl[kWaves];
    uint32_t red[2 * kWaves];
};

// Stable ranking of the cnt (<= kSortLds) entries of src by the digit
// (key >> shift) & 255: put(entry, digit, place) receives every entry with
// its place in the chunk's digit-sorted order.  Leaves the chunk's digit
// counts in dcount and their exclusive scan in dstart.
template <class Put>
__device__ __forceinline__ void rank_chunk(SortLds &S, const uint2 *src, int cnt, int shift, Put put)
{
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    for (int d = threadIdx.x; d < kWaves * kDigits; d += kBlock) (&S.wh[0][0])[d] = 0u;
    __syncthreads();
    // wave w takes the consecutive entries [w q, (w + 1) q), q a multiple of 64
    const int q = ((cnt + kWaves * kWave - 1) / (kWaves * kWave)) * kWave;
    const int wb = w * q;
    const uint64_t lt_mask = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
    uint32_t rank[kSortRounds];
    uint2 e[kSortRounds];
#pragma unroll
    for (int rr = 0; rr < kSortRounds; ++rr) {
        const int j = wb + rr * kWave + lane;
        const bool ok = rr * kWave < q && j < cnt;
        e[rr] = ok ? src[j] : make_uint2(0u, 0u);
        rank[rr] = 0u;
        if (rr * kWave >= q) continue;  // uniform over the wave
        const uint32_t dg = (e[rr].x >> shift) & 255u;
        uint64_t peers = __ballot(ok);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (dg >> b) & 1u;
            const uint64_t bal = __ballot(bit);
            peers &= bit ? bal : ~bal;
        }
        const uint32_t below = (uint32_t)__popcll(peers & lt_mask);
        uint32_t prev = 0;
        if (ok) prev = S.wh[w][dg];
        __builtin_amdgcn_wave_barrier();
        if (ok && below == 0) S.wh[w][dg] = prev + (uint32_t)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
        rank[rr] = prev + below;
    }
    __syncthreads();
    {
        // thread d owns digit d: offsets of the waves, then the digit starts
        const int d = threadIdx.x;
        const uint32_t c0 = S.wh[0][d], c1 = S.wh[1][d], c2 = S.wh[2][d], c3 = S.wh[3][d];
        S.wh[0][d] = 0u;
        S.wh[1][d] = c0;
        S.wh[2][d] = c0 + c1;
        S.wh[3][d] = c0 + c1 + c2;
        uint32_t tot;
        S.dstart[d] = block_scan(c0 + c1 + c2 + c3, S.wl, tot);
        S.dcount[d] = c0 + c1 + c2 + c3;
    }
    __syncthreads();
#pragma unroll
    for (int rr = 0; rr < kSortRounds; ++rr) {
        const int j = wb + rr * kWave + lane;
        if (rr * kWave < q && j < cnt) {
            const uint32_t dg = (e[rr].x >> shift) & 255u;
            put(e[rr], dg, S.dstart[dg] + S.wh[w][dg] + rank[rr]);
        }
    }
}

__device__ __forceinline__ int bit_length(uint32_t x) { return x ? 32 - __clz((int)x) : 0; }

__global__ __launch_bounds__(kBlock) void tile_sort_kernel(const uint2 *ranges, int n_tiles, uint2 *ent,
                                                           uint2 *tmp, uint32_t *tval)
{
    __shared__ SortLds S;
    const int tile = blockIdx.x;
    if (tile >= n_tiles) return;
    const uint2 rg = ranges[tile];
    const int len = (int)(rg.y - rg.x);
    if (len <= 0) return;
    uint2 *g = ent + rg.x;
    uint2 *g2 = tmp + rg.x;
    const int tid = threadIdx.x;
    if (len == 1) {
        if (tid == 0) tval[rg.x] = g[0].y;
        return;
    }
    // smallest and largest key of the tile
    uint32_t kmin = 0xFFFFFFFFu, kmax = 0u;
    for (int j = tid; j < len; j += kBlock) {
        const uint32_t k = g[j].x;
        kmin = min(kmin, k);
        kmax = max(kmax, k);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        kmin = min(kmin, (uint32_t)__shfl_xor((int)kmin, o, kWave));
        kmax = max(kmax, (uint32_t)__shfl_xor((int)kmax, o, kWave));
    }
    const int lane = tid & (kWave - 1), w = tid / kWave;
    if (lane == 0) {
        S.red[w] = kmin;
        S.red[kWaves + w] = kmax;
    }
    __syncthreads();
    kmin = min(min(S.red[0], S.red[1]), min(S.red[2], S.red[3]));
    kmax = max(max(S.red[4], S.red[5]), max(S.red[6], S.red[7]));
    const int passes = (bit_length(kmax - kmin) + 7) / 8;
    __syncthreads();

    uint2 *out;  // LDS or global buffer holding the key-sorted range
    if (len <= kSortLds) {
        // the whole range in LDS, keys relative to the minimum
        for (int j = tid; j < len; j += kBlock) {
            const uint2 x = g[j];
            S.a[j] = make_uint2(x.x - kmin, x.y);
        }
        __syncthreads();
        uint2 *src = S.a, *dst = S.b;
        for (int p = 0; p < passes; ++p) {
            rank_chunk(S, src, len, 8 * p, [&](uint2 x, uint32_t, uint32_t pos) { dst[pos] = x; });
            __syncthreads();
            uint2 *t = src;
            src = dst;
            dst = t;
        }
        out = src;
    } else {
        // chunks of kSortLds from global memory, ping-pong between the range
        // and the same range of tmp
        for (int j = tid; j < len; j += kBlock) {
            const uint2 x = g[j];
            g[j] = make_uint2(x.x - kmin, x.y);
        }
        __syncthreads();
        uint2 *src = g, *dst = g2;
        for (int p = 0; p < passes; ++p) {
            const int shift = 8 * p;
            // digit totals of the whole range, then their starts
            S.run[tid] = 0u;
            __syncthreads();
            for (int j = tid; j < len; j += kBlock) atomicAdd(&S.run[(src[j].x >> shift) & 255u], 1u);
            __syncthreads();
            {
                uint32_t tot;
                const uint32_t c = S.run[tid];
                __syncthreads();
                const uint32_t st = block_scan(c, S.wl, tot);
                S.run[tid] = st;  // running start of digit tid in the range
            }
            __syncthreads();
            for (int c0 = 0; c0 < len; c0 += kSortLds) {
                const int cnt = min(kSortLds, len - c0);
                for (int j = tid; j < cnt; j += kBlock) S.a[j] = src[c0 + j];
                __syncthreads();
                rank_chunk(S, S.a, cnt, shift, [&](uint2 x, uint32_t dg, uint32_t pos) {
                    dst[S.run[dg] + (pos - S.dstart[dg])] = x;
                });
                __syncthreads();
                S.run[tid] += S.dcount[tid];
                __syncthreads();
            }
            uint2 *t = src;
            src = dst;
            dst = t;
        }
        out = src;
    }
    __syncthreads();
    // runs of equal keys in index order: entry j of a run [s, e) goes to
    // s + (entries of the run with a smaller index)
    for (int j = tid; j < len; j += kBlock) {
        const uint2 x = out[j];
        int s = j, e = j + 1;
        while (s > 0 && out[s - 1].x == x.x) --s;
        while (e < len && out[e].x == x.x) ++e;
        int r = s;
        if (e - s > 1)
            for (int m = s; m < e; ++m) r += out[m].y < x.y ? 1 : 0;
        tval[rg.x + r] = x.y;
    }
}

}  // namespace

hipError_t launch_tile_scan(const uint32_t *tile_cnt, int n_tiles, uint2 *ranges, uint32_t *cursor,
                            uint32_t capacity, uint64_t *total, uint32_t *m_out, uint32_t *flags,
                            uint32_t *skipped, unsigned long long *need, uint32_t *slot_btot, int64_t slot_nb,
                            uint64_t *bsum, size_t bsum_words, hipStream_t s)
{
    ScanArgs a{tile_cnt, n_tiles, ranges, cursor, capacity, total, m_out, flags, skipped, need, slot_btot, slot_nb};
    const int nb = (n_tiles + kBlock - 1) / kBlock;
    if (n_tiles <= kTileScanSelfMax) {
        tile_scan_self_kernel<<<std::max(1, nb), kBlock, 0, s>>>(a);
        return hipGetLastError();
    }
    if (!bsum || (size_t)nb > bsum_words) return hipErrorInvalidValue;
    tile_sum_kernel<<<nb, kBlock, 0, s>>>(tile_cnt, n_tiles, bsum);
    tile_top_kernel<<<1, 1024, 0, s>>>(bsum, nb, a);
    tile_apply_kernel<<<nb, kBlock, 0, s>>>(bsum, a);
    return hipGetLastError();
}

hipError_t launch_bin_scatter(int64_t VN, int n, const uint32_t *cnt, const uint2 *rect, const uint32_t *zkey,
                              const ViewDev *views, uint32_t *cursor, uint32_t capacity, uint2 *out,
                              uint32_t *tile_cnt, int n_tiles, hipStream_t s)
{
    const int64_t nb = std::max<int64_t>((VN + kBlock - 1) / kBlock, (n_tiles + kBlock - 1) / kBlock);
    if (nb <= 0) return hipSuccess;
    bin_scatter_kernel<<<(unsigned)nb, kBlock, 0, s>>>(VN, n, cnt, rect, zkey, views, cursor, capacity, out,
                                                       tile_cnt, n_tiles);
    return hipGetLastError();
}

hipError_t launch_tile_sort(const uint2 *ranges, int n_tiles, uint2 *ent, uint2 *tmp, uint32_t *tval, hipStream_t s)
{
    if (n_tiles <= 0) return hipSuccess;
    tile_sort_kernel<<<n_tiles, kBlock, 0, s>>>(ranges, n_tiles, ent, tmp, tval);
    return hipGetLastError();
}

}  // namespace ddgs
