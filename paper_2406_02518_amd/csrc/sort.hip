// sort.hip -- scans and the hand-written stable LSD radix sort on gfx950:
// exclusive scans of u32 arrays (with 64-bit totals), the work items of the
// chunked raster, a stable LSD radix sort of (key, value) u32 pairs (the
// persistent raster's tile queue, the dual-sampling subsample, and an entry
// point of its own), and per-tile [start, end) ranges of a sorted key array.
// The tile lists of the render path are built by binning (bin.hip), which
// needs no global sort.
#include "internal.h"

namespace ddgs {

namespace {

constexpr int kBlock = 256;
constexpr int kScanIPT = kScanTile / kBlock;  // 16
// keys per thread of a radix block: 16 (4096 keys per block) for large sorts,
// 4 (1024 keys) below kRadixSmallN keys so that a pass still spreads over
// every compute unit.  (32 per thread, for longer write runs per digit, was
// measured slower on 64M keys: the scatter's 215 VGPRs halve occupancy.)
constexpr int kRadixIPTLarge = 16, kRadixIPTSmall = 4;
constexpr int64_t kRadixSmallN = (int64_t)2 << 20;
constexpr int kRadixMaxDigits = kSortTotWords;  // digit values of the widest (9-bit) pass
constexpr int kWaves = kBlock / kWave;

// exclusive scan over a block of 256 threads; returns the block total
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t *lds /* >= 4 */, uint32_t &total)
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

// ------------------------------------------------------------------- scan
// Two launches: per-block sums, then every block adds the sums of the blocks
// before it (read by the block itself, at most kScanSelfMax of them) to its
// own in-block exclusive scan.  Longer inputs scan the block sums in a third
// launch in between.  (Chained single-pass scans were measured slower here:
// every look-back hop is a cross-die round trip.)
constexpr int64_t kScanSelfMax = (int64_t)kBlock * 16;

// Scan inputs: a plain (optionally gathered) array, or the number of
// `split`-entry work items of each tile range.
struct PlainIn {
    const uint32_t *in, *gather;
    __device__ uint32_t operator()(int64_t i) const { return in[gather ? gather[i] : i]; }
};
struct ChunkIn {
    const uint2 *ranges;
    uint32_t split;
    __device__ uint32_t operator()(int64_t t) const
    {
        const uint2 r = ranges[t];
        return (r.y - r.x + split - 1u) / split;
    }
};

// The IPT inputs of a thread at base + q * kBlock + threadIdx.x, all read
// before any is used so that the loads overlap; indices are clamped to the
// last element (n > base), callers zero what lies past the end.
template <int IPT, class In>
__device__ __forceinline__ void load_inputs(const In &f, int64_t base, int64_t n, uint32_t (&x)[IPT])
{
#pragma unroll
    for (int q = 0; q < IPT; ++q) x[q] = f(min(base + q * kBlock + threadIdx.x, n - 1));
}
// (gathered input: every index first, then every value)
template <int IPT>
__device__ __forceinline__ void load_inputs(const PlainIn &f, int64_t base, int64_t n, uint32_t (&x)[IPT])
{
    if (f.gather) {
        uint32_t g[IPT];
#pragma unroll
        for (int q = 0; q < IPT; ++q) g[q] = f.gather[min(base + q * kBlock + threadIdx.x, n - 1)];
#pragma unroll
        for (int q = 0; q < IPT; ++q) x[q] = f.in[g[q]];
    } else {
#pragma unroll
        for (int q = 0; q < IPT; ++q) x[q] = f.in[min(base + q * kBlock + threadIdx.x, n - 1)];
    }
}

template <class In, int IPT>
__global__ __launch_bounds__(kBlock) void scan_reduce_kernel(In f, int64_t n, uint64_t *blocksum)
{
    const int64_t base = (int64_t)blockIdx.x * (kBlock * IPT);
    uint32_t x[IPT];
    load_inputs(f, base, n, x);
    uint64_t s = 0;
#pragma unroll
    for (int q = 0; q < IPT; ++q)
        if (base + q * kBlock + threadIdx.x < n) s += x[q];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, kWave);
    __shared__ uint64_t red[kWaves];
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
        for (int q = 0; q < kWaves; ++q) t += red[q];
        blocksum[blockIdx.x] = t;
    }
}

// single block: exclusive scan of the block sums with a running carry
__global__ __launch_bounds__(1024) void scan_top_kernel(uint64_t *blocksum, int64_t nb, uint64_t *total)
{
    __shared__ uint64_t wt[16];
    __shared__ uint64_t carry_s;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    if (threadIdx.x == 0) carry_s = 0;
    __syncthreads();
    for (int64_t c0 = 0; c0 < nb; c0 += 1024) {
        const int64_t idx = c0 + threadIdx.x;
        const uint64_t x = idx < nb ? blocksum[idx] : 0;
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
        if (idx < nb) blocksum[idx] = before + inc - x;
        __syncthreads();
        if (threadIdx.x == 0) carry_s += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0 && total) *total = carry_s;
}

// Scan outputs: the exclusive prefix, or the work items of each tile (its
// item count, first item, and the (tile, chunk) list; finish() stores the
// item count and clears the two work-queue counters).
struct PlainOut {
    uint32_t *out;
    __device__ void operator()(int64_t i, uint32_t pre, uint32_t) const { out[i] = pre; }
    __device__ void finish(uint64_t) const {}
};
struct ItemsOut {
    uint32_t *cnt, *base;
    uint2 *items;
    uint32_t max_items;
    uint32_t *n_items, *counter;
    __device__ void operator()(int64_t t, uint32_t pre, uint32_t v) const
    {
        cnt[t] = v;
        base[t] = pre;
        for (uint32_t k = 0; k < v && pre + k < max_items; ++k) items[pre + k] = make_uint2((uint32_t)t, k);
    }
    __device__ void finish(uint64_t total) const
    {
        *n_items = total > (uint64_t)max_items ? max_items : (uint32_t)total;
        counter[0] = 0;
        counter[1] = 0;
    }
};

// prescanned: blocksum holds exclusive block offsets (scan_top ran and wrote
// *total); otherwise the block sums the raw block sums before it, and the
// last block writes the total.
template <class In, class Out, int IPT>
__global__ __launch_bounds__(kBlock) void scan_apply_kernel(In f, int64_t n, const uint64_t *blocksum, int prescanned,
                                                            Out o, uint64_t *total)
{
    constexpr int TILE = kBlock * IPT;
    __shared__ uint32_t tile[TILE];
    __shared__ uint32_t vals[TILE];
    __shared__ uint32_t wl[kWaves];
    __shared__ uint64_t red[kWaves];
    const int64_t base = (int64_t)blockIdx.x * TILE;
    {
        uint32_t xs[IPT];
        load_inputs(f, base, n, xs);
#pragma unroll
        for (int q = 0; q < IPT; ++q) {
            const uint32_t x = base + q * kBlock + threadIdx.x < n ? xs[q] : 0u;
            tile[q * kBlock + threadIdx.x] = x;
            vals[q * kBlock + threadIdx.x] = x;
        }
    }
    uint64_t off;
    if (prescanned) {
        off = blocksum[blockIdx.x];
    } else {
        uint64_t s = 0;
        for (int j = threadIdx.x; j < (int)blockIdx.x; j += kBlock) s += blocksum[j];
#pragma unroll
        for (int k = 32; k > 0; k >>= 1) s += __shfl_xor(s, k, kWave);
        if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = s;
    }
    __syncthreads();
    if (!prescanned) {
        off = 0;
#pragma unroll
        for (int q = 0; q < kWaves; ++q) off += red[q];
    }
    if (threadIdx.x == 0 && blockIdx.x == gridDim.x - 1) {
        const uint64_t t = prescanned ? *total : off + blocksum[blockIdx.x];
        if (!prescanned && total) *total = t;
        o.finish(t);
    }
    uint32_t v[IPT], s = 0;
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        v[q] = tile[threadIdx.x * IPT + q];
        s += v[q];
    }
    uint32_t tot;
    uint32_t pre = block_excl_scan(s, wl, tot);
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        tile[threadIdx.x * IPT + q] = pre;
        pre += v[q];
    }
    __syncthreads();
    const uint32_t off32 = (uint32_t)off;
#pragma unroll 4
    for (int q = 0; q < IPT; ++q) {
        const int64_t idx = base + q * kBlock + threadIdx.x;
        if (idx < n) o(idx, off32 + tile[q * kBlock + threadIdx.x], vals[q * kBlock + threadIdx.x]);
    }
}

// ------------------------------------------------------------- radix sort
// One pass = three launches: per-block digit counts (digit-major), one block
// per digit turning its row into offsets across blocks plus the digit total,
// and the stable scatter, which adds the digit's start to its own offset.

__device__ __forceinline__ int64_t runtime_n(int64_t n_cap, const uint32_t *n_dev)
{
    if (!n_dev) return n_cap;
    const int64_t m = (int64_t)*n_dev;
    return m < n_cap ? m : n_cap;
}

// NB: digit values of a pass (256, or 512 where 9-bit digits save a pass)
template <int IPT, int NB>
__global__ __launch_bounds__(kBlock) void radix_count_kernel(const uint32_t *kin, int64_t n_cap, const uint32_t *n_dev,
                                                             int shift, uint32_t mask, uint32_t *counts, int nblocks)
{
    constexpr int kRadixTile = kBlock * IPT;
    __shared__ uint32_t h[kWaves][NB];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
#pragma unroll
    for (int q = 0; q < NB / kWave; ++q) h[w][lane + q * kWave] = 0;
    __syncthreads();
    const int64_t n = runtime_n(n_cap, n_dev);
    const int64_t wbase = (int64_t)blockIdx.x * kRadixTile + w * (kRadixTile / kWaves);
    // every round's key is loaded before the first is counted, so the loads
    // overlap (lanes past the end read the last key and count nothing)
    const int64_t last = n > 0 ? n - 1 : 0;
    uint32_t kk[IPT];
#pragma unroll
    for (int r = 0; r < IPT; ++r) kk[r] = kin[min(wbase + r * kWave + lane, last)];
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        const int64_t idx = wbase + r * kWave + lane;
        if (idx < n) atomicAdd(&h[w][(kk[r] >> shift) & mask], 1u);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < NB; d += kBlock)
        counts[(size_t)d * nblocks + blockIdx.x] = h[0][d] + h[1][d] + h[2][d] + h[3][d];
}

// Block d: exclusive scan of counts[d][0, nblocks) in place; tot[d] = row sum.
__global__ __launch_bounds__(kBlock) void radix_prefix_kernel(uint32_t *counts, int nblocks, uint32_t *tot)
{
    __shared__ uint32_t tile[kScanTile];
    __shared__ uint32_t wl[kWaves];
    uint32_t *row = counts + (size_t)blockIdx.x * nblocks;
    uint32_t carry = 0;
    for (int c0 = 0; c0 < nblocks; c0 += kScanTile) {
        __syncthreads();
#pragma unroll 4
        for (int q = 0; q < kScanIPT; ++q) {
            const int idx = c0 + q * kBlock + threadIdx.x;
            tile[q * kBlock + threadIdx.x] = idx < nblocks ? row[idx] : 0u;
        }
        __syncthreads();
        uint32_t v[kScanIPT], sum = 0;
#pragma unroll
        for (int q = 0; q < kScanIPT; ++q) {
            v[q] = tile[threadIdx.x * kScanIPT + q];
            sum += v[q];
        }
        uint32_t t;
        uint32_t pre = carry + block_excl_scan(sum, wl, t);
#pragma unroll
        for (int q = 0; q < kScanIPT; ++q) {
            tile[threadIdx.x * kScanIPT + q] = pre;
            pre += v[q];
        }
        __syncthreads();
#pragma unroll 4
        for (int q = 0; q < kScanIPT; ++q) {
            const int idx = c0 + q * kBlock + threadIdx.x;
            if (idx < nblocks) row[idx] = tile[q * kBlock + threadIdx.x];
        }
        carry += t;
    }
    if (threadIdx.x == 0) tot[blockIdx.x] = carry;
}

// Stable scatter: every wave ranks its IPT rounds of 64 consecutive keys with
// ballots (lanes sharing the digit), the block combines the 4 wave
// histograms, the keys are staged in LDS in digit order and written out
// with consecutive lanes on consecutive addresses.
template <int IPT, int NB>
__global__ __launch_bounds__(kBlock) void radix_scatter_kernel(const uint32_t *kin, const uint32_t *vin,
                                                               uint32_t *kout, uint32_t *vout, int64_t n_cap,
                                                               const uint32_t *n_dev, int shift, int nbits,
                                                               const uint32_t *offsets, const uint32_t *tot,
                                                               int nblocks, const uint32_t *gsrc, uint32_t *gdst)
{
    constexpr int kRadixTile = kBlock * IPT;
    constexpr int DPT = NB / kBlock;  // digits per thread in the block-wide steps
    __shared__ uint32_t wh[kWaves][NB];
    __shared__ uint32_t bstart[NB];
    __shared__ uint32_t gbase[NB];
    __shared__ uint32_t sk[kRadixTile];
    __shared__ uint32_t sv[kRadixTile];
    __shared__ uint32_t wl[kWaves];
    const int64_t n = runtime_n(n_cap, n_dev);
    const int64_t base = (int64_t)blockIdx.x * kRadixTile;
    if (base >= n) return;  // uniform over the block
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const uint32_t mask = (1u << nbits) - 1u;
#pragma unroll
    for (int q = 0; q < NB / kWave; ++q) wh[w][lane + q * kWave] = 0;
    __syncthreads();
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
    uint32_t key[IPT], val[IPT], rank[IPT];
    const int64_t wbase = base + w * (kRadixTile / kWaves);
    // all rounds' keys and values are loaded before the first is ranked, so
    // the loads overlap (lanes past the end read the last pair, n > base)
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        const int64_t li = min(wbase + r * kWave + lane, n - 1);
        key[r] = kin[li];
        val[r] = vin[li];
    }
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        const int64_t idx = wbase + r * kWave + lane;
        const bool ok = idx < n;
        const uint32_t d = (key[r] >> shift) & mask;
        uint64_t peers = __ballot(ok);
        for (int b = 0; b < nbits; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bal = __ballot(bit);
            peers &= bit ? bal : ~bal;
        }
        const uint32_t below = (uint32_t)__popcll(peers & lt_mask);
        uint32_t prev = 0;
        if (ok) prev = wh[w][d];
        __builtin_amdgcn_wave_barrier();
        if (ok && below == 0) wh[w][d] = prev + (uint32_t)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
        rank[r] = prev + below;
    }
    __syncthreads();
    {
        // thread t owns digits t DPT .. t DPT + DPT - 1, so the block scans
        // over threads run in digit order
        uint32_t csum[DPT], cs = 0, ts = 0;
#pragma unroll
        for (int j = 0; j < DPT; ++j) {
            const int d = threadIdx.x * DPT + j;
            const uint32_t c0 = wh[0][d], c1 = wh[1][d], c2 = wh[2][d], c3 = wh[3][d];
            wh[0][d] = 0;
            wh[1][d] = c0;
            wh[2][d] = c0 + c1;
            wh[3][d] = c0 + c1 + c2;
            csum[j] = c0 + c1 + c2 + c3;
            cs += csum[j];
            ts += tot[d];
        }
        uint32_t t;
        uint32_t bs = block_excl_scan(cs, wl, t);
        uint32_t ds = block_excl_scan(ts, wl, t);
#pragma unroll
        for (int j = 0; j < DPT; ++j) {
            const int d = threadIdx.x * DPT + j;
            bstart[d] = bs;
            gbase[d] = ds + offsets[(size_t)d * nblocks + blockIdx.x];
            bs += csum[j];
            ds += tot[d];
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        const int64_t idx = wbase + r * kWave + lane;
        if (idx < n) {
            const uint32_t d = (key[r] >> shift) & mask;
            const uint32_t pos = bstart[d] + wh[w][d] + rank[r];
            sk[pos] = key[r];
            sv[pos] = val[r];
        }
    }
    __syncthreads();
    const int cnt = (int)min((int64_t)kRadixTile, n - base);
    for (int j = threadIdx.x; j < cnt; j += kBlock) {
        const uint32_t kk = sk[j];
        const uint32_t d = (kk >> shift) & mask;
        const uint32_t o = gbase[d] + (uint32_t)j - bstart[d];
        kout[o] = kk;
        vout[o] = sv[j];
        if (gsrc) gdst[o] = gsrc[sv[j]];
    }
}

__global__ void zero_u64_kernel(uint64_t *p) { *p = 0; }

__global__ __launch_bounds__(kBlock) void fill_u32_kernel(uint32_t *p, uint32_t v, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ __launch_bounds__(kBlock) void copy_u32_kernel(uint32_t *dst, const uint32_t *src, const uint32_t *n_dev,
                                                          int64_t n_cap)
{
    const int64_t n = runtime_n(n_cap, n_dev);
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        dst[i] = src[i];
}

// Each thread takes kRangesIPT consecutive sorted keys (one 16-byte load
// where all four exist, plus the key before and the key after) and marks
// where a tile's run starts and ends.
constexpr int kRangesIPT = 4;

__global__ __launch_bounds__(kBlock) void ranges_kernel(const uint32_t *keys, const uint32_t *m_dev, int64_t m_cap,
                                                        uint2 *ranges, int n_tiles)
{
    const int64_t m = runtime_n(m_cap, m_dev);
    const int64_t stride = (int64_t)gridDim.x * kBlock * kRangesIPT;
    for (int64_t j0 = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * kRangesIPT; j0 < m; j0 += stride) {
        // k[q + 1] = keys[j0 + q]; k[0], k[kRangesIPT + 1]: the neighbours
        // (indices clamped into [0, m); the ends are tested by position)
        uint32_t k[kRangesIPT + 2];
        k[0] = keys[j0 > 0 ? j0 - 1 : 0];
        k[kRangesIPT + 1] = keys[j0 + kRangesIPT < m ? j0 + kRangesIPT : m - 1];
        if (j0 + kRangesIPT <= m) {
            const uint4 x = *reinterpret_cast<const uint4 *>(keys + j0);
            k[1] = x.x; k[2] = x.y; k[3] = x.z; k[4] = x.w;
        } else {
#pragma unroll
            for (int q = 1; q <= kRangesIPT; ++q) k[q] = keys[j0 - 1 + q < m ? j0 - 1 + q : m - 1];
        }
#pragma unroll
        for (int q = 0; q < kRangesIPT; ++q) {
            const int64_t j = j0 + q;
            const uint32_t kk = k[q + 1];
            if (j < m && kk < (uint32_t)n_tiles) {
                if (j == 0 || k[q] != kk) ranges[kk].x = (uint32_t)j;
                if (j == m - 1 || k[q + 2] != kk) ranges[kk].y = (uint32_t)(j + 1);
            }
        }
    }
}

__global__ __launch_bounds__(kBlock) void zero_ranges_kernel(uint2 *ranges, int n_tiles)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n_tiles) ranges[i] = make_uint2(0, 0);
}

int64_t blocks_for(int64_t n, int64_t per) { return (n + per - 1) / per; }

}  // namespace

int radix_ipt(int64_t n) { return n < kRadixSmallN ? kRadixIPTSmall : kRadixIPTLarge; }

// (monotone in n, so a workspace sized for n also serves every smaller sort)
size_t sort_counts_words(int64_t n)
{
    const int64_t small = blocks_for(std::min(n, kRadixSmallN), (int64_t)kBlock * kRadixIPTSmall);
    const int64_t large = blocks_for(n, (int64_t)kBlock * kRadixIPTLarge);
    return (size_t)kRadixMaxDigits * (size_t)std::max<int64_t>({1, small, large});
}
// (enough for the 256-per-block item scans too: their inputs are tile counts)
size_t sort_blocksum_words(int64_t n) { return (size_t)std::max<int64_t>(1, blocks_for(n, kBlock)) + 1; }

namespace {

// IPT values per thread: kScanIPT (4096 per block) for long inputs, 1 (256
// per block) where per-element output work dominates (the item lists)
template <int IPT, class In, class Out>
hipError_t scan_launch(In f, int64_t n, Out o, const SortWs &ws, uint64_t *total, hipStream_t s)
{
    const int64_t nb = blocks_for(n, (int64_t)kBlock * IPT);
    if (!ws.blocksum || (size_t)nb + 1 > ws.blocksum_words || nb > 0x7FFFFFFF) return hipErrorInvalidValue;
    scan_reduce_kernel<In, IPT><<<(unsigned)nb, kBlock, 0, s>>>(f, n, ws.blocksum);
    const bool pre = nb > kScanSelfMax;
    if (pre) scan_top_kernel<<<1, 1024, 0, s>>>(ws.blocksum, nb, total);
    scan_apply_kernel<In, Out, IPT><<<(unsigned)nb, kBlock, 0, s>>>(f, n, ws.blocksum, pre ? 1 : 0, o, total);
    return hipGetLastError();
}

// Work items in one launch for up to kItemsSelfMax tiles: block b (one tile
// per thread) first sums the item counts of the tiles before its own, read
// directly from the ranges, then scans its own; the last block stores the
// total.
constexpr int64_t kItemsSelfMax = 16384;

__global__ __launch_bounds__(kBlock) void items_self_kernel(ChunkIn f, int n, ItemsOut o, uint64_t *total)
{
    __shared__ uint32_t wl[kWaves];
    const int base = blockIdx.x * kBlock;
    uint32_t c = 0;
#pragma unroll 4
    for (int t = threadIdx.x; t < base; t += kBlock) c += f(t);
    uint32_t carry;
    (void)block_excl_scan(c, wl, carry);
    const int t = base + threadIdx.x;
    const uint32_t v = t < n ? f(t) : 0u;
    uint32_t tot;
    const uint32_t pre = carry + block_excl_scan(v, wl, tot);
    if (t < n) o(t, pre, v);
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
        if (total) *total = carry + tot;
        o.finish(carry + tot);
    }
}

__global__ void items_empty_kernel(uint32_t *n_items, uint32_t *counter)
{
    *n_items = 0;
    counter[0] = 0;
    counter[1] = 0;
}

}  // namespace

hipError_t launch_exclusive_scan(const uint32_t *in, const uint32_t *gather, uint32_t *out, int64_t n,
                                 const SortWs &ws, uint64_t *total, hipStream_t s)
{
    if (n == 0) return total ? launch_zero_u64(total, s) : hipSuccess;
    if (!total) return hipErrorInvalidValue;
    return scan_launch<kScanIPT>(PlainIn{in, gather}, n, PlainOut{out}, ws, total, s);
}

hipError_t launch_items(const uint2 *ranges, int n_tiles, int split, uint32_t *cnt, uint32_t *base, uint2 *items,
                        uint32_t max_items, const SortWs &ws, uint64_t *scan_total, uint32_t *n_items,
                        uint32_t *counter, hipStream_t s)
{
    if (split <= 0) return hipErrorInvalidValue;
    if (n_tiles == 0) {
        items_empty_kernel<<<1, 1, 0, s>>>(n_items, counter);
        return hipGetLastError();
    }
    const ChunkIn f{ranges, (uint32_t)split};
    const ItemsOut o{cnt, base, items, max_items, n_items, counter};
    if (n_tiles <= kItemsSelfMax) {
        items_self_kernel<<<(unsigned)blocks_for(n_tiles, kBlock), kBlock, 0, s>>>(f, n_tiles, o, scan_total);
        return hipGetLastError();
    }
    return scan_launch<1>(f, n_tiles, o, ws, scan_total, s);
}

hipError_t radix_sort_pairs(uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1, int64_t n_cap,
                            const uint32_t *n_dev, int bits, const SortWs &ws, bool *in_k1, hipStream_t s,
                            const uint32_t *gsrc, uint32_t *gdst)
{
    *in_k1 = false;
    if (n_cap <= 0 || bits <= 0) return hipSuccess;
    if (bits > 32 || !ws.counts || !ws.tot || sort_counts_words(n_cap) > ws.counts_words) return hipErrorInvalidValue;
    const int ipt = radix_ipt(n_cap);
    const int64_t nblocks = blocks_for(n_cap, (int64_t)kBlock * ipt);
    if (nblocks > 0x7FFFFFFF) return hipErrorInvalidValue;
    // passes of 8-bit digits, or of up to 9 bits (512 digit values) where that
    // takes fewer passes (9, 17 or 25 key bits), the bits then spread evenly
    // (three 11-bit passes for 32-bit keys were measured slower than four
    // 8-bit ones: the wider histograms cost more per pass than a pass saves)
    const int passes8 = (bits + 7) / 8, passes9 = (bits + 8) / 9;
    const bool wide = passes9 < passes8;
    const int passes = wide ? passes9 : passes8;
    uint32_t *ka = k0, *va = v0, *kb = k1, *vb = v1;
    int shift = 0;
    for (int p = 0; p < passes; ++p) {
        const int nbits = wide ? bits / passes + (p < bits % passes ? 1 : 0) : std::min(8, bits - shift);
        const uint32_t mask = (1u << nbits) - 1u;
        const bool last = p == passes - 1;
        const uint32_t *gs = last ? gsrc : nullptr;
        uint32_t *gd = last ? gdst : nullptr;
        auto pass = [&](auto ipt_c, auto nb_c) {
            constexpr int IPT = decltype(ipt_c)::value, NB = decltype(nb_c)::value;
            radix_count_kernel<IPT, NB><<<(unsigned)nblocks, kBlock, 0, s>>>(ka, n_cap, n_dev, shift, mask,
                                                                            ws.counts, (int)nblocks);
            radix_prefix_kernel<<<NB, kBlock, 0, s>>>(ws.counts, (int)nblocks, ws.tot);
            radix_scatter_kernel<IPT, NB><<<(unsigned)nblocks, kBlock, 0, s>>>(
                ka, va, kb, vb, n_cap, n_dev, shift, nbits, ws.counts, ws.tot, (int)nblocks, gs, gd);
        };
        using Small = std::integral_constant<int, kRadixIPTSmall>;
        using Large = std::integral_constant<int, kRadixIPTLarge>;
        using D8 = std::integral_constant<int, 256>;
        using D9 = std::integral_constant<int, kRadixMaxDigits>;
        if (ipt == kRadixIPTSmall) {
            if (wide) pass(Small{}, D9{});
            else pass(Small{}, D8{});
        } else {
            if (wide) pass(Large{}, D9{});
            else pass(Large{}, D8{});
        }
        shift += nbits;
        std::swap(ka, kb);
        std::swap(va, vb);
        *in_k1 = !*in_k1;
    }
    return hipGetLastError();
}

hipError_t launch_ranges(const uint32_t *keys, const uint32_t *m_dev, int64_t m_cap, uint2 *ranges, int n_tiles,
                         bool zero, hipStream_t s)
{
    if (zero && n_tiles > 0) zero_ranges_kernel<<<(unsigned)blocks_for(n_tiles, kBlock), kBlock, 0, s>>>(ranges, n_tiles);
    if (m_cap > 0) {
        const int64_t nb = std::min<int64_t>(blocks_for(m_cap, (int64_t)kBlock * kRangesIPT), 65536);
        ranges_kernel<<<(unsigned)nb, kBlock, 0, s>>>(keys, m_dev, m_cap, ranges, n_tiles);
    }
    return hipGetLastError();
}

hipError_t launch_zero_u64(uint64_t *p, hipStream_t s)
{
    zero_u64_kernel<<<1, 1, 0, s>>>(p);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    fill_u32_kernel<<<(unsigned)blocks_for(n, kBlock), kBlock, 0, s>>>(p, v, n);
    return hipGetLastError();
}

hipError_t launch_copy_u32(uint32_t *dst, const uint32_t *src, const uint32_t *n_dev, int64_t n_cap, hipStream_t s)
{
    if (n_cap <= 0) return hipSuccess;
    const int64_t nb = std::min<int64_t>(blocks_for(n_cap, kBlock), 65536);
    copy_u32_kernel<<<(unsigned)nb, kBlock, 0, s>>>(dst, src, n_dev, n_cap);
    return hipGetLastError();
}

}  // namespace ddgs
