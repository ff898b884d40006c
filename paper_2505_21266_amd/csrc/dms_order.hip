// dms_order.hip -- global vertex order (Section 2.1; Array Preconditioning,
// Section 3) as a stable least-significant-digit radix sort of
// (value key, vertex id) pairs on one GPU.
//
// The paper sorts (value, global id, owner) tuples with a distributed sort;
// on one GPU the same order comes from a stable LSD radix sort: vertices start
// in id order, every pass is stable, so equal values stay in id order, which
// is exactly the tie-break of Section 2.1.  Values become order-preserving
// unsigned keys (-0.0 -> +0.0; NaN flagged).  8-bit digits: 4 passes for
// float32, 8 for float64.  The last pass hands each vertex's final position
// to order[id] through (id, position) pairs grouped into 256 id buckets, so
// that the inversion's scattered writes stay inside a window of a few
// buckets instead of covering the whole order array.
//
// Each pass: (1) per-tile digit histograms (LDS atomics), (2) a device-wide
// exclusive scan of the digit-major histogram matrix, (3) a stable per-tile
// scatter.  Tiles
// hold 4096 keys (256 threads x 16 items, wave-striped so that a wave's items
// are in element order); ranks inside a wave come from ballot-based digit
// matching, ranks across waves from per-wave digit counts in LDS.
#include "dms_common.hpp"
#include "dms_internal.hpp"
#include "dms_scan.hpp"

namespace dms {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / kWave;
constexpr int kItems = 16;
constexpr int kTile = kThreads * kItems;
constexpr int kRadix = 256;

// Key types: uint32_t for float32, uint64_t for float64 and for batches
// (field index in bits 32..39 above the float32 key).
constexpr int kBatchPasses = 5;

// field of element i: the last f with foff[f] <= i (binary search)
__device__ __forceinline__ int field_of(const int64_t *foff, int nfields, int64_t i)
{
    int lo = 0, hi = nfields - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (foff[mid] <= i) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Tile processed by this block.  Blocks are dealt round-robin to the 8 XCDs
// (each with its own L2); giving each XCD a contiguous range of tiles lets
// neighbouring tiles, whose digit runs share cache lines, merge in one L2.
__device__ __forceinline__ int64_t tile_of_block(int64_t ntiles)
{
    const int64_t b = blockIdx.x;
    const int64_t per = ntiles / 8;
    if (per == 0 || b >= 8 * per) return b;  // the ragged tail keeps its place
    return (b % 8) * per + b / 8;
}

__device__ __forceinline__ int64_t elem_index(int64_t tile, int wave, int k, int lane)
{
    return tile * kTile + (int64_t)wave * (kItems * kWave) + k * kWave + lane;
}

// Histogram update for one item per lane (counts only, no ranks): an LDS
// atomic per lane, or a single add when the whole wave holds one digit, as
// it does for the high key bytes of smooth fields.
__device__ __forceinline__ void hist_add(uint32_t *h, uint32_t d, bool valid)
{
    const uint64_t act = __ballot(valid);
    if (act == 0) return;
    const uint32_t d0 = __builtin_amdgcn_readfirstlane(valid ? d : 0xffffffffu);
    const uint64_t same = __ballot(valid && d == d0);
    if (same == act) {
        if (lane_id() == (int)__builtin_ctzll(act)) atomicAdd(&h[d0], (uint32_t)__popcll(act));
    } else if (valid) {
        atomicAdd(&h[d], 1u);
    }
}

template <typename V, typename K, bool kFirst>
__device__ __forceinline__ K load_key(const void *src, int64_t i, bool &nan)
{
    if constexpr (kFirst) {
        return (K)key_of(((const V *)src)[i], nan);
    } else {
        nan = false;
        return ((const K *)src)[i];
    }
}

// (1) per-tile histogram of the digit at `shift`; counts is digit-major:
// counts[d * ntiles + tile].
// With ids != null (the last pass) it also histograms the vertex ids by
// bucket (id >> bshift) into bcounts, for the grouped inversion.
template <typename V, typename K, bool kFirst>
__global__ __launch_bounds__(kThreads) void k_tile_hist(const void *src, int64_t n, int shift,
                                                        uint32_t *counts, int64_t ntiles,
                                                        uint32_t *flags, const uint32_t *ids,
                                                        int bshift, uint32_t *bcounts)
{
    __shared__ uint32_t hist[kWaves][kRadix];
    __shared__ uint32_t bhist[kWaves][kRadix];
    const int tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
    for (int i = tid; i < kWaves * kRadix; i += kThreads) {
        (&hist[0][0])[i] = 0;
        (&bhist[0][0])[i] = 0;
    }
    __syncthreads();
    const int64_t tile = tile_of_block(ntiles);
    bool nan_any = false;
    uint32_t dig[kItems];
    if (ids) {
        uint32_t bk[kItems];
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            const int64_t i = elem_index(tile, wave, k, lane);
            bk[k] = i < n ? (ids[i] >> bshift) & (kRadix - 1) : (uint32_t)kRadix;
        }
#pragma unroll
        for (int k = 0; k < kItems; ++k) hist_add(bhist[wave], bk[k], bk[k] < (uint32_t)kRadix);
    }
#pragma unroll
    for (int k = 0; k < kItems; ++k) {  // all loads first
        const int64_t i = elem_index(tile, wave, k, lane);
        dig[k] = kRadix;
        if (i < n) {
            bool nan;
            K key = load_key<V, K, kFirst>(src, i, nan);
            nan_any |= nan;
            dig[k] = (uint32_t)(key >> shift) & (kRadix - 1);
        }
    }
#pragma unroll
    for (int k = 0; k < kItems; ++k) hist_add(hist[wave], dig[k], dig[k] < (uint32_t)kRadix);
    __syncthreads();
    uint32_t tot = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) tot += hist[w][tid];
    counts[(int64_t)tid * ntiles + tile] = tot;  // digit-major, tiles in tile order
    if (ids) {
        uint32_t bt = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) bt += bhist[w][tid];
        bcounts[(int64_t)tid * ntiles + tile] = bt;
    }
    if (kFirst && __ballot(nan_any) && lane == 0) atomicOr(flags, (uint32_t)DMS_FLAG_NAN);
}

// Rank of an item among the wave's items with the same 8-bit digit, counting
// this k and all earlier ones; wh is the wave's row of counts.  Items of a
// wave are in element order (k major, lane minor), so ranks are stable.
__device__ __forceinline__ uint32_t wave_rank(uint32_t d, bool valid, uint32_t *wh)
{
    const uint64_t peers = match_digit8(d, __ballot(valid));
    uint32_t base = 0;
    if (valid) base = wh[d];
    const uint32_t below = (uint32_t)__popcll(peers & lanemask_lt());
    if (valid && below == 0) wh[d] = base + (uint32_t)__popcll(peers);
    return base + below;
}

// Thread tid owns digit tid: the per-wave counts become exclusive prefixes
// over the waves; returns the tile's count of the digit.
__device__ __forceinline__ uint32_t wave_prefix(uint32_t (*wh)[kRadix])
{
    static_assert(kRadix == kThreads, "one thread per digit");
    const int tid = threadIdx.x;
    uint32_t run = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        const uint32_t c = wh[w][tid];
        wh[w][tid] = run;
        run += c;
    }
    return run;
}

// (3) stable scatter of one tile by the digit at `shift`.  offsets holds the
// scanned counts (global start of digit d in tile `tile`).
// foff (nfields + 1 offsets) is non-null for batches: the first pass puts
// the field index above the value key.
template <typename V, typename K, bool kFirst>
__global__ __launch_bounds__(kThreads) void k_scatter(const void *src, const uint32_t *src_ids,
                                                      int64_t n, int shift,
                                                      const uint32_t *offsets, int64_t ntiles,
                                                      K *dst_keys, uint32_t *dst_ids,
                                                      const int64_t *foff, int nfields)
{
    __shared__ uint32_t whist[kWaves][kRadix];
    __shared__ uint32_t digit_start[kRadix];
    __shared__ uint32_t gbase[kRadix];
    __shared__ K skey[kTile];
    __shared__ uint32_t sid[kTile];

    const int tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
    for (int i = tid; i < kWaves * kRadix; i += kThreads) (&whist[0][0])[i] = 0;
    __syncthreads();

    const int64_t tile = tile_of_block(ntiles);
    K key[kItems];
    uint32_t id[kItems];
    uint32_t rank[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int64_t i = elem_index(tile, wave, k, lane);
        const bool valid = i < n;
        key[k] = 0;
        id[k] = 0;
        if (valid) {
            bool nan;
            key[k] = load_key<V, K, kFirst>(src, i, nan);
            if constexpr (kFirst && sizeof(K) == 8) {
                if (foff) key[k] |= (K)field_of(foff, nfields, i) << 32;
            }
            id[k] = kFirst ? (uint32_t)i : src_ids[i];
        }
        rank[k] = wave_rank((uint32_t)(key[k] >> shift) & (kRadix - 1), valid, whist[wave]);
    }
    __syncthreads();
    {
        uint32_t total;
        digit_start[tid] = block_exclusive_scan<uint32_t>(wave_prefix(whist), &total);
        gbase[tid] = offsets[(int64_t)tid * ntiles + tile];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int64_t i = elem_index(tile, wave, k, lane);
        if (i < n) {
            const uint32_t d = (uint32_t)(key[k] >> shift) & (kRadix - 1);
            const uint32_t pos = digit_start[d] + whist[wave][d] + rank[k];
            skey[pos] = key[k];
            sid[pos] = id[k];
        }
    }
    __syncthreads();
    const int64_t left = n - tile * kTile;
    const int count = left < kTile ? (int)left : kTile;
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        const int p = tid + j * kThreads;
        if (p < count) {
            const K kk = skey[p];
            const uint32_t d = (uint32_t)(kk >> shift) & (kRadix - 1);
            const uint32_t g = gbase[d] + (uint32_t)(p - (int)digit_start[d]);
            // the ranks make g < n; the guard keeps any breach of that in bounds
            if ((int64_t)g < n) {
                dst_keys[g] = kk;
                dst_ids[g] = sid[p];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Inverting the sorted sequence into order[id] = position.
//
// Writing order[id] straight from the last pass would scatter 4-byte writes
// over the whole array.  Instead the position is carried as an (id, position)
// pair and the pairs are grouped by id in up to two partition levels, after
// which each window of ids is assembled in LDS and written out contiguously.
// Since the ids are a permutation of [0, n), bucket b of width 2^s holds
// exactly the ids [b 2^s, (b+1) 2^s) and so starts at position b 2^s: the
// bucket layout needs no counting, only each tile's place inside a bucket.
//   level 0 (last radix pass): 256 coarse buckets, id >> bshift;
//   level 1 (when a coarse bucket is wider than one LDS window): a stable
//     partition of each coarse bucket by the fine digit (id >> fshift) & (F-1);
//   window: one block per 2^wshift ids.
struct InvertPlan {
    int bshift;       // coarse bucket = id >> bshift (at most 256 buckets)
    bool fine;        // level 1 runs
    int fshift, flog; // fine digit = (id >> fshift) & ((1 << flog) - 1)
    int qlog;         // log2 of the kTile chunks per coarse bucket
    int64_t nchunks;  // level-1 chunks, ncb << qlog
    int wshift;       // LDS window = 2^wshift ids
};

constexpr int kTileLog = 12;
static_assert((1 << kTileLog) == kTile, "tile size");
constexpr int kMaxWinLog = 14;  // 64 KiB window: two blocks share a CU's LDS;
                                // only n > 2^30 needs 2^15 (128 KiB)

InvertPlan invert_plan(int64_t n)
{
    InvertPlan P{};
    int bits = 0;
    while (bits < 31 && (1ll << bits) < n) ++bits;
    P.bshift = bits > 8 ? bits - 8 : 0;
    const int64_t ncb = (n + (1ll << P.bshift) - 1) >> P.bshift;
    P.fine = P.bshift > kMaxWinLog;
    if (P.fine) {
        P.fshift = P.bshift - 8 > kMaxWinLog ? P.bshift - 8 : kMaxWinLog;
        P.flog = P.bshift - P.fshift;
        P.qlog = P.bshift - kTileLog;
        P.nchunks = ncb << P.qlog;
        P.wshift = P.fshift;
    } else {
        P.wshift = P.bshift;
    }
    return P;
}

// Level 0: the last radix pass.  Each item's final position g comes from the
// digit ranks as in k_scatter; the tile is then re-ranked by coarse bucket
// and staged in LDS in bucket order, so that a bucket's pairs from this tile
// leave as one contiguous run at the bucket's scanned offset (boffsets).
// For batches the position is taken relative to the field's first vertex.
template <typename K>
__global__ __launch_bounds__(kThreads) void k_scatter_last(const K *src, const uint32_t *src_ids,
                                                           int64_t n, int shift,
                                                           const uint32_t *offsets,
                                                           const uint32_t *boffsets, int64_t ntiles,
                                                           const int64_t *foff, int bshift,
                                                           uint32_t *pair_id, int32_t *pair_pos)
{
    __shared__ uint32_t dwh[kWaves][kRadix];
    __shared__ uint32_t bwh[kWaves][kRadix];
    __shared__ uint32_t gbase[kRadix];
    __shared__ uint32_t bstart[kRadix];
    __shared__ uint32_t bbase[kRadix];
    __shared__ uint32_t sid[kTile];
    __shared__ int32_t spos[kTile];

    const int tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
    for (int i = tid; i < kWaves * kRadix; i += kThreads) {
        (&dwh[0][0])[i] = 0;
        (&bwh[0][0])[i] = 0;
    }
    __syncthreads();

    const int64_t tile = tile_of_block(ntiles);
    // per item after the ranking: id, (digit rank | digit << 16) and
    // (bucket rank | field << 16); ranks are below kTile = 2^12
    uint32_t id[kItems], dr[kItems], br[kItems];
    {
        K key[kItems];
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            const int64_t i = elem_index(tile, wave, k, lane);
            const bool valid = i < n;
            key[k] = valid ? src[i] : K(0);
            id[k] = valid ? src_ids[i] : 0u;
        }
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            const bool valid = elem_index(tile, wave, k, lane) < n;
            const uint32_t d = (uint32_t)(key[k] >> shift) & (kRadix - 1);
            dr[k] = wave_rank(d, valid, dwh[wave]) | d << 16;
            uint32_t field = 0;
            if constexpr (sizeof(K) == 8) field = (uint32_t)(key[k] >> 32);
            br[k] = wave_rank((id[k] >> bshift) & (kRadix - 1), valid, bwh[wave]) | field << 16;
        }
    }
    __syncthreads();
    {
        wave_prefix(dwh);
        uint32_t total;
        bstart[tid] = block_exclusive_scan<uint32_t>(wave_prefix(bwh), &total);
        gbase[tid] = offsets[(int64_t)tid * ntiles + tile];
        bbase[tid] = boffsets[(int64_t)tid * ntiles + tile];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        if (elem_index(tile, wave, k, lane) < n) {
            const uint32_t d = dr[k] >> 16;
            const uint32_t b = (id[k] >> bshift) & (kRadix - 1);
            const int64_t g = (int64_t)gbase[d] + dwh[wave][d] + (dr[k] & 0xffffu);
            int64_t base = 0;
            if constexpr (sizeof(K) == 8) {
                if (foff) base = foff[br[k] >> 16];
            }
            const uint32_t pos = bstart[b] + bwh[wave][b] + (br[k] & 0xffffu);
            if (pos < (uint32_t)kTile) {
                sid[pos] = id[k];
                spos[pos] = (int32_t)(g - base);
            }
        }
    }
    __syncthreads();
    const int64_t left = n - tile * kTile;
    const int count = left < kTile ? (int)left : kTile;
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        const int p = tid + j * kThreads;
        if (p < count) {
            const uint32_t who = sid[p];
            const uint32_t b = (who >> bshift) & (kRadix - 1);
            const int64_t dst = (int64_t)bbase[b] + (p - (int)bstart[b]);
            if (dst < n) {
                pair_id[dst] = who;
                pair_pos[dst] = spos[p];
            }
        }
    }
}

// Level 1 counts: chunk c (kTile positions) lies in coarse bucket c >> qlog;
// counts are coarse-bucket major, then fine digit, then chunk, so that one
// exclusive scan gives every chunk its output offset for every fine digit.
__device__ __forceinline__ int64_t fine_count_index(int64_t c, int f, int flog, int qlog)
{
    const int64_t cb = c >> qlog, q = c & ((1ll << qlog) - 1);
    return (((cb << flog) | f) << qlog) | q;
}

__global__ __launch_bounds__(kThreads) void k_fine_hist(const uint32_t *pair_id, int64_t n,
                                                        int fshift, int flog, int qlog,
                                                        int64_t nchunks, uint32_t *counts)
{
    __shared__ uint32_t hist[kWaves][kRadix];
    const int tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
    for (int i = tid; i < kWaves * kRadix; i += kThreads) (&hist[0][0])[i] = 0;
    __syncthreads();
    const int64_t c = tile_of_block(nchunks);
    const uint32_t fmask = (1u << flog) - 1u;
    uint32_t dig[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int64_t i = elem_index(c, wave, k, lane);
        dig[k] = i < n ? (pair_id[i] >> fshift) & fmask : (uint32_t)kRadix;
    }
#pragma unroll
    for (int k = 0; k < kItems; ++k) hist_add(hist[wave], dig[k], dig[k] < (uint32_t)kRadix);
    __syncthreads();
    if (tid <= (int)fmask) {
        uint32_t tot = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) tot += hist[w][tid];
        counts[fine_count_index(c, tid, flog, qlog)] = tot;
    }
}

__global__ __launch_bounds__(kThreads) void k_fine_scatter(const uint32_t *in_id, const int32_t *in_pos,
                                                           int64_t n, int fshift, int flog, int qlog,
                                                           int64_t nchunks, const uint32_t *offsets,
                                                           uint32_t *out_id, int32_t *out_pos)
{
    __shared__ uint32_t wh[kWaves][kRadix];
    __shared__ uint32_t dstart[kRadix];
    __shared__ uint32_t gbase[kRadix];
    __shared__ uint32_t sid[kTile];
    __shared__ int32_t spos[kTile];

    const int tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
    for (int i = tid; i < kWaves * kRadix; i += kThreads) (&wh[0][0])[i] = 0;
    __syncthreads();
    const int64_t c = tile_of_block(nchunks);
    const uint32_t fmask = (1u << flog) - 1u;
    uint32_t id[kItems], r[kItems];
    int32_t pos[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int64_t i = elem_index(c, wave, k, lane);
        const bool valid = i < n;
        id[k] = valid ? in_id[i] : 0u;
        pos[k] = valid ? in_pos[i] : 0;
    }
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const bool valid = elem_index(c, wave, k, lane) < n;
        r[k] = wave_rank((id[k] >> fshift) & fmask, valid, wh[wave]);
    }
    __syncthreads();
    {
        uint32_t total;
        dstart[tid] = block_exclusive_scan<uint32_t>(wave_prefix(wh), &total);
        gbase[tid] = tid <= (int)fmask ? offsets[fine_count_index(c, tid, flog, qlog)] : 0u;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        if (elem_index(c, wave, k, lane) < n) {
            const uint32_t d = (id[k] >> fshift) & fmask;
            const uint32_t at = dstart[d] + wh[wave][d] + r[k];
            if (at < (uint32_t)kTile) {
                sid[at] = id[k];
                spos[at] = pos[k];
            }
        }
    }
    __syncthreads();
    const int64_t left = n - c * kTile;
    const int count = left <= 0 ? 0 : (left < kTile ? (int)left : kTile);
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        const int p = tid + j * kThreads;
        if (p < count) {
            const uint32_t who = sid[p];
            const uint32_t d = (who >> fshift) & fmask;
            const int64_t dst = (int64_t)gbase[d] + (p - (int)dstart[d]);
            if (dst < n) {
                out_id[dst] = who;
                out_pos[dst] = spos[p];
            }
        }
    }
}

// Window w holds the pairs of ids [w 2^wshift, (w+1) 2^wshift): the block
// places the positions into LDS by id, then writes the window contiguously.
constexpr int kInvThreads = 1024;
constexpr int kInvUnroll = 4;

template <int kWinLog>
__global__ __launch_bounds__(kInvThreads) void k_invert_window(const uint32_t *__restrict__ pair_id,
                                                               const int32_t *__restrict__ pair_pos,
                                                               int64_t n, int wshift,
                                                               int32_t *__restrict__ order)
{
    __shared__ int32_t win[1 << kWinLog];
    if (wshift > kWinLog) return;  // the host picks an instance that fits
    const int64_t base = (int64_t)blockIdx.x << wshift;
    const int64_t left = n - base;
    const int cnt = left < (1ll << wshift) ? (int)left : (1 << wshift);
    for (int i0 = 0; i0 < cnt; i0 += kInvThreads * kInvUnroll) {
        uint32_t v[kInvUnroll];
        int32_t r[kInvUnroll];
#pragma unroll
        for (int u = 0; u < kInvUnroll; ++u) {
            const int i = i0 + u * kInvThreads + (int)threadIdx.x;
            v[u] = i < cnt ? pair_id[base + i] : 0xffffffffu;
            r[u] = i < cnt ? pair_pos[base + i] : 0;
        }
#pragma unroll
        for (int u = 0; u < kInvUnroll; ++u) {
            const int64_t off = (int64_t)v[u] - base;
            if (off >= 0 && off < cnt) win[off] = r[u];
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < cnt; i += kInvThreads) order[base + i] = win[i];
}

struct OrderLayout {
    size_t keys0, keys1, ids0, ids1, counts, partials, bcounts, bpartials, total;
};

template <typename K>
OrderLayout order_layout(int64_t n)
{
    const int64_t ntiles = (n + kTile - 1) / kTile;
    const InvertPlan P = invert_plan(n);
    const int64_t chunks = P.fine && P.nchunks > ntiles ? P.nchunks : ntiles;
    const int64_t clen = chunks * kRadix;
    const int64_t blen = ntiles * kRadix;
    OrderLayout L{};
    size_t off = 0;
    L.keys0 = off; off += align_up((size_t)n * sizeof(K), 256);
    L.keys1 = off; off += align_up((size_t)n * sizeof(K), 256);
    L.ids0 = off; off += align_up((size_t)n * 4, 256);
    L.ids1 = off; off += align_up((size_t)n * 4, 256);
    L.counts = off; off += align_up((size_t)clen * 4, 256);
    L.partials = off; off += scan_partials_bytes(clen, 4);
    L.bcounts = off; off += align_up((size_t)blen * 4, 256);
    L.bpartials = off; off += scan_partials_bytes(blen, 4);
    L.total = off;
    return L;
}

template <typename V, typename K>
int run_order(const void *values, int64_t n, int passes, int32_t *order, char *ws, uint32_t *flags,
              const int64_t *foff, int nfields, hipStream_t s)
{
    if (passes < 2) return DMS_E_ARG;
    const OrderLayout L = order_layout<K>(n);
    const InvertPlan P = invert_plan(n);
    const int64_t ntiles = (n + kTile - 1) / kTile;
    K *keys[2] = {(K *)(ws + L.keys0), (K *)(ws + L.keys1)};
    uint32_t *ids[2] = {(uint32_t *)(ws + L.ids0), (uint32_t *)(ws + L.ids1)};
    uint32_t *counts = (uint32_t *)(ws + L.counts);
    uint32_t *partials = (uint32_t *)(ws + L.partials);
    uint32_t *bcounts = (uint32_t *)(ws + L.bcounts);
    uint32_t *bpartials = (uint32_t *)(ws + L.bpartials);
    const dim3 grid((unsigned)ntiles), block(kThreads);
    for (int p = 0; p < passes; ++p) {
        const int shift = 8 * p;
        const bool last = p == passes - 1;
        const void *src = p == 0 ? values : (const void *)keys[(p - 1) & 1];
        const uint32_t *sids = p == 0 ? nullptr : ids[(p - 1) & 1];
        if (p == 0)
            hipLaunchKernelGGL((k_tile_hist<V, K, true>), grid, block, 0, s, src, n, shift, counts,
                               ntiles, flags, nullptr, 0, nullptr);
        else
            hipLaunchKernelGGL((k_tile_hist<V, K, false>), grid, block, 0, s, src, n, shift, counts,
                               ntiles, flags, last ? sids : nullptr, P.bshift, bcounts);
        exclusive_scan<uint32_t>(counts, ntiles * kRadix, partials, s);
        if (!last) {
            if (p == 0)
                hipLaunchKernelGGL((k_scatter<V, K, true>), grid, block, 0, s, src, sids, n, shift,
                                   counts, ntiles, keys[p & 1], ids[p & 1], foff, nfields);
            else
                hipLaunchKernelGGL((k_scatter<V, K, false>), grid, block, 0, s, src, sids, n, shift,
                                   counts, ntiles, keys[p & 1], ids[p & 1], foff, nfields);
            continue;
        }
        exclusive_scan<uint32_t>(bcounts, ntiles * kRadix, bpartials, s);
        // level 0 into the free buffers; level 1 back into the last pass's
        // source buffers once they are read
        uint32_t *aid = (uint32_t *)keys[p & 1];
        int32_t *apos = (int32_t *)ids[p & 1];
        hipLaunchKernelGGL((k_scatter_last<K>), grid, block, 0, s, (const K *)src, sids, n, shift,
                           counts, bcounts, ntiles, foff, P.bshift, aid, apos);
        if (P.fine) {
            uint32_t *fid = (uint32_t *)keys[(p - 1) & 1];
            int32_t *fpos = (int32_t *)ids[(p - 1) & 1];
            const dim3 cgrid((unsigned)P.nchunks);
            hipLaunchKernelGGL(k_fine_hist, cgrid, block, 0, s, aid, n, P.fshift, P.flog, P.qlog,
                               P.nchunks, counts);
            exclusive_scan<uint32_t>(counts, P.nchunks << P.flog, partials, s);
            hipLaunchKernelGGL(k_fine_scatter, cgrid, block, 0, s, aid, apos, n, P.fshift, P.flog,
                               P.qlog, P.nchunks, counts, fid, fpos);
            aid = fid;
            apos = fpos;
        }
        const int64_t nwin = (n + (1ll << P.wshift) - 1) >> P.wshift;
        if (P.wshift <= kMaxWinLog)
            hipLaunchKernelGGL(k_invert_window<kMaxWinLog>, dim3((unsigned)nwin), dim3(kInvThreads), 0,
                               s, aid, apos, n, P.wshift, order);
        else if (P.wshift == kMaxWinLog + 1)
            hipLaunchKernelGGL(k_invert_window<kMaxWinLog + 1>, dim3((unsigned)nwin),
                               dim3(kInvThreads), 0, s, aid, apos, n, P.wshift, order);
        else
            return DMS_E_SIZE;
    }
    return launch_status();
}

}  // namespace

size_t order_batch_workspace_size(int64_t n) { return order_layout<uint64_t>(n > 0 ? n : 1).total; }

int launch_order_batch(const float *values, int64_t n, const int64_t *foff, int nfields,
                       int32_t *order, char *ws, uint32_t *flags, hipStream_t s)
{
    if (n == 0) return DMS_OK;
    return run_order<float, uint64_t>(values, n, kBatchPasses, order, ws, flags, foff, nfields, s);
}

}  // namespace dms

extern "C" size_t dms_order_workspace_size(int64_t n, int dtype)
{
    if (n <= 0) return 256;
    if (dtype == DMS_F32) return dms::order_layout<uint32_t>(n).total;
    if (dtype == DMS_F64) return dms::order_layout<uint64_t>(n).total;
    return 0;
}

extern "C" int dms_order(const void *values, int dtype, int64_t n, int32_t *order, void *workspace,
                         size_t workspace_bytes, uint32_t *dev_flags, void *stream)
{
    if (n < 0 || (dtype != DMS_F32 && dtype != DMS_F64)) return DMS_E_ARG;
    if (n > 2147483647LL) return DMS_E_SIZE;
    if (n == 0) return DMS_OK;
    if (!values || !order || !dev_flags) return DMS_E_ARG;
    if (!workspace || workspace_bytes < dms_order_workspace_size(n, dtype)) return DMS_E_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    if (dtype == DMS_F32)
        return dms::run_order<float, uint32_t>(values, n, 4, order, (char *)workspace, dev_flags,
                                               nullptr, 0, s);
    return dms::run_order<double, uint64_t>(values, n, 8, order, (char *)workspace, dev_flags, nullptr,
                                            0, s);
}
