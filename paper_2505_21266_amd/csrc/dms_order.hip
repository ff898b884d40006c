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
// scatter.  A tile holds 16 items per thread (8192 keys in 512-thread blocks
// for 4-byte keys, 4096 in 256-thread blocks for 8-byte keys), wave-striped
// so that a wave's items are in element order; ranks inside a wave come from
// digit matching (LDS lane masks or ballots), ranks across waves from
// per-wave digit counts in LDS.
#include "dms_common.hpp"
#include "dms_internal.hpp"
#include "dms_scan.hpp"

#include <type_traits>

namespace dms {
namespace {

constexpr int kThreads = 256;
constexpr int kItems = 16;
constexpr int kTile = kThreads * kItems;
constexpr int kRadix = 256;
// The radix passes run 512-thread blocks (8192-key tiles) for 4-byte keys: a
// tile's run of one digit (or, in the last pass, of one id bucket) is then
// about 32 keys, a whole 128-byte line, and the scattered writes cost less
// (about 0.1 ms per histogram and 0.5-0.7 ms per scatter at 2^30 keys).
// 8-byte keys keep 256 threads: two 512-thread blocks of those would not fit
// one CU's LDS and registers.  The fine partition of the inversion keeps 256.
constexpr int kWideThreads = 512;

// Key types: uint32_t for float32, uint64_t for float64 and for batches
// (field index from bit 32 up, above the float32 key): a batch sorts the four
// value bytes and then as many bytes of the field index as the number of
// fields needs.
__host__ __device__ constexpr int batch_passes(int nfields)
{
    int p = 4;
    for (int64_t span = 1; span < nfields; span <<= 8) ++p;
    return p < 5 ? 5 : p;
}
static_assert(batch_passes(1) == 5 && batch_passes(256) == 5 && batch_passes(257) == 6 &&
                  batch_passes(kMaxBatchFields) == 6,
              "field bytes sorted by a batch");

// field of element i: the last f in [lo, hi] with foff[f] <= i (binary
// search; the caller knows i lies in one of fields lo..hi)
__device__ __forceinline__ int field_between(const int64_t *foff, int lo, int hi, int64_t i)
{
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (foff[mid] <= i) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int field_of(const int64_t *foff, int nfields, int64_t i)
{
    return field_between(foff, 0, nfields - 1, i);
}

// Coarse field table of a field pass, in LDS: entry j is the field of vertex
// j << s (of the last vertex for entries past it), s being the smallest shift
// that keeps the entries for [0, n) plus one within kFieldTable.  Vertex v's
// field lies between entries v >> s and (v >> s) + 1: one or two fields unless
// fields are shorter than 2^s vertices, in place of a search over all of them.
constexpr int kFieldTable = 1024;

__device__ __forceinline__ int field_table_shift(int64_t n)
{
    int s = 0;
    while (((n - 1) >> s) + 2 > kFieldTable) ++s;
    return s;
}

// The block fills tab from the LDS field offsets fo (n >= 1).
__device__ __forceinline__ void build_field_table(uint16_t *tab, const int64_t *fo, int nfields, int64_t n, int s)
{
    const int64_t nent = ((n - 1) >> s) + 2;
    for (int64_t j = threadIdx.x; j < nent; j += blockDim.x) {
        const int64_t v = (j << s) < n ? (j << s) : n - 1;
        tab[j] = (uint16_t)field_of(fo, nfields, v);
    }
}

__device__ __forceinline__ int field_by_table(const uint16_t *tab, const int64_t *fo, int s, uint32_t v)
{
    const uint32_t j = v >> s;
    return field_between(fo, tab[j], tab[j + 1], (int64_t)v);
}

// Batches of up to kFieldPassFields fields sort 4-byte value keys and then,
// in a last pass, by the field of each vertex id, found in an LDS copy of the
// field offsets (fo, nfields + 1 entries) narrowed by a coarse table.
constexpr int kFieldPassFields = 256;

__device__ __forceinline__ void load_field_offsets(int64_t *fo, const int64_t *foff, int nfields)
{
    for (int i = threadIdx.x; i <= nfields; i += blockDim.x) fo[i] = foff[i];
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


// The value as computed at this point: an empty asm statement that the
// compiler must treat as reading and rewriting the register, so the
// computation cannot move below it.
__device__ __forceinline__ uint32_t settled(uint32_t v)
{
    asm volatile("" : "+v"(v));
    return v;
}

// Element k of this lane in its tile (wave-striped), as an offset from the
// tile's first element.
__device__ __forceinline__ int local_index(int wave, int k, int lane)
{
    return wave * (kItems * kWave) + k * kWave + lane;
}

template <int kT = kTile>
__device__ __forceinline__ int tile_count(int64_t n, int64_t tile)
{
    const int64_t left = n - tile * kT;
    return left <= 0 ? 0 : (left < kT ? (int)left : kT);
}

// Histogram counters of a block: kCopies copies of the kRadix counts, lane l
// adding into copy l % kCopies, so that at most kWave / kCopies lanes of one
// LDS atomic instruction hit the same counter.  A digit that takes few values
// in random order (the top byte after the lower bytes have been sorted) would
// otherwise serialise most of a wave on one or two addresses.  Rows are
// padded by one word so that a digit's copies sit in different banks.
constexpr int kCopies = 16;
using HistRows = uint32_t[kCopies][kRadix + 1];

// One item per lane; a wave whose items share one digit adds them with one
// atomic.
__device__ __forceinline__ void hist_add(HistRows &h, uint32_t d, bool valid)
{
    const uint64_t act = __ballot(valid);
    const uint32_t d0 = __builtin_amdgcn_readfirstlane(valid ? d : 0xffffffffu);
    if (__ballot(valid && d == d0) == act) {
        if (act != 0 && lane_id() == (int)__builtin_ctzll(act)) atomicAdd(&h[0][d0], (uint32_t)__popcll(act));
        return;
    }
    if (valid) atomicAdd(&h[lane_id() & (kCopies - 1)][d], 1u);
}

// Element type read by a pass: the caller's values in the first pass, the
// sort keys after.
template <typename V, typename K, bool kFirst>
using SrcT = std::conditional_t<kFirst, V, K>;

template <typename V, typename K, bool kFirst>
__device__ __forceinline__ K to_key(SrcT<V, K, kFirst> r, bool &nan)
{
    if constexpr (kFirst) {
        return (K)key_of(r, nan);
    } else {
        nan = false;
        return r;
    }
}

// Loads of a tile's items are unconditional: items past the tile's end read
// its last element (every launched tile holds at least one) and are masked
// afterwards.  A load behind a per-item branch would make the compiler wait
// for it before the next item's load; this way all of them are in flight at
// once.
__device__ __forceinline__ int64_t item_at(int64_t t0, int li, int last)
{
    return t0 + (li < last ? li : last);
}

// (1) per-tile histogram of the digit at `shift`; counts is digit-major:
// counts[d * ntiles + tile].
// ids: the vertex ids, read by the field pass of a batch, whose digit is
// each id's field.
// kField (the last pass of a batch with 4-byte keys): the digit is the field
// of the vertex id instead of a byte of the key.
template <typename V, typename K, bool kFirst, int kThr, bool kField = false>
__global__ __launch_bounds__(kThr) void k_tile_hist(const void *src, int64_t n, int shift,
                                                        uint32_t *counts, int64_t ntiles,
                                                        uint32_t *flags, const uint32_t *ids,
                                                        const int64_t *foff, int nfields)
{
    __shared__ int64_t fo[kField ? kFieldPassFields + 1 : 1];
    __shared__ uint16_t ftab[kField ? kFieldTable : 1];
    __shared__ HistRows hist;
    const int tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
    const int64_t tile = tile_of_block(ntiles);
    const int64_t t0 = tile * (kThr * kItems);
    const int count = tile_count<kThr * kItems>(n, tile);
    if (count == 0) return;  // block-uniform
    const int last = count - 1;
    using R = SrcT<V, K, kFirst>;
    R raw[kItems];
    uint32_t bid[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k)
        if constexpr (!kField) raw[k] = ((const R *)src)[item_at(t0, local_index(wave, k, lane), last)];
    if (ids) {
#pragma unroll
        for (int k = 0; k < kItems; ++k) bid[k] = ids[item_at(t0, local_index(wave, k, lane), last)];
    }
    for (int i = tid; i < kCopies * (kRadix + 1); i += kThr) (&hist[0][0])[i] = 0;
    if constexpr (kField) load_field_offsets(fo, foff, nfields);
    __syncthreads();
    const int fsh = kField ? field_table_shift(n) : 0;
    if constexpr (kField) {
        build_field_table(ftab, fo, nfields, n, fsh);
        __syncthreads();
    }
    bool nan_any = false;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const bool valid = local_index(wave, k, lane) < count;
        uint32_t d;
        if constexpr (kField) {
            d = (uint32_t)field_by_table(ftab, fo, fsh, bid[k]);
        } else {
            bool nan;
            const K key = to_key<V, K, kFirst>(raw[k], nan);
            nan_any |= valid && nan;
            d = (uint32_t)(key >> shift) & (kRadix - 1);
        }
        hist_add(hist, d, valid);
    }
    __syncthreads();
    if (kFirst && __ballot(nan_any) && lane == 0) atomicOr(flags, (uint32_t)DMS_FLAG_NAN);
    if (tid >= kRadix) return;  // a thread per digit
    uint32_t tot = 0;
#pragma unroll
    for (int c = 0; c < kCopies; ++c) tot += hist[c][tid];
    counts[(int64_t)tid * ntiles + tile] = tot;  // digit-major, tiles in tile order
}

// Key storage between passes.  Every pass sorts by one byte of the stored
// key.  Except for batches of more than kFieldPassFields fields (whose last
// pass reads the field from the top of the 64-bit key), a pass writes the
// key without the byte it consumed, in the narrowest type that holds the
// rest, so that later passes read and write fewer bytes; the digit is then
// always the stored key's low byte.  NoKey: nothing left to store.
struct NoKey {};

// Rank of an item among the wave's items with the same 8-bit digit, counting
// this k and all earlier ones; wh is the wave's row of counts.  Items of a
// wave are in element order (k major, lane minor), so ranks are stable.
// The lanes holding the same digit are found either by eight ballots
// (kLds false) or through LDS (kLds true): each lane ORs its lane bit into
// the wave's mask slot of its digit (mk, zero between uses), reads the slot
// back and clears it -- three LDS operations in place of some forty vector
// instructions, which pays where the vector units are the busier resource
// (measured per kernel: the radix scatters and the id buckets use LDS, the
// last pass's digit and the fine partition the ballots).  A wave whose lanes share one digit (the high bytes of a smooth
// field) skips either.
template <bool kLds, typename CT>
__device__ __forceinline__ uint32_t wave_rank(uint32_t d, bool valid, CT *wh, uint64_t *mk)
{
    const uint64_t act = __ballot(valid);
    const uint32_t d0 = __builtin_amdgcn_readfirstlane(valid ? d : 0xffffffffu);
    uint64_t peers;
    if (__ballot(valid && d == d0) == act) {
        peers = act;
    } else if constexpr (kLds) {
        if (valid) atomicOr((unsigned long long *)&mk[d], 1ull << lane_id());
        peers = valid ? mk[d] : 0ull;
        if (valid) mk[d] = 0ull;
    } else {
        peers = match_digit8(d, act);
    }
    uint32_t base = 0;
    if (valid) base = wh[d];
    const uint32_t below = (uint32_t)__popcll(peers & lanemask_lt());
    if (valid && below == 0) wh[d] = (CT)(base + (uint32_t)__popcll(peers));
    return base + below;
}

// Thread tid < kRadix owns digit tid: the per-wave counts become exclusive
// prefixes over the waves; returns the tile's count of the digit (0 on the
// other threads).
template <int kThr = kThreads, typename CT>
__device__ __forceinline__ uint32_t wave_prefix(CT (*wh)[kRadix])
{
    static_assert(kThr >= kRadix, "a thread per digit");
    const int tid = threadIdx.x;
    if (tid >= kRadix) return 0;
    uint32_t run = 0;
#pragma unroll
    for (int w = 0; w < kThr / kWave; ++w) {
        const uint32_t c = wh[w][tid];
        wh[w][tid] = (CT)run;
        run += c;
    }
    return run;
}

// (3) stable scatter of one tile by the digit at `shift`.  offsets holds the
// scanned counts (global start of digit d in tile `tile`).
// foff (nfields + 1 offsets) is non-null for batches: the first pass puts
// the field index above the value key.
// LDS staging of a tile; the digit masks of the ranking phase live in the
// same bytes (the phases are separated by a barrier).
// A and B of at most 4 bytes each are staged packed in one 64-bit word (a in
// the low half): one LDS write and one read per item instead of two each.
template <typename A, typename B, int kThr = kThreads>
union Staging {
    struct {
        A a[kThr * kItems];
        B b[kThr * kItems];
    } st;
    uint64_t ab[kThr * kItems];
    uint64_t mk[kThr / kWave][kRadix];
    uint16_t ftab[kFieldTable];  // a field pass's coarse field table, while ranking by ballots
};

template <typename A, typename B>
constexpr bool kPacked = sizeof(A) <= 4 && sizeof(B) <= 4;

template <typename A, typename B, int kThr>
__device__ __forceinline__ void stage_put(Staging<A, B, kThr> &S, uint32_t pos, A a, B b)
{
    if constexpr (kPacked<A, B>) {
        S.ab[pos] = (uint64_t)(uint32_t)b << 32 | (uint64_t)a;
    } else {
        S.st.a[pos] = a;
        S.st.b[pos] = b;
    }
}

template <typename A, typename B, int kThr>
__device__ __forceinline__ void stage_get(const Staging<A, B, kThr> &S, int p, A &a, B &b)
{
    if constexpr (kPacked<A, B>) {
        const uint64_t v = S.ab[p];
        a = (A)v;
        b = (B)(uint32_t)(v >> 32);
    } else {
        a = S.st.a[p];
        b = S.st.b[p];
    }
}

template <typename A, typename B, int kThr>
__device__ __forceinline__ void zero_masks(Staging<A, B, kThr> &S)
{
    for (int i = threadIdx.x; i < (kThr / kWave) * kRadix; i += kThr) (&S.mk[0][0])[i] = 0ull;
}

// KD: the type the keys are written in, (KD)(key >> strip); NoKey when the
// next pass reads no key.
template <typename V, typename K, typename KD, bool kFirst, int kThr>
__global__ __launch_bounds__(kThr) void k_scatter(const void *src, const uint32_t *src_ids,
                                                      int64_t n, int shift, int strip,
                                                      const uint32_t *offsets, int64_t ntiles,
                                                      void *dst_keys, uint32_t *dst_ids,
                                                      const int64_t *foff, int nfields)
{
    constexpr int kW = kThr / kWave;
    __shared__ uint32_t whist[kW][kRadix];
    __shared__ uint32_t gbase[kRadix];
    __shared__ Staging<K, uint32_t, kThr> S;

    const int tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
    const int64_t tile = tile_of_block(ntiles);
    const int64_t t0 = tile * (kThr * kItems);
    const int count = tile_count<kThr * kItems>(n, tile);
    if (count == 0) return;  // block-uniform
    const int last = count - 1;
    using R = SrcT<V, K, kFirst>;
    R raw[kItems];
    uint32_t id[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int64_t at = item_at(t0, local_index(wave, k, lane), last);
        raw[k] = ((const R *)src)[at];
        id[k] = kFirst ? (uint32_t)at : src_ids[at];
    }
    for (int i = tid; i < kW * kRadix; i += kThr) (&whist[0][0])[i] = 0;
    zero_masks(S);
    __syncthreads();

    K key[kItems];
    uint32_t rank[kItems];
    // a batch tile usually lies in one field: the fields of its first and
    // last elements bound the search for the others
    int f_first = 0, f_last = 0;
    if constexpr (kFirst && sizeof(K) == 8) {
        if (foff && count > 0) {
            f_first = field_of(foff, nfields, t0);
            f_last = field_of(foff, nfields, t0 + count - 1);
        }
    }
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int li = local_index(wave, k, lane);
        bool nan;
        key[k] = to_key<V, K, kFirst>(raw[k], nan);
        if constexpr (kFirst && sizeof(K) == 8) {
            if (foff && li < count) {
                const int f = f_first == f_last ? f_first : field_between(foff, f_first, f_last, t0 + li);
                key[k] |= (K)f << 32;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < kItems; ++k)
        rank[k] = wave_rank<true>((uint32_t)(key[k] >> shift) & (kRadix - 1),
                                     local_index(wave, k, lane) < count, whist[wave], S.mk[wave]);
    __syncthreads();
    {
        uint32_t total;
        const uint32_t start = block_exclusive_scan<uint32_t, kThr>(wave_prefix<kThr>(whist), &total);
        // whist[w][d] becomes the tile position of wave w's first item of
        // digit d; the global position of the tile's element at local
        // position p of digit d is gbase[d] + p (gbase holds the scanned
        // offset minus the local start)
        if (tid < kRadix) {
#pragma unroll
            for (int w = 0; w < kW; ++w) whist[w][tid] += start;
            gbase[tid] = offsets[(int64_t)tid * ntiles + tile] - start;
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        if (local_index(wave, k, lane) < count) {
            const uint32_t d = (uint32_t)(key[k] >> shift) & (kRadix - 1);
            stage_put(S, whist[wave][d] + rank[k], key[k], id[k]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        const int p = tid + j * kThr;
        if (p < count) {
            K kk;
            uint32_t who;
            stage_get(S, p, kk, who);
            const uint32_t g = gbase[(uint32_t)(kk >> shift) & (kRadix - 1)] + (uint32_t)p;
            // the ranks make g < n; the guard keeps any breach of that in bounds
            if ((int64_t)g < n) {
                if constexpr (!std::is_same_v<KD, NoKey>) ((KD *)dst_keys)[g] = (KD)(kk >> strip);
                dst_ids[g] = who;
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
// leave as one contiguous run.  The run's place inside its bucket is taken
// from the bucket's fill counter (bfill, zeroed beforehand) by one atomic
// add per bucket and tile: the order of the pairs inside a bucket does not
// matter to the inversion, which places them by id, and bucket b starts at
// position b << bshift because the ids are a permutation.
// For batches the position is taken relative to the field's first vertex.
// Per-wave counts are 16-bit (at most a tile), so that the block's LDS stays
// just under 40 KiB at 256 threads (four blocks per CU) and 75 KiB at 512
// (two).
template <typename K, int kThr, bool kField = false>
__global__ __launch_bounds__(kThr) void k_scatter_last(const K *src, const uint32_t *src_ids,
                                                           int64_t n, int shift,
                                                           const uint32_t *offsets,
                                                           uint32_t *bfill, int64_t ntiles,
                                                           const int64_t *foff, int nfields, int bshift,
                                                           uint32_t *pair_id, int32_t *pair_pos)
{
    __shared__ int64_t fo[kField ? kFieldPassFields + 1 : 1];
    constexpr int kW = kThr / kWave, kT = kThr * kItems;
    // dwh: per-wave digit counts while ranking, then the final position of
    // wave w's first item of digit d (for a field pass, relative to the
    // field's first vertex)
    __shared__ uint32_t dwh[kW][kRadix];
    __shared__ uint32_t bcnt[kRadix];
    __shared__ uint32_t bstart[kRadix];
    __shared__ uint32_t bbase[kRadix];
    __shared__ Staging<uint32_t, int32_t, kThr> S;

    const int tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
    for (int i = tid; i < kW * kRadix; i += kThr) (&dwh[0][0])[i] = 0;
    if (tid < kRadix) bcnt[tid] = 0;
    if constexpr (kField) load_field_offsets(fo, foff, nfields);
    __syncthreads();

    const int64_t tile = tile_of_block(ntiles);
    const int64_t t0 = tile * kT;
    const int count = tile_count<kT>(n, tile);
    if (count == 0) return;  // block-uniform
    // per item after the ranking: the id and, packed, its digit rank inside
    // the wave (below 16 x 64 = 2^10), its digit and its slot among the
    // tile's pairs of its bucket (below 2^13); batches of 8-byte keys also
    // keep the field.
    // The digit ranks must be stable (they give the sorted position); the
    // bucket slots need not be (the inversion places pairs by id), so they
    // come from one LDS atomic per item.
    uint32_t id[kItems], pk[kItems];
    uint32_t fld[sizeof(K) == 8 ? kItems : 1];
    {
        K key[kItems];
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            const int64_t at = item_at(t0, local_index(wave, k, lane), count - 1);
            if constexpr (!kField) key[k] = src[at];  // the field pass needs only the ids
            id[k] = src_ids[at];
        }
        // the field table lives in the staging bytes, unused until the
        // ranking's barrier (the ranking matches by ballots, without the
        // LDS masks)
        const int fsh = kField ? field_table_shift(n) : 0;
        if constexpr (kField) {
            build_field_table(S.ftab, fo, nfields, n, fsh);
            __syncthreads();
        }
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            const bool valid = local_index(wave, k, lane) < count;
            uint32_t d;
            if constexpr (kField)
                d = (uint32_t)field_by_table(S.ftab, fo, fsh, id[k]);
            else
                d = (uint32_t)(key[k] >> shift) & (kRadix - 1);
            // the top byte (sign and exponent) takes few values, and a tile
            // spans few fields: ballots match it faster than the LDS masks,
            // which serve the random id buckets
            const uint32_t rd = wave_rank<false>(d, valid, dwh[wave], S.mk[wave]);
            const uint32_t rb = valid ? atomicAdd(&bcnt[(id[k] >> bshift) & (kRadix - 1)], 1u) : 0u;
            // settled here: otherwise the compiler sinks the rank popcounts past
            // the barrier and keeps every item's two 64-bit lane masks alive
            pk[k] = settled(rd | d << 10 | rb << 18);
            if constexpr (!kField && sizeof(K) == 8) fld[k] = (uint32_t)(key[k] >> 32);
        }
    }
    __syncthreads();
    {
        wave_prefix<kThr>(dwh);
        uint32_t total;
        const uint32_t nb = tid < kRadix ? bcnt[tid] : 0u;  // the tile's pairs of bucket tid
        const uint32_t start = block_exclusive_scan<uint32_t, kThr>(nb, &total);
        if (tid < kRadix) {
            bstart[tid] = start;
            uint32_t gb = offsets[(int64_t)tid * ntiles + tile];
            if constexpr (kField) gb -= tid <= nfields ? (uint32_t)fo[tid] : 0u;  // the digit is the field
#pragma unroll
            for (int w = 0; w < kW; ++w) dwh[w][tid] += gb;
            bbase[tid] = nb ? ((uint32_t)tid << bshift) + atomicAdd(&bfill[tid], nb) - start : 0u;
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        if (local_index(wave, k, lane) < count) {
            const uint32_t d = (pk[k] >> 10) & (kRadix - 1);
            const uint32_t b = (id[k] >> bshift) & (kRadix - 1);
            int64_t g = (int64_t)(dwh[wave][d] + (pk[k] & 1023u));
            if constexpr (!kField && sizeof(K) == 8) {
                if (foff) g -= foff[fld[k]];
            }
            const uint32_t pos = bstart[b] + (pk[k] >> 18);
            if (pos < (uint32_t)kT) stage_put(S, pos, id[k], (int32_t)g);
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        const int p = tid + j * kThr;
        if (p < count) {
            uint32_t who;
            int32_t at;
            stage_get(S, p, who, at);
            const uint32_t dst = bbase[(who >> bshift) & (kRadix - 1)] + (uint32_t)p;
            if ((int64_t)dst < n) {
                pair_id[dst] = who;
                pair_pos[dst] = at;
            }
        }
    }
}

// Level 1: a partition of each chunk of a coarse bucket by the fine digit
// into the windows of ids.  As in level 0, a chunk's run for window w is
// placed by one atomic add on the window's fill counter (wfill, zeroed
// beforehand; window w starts at position w << fshift).  The ids are written
// relative to their window (fshift <= 16 bits), 2 bytes instead of 4.
__global__ __launch_bounds__(kThreads) void k_fine_scatter(const uint32_t *in_id, const int32_t *in_pos,
                                                           int64_t n, int fshift, int flog, int qlog,
                                                           int64_t nchunks, uint32_t *wfill,
                                                           uint16_t *out_id, int32_t *out_pos)
{
    __shared__ uint32_t cnt[kRadix];
    __shared__ uint32_t dstart[kRadix];
    __shared__ uint32_t gbase[kRadix];
    __shared__ uint32_t sid[kTile];
    __shared__ int32_t spos[kTile];

    const int tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
    if (tid < kRadix) cnt[tid] = 0;
    __syncthreads();
    const int64_t c = tile_of_block(nchunks);
    const int64_t t0 = c * kTile;
    const int count = tile_count(n, c);
    if (count == 0) return;  // block-uniform
    const uint32_t fmask = (1u << flog) - 1u;
    uint32_t id[kItems], slot[kItems];
    int32_t pos[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k) {  // unconditional loads (count >= 1)
        const int64_t at = item_at(t0, local_index(wave, k, lane), count - 1);
        id[k] = in_id[at];
        pos[k] = in_pos[at];
    }
    // the order inside a window is free: a slot per item from one LDS atomic
#pragma unroll
    for (int k = 0; k < kItems; ++k)
        slot[k] = local_index(wave, k, lane) < count ? atomicAdd(&cnt[(id[k] >> fshift) & fmask], 1u) : 0u;
    __syncthreads();
    {
        uint32_t total;
        const uint32_t nw = tid <= (int)fmask ? cnt[tid] : 0u;  // the chunk's pairs of window digit tid
        const uint32_t start = block_exclusive_scan<uint32_t>(nw, &total);
        dstart[tid] = start;
        const int64_t w = ((c >> qlog) << flog) | tid;
        gbase[tid] = nw ? (uint32_t)(w << fshift) + atomicAdd(&wfill[w], nw) - start : 0u;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        if (local_index(wave, k, lane) < count) {
            const uint32_t at = dstart[(id[k] >> fshift) & fmask] + slot[k];
            if (at < (uint32_t)kTile) {
                sid[at] = id[k];
                spos[at] = pos[k];
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        const int p = tid + j * kThreads;
        if (p < count) {
            const uint32_t who = sid[p];
            const uint32_t dst = gbase[(who >> fshift) & fmask] + (uint32_t)p;
            if ((int64_t)dst < n) {
                out_id[dst] = (uint16_t)(who & ((1u << fshift) - 1u));  // the id within its window
                out_pos[dst] = spos[p];
            }
        }
    }
}

// Window w holds the pairs of ids [w 2^wshift, (w+1) 2^wshift): the block
// places the positions into LDS by id, then writes the window contiguously.
constexpr int kInvThreads = 1024;
constexpr int kInvUnroll = 4;

// ID: uint32_t ids (windows straight from the coarse buckets), or uint16_t
// ids relative to the window's first id (written by the fine level).
template <int kWinLog, typename ID>
__global__ __launch_bounds__(kInvThreads) void k_invert_window(const ID *__restrict__ pair_id,
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
        int64_t off[kInvUnroll];
        int32_t r[kInvUnroll];
#pragma unroll
        for (int u = 0; u < kInvUnroll; ++u) {  // unconditional loads (cnt >= 1)
            const int i = i0 + u * kInvThreads + (int)threadIdx.x;
            const int64_t at = base + (i < cnt ? i : cnt - 1);
            const int64_t v = (int64_t)pair_id[at];
            r[u] = pair_pos[at];
            off[u] = i >= cnt ? -1 : (sizeof(ID) == 2 ? v : v - base);
        }
#pragma unroll
        for (int u = 0; u < kInvUnroll; ++u)
            if (off[u] >= 0 && off[u] < cnt) win[off[u]] = r[u];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < cnt; i += kInvThreads) order[base + i] = win[i];
}

struct OrderLayout {
    size_t keys0, keys1, ids0, ids1, counts, partials, fill, total;
};

// Fill counters of the inversion: the kRadix coarse buckets, then the windows.
inline int64_t fill_words(int64_t n, const InvertPlan &P) { return kRadix + ((n + (1ll << P.wshift) - 1) >> P.wshift); }

template <typename K>
OrderLayout order_layout(int64_t n)
{
    const int64_t ntiles = (n + kTile - 1) / kTile;
    const InvertPlan P = invert_plan(n);
    const int64_t chunks = P.fine && P.nchunks > ntiles ? P.nchunks : ntiles;
    const int64_t clen = chunks * kRadix;
    OrderLayout L{};
    size_t off = 0;
    L.keys0 = off; off += align_up((size_t)n * sizeof(K), 256);
    L.keys1 = off; off += align_up((size_t)n * sizeof(K), 256);
    L.ids0 = off; off += align_up((size_t)n * 4, 256);
    L.ids1 = off; off += align_up((size_t)n * 4, 256);
    L.counts = off; off += align_up((size_t)clen * 4, 256);
    L.partials = off; off += scan_partials_bytes(clen, 4);
    L.fill = off; off += align_up((size_t)fill_words(n, P) * 4, 256);
    L.total = off;
    return L;
}

// Bytes of the stored key when `bits` bits of it remain (0: none left).
constexpr int key_bytes(int bits) { return bits <= 0 ? 0 : bits <= 8 ? 1 : bits <= 16 ? 2 : bits <= 32 ? 4 : 8; }

// One radix pass other than the last (histogram, scan, scatter).
struct PassArgs {
    const void *src;
    const uint32_t *sids;
    int64_t n;
    int shift, strip;
    uint32_t *counts, *partials, *flags;
    void *dkeys;
    uint32_t *dids;
    const int64_t *foff;
    int nfields;
    hipStream_t s;
};

// Blocks of 512 threads (8192-key tiles) for keys up to 4 bytes, 256 for
// 8-byte keys (two 512-thread blocks of those would not fit one CU's LDS).
template <typename K>
constexpr int pass_threads() { return sizeof(K) == 8 ? kThreads : kWideThreads; }

template <typename V, typename K, typename KD, bool kFirst>
void radix_pass(const PassArgs &A)
{
    constexpr int kW = pass_threads<K>();
    const int64_t nt = (A.n + kW * kItems - 1) / (kW * kItems);
    hipLaunchKernelGGL((k_tile_hist<V, K, kFirst, kW>), dim3((unsigned)nt), dim3(kW), 0, A.s, A.src, A.n,
                       A.shift, A.counts, nt, A.flags, (const uint32_t *)nullptr, (const int64_t *)nullptr, 0);
    exclusive_scan<uint32_t>(A.counts, nt * kRadix, A.partials, A.s);
    hipLaunchKernelGGL((k_scatter<V, K, KD, kFirst, kW>), dim3((unsigned)nt), dim3(kW), 0, A.s, A.src, A.sids,
                       A.n, A.shift, A.strip, A.counts, nt, A.dkeys, A.dids, A.foff, A.nfields);
}

// A middle pass by the stored key's bytes before (ks) and after (kd) it.
int radix_mid_pass(int ks, int kd, const PassArgs &A)
{
    switch (ks * 16 + kd) {
    case 8 * 16 + 8: radix_pass<uint64_t, uint64_t, uint64_t, false>(A); return DMS_OK;
    case 8 * 16 + 4: radix_pass<uint64_t, uint64_t, uint32_t, false>(A); return DMS_OK;
    case 4 * 16 + 4: radix_pass<uint32_t, uint32_t, uint32_t, false>(A); return DMS_OK;
    case 4 * 16 + 2: radix_pass<uint32_t, uint32_t, uint16_t, false>(A); return DMS_OK;
    case 2 * 16 + 1: radix_pass<uint16_t, uint16_t, uint8_t, false>(A); return DMS_OK;
    case 1 * 16 + 0: radix_pass<uint8_t, uint8_t, NoKey, false>(A); return DMS_OK;
    default: return DMS_E_ARG;
    }
}

// The last pass (histogram of the digit, its scan, level-0 scatter of the
// (id, position) pairs into the coarse buckets, placed through bfill) on
// stored keys KS.
template <typename KS, bool kField>
void last_pass(const void *src, const uint32_t *sids, int64_t n, int shift, const InvertPlan &P,
               uint32_t *counts, uint32_t *partials, uint32_t *bfill, uint32_t *flags, const int64_t *foff,
               int nfields, uint32_t *aid, int32_t *apos, hipStream_t s)
{
    constexpr int kW = pass_threads<KS>();
    const int64_t nt = (n + kW * kItems - 1) / (kW * kItems);
    hipLaunchKernelGGL((k_tile_hist<KS, KS, false, kW, kField>), dim3((unsigned)nt), dim3(kW), 0, s, src, n,
                       shift, counts, nt, flags, kField ? sids : nullptr, foff, nfields);
    exclusive_scan<uint32_t>(counts, nt * kRadix, partials, s);
    hipLaunchKernelGGL((k_scatter_last<KS, kW, kField>), dim3((unsigned)nt), dim3(kW), 0, s, (const KS *)src,
                       sids, n, shift, counts, bfill, nt, foff, nfields, P.bshift, aid, apos);
}

__global__ void k_zero_words(uint32_t *__restrict__ w, int64_t nw)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nw) w[i] = 0u;
}

// field_last: a batch of at most kFieldPassFields fields with 4-byte keys;
// passes - 1 value passes, then the last pass orders by the field of each id.
// Keys are stored stripped of consumed bytes (NoKey) except for batches
// with 64-bit keys.
template <typename V, typename K>
int run_order(const void *values, int64_t n, int passes, int32_t *order, char *ws, uint32_t *flags,
              const int64_t *foff, int nfields, hipStream_t s, bool field_last = false)
{
    if (passes < 2) return DMS_E_ARG;
    if (field_last && (sizeof(K) != 4 || !foff || nfields > kFieldPassFields)) return DMS_E_ARG;
    const OrderLayout L = order_layout<K>(n);
    const InvertPlan P = invert_plan(n);
    const bool strip = !(sizeof(K) == 8 && foff);
    const int key_bits = field_last ? 32 : 8 * passes;
    char *keys[2] = {ws + L.keys0, ws + L.keys1};
    uint32_t *ids[2] = {(uint32_t *)(ws + L.ids0), (uint32_t *)(ws + L.ids1)};
    uint32_t *counts = (uint32_t *)(ws + L.counts);
    uint32_t *partials = (uint32_t *)(ws + L.partials);
    uint32_t *bfill = (uint32_t *)(ws + L.fill), *wfill = bfill + kRadix;
    for (int p = 0; p < passes; ++p) {
        // digits: the stored key's low byte, or byte p of the whole key
        const int shift = strip ? 0 : 8 * p;
        const bool last = p == passes - 1;
        const void *src = p == 0 ? values : (const void *)keys[(p - 1) & 1];
        const uint32_t *sids = p == 0 ? nullptr : ids[(p - 1) & 1];
        if (!last) {
            PassArgs A{src, sids, n, shift, strip ? 8 : 0, counts, partials, flags, keys[p & 1], ids[p & 1],
                       foff, nfields, s};
            if (p == 0) {
                // the first pass writes K: at least 24 bits of a 32-bit key and 56 of a 64-bit one remain
                if (strip && key_bytes(key_bits - 8) != (int)sizeof(K)) return DMS_E_ARG;
                radix_pass<V, K, K, true>(A);
            } else {
                const int ks = strip ? key_bytes(key_bits - 8 * p) : (int)sizeof(K);
                const int kd = strip ? key_bytes(key_bits - 8 * (p + 1)) : (int)sizeof(K);
                if (const int st = radix_mid_pass(ks, kd, A)) return st;
            }
            continue;
        }
        // level 0 into the free buffers; level 1 back into the last pass's
        // source buffers once they are read
        uint32_t *aid = (uint32_t *)keys[p & 1];
        int32_t *apos = (int32_t *)ids[p & 1];
        const int64_t nfill = fill_words(n, P);
        hipLaunchKernelGGL(k_zero_words, dim3((unsigned)((nfill + 255) / 256)), dim3(256), 0, s, bfill, nfill);
        if (field_last)
            last_pass<uint32_t, true>(src, sids, n, 0, P, counts, partials, bfill, flags, foff, nfields, aid,
                                      apos, s);
        else if (strip)
            last_pass<uint8_t, false>(src, sids, n, 0, P, counts, partials, bfill, flags, foff, nfields, aid,
                                      apos, s);
        else
            last_pass<uint64_t, false>(src, sids, n, shift, P, counts, partials, bfill, flags, foff, nfields,
                                       aid, apos, s);
        const int64_t nwin = (n + (1ll << P.wshift) - 1) >> P.wshift;
        if (P.wshift > kMaxWinLog + 1) return DMS_E_SIZE;
        if (P.fine) {
            uint16_t *fid = (uint16_t *)keys[(p - 1) & 1];
            int32_t *fpos = (int32_t *)ids[(p - 1) & 1];
            const dim3 cgrid((unsigned)P.nchunks);
            hipLaunchKernelGGL(k_fine_scatter, cgrid, dim3(kThreads), 0, s, aid, apos, n, P.fshift, P.flog,
                               P.qlog, P.nchunks, wfill, fid, fpos);
            if (P.wshift <= kMaxWinLog)
                hipLaunchKernelGGL((k_invert_window<kMaxWinLog, uint16_t>), dim3((unsigned)nwin),
                                   dim3(kInvThreads), 0, s, fid, fpos, n, P.wshift, order);
            else
                hipLaunchKernelGGL((k_invert_window<kMaxWinLog + 1, uint16_t>), dim3((unsigned)nwin),
                                   dim3(kInvThreads), 0, s, fid, fpos, n, P.wshift, order);
        } else {
            if (P.wshift <= kMaxWinLog)
                hipLaunchKernelGGL((k_invert_window<kMaxWinLog, uint32_t>), dim3((unsigned)nwin),
                                   dim3(kInvThreads), 0, s, aid, apos, n, P.wshift, order);
            else
                hipLaunchKernelGGL((k_invert_window<kMaxWinLog + 1, uint32_t>), dim3((unsigned)nwin),
                                   dim3(kInvThreads), 0, s, aid, apos, n, P.wshift, order);
        }
    }
    return launch_status();
}

}  // namespace

size_t rank_u64_workspace_size(int64_t n) { return order_layout<uint64_t>(n > 0 ? n : 1).total; }

int launch_rank_u64(const uint64_t *keys, int64_t n, int32_t *rank, char *ws, uint32_t *flags,
                    hipStream_t s)
{
    if (n == 0) return DMS_OK;
    return run_order<uint64_t, uint64_t>(keys, n, 8, rank, ws, flags, nullptr, 0, s);
}

size_t order_batch_workspace_size(int64_t n) { return order_layout<uint64_t>(n > 0 ? n : 1).total; }

int launch_order_batch(const float *values, int64_t n, const int64_t *foff, int nfields,
                       int32_t *order, char *ws, uint32_t *flags, hipStream_t s)
{
    if (n == 0) return DMS_OK;
    if (nfields <= kFieldPassFields)  // four value passes, then one field pass
        return run_order<float, uint32_t>(values, n, 5, order, ws, flags, foff, nfields, s, true);
    return run_order<float, uint64_t>(values, n, batch_passes(nfields), order, ws, flags, foff, nfields, s);
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
    if (const int dc = dms::device_check()) return dc;
    hipStream_t s = (hipStream_t)stream;
    if (dtype == DMS_F32)
        return dms::run_order<float, uint32_t>(values, n, 4, order, (char *)workspace, dev_flags,
                                               nullptr, 0, s);
    return dms::run_order<double, uint64_t>(values, n, 8, order, (char *)workspace, dev_flags, nullptr,
                                            0, s);
}
