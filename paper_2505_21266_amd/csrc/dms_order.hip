// dms_order.hip -- global vertex order (Section 2.1; Array Preconditioning,
// Section 3) as a stable least-significant-digit radix sort of
// (value key, vertex id) pairs on one GPU.
//
// The paper sorts (value, global id, owner) tuples with a distributed sort;
// on one GPU the same order comes from a stable LSD radix sort: vertices start
// in id order, every pass is stable, so equal values stay in id order, which
// is exactly the tie-break of Section 2.1.  Values become order-preserving
// unsigned keys (-0.0 -> +0.0; NaN flagged).  8-bit digits: 4 passes for
// float32, 8 for float64.  The last pass scatters each vertex's final
// position straight into order[id].
//
// Each pass: (1) per-tile digit histograms, (2) a device-wide exclusive scan
// of the digit-major histogram matrix, (3) a stable per-tile scatter.  Tiles
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

__device__ __forceinline__ int64_t elem_index(int64_t tile, int wave, int k, int lane)
{
    return tile * kTile + (int64_t)wave * (kItems * kWave) + k * kWave + lane;
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
template <typename V, typename K, bool kFirst>
__global__ __launch_bounds__(kThreads) void k_tile_hist(const void *src, int64_t n, int shift,
                                                        uint32_t *counts, int64_t ntiles,
                                                        uint32_t *flags)
{
    __shared__ uint32_t hist[kWaves][kRadix];
    const int tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
    for (int i = tid; i < kWaves * kRadix; i += kThreads) (&hist[0][0])[i] = 0;
    __syncthreads();
    const int64_t tile = blockIdx.x;
    bool nan_any = false;
    for (int k = 0; k < kItems; ++k) {
        const int64_t i = elem_index(tile, wave, k, lane);
        const bool valid = i < n;
        uint32_t d = 0;
        if (valid) {
            bool nan;
            K key = load_key<V, K, kFirst>(src, i, nan);
            nan_any |= nan;
            d = (uint32_t)(key >> shift) & (kRadix - 1);
        }
        const uint64_t peers = match_digit8(d, __ballot(valid));
        if (valid && (peers & lanemask_lt()) == 0) hist[wave][d] += (uint32_t)__popcll(peers);
    }
    __syncthreads();
    uint32_t tot = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) tot += hist[w][tid];
    counts[(int64_t)tid * ntiles + tile] = tot;
    if (kFirst && __ballot(nan_any) && lane == 0) atomicOr(flags, (uint32_t)DMS_FLAG_NAN);
}

// (3) stable scatter of one tile by the digit at `shift`.  offsets holds the
// scanned counts (global start of digit d in tile `tile`).
// foff (nfields + 1 offsets) is non-null for batches: the first pass puts
// the field index above the value key, the last writes order = position
// minus the field's offset.
template <typename V, typename K, bool kFirst, bool kLast>
__global__ __launch_bounds__(kThreads) void k_scatter(const void *src, const uint32_t *src_ids,
                                                      int64_t n, int shift,
                                                      const uint32_t *offsets, int64_t ntiles,
                                                      K *dst_keys, uint32_t *dst_ids, int32_t *order,
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

    const int64_t tile = blockIdx.x;
    K key[kItems];
    uint32_t id[kItems];
    uint32_t rank[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int64_t i = elem_index(tile, wave, k, lane);
        const bool valid = i < n;
        uint32_t d = 0;
        key[k] = 0;
        id[k] = 0;
        if (valid) {
            bool nan;
            key[k] = load_key<V, K, kFirst>(src, i, nan);
            if constexpr (kFirst && sizeof(K) == 8) {
                if (foff) key[k] |= (K)field_of(foff, nfields, i) << 32;
            }
            id[k] = kFirst ? (uint32_t)i : src_ids[i];
            d = (uint32_t)(key[k] >> shift) & (kRadix - 1);
        }
        const uint64_t peers = match_digit8(d, __ballot(valid));
        uint32_t base = 0;
        if (valid) base = whist[wave][d];
        rank[k] = base + (uint32_t)__popcll(peers & lanemask_lt());
        if (valid && (peers & lanemask_lt()) == 0) whist[wave][d] = base + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    {
        // thread tid owns digit tid: prefix over waves, then over digits
        uint32_t c[kWaves], run = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            c[w] = whist[w][tid];
            whist[w][tid] = run;
            run += c[w];
        }
        uint32_t total;
        const uint32_t start = block_exclusive_scan<uint32_t>(run, &total);
        digit_start[tid] = start;
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
            const uint32_t who = sid[p];
            // the ranks make g < n and who < n; the guard keeps any breach of
            // that in bounds
            if ((int64_t)g < n && (int64_t)who < n) {
                if (kLast) {
                    int64_t base = 0;
                    if constexpr (sizeof(K) == 8) {
                        if (foff) base = foff[(int)(kk >> 32)];
                    }
                    order[who] = (int32_t)((int64_t)g - base);
                } else {
                    dst_keys[g] = kk;
                    dst_ids[g] = who;
                }
            }
        }
    }
}

struct OrderLayout {
    size_t keys0, keys1, ids0, ids1, counts, partials, total;
};

template <typename K>
OrderLayout order_layout(int64_t n)
{
    const int64_t ntiles = (n + kTile - 1) / kTile;
    const int64_t clen = ntiles * kRadix;
    OrderLayout L{};
    size_t off = 0;
    L.keys0 = off; off += align_up((size_t)n * sizeof(K), 256);
    L.keys1 = off; off += align_up((size_t)n * sizeof(K), 256);
    L.ids0 = off; off += align_up((size_t)n * 4, 256);
    L.ids1 = off; off += align_up((size_t)n * 4, 256);
    L.counts = off; off += align_up((size_t)clen * 4, 256);
    L.partials = off; off += scan_partials_bytes(clen, 4);
    L.total = off;
    return L;
}

template <typename V, typename K>
int run_order(const void *values, int64_t n, int passes, int32_t *order, char *ws, uint32_t *flags,
              const int64_t *foff, int nfields, hipStream_t s)
{
    const OrderLayout L = order_layout<K>(n);
    const int64_t ntiles = (n + kTile - 1) / kTile;
    K *keys[2] = {(K *)(ws + L.keys0), (K *)(ws + L.keys1)};
    uint32_t *ids[2] = {(uint32_t *)(ws + L.ids0), (uint32_t *)(ws + L.ids1)};
    uint32_t *counts = (uint32_t *)(ws + L.counts);
    uint32_t *partials = (uint32_t *)(ws + L.partials);
    const dim3 grid((unsigned)ntiles), block(kThreads);
    for (int p = 0; p < passes; ++p) {
        const int shift = 8 * p;
        const void *src = p == 0 ? values : (const void *)keys[(p - 1) & 1];
        const uint32_t *sids = p == 0 ? nullptr : ids[(p - 1) & 1];
        if (p == 0)
            hipLaunchKernelGGL((k_tile_hist<V, K, true>), grid, block, 0, s, src, n, shift, counts,
                               ntiles, flags);
        else
            hipLaunchKernelGGL((k_tile_hist<V, K, false>), grid, block, 0, s, src, n, shift, counts,
                               ntiles, flags);
        exclusive_scan<uint32_t>(counts, ntiles * kRadix, partials, s);
        if (p == 0)
            hipLaunchKernelGGL((k_scatter<V, K, true, false>), grid, block, 0, s, src, sids, n, shift,
                               counts, ntiles, keys[p & 1], ids[p & 1], order, foff, nfields);
        else if (p == passes - 1)
            hipLaunchKernelGGL((k_scatter<V, K, false, true>), grid, block, 0, s, src, sids, n, shift,
                               counts, ntiles, keys[p & 1], ids[p & 1], order, foff, nfields);
        else
            hipLaunchKernelGGL((k_scatter<V, K, false, false>), grid, block, 0, s, src, sids, n, shift,
                               counts, ntiles, keys[p & 1], ids[p & 1], order, foff, nfields);
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
