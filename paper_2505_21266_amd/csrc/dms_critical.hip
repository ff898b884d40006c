// dms_critical.hip -- extraction of the critical simplices from the
// lower-star records (Section 2.6, zero-persistence skip: a cell that is
// neither tail nor head of a discrete vector is critical; Section 3, Extract).
//
// Three steps over the owned box, in box order (which is vertex-id order):
//  count  per 1024-record tile, the number of critical cells of each
//         dimension, from popcounts of the record fields (no table walk),
//         and the list of the tile's records that hold any (up to kCand);
//  scan   an exclusive scan of the 4 x ntiles tile counts;
//  fill   per listed record, the critical cells in (dimension, local index)
//         order, written at tile offset + scan offset as int64 codes
//         (max vertex id << 8) | local index.  A tile with more than kCand
//         such records is re-read whole.
// With the critical mask of the gradient call, count and fill read only the
// flagged records instead, one wave per tile, and no candidate lists.
#include <atomic>

#include "dms_common.hpp"
#include "dms_internal.hpp"
#include "dms_scan.hpp"
#include "dms_tables.hpp"

namespace dms {
namespace {

constexpr int kThreads = 256;
constexpr int kPerThread = 4;
constexpr int kTileRecs = kThreads * kPerThread;  // records per block
constexpr int kCand = 32;  // records with critical cells listed per tile

struct Fields {
    uint64_t lo, hi;
};

// L(x) edge mask from the edge fields: bit e set iff edge field e is non-zero
// (nibble-wise OR, then the 14 nibble bits compressed into 14 adjacent bits)
__device__ __forceinline__ uint32_t lower_edges(uint64_t lo)
{
    uint64_t x = lo | (lo >> 1);
    x |= x >> 2;
    x &= 0x0011111111111111ull;                   // bit 4e
    x = (x | (x >> 3)) & 0x0003030303030303ull;   // bits 8j, 8j+1
    x = (x | (x >> 6)) & 0x000f000f000f000full;   // nibbles at 16j
    x = (x | (x >> 12)) & 0x000000ff000000ffull;  // bytes at 32j
    x = (x | (x >> 24)) & 0xffffull;
    return (uint32_t)x;
}

// Number of star triangles (low byte) and tets (high byte) in L(x) for each
// 14-bit lower-neighbour mask: the cells all of whose other vertices are
// lower neighbours.
struct CellCounts {
    uint16_t n[1 << 14];
};

// Built incrementally: adding the highest lower neighbour e to a mask adds
// the triangles {e, a} with a lower (a in the link of e) and the tets {e, a,
// b} with a and b lower.
constexpr CellCounts make_cell_counts()
{
    CellCounts C{};
    const Tables &T = kTables;
    uint16_t tet_pairs[14][24] = {};
    int npairs[14] = {};
    for (int q = 0; q < 24; ++q)
        for (int c = 0; c < 3; ++c) {
            const int e = T.tet[q][c];
            uint16_t m = 0;
            for (int d = 0; d < 3; ++d)
                if (d != c) m = (uint16_t)(m | (1u << T.tet[q][d]));
            tet_pairs[e][npairs[e]++] = m;
        }
    C.n[0] = 0;
    for (uint32_t low = 1; low < (1u << 14); ++low) {
        int e = 13;
        while (!((low >> e) & 1u)) --e;
        const uint32_t rest = low & ~(1u << e);
        uint32_t nt = 0, nq = 0;
        for (uint32_t m = T.link[e] & rest; m; m &= m - 1) ++nt;
        for (int k = 0; k < npairs[e]; ++k)
            if ((tet_pairs[e][k] & rest) == tet_pairs[e][k]) ++nq;
        const uint32_t prev = C.n[rest];
        C.n[low] = (uint16_t)(((prev & 0xffu) + nt) | (((prev >> 8) + nq) << 8));
    }
    return C;
}

__device__ const CellCounts g_cell_counts = make_cell_counts();

constexpr uint64_t kNib14 = 0x00ffffffffffffffull;  // 14 nibbles

__device__ __forceinline__ void count_critical(uint64_t lo, uint64_t hi, uint32_t c[4])
{
    const uint64_t ef = lo & kNib14;
    const uint32_t low = lower_edges(lo);
    // fields equal to 2 (critical edges)
    const uint64_t y = ef ^ (0x0022222222222222ull);
    const uint64_t nz = (y | (y >> 1) | (y >> 2) | (y >> 3)) & 0x0011111111111111ull;
    const uint32_t crit_e = 14u - (uint32_t)__popcll(nz);
    // fields >= 3 (edges paired with a triangle: one head triangle each)
    const uint32_t heads_t = (uint32_t)__popcll((ef + 0x0055555555555555ull) & 0x0088888888888888ull);
    // non-zero triangle fields (triangles paired with a tet: one head tet each)
    const uint64_t t0 = lo >> 56, t1 = hi;
    const uint32_t tails_t = (uint32_t)__popcll((t0 | (t0 >> 1)) & 0x55ull) +
                             (uint32_t)__popcll((t1 | (t1 >> 1)) & 0x5555555555555555ull);
    c[0] = low == 0 ? 1u : 0u;
    c[1] = crit_e;
    const uint32_t cells = g_cell_counts.n[low];
    c[2] = (cells & 0xffu) - tails_t - heads_t;
    c[3] = (cells >> 8) - tails_t;
}

__device__ __forceinline__ int64_t box_vertex(int64_t r, int64_t w0, int64_t w1, int64_t lo0,
                                              int64_t lo1, int64_t lo2, int64_t nx, int64_t ny)
{
    const int64_t i = lo0 + r % w0, j = lo1 + (r / w0) % w1, k = lo2 + r / (w0 * w1);
    return i + nx * (j + ny * k);
}

// Star triangles (bits 0..35) and star tets (bits 36..59) of L(x) for each
// 14-bit lower-neighbour mask: the cells all of whose edges are lower.
// Built like CellCounts: adding the highest lower neighbour e adds the
// triangles and tets through e whose other edges are already lower.
struct LowerCells {
    uint64_t m[1 << 14];
};

constexpr LowerCells make_lower_cells()
{
    LowerCells L{};
    const Tables &T = kTables;
    // per edge e: its star triangles and tets, each with the mask of its
    // other edges
    int n[14] = {};
    uint8_t bit[14][12] = {};
    uint16_t other[14][12] = {};
    for (int t = 0; t < 36; ++t)
        for (int c = 0; c < 2; ++c) {
            const int e = T.tri[t][c];
            bit[e][n[e]] = (uint8_t)t;
            other[e][n[e]++] = (uint16_t)(1u << T.tri[t][1 - c]);
        }
    for (int q = 0; q < 24; ++q)
        for (int c = 0; c < 3; ++c) {
            const int e = T.tet[q][c];
            uint16_t m = 0;
            for (int d = 0; d < 3; ++d)
                if (d != c) m = (uint16_t)(m | (1u << T.tet[q][d]));
            bit[e][n[e]] = (uint8_t)(36 + q);
            other[e][n[e]++] = m;
        }
    L.m[0] = 0;
    for (uint32_t low = 1; low < (1u << 14); ++low) {
        int e = 13;
        while (!((low >> e) & 1u)) --e;
        const uint32_t rest = low & ~(1u << e);
        uint64_t m = L.m[rest];
        for (int k = 0; k < n[e]; ++k)
            if ((other[e][k] & rest) == other[e][k]) m |= 1ull << bit[e][k];
        L.m[low] = m;
    }
    return L;
}

constexpr LowerCells kLowerCells = make_lower_cells();
static_assert(kLowerCells.m[(1u << 14) - 1] == (1ull << 60) - 1 && kLowerCells.m[1u << 13] == 0,
              "all 60 cells when every neighbour is lower, none for a single edge");
__device__ const LowerCells g_lower_cells = kLowerCells;

// Star triangles of each edge (edge_tris) and star tets of each triangle
// (tri_tets), staged in LDS by the fill kernels so that a field names its
// partner with one read.
struct EdgeTris {
    uint8_t t[14][8];
    uint8_t q[36][2];
};

__device__ __forceinline__ void load_edge_tris(EdgeTris &E)
{
    const int i = threadIdx.x;
    if (i < 14 * 8) {
        const int e = i / 8, j = i % 8;
        E.t[e][j] = (uint8_t)(j < kTables.edge_ntri[e] ? kTables.edge_tris[e][j] : 0);
    } else if (i < 14 * 8 + 36 * 2) {
        const int k = i - 14 * 8;
        E.q[k / 2][k % 2] = (uint8_t)kTables.tri_tets[k / 2][k % 2];
    }
}

// Writes the critical cells of one record (counts c, first slots at) as
// codes base | local index.  Only the fields that name a partner are
// visited (bit tricks on the nibbles and 2-bit fields), and the cells of
// L(x) come from one table read.
__device__ __forceinline__ void write_codes(uint64_t lo, uint64_t hi, const uint32_t *c, const uint64_t *at,
                                            int64_t base, const EdgeTris &E, int64_t *crit0, int64_t *crit1,
                                            int64_t *crit2, int64_t *crit3, int64_t cap0, int64_t cap1,
                                            int64_t cap2, int64_t cap3)
{
    if (c[0]) {
        if ((int64_t)at[0] < cap0) crit0[at[0]] = base;
        return;  // a minimum has an empty lower star beyond itself
    }
    const uint64_t ef = lo & kNib14;
    const uint64_t cells = g_lower_cells.m[lower_edges(lo)];
    // edge fields equal to 2 (critical edges): bit 4e
    const uint64_t y = ef ^ 0x0022222222222222ull;
    uint64_t me = ~(y | (y >> 1) | (y >> 2) | (y >> 3)) & 0x0011111111111111ull;
    // edge fields >= 3 (paired with triangle field - 3 of the edge): bit 4e + 3
    uint64_t mh = (ef + 0x0055555555555555ull) & 0x0088888888888888ull;
    uint64_t head_t = 0;
    while (mh) {
        const int b = __ffsll((unsigned long long)mh) - 1;
        mh &= mh - 1;
        const int e = b >> 2;
        head_t |= 1ull << E.t[e][((uint32_t)(ef >> (4 * e)) & 15u) - 3u];
    }
    // non-zero triangle fields (paired with star tet field - 1 of the triangle)
    uint64_t tail_t = 0;
    uint32_t head_q = 0;
    const uint64_t f0 = lo >> 56, f1 = hi;
    uint64_t n0 = (f0 | (f0 >> 1)) & 0x55ull;
    uint64_t n1 = (f1 | (f1 >> 1)) & 0x5555555555555555ull;
    while (n0) {
        const int b = __ffsll((unsigned long long)n0) - 1;
        n0 &= n0 - 1;
        const int t = b >> 1;
        tail_t |= 1ull << t;
        head_q |= 1u << E.q[t][((uint32_t)(f0 >> b) & 3u) - 1u];
    }
    while (n1) {
        const int b = __ffsll((unsigned long long)n1) - 1;
        n1 &= n1 - 1;
        const int t = 4 + (b >> 1);
        tail_t |= 1ull << t;
        head_q |= 1u << E.q[t][((uint32_t)(f1 >> b) & 3u) - 1u];
    }
    uint64_t mt = cells & ((1ull << 36) - 1) & ~head_t & ~tail_t;
    uint32_t mq = (uint32_t)(cells >> 36) & ~head_q;
    int64_t a = (int64_t)at[1];
    while (me) {
        const int e = (__ffsll((unsigned long long)me) - 1) >> 2;
        me &= me - 1;
        if (a < cap1) crit1[a] = base | e;
        ++a;
    }
    a = (int64_t)at[2];
    while (mt) {
        const int t = __ffsll((unsigned long long)mt) - 1;
        mt &= mt - 1;
        if (a < cap2) crit2[a] = base | t;
        ++a;
    }
    a = (int64_t)at[3];
    while (mq) {
        const int q = __ffs(mq) - 1;
        mq &= mq - 1;
        if (a < cap3) crit3[a] = base | q;
        ++a;
    }
}

// Byte tables that decode a record without walking its fields:
//   he[j][b], record byte j < 7 (edge fields 2j and 2j + 1): bits 0..35 the
//     head triangles the two fields name, bits 36 + k the edge 2j + k is
//     critical (field 2), bits 38 + k it is in L(x) (field non-zero);
//   hq[j][b], record byte 7 + j (triangle fields 4j .. 4j + 3): bits 0..23
//     the head tets they name, bits 24 + i triangle 4j + i is a tail
//     (field non-zero).
struct DecodeTables {
    uint64_t he[7][256];
    uint32_t hq[9][256];
};

constexpr DecodeTables make_decode_tables()
{
    DecodeTables D{};
    const Tables &T = kTables;
    for (int j = 0; j < 7; ++j)
        for (uint32_t b = 0; b < 256; ++b) {
            uint64_t v = 0;
            for (int k = 0; k < 2; ++k) {
                const int e = 2 * j + k;
                const uint32_t f = (b >> (4 * k)) & 15u;
                if (f == 2) v |= 1ull << (36 + k);
                if (f != 0) v |= 1ull << (38 + k);
                if (f >= 3 && (int)(f - 3) < T.edge_ntri[e]) v |= 1ull << T.edge_tris[e][f - 3];
            }
            D.he[j][b] = v;
        }
    for (int j = 0; j < 9; ++j)
        for (uint32_t b = 0; b < 256; ++b) {
            uint32_t v = 0;
            for (int i = 0; i < 4; ++i) {
                const int t = 4 * j + i;
                const uint32_t g = (b >> (2 * i)) & 3u;
                if (g == 0) continue;
                v |= 1u << (24 + i);
                if (g <= 2) v |= 1u << T.tri_tets[t][g - 1];
            }
            D.hq[j][b] = v;
        }
    return D;
}

__device__ const DecodeTables g_decode = make_decode_tables();

__device__ __forceinline__ void load_decode(DecodeTables &D)
{
    const uint32_t *src = (const uint32_t *)&g_decode;
    uint32_t *dst = (uint32_t *)&D;
    for (int i = threadIdx.x; i < (int)(sizeof(DecodeTables) / 4); i += blockDim.x) dst[i] = src[i];
}

// Critical cells of one record: edges ce (by neighbour), triangles ct and
// tets cq (by star index); returns the packed counts (pack4).
__device__ __forceinline__ uint64_t decode_record(uint64_t lo, uint64_t hi, const DecodeTables &D, uint32_t &ce,
                                                  uint64_t &ct, uint32_t &cq)
{
    uint64_t head_t = 0;
    uint32_t low = 0;
    ce = 0;
#pragma unroll
    for (int j = 0; j < 7; ++j) {
        const uint64_t v = D.he[j][(uint32_t)(lo >> (8 * j)) & 255u];
        head_t |= v;
        ce |= ((uint32_t)(v >> 36) & 3u) << (2 * j);
        low |= ((uint32_t)(v >> 38) & 3u) << (2 * j);
    }
    uint32_t head_q = 0;
    uint64_t tail_t = 0;
#pragma unroll
    for (int j = 0; j < 9; ++j) {
        const uint32_t b = j == 0 ? (uint32_t)(lo >> 56) : (uint32_t)(hi >> (8 * (j - 1))) & 255u;
        const uint32_t v = D.hq[j][b];
        head_q |= v;
        tail_t |= (uint64_t)(v >> 24) << (4 * j);
    }
    const uint64_t cells = g_lower_cells.m[low];
    ct = cells & ~head_t & ~tail_t & ((1ull << 36) - 1);
    cq = (uint32_t)(cells >> 36) & ~head_q & 0xffffffu;
    const uint64_t c0 = low == 0 ? 1u : 0u;  // L(x) = {x}: nothing else is in it
    return c0 | ((uint64_t)__popc(ce) << 16) | ((uint64_t)__popcll((unsigned long long)ct) << 32) |
           ((uint64_t)__popc(cq) << 48);
}

// Per-record counts packed in 16-bit lanes (dimension d in bits 16d..16d+15);
// a block's sums fit: at most 36 x 1024 cells of one dimension.
__device__ __forceinline__ uint64_t pack4(const uint32_t *c)
{
    return (uint64_t)c[0] | ((uint64_t)c[1] << 16) | ((uint64_t)c[2] << 32) | ((uint64_t)c[3] << 48);
}

__device__ __forceinline__ uint32_t lane16(uint64_t v, int d) { return (uint32_t)(v >> (16 * d)) & 0xffffu; }

__device__ __forceinline__ void load_recs(const uint4 *__restrict__ rec, int64_t nbox, int64_t r0,
                                          uint64_t *lo, uint64_t *hi, uint64_t *packed)
{
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
        uint32_t c[4] = {0, 0, 0, 0};
        lo[k] = hi[k] = 0;
        if (r0 + k < nbox) {
            const uint4 w = rec[r0 + k];
            lo[k] = (uint64_t)w.x | ((uint64_t)w.y << 32);
            hi[k] = (uint64_t)w.z | ((uint64_t)w.w << 32);
            count_critical(lo[k], hi[k], c);
        }
        packed[k] = pack4(c);
    }
}

// cand (may be null): kCand uint16 tile positions per tile, ncand: their
// number per tile (the true number, also beyond kCand).  Records are read
// striped (record k * kThreads + tid of the tile), so the loads coalesce;
// the candidates are listed in record order (row k before row k + 1).
__global__ __launch_bounds__(kThreads) void k_crit_count(const uint4 *__restrict__ rec, int64_t nbox,
                                                         uint64_t *__restrict__ tile_counts,
                                                         int64_t ntiles, uint16_t *__restrict__ cand,
                                                         uint32_t *__restrict__ ncand)
{
    __shared__ uint64_t wsum[kThreads / kWave];
    const int tid = threadIdx.x;
    const int64_t t0 = (int64_t)blockIdx.x * kTileRecs;
    uint64_t pk[kPerThread];
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
        const int64_t r = t0 + k * kThreads + tid;
        uint32_t c[4] = {0, 0, 0, 0};
        if (r < nbox) {
            const uint4 w = rec[r];
            count_critical((uint64_t)w.x | ((uint64_t)w.y << 32), (uint64_t)w.z | ((uint64_t)w.w << 32), c);
        }
        pk[k] = pack4(c);
    }
    uint64_t sum = pk[0] + pk[1] + pk[2] + pk[3];
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
    if (lane_id() == 0) wsum[tid / kWave] = sum;
    __syncthreads();
    if (tid < 4) {
        uint64_t t = 0;
#pragma unroll
        for (int w = 0; w < kThreads / kWave; ++w) t += wsum[w];
        tile_counts[(int64_t)tid * ntiles + blockIdx.x] = lane16(t, tid);
    }
    if (blockIdx.x == 0 && tid == 0) tile_counts[4 * ntiles] = 0;
    if (cand) {
        // one 16-bit field per row: the row's candidates, scanned over the block
        uint64_t mine = 0;
#pragma unroll
        for (int k = 0; k < kPerThread; ++k) mine |= (uint64_t)(pk[k] != 0 ? 1u : 0u) << (16 * k);
        uint64_t tot;
        const uint64_t ex = block_exclusive_scan<uint64_t>(mine, &tot);
        uint32_t row_base = 0;
#pragma unroll
        for (int k = 0; k < kPerThread; ++k) {
            if (pk[k] != 0) {
                const uint32_t a = row_base + lane16(ex, k);
                if (a < (uint32_t)kCand)
                    cand[(int64_t)blockIdx.x * kCand + a] = (uint16_t)(k * kThreads + tid);
            }
            row_base += lane16(tot, k);
        }
        if (tid == 0) ncand[blockIdx.x] = row_base;
    }
}

// Shared by the single-field and batched fill: records [r0, r0 + 4) of
// this thread, their packed counts, and the first slot of each list for
// the first of them.
__device__ __forceinline__ void fill_slots(const uint64_t *pk, const uint64_t *__restrict__ offs,
                                           int64_t ntiles, uint64_t at[kPerThread][4])
{
    uint64_t total;
    uint64_t run = block_exclusive_scan<uint64_t>(pk[0] + pk[1] + pk[2] + pk[3], &total);
    uint64_t base[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) base[d] = offs[(int64_t)d * ntiles + blockIdx.x] - offs[(int64_t)d * ntiles];
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
#pragma unroll
        for (int d = 0; d < 4; ++d) at[k][d] = base[d] + lane16(run, d);
        run += pk[k];
    }
}

// All records of one tile (the whole block).
__device__ __forceinline__ void fill_tile_full(
    const uint4 *__restrict__ rec, int64_t nbox, const uint64_t *__restrict__ offs, int64_t ntiles,
    int64_t w0, int64_t w1, int64_t lo0, int64_t lo1, int64_t lo2, int64_t nx, int64_t ny, const EdgeTris &E,
    int64_t *crit0, int64_t *crit1, int64_t *crit2, int64_t *crit3, int64_t cap0, int64_t cap1,
    int64_t cap2, int64_t cap3)
{
    const int64_t r0 = (int64_t)blockIdx.x * kTileRecs + (int64_t)threadIdx.x * kPerThread;
    uint64_t lo[kPerThread], hi[kPerThread], pk[kPerThread], at[kPerThread][4];
    load_recs(rec, nbox, r0, lo, hi, pk);
    fill_slots(pk, offs, ntiles, at);
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
        if (r0 + k >= nbox || pk[k] == 0) continue;
        uint32_t c[4];
#pragma unroll
        for (int d = 0; d < 4; ++d) c[d] = lane16(pk[k], d);
        const int64_t v = box_vertex(r0 + k, w0, w1, lo0, lo1, lo2, nx, ny);
        write_codes(lo[k], hi[k], c, at[k], v << 8, E, crit0, crit1, crit2, crit3, cap0, cap1, cap2,
                           cap3);
    }
}

// Fill from the candidate lists: a tile with at most kCand listed records
// reads only those (one wave; their slots from a wave scan of the packed
// counts), a tile with more is re-read whole, a tile with none is skipped.
__global__ __launch_bounds__(kThreads) void k_crit_fill(
    const uint4 *__restrict__ rec, int64_t nbox, const uint64_t *__restrict__ offs, int64_t ntiles,
    const uint16_t *__restrict__ cand, const uint32_t *__restrict__ ncand, int64_t w0, int64_t w1,
    int64_t lo0, int64_t lo1, int64_t lo2, int64_t nx, int64_t ny, int64_t *crit0, int64_t *crit1,
    int64_t *crit2, int64_t *crit3, int64_t cap0, int64_t cap1, int64_t cap2, int64_t cap3)
{
    __shared__ EdgeTris E;
    const uint32_t n = ncand[blockIdx.x];
    if (n == 0) return;  // uniform
    load_edge_tris(E);
    __syncthreads();
    if (n > (uint32_t)kCand) {
        fill_tile_full(rec, nbox, offs, ntiles, w0, w1, lo0, lo1, lo2, nx, ny, E, crit0, crit1, crit2,
                       crit3, cap0, cap1, cap2, cap3);
        return;
    }
    if (threadIdx.x >= kWave) return;
    const int lane = threadIdx.x;
    const bool active = (uint32_t)lane < n;
    uint64_t lo = 0, hi = 0, pk = 0;
    int64_t r = 0;
    if (active) {
        r = (int64_t)blockIdx.x * kTileRecs + cand[(int64_t)blockIdx.x * kCand + lane];
        if (r < nbox) {
            const uint4 w = rec[r];
            lo = (uint64_t)w.x | ((uint64_t)w.y << 32);
            hi = (uint64_t)w.z | ((uint64_t)w.w << 32);
            uint32_t c[4];
            count_critical(lo, hi, c);
            pk = pack4(c);
        }
    }
    // exclusive scan of the packed counts over the wave
    uint64_t inc = pk;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const uint64_t t = __shfl_up(inc, off);
        if (lane >= off) inc += t;
    }
    const uint64_t ex = inc - pk;
    if (pk == 0) return;
    uint64_t at[4];
    uint32_t c[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        at[d] = offs[(int64_t)d * ntiles + blockIdx.x] - offs[(int64_t)d * ntiles] + lane16(ex, d);
        c[d] = lane16(pk, d);
    }
    const int64_t v = box_vertex(r, w0, w1, lo0, lo1, lo2, nx, ny);
    write_codes(lo, hi, c, at, v << 8, E, crit0, crit1, crit2, crit3, cap0, cap1, cap2, cap3);
}

// Position of the n-th set bit (n < popc(x)), by halving.
__device__ __forceinline__ uint32_t select_bit(uint32_t x, uint32_t n)
{
    uint32_t pos = 0;
#pragma unroll
    for (uint32_t s = 16; s > 0; s >>= 1) {
        const uint32_t c = (uint32_t)__popc(x & ((1u << s) - 1u));
        if (n >= c) {
            n -= c;
            x >>= s;
            pos += s;
        }
    }
    return pos;
}

// Writes the critical cells of a wave's records, one record per lane (ce,
// ct, cq from decode_record; v its vertex id as the codes carry it; pk its
// packed counts, zero for lanes without a record), in lane order: the codes
// of list d go to slots at[d] .. at[d] + (its total) - 1, one code per lane
// per round, so each store is contiguous.  Code j of list d belongs to the
// first lane whose inclusive count exceeds j (a binary search over the
// wave's scan) and names that record's (j - earlier)-th cell.  Returns the
// wave's packed totals.  Every lane of the wave must call it.
__device__ __forceinline__ uint64_t emit_codes(uint32_t ce, uint64_t ct, uint32_t cq, int64_t v, uint64_t pk,
                                               const uint64_t *at, int64_t *crit0, int64_t *crit1,
                                               int64_t *crit2, int64_t *crit3, int64_t cap0, int64_t cap1,
                                               int64_t cap2, int64_t cap3)
{
    const int lane = lane_id();
    uint64_t inc = pk;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const uint64_t u = __shfl_up(inc, off);
        if (lane >= off) inc += u;
    }
    const uint64_t tot = __shfl(inc, kWave - 1);
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const uint32_t total = lane16(tot, d);
        const uint32_t incd = lane16(inc, d);
        int64_t *const out = d == 0 ? crit0 : d == 1 ? crit1 : d == 2 ? crit2 : crit3;
        const int64_t cap = d == 0 ? cap0 : d == 1 ? cap1 : d == 2 ? cap2 : cap3;
        for (uint32_t j0 = 0; j0 < total; j0 += kWave) {
            const uint32_t j = j0 + (uint32_t)lane;
            int w = 0;
#pragma unroll
            for (int step = kWave / 2; step > 0; step >>= 1)
                if (__shfl(incd, w + step - 1) <= j) w += step;
            const uint32_t prev = __shfl(incd, w > 0 ? w - 1 : 0);
            const uint32_t n = j - (w > 0 ? prev : 0u);
            const int64_t ov = __shfl(v, w);
            uint32_t local = 0;
            if (d == 1) {
                local = select_bit(__shfl(ce, w), n);
            } else if (d == 2) {
                const uint64_t m = __shfl(ct, w);
                const uint32_t m0 = (uint32_t)m, c = (uint32_t)__popc(m0);
                local = n < c ? select_bit(m0, n) : 32u + select_bit((uint32_t)(m >> 32), n - c);
            } else if (d == 3) {
                local = select_bit(__shfl(cq, w), n);
            }
            const int64_t a = (int64_t)at[d] + (int64_t)j;
            if (j < total && a < cap) out[a] = (ov << 8) | (int64_t)local;
        }
    }
    return tot;
}

// ---------------------------------------------------------------------------
// Masked extraction: the gradient set bit r of the mask for every record r
// holding a critical cell, so the other records need not be read.  A wave
// takes kTilesPerWave consecutive tiles, whose mask words it holds one per
// lane, and their flagged records kWave at a time in record order: lane j
// takes the chunk's j-th.  A smooth field flags few records (one chunk, one
// load for the whole wave); a noise field flags about a quarter, most rows
// of 64 records among them, so a walk by rows would read and decode nearly
// all.  The tiles' slots in the scanned counts are consecutive, so one
// running offset serves both tiles.
constexpr int kTileWords = kTileRecs / 32;
constexpr int kTilesPerWave = kWave / kTileWords;
constexpr int kWavesPerBlock = kThreads / kWave;
static_assert(kWave == 64 && kTilesPerWave == 2, "one mask word per lane");

// The wave's flagged records: word = mask word `lane` of the wave's tiles.
// flag_scan returns their number and sets inc (inclusive scan of the words'
// bit counts over the lanes); flag_at gives the j-th flagged record's
// position from the first tile's start (j below the number).
__device__ __forceinline__ uint32_t flag_scan(uint32_t word, int lane, uint32_t &inc)
{
    inc = (uint32_t)__popc(word);
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const uint32_t t = __shfl_up(inc, off);
        if (lane >= off) inc += t;
    }
    return __shfl(inc, kWave - 1);
}

__device__ __forceinline__ uint32_t flag_at(uint32_t word, uint32_t inc, uint32_t j)
{
    // the word holding flagged record j: the first w with inc[w] > j
    int w = 0;
#pragma unroll
    for (int step = kWave / 2; step > 0; step >>= 1)
        if (__shfl(inc, w + step - 1) <= j) w += step;
    const uint32_t ww = __shfl(word, w);
    const uint32_t before = __shfl(inc, w) - (uint32_t)__popc(ww);
    return (uint32_t)w * 32u + select_bit(ww, j - before);
}

__device__ __forceinline__ uint64_t count_record(const uint4 *__restrict__ rec, int64_t r, uint64_t &lo,
                                                 uint64_t &hi)
{
    const uint4 w = rec[r];
    lo = (uint64_t)w.x | ((uint64_t)w.y << 32);
    hi = (uint64_t)w.z | ((uint64_t)w.w << 32);
    uint32_t c[4];
    count_critical(lo, hi, c);
    return pack4(c);
}

__global__ __launch_bounds__(kThreads) void k_crit_count_masked(const uint4 *__restrict__ rec,
                                                                const uint32_t *__restrict__ mask,
                                                                int64_t nbox,
                                                                uint64_t *__restrict__ tile_counts,
                                                                int64_t ntiles)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) tile_counts[4 * ntiles] = 0;
    const int lane = lane_id();
    const int64_t tile0 =
        (int64_t)__builtin_amdgcn_readfirstlane((int)(blockIdx.x * kWavesPerBlock + threadIdx.x / kWave)) *
        kTilesPerWave;
    if (tile0 >= ntiles) return;
    const int64_t wi = tile0 * kTileWords + lane;
    const uint32_t word = wi < (nbox + 31) / 32 ? mask[wi] : 0u;
    const int64_t r0 = tile0 * kTileRecs;
    uint32_t inc;
    const uint32_t total = flag_scan(word, lane, inc);
    uint64_t sum[kTilesPerWave] = {0, 0};
#pragma unroll 1
    for (uint32_t c0 = 0; c0 < total; c0 += kWave) {
        const uint32_t j = c0 + (uint32_t)lane;
        const uint32_t rel = flag_at(word, inc, j < total ? j : c0);  // every lane takes part in the shuffles
        uint64_t lo, hi;
        if (j < total && r0 + rel < nbox) {
            const uint64_t pk = count_record(rec, r0 + rel, lo, hi);
            if (rel < (uint32_t)kTileRecs) sum[0] += pk; else sum[1] += pk;
        }
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        sum[0] += __shfl_xor(sum[0], off);
        sum[1] += __shfl_xor(sum[1], off);
    }
#pragma unroll
    for (int t = 0; t < kTilesPerWave; ++t)
        if (lane < 4 && tile0 + t < ntiles) tile_counts[(int64_t)lane * ntiles + tile0 + t] = lane16(sum[t], lane);
}

__global__ __launch_bounds__(kThreads) void k_crit_fill_masked(
    const uint4 *__restrict__ rec, const uint32_t *__restrict__ mask, int64_t nbox,
    const uint64_t *__restrict__ offs, int64_t ntiles, int64_t w0, int64_t w1, int64_t lo0, int64_t lo1,
    int64_t lo2, int64_t nx, int64_t ny, int64_t *crit0, int64_t *crit1, int64_t *crit2, int64_t *crit3,
    int64_t cap0, int64_t cap1, int64_t cap2, int64_t cap3)
{
    // few records per block: the decode tables are read where they are
    // (cached) rather than staged in LDS
    const DecodeTables &D = g_decode;
    const int lane = lane_id();
    const int64_t tile0 =
        (int64_t)__builtin_amdgcn_readfirstlane((int)(blockIdx.x * kWavesPerBlock + threadIdx.x / kWave)) *
        kTilesPerWave;
    if (tile0 >= ntiles) return;
    const int64_t wi = tile0 * kTileWords + lane;
    const uint32_t word = wi < (nbox + 31) / 32 ? mask[wi] : 0u;
    if (!__ballot(word != 0u)) return;
    uint64_t at[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) at[d] = offs[(int64_t)d * ntiles + tile0] - offs[(int64_t)d * ntiles];
    const int64_t r0 = tile0 * kTileRecs;
    uint32_t inc;
    const uint32_t total = flag_scan(word, lane, inc);
#pragma unroll 1
    for (uint32_t c0 = 0; c0 < total; c0 += kWave) {
        const uint32_t j = c0 + (uint32_t)lane;
        const bool take = j < total;
        const int64_t r = r0 + flag_at(word, inc, take ? j : c0);
        uint64_t pk = 0;
        uint32_t ce = 0, cq = 0;
        uint64_t ct = 0;
        int64_t v = 0;
        if (take && r < nbox) {
            const uint4 w = rec[r];
            pk = decode_record((uint64_t)w.x | ((uint64_t)w.y << 32), (uint64_t)w.z | ((uint64_t)w.w << 32), D,
                               ce, ct, cq);
            v = box_vertex(r, w0, w1, lo0, lo1, lo2, nx, ny);
        }
        if (!__ballot(pk != 0)) continue;
        const uint64_t tot =
            emit_codes(ce, ct, cq, v, pk, at, crit0, crit1, crit2, crit3, cap0, cap1, cap2, cap3);
#pragma unroll
        for (int d = 0; d < 4; ++d) at[d] += lane16(tot, d);
    }
}

__global__ void k_crit_finish(const uint64_t *offs, int64_t ntiles, int64_t *counts, int64_t cap0,
                              int64_t cap1, int64_t cap2, int64_t cap3, uint32_t *flags)
{
    if (threadIdx.x != 0) return;
    const int64_t cap[4] = {cap0, cap1, cap2, cap3};
    bool over = false;
    for (int d = 0; d < 4; ++d) {
        const int64_t tot = (int64_t)(offs[(int64_t)(d + 1) * ntiles] - offs[(int64_t)d * ntiles]);
        counts[d] = tot;
        over = over || tot > cap[d];
    }
    if (over) atomicOr(flags, (uint32_t)DMS_FLAG_CAPACITY);
}


// Batched fill from the critical mask: records of whole fields
// concatenated; codes carry the field-local vertex id.  A wave takes
// kTilesPerWave consecutive tiles (one mask word per lane) and their flagged
// records kWave at a time, in record order (lane j the chunk's j-th), so that
// every decode serves a flagged record; a chunk's codes leave as one run at
// the running offset.  Most records of a noise field hold no critical cell,
// but most rows of 64 records hold one, so walking rows would decode them all.
__global__ __launch_bounds__(kThreads) void k_crit_fill_batch(
    const uint4 *__restrict__ rec, const uint32_t *__restrict__ mask, int64_t nbox,
    const uint64_t *__restrict__ offs, int64_t ntiles, const int64_t *__restrict__ foff, int nfields,
    int64_t *crit0, int64_t *crit1, int64_t *crit2, int64_t *crit3, int64_t cap0, int64_t cap1, int64_t cap2,
    int64_t cap3)
{
    __shared__ int64_t so[kMaxBatchFields + 1];
    __shared__ DecodeTables D;
    for (int i = threadIdx.x; i <= nfields; i += kThreads) so[i] = foff[i];
    load_decode(D);
    __syncthreads();
    const int lane = lane_id();
    const int64_t tile0 =
        (int64_t)__builtin_amdgcn_readfirstlane((int)(blockIdx.x * kWavesPerBlock + threadIdx.x / kWave)) *
        kTilesPerWave;
    if (tile0 >= ntiles) return;
    const int64_t wi = tile0 * kTileWords + lane;
    const uint32_t word = wi < (nbox + 31) / 32 ? mask[wi] : 0u;
    if (!__ballot(word != 0u)) return;
    uint64_t at[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) at[d] = offs[(int64_t)d * ntiles + tile0] - offs[(int64_t)d * ntiles];
    const int64_t r0 = tile0 * kTileRecs;
    // field of the wave's first record (uniform); a lane's record lies in it
    // or in a later field
    int f0 = 0;
    for (int step = 1 << 10; step > 0; step >>= 1)
        if (f0 + step < nfields && so[f0 + step] <= r0) f0 += step;
    uint32_t inc;
    const uint32_t total = flag_scan(word, lane, inc);
#pragma unroll 1
    for (uint32_t c0 = 0; c0 < total; c0 += kWave) {
        const uint32_t j = c0 + (uint32_t)lane;
        const bool take = j < total;
        const int64_t r = r0 + flag_at(word, inc, take ? j : c0);
        uint64_t pk = 0;
        uint32_t ce = 0, cq = 0;
        uint64_t ct = 0;
        int f = f0;
        if (take && r < nbox) {
            const uint4 w = rec[r];
            pk = decode_record((uint64_t)w.x | ((uint64_t)w.y << 32), (uint64_t)w.z | ((uint64_t)w.w << 32), D,
                               ce, ct, cq);
            while (f + 1 < nfields && so[f + 1] <= r) ++f;
        }
        if (!__ballot(pk != 0)) continue;
        const uint64_t tot =
            emit_codes(ce, ct, cq, r - so[f], pk, at, crit0, crit1, crit2, crit3, cap0, cap1, cap2, cap3);
#pragma unroll
        for (int d = 0; d < 4; ++d) at[d] += lane16(tot, d);
    }
}

// First slot of every field in every list: the scanned count of its first
// record's tile plus the counts of the tile's records before it (one block
// per field).
__global__ __launch_bounds__(kThreads) void k_crit_fstart_batch(const uint4 *__restrict__ rec,
                                                                const uint64_t *__restrict__ offs,
                                                                int64_t ntiles,
                                                                const int64_t *__restrict__ foff,
                                                                int nfields, int64_t *fstart)
{
    const int f = blockIdx.x;
    const int64_t r = foff[f];
    const int64_t tile = r / kTileRecs;
    uint64_t sum = 0;
    for (int64_t q = tile * kTileRecs + threadIdx.x; q < r; q += kThreads) {
        const uint4 w = rec[q];
        uint32_t c[4];
        count_critical((uint64_t)w.x | ((uint64_t)w.y << 32), (uint64_t)w.z | ((uint64_t)w.w << 32), c);
        sum += pack4(c);
    }
    uint64_t total;
    block_exclusive_scan<uint64_t>(sum, &total);
    if (threadIdx.x == 0 && tile < ntiles)
        for (int d = 0; d < 4; ++d)
            fstart[(int64_t)d * (nfields + 1) + f] =
                (int64_t)(offs[(int64_t)d * ntiles + tile] - offs[(int64_t)d * ntiles] + lane16(total, d));
}

__global__ void k_crit_finish_batch(const uint64_t *offs, int64_t ntiles, int nfields, int64_t *fstart,
                                    int64_t *counts, int64_t cap0, int64_t cap1, int64_t cap2,
                                    int64_t cap3, uint32_t *flags)
{
    const int64_t cap[4] = {cap0, cap1, cap2, cap3};
    for (int d = 0; d < 4; ++d) {
        const int64_t tot = (int64_t)(offs[(int64_t)(d + 1) * ntiles] - offs[(int64_t)d * ntiles]);
        if (threadIdx.x == 0) {
            fstart[(int64_t)d * (nfields + 1) + nfields] = tot;
            if (tot > cap[d]) atomicOr(flags, (uint32_t)DMS_FLAG_CAPACITY);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 4 * nfields; i += blockDim.x) {
        const int f = i / 4, d = i % 4;
        const int64_t *fs = fstart + (int64_t)d * (nfields + 1);
        counts[i] = fs[f + 1] - fs[f];
    }
}

__global__ void k_crit_empty(int64_t *counts)
{
    if (threadIdx.x < 4) counts[threadIdx.x] = 0;
}

}  // namespace
}  // namespace dms


namespace dms {

// Single-field workspace: tile counts (4 x ntiles + 1, scanned in place),
// scan partials, candidate positions (kCand per tile), candidate counts.
struct CritLayout {
    size_t partials, cand, ncand, total;
};

constexpr CritLayout crit_layout(int64_t ntiles)
{
    const int64_t len = 4 * ntiles + 1;
    CritLayout L{};
    size_t off = align_up((size_t)len * 8, 256);
    L.partials = off; off += scan_partials_bytes(len, 8);
    L.cand = off; off += align_up((size_t)ntiles * kCand * 2, 256);
    L.ncand = off; off += align_up((size_t)ntiles * 4, 256);
    L.total = off;
    return L;
}

// Allocation-free extraction: its workspace lives in this file-scope device
// array, one per device, for boxes of up to kNoAllocTiles tiles of
// kTileRecs records.  Host code reaches the array only through the address
// hipGetSymbolAddress gives on each device (init_critical_scratch).
constexpr int64_t kNoAllocTiles = 160 * 1024;  // boxes of up to 167,772,160 vertices
constexpr size_t kNoAllocBytes = crit_layout(kNoAllocTiles).total;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];
static std::atomic<char *> g_scratch[64];  // per device: the array's device address

// Enqueues the extraction of box [lo, hi) into crit0..3 with the workspace
// ws (crit_layout of the box's tiles); arguments already checked.
int launch_critical(const uint32_t *rec, const uint32_t *mask, const int64_t *dims, const int64_t *lo,
                    const int64_t *hi, int64_t *crit0, int64_t *crit1, int64_t *crit2, int64_t *crit3, const int64_t *cap,
                    int64_t *counts, char *workspace, uint32_t *dev_flags, hipStream_t s)
{
    const int64_t w0 = hi[0] - lo[0], w1 = hi[1] - lo[1], w2 = hi[2] - lo[2];
    const int64_t nbox = w0 * w1 * w2;
    const int64_t ntiles = (nbox + kTileRecs - 1) / kTileRecs;
    const int64_t len = 4 * ntiles + 1;
    const CritLayout L = crit_layout(ntiles);
    uint64_t *tc = (uint64_t *)workspace;
    uint64_t *partials = (uint64_t *)(workspace + L.partials);
    uint16_t *cand = (uint16_t *)(workspace + L.cand);
    uint32_t *ncand = (uint32_t *)(workspace + L.ncand);
    if (ntiles == 0) {
        hipLaunchKernelGGL(k_crit_empty, dim3(1), dim3(64), 0, s, counts);
        return launch_status();
    }
    if (mask) {
        const int64_t per_block = (int64_t)kWavesPerBlock * kTilesPerWave;
        const unsigned blocks = (unsigned)((ntiles + per_block - 1) / per_block);
        hipLaunchKernelGGL(k_crit_count_masked, dim3(blocks), dim3(kThreads), 0, s, (const uint4 *)rec, mask,
                           nbox, tc, ntiles);
        exclusive_scan<uint64_t>(tc, len, partials, s);
        hipLaunchKernelGGL(k_crit_fill_masked, dim3(blocks), dim3(kThreads), 0, s, (const uint4 *)rec, mask,
                           nbox, tc, ntiles, w0, w1, lo[0], lo[1], lo[2], dims[0], dims[1], crit0, crit1,
                           crit2, crit3, cap[0], cap[1], cap[2], cap[3]);
    } else {
        hipLaunchKernelGGL(k_crit_count, dim3((unsigned)ntiles), dim3(kThreads), 0, s, (const uint4 *)rec,
                           nbox, tc, ntiles, cand, ncand);
        exclusive_scan<uint64_t>(tc, len, partials, s);
        hipLaunchKernelGGL(k_crit_fill, dim3((unsigned)ntiles), dim3(kThreads), 0, s, (const uint4 *)rec,
                           nbox, tc, ntiles, cand, ncand, w0, w1, lo[0], lo[1], lo[2], dims[0], dims[1],
                           crit0, crit1, crit2, crit3, cap[0], cap[1], cap[2], cap[3]);
    }
    hipLaunchKernelGGL(k_crit_finish, dim3(1), dim3(64), 0, s, tc, ntiles, counts, cap[0], cap[1],
                       cap[2], cap[3], dev_flags);
    return launch_status();
}

// Argument checks shared by both extraction entry points.
int check_critical_args(const uint32_t *rec, const int64_t *dims, const int64_t *lo, const int64_t *hi,
                        int64_t *crit0, int64_t *crit1, int64_t *crit2, int64_t *crit3, const int64_t *cap,
                        const int64_t *counts, const uint32_t *dev_flags)
{
    if (!box_valid(dims, lo, hi) || !cap || !counts || !dev_flags) return DMS_E_ARG;
    if (!grid_size_values_ok(dims)) return DMS_E_SIZE;
    for (int d = 0; d < 4; ++d)
        if (cap[d] < 0) return DMS_E_ARG;
    if ((cap[0] && !crit0) || (cap[1] && !crit1) || (cap[2] && !crit2) || (cap[3] && !crit3))
        return DMS_E_ARG;
    const int64_t nbox = (hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2]);
    if (nbox > 0 && !rec) return DMS_E_ARG;
    return DMS_OK;
}

size_t critical_batch_workspace_size(int64_t n, int nfields)
{
    (void)nfields;
    return crit_layout((n + kTileRecs - 1) / kTileRecs).total;
}

int launch_critical_batch(const uint32_t *rec, const uint32_t *mask, int64_t n, const int64_t *foff,
                          int nfields, const BatchField *fields, int64_t *const crit[4], const int64_t cap[4],
                          int64_t *counts, int64_t *offsets, char *ws, uint32_t *flags, hipStream_t s)
{
    (void)fields;
    if (!mask) return DMS_E_ARG;
    const int64_t ntiles = (n + kTileRecs - 1) / kTileRecs;
    const int64_t len = 4 * ntiles + 1;
    const CritLayout L = crit_layout(ntiles);
    uint64_t *tc = (uint64_t *)ws;
    uint64_t *partials = (uint64_t *)(ws + L.partials);
    const int64_t per_block = (int64_t)kWavesPerBlock * kTilesPerWave;
    const unsigned blocks = (unsigned)((ntiles + per_block - 1) / per_block);
    hipLaunchKernelGGL(k_crit_count_masked, dim3(blocks), dim3(kThreads), 0, s, (const uint4 *)rec, mask, n, tc,
                       ntiles);
    exclusive_scan<uint64_t>(tc, len, partials, s);
    hipLaunchKernelGGL(k_crit_fill_batch, dim3(blocks), dim3(kThreads), 0, s, (const uint4 *)rec, mask, n, tc,
                       ntiles, foff, nfields, crit[0], crit[1], crit[2], crit[3], cap[0], cap[1], cap[2], cap[3]);
    hipLaunchKernelGGL(k_crit_fstart_batch, dim3((unsigned)nfields), dim3(kThreads), 0, s, (const uint4 *)rec,
                       tc, ntiles, foff, nfields, offsets);
    hipLaunchKernelGGL(k_crit_finish_batch, dim3(1), dim3(256), 0, s, tc, ntiles, nfields, offsets,
                       counts, cap[0], cap[1], cap[2], cap[3], flags);
    return launch_status();
}

int init_critical_scratch()
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return DMS_E_HIP;
    if (g_scratch[dev].load()) return DMS_OK;
    char *ptr = nullptr;
    if (hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return DMS_E_HIP;
    g_scratch[dev].store(ptr);
    return DMS_OK;
}

}  // namespace dms

extern "C" size_t dms_critical_workspace_size(const int64_t dims[3], const int64_t lo[3],
                                              const int64_t hi[3])
{
    using namespace dms;
    if (!box_valid(dims, lo, hi)) return 0;
    const int64_t nbox = (hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2]);
    return crit_layout((nbox + kTileRecs - 1) / kTileRecs).total;
}

extern "C" int dms_critical_simplices(const uint32_t *rec, const uint32_t *critical_mask,
                                      const int64_t dims[3], const int64_t lo[3],
                                      const int64_t hi[3], int64_t *crit0, int64_t *crit1,
                                      int64_t *crit2, int64_t *crit3, const int64_t cap[4],
                                      int64_t *counts, void *workspace, size_t workspace_bytes,
                                      uint32_t *dev_flags, void *stream)
{
    using namespace dms;
    if (const int st = check_critical_args(rec, dims, lo, hi, crit0, crit1, crit2, crit3, cap, counts, dev_flags))
        return st;
    const size_t need = dms_critical_workspace_size(dims, lo, hi);
    if (!workspace || workspace_bytes < need) return DMS_E_WORKSPACE;
    if (const int dc = device_check()) return dc;
    return launch_critical(rec, critical_mask, dims, lo, hi, crit0, crit1, crit2, crit3, cap, counts,
                           (char *)workspace,
                           dev_flags, (hipStream_t)stream);
}

extern "C" int dms_critical_simplices_noalloc(const uint32_t *rec, const uint32_t *critical_mask,
                                              const int64_t dims[3], const int64_t lo[3],
                                              const int64_t hi[3], int64_t *crit0, int64_t *crit1,
                                              int64_t *crit2, int64_t *crit3, const int64_t cap[4],
                                              int64_t *counts, uint32_t *dev_flags, void *stream)
{
    using namespace dms;
    if (const int st = check_critical_args(rec, dims, lo, hi, crit0, crit1, crit2, crit3, cap, counts, dev_flags))
        return st;
    const int64_t nbox = (hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2]);
    if ((nbox + kTileRecs - 1) / kTileRecs > kNoAllocTiles) return DMS_E_SIZE;
    if (const int dc = device_check()) return dc;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return DMS_E_HIP;
    char *ws = g_scratch[dev].load();
    if (!ws) return DMS_E_NOT_INITIALISED;
    return launch_critical(rec, critical_mask, dims, lo, hi, crit0, crit1, crit2, crit3, cap, counts, ws,
                           dev_flags,
                           (hipStream_t)stream);
}
