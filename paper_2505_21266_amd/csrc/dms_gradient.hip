// dms_gradient.hip -- discrete gradient by Robins et al.'s ProcessLowerStars,
// one GPU thread per vertex (Section 2.3: the gradient is computed by
// inspecting the local neighbourhood of each vertex, which makes the step
// embarrassingly parallel; cells are compared as in Section 2.1).
//
// Per vertex x, with the orders of x and its 14 neighbours staged in LDS:
//  1. the lower neighbours are ranked among themselves; the key of a cell of
//     the lower star L(x) (its vertex orders listed decreasingly, compared
//     lexicographically) then equals the integer whose bits are the ranks of
//     its lower vertices, so faces precede cofaces and "smallest" is an
//     integer minimum, found by a bit-sliced scan over per-rank planes;
//  2. Robins' pairing runs in registers on bitsets over the star's cells
//     (unpaired cells, and a bit-sliced count of each cell's unpaired facets)
//     -- see process_vertex for why the two priority queues need no storage;
//  3. the outcome is packed into the 16-byte record described in dms.h.
// Readings: "unpaired" = neither paired nor critical; only unpaired cells
// enter the one-facet queue; entries of the zero queue that get paired are
// dropped (Robins' lazy deletion gives the same pops).
#include <atomic>
#include <mutex>

#include "dms_common.hpp"
#include "dms_internal.hpp"
#include "dms_tables.hpp"

namespace dms {
namespace {

constexpr int kThreads = 256;      // threads per block
constexpr int kTileVerts = 1024;  // vertices per tile (4 per thread)
constexpr int32_t kAbsent = 0x7fffffff;
constexpr int kSizeBins = 77;  // keys 1 + lower-star size (1..75); bin 76 stays empty

// Star cells other than x and the edges: triangles t -> bit t, tets q -> bit
// 36 + q of a 64-bit mask ("TQ space").
constexpr uint64_t kTriBits = (1ull << 36) - 1;

struct SharedTables {
    uint64_t cont[14];     // TQ cells containing neighbour e
    uint64_t facet[60];    // triangle: its two edges (neighbour bits); tet: its 3 triangles (TQ bits)
    uint64_t cofacet[60];  // triangle: the tets containing it (TQ bits); tet: 0
    uint8_t tri_ab[36];    // a | b << 4
    uint8_t tri_slot[36];  // slot of t in the triangle list of a | of b << 4
    uint8_t tri_tet0[36];  // first star tet containing t
    uint8_t tet_abc[24][3];
    uint8_t pad[4];
};

constexpr SharedTables make_shared_tables()
{
    SharedTables d{};
    const Tables &T = kTables;
    for (int e = 0; e < 14; ++e) d.cont[e] = T.edge_trimask[e] | ((uint64_t)T.edge_tetmask[e] << 36);
    for (int t = 0; t < 36; ++t) {
        d.facet[t] = T.tri_edgemask[t];
        d.cofacet[t] = (uint64_t)T.tri_tetmask[t] << 36;
        d.tri_ab[t] = (uint8_t)(T.tri[t][0] | (T.tri[t][1] << 4));
        d.tri_slot[t] = (uint8_t)(T.tri_slot[t][0] | (T.tri_slot[t][1] << 4));
        d.tri_tet0[t] = (uint8_t)T.tri_tets[t][0];
    }
    for (int q = 0; q < 24; ++q) {
        d.facet[36 + q] = T.tet_trimask[q];
        d.cofacet[36 + q] = 0;
        for (int c = 0; c < 3; ++c) d.tet_abc[q][c] = (uint8_t)T.tet[q][c];
    }
    return d;
}

__constant__ SharedTables g_tables = make_shared_tables();
static_assert(sizeof(SharedTables) % 4 == 0, "copied as words");

// Free-facet counts of the TQ cells, bit-sliced: count = 2*b1 + b0.
struct Counts {
    uint64_t b0, b1;
    __device__ __forceinline__ void dec(uint64_t d)
    {
        b1 ^= d & ~b0;
        b0 ^= d;
    }
};

__device__ __forceinline__ uint32_t nib(uint64_t packed, int i) { return (uint32_t)(packed >> (4 * i)) & 15u; }

// Comparison keys.  The gradient only compares x with its neighbours and
// the neighbours among themselves, in the order of Section 2.1: by value,
// ties by vertex id.  Ranks (the global order) are one encoding of it; the
// values themselves are another (the equivalent form that needs no sort).
//  RankKeys: the LDS halo holds int32 ranks, compared directly.
//  F32Keys / F64Keys: the halo holds order-preserving unsigned keys of the
//    values (-0.0 as +0.0); a comparison value is key << 4 | slot, where the
//    slot orders x and its neighbours by id (neighbours 0..6 precede x, 7..13
//    follow it), so equal values break ties by id.
// Id-order slot of neighbour e relative to x (x itself is slot 7).
__device__ __forceinline__ constexpr int id_slot(int e) { return e < 7 ? e : e + 1; }

template <typename C>
__device__ __forceinline__ C cmin(C a, C b) { return b < a ? b : a; }

// A comparison value above every real one.
template <typename C> __device__ __forceinline__ constexpr C c_highest();
template <> __device__ __forceinline__ constexpr int32_t c_highest<int32_t>() { return 0x7fffffff; }
template <> __device__ __forceinline__ constexpr uint64_t c_highest<uint64_t>() { return ~0ull; }
template <> __device__ __forceinline__ constexpr unsigned __int128 c_highest<unsigned __int128>()
{
    return ~(unsigned __int128)0;
}

struct RankKeys {
    using H = int32_t;
    using C = int32_t;
    static constexpr H kAbsentH = kAbsent;
    __device__ static H load(const void *f, int64_t i, bool &nan)
    {
        nan = false;
        return ((const int32_t *)f)[i];
    }
    __device__ static C cmp(H h, int) { return h; }
};

struct F32Keys {
    using H = uint32_t;
    using C = uint64_t;
    static constexpr H kAbsentH = 0xffffffffu;  // a NaN's key: never a valid input
    __device__ static H load(const void *f, int64_t i, bool &nan) { return key_of(((const float *)f)[i], nan); }
    __device__ static C cmp(H h, int slot) { return h == kAbsentH ? c_highest<C>() : ((C)h << 4) | (C)slot; }
};

struct F64Keys {
    using H = uint64_t;
    using C = unsigned __int128;
    static constexpr H kAbsentH = ~0ull;
    __device__ static H load(const void *f, int64_t i, bool &nan) { return key_of(((const double *)f)[i], nan); }
    __device__ static C cmp(H h, int slot) { return h == kAbsentH ? c_highest<C>() : ((C)h << 4) | (C)slot; }
};

// Lower-neighbour mask of x: bit e set if neighbour e precedes x.
template <typename C>
__device__ __forceinline__ uint32_t lower_mask(const C *o, C ox)
{
    uint32_t low = 0;
#pragma unroll
    for (int e = 0; e < 14; ++e) low |= (o[e] < ox ? 1u : 0u) << e;
    return low;
}

// TQ cells of L(x): those with no vertex outside the lower set.
__device__ __forceinline__ uint64_t lower_star_tq(uint32_t low)
{
    uint64_t out_tq = 0;
#pragma unroll
    for (int e = 0; e < 14; ++e)
        if (!((low >> e) & 1u)) out_tq |= kTables.edge_trimask[e] | ((uint64_t)kTables.edge_tetmask[e] << 36);
    return ~out_tq & ((1ull << 60) - 1);
}

// Ranks of the lower neighbours among themselves, 4 bits per neighbour
// (15 for a neighbour that is not lower).
template <typename C>
__device__ __forceinline__ uint64_t lower_ranks(const C *o, uint32_t low)
{
    C ol[14];
    uint32_t r[14];
#pragma unroll
    for (int e = 0; e < 14; ++e) {
        ol[e] = (low >> e) & 1u ? o[e] : c_highest<C>();
        r[e] = 0;
    }
#pragma unroll
    for (int a = 0; a < 14; ++a)
#pragma unroll
        for (int b = a + 1; b < 14; ++b) {
            const uint32_t c = ol[b] < ol[a] ? 1u : 0u;
            r[a] += c;
            r[b] += 1u - c;
        }
    uint64_t rank_of = 0;
#pragma unroll
    for (int e = 0; e < 14; ++e) rank_of |= (uint64_t)((low >> e) & 1u ? r[e] : 15u) << (4 * e);
    return rank_of;
}

__device__ __forceinline__ uint32_t low_of_ranks(uint64_t rank_of)
{
    uint32_t low = 0;
#pragma unroll
    for (int e = 0; e < 14; ++e) low |= (nib(rank_of, e) != 15u ? 1u : 0u) << e;
    return low;
}

__device__ __forceinline__ bool robins(uint64_t rank_of, const SharedTables &T, uint4 &out);

// The cell of S with the smallest key, as a one-bit set (S if S has at
// most one cell), bit-sliced from the top rank plane down: keep the cells
// without rank b when there are any.  All 14 planes are walked, as
// straight-line code; planes at or above the lower-neighbour count are all
// ones and change nothing.  (Entering the walk at the wave's largest lower
// count instead, through a switch, cost a branch chain and register copies
// in every step; instances for a few plane counts raised register pressure
// into spills; stopping early once no lane has two candidates left cost more
// in checks than it saved in planes.)
__device__ __forceinline__ uint64_t smallest_by_key(uint64_t S, const uint64_t *nkp)
{
#pragma unroll
    for (int b = 13; b >= 0; --b) {
        const uint64_t z = S & nkp[b];
        S = z ? z : S;
    }
    return S;
}

// Robins' ProcessLowerStars for one vertex, from the orders of x and its 14
// neighbours (kAbsent for neighbours outside the grid).
// Returns whether L(x) holds a critical cell.
template <typename C>
__device__ __forceinline__ bool process_vertex(const C *o, C ox, const SharedTables &T, uint4 &out)
{
    const uint32_t low = lower_mask(o, ox);
    if (low == 0) {  // L(x) = {x}: x is critical
        out = make_uint4(0, 0, 0, 0);
        return true;
    }
    return robins(lower_ranks(o, low), T, out);
}

// The pairing itself, from the ranks of the lower neighbours (lower_ranks).
//
// The two priority queues of Robins' formulation are not stored: at any time
// the one-facet queue, minus entries that have meanwhile lost their last
// unpaired facet, is exactly the set of unpaired cells with one unpaired
// facet (every cell enters it at the moment its count drops from two to
// one), and when that set is empty the zero queue's live entries are exactly
// the unpaired edges and the unpaired cells with no unpaired facet.  So each
// step takes the smallest cell of the first set and pairs it with its
// unpaired facet, or, if that set is empty, declares the smallest cell of the
// second set critical.  "Smallest" is a bit-sliced minimum over key planes:
// plane b holds the cells that contain the neighbour of rank b, and the key
// of a cell is the integer with those bits (Section 2.1 comparison).
// Returns whether some cell of L(x) ends critical.
__device__ __forceinline__ bool robins(uint64_t rank_of, const SharedTables &T, uint4 &out)
{
    const uint32_t low = low_of_ranks(rank_of);
    if (low == 0) {
        out = make_uint4(0, 0, 0, 0);
        return true;
    }
    bool crit = false;
    uint64_t nb_at = 0;  // rank -> neighbour (4 bits each)
#pragma unroll
    for (int e = 0; e < 14; ++e)
        if ((low >> e) & 1u) nb_at |= (uint64_t)e << (4 * nib(rank_of, e));
    const int m = __popc(low);
    // complement of the key planes: nkp[b] = TQ cells NOT containing rank b
    uint64_t nkp[14];
#pragma unroll
    for (int b = 0; b < 14; ++b) nkp[b] = b < m ? ~T.cont[nib(nb_at, b)] : ~0ull;

    uint64_t ftq = lower_star_tq(low);  // unpaired TQ cells
    uint32_t fe = low;                  // unpaired edges, by neighbour
    uint32_t fr = (1u << m) - 1u;       // unpaired edges, by rank
    Counts cnt{(1ull << 60) - 1 - kTriBits, (1ull << 60) - 1};  // triangles 2, tets 3
    uint64_t rec_lo = 0, rec_hi = 0;

    // pair x with its smallest edge (the lowest lower neighbour)
    {
        const int d = nib(nb_at, 0);
        fe &= ~(1u << d);
        fr &= ~1u;
        rec_lo |= 1ull << (4 * d);
        cnt.dec(T.cont[d] & kTriBits);
    }
    for (int step = 0; step < 80; ++step) {
        // the cells with one unpaired facet if there are any, else the
        // unpaired cells without one; one bit-sliced minimum serves both
        // cases, so lanes of a wave that are in different cases share it
        const uint64_t one = ftq & cnt.b0 & ~cnt.b1;
        uint64_t S = one ? one : (ftq & ~cnt.b0 & ~cnt.b1);
        if (S == 0 && fr == 0) break;
        S = smallest_by_key(S, nkp);
        const bool have_a = S != 0;
        const int a = have_a ? __ffsll((unsigned long long)S) - 1 : 0;
        if (one) {
            // pair the smallest cell with one unpaired facet with that facet
            const uint64_t fa = T.facet[a];
            uint64_t D;
            if (a < 36) {  // triangle a takes its only unpaired edge e
                const int e = __ffs((uint32_t)fa & fe) - 1;
                fe &= ~(1u << e);
                fr &= ~(1u << nib(rank_of, e));
                const uint32_t ab = T.tri_ab[a], sl = T.tri_slot[a];
                const uint32_t slot = (int)(ab & 15u) == e ? (sl & 15u) : (sl >> 4);
                rec_lo |= (uint64_t)(3u + slot) << (4 * e);
                D = (T.cont[e] & kTriBits) | T.cofacet[a];
            } else {  // tet a takes its only unpaired triangle t
                const int t = __ffsll((unsigned long long)(fa & ftq)) - 1;
                ftq &= ~(1ull << t);
                D = T.cofacet[t];
                const uint64_t v = T.tri_tet0[t] == a - 36 ? 1u : 2u;
                const int bit = 56 + 2 * t;
                if (bit < 64) rec_lo |= v << bit; else rec_hi |= v << (bit - 64);
            }
            ftq &= ~(1ull << a);
            cnt.dec(D);
            continue;
        }
        // no cell has exactly one unpaired facet: the smallest unpaired edge or
        // cell without unpaired facets is critical
        crit = true;
        bool edge_wins = fr != 0 && !have_a;
        const int re = fr ? __ffs(fr) - 1 : 31;
        if (fr != 0 && have_a) {
            // the edge of rank re is smaller iff re <= the top rank of cell a
            int top;
            if (a < 36) {
                const uint32_t ab = T.tri_ab[a];
                top = max(nib(rank_of, ab & 15u), nib(rank_of, ab >> 4));
            } else {
                const int q = a - 36;
                top = max(max(nib(rank_of, T.tet_abc[q][0]), nib(rank_of, T.tet_abc[q][1])),
                          nib(rank_of, T.tet_abc[q][2]));
            }
            edge_wins = re <= top;
        }
        if (edge_wins) {
            const int e = nib(nb_at, re);
            fe &= ~(1u << e);
            fr &= ~(1u << re);
            rec_lo |= 2ull << (4 * e);
            cnt.dec(T.cont[e] & kTriBits);
        } else {
            ftq &= ~(1ull << a);
            cnt.dec(T.cofacet[a]);
        }
    }
    out = make_uint4((uint32_t)rec_lo, (uint32_t)(rec_lo >> 32), (uint32_t)rec_hi,
                     (uint32_t)(rec_hi >> 32));
    return crit;
}

// ---------------------------------------------------------------------------
// Antipodal-regular vertices.  Neighbour e and neighbour 13 - e are opposite
// offsets.  When exactly one of each of the 7 opposite pairs precedes x (the
// common case of a smooth field: the lower link is a hemisphere), L(x) is
// fixed by which member of each pair is lower (7 bits) and by the order of
// those 7 neighbours (a permutation of 7).  Robins' result for all 128 x 5040
// such configurations is computed once per device by process_vertex itself
// and kept in a device table; such vertices then cost a table lookup.
constexpr int kPerm7 = 5040;
constexpr int kRegular = 128 * kPerm7;
__device__ uint4 g_regular[kRegular];

// One-defect vertices: six pairs have one lower member and the seventh has
// both (8 lower neighbours) or neither (6).  All three families are looked
// up from one set of eight slots: v[i] = the member of pair i on the lower
// side (neighbour 13 - i when side bit i is set, else i) for i < 7, and
// v[7] = the smallest order among the other members -- neighbour j itself
// when pair j is wholly lower, else an upper order (replaced by a value
// above every order).  The Lehmer digits l_i count the later slots holding
// smaller orders; the codes are fixed-radix factorial sums of them:
//   code7 = sum over i < 7 of l_i (6 - i)!   (regular and |L| = 6)
//   code8 = sum over i < 8 of l_i (7 - i)!   (|L| = 8)
// For |L| = 6 slot j holds an upper order, larger than every lower one, so
// its digit is always 6 - j: the code is injective but sparse (one code in
// seven is used), which keeps the lookup free of any per-lane dependence on
// j beyond the table offset.
//   regular: index side * 7! + code7                       (10 MB)
//   |L| = 6: index (j * 64 + side6) * 7! + code7            (36 MB, sparse)
//   |L| = 8: index (j * 64 + side6) * 8! + code8            (289 MB, allocated
//            once per device)
// side6 is the 7-bit side pattern with bit j removed.
constexpr int kPerm8 = 40320;
constexpr int kDefect6 = 7 * 64 * kPerm7;
constexpr int64_t kDefect8 = 7ll * 64 * kPerm8;
__device__ uint4 g_defect6[kDefect6];
// One bit per table entry: whether the entry's lower star holds a critical
// cell (set by the table fillers, read to mark records for the extraction).
static_assert(kRegular % 64 == 0 && kDefect6 % 64 == 0 && kDefect8 % 64 == 0, "flag words per wave");
__device__ uint32_t g_regular_flags[kRegular / 32];
__device__ uint32_t g_defect6_flags[kDefect6 / 32];
__device__ uint32_t g_defect8_flags[kDefect8 / 32];

// A table lookup: the entry's record (null when x is in no tabulated
// family), the family's flag bits and the entry index.
struct TabHit {
    const uint4 *rec;
    const uint32_t *flags;
    uint32_t idx;
};

// Table entry of x, or a null record when x is in none of the families
// (defect8 may be null: that family then takes the general path).
template <typename C>
__device__ __forceinline__ TabHit table_entry(uint32_t low, const C *o, const uint4 *__restrict__ defect8)
{
    const C kHigh = c_highest<C>();
    const uint32_t rev = __brev(low) >> 18;  // bit e -> bit 13 - e
    const uint32_t one = (low ^ rev) & 0x7fu;
    const int npair = __popc(one);
    if (npair < 6) return TabHit{nullptr, nullptr, 0};
    const uint32_t side = __brev((low >> 7) & 0x7fu) >> 25;  // bit i: the lower member is 13 - i
    const uint32_t both = low & rev & 0x7fu;                   // pairs wholly lower
    // slot values without selecting between array elements by a per-lane
    // index (which the compiler expands into chains of compares): the lower
    // member of a single pair is the smaller order of the two; a wholly lower
    // pair (side bit set) takes neighbour 13 - i, and neighbour i goes to
    // slot 7
    C v[8];
    C v7 = kHigh;
#pragma unroll
    for (int i = 0; i < 7; ++i) {
        const C a = o[i], b = o[13 - i];
        const bool w = (both >> i) & 1u;
        v[i] = w ? b : cmin(a, b);
        v7 = cmin(v7, w ? a : kHigh);
    }
    const bool eight = both != 0;
    if (eight && !defect8) return TabHit{nullptr, nullptr, 0};
    v[7] = v7;
    uint32_t l[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        l[i] = 0;
#pragma unroll
        for (int k = i + 1; k < 8; ++k) l[i] += v[k] < v[i] ? 1u : 0u;
    }
    constexpr uint32_t f7[7] = {720, 120, 24, 6, 2, 1, 1};
    constexpr uint32_t f8[8] = {5040, 720, 120, 24, 6, 2, 1, 1};
    uint32_t code7 = 0, code8 = 0;
#pragma unroll
    for (int i = 0; i < 7; ++i) code7 += l[i] * f7[i];
#pragma unroll
    for (int i = 0; i < 8; ++i) code8 += l[i] * f8[i];
    if (npair == 7) {
        const uint32_t i = side * kPerm7 + code7;
        return TabHit{&g_regular[i], g_regular_flags, i};
    }
    const uint32_t j = (uint32_t)__ffs(~one & 0x7fu) - 1u;
    const uint32_t side6 = (side & ((1u << j) - 1u)) | ((side >> (j + 1u)) << j);
    static_assert(kDefect8 < (1ll << 32), "32-bit index into the wholly-lower table");
    if (eight) {
        const uint32_t i = (j * 64u + side6) * (uint32_t)kPerm8 + code8;
        return TabHit{defect8 + i, g_defect8_flags, i};
    }
    const uint32_t i = (j * 64u + side6) * kPerm7 + code7;
    return TabHit{&g_defect6[i], g_defect6_flags, i};
}

template <int GX, int GY>
struct Tile {
    static_assert(GX * GY == kTileVerts, "tile holds kTileVerts vertices");
    static constexpr int HX = GX + 2, HY = GY + 2, HZ = 3;
    static constexpr int kHalo = HX * HY * HZ;
};

// Comparison values of x's 14 neighbours (in neighbour order) and of x.
template <typename Keys, int GX, int GY>
__device__ __forceinline__ void gather_orders(const typename Keys::H *tile, int c, typename Keys::C *o,
                                              typename Keys::C &ox)
{
    using S = Tile<GX, GY>;
#pragma unroll
    for (int e = 0; e < 14; ++e)
        o[e] = Keys::cmp(tile[c + kTables.nb[e][0] + S::HX * (kTables.nb[e][1] + S::HY * kTables.nb[e][2])],
                         id_slot(e));
    ox = Keys::cmp(tile[c], 7);
}

// Vertices that no table covers ("general" vertices) need Robins' loop,
// whose length varies with the lower star.  A tile with many of them pairs
// them itself, dealt to threads by increasing size (pass 2).  A tile with
// few -- the common case of a smooth field -- would leave one sparse wave
// running a long loop while the block holds its slot, so it ranks them and
// appends compact entries to a device queue instead; a second kernel pairs
// the queue in full waves sorted by size.
//   entry: x, y = ranks of the lower neighbours (lower_ranks, 56 bits), the
//          record index (40 bits: z, and the top byte of y), w = size key.
constexpr int kQueueChunk = 1024;  // entries per block of the queue kernel

// The ranks take 56 bits (14 nibbles); the record index takes 40 bits, its
// top 8 in the free byte above the ranks.
__device__ __forceinline__ uint4 queue_entry(uint64_t rk, int64_t ridx, uint32_t key)
{
    const uint64_t r = (uint64_t)ridx;
    return make_uint4((uint32_t)rk, ((uint32_t)(rk >> 32) & 0x00ffffffu) | ((uint32_t)(r >> 32) << 24),
                      (uint32_t)r, key);
}
__device__ __forceinline__ uint64_t entry_ranks(const uint4 &e)
{
    return (uint64_t)e.x | (uint64_t)(e.y & 0x00ffffffu) << 32;
}
__device__ __forceinline__ int64_t entry_record(const uint4 &e)
{
    return (int64_t)((uint64_t)e.z | (uint64_t)(e.y >> 24) << 32);
}

struct BlockShared {
    SharedTables T;
    uint32_t bins[kSizeBins];
    uint32_t qbase;
    uint32_t nlist;
    uint16_t list[kTileVerts];  // general vertices of the tile (tile positions)
    uint16_t perm[kTileVerts];  // the same, sorted by size key (dense tiles)
};

__device__ __forceinline__ void load_tables(SharedTables &T)
{
    const uint32_t *src = (const uint32_t *)&g_tables;
    uint32_t *dst = (uint32_t *)&T;
    for (int i = threadIdx.x; i < (int)(sizeof(SharedTables) / 4); i += kThreads) dst[i] = src[i];
}

// Exclusive scan of sh.bins (kSizeBins <= 2 * kWave) by the first wave.
__device__ __forceinline__ void scan_bins(uint32_t *bins)
{
    const int tid = threadIdx.x;
    if (tid < kWave) {
        const uint32_t v0 = tid < kSizeBins ? bins[tid] : 0u;
        const uint32_t v1 = tid + kWave < kSizeBins ? bins[tid + kWave] : 0u;
        uint32_t i0 = v0, i1 = v1;
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const uint32_t t0 = __shfl_up(i0, off), t1 = __shfl_up(i1, off);
            if (tid >= off) { i0 += t0; i1 += t1; }
        }
        const uint32_t tot0 = __shfl(i0, kWave - 1);
        if (tid < kSizeBins) bins[tid] = i0 - v0;
        if (tid + kWave < kSizeBins) bins[tid + kWave] = tot0 + i1 - v1;
    }
}

// Size key of a general vertex: 1 + lower neighbours + lower-star triangles
// and tets (at most 75).
__device__ __forceinline__ uint32_t size_key(uint32_t low)
{
    return 1u + (uint32_t)__popc(low) + (uint32_t)__popcll(lower_star_tq(low));
}

// Marks record r (box index) as holding a critical cell: bit r of the mask.
__device__ __forceinline__ void mark_critical(uint32_t *mark, int64_t r)
{
    atomicOr(&mark[r >> 5], 1u << (uint32_t)(r & 31));
}

// One GX x GY x 1 tile (1024 vertices) of the owned box [lo, lo + w) of a
// grid of dims n; record indices are rec_off + position in the owned box.
// The orders of the tile plus a one-vertex halo are staged in LDS.  Pass 1
// visits the tile in order (4 vertices per thread): a regular or one-defect
// vertex takes its record from the precomputed tables; any other vertex is
// listed.  A tile with fewer than kThreads listed vertices ranks them and
// queues as many as fit (pairing any others itself); a denser tile sorts
// them by size and pairs them itself.  Must be entered by the whole block.
template <typename Keys, int GX, int GY>
__device__ __forceinline__ void gradient_tile(const void *__restrict__ field, int64_t nx,
                                              int64_t ny, int64_t nz, int64_t lo0, int64_t lo1,
                                              int64_t lo2, int64_t w0, int64_t w1, int64_t w2,
                                              int64_t bx, int64_t by, int64_t bz, int64_t rec_off,
                                              uint4 *__restrict__ rec, const uint4 *__restrict__ defect8,
                                              uint4 *__restrict__ queue, uint32_t *qcount, uint32_t qcap,
                                              uint32_t *flags, uint32_t *__restrict__ mark, BlockShared &sh,
                                              typename Keys::H *tile)
{
    using S = Tile<GX, GY>;
    using C = typename Keys::C;
    const int tid = threadIdx.x;
    if (tid == 0) sh.nlist = 0;
    const int64_t x0 = lo0 + bx * GX - 1, y0 = lo1 + by * GY - 1, z0 = lo2 + bz - 1;
    const bool full = x0 >= 0 && y0 >= 0 && z0 >= 0 && x0 + S::HX <= nx && y0 + S::HY <= ny &&
                      z0 + S::HZ <= nz;
    bool nan = false, nan_any = false;
    bool staged = false;  // uniform
    if constexpr (GX == kWave) {
      if (full) {
        // inside the grid, rows of 66 orders: wave w loads rows w, w + 4, ...
        // (64 consecutive orders from a row base computed in scalar
        // registers, so the loads need no per-lane address arithmetic), and
        // the first 2 x 54 threads load the rows' last two orders; every
        // load is issued before any LDS store
        constexpr int kRows = S::HY * S::HZ;
        constexpr int kWavesB = kThreads / kWave;
        constexpr int kPerRow = (kRows + kWavesB - 1) / kWavesB;
        static_assert(S::HX == kWave + 2 && 2 * kRows <= kThreads, "row split");
        const int wave = __builtin_amdgcn_readfirstlane(tid / kWave), lane = tid % kWave;
        const int64_t base0 = x0 + nx * (y0 + ny * z0), pstride = nx * ny;
        typename Keys::H hv[kPerRow];
#pragma unroll
        for (int k = 0; k < kPerRow; ++k) {
            const int r = min(wave + kWavesB * k, kRows - 1);
            const int hz = r / S::HY, hy = r - hz * S::HY;
            hv[k] = Keys::load(field, base0 + hz * pstride + hy * nx + lane, nan);
            nan_any |= nan;
        }
        const int er = tid < 2 * kRows ? tid >> 1 : 0;
        const int ez = er / S::HY, ey = er - ez * S::HY;
        const typename Keys::H ev = Keys::load(field, base0 + ez * pstride + ey * nx + kWave + (tid & 1), nan);
        nan_any |= nan;
#pragma unroll
        for (int k = 0; k < kPerRow; ++k) {
            const int r = wave + kWavesB * k;
            if (r < kRows) tile[r * S::HX + lane] = hv[k];
        }
        if (tid < 2 * kRows) tile[er * S::HX + kWave + (tid & 1)] = ev;
        staged = true;
      }
    }
    if (staged) {
    } else if (full && nx * S::HY < (1ll << 31)) {
        // inside the grid: each thread issues a fixed number of loads (its
        // last one clamped into the halo) before any LDS store, so that all
        // are in flight at once; a 64-bit base per halo plane and a 32-bit
        // offset within the plane
        static_assert(S::HZ == 3, "three halo planes");
        constexpr int kPlane = S::HX * S::HY;
        constexpr int kPer = (S::kHalo + kThreads - 1) / kThreads;
        const int nxi = (int)nx;
        const int64_t base0 = x0 + nx * (y0 + ny * z0), pstride = nx * ny;
        typename Keys::H hv[kPer];
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const int i = min(tid + j * kThreads, S::kHalo - 1);
            const int hz = i / kPlane, r = i - hz * kPlane;
            const int hy = r / S::HX, hx = r - hy * S::HX;
            const int64_t pb = hz == 0 ? base0 : (hz == 1 ? base0 + pstride : base0 + 2 * pstride);
            hv[j] = Keys::load(field, pb + hx + hy * nxi, nan);
            nan_any |= nan;
        }
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const int i = tid + j * kThreads;
            if (i < S::kHalo) tile[i] = hv[j];
        }
    } else {
        for (int i = tid; i < S::kHalo; i += kThreads) {
            const int hx = i % S::HX, hy = (i / S::HX) % S::HY, hz = i / (S::HX * S::HY);
            const int64_t x = x0 + hx, y = y0 + hy, z = z0 + hz;
            typename Keys::H v = Keys::kAbsentH;
            if (x >= 0 && y >= 0 && z >= 0 && x < nx && y < ny && z < nz) {
                v = Keys::load(field, x + nx * (y + ny * z), nan);
                nan_any |= nan;
            }
            tile[i] = v;
        }
    }
    if (flags && __ballot(nan_any) && lane_id() == 0) atomicOr(flags, (uint32_t)DMS_FLAG_NAN);
    __syncthreads();

    // pass 1: table vertices; the others are listed
    const int64_t rbase = rec_off + (bx * GX) + w0 * ((by * GY) + w1 * bz);
    // a 64-wide tile: vertex k of a thread lies in column lane and row
    // wave + 4 k, the same row for the whole wave, so the row's part of the
    // LDS and record addresses stays in scalar registers
    const int wave_u = __builtin_amdgcn_readfirstlane(tid / kWave);
    // all of a thread's table reads are issued (a vertex with no entry reads
    // a dummy one) before any record is stored, so that their latencies
    // overlap instead of adding up
    constexpr int kPer = kTileVerts / kThreads;
    uint32_t gx[kPer], gy[kPer], gz[kPer], gw[kPer];  // the entries, as plain words
    uint32_t fw[kPer];   // the flag words of the entries
    uint32_t fbit = 0;   // 5 bits per vertex: the entry's bit in its flag word
    uint32_t state = 0;  // bit k: vertex k in the box; bit kPer + k: it has an entry
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int v = tid + k * kThreads;
        const int tx = GX == kWave ? tid % kWave : v % GX;
        const int ty = GX == kWave ? wave_u + (kThreads / kWave) * k : v / GX;
        TabHit hit{nullptr, g_regular_flags, 0};
        if (bx * GX + tx < w0 && by * GY + ty < w1 && bz < w2) {
            const int c = (tx + 1) + S::HX * ((ty + 1) + S::HY);
            C o[14], ox;
            gather_orders<Keys, GX, GY>(tile, c, o, ox);
            hit = table_entry(lower_mask(o, ox), o, defect8);
            state |= 1u << k;
        }
        if (hit.rec) state |= 1u << (kPer + k);
        const uint4 e = *(hit.rec ? hit.rec : g_regular);
        gx[k] = e.x;
        gy[k] = e.y;
        gz[k] = e.z;
        gw[k] = e.w;
        fw[k] = hit.rec ? hit.flags[hit.idx >> 5] : 0u;
        fbit |= (hit.idx & 31u) << (5 * k);
    }
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        if (!((state >> k) & 1u)) continue;
        const int v = tid + k * kThreads;
        const int tx = GX == kWave ? tid % kWave : v % GX;
        const int ty = GX == kWave ? wave_u + (kThreads / kWave) * k : v / GX;
        if ((state >> (kPer + k)) & 1u) {
            const int64_t r = rbase + tx + w0 * ty;
            rec[r] = make_uint4(gx[k], gy[k], gz[k], gw[k]);
            if (mark && ((fw[k] >> ((fbit >> (5 * k)) & 31u)) & 1u)) mark_critical(mark, r);
        } else {
            sh.list[atomicAdd(&sh.nlist, 1u)] = (uint16_t)v;
        }
    }
    __syncthreads();
    const uint32_t total = sh.nlist;
    if (total == 0) return;

    if (queue && total < (uint32_t)kThreads) {
        // reserve queue slots; the ranking below overlaps the atomic
        if (tid == 0) sh.qbase = atomicAdd(qcount, total);
        const bool mine = (uint32_t)tid < total;
        const int v = mine ? sh.list[tid] : 0;
        const int tx = v % GX, ty = v / GX;
        const int c = (tx + 1) + S::HX * ((ty + 1) + S::HY);
        C o[14], ox;
        gather_orders<Keys, GX, GY>(tile, c, o, ox);
        const uint32_t low = mine ? lower_mask(o, ox) : 0u;
        const uint64_t rk = mine ? lower_ranks(o, low) : 0xffffffffffffffull;
        __syncthreads();
        // queue as many as fit below qcap, so that every slot the queue
        // kernel reads, [0, min(count, qcap)), has been written by this launch
        const uint32_t qb = sh.qbase;
        const uint32_t nq = qb >= qcap ? 0u : min(total, qcap - qb);  // uniform
        const int64_t ridx = rbase + tx + w0 * ty;
        if ((uint32_t)tid < nq)
            queue[qb + tid] = queue_entry(rk, ridx, size_key(low));
        if (nq == total) return;
        // the queue is full: pair the rest here (rare, so unsorted)
        const bool here = (uint32_t)tid >= nq && mine;
        if (here) {
            uint4 r;
            const bool crit = robins(rk, sh.T, r);
            rec[ridx] = r;
            if (mark && crit) mark_critical(mark, ridx);
        }
        return;
    }

    // a dense tile: deal its general vertices into perm by size key (the key
    // is computed twice rather than stored: LDS is kept for occupancy)
    for (int i = tid; i < kSizeBins; i += kThreads) sh.bins[i] = 0;
    __syncthreads();
    for (uint32_t i = tid; i < total; i += kThreads) {
        const int v = sh.list[i];
        const int c = (v % GX + 1) + S::HX * ((v / GX + 1) + S::HY);
        C o[14], ox;
        gather_orders<Keys, GX, GY>(tile, c, o, ox);
        atomicAdd(&sh.bins[size_key(lower_mask(o, ox))], 1u);
    }
    __syncthreads();
    scan_bins(sh.bins);
    __syncthreads();
    for (uint32_t i = tid; i < total; i += kThreads) {
        const int v = sh.list[i];
        const int c = (v % GX + 1) + S::HX * ((v / GX + 1) + S::HY);
        C o[14], ox;
        gather_orders<Keys, GX, GY>(tile, c, o, ox);
        sh.perm[atomicAdd(&sh.bins[size_key(lower_mask(o, ox))], 1u)] = (uint16_t)v;
    }
    __syncthreads();

    // pass 2: general vertices by increasing lower-star size
    for (uint32_t base = 0; base < total; base += kThreads) {
        const uint32_t i = base + tid;
        const bool active = i < total;
        const int v = active ? sh.perm[i] : 0;
        const int tx = v % GX, ty = v / GX;
        const int c = (tx + 1) + S::HX * ((ty + 1) + S::HY);
        C o[14], ox;
        gather_orders<Keys, GX, GY>(tile, c, o, ox);
        if (active) {
            uint4 r;
            const bool crit = process_vertex(o, ox, sh.T, r);
            const int64_t ri = rbase + tx + w0 * ty;
            rec[ri] = r;
            if (mark && crit) mark_critical(mark, ri);
        }
    }
}

// Keys: RankKeys reads the int32 order; F32Keys / F64Keys read the values
// (flags receives DMS_FLAG_NAN for a NaN among them).
template <typename Keys, int GX, int GY>
__global__ __launch_bounds__(kThreads, 8) void k_gradient(const void *__restrict__ field,
                                                       int64_t nx, int64_t ny, int64_t nz,
                                                       int64_t lo0, int64_t lo1, int64_t lo2,
                                                       int64_t w0, int64_t w1, int64_t w2,
                                                       int64_t bx_count, int64_t by_count,
                                                       uint4 *__restrict__ rec,
                                                       const uint4 *__restrict__ defect8,
                                                       uint4 *__restrict__ queue, uint32_t *qcount,
                                                       uint32_t qcap, uint32_t *flags,
                                                       uint32_t *__restrict__ mark)
{
    __shared__ BlockShared sh;
    __shared__ typename Keys::H tile[Tile<GX, GY>::kHalo];
    load_tables(sh.T);
    // tiles in column order, z fastest: the tiles running at the same time
    // then include each tile's neighbours above and below, which read two of
    // its three halo planes, so most halo reads hit a cache (row order, with
    // z slowest, put those neighbours a whole plane of tiles apart)
    const int64_t t = blockIdx.x;
    const int64_t bz = t % w2, col = t / w2, bx = col % bx_count, by = col / bx_count;
    gradient_tile<Keys, GX, GY>(field, nx, ny, nz, lo0, lo1, lo2, w0, w1, w2, bx, by, bz, 0, rec, defect8,
                                queue, qcount, qcap, flags, mark, sh, tile);
}

// Batched form: many whole fields, concatenated; one block per tile of the
// (field, tile) list, field f owning tiles [tile_start[f], tile_start[f+1]).
// tile_field[t] names the field of tile t, so a block finds its field with
// one read, and the kernel keeps the single-field kernel's registers and LDS
// (a persistent grid walking the tiles held the walk's 64-bit state in
// scalar registers and spilled).
template <int GX, int GY>
__global__ __launch_bounds__(kThreads, 8) void k_gradient_batch(const int32_t *__restrict__ order,
                                                                const BatchField *__restrict__ fields,
                                                                const int64_t *__restrict__ tile_start,
                                                                const uint16_t *__restrict__ tile_field,
                                                                uint4 *__restrict__ rec,
                                                                const uint4 *__restrict__ defect8,
                                                                uint4 *__restrict__ queue,
                                                                uint32_t *qcount, uint32_t qcap,
                                                                uint32_t *__restrict__ mark)
{
    __shared__ BlockShared sh;
    __shared__ int32_t tile[Tile<GX, GY>::kHalo];
    load_tables(sh.T);
    const int64_t t = blockIdx.x;
    const int f = tile_field[t];
    const BatchField F = fields[f];
    const int64_t bxc = (F.n[0] + GX - 1) / GX, byc = (F.n[1] + GY - 1) / GY;
    // column order inside the field, as in k_gradient
    const int64_t k = t - tile_start[f];
    const int64_t bz = k % F.n[2], col = k / F.n[2], bx = col % bxc, by = col / bxc;
    gradient_tile<RankKeys, GX, GY>(order + F.off, F.n[0], F.n[1], F.n[2], 0, 0, 0, F.n[0], F.n[1], F.n[2], bx,
                                    by, bz, F.off, rec, defect8, queue, qcount, qcap, nullptr, mark, sh,
                                    tile);
}

__global__ void k_queue_reset(uint32_t *qcount) { *qcount = 0; }

__global__ void k_mark_zero(uint32_t *__restrict__ mark, int64_t words)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < words) mark[i] = 0u;
}

// Pairs the queued general vertices: block b takes entries
// [b kQueueChunk, (b+1) kQueueChunk) of the filled part, sorts them by size
// key and runs Robins' loop on them in full rounds.
__global__ __launch_bounds__(kThreads) void k_gradient_queue(const uint4 *__restrict__ queue,
                                                             const uint32_t *qcount, uint32_t qcap,
                                                             uint4 *__restrict__ rec,
                                                             uint32_t *__restrict__ mark)
{
    __shared__ SharedTables T;
    __shared__ uint32_t bins[kSizeBins];
    __shared__ uint16_t perm[kQueueChunk];
    const int tid = threadIdx.x;
    const uint32_t filled = min(*qcount, qcap);
    const uint64_t start = (uint64_t)blockIdx.x * kQueueChunk;
    if (start >= filled) return;  // uniform
    const uint32_t cnt = (uint32_t)min<uint64_t>(kQueueChunk, filled - start);
    load_tables(T);
    for (int i = tid; i < kSizeBins; i += kThreads) bins[i] = 0;
    __syncthreads();
    for (uint32_t i = tid; i < cnt; i += kThreads) atomicAdd(&bins[min(queue[start + i].w, (uint32_t)kSizeBins - 1u)], 1u);
    __syncthreads();
    scan_bins(bins);
    __syncthreads();
    for (uint32_t i = tid; i < cnt; i += kThreads)
        perm[atomicAdd(&bins[min(queue[start + i].w, (uint32_t)kSizeBins - 1u)], 1u)] = (uint16_t)i;
    __syncthreads();
    for (uint32_t base = 0; base < cnt; base += kThreads) {
        const uint32_t i = base + tid;
        const bool active = i < cnt;
        uint4 e = make_uint4(0xffffffffu, 0x00ffffffu, 0u, 0u);  // no lower neighbour
        if (active) e = queue[start + perm[i]];
        const uint64_t rk = entry_ranks(e);
        if (active) {
            uint4 r;
            const bool crit = robins(rk, T, r);
            const int64_t ri = entry_record(e);
            rec[ri] = r;
            if (mark && crit) mark_critical(mark, ri);
        }
    }
}

// Decodes a Lehmer code (factorial base, first item most significant) of
// N items into their ranks.
template <int N>
__device__ void lehmer_decode(uint32_t code, uint32_t *rank)
{
    uint32_t w = 1;
    for (int i = 2; i < N; ++i) w *= (uint32_t)i;  // (N - 1)!
    uint32_t used = 0;
    for (int i = 0; i < N; ++i) {
        uint32_t l = code / w;
        code %= w;
        if (i < N - 1) w /= (uint32_t)(N - 1 - i);
        int r = 0;  // the l-th smallest unused rank
        for (;; ++r)
            if (!((used >> r) & 1u)) {
                if (l == 0) break;
                --l;
            }
        used |= 1u << r;
        rank[i] = (uint32_t)r;
    }
}

// Fills the regular-vertex table: entry side * 5040 + code holds the record of
// the configuration whose lower neighbours are, for pair i, neighbour i or
// 13 - i (bit i of side), ordered by the permutation with Lehmer code `code`.
__global__ __launch_bounds__(kThreads) void k_regular_table()
{
    __shared__ SharedTables T;
    load_tables(T);
    __syncthreads();
    const int idx = blockIdx.x * kThreads + threadIdx.x;  // a wave covers 64 aligned entries
    bool crit = false;
    if (idx < kRegular) {
        const uint32_t side = idx / kPerm7;
        uint32_t rank[7];
        lehmer_decode<7>(idx % kPerm7, rank);
        int32_t o[14];
        for (int i = 0; i < 7; ++i) {
            const int lowm = ((side >> i) & 1u) ? 13 - i : i;
            o[lowm] = (int32_t)rank[i];
            o[13 - lowm] = 100 + i;  // above x
        }
        uint4 r;
        crit = process_vertex(o, 50, T, r);
        g_regular[idx] = r;
    }
    const uint64_t m = __ballot(crit);
    if (lane_id() == 0 && idx < kRegular) {
        g_regular_flags[idx / 32] = (uint32_t)m;
        g_regular_flags[idx / 32 + 1] = (uint32_t)(m >> 32);
    }
}

// Fills a one-defect table in the layout table_entry reads: for |L| = 8 the
// code is that of 8 slots (slot 7 = neighbour j); for |L| = 6 that of 7
// slots where slot j (pair j, wholly upper) ranks above the other six --
// entries whose code puts it elsewhere are never read and stay zero.
template <bool kEight>
__global__ __launch_bounds__(kThreads) void k_defect_table(uint4 *table)
{
    __shared__ SharedTables T;
    load_tables(T);
    __syncthreads();
    constexpr int N = kEight ? 8 : 7;
    constexpr int64_t perms = kEight ? kPerm8 : kPerm7;
    constexpr int64_t total = 7 * 64 * perms;
    uint32_t *flags = kEight ? g_defect8_flags : g_defect6_flags;
    const int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x;  // a wave covers 64 aligned entries
    bool crit = false;
    if (idx < total) {
        const uint32_t code = (uint32_t)(idx % perms);
        const uint32_t js = (uint32_t)(idx / perms);
        const uint32_t j = js / 64, side6 = js % 64;
        // the 7-bit side pattern with bit j (pair j) set for both lower
        const uint32_t side = (side6 & ((1u << j) - 1u)) | ((side6 >> j) << (j + 1u)) |
                              (kEight ? 1u << j : 0u);
        uint32_t rank[N];
        lehmer_decode<N>(code, rank);
        uint4 r = make_uint4(0, 0, 0, 0);
        if (kEight || rank[j] == 6u) {  // other |L| = 6 codes are never read
            int32_t o[14];
            for (int e = 0; e < 14; ++e) o[e] = 100 + e;  // above x unless set below
            for (int i = 0; i < 7; ++i) {
                if (!kEight && (uint32_t)i == j) continue;
                o[((side >> i) & 1u) ? 13 - i : i] = (int32_t)rank[i];
            }
            if (kEight) o[j] = (int32_t)rank[7];
            crit = process_vertex(o, 50, T, r);
        }
        table[idx] = r;
    }
    const uint64_t m = __ballot(crit);
    if (lane_id() == 0 && idx < total) {
        flags[idx / 32] = (uint32_t)m;
        flags[idx / 32 + 1] = (uint32_t)(m >> 32);
    }
}

}  // namespace
}  // namespace dms

namespace dms {

namespace {
std::atomic<uint64_t> g_regular_ready{0};  // one bit per device that holds the tables
std::mutex g_table_mutex;
uint4 *g_defect8_ptr[64];  // per device, held until the process ends
}

int init_tables(hipStream_t s)
{
    if (const int dc = device_check()) return dc;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return DMS_E_HIP;
    const uint64_t bit = 1ull << dev;
    if (g_regular_ready.load() & bit) return DMS_OK;
    std::lock_guard<std::mutex> lock(g_table_mutex);
    if (g_regular_ready.load() & bit) return DMS_OK;
    if (!g_defect8_ptr[dev]) {
        void *p = nullptr;
        if (hipMalloc(&p, (size_t)kDefect8 * sizeof(uint4)) != hipSuccess) return DMS_E_HIP;
        g_defect8_ptr[dev] = (uint4 *)p;
    }
    uint4 *d6 = nullptr;
    if (hipGetSymbolAddress((void **)&d6, HIP_SYMBOL(g_defect6)) != hipSuccess) return DMS_E_HIP;
    hipLaunchKernelGGL(k_regular_table, dim3((kRegular + kThreads - 1) / kThreads), dim3(kThreads), 0, s);
    hipLaunchKernelGGL(k_defect_table<false>, dim3((kDefect6 + kThreads - 1) / kThreads), dim3(kThreads),
                       0, s, d6);
    hipLaunchKernelGGL(k_defect_table<true>, dim3((unsigned)((kDefect8 + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, s, g_defect8_ptr[dev]);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) return DMS_E_HIP;
    g_regular_ready.fetch_or(bit);
    return DMS_OK;
}

// The current device's |L| = 8 table (null before init_tables).
static const uint4 *defect8_table()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    return (g_regular_ready.load() >> dev) & 1u ? g_defect8_ptr[dev] : nullptr;
}

// DMS_OK when the current device is a gfx950 whose tables init_tables has
// filled; DMS_E_UNSUPPORTED or DMS_E_NOT_INITIALISED otherwise.
int tables_ready()
{
    if (const int dc = device_check()) return dc;
    return defect8_table() ? DMS_OK : DMS_E_NOT_INITIALISED;
}


// Queue of general vertices: a counter, then qcap 16-byte entries; room for
// one vertex in 16 plus a chunk.
static uint32_t queue_cap(int64_t owned)
{
    const int64_t c = owned / 16 + kQueueChunk;
    return (uint32_t)(c < 0x7fffffffLL ? c : 0x7fffffffLL);
}

size_t gradient_workspace_size(int64_t owned) { return 256 + (size_t)queue_cap(owned) * sizeof(uint4); }

// Resets the queue counter; returns (queue, counter, capacity) carved from ws
// (all null / 0 when ws is null: every tile then pairs its own vertices).
static void queue_begin(char *ws, int64_t owned, hipStream_t s, uint4 **queue, uint32_t **qcount,
                        uint32_t *qcap)
{
    *queue = nullptr;
    *qcount = nullptr;
    *qcap = 0;
    if (!ws) return;
    *qcount = (uint32_t *)ws;
    *queue = (uint4 *)(ws + 256);
    *qcap = queue_cap(owned);
    hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(1), 0, s, *qcount);
}

static void queue_finish(const uint4 *queue, const uint32_t *qcount, uint32_t qcap, uint32_t *rec,
                         uint32_t *mark, hipStream_t s)
{
    if (!queue) return;
    const unsigned blocks = (unsigned)((qcap + kQueueChunk - 1) / kQueueChunk);
    hipLaunchKernelGGL(k_gradient_queue, dim3(blocks), dim3(kThreads), 0, s, queue, qcount, qcap,
                       (uint4 *)rec, mark);
}

template <typename Keys>
static int launch_gradient_keys(int variant, const void *field, const int64_t *dims, const int64_t *lo,
                                const int64_t *hi, uint32_t *rec, uint32_t *mark, char *ws, uint32_t *flags,
                                hipStream_t s)
{
    const int64_t w0 = hi[0] - lo[0], w1 = hi[1] - lo[1], w2 = hi[2] - lo[2];
    if (w0 == 0 || w1 == 0 || w2 == 0) return DMS_OK;
    if (mark) {
        const int64_t words = (w0 * w1 * w2 + 31) / 32;
        hipLaunchKernelGGL(k_mark_zero, dim3((unsigned)((words + kThreads - 1) / kThreads)), dim3(kThreads), 0, s,
                           mark, words);
    }
    const int gx = kTileX[variant], gy = kTileVerts / gx;
    const int64_t bxc = (w0 + gx - 1) / gx, byc = (w1 + gy - 1) / gy;
    const int64_t blocks = bxc * byc * w2;
    if (blocks > 2147483647LL) return DMS_E_SIZE;
    const uint4 *d8 = defect8_table();
    uint4 *queue;
    uint32_t *qcount, qcap;
    queue_begin(ws, w0 * w1 * w2, s, &queue, &qcount, &qcap);
#define DMS_LAUNCH(GXV)                                                                              \
    hipLaunchKernelGGL((k_gradient<Keys, GXV, kTileVerts / GXV>), dim3((unsigned)blocks), dim3(kThreads), \
                       0, s, field, dims[0], dims[1], dims[2], lo[0], lo[1], lo[2], w0, w1, w2, bxc, byc, \
                       (uint4 *)rec, d8, queue, qcount, qcap, flags, mark)
    switch (variant) {
    case 0: DMS_LAUNCH(64); break;
    case 1: DMS_LAUNCH(32); break;
    default: DMS_LAUNCH(16); break;
    }
#undef DMS_LAUNCH
    queue_finish(queue, qcount, qcap, rec, mark, s);
    return launch_status();
}

int launch_gradient(int variant, const int32_t *order, const int64_t *dims, const int64_t *lo,
                    const int64_t *hi, uint32_t *rec, uint32_t *mark, char *ws, hipStream_t s)
{
    return launch_gradient_keys<RankKeys>(variant, order, dims, lo, hi, rec, mark, ws, nullptr, s);
}

int launch_gradient_batch(int variant, const int32_t *order, const BatchField *fields, int nfields,
                          const int64_t *tile_start, const uint16_t *tile_field, int64_t total_tiles,
                          int64_t total_verts, uint32_t *rec, uint32_t *mark, char *ws, hipStream_t s)
{
    (void)nfields;
    if (total_tiles == 0) return DMS_OK;
    if (total_tiles > 2147483647LL) return DMS_E_SIZE;
    if (mark) {
        const int64_t words = (total_verts + 31) / 32;
        hipLaunchKernelGGL(k_mark_zero, dim3((unsigned)((words + kThreads - 1) / kThreads)), dim3(kThreads), 0, s,
                           mark, words);
    }
    const uint4 *d8 = defect8_table();
    uint4 *queue;
    uint32_t *qcount, qcap;
    queue_begin(ws, total_verts, s, &queue, &qcount, &qcap);
#define DMS_LAUNCH(GXV)                                                                               \
    hipLaunchKernelGGL((k_gradient_batch<GXV, kTileVerts / GXV>), dim3((unsigned)total_tiles), dim3(kThreads), \
                       0, s, order, fields, tile_start, tile_field, (uint4 *)rec, d8, queue, qcount, qcap, mark)
    switch (variant) {
    case 0: DMS_LAUNCH(64); break;
    case 1: DMS_LAUNCH(32); break;
    default: DMS_LAUNCH(16); break;
    }
#undef DMS_LAUNCH
    queue_finish(queue, qcount, qcap, rec, mark, s);
    return launch_status();
}

}  // namespace dms

extern "C" size_t dms_gradient_workspace_size(const int64_t dims[3], const int64_t lo[3],
                                              const int64_t hi[3])
{
    using namespace dms;
    if (!box_valid(dims, lo, hi) || !grid_size_values_ok(dims)) return 0;
    return gradient_workspace_size((hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2]));
}

extern "C" int dms_discrete_gradient(const int32_t *order, const int64_t dims[3], const int64_t lo[3],
                                     const int64_t hi[3], uint32_t *rec, uint32_t *critical_mask,
                                     void *workspace, size_t workspace_bytes, void *stream)
{
    using namespace dms;
    if (!box_valid(dims, lo, hi)) return DMS_E_ARG;
    if (!grid_size_ok(dims)) return DMS_E_SIZE;
    const int64_t w0 = hi[0] - lo[0], w1 = hi[1] - lo[1], w2 = hi[2] - lo[2];
    if (w0 == 0 || w1 == 0 || w2 == 0) return DMS_OK;
    if (!order || !rec) return DMS_E_ARG;
    if (workspace && workspace_bytes < gradient_workspace_size(w0 * w1 * w2)) return DMS_E_WORKSPACE;
    if (const int st = tables_ready()) return st;
    return launch_gradient(0, order, dims, lo, hi, rec, critical_mask, (char *)workspace, (hipStream_t)stream);
}

extern "C" int dms_discrete_gradient_values(const void *values, int dtype, const int64_t dims[3],
                                            const int64_t lo[3], const int64_t hi[3], uint32_t *rec,
                                            uint32_t *critical_mask, void *workspace, size_t workspace_bytes,
                                            uint32_t *dev_flags, void *stream)
{
    using namespace dms;
    if (dtype != DMS_F32 && dtype != DMS_F64) return DMS_E_ARG;
    if (!box_valid(dims, lo, hi)) return DMS_E_ARG;
    if (!grid_size_values_ok(dims)) return DMS_E_SIZE;
    const int64_t w0 = hi[0] - lo[0], w1 = hi[1] - lo[1], w2 = hi[2] - lo[2];
    if (w0 == 0 || w1 == 0 || w2 == 0) return DMS_OK;
    if (!values || !rec || !dev_flags) return DMS_E_ARG;
    if (workspace && workspace_bytes < gradient_workspace_size(w0 * w1 * w2)) return DMS_E_WORKSPACE;
    if (const int st = tables_ready()) return st;
    if (dtype == DMS_F32)
        return launch_gradient_keys<F32Keys>(0, values, dims, lo, hi, rec, critical_mask, (char *)workspace,
                                             dev_flags,
                                             (hipStream_t)stream);
    return launch_gradient_keys<F64Keys>(0, values, dims, lo, hi, rec, critical_mask, (char *)workspace,
                                         dev_flags,
                                         (hipStream_t)stream);
}

extern "C" int dms_init(void *stream)
{
    if (const int st = dms::init_tables((hipStream_t)stream)) return st;
    return dms::init_critical_scratch();
}
