// dms_filtration.hip -- critical cells of one dimension in the filtration
// order of Section 2.1: a cell's key is the list of its vertex orders sorted
// decreasingly, and keys of one dimension compare lexicographically.
//
// A key holds at most four orders, each below 2^31.  It is packed into two
// 64-bit words, hi = o1 << 32 | o2 and lo = o3 << 32 | o4 (absent entries
// 0), and the list is ranked by the radix passes: by lo first, then stably by
// hi, which is the lexicographic order of (hi, lo).  Vertices and edges need
// the hi word only.
#include "dms_common.hpp"
#include "dms_internal.hpp"
#include "dms_tables.hpp"

namespace dms {
namespace {

constexpr int kThreads = 256;

// The star geometry a cell code refers to (kernel argument).
struct Geom {
    int8_t nb[14][3];  // (dx, dy, dz) of neighbour e
    uint8_t tri[36][2];
    uint8_t tet[24][3];
};

Geom make_geom()
{
    Geom g{};
    const Tables &T = kTables;
    for (int e = 0; e < 14; ++e)
        for (int c = 0; c < 3; ++c) g.nb[e][c] = (int8_t)T.nb[e][c];
    for (int t = 0; t < 36; ++t)
        for (int c = 0; c < 2; ++c) g.tri[t][c] = (uint8_t)T.tri[t][c];
    for (int q = 0; q < 24; ++q)
        for (int c = 0; c < 3; ++c) g.tet[q][c] = (uint8_t)T.tet[q][c];
    return g;
}

__device__ __forceinline__ void cswap_desc(uint32_t &a, uint32_t &b)
{
    const uint32_t hi = max(a, b), lo = min(a, b);
    a = hi;
    b = lo;
}

// Keys of the cells: code = (maxv << 8) | local index (0 for a vertex,
// neighbour e for an edge, star triangle t, star tet q).  A code naming no
// cell of the grid gets the largest key and raises DMS_FLAG_BADCODE.
__global__ __launch_bounds__(kThreads) void k_cell_keys(const int64_t *__restrict__ codes, int64_t count,
                                                        int dim, const int32_t *__restrict__ order,
                                                        int64_t nx, int64_t ny, int64_t nz, Geom g,
                                                        uint64_t *__restrict__ hi, uint64_t *__restrict__ lo,
                                                        uint32_t *flags)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= count) return;
    const int64_t code = codes[i];
    const int64_t v = code >> 8;
    const int loc = (int)(code & 255);
    const int64_t n = nx * ny * nz;
    int oth[3] = {0, 0, 0};
    bool bad = v < 0 || v >= n;
    if (dim == 0) {
        bad = bad || loc != 0;
    } else if (dim == 1) {
        bad = bad || loc >= 14;
        oth[0] = loc < 14 ? loc : 0;
    } else if (dim == 2) {
        bad = bad || loc >= 36;
        const int t = loc < 36 ? loc : 0;
        oth[0] = g.tri[t][0];
        oth[1] = g.tri[t][1];
    } else {
        bad = bad || loc >= 24;
        const int q = loc < 24 ? loc : 0;
        oth[0] = g.tet[q][0];
        oth[1] = g.tet[q][1];
        oth[2] = g.tet[q][2];
    }
    uint32_t o[4] = {0u, 0u, 0u, 0u};
    if (!bad) {
        const int64_t x = v % nx, y = (v / nx) % ny, z = v / (nx * ny);
        o[0] = (uint32_t)order[v];
        for (int k = 0; k < dim; ++k) {
            const int e = oth[k];
            const int64_t a = x + g.nb[e][0], b = y + g.nb[e][1], c = z + g.nb[e][2];
            if (a < 0 || b < 0 || c < 0 || a >= nx || b >= ny || c >= nz) {
                bad = true;
                break;
            }
            o[k + 1] = (uint32_t)order[a + nx * (b + ny * c)];
        }
    }
    // decreasing: a five-comparator network on four entries; the absent ones
    // (0) end up last, where every cell of the dimension has them
    cswap_desc(o[0], o[1]);
    cswap_desc(o[2], o[3]);
    cswap_desc(o[0], o[2]);
    cswap_desc(o[1], o[3]);
    cswap_desc(o[1], o[2]);
    if (bad) {
        atomicOr(flags, (uint32_t)DMS_FLAG_BADCODE);
        hi[i] = ~0ull;
        lo[i] = ~0ull;
        return;
    }
    hi[i] = ((uint64_t)o[0] << 32) | o[1];
    lo[i] = ((uint64_t)o[2] << 32) | o[3];
}

// out[rank[i]] = in[i] for the codes, and (optionally) the keys.
__global__ __launch_bounds__(kThreads) void k_cell_place(const int32_t *__restrict__ rank, int64_t count,
                                                         const int64_t *__restrict__ in_codes,
                                                         const uint64_t *__restrict__ in_key,
                                                         int64_t *__restrict__ out_codes,
                                                         uint64_t *__restrict__ out_key)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= count) return;
    const int32_t r = rank[i];
    if (r < 0 || r >= count) return;
    if (out_codes) out_codes[r] = in_codes[i];
    if (out_key) out_key[r] = in_key[i];
}

// rank[i] = second[first[i]]: the position after the low-word pass, then
// after the high-word pass.
__global__ __launch_bounds__(kThreads) void k_compose(const int32_t *__restrict__ first,
                                                      const int32_t *__restrict__ second, int64_t count,
                                                      int32_t *__restrict__ rank)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= count) return;
    const int32_t a = first[i];
    rank[i] = a >= 0 && a < count ? second[a] : a;
}

struct RankLayout {
    size_t hi, lo, hi2, r1, r2, rws, total;
};

RankLayout rank_layout(int64_t count)
{
    const size_t c = (size_t)(count > 0 ? count : 1);
    RankLayout L{};
    size_t off = 0;
    L.hi = off; off += align_up(c * 8, 256);
    L.lo = off; off += align_up(c * 8, 256);
    L.hi2 = off; off += align_up(c * 8, 256);
    L.r1 = off; off += align_up(c * 4, 256);
    L.r2 = off; off += align_up(c * 4, 256);
    L.rws = off; off += rank_u64_workspace_size(count);
    L.total = off;
    return L;
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

}  // namespace

size_t cell_rank_workspace_size(int64_t count) { return rank_layout(count).total; }

int launch_cell_ranks(const int64_t *codes, int64_t count, int dim, const int32_t *order, const int64_t *dims,
                      int32_t *rank, char *ws, uint32_t *flags, hipStream_t s)
{
    if (count == 0) return DMS_OK;
    const RankLayout L = rank_layout(count);
    uint64_t *hi = (uint64_t *)(ws + L.hi), *lo = (uint64_t *)(ws + L.lo), *hi2 = (uint64_t *)(ws + L.hi2);
    int32_t *r1 = (int32_t *)(ws + L.r1), *r2 = (int32_t *)(ws + L.r2);
    const unsigned blocks = blocks_for(count);
    hipLaunchKernelGGL(k_cell_keys, dim3(blocks), dim3(kThreads), 0, s, codes, count, dim, order, dims[0],
                       dims[1], dims[2], make_geom(), hi, lo, flags);
    if (dim < 2) return launch_rank_u64(hi, count, rank, ws + L.rws, flags, s);
    // the low word first; the high word's stable ranking then orders by
    // (hi, lo)
    int st = launch_rank_u64(lo, count, r1, ws + L.rws, flags, s);
    if (st) return st;
    hipLaunchKernelGGL(k_cell_place, dim3(blocks), dim3(kThreads), 0, s, r1, count, (const int64_t *)nullptr,
                       hi, (int64_t *)nullptr, hi2);
    st = launch_rank_u64(hi2, count, r2, ws + L.rws, flags, s);
    if (st) return st;
    hipLaunchKernelGGL(k_compose, dim3(blocks), dim3(kThreads), 0, s, r1, r2, count, rank);
    return launch_status();
}

}  // namespace dms

namespace {
size_t sort_rank_offset(int64_t count)
{
    return dms::align_up((size_t)(count > 0 ? count : 1) * 4, 256);
}
}  // namespace

extern "C" size_t dms_critical_sort_workspace_size(int64_t count)
{
    if (count < 0) return 0;
    return sort_rank_offset(count) + dms::cell_rank_workspace_size(count);
}

extern "C" int dms_critical_sort(const int64_t *codes, int64_t count, int dim, const int32_t *order,
                                 const int64_t dims[3], int64_t *sorted, void *workspace,
                                 size_t workspace_bytes, uint32_t *dev_flags, void *stream)
{
    using namespace dms;
    if (!dims || dims[0] < 1 || dims[1] < 1 || dims[2] < 1 || count < 0 || dim < 0 || dim > 3)
        return DMS_E_ARG;
    if (!grid_size_ok(dims)) return DMS_E_SIZE;
    if (count > 2147483647LL) return DMS_E_SIZE;
    if (count == 0) return DMS_OK;
    if (!codes || !order || !sorted || !dev_flags || sorted == codes) return DMS_E_ARG;
    if (!workspace || workspace_bytes < dms_critical_sort_workspace_size(count)) return DMS_E_WORKSPACE;
    if (const int dc = device_check()) return dc;
    hipStream_t s = (hipStream_t)stream;
    char *ws = (char *)workspace;
    int32_t *rank = (int32_t *)ws;
    const int st = launch_cell_ranks(codes, count, dim, order, dims, rank, ws + sort_rank_offset(count),
                                     dev_flags, s);
    if (st) return st;
    hipLaunchKernelGGL(k_cell_place, dim3(blocks_for(count)), dim3(kThreads), 0, s, rank, count, codes,
                       (const uint64_t *)nullptr, sorted, (uint64_t *)nullptr);
    return launch_status();
}
