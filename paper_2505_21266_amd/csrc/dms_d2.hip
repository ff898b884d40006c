// dms_d2.hip -- the extremum-graph half of the D2 pairing on the GPU
// (Section 2.6: D2 is computed like D0 on the dual complex, where every
// discrete vector is reversed).  The dual graph has one node per tet and one
// for the outside of the grid; a triangle on the grid boundary joins its one
// tet to the outside node.
//
//   trip   one thread per critical triangle: from each of its two cofacet
//          tets (the outside node where one is missing) the dual v-path is
//          followed -- a tet that is the head of a gradient pair is left
//          through its tail triangle to the other tet containing it -- until
//          a critical tet (a maximum) or the outside node.  Maxima become
//          indices into the critical tet list (a binary search: the list is
//          in code order); the outside node is index n3.
//   order  the triplets whose maxima differ, by decreasing triangle (the
//          Section 2.1 ranking of the critical triangles, reversed, and a
//          scan over the kept ones); the maxima's own ranks for the
//          union-find's comparisons.
// Paths are acyclic (the gradient has no closed v-path), so every walk ends;
// a walk longer than the number of tets raises DMS_FLAG_CAPACITY instead of
// running on.  The union-find itself (dms_d2_pairs_sorted_host) runs on the
// host, like Algorithm 1's.
#include "dms_common.hpp"
#include "dms_internal.hpp"
#include "dms_scan.hpp"
#include "dms_tables.hpp"

namespace dms {
namespace {

constexpr int kThreads = 256;

struct D2Tables {
    int8_t nb[14][3];
    int8_t nb_of[27];  // neighbour index of offset d, at (dx+1) + 3 (dy+1) + 9 (dz+1); -1 if none
    int8_t tet[24][3];
    int8_t tet_tris[24][3];
    int8_t tri[36][2];
    int8_t tri_tets[36][2];
    int8_t tet_id[14][14][14];
};

constexpr D2Tables make_d2_tables()
{
    D2Tables D{};
    const Tables &T = kTables;
    for (int i = 0; i < 27; ++i) D.nb_of[i] = -1;
    for (int e = 0; e < 14; ++e) {
        for (int c = 0; c < 3; ++c) D.nb[e][c] = (int8_t)T.nb[e][c];
        D.nb_of[(T.nb[e][0] + 1) + 3 * (T.nb[e][1] + 1) + 9 * (T.nb[e][2] + 1)] = (int8_t)e;
    }
    for (int q = 0; q < 24; ++q)
        for (int c = 0; c < 3; ++c) {
            D.tet[q][c] = (int8_t)T.tet[q][c];
            D.tet_tris[q][c] = (int8_t)T.tet_tris[q][c];
        }
    for (int t = 0; t < 36; ++t)
        for (int c = 0; c < 2; ++c) {
            D.tri[t][c] = (int8_t)T.tri[t][c];
            D.tri_tets[t][c] = (int8_t)T.tri_tets[t][c];
        }
    for (int a = 0; a < 14; ++a)
        for (int b = 0; b < 14; ++b)
            for (int c = 0; c < 14; ++c) D.tet_id[a][b][c] = (int8_t)T.tet_id[a][b][c];
    return D;
}

__constant__ D2Tables c_d2 = make_d2_tables();

struct Grid {
    int64_t nx, ny, nz;
};

// Triangle field t (2 bits at 56 + 2t of the 128-bit record): 0 not paired
// with a tet, 1 + j paired with the j-th star tet containing t.
__device__ __forceinline__ int tri_state(const uint4 &w, int t)
{
    const int b = 56 + 2 * t;
    const uint32_t word = b < 64 ? w.y : (b < 96 ? w.z : w.w);
    return (int)((word >> (b & 31)) & 3u);
}

// Code of the tet made of v and the star tet q of v, whose vertices must lie
// in the grid: (highest vertex << 8) | local index in that vertex's star; -1
// if the star tables do not place it (cannot happen: the Kuhn complex is a
// flag complex, so the four pairwise adjacent vertices form a star tet of
// each of them).
__device__ int64_t tet_code(const int32_t *__restrict__ order, int64_t nx, int64_t ny, int64_t v, int q)
{
    int off[4][3];
    int64_t id[4];
    int32_t o[4];
    off[0][0] = off[0][1] = off[0][2] = 0;
    id[0] = v;
    o[0] = order[v];
    int top = 0;
    for (int k = 0; k < 3; ++k) {
        const int e = c_d2.tet[q][k];
        for (int c = 0; c < 3; ++c) off[k + 1][c] = c_d2.nb[e][c];
        id[k + 1] = v + off[k + 1][0] + nx * (off[k + 1][1] + ny * off[k + 1][2]);
        o[k + 1] = order[id[k + 1]];
        if (o[k + 1] > o[top]) top = k + 1;
    }
    if (top == 0) return (v << 8) | q;
    int es[3], ne = 0;
    for (int k = 0; k < 4; ++k) {
        if (k == top) continue;
        const int dx = off[k][0] - off[top][0], dy = off[k][1] - off[top][1], dz = off[k][2] - off[top][2];
        const bool near = dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1 && dz >= -1 && dz <= 1;
        es[ne] = near ? c_d2.nb_of[(dx + 1) + 3 * (dy + 1) + 9 * (dz + 1)] : -1;
        if (es[ne] < 0) return -1;
        ++ne;
    }
    const int loc = c_d2.tet_id[es[0]][es[1]][es[2]];
    return loc < 0 ? -1 : (id[top] << 8) | loc;
}

// Whether every vertex of star tet q of v = (x, y, z) lies in the grid.
__device__ __forceinline__ bool tet_inside(const Grid &g, int64_t x, int64_t y, int64_t z, int q)
{
    bool in = true;
    for (int k = 0; k < 3; ++k) {
        const int e = c_d2.tet[q][k];
        const int64_t a = x + c_d2.nb[e][0], b = y + c_d2.nb[e][1], c = z + c_d2.nb[e][2];
        in = in && a >= 0 && b >= 0 && c >= 0 && a < g.nx && b < g.ny && c < g.nz;
    }
    return in;
}

// The maximum reached from tet `code` along the dual v-path, or -1 for the
// outside node.
__device__ int64_t walk_up(const uint4 *__restrict__ rec, const int32_t *__restrict__ order, const Grid &g,
                           int64_t code, int64_t limit, bool &stall)
{
    for (int64_t step = 0;; ++step) {
        if (step > limit || code < 0) {
            stall = true;
            return -1;
        }
        const int64_t m = code >> 8;
        const int q = (int)(code & 255);
        if (q >= 24) {
            stall = true;
            return -1;
        }
        const uint4 w = rec[m];
        int tail = -1;
        for (int s = 0; s < 3; ++s) {
            const int t = c_d2.tet_tris[q][s];
            const int st = tri_state(w, t);
            if (st && c_d2.tri_tets[t][st - 1] == q) tail = t;
        }
        if (tail < 0) return code;  // a critical tet
        const int q2 = c_d2.tri_tets[tail][0] == q ? c_d2.tri_tets[tail][1] : c_d2.tri_tets[tail][0];
        const int64_t x = m % g.nx, y = (m / g.nx) % g.ny, z = m / (g.nx * g.ny);
        if (!tet_inside(g, x, y, z, q2)) return -1;
        code = tet_code(order, g.nx, g.ny, m, q2);
    }
}

// index of code in the sorted list, or -1
__device__ __forceinline__ int64_t find_code(const int64_t *__restrict__ list, int64_t n, int64_t code)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (list[mid] < code) lo = mid + 1; else hi = mid;
    }
    return lo < n && list[lo] == code ? lo : -1;
}

__global__ __launch_bounds__(kThreads) void k_d2_trip(const uint4 *__restrict__ rec,
                                                      const int32_t *__restrict__ order, Grid g,
                                                      const int64_t *__restrict__ crit2, int64_t n2,
                                                      const int64_t *__restrict__ crit3, int64_t n3,
                                                      int32_t *__restrict__ m0, int32_t *__restrict__ m1,
                                                      uint32_t *__restrict__ keep, unsigned long long *ntri,
                                                      uint32_t *flags)
{
    const int64_t s = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    bool valid = false;
    if (s < n2) {
        const int64_t v = crit2[s] >> 8;
        const int t = (int)(crit2[s] & 255);
        const int64_t n = g.nx * g.ny * g.nz;
        int64_t idx[2] = {n3, n3};
        bool bad = v < 0 || v >= n || t >= 36, stall = false;
        if (!bad) {
            const int64_t x = v % g.nx, y = (v / g.nx) % g.ny, z = v / (g.nx * g.ny);
            for (int c = 0; c < 2; ++c) {
                const int q = c_d2.tri_tets[t][c];
                if (!tet_inside(g, x, y, z, q)) continue;  // outside node
                const int64_t top = walk_up(rec, order, g, tet_code(order, g.nx, g.ny, v, q), 6 * n, stall);
                idx[c] = top < 0 ? n3 : find_code(crit3, n3, top);
            }
        }
        if (bad || stall || idx[0] < 0 || idx[1] < 0) {
            atomicOr(flags, (uint32_t)DMS_FLAG_CAPACITY);  // a maximum missing from crit3, or a bad code
        } else {
            valid = idx[0] != idx[1];
        }
        m0[s] = (int32_t)(idx[0] < 0 ? n3 : idx[0]);
        m1[s] = (int32_t)(idx[1] < 0 ? n3 : idx[1]);
    }
    const uint64_t b = __ballot(valid);
    if (lane_id() == 0 && b) atomicAdd(ntri, (unsigned long long)__popcll(b));
    if (s < n2) keep[s] = valid ? 1u : 0u;
}

// at[n2 - 1 - rank[s]] = keep[s]: the kept flags in decreasing triangle order
__global__ __launch_bounds__(kThreads) void k_d2_flags(const int32_t *__restrict__ rank, int64_t n2,
                                                       const uint32_t *__restrict__ keep, uint32_t *__restrict__ at)
{
    const int64_t s = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (s >= n2) return;
    const int64_t p = n2 - 1 - rank[s];
    if (p >= 0 && p < n2) at[p] = keep[s];
}

__global__ __launch_bounds__(kThreads) void k_d2_place(const int32_t *__restrict__ rank, int64_t n2,
                                                       const uint32_t *__restrict__ keep,
                                                       const uint32_t *__restrict__ pos,
                                                       const int64_t *__restrict__ crit2,
                                                       const int32_t *__restrict__ m0,
                                                       const int32_t *__restrict__ m1,
                                                       int64_t *__restrict__ tri_code,
                                                       int32_t *__restrict__ tri_max0,
                                                       int32_t *__restrict__ tri_max1)
{
    const int64_t s = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (s >= n2 || !keep[s]) return;
    const int64_t p = n2 - 1 - rank[s];
    if (p < 0 || p >= n2) return;
    const uint32_t r = pos[p];
    if ((int64_t)r >= n2) return;
    tri_code[r] = crit2[s];
    tri_max0[r] = m0[s];
    tri_max1[r] = m1[s];
}

__global__ void k_d2_zero(unsigned long long *p) { *p = 0ull; }

struct D2Layout {
    size_t m0, m1, keep, at, rank, partials, rws, total;
};

D2Layout d2_layout(int64_t n2, int64_t n3)
{
    const size_t c2 = (size_t)(n2 > 0 ? n2 : 1);
    D2Layout L{};
    size_t off = 0;
    L.m0 = off; off += align_up(c2 * 4, 256);
    L.m1 = off; off += align_up(c2 * 4, 256);
    L.keep = off; off += align_up(c2 * 4, 256);
    L.at = off; off += align_up(c2 * 4, 256);
    L.rank = off; off += align_up(c2 * 4, 256);
    L.partials = off; off += align_up(scan_partials_bytes(n2 > 0 ? n2 : 1, 4), 256);
    const size_t r2 = cell_rank_workspace_size(n2 > 0 ? n2 : 1), r3 = cell_rank_workspace_size(n3 > 0 ? n3 : 1);
    L.rws = off; off += r2 > r3 ? r2 : r3;
    L.total = off;
    return L;
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

}  // namespace
}  // namespace dms

extern "C" size_t dms_d2_workspace_size(int64_t n2, int64_t n3)
{
    if (n2 < 0 || n3 < 0) return 0;
    return dms::d2_layout(n2, n3).total;
}

extern "C" int dms_d2_triplets(const uint32_t *rec, const int32_t *order, const int64_t dims[3],
                               const int64_t *crit2, int64_t n2, const int64_t *crit3, int64_t n3,
                               int64_t *tri_code, int32_t *tri_max0, int32_t *tri_max1, int32_t *max_rank,
                               int64_t *ntri, void *workspace, size_t workspace_bytes, uint32_t *dev_flags,
                               void *stream)
{
    using namespace dms;
    if (!dims || dims[0] < 1 || dims[1] < 1 || dims[2] < 1 || n2 < 0 || n3 < 0) return DMS_E_ARG;
    if (!grid_size_ok(dims)) return DMS_E_SIZE;
    if (n2 > 2147483647LL || n3 >= 2147483647LL) return DMS_E_SIZE;
    if (!rec || !order || !ntri || !dev_flags) return DMS_E_ARG;
    if ((n2 > 0 && (!crit2 || !tri_code || !tri_max0 || !tri_max1)) || (n3 > 0 && (!crit3 || !max_rank)))
        return DMS_E_ARG;
    const D2Layout L = d2_layout(n2, n3);
    if (!workspace || workspace_bytes < L.total) return DMS_E_WORKSPACE;
    if (const int dc = device_check()) return dc;
    hipStream_t s = (hipStream_t)stream;
    char *ws = (char *)workspace;
    int32_t *m0 = (int32_t *)(ws + L.m0), *m1 = (int32_t *)(ws + L.m1), *rank = (int32_t *)(ws + L.rank);
    uint32_t *keep = (uint32_t *)(ws + L.keep), *at = (uint32_t *)(ws + L.at);
    unsigned long long *count = (unsigned long long *)ntri;  // counted in place
    hipLaunchKernelGGL(k_d2_zero, dim3(1), dim3(1), 0, s, count);
    if (n3 > 0) {
        const int st = launch_cell_ranks(crit3, n3, 3, order, dims, max_rank, ws + L.rws, dev_flags, s);
        if (st) return st;
    }
    if (n2 > 0) {
        const Grid g{dims[0], dims[1], dims[2]};
        hipLaunchKernelGGL(k_d2_trip, dim3(blocks_for(n2)), dim3(kThreads), 0, s, (const uint4 *)rec, order, g,
                           crit2, n2, crit3, n3, m0, m1, keep, count, dev_flags);
        const int st = launch_cell_ranks(crit2, n2, 2, order, dims, rank, ws + L.rws, dev_flags, s);
        if (st) return st;
        hipLaunchKernelGGL(k_d2_flags, dim3(blocks_for(n2)), dim3(kThreads), 0, s, rank, n2, keep, at);
        exclusive_scan<uint32_t>(at, n2, (uint32_t *)(ws + L.partials), s);
        hipLaunchKernelGGL(k_d2_place, dim3(blocks_for(n2)), dim3(kThreads), 0, s, rank, n2, keep, at, crit2, m0,
                           m1, tri_code, tri_max0, tri_max1);
    }
    return launch_status();
}
