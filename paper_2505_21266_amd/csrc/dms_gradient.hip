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
//     integer minimum;
//  2. the cells of L(x) are enumerated in increasing key order (by highest
//     rank, then second, then third), giving each its position p;
//  3. Robins' two priority queues become bitsets over positions (pop-min is
//     find-first-set), the unpaired ("free") cells bitsets over star-table
//     indices, and the pairing runs in registers, with the two position maps
//     in per-thread LDS;
//  4. the outcome is packed into the 16-byte record described in dms.h.
// Readings: "unpaired" = neither paired nor critical; only unpaired cells are
// pushed onto the one-facet queue; the zero queue drops a cell as soon as it
// is paired, which yields what lazy deletion yields.
#include "dms_common.hpp"
#include "dms_tables.hpp"

namespace dms {
namespace {

constexpr int GX = 64, GY = 4, GZ = 1;  // owned vertices per block
constexpr int kThreads = GX * GY * GZ;
constexpr int HX = GX + 2, HY = GY + 2, HZ = GZ + 2;
constexpr int kHalo = HX * HY * HZ;
constexpr int32_t kAbsent = 0x7fffffff;

// cell ids inside one star: edges 0..13, triangles 14..49, tets 50..73
constexpr int kCellT = 14, kCellQ = 50, kCells = 74;

struct SharedTables {
    uint8_t tri_id[14][14];
    uint8_t tet_id[14][14][14];
    uint8_t tri_ab[36];        // a | b << 4
    uint8_t tri_slot[36];      // slot in edge_tris of a | slot of b << 4
    uint8_t tri_tet0[36];      // first star tet of the triangle
    uint16_t tri_edgemask[36];
    uint32_t tri_tetmask[36];
    uint64_t edge_trimask[14];
    uint64_t tet_trimask[24];
};

struct DeviceTables {
    SharedTables t;
};

constexpr DeviceTables make_device_tables()
{
    DeviceTables d{};
    const Tables &T = kTables;
    for (int a = 0; a < 14; ++a)
        for (int b = 0; b < 14; ++b) {
            d.t.tri_id[a][b] = (uint8_t)(T.tri_id[a][b] < 0 ? 255 : T.tri_id[a][b]);
            for (int c = 0; c < 14; ++c)
                d.t.tet_id[a][b][c] = (uint8_t)(T.tet_id[a][b][c] < 0 ? 255 : T.tet_id[a][b][c]);
        }
    for (int t = 0; t < 36; ++t) {
        d.t.tri_ab[t] = (uint8_t)(T.tri[t][0] | (T.tri[t][1] << 4));
        d.t.tri_slot[t] = (uint8_t)(T.tri_slot[t][0] | (T.tri_slot[t][1] << 4));
        d.t.tri_tet0[t] = (uint8_t)T.tri_tets[t][0];
        d.t.tri_edgemask[t] = T.tri_edgemask[t];
        d.t.tri_tetmask[t] = T.tri_tetmask[t];
    }
    for (int e = 0; e < 14; ++e) d.t.edge_trimask[e] = T.edge_trimask[e];
    for (int q = 0; q < 24; ++q) d.t.tet_trimask[q] = T.tet_trimask[q];
    return d;
}

__constant__ DeviceTables g_tables = make_device_tables();

struct Bits128 {
    uint64_t lo, hi;
    __device__ __forceinline__ void set(int p)
    {
        if (p < 64) lo |= 1ull << p; else hi |= 1ull << (p - 64);
    }
    __device__ __forceinline__ void clear(int p)
    {
        if (p < 64) lo &= ~(1ull << p); else hi &= ~(1ull << (p - 64));
    }
    __device__ __forceinline__ bool any() const { return (lo | hi) != 0; }
    // index of the lowest set bit, which is cleared
    __device__ __forceinline__ int pop_lowest()
    {
        if (lo) {
            int p = __ffsll((unsigned long long)lo) - 1;
            lo &= lo - 1;
            return p;
        }
        int p = __ffsll((unsigned long long)hi) - 1;
        hi &= hi - 1;
        return p + 64;
    }
};

// per-thread arrays, interleaved by thread so that equal indices of
// neighbouring lanes sit in neighbouring bytes
struct ThreadScratch {
    uint8_t pos_of[kCells][kThreads];
    uint8_t cell_at[kCells][kThreads];
    uint8_t nb_at[14][kThreads];
    uint16_t adj[14][kThreads];
};

struct Star {
    const SharedTables &T;
    ThreadScratch &S;
    int tid;
    uint32_t fe;   // free edges (neighbour bits)
    uint64_t ft;   // free triangles
    uint32_t fq;   // free tets
    Bits128 q1, q0;
    uint64_t rec_lo, rec_hi;

    __device__ __forceinline__ int pos(int cell) const { return S.pos_of[cell][tid]; }

    __device__ __forceinline__ void set_tri_field(int t, uint32_t v)
    {
        const int b = 56 + 2 * t;
        if (b < 64) rec_lo |= (uint64_t)v << b; else rec_hi |= (uint64_t)v << (b - 64);
    }

    // push free triangles of edge e with exactly one free edge
    __device__ __forceinline__ void push_cofacets_edge(int e)
    {
        uint64_t m = T.edge_trimask[e] & ft;
        while (m) {
            const int t = __ffsll((unsigned long long)m) - 1;
            m &= m - 1;
            if (__popc(T.tri_edgemask[t] & fe) == 1) q1.set(pos(kCellT + t));
        }
    }

    // push free tets of triangle t with exactly one free triangle
    __device__ __forceinline__ void push_cofacets_tri(int t)
    {
        uint32_t m = T.tri_tetmask[t] & fq;
        while (m) {
            const int q = __ffs(m) - 1;
            m &= m - 1;
            if (__popcll(T.tet_trimask[q] & ft) == 1) q1.set(pos(kCellQ + q));
        }
    }
};

__device__ void process_vertex(const int32_t *o, int32_t ox, const SharedTables &T,
                               ThreadScratch &S, int tid, uint4 &out)
{
    uint32_t low = 0;
#pragma unroll
    for (int e = 0; e < 14; ++e) low |= (o[e] < ox ? 1u : 0u) << e;
    if (low == 0) {  // L(x) = {x}: x is critical
        out = make_uint4(0, 0, 0, 0);
        return;
    }
    // 1. ranks among the lower neighbours (non-lower ones rank above them)
    uint32_t ol[14], r[14];
#pragma unroll
    for (int e = 0; e < 14; ++e) {
        ol[e] = (low >> e) & 1u ? (uint32_t)o[e] : 0xffffffffu;
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
    uint32_t bitv[14];
#pragma unroll
    for (int e = 0; e < 14; ++e) bitv[e] = (low >> e) & 1u ? 1u << r[e] : 0u;
#pragma unroll
    for (int e = 0; e < 14; ++e) {
        if ((low >> e) & 1u) {
            uint32_t a = 0;
#pragma unroll
            for (int f = 0; f < 14; ++f)
                if ((kTables.link[e] >> f) & 1u) a |= bitv[f];
            S.nb_at[r[e]][tid] = (uint8_t)e;
            S.adj[r[e]][tid] = (uint16_t)a;
        }
    }
    const int m = __popc(low);

    // 2. enumerate L(x) \ {x} in key order
    Star st{T, S, tid, 0, 0, 0, {0, 0}, {0, 0}, 0, 0};
    uint64_t in_t = 0;
    uint32_t in_q = 0;
    int P = 0;
    for (int h = 0; h < m; ++h) {
        const int e = S.nb_at[h][tid];
        const uint32_t ah = S.adj[h][tid];
        S.pos_of[e][tid] = (uint8_t)P;
        S.cell_at[P][tid] = (uint8_t)e;
        if (h > 0) st.q0.set(P);
        ++P;
        uint32_t A = ah & ((1u << h) - 1u);
        while (A) {
            const int s = __ffs(A) - 1;
            A &= A - 1;
            const int f = S.nb_at[s][tid];
            const int t = T.tri_id[e][f];
            in_t |= 1ull << t;
            S.pos_of[kCellT + t][tid] = (uint8_t)P;
            S.cell_at[P][tid] = (uint8_t)(kCellT + t);
            ++P;
            uint32_t B = ah & S.adj[s][tid] & ((1u << s) - 1u);
            while (B) {
                const int u = __ffs(B) - 1;
                B &= B - 1;
                const int g = S.nb_at[u][tid];
                const int q = T.tet_id[e][f][g];
                in_q |= 1u << q;
                S.pos_of[kCellQ + q][tid] = (uint8_t)P;
                S.cell_at[P][tid] = (uint8_t)(kCellQ + q);
                ++P;
            }
        }
    }

    // 3. Robins' pairing
    const int delta = S.nb_at[0][tid];  // smallest edge: lowest lower neighbour, position 0
    st.fe = low & ~(1u << delta);
    st.ft = in_t;
    st.fq = in_q;
    st.rec_lo = 1ull << (4 * delta);  // delta is paired with x
    st.push_cofacets_edge(delta);
    for (;;) {
        while (st.q1.any()) {
            const int p = st.q1.pop_lowest();
            const int c = S.cell_at[p][tid];
            if (c < kCellQ) {  // triangle
                const int t = c - kCellT;
                const uint32_t fm = T.tri_edgemask[t] & st.fe;
                if (fm == 0) {
                    st.q0.set(p);
                } else {
                    const int b = __ffs(fm) - 1;  // its only free edge
                    st.fe &= ~(1u << b);
                    st.ft &= ~(1ull << t);
                    const uint32_t ab = T.tri_ab[t], sl = T.tri_slot[t];
                    const uint32_t slot = (int)(ab & 15u) == b ? (sl & 15u) : (sl >> 4);
                    st.rec_lo |= (uint64_t)(3u + slot) << (4 * b);
                    st.q0.clear(st.pos(b));
                    st.push_cofacets_tri(t);
                    st.push_cofacets_edge(b);
                }
            } else {  // tet
                const int q = c - kCellQ;
                const uint64_t fm = T.tet_trimask[q] & st.ft;
                if (fm == 0) {
                    st.q0.set(p);
                } else {
                    const int b = __ffsll((unsigned long long)fm) - 1;  // its only free triangle
                    st.ft &= ~(1ull << b);
                    st.fq &= ~(1u << q);
                    st.set_tri_field(b, T.tri_tet0[b] == q ? 1u : 2u);
                    st.q0.clear(st.pos(kCellT + b));
                    st.push_cofacets_tri(b);
                }
            }
        }
        if (!st.q0.any()) break;
        const int p = st.q0.pop_lowest();
        const int c = S.cell_at[p][tid];
        if (c < kCellT) {  // critical edge
            st.fe &= ~(1u << c);
            st.rec_lo |= 2ull << (4 * c);
            st.push_cofacets_edge(c);
        } else if (c < kCellQ) {  // critical triangle
            st.ft &= ~(1ull << (c - kCellT));
            st.push_cofacets_tri(c - kCellT);
        } else {  // critical tet
            st.fq &= ~(1u << (c - kCellQ));
        }
    }
    out = make_uint4((uint32_t)st.rec_lo, (uint32_t)(st.rec_lo >> 32), (uint32_t)st.rec_hi,
                     (uint32_t)(st.rec_hi >> 32));
}

__global__ __launch_bounds__(kThreads) void k_gradient(const int32_t *__restrict__ order,
                                                       int64_t nx, int64_t ny, int64_t nz,
                                                       int64_t lo0, int64_t lo1, int64_t lo2,
                                                       int64_t w0, int64_t w1, int64_t w2,
                                                       int64_t bx_count, int64_t by_count,
                                                       uint4 *__restrict__ rec)
{
    __shared__ SharedTables T;
    __shared__ int32_t tile[kHalo];
    __shared__ ThreadScratch S;

    const int tid = threadIdx.x;
    {
        const uint32_t *src = (const uint32_t *)&g_tables.t;
        uint32_t *dst = (uint32_t *)&T;
        for (int i = tid; i < (int)(sizeof(SharedTables) / 4); i += kThreads) dst[i] = src[i];
    }
    const int64_t b = blockIdx.x;
    const int64_t bx = b % bx_count, by = (b / bx_count) % by_count, bz = b / (bx_count * by_count);
    const int64_t x0 = lo0 + bx * GX - 1, y0 = lo1 + by * GY - 1, z0 = lo2 + bz * GZ - 1;
    for (int i = tid; i < kHalo; i += kThreads) {
        const int hx = i % HX, hy = (i / HX) % HY, hz = i / (HX * HY);
        const int64_t x = x0 + hx, y = y0 + hy, z = z0 + hz;
        int32_t v = kAbsent;
        if (x >= 0 && y >= 0 && z >= 0 && x < nx && y < ny && z < nz) v = order[x + nx * (y + ny * z)];
        tile[i] = v;
    }
    __syncthreads();

    const int tx = tid % GX, ty = (tid / GX) % GY, tz = tid / (GX * GY);
    const int64_t ox_ = bx * GX + tx, oy_ = by * GY + ty, oz_ = bz * GZ + tz;  // box coordinates
    if (ox_ >= w0 || oy_ >= w1 || oz_ >= w2) return;
    const int c = (tx + 1) + HX * ((ty + 1) + HY * (tz + 1));
    int32_t o[14];
#pragma unroll
    for (int e = 0; e < 14; ++e)
        o[e] = tile[c + kTables.nb[e][0] + HX * (kTables.nb[e][1] + HY * kTables.nb[e][2])];
    uint4 r;
    process_vertex(o, tile[c], T, S, tid, r);
    rec[ox_ + w0 * (oy_ + w1 * oz_)] = r;
}

}  // namespace
}  // namespace dms

extern "C" int dms_discrete_gradient(const int32_t *order, const int64_t dims[3], const int64_t lo[3],
                                     const int64_t hi[3], uint32_t *rec, void *stream)
{
    using namespace dms;
    if (!box_valid(dims, lo, hi)) return DMS_E_ARG;
    if (!grid_size_ok(dims)) return DMS_E_SIZE;
    const int64_t w0 = hi[0] - lo[0], w1 = hi[1] - lo[1], w2 = hi[2] - lo[2];
    if (w0 == 0 || w1 == 0 || w2 == 0) return DMS_OK;
    if (!order || !rec) return DMS_E_ARG;
    const int64_t bxc = (w0 + GX - 1) / GX, byc = (w1 + GY - 1) / GY, bzc = (w2 + GZ - 1) / GZ;
    const int64_t blocks = bxc * byc * bzc;
    if (blocks > 2147483647LL) return DMS_E_SIZE;
    hipLaunchKernelGGL(k_gradient, dim3((unsigned)blocks), dim3(kThreads), 0, (hipStream_t)stream,
                       order, dims[0], dims[1], dims[2], lo[0], lo[1], lo[2], w0, w1, w2, bxc, byc,
                       (uint4 *)rec);
    return launch_status();
}
