// dms_d0.hip -- the extremum-graph half of the D0 pairing on the GPU
// (Section 2.6: from both vertices of every critical edge, descend along the
// vertex-edge vectors of the gradient to a minimum; Algorithm 1 then visits
// the triplets (edge, minimum, minimum) in increasing edge order).
//
//   next   v -> the other vertex of the edge v is paired with, or v itself
//          when v is critical (a minimum: its record pairs it with nothing);
//   jump   pointer doubling until every vertex points at its minimum;
//   trip   per critical edge: the indices (in the critical-vertex list) of
//          its two minima and its key -- the order of its higher vertex, then
//          of its lower one (Section 2.1); an edge whose minima coincide gets
//          the largest key and is not counted;
//   sort   ranks of the keys by the radix passes, then placement.
// The union-find of Algorithm 1 stays on the host (dms_d0_pairs_sorted_host):
// it is sequential and touches only the minima.
#include "dms_common.hpp"
#include "dms_internal.hpp"
#include "dms_tables.hpp"

namespace dms {
namespace {

constexpr int kThreads = 256;

struct Steps {
    int64_t s[14];  // vertex-id offset of neighbour e
};

__device__ __forceinline__ bool in_grid(int64_t v, int64_t n) { return v >= 0 && v < n; }

__global__ __launch_bounds__(kThreads) void k_d0_next(const uint4 *__restrict__ rec, int64_t n, Steps st,
                                                      int32_t *__restrict__ next)
{
    const int64_t v = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (v >= n) return;
    const uint4 w = rec[v];
    const uint64_t lo = (uint64_t)w.x | ((uint64_t)w.y << 32);
    int64_t to = v;
#pragma unroll
    for (int e = 0; e < 14; ++e)
        if (((lo >> (4 * e)) & 15u) == 1u) to = v + st.s[e];  // at most one edge field is 1
    next[v] = (int32_t)(in_grid(to, n) ? to : v);
}

__global__ __launch_bounds__(kThreads) void k_d0_jump(const int32_t *__restrict__ src,
                                                      int32_t *__restrict__ dst, int64_t n)
{
    const int64_t v = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (v >= n) return;
    const int32_t a = src[v];
    dst[v] = in_grid(a, n) ? src[a] : a;
}

__global__ __launch_bounds__(kThreads) void k_d0_fill(int32_t *__restrict__ p, int64_t n, int32_t value)
{
    const int64_t v = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (v < n) p[v] = value;
}

// minidx[v] = index of minimum v in crit0; min_order[i] = order of minimum i.
__global__ __launch_bounds__(kThreads) void k_d0_minima(const int64_t *__restrict__ crit0, int64_t n0,
                                                        const int32_t *__restrict__ order, int64_t n,
                                                        int32_t *__restrict__ minidx,
                                                        int32_t *__restrict__ min_order)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n0) return;
    const int64_t v = crit0[i] >> 8;
    if (!in_grid(v, n)) return;
    minidx[v] = (int32_t)i;
    min_order[i] = order[v];
}

__global__ __launch_bounds__(kThreads) void k_d0_trip(const int64_t *__restrict__ crit1, int64_t n1,
                                                      const int32_t *__restrict__ root,
                                                      const int32_t *__restrict__ minidx,
                                                      const int32_t *__restrict__ order, int64_t n,
                                                      Steps st, uint64_t *__restrict__ key,
                                                      int32_t *__restrict__ m0, int32_t *__restrict__ m1,
                                                      unsigned long long *ntri, uint32_t *flags)
{
    const int64_t s = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    bool valid = false;
    if (s < n1) {
        const int64_t a = crit1[s] >> 8;
        const int e = (int)(crit1[s] & 255);
        int32_t t0 = -1, t1 = -1;
        uint64_t k = ~0ull;
        if (e < 14 && in_grid(a, n) && in_grid(a + st.s[e], n)) {
            const int64_t b = a + st.s[e];
            const int32_t r0 = root[a], r1 = root[b];
            t0 = in_grid(r0, n) ? minidx[r0] : -1;
            t1 = in_grid(r1, n) ? minidx[r1] : -1;
            if (t0 < 0 || t1 < 0) {
                atomicOr(flags, (uint32_t)DMS_FLAG_CAPACITY);  // a minimum missing from crit0
            } else if (t0 != t1) {
                valid = true;
                k = ((uint64_t)(uint32_t)order[a] << 32) | (uint32_t)order[b];
            }
        } else {
            atomicOr(flags, (uint32_t)DMS_FLAG_CAPACITY);
        }
        key[s] = k;
        m0[s] = t0;
        m1[s] = t1;
    }
    const uint64_t b = __ballot(valid);
    if (lane_id() == 0 && b) atomicAdd(ntri, (unsigned long long)__popcll(b));
}

__global__ __launch_bounds__(kThreads) void k_d0_place(const int32_t *__restrict__ rank, int64_t n1,
                                                       const int64_t *__restrict__ crit1,
                                                       const int32_t *__restrict__ m0,
                                                       const int32_t *__restrict__ m1,
                                                       int64_t *__restrict__ tri_edge,
                                                       int32_t *__restrict__ tri_min0,
                                                       int32_t *__restrict__ tri_min1)
{
    const int64_t s = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (s >= n1) return;
    const int32_t r = rank[s];
    if (r < 0 || r >= n1) return;
    tri_edge[r] = crit1[s];
    tri_min0[r] = m0[s];
    tri_min1[r] = m1[s];
}

__global__ void k_d0_zero(unsigned long long *p) { *p = 0ull; }

struct D0Layout {
    size_t next, root, minidx, key, m0, m1, rank, count, rws, total;
};

D0Layout d0_layout(int64_t n, int64_t n1)
{
    D0Layout L{};
    size_t off = 0;
    L.next = off; off += align_up((size_t)n * 4, 256);
    L.root = off; off += align_up((size_t)n * 4, 256);
    L.minidx = off; off += align_up((size_t)n * 4, 256);
    L.key = off; off += align_up((size_t)(n1 > 0 ? n1 : 1) * 8, 256);
    L.m0 = off; off += align_up((size_t)(n1 > 0 ? n1 : 1) * 4, 256);
    L.m1 = off; off += align_up((size_t)(n1 > 0 ? n1 : 1) * 4, 256);
    L.rank = off; off += align_up((size_t)(n1 > 0 ? n1 : 1) * 4, 256);
    L.count = off; off += 256;  // the rank flags word
    L.rws = off; off += rank_u64_workspace_size(n1);
    L.total = off;
    return L;
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

}  // namespace
}  // namespace dms

extern "C" size_t dms_d0_workspace_size(const int64_t dims[3], int64_t n1)
{
    using namespace dms;
    if (!dims || dims[0] < 1 || dims[1] < 1 || dims[2] < 1 || n1 < 0 || !grid_size_ok(dims)) return 0;
    return d0_layout(dims[0] * dims[1] * dims[2], n1).total;
}

extern "C" int dms_d0_triplets(const uint32_t *rec, const int32_t *order, const int64_t dims[3],
                               const int64_t *crit0, int64_t n0, const int64_t *crit1, int64_t n1,
                               int64_t *tri_edge, int32_t *tri_min0, int32_t *tri_min1,
                               int32_t *min_order, int64_t *ntri, void *workspace,
                               size_t workspace_bytes, uint32_t *dev_flags, void *stream)
{
    using namespace dms;
    if (!dims || dims[0] < 1 || dims[1] < 1 || dims[2] < 1 || n0 < 0 || n1 < 0) return DMS_E_ARG;
    if (!grid_size_ok(dims)) return DMS_E_SIZE;
    if (!rec || !order || !ntri || !dev_flags) return DMS_E_ARG;
    if ((n0 > 0 && (!crit0 || !min_order)) || (n1 > 0 && (!crit1 || !tri_edge || !tri_min0 || !tri_min1)))
        return DMS_E_ARG;
    const int64_t n = dims[0] * dims[1] * dims[2];
    const D0Layout L = d0_layout(n, n1);
    if (!workspace || workspace_bytes < L.total) return DMS_E_WORKSPACE;
    if (const int dc = device_check()) return dc;
    hipStream_t s = (hipStream_t)stream;
    char *ws = (char *)workspace;
    int32_t *next = (int32_t *)(ws + L.next), *root = (int32_t *)(ws + L.root);
    int32_t *minidx = (int32_t *)(ws + L.minidx);
    uint64_t *key = (uint64_t *)(ws + L.key);
    int32_t *m0 = (int32_t *)(ws + L.m0), *m1 = (int32_t *)(ws + L.m1), *rank = (int32_t *)(ws + L.rank);
    unsigned long long *count = (unsigned long long *)ntri;  // counted in place
    uint32_t *rflags = (uint32_t *)(ws + L.count);

    Steps st;
    const Tables &T = kTables;
    for (int e = 0; e < 14; ++e) st.s[e] = T.nb[e][0] + dims[0] * (T.nb[e][1] + dims[1] * T.nb[e][2]);

    hipLaunchKernelGGL(k_d0_zero, dim3(1), dim3(1), 0, s, count);
    hipLaunchKernelGGL(k_d0_next, dim3(blocks_for(n)), dim3(kThreads), 0, s, (const uint4 *)rec, n, st, next);
    // pointer doubling: after j rounds every vertex points 2^j steps down its
    // path (or at its minimum); paths are shorter than n
    int32_t *a = next, *b = root;
    for (int64_t reach = 1; reach < n; reach <<= 1) {
        hipLaunchKernelGGL(k_d0_jump, dim3(blocks_for(n)), dim3(kThreads), 0, s, a, b, n);
        int32_t *t = a;
        a = b;
        b = t;
    }
    const int32_t *roots = a;
    hipLaunchKernelGGL(k_d0_fill, dim3(blocks_for(n)), dim3(kThreads), 0, s, minidx, n, -1);
    if (n0 > 0)
        hipLaunchKernelGGL(k_d0_minima, dim3(blocks_for(n0)), dim3(kThreads), 0, s, crit0, n0, order, n,
                           minidx, min_order);
    if (n1 > 0) {
        hipLaunchKernelGGL(k_d0_trip, dim3(blocks_for(n1)), dim3(kThreads), 0, s, crit1, n1, roots, minidx,
                           order, n, st, key, m0, m1, count, dev_flags);
        const int st2 = launch_rank_u64(key, n1, rank, ws + L.rws, rflags, s);
        if (st2) return st2;
        hipLaunchKernelGGL(k_d0_place, dim3(blocks_for(n1)), dim3(kThreads), 0, s, rank, n1, crit1, m0, m1,
                           tri_edge, tri_min0, tri_min1);
    }
    return launch_status();
}
