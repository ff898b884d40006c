// dms_d0_host.cpp -- host D0 pairing of the differentiable form (Section 2.6
// and Algorithm 1, PairExtremaSaddles), run on the CPU after the GPU
// gradient, the split the paper suggests for CPU+GPU nodes (Section 7).
//
// Extremum graph: from both vertices of every critical edge, follow the
// vertex-edge vectors of the gradient down to a minimum (a vertex whose
// record pairs it with nothing).  Triplets (edge, t0, t1) with t0 != t1 are
// visited by increasing edge (Section 2.1 comparison: the edge's two vertex
// orders, higher first); each joins the components of t0 and t1, and the
// younger representative (higher order) dies at the edge.  Descents are
// memoised per vertex.
#include <algorithm>
#include <cstdint>
#include <vector>

#include "dms.h"
#include "dms_tables.hpp"

namespace {

struct Triplet {
    int32_t k0, k1;  // orders of the higher and lower vertex of the edge
    int64_t edge, t0, t1;
};

}  // namespace

extern "C" int dms_d0_pairs_host(const uint32_t *rec, const int32_t *order, const int64_t dims[3],
                                 const int64_t *crit1, int64_t n1, int64_t *pair_edge,
                                 int64_t *pair_min, int64_t capacity, int64_t *npairs)
{
    if (!rec || !order || !dims || !npairs || n1 < 0 || capacity < 0) return DMS_E_ARG;
    if (n1 > 0 && !crit1) return DMS_E_ARG;
    if (capacity > 0 && (!pair_edge || !pair_min)) return DMS_E_ARG;
    const int64_t nx = dims[0], ny = dims[1], nz = dims[2];
    if (nx < 1 || ny < 1 || nz < 1) return DMS_E_ARG;
    const int64_t n = nx * ny * nz;
    const dms::Tables &T = dms::kTables;
    int64_t step[14];
    for (int e = 0; e < 14; ++e) step[e] = T.nb[e][0] + nx * (T.nb[e][1] + ny * T.nb[e][2]);

    // memoised descent: target[v] = minimum reached from v, -1 = not yet known
    std::vector<int64_t> target(n, -1);
    std::vector<int64_t> path;
    auto descend = [&](int64_t v) -> int64_t {
        path.clear();
        while (target[v] < 0) {
            const uint32_t *w = rec + 4 * v;
            const uint64_t lo = (uint64_t)w[0] | ((uint64_t)w[1] << 32);
            int delta = -1;
            for (int e = 0; e < 14; ++e)
                if (((lo >> (4 * e)) & 15u) == 1u) { delta = e; break; }
            if (delta < 0) { target[v] = v; break; }
            path.push_back(v);
            v += step[delta];
        }
        const int64_t t = target[v];
        for (int64_t u : path) target[u] = t;
        return t;
    };

    std::vector<Triplet> trip;
    trip.reserve((size_t)n1);
    for (int64_t s = 0; s < n1; ++s) {
        const int64_t a = crit1[s] >> 8;
        const int e = (int)(crit1[s] & 255);
        if (a < 0 || a >= n || e >= 14) return DMS_E_ARG;
        const int64_t b = a + step[e];
        if (b < 0 || b >= n) return DMS_E_ARG;
        const int64_t t0 = descend(a), t1 = descend(b);
        if (t0 != t1) trip.push_back({order[a], order[b], crit1[s], t0, t1});
    }
    std::sort(trip.begin(), trip.end(), [](const Triplet &x, const Triplet &y) {
        return x.k0 != y.k0 ? x.k0 < y.k0 : x.k1 < y.k1;
    });
    std::vector<int64_t> rep(n);
    for (int64_t v = 0; v < n; ++v) rep[v] = v;
    auto find = [&](int64_t v) {
        while (rep[v] != v) v = rep[v];
        return v;
    };
    int64_t np = 0;
    for (const Triplet &tr : trip) {
        int64_t r0 = find(tr.t0), r1 = find(tr.t1);
        if (r0 == r1) continue;
        if (order[r0] < order[r1]) std::swap(r0, r1);
        if (np < capacity) {
            pair_edge[np] = tr.edge;
            pair_min[np] = r0;
        }
        ++np;
        rep[r0] = r1;
        rep[tr.t0] = r1;
    }
    *npairs = np;
    return np > capacity ? DMS_E_WORKSPACE : DMS_OK;
}

// Algorithm 1 on triplets already in increasing edge order (dms_d0_triplets):
// minima are indices 0..n0-1 of the critical-vertex list, min_order their
// orders.  pair_min receives minimum indices.
extern "C" int dms_d0_pairs_sorted_host(const int64_t *tri_edge, const int32_t *tri_min0,
                                        const int32_t *tri_min1, int64_t ntri, const int32_t *min_order,
                                        int64_t n0, int64_t *pair_edge, int32_t *pair_min,
                                        int64_t capacity, int64_t *npairs)
{
    if (!npairs || ntri < 0 || n0 < 0 || capacity < 0) return DMS_E_ARG;
    if (ntri > 0 && (!tri_edge || !tri_min0 || !tri_min1)) return DMS_E_ARG;
    if (n0 > 0 && !min_order) return DMS_E_ARG;
    if (capacity > 0 && (!pair_edge || !pair_min)) return DMS_E_ARG;
    std::vector<int32_t> rep((size_t)n0);
    for (int64_t i = 0; i < n0; ++i) rep[(size_t)i] = (int32_t)i;
    auto find = [&](int32_t v) {
        while (rep[(size_t)v] != v) v = rep[(size_t)v];
        return v;
    };
    int64_t np = 0;
    for (int64_t j = 0; j < ntri; ++j) {
        const int32_t t0 = tri_min0[j], t1 = tri_min1[j];
        if (t0 < 0 || t1 < 0 || t0 >= n0 || t1 >= n0) return DMS_E_ARG;
        int32_t r0 = find(t0), r1 = find(t1);
        if (r0 == r1) continue;
        if (min_order[r0] < min_order[r1]) std::swap(r0, r1);
        if (np < capacity) {
            pair_edge[np] = tri_edge[j];
            pair_min[np] = r0;
        }
        ++np;
        rep[(size_t)r0] = r1;
        rep[(size_t)t0] = r1;
    }
    *npairs = np;
    return np > capacity ? DMS_E_WORKSPACE : DMS_OK;
}


// The dual of Algorithm 1 for D2, over the triplets of dms_d2_triplets in
// decreasing triangle order: each triplet joins the classes of its maxima;
// the lower representative (smaller filtration rank; the outside node, index
// n3, is above every tet) dies at the triangle.
extern "C" int dms_d2_pairs_sorted_host(const int64_t *tri_code, const int32_t *tri_max0,
                                        const int32_t *tri_max1, int64_t ntri, const int32_t *max_rank,
                                        int64_t n3, int64_t *pair_tri, int32_t *pair_max, int64_t capacity,
                                        int64_t *npairs)
{
    if (!npairs || ntri < 0 || n3 < 0 || capacity < 0) return DMS_E_ARG;
    if (ntri > 0 && (!tri_code || !tri_max0 || !tri_max1)) return DMS_E_ARG;
    if (n3 > 0 && !max_rank) return DMS_E_ARG;
    if (capacity > 0 && (!pair_tri || !pair_max)) return DMS_E_ARG;
    std::vector<int64_t> rep((size_t)n3 + 1);
    for (int64_t i = 0; i <= n3; ++i) rep[(size_t)i] = i;
    auto find = [&](int64_t a) {
        while (rep[(size_t)a] != a) a = rep[(size_t)a];
        return a;
    };
    auto lower = [&](int64_t a, int64_t b) {  // a below b
        if (a == n3) return false;
        if (b == n3) return true;
        return max_rank[a] < max_rank[b];
    };
    int64_t np = 0;
    for (int64_t s = 0; s < ntri; ++s) {
        const int64_t t0 = tri_max0[s], t1 = tri_max1[s];
        if (t0 < 0 || t0 > n3 || t1 < 0 || t1 > n3) return DMS_E_ARG;
        int64_t r0 = find(t0), r1 = find(t1);
        if (r0 == r1) continue;
        if (lower(r1, r0)) std::swap(r0, r1);
        if (np < capacity) {
            pair_tri[np] = tri_code[s];
            pair_max[np] = (int32_t)r0;
        }
        ++np;
        rep[(size_t)r0] = r1;
        rep[(size_t)t0] = r1;
    }
    *npairs = np;
    return np > capacity ? DMS_E_WORKSPACE : DMS_OK;
}
