// dms_d0_host.cpp -- host pairings of the differentiable forms (Section 2.6:
// D0 by Algorithm 1, PairExtremaSaddles; D2 by its dual), run on the CPU after
// the GPU gradient, the split the paper suggests for CPU+GPU nodes (Section 7).
//
// Extremum graph: from both vertices of every critical edge, follow the
// vertex-edge vectors of the gradient down to a minimum (a vertex whose
// record pairs it with nothing).  The saddles are visited in filtration
// order (Section 2.1 comparison); each joins the classes of its two
// extrema, and by the elder rule the extremum born later of the two classes'
// eldest dies at the saddle.  Algorithm 1 keeps a class's eldest extremum as
// its representative; here a union-find with union by rank and path halving
// stores each class's eldest at its root instead, which gives the same
// pairs.  Descents are memoised per vertex.
#include <algorithm>
#include <cstdint>
#include <utility>
#include <vector>

#include "dms.h"
#include "dms_tables.hpp"

namespace {

struct Triplet {
    int32_t k0, k1;  // orders of the higher and lower vertex of the edge
    int64_t edge, t0, t1;
};

// Classes of extrema 0..n-1.  join(a, b) merges the classes of a and b and
// returns the eldest of the younger class (the extremum that dies), or -1
// when they are one class already.  older(x, y): x was born before y.
class ElderForest {
  public:
    explicit ElderForest(int64_t n) : parent_((size_t)n), rank_((size_t)n, 0), eldest_((size_t)n)
    {
        for (int64_t i = 0; i < n; ++i) parent_[(size_t)i] = eldest_[(size_t)i] = i;
    }

    int64_t root(int64_t a)
    {
        while (parent_[(size_t)a] != a) {
            parent_[(size_t)a] = parent_[(size_t)parent_[(size_t)a]];
            a = parent_[(size_t)a];
        }
        return a;
    }

    template <typename Older>
    int64_t join(int64_t a, int64_t b, Older older)
    {
        int64_t ra = root(a), rb = root(b);
        if (ra == rb) return -1;
        const int64_t ea = eldest_[(size_t)ra], eb = eldest_[(size_t)rb];
        const bool a_survives = older(ea, eb);
        if (rank_[(size_t)ra] < rank_[(size_t)rb]) std::swap(ra, rb);
        parent_[(size_t)rb] = ra;
        if (rank_[(size_t)ra] == rank_[(size_t)rb]) ++rank_[(size_t)ra];
        eldest_[(size_t)ra] = a_survives ? ea : eb;
        return a_survives ? eb : ea;
    }

  private:
    std::vector<int64_t> parent_;
    std::vector<uint8_t> rank_;
    std::vector<int64_t> eldest_;
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
    ElderForest minima(n);
    const auto older = [&](int64_t x, int64_t y) { return order[x] < order[y]; };
    int64_t np = 0;
    for (const Triplet &tr : trip) {
        const int64_t dies = minima.join(tr.t0, tr.t1, older);
        if (dies < 0) continue;
        if (np < capacity) {
            pair_edge[np] = tr.edge;
            pair_min[np] = dies;
        }
        ++np;
    }
    *npairs = np;
    return np > capacity ? DMS_E_WORKSPACE : DMS_OK;
}

// The same pairing on triplets already in increasing edge order
// (dms_d0_triplets): minima are indices 0..n0-1 of the critical-vertex list,
// min_order their orders.  pair_min receives minimum indices.
extern "C" int dms_d0_pairs_sorted_host(const int64_t *tri_edge, const int32_t *tri_min0,
                                        const int32_t *tri_min1, int64_t ntri, const int32_t *min_order,
                                        int64_t n0, int64_t *pair_edge, int32_t *pair_min,
                                        int64_t capacity, int64_t *npairs)
{
    if (!npairs || ntri < 0 || n0 < 0 || capacity < 0) return DMS_E_ARG;
    if (ntri > 0 && (!tri_edge || !tri_min0 || !tri_min1)) return DMS_E_ARG;
    if (n0 > 0 && !min_order) return DMS_E_ARG;
    if (capacity > 0 && (!pair_edge || !pair_min)) return DMS_E_ARG;
    ElderForest minima(n0);
    const auto older = [&](int64_t x, int64_t y) { return min_order[x] < min_order[y]; };
    int64_t np = 0;
    for (int64_t j = 0; j < ntri; ++j) {
        const int32_t t0 = tri_min0[j], t1 = tri_min1[j];
        if (t0 < 0 || t1 < 0 || t0 >= n0 || t1 >= n0) return DMS_E_ARG;
        const int64_t dies = minima.join(t0, t1, older);
        if (dies < 0) continue;
        if (np < capacity) {
            pair_edge[np] = tri_edge[j];
            pair_min[np] = (int32_t)dies;
        }
        ++np;
    }
    *npairs = np;
    return np > capacity ? DMS_E_WORKSPACE : DMS_OK;
}


// The dual pairing for D2, over the triplets of dms_d2_triplets in
// decreasing triangle order: each triplet joins the classes of its maxima;
// the lower of the two classes' highest maxima (smaller filtration rank; the
// outside node, index n3, is above every tet) dies at the triangle.
extern "C" int dms_d2_pairs_sorted_host(const int64_t *tri_code, const int32_t *tri_max0,
                                        const int32_t *tri_max1, int64_t ntri, const int32_t *max_rank,
                                        int64_t n3, int64_t *pair_tri, int32_t *pair_max, int64_t capacity,
                                        int64_t *npairs)
{
    if (!npairs || ntri < 0 || n3 < 0 || capacity < 0) return DMS_E_ARG;
    if (ntri > 0 && (!tri_code || !tri_max0 || !tri_max1)) return DMS_E_ARG;
    if (n3 > 0 && !max_rank) return DMS_E_ARG;
    if (capacity > 0 && (!pair_tri || !pair_max)) return DMS_E_ARG;
    // on the dual the sweep runs downwards: a maximum is born before another
    // when it is higher; the outside node (index n3) is above every tet
    ElderForest maxima(n3 + 1);
    const auto older = [&](int64_t a, int64_t b) {
        if (a == n3) return true;
        if (b == n3) return false;
        return max_rank[a] > max_rank[b];
    };
    int64_t np = 0;
    for (int64_t s = 0; s < ntri; ++s) {
        const int64_t t0 = tri_max0[s], t1 = tri_max1[s];
        if (t0 < 0 || t0 > n3 || t1 < 0 || t1 > n3) return DMS_E_ARG;
        const int64_t dies = maxima.join(t0, t1, older);
        if (dies < 0) continue;
        if (np < capacity) {
            pair_tri[np] = tri_code[s];
            pair_max[np] = (int32_t)dies;
        }
        ++np;
    }
    *npairs = np;
    return np > capacity ? DMS_E_WORKSPACE : DMS_OK;
}
