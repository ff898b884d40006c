// dms_tables.hpp -- compile-time star tables of the Freudenthal (Kuhn)
// triangulation of a 3D grid, for the GPU library.
//
// Section 2.1 of the paper triangulates a regular grid with the Freudenthal
// triangulation without fixing the diagonal; this library uses the Kuhn
// triangulation along +(1,1,1): the unit cube with lowest corner c is split
// into the six tetrahedra {c, c+e_p0, c+e_p0+e_p1, c+(1,1,1)}, one per
// permutation p of the axes.  The star of a vertex is built here from the
// tetrahedra of the eight cubes that touch it:
//   * neighbours: the vertices of those star tetrahedra other than the centre,
//     numbered by (dz, dy, dx), i.e. by linear memory offset;
//   * star triangles: neighbour pairs {a < b} that share a star tetrahedron,
//     numbered lexicographically; star tetrahedra likewise by {a < b < c}.
// Everything is computed by constexpr code at compile time.
#pragma once
#include <cstdint>

namespace dms {

struct Tables {
    int nb[14][3];          // (dx, dy, dz) of neighbour e
    int ntri, ntet;
    int tri[36][2];         // star triangle {x, a, b}, a < b
    int tet[24][3];         // star tet {x, a, b, c}, a < b < c
    int tri_id[14][14];     // triangle of {a, b}, -1 if none
    int tet_id[14][14][14]; // tet of {a, b, c} (any order), -1 if none
    int edge_tris[14][6];   // star triangles containing edge e, ascending, -1 padded
    int edge_ntri[14];
    int tri_tets[36][2];    // the two star tets containing triangle t, ascending
    int tet_tris[24][3];    // triangles of tet q that contain x
    int tri_slot[36][2];    // slot of triangle t in edge_tris of tri[t][0] / tri[t][1]
    uint16_t link[14];      // neighbours joined to e by a star triangle
    uint64_t edge_trimask[14];
    uint16_t tri_edgemask[36];
    uint32_t tri_tetmask[36];
    uint64_t tet_trimask[24];
    uint32_t edge_tetmask[14];
};

namespace detail {

constexpr int lin(int dx, int dy, int dz) { return dx + 3 * (dy + 3 * dz); }  // within a 3x3x3 patch

constexpr Tables build()
{
    Tables T{};
    // 1. star tetrahedra as sets of patch cells (offset + 1 in each axis)
    int tets[64][4] = {};
    int nt = 0;
    const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    for (int cz = -1; cz <= 0; ++cz)
        for (int cy = -1; cy <= 0; ++cy)
            for (int cx = -1; cx <= 0; ++cx)
                for (int p = 0; p < 6; ++p) {
                    int c[3] = {cx, cy, cz};
                    int v[4] = {};
                    v[0] = lin(c[0] + 1, c[1] + 1, c[2] + 1);
                    for (int s = 0; s < 3; ++s) {
                        c[perms[p][s]] += 1;
                        v[s + 1] = lin(c[0] + 1, c[1] + 1, c[2] + 1);
                    }
                    const int centre = lin(1, 1, 1);
                    bool has = false;
                    for (int s = 0; s < 4; ++s) has = has || v[s] == centre;
                    if (!has) continue;
                    for (int s = 0; s < 4; ++s) tets[nt][s] = v[s];
                    ++nt;
                }
    // 2. neighbours: patch cells other than the centre that lie in a star tet
    bool used[27] = {};
    for (int q = 0; q < nt; ++q)
        for (int s = 0; s < 4; ++s) used[tets[q][s]] = true;
    used[lin(1, 1, 1)] = false;
    int nb_of_cell[27] = {};
    int ne = 0;
    for (int cell = 0; cell < 27; ++cell) {  // patch order is (dz, dy, dx) order
        nb_of_cell[cell] = -1;
        if (!used[cell]) continue;
        T.nb[ne][0] = cell % 3 - 1;
        T.nb[ne][1] = (cell / 3) % 3 - 1;
        T.nb[ne][2] = cell / 9 - 1;
        nb_of_cell[cell] = ne++;
    }
    // 3. tets as neighbour triples
    bool tetset[14][14][14] = {};
    for (int q = 0; q < nt; ++q) {
        int w[3] = {}, k = 0;
        for (int s = 0; s < 4; ++s)
            if (tets[q][s] != lin(1, 1, 1)) w[k++] = nb_of_cell[tets[q][s]];
        for (int a = 0; a < 3; ++a)
            for (int b = a + 1; b < 3; ++b)
                if (w[b] < w[a]) { int t = w[a]; w[a] = w[b]; w[b] = t; }
        tetset[w[0]][w[1]][w[2]] = true;
    }
    for (int a = 0; a < 14; ++a)
        for (int b = 0; b < 14; ++b) {
            T.tri_id[a][b] = -1;
            for (int c = 0; c < 14; ++c) T.tet_id[a][b][c] = -1;
        }
    T.ntet = 0;
    for (int a = 0; a < 14; ++a)
        for (int b = a + 1; b < 14; ++b)
            for (int c = b + 1; c < 14; ++c)
                if (tetset[a][b][c]) {
                    int q = T.ntet++;
                    T.tet[q][0] = a; T.tet[q][1] = b; T.tet[q][2] = c;
                    int w[3] = {a, b, c};
                    for (int i = 0; i < 3; ++i)
                        for (int j = 0; j < 3; ++j)
                            for (int k = 0; k < 3; ++k)
                                if (i != j && j != k && i != k) T.tet_id[w[i]][w[j]][w[k]] = q;
                }
    // 4. triangles: pairs inside some star tet
    T.ntri = 0;
    for (int a = 0; a < 14; ++a)
        for (int b = a + 1; b < 14; ++b) {
            bool in = false;
            for (int q = 0; q < T.ntet; ++q) {
                bool ha = false, hb = false;
                for (int s = 0; s < 3; ++s) { ha = ha || T.tet[q][s] == a; hb = hb || T.tet[q][s] == b; }
                in = in || (ha && hb);
            }
            if (!in) continue;
            int t = T.ntri++;
            T.tri[t][0] = a; T.tri[t][1] = b;
            T.tri_id[a][b] = T.tri_id[b][a] = t;
        }
    // 5. incidences
    for (int e = 0; e < 14; ++e) {
        T.edge_ntri[e] = 0;
        for (int s = 0; s < 6; ++s) T.edge_tris[e][s] = -1;
        T.link[e] = 0; T.edge_trimask[e] = 0; T.edge_tetmask[e] = 0;
    }
    for (int t = 0; t < T.ntri; ++t) {
        int a = T.tri[t][0], b = T.tri[t][1];
        T.tri_slot[t][0] = T.edge_ntri[a];
        T.edge_tris[a][T.edge_ntri[a]++] = t;
        T.tri_slot[t][1] = T.edge_ntri[b];
        T.edge_tris[b][T.edge_ntri[b]++] = t;
        T.link[a] |= uint16_t(1u << b);
        T.link[b] |= uint16_t(1u << a);
        T.edge_trimask[a] |= 1ull << t;
        T.edge_trimask[b] |= 1ull << t;
        T.tri_edgemask[t] = uint16_t((1u << a) | (1u << b));
        T.tri_tetmask[t] = 0;
    }
    int ntt[36] = {};
    for (int q = 0; q < T.ntet; ++q) {
        int a = T.tet[q][0], b = T.tet[q][1], c = T.tet[q][2];
        int f[3] = {T.tri_id[a][b], T.tri_id[a][c], T.tri_id[b][c]};
        T.tet_trimask[q] = 0;
        for (int s = 0; s < 3; ++s) {
            T.tet_tris[q][s] = f[s];
            T.tri_tets[f[s]][ntt[f[s]]++] = q;
            T.tri_tetmask[f[s]] |= 1u << q;
            T.tet_trimask[q] |= 1ull << f[s];
        }
        T.edge_tetmask[a] |= 1u << q;
        T.edge_tetmask[b] |= 1u << q;
        T.edge_tetmask[c] |= 1u << q;
    }
    return T;
}

}  // namespace detail

inline constexpr Tables kTables = detail::build();

static_assert(kTables.ntri == 36 && kTables.ntet == 24, "Kuhn star must have 36 triangles, 24 tets");
static_assert(kTables.nb[0][0] == -1 && kTables.nb[0][1] == -1 && kTables.nb[0][2] == -1, "numbering");
static_assert(kTables.nb[13][0] == 1 && kTables.nb[13][1] == 1 && kTables.nb[13][2] == 1, "numbering");

}  // namespace dms
