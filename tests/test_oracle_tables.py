"""Pins of the oracle's Kuhn star tables against the six-tets-per-cube
definition of the Freudenthal triangulation (Section 2.1 reading)."""
import itertools

import numpy as np
import pytest

import brute
import oracle


def test_counts(tables):
    assert tables["nb"].shape == (14, 3)
    assert len({tuple(r) for r in tables["nb"]}) == 14
    assert tables["tri"].shape == (36, 2) and tables["tet"].shape == (24, 3)
    # link of a vertex is a 2-sphere: chi = V - E + F = 2
    assert 14 - 36 + 24 == 2
    # every star triangle lies in exactly 2 star tets; edges in 4 or 6 triangles
    tt = tables["tri_tets"]
    assert all(tt[t][0] != tt[t][1] for t in range(36))
    deg = (tables["edge_tris"] >= 0).sum(axis=1)
    assert set(deg.tolist()) == {4, 6} and deg.sum() == 72


def test_neighbour_numbering_is_memory_order(tables):
    nb = tables["nb"]
    nx, ny = 7, 5
    lin = [int(dx + nx * (dy + ny * dz)) for dx, dy, dz in nb]
    assert lin == sorted(lin)
    # symmetric numbering: neighbour 13 - e is -neighbour e
    for e in range(14):
        assert (nb[13 - e] == -nb[e]).all()


def test_star_matches_cube_decomposition(tables):
    """The star of the centre of a 3x3x3 grid, rebuilt from the 6 Kuhn tets of
    each of its 8 cubes, equals the oracle's tables."""
    dims = (3, 3, 3)
    simp = brute.kuhn_simplices(dims)
    centre = brute.vid(dims, 1, 1, 1)

    def off(v):
        i, j, k = v % 3, (v // 3) % 3, v // 9
        return (i - 1, j - 1, k - 1)

    nb = [tuple(int(c) for c in r) for r in tables["nb"]]
    star = [set(), set(), set()]
    for d in (1, 2, 3):
        for s in simp[d]:
            if centre in s:
                star[d - 1].add(frozenset(off(v) for v in s if v != centre))
    assert star[0] == {frozenset([o]) for o in nb}
    assert star[1] == {frozenset([nb[a], nb[b]]) for a, b in tables["tri"]}
    assert star[2] == {frozenset([nb[a], nb[b], nb[c]]) for a, b, c in tables["tet"]}
    # incidence tables
    for e in range(14):
        tris = [t for t in range(36) if e in tables["tri"][t]]
        assert tables["edge_tris"][e][: len(tris)].tolist() == tris
    for t in range(36):
        a, b = tables["tri"][t]
        tets = [q for q in range(24) if a in tables["tet"][q] and b in tables["tet"][q]]
        assert sorted(tables["tri_tets"][t].tolist()) == tets


@pytest.mark.parametrize("n", [2, 3, 4, 6, 9])
def test_closed_form_counts(n):
    """Cubic grid of N = n + 1 vertices per side: E = 7n^3 + 9n^2 + 3n,
    F = 12n^3 + 6n^2, T = 6n^3, V - E + F - T = 1."""
    N = n + 1
    simp = brute.kuhn_simplices((N, N, N))
    V, E, F, T = (len(s) for s in simp)
    assert V == N ** 3
    assert E == 7 * n ** 3 + 9 * n ** 2 + 3 * n
    assert F == 12 * n ** 3 + 6 * n ** 2
    assert T == 6 * n ** 3
    assert V - E + F - T == 1


@pytest.mark.parametrize("dims", [(2, 2, 2), (3, 4, 5), (6, 5, 4), (5, 5, 5)])
def test_lower_stars_partition_the_complex(dims):
    """Every simplex has exactly one max vertex, so the lower stars partition
    the complex: summing L(x) sizes per dimension gives the simplex counts."""
    nx, ny, nz = dims
    v = np.random.default_rng(7).random((nz, ny, nx))
    o = oracle.order(v)
    rec, counts, an = oracle.lower_stars(o, dims)
    assert an == 0
    tot = [0, 0, 0, 0]
    for x in range(rec.shape[0]):
        st = oracle.decode_record(rec[x])
        tot[0] += 1
        tot[1] += int((st[1:15] != oracle.ST_OUT).sum())
        tot[2] += int((st[15:51] != oracle.ST_OUT).sum())
        tot[3] += int((st[51:75] != oracle.ST_OUT).sum())
    simp = brute.kuhn_simplices(dims)
    assert tot == [len(s) for s in simp]
