"""Pins of the oracle's filtration sort (Section 2.1): a hand-worked cube,
the vertex case against numpy's argsort, and invariants on random fields."""
import json
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import oracle  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "filtration_cube2.json")


def _coords(v, dims):
    nx, ny, _ = dims
    return np.array([v % nx, (v // nx) % ny, v // (nx * ny)])


def code_of(cell, order, dims, T):
    """(maxv << 8) | local index of a cell given by its vertex ids, through
    the oracle's star tables."""
    cell = list(cell)
    m = max(cell, key=lambda u: order[u])
    es = []
    for u in cell:
        if u == m:
            continue
        d = _coords(u, dims) - _coords(m, dims)
        hit = [e for e in range(14) if (T["nb"][e] == d).all()]
        assert len(hit) == 1, (cell, u, d)
        es.append(hit[0])
    es.sort()
    if len(cell) == 1:
        loc = 0
    elif len(cell) == 2:
        loc = es[0]
    elif len(cell) == 3:
        loc = [t for t in range(36) if sorted(T["tri"][t]) == es][0]
    else:
        loc = [q for q in range(24) if sorted(T["tet"][q]) == es][0]
    return (m << 8) | loc


@pytest.mark.parametrize("name,dim", [("vertices", 0), ("edges", 1), ("triangles", 2), ("tets", 3)])
def test_hand_worked_cube(name, dim):
    g = json.load(open(GOLDEN))
    dims, order = tuple(g["dims"]), g["order"]
    T = oracle.star_tables()
    cells = g[name]["input"]
    want = g[name]["sorted"]
    if dim == 0:
        cells = [[c] for c in cells]
        want = [[c] for c in want]
    codes = [code_of(c, order, dims, T) for c in cells]
    got = oracle.filtration_sort(np.array(order, np.int32), dims, codes, dim)
    assert got.tolist() == [code_of(c, order, dims, T) for c in want]


def test_vertices_are_sorted_by_order():
    rng = np.random.default_rng(5)
    dims = (9, 7, 5)
    n = 9 * 7 * 5
    order = rng.permutation(n).astype(np.int32)
    ids = rng.permutation(n)[: n // 2]
    got = oracle.filtration_sort(order, dims, ids.astype(np.int64) << 8, 0)
    want = ids[np.argsort(order[ids], kind="stable")]
    assert ((got >> 8) == want).all() and ((got & 255) == 0).all()


@pytest.mark.parametrize("seed", [1, 2])
def test_invariants_on_a_field(seed):
    rng = np.random.default_rng(seed)
    dims = (10, 9, 8)
    v = rng.random((8, 9, 10), dtype=np.float32)
    o = oracle.order(v)
    rec, _, _ = oracle.lower_stars(o, dims)
    crit, _ = oracle.critical_simplices(rec, dims)
    flat = o.reshape(-1)
    for d in range(4):
        c = np.asarray(crit[d], np.int64)
        got = oracle.filtration_sort(o, dims, c[::-1], d)
        assert sorted(got.tolist()) == sorted(c.tolist())  # a permutation
        top = flat[got >> 8]
        assert (np.diff(top) >= 0).all()  # the highest vertex's order leads


def test_rejects_bad_codes():
    o = np.arange(8, dtype=np.int32)
    with pytest.raises(ValueError):
        oracle.filtration_sort(o, (2, 2, 2), [(0 << 8) | 40], 2)  # no star triangle 40
    with pytest.raises(ValueError):
        oracle.filtration_sort(o, (2, 2, 2), [(7 << 8) | 13], 1)  # neighbour outside the grid
