"""Pins of the oracle's D2 pairing (the dual of Algorithm 1 on the tets,
Section 2.6): equality with the (triangle, tet) pairs of non-zero
persistence of a mod-2 boundary-matrix reduction of the lexicographic
filtration, and every maximum paired (the grid is a ball)."""
import numpy as np
import pytest

import brute
import oracle
from paper_2505_21266_amd import inputs


def _field(dims, kind, seed):
    nx, ny, nz = dims
    rng = np.random.default_rng(seed)
    if kind == "noise":
        return rng.random((nz, ny, nx))
    if kind == "ties":
        return rng.integers(0, 4, (nz, ny, nx)).astype(np.float64)
    return inputs.mixture_field((nz, ny, nx), 4, rng, 1e-3, np.float64)


def _run(v, dims):
    o = oracle.order(v)
    rec, counts, an = oracle.lower_stars(o, dims)
    assert an == 0
    crit, _ = oracle.critical_simplices(rec, dims)
    pt, pq = oracle.d2_pairs(o, rec, dims, crit[2], crit[3])
    return o.reshape(-1), rec, counts, crit, pt, pq


def _verts(code, k, dims, T):
    nx, ny, _ = dims
    x, loc = int(code) >> 8, int(code) & 255
    i, j, kk = x % nx, (x // nx) % ny, x // (nx * ny)
    offs = [] if k == 1 else [loc] if k == 2 else list(T["tri"][loc]) if k == 3 else list(T["tet"][loc])
    vs = [x] + [brute.vid(dims, i + T["nb"][e][0], j + T["nb"][e][1], kk + T["nb"][e][2]) for e in offs]
    return tuple(sorted(vs))


@pytest.mark.parametrize("dims,kind,seed", [((3, 3, 3), "noise", 31), ((4, 4, 4), "noise", 32),
                                            ((5, 4, 3), "ties", 33), ((5, 5, 5), "mixture", 34),
                                            ((4, 5, 5), "noise", 35), ((6, 5, 4), "noise", 36)])
def test_d2_equals_boundary_reduction(dims, kind, seed, tables):
    o, rec, counts, crit, pt, pq = _run(_field(dims, kind, seed), dims)
    assert len(pt) == counts[3]  # every maximum dies
    simp = brute.kuhn_simplices(dims)
    ppairs, _ = brute.persistence_pairs(o, simp)
    want = {(b, d) for b, d in ppairs if len(b) == 3 and brute.maxv(o, b) != brute.maxv(o, d)}
    got = {(_verts(a, 3, dims, tables), _verts(b, 4, dims, tables)) for a, b in zip(pt, pq)}
    assert got == want


@pytest.mark.parametrize("dims,seed", [((10, 9, 8), 41), ((12, 12, 12), 42)])
def test_d2_invariants(dims, seed):
    """Larger grids (no brute force): every critical tet is paired once, with
    a critical triangle, and persistence is positive (the tet's highest
    vertex comes after the triangle's)."""
    o, rec, counts, crit, pt, pq = _run(_field(dims, "noise", seed), dims)
    assert len(pq) == counts[3] and sorted(pq.tolist()) == sorted(np.asarray(crit[3]).tolist())
    assert set(pt.tolist()) <= set(np.asarray(crit[2]).tolist()) and len(set(pt.tolist())) == len(pt)
    assert (o[pq >> 8] > o[pt >> 8]).all()


def test_d2_flat_grid_is_empty():
    dims = (7, 6, 1)
    o, rec, counts, crit, pt, pq = _run(_field(dims, "noise", 5), dims)
    assert counts[3] == 0 and len(pt) == 0
