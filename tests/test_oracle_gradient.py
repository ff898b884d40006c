"""Pins of the oracle's ProcessLowerStars and critical extraction against what
the paper and the mathematics fix (Sections 2.1, 2.3, 2.5, 2.6)."""
import json
import os

import numpy as np
import pytest

import brute
import oracle
from paper_2505_21266_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _grid(dims, kind, seed):
    nx, ny, nz = dims
    rng = np.random.default_rng(seed)
    if kind == "noise":
        return rng.random((nz, ny, nx))
    if kind == "ties":  # four levels only: most comparisons are decided by id
        return rng.integers(0, 4, (nz, ny, nx)).astype(np.float32)
    if kind == "mixture":
        return inputs.mixture_field((nz, ny, nx), 6, rng, 1e-3, np.float64)
    raise ValueError(kind)


def _whole(values, dims):
    o = oracle.order(values)
    rec, counts, an = oracle.lower_stars(o, dims)
    assert an == 0
    return o.reshape(-1), rec, counts


SMALL = [((2, 2, 2), "noise", 1), ((3, 3, 3), "noise", 2), ((4, 3, 5), "noise", 3),
         ((5, 5, 5), "ties", 4), ((6, 5, 4), "mixture", 5), ((8, 8, 8), "noise", 6),
         ((8, 7, 6), "ties", 7), ((8, 8, 8), "mixture", 8)]


@pytest.mark.parametrize("dims,kind,seed", SMALL)
def test_matching_and_acyclic(dims, kind, seed, tables):
    """Discrete vectors are facet-cofacet pairs inside one lower star, each
    simplex is in at most one, the critical cells are exactly the unpaired
    ones, and no v-path closes a loop (Section 2.3)."""
    o, rec, counts = _whole(_grid(dims, kind, seed), dims)
    simp = brute.kuhn_simplices(dims)
    pairs = brute.gradient_pairs(rec, dims, tables)
    unpaired = brute.check_matching(pairs, simp, o)
    assert brute.critical_by_dim(unpaired) == counts.tolist()
    crit, cnt = oracle.critical_simplices(rec, dims)
    assert (cnt == counts).all()
    assert brute.is_acyclic(pairs, simp)
    # the listed codes name exactly the unpaired simplices
    nb = tables["nb"]
    listed = set()
    for d in range(4):
        for code in crit[d]:
            x, idx = int(code) >> 8, int(code) & 255
            i, j, k = x % dims[0], (x // dims[0]) % dims[1], x // (dims[0] * dims[1])
            if d == 0:
                offs = []
            elif d == 1:
                offs = [idx]
            elif d == 2:
                offs = list(tables["tri"][idx])
            else:
                offs = list(tables["tet"][idx])
            s = [x] + [brute.vid(dims, i + nb[e][0], j + nb[e][1], k + nb[e][2]) for e in offs]
            listed.add(tuple(sorted(s)))
        assert list(crit[d]) == sorted(crit[d])
    assert listed == unpaired


@pytest.mark.parametrize("dims,kind,seed", SMALL + [((16, 16, 16), "noise", 9),
                                                     ((20, 9, 13), "mixture", 10)])
def test_euler_characteristic(dims, kind, seed):
    _, _, c = _whole(_grid(dims, kind, seed), dims)
    assert c[0] - c[1] + c[2] - c[3] == 1


@pytest.mark.parametrize("direction", [(1, 2, 4), (1, 1, 1), (3, -1, 2), (0, 0, 1), (-1, 0, 0),
                                       (1e-9, 1e-9, 1e-9)])
def test_ramp_single_minimum(direction):
    """Elevation case (Section 6.1): a linear field, ties broken by id, has a
    single critical cell, the global minimum."""
    dims = (9, 7, 8)
    v = inputs.ramp(dims[::-1], direction)
    o, rec, c = _whole(v, dims)
    assert c.tolist() == [1, 0, 0, 0]
    crit, _ = oracle.critical_simplices(rec, dims)
    assert int(crit[0][0]) >> 8 == int(np.argmin(o))


def test_separated_gaussians_k_maxima():
    """k positive Gaussians, 8 sigma apart and 4 sigma from the faces, give
    exactly k maxima (critical tets)."""
    n = 40
    rng = np.random.default_rng(11)
    centres = [(a, b, c) for a in (10, 30) for b in (10, 30) for c in (10, 30)]
    k_, j_, i_ = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    f = np.zeros((n, n, n))
    for (cx, cy, cz) in centres:
        cx, cy, cz = cx + rng.uniform(-0.5, 0.5), cy + rng.uniform(-0.5, 0.5), cz + rng.uniform(-0.5, 0.5)
        a = rng.uniform(0.5, 1.0)
        f += a * np.exp(-((i_ - cx) ** 2 + (j_ - cy) ** 2 + (k_ - cz) ** 2) / (2 * 2.5 ** 2))
    _, _, c = _whole(f, (n, n, n))
    assert c[3] == len(centres)
    assert c[0] - c[1] + c[2] - c[3] == 1


@pytest.mark.parametrize("dims,kind,seed", [((12, 12, 12), "noise", 12), ((10, 12, 9), "ties", 13),
                                            ((14, 10, 12), "mixture", 14)])
def test_lower_link_betti(dims, kind, seed, tables):
    """Robins' guarantee up to 3D (Sections 2.3, 6.6): the number of critical
    k-cells in L(x) equals the reduced Betti number b~_{k-1} of the lower link."""
    v = _grid(dims, kind, seed)
    o, rec, _ = _whole(v, dims)
    nx, ny, nz = dims
    for x in range(rec.shape[0]):
        i, j, k = x % nx, (x // nx) % ny, x // (nx * ny)
        st = oracle.decode_record(rec[x])
        got = (int(st[0] == oracle.ST_CRIT), int((st[1:15] == oracle.ST_CRIT).sum()),
               int((st[15:51] == oracle.ST_CRIT).sum()), int((st[51:75] == oracle.ST_CRIT).sum()))
        assert got == brute.lower_link_betti(o, dims, tables, i, j, k), (x, got)


@pytest.mark.parametrize("dims,kind,seed", [((6, 6, 6), "noise", 15), ((7, 5, 6), "ties", 16),
                                            ((8, 8, 8), "mixture", 17)])
def test_vertex_edge_pairs_are_union_find_zero_persistence(dims, kind, seed, tables):
    """Textbook D0 by union-find over edges in filtration order: a vertex joins
    the complex through its smallest lower edge with zero persistence; those
    merges are exactly the gradient's vertex-edge pairs."""
    o, rec, _ = _whole(_grid(dims, kind, seed), dims)
    simp = brute.kuhn_simplices(dims)
    merges = brute.union_find_d0(o, simp)
    zero = {((young,), e) for e, young in merges if brute.maxv(o, e) == young}
    pairs = brute.gradient_pairs(rec, dims, tables)
    ve = {(t, h) for t, h in pairs if len(t) == 1}
    assert ve == zero


@pytest.mark.parametrize("dims,kind,seed", [((3, 3, 3), "noise", 18), ((4, 4, 4), "noise", 19),
                                            ((5, 4, 3), "ties", 20), ((5, 5, 5), "mixture", 21),
                                            ((4, 5, 5), "noise", 22)])
def test_gradient_pairs_are_zero_persistence_pairs(dims, kind, seed, tables):
    """Zero-persistence skip (Section 2.6), checked by mod-2 boundary-matrix
    reduction of the lexicographic filtration on tiny grids: the simplices the
    gradient pairs are exactly those in persistence pairs whose two simplices
    share their max vertex (zero persistence), and the critical simplices are
    exactly those of the non-zero and infinite pairs.  Finding: inside one
    lower star the gradient may match these simplices with different partners
    than the simplex-wise reduction does (both pairings have zero persistence),
    so partner identity is not pinned here."""
    o, rec, _ = _whole(_grid(dims, kind, seed), dims)
    simp = brute.kuhn_simplices(dims)
    ppairs, essential = brute.persistence_pairs(o, simp)
    zero = {(b, d) for b, d in ppairs if brute.maxv(o, b) == brute.maxv(o, d)}
    grad = set(brute.gradient_pairs(rec, dims, tables))
    assert len(grad) == len(zero)
    assert {s for p in grad for s in p} == {s for p in zero for s in p}
    for t, h in grad:
        assert brute.maxv(o, t) == brute.maxv(o, h)
    crit = set().union(*simp) - {s for p in grad for s in p}
    nonzero = {s for b, d in ppairs if (b, d) not in zero for s in (b, d)}
    assert crit == nonzero | essential
    # per dimension, the zero-persistence pairs and the gradient pairs agree
    # in number (the matching differs only by swaps inside lower stars)
    for dim in (1, 2, 3):
        assert sum(len(t) == dim for t, _ in grad) == sum(len(b) == dim for b, _ in zero)


def test_hand_worked_cube(tables):
    """Hand-derived lower stars of one cube (tests/golden/cube2_hand.md)."""
    with open(os.path.join(GOLDEN, "cube2_hand.json")) as fh:
        g = json.load(fh)
    dims = tuple(g["dims"])
    o = np.array(g["order"], np.int32)
    rec, counts, an = oracle.lower_stars(o, dims)
    assert an == 0
    pairs = {(tuple(t), tuple(h)) for t, h in brute.gradient_pairs(rec, dims, tables)}
    assert pairs == {(tuple(t), tuple(h)) for t, h in g["pairs"]}
    simp = brute.kuhn_simplices(dims)
    crit = set().union(*simp) - {s for p in pairs for s in p}
    assert crit == {tuple(c) for c in g["critical"]}
    crit_codes, _ = oracle.critical_simplices(rec, dims)
    pe, pm = oracle.d0_pairs(o, rec, dims, crit_codes[1])
    got = []
    nb = tables["nb"]
    for code, m in zip(pe, pm):
        x, e = int(code) >> 8, int(code) & 255
        i, j, k = x % 2, (x // 2) % 2, x // 4
        y = brute.vid(dims, i + nb[e][0], j + nb[e][1], k + nb[e][2])
        got.append([sorted([x, y]), int(m)])
    assert got == g["d0_pairs"]


@pytest.mark.parametrize("kind,seed", [("noise", 23), ("ties", 24), ("mixture", 25)])
def test_literal_reading_agrees(kind, seed):
    """Robins' steps with pushes that ignore the cell's own state never pair a
    cell twice, so they give the same records as the free-only reading."""
    dims = (24, 20, 22)
    v = _grid(dims, kind, seed)
    o = oracle.order(v)
    r0, c0, a0 = oracle.lower_stars(o, dims, literal=False)
    r1, c1, a1 = oracle.lower_stars(o, dims, literal=True)
    assert a0 == 0 and a1 == 0
    assert (r0 == r1).all() and (c0 == c1).all()


def test_sampled_matches_whole_grid():
    """Per-vertex records from (value, id) comparisons equal the records from
    the global order (the lower star only sees relative order)."""
    dims = (17, 13, 11)
    v = _grid(dims, "ties", 26)
    o = oracle.order(v)
    rec, _, _ = oracle.lower_stars(o, dims)
    vids = np.arange(rec.shape[0])
    rs = oracle.lower_stars_sampled(v, dims, vids)
    assert (rs == rec).all()


def test_ghost_box_equals_restriction():
    """Processing only an owned box of a ghosted block (Section 2.2) reproduces
    the whole-grid records of that box."""
    dims = (14, 12, 10)
    v = _grid(dims, "noise", 27)
    o = oracle.order(v)
    rec, _, _ = oracle.lower_stars(o, dims)
    lo, hi = (1, 2, 1), (13, 11, 9)
    rb, _, _ = oracle.lower_stars(o, dims, lo, hi)
    full = rec.reshape(dims[2], dims[1], dims[0], 4)
    assert (rb == full[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]].reshape(-1, 4)).all()
    # a block's local order gives the same records as the global one
    sub = v[lo[2] - 1:hi[2] + 1, lo[1] - 1:hi[1] + 1, lo[0] - 1:hi[0] + 1]
    so = oracle.order(np.ascontiguousarray(sub))
    sd = (sub.shape[2], sub.shape[1], sub.shape[0])
    rs, _, _ = oracle.lower_stars(so, sd, (1, 1, 1), (sd[0] - 1, sd[1] - 1, sd[2] - 1))
    assert (rs == rb).all()


@pytest.mark.parametrize("dims", [(1, 1, 1), (7, 1, 1), (1, 6, 1), (1, 1, 5), (5, 4, 1), (1, 4, 5),
                                  (6, 1, 3)])
def test_degenerate_grids(dims):
    """Grids with a side of one vertex are lower-dimensional triangulations;
    the Euler characteristic is still 1, and a path graph has c1 = c0 - 1."""
    nx, ny, nz = dims
    v = np.random.default_rng(28).random((nz, ny, nx))
    _, rec, c = _whole(v, dims)
    assert c[0] - c[1] + c[2] - c[3] == 1
    if sorted(dims)[:2] == [1, 1]:
        f = v.reshape(-1)
        n = f.size
        mins = sum(1 for a in range(n)
                   if (a == 0 or f[a - 1] > f[a]) and (a == n - 1 or f[a + 1] > f[a]))
        assert c[0] == mins and c[1] == mins - 1


def test_min_count_plain_definition():
    """c0 = number of vertices without a lower neighbour, counted directly."""
    dims = (16, 15, 14)
    v = _grid(dims, "ties", 29)
    o, rec, c = _whole(v, dims)
    nx, ny, nz = dims
    t = oracle.star_tables()
    oo = o.reshape(nz, ny, nx)
    mins = 0
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                low = False
                for dx, dy, dz in t["nb"]:
                    a, b, cc = i + dx, j + dy, k + dz
                    if 0 <= a < nx and 0 <= b < ny and 0 <= cc < nz and oo[cc, b, a] < oo[k, j, i]:
                        low = True
                        break
                mins += not low
    assert c[0] == mins


@pytest.mark.parametrize("dims,lo,hi", [((40, 31, 22), None, None), ((34, 34, 9), (1, 1, 1), (33, 33, 8))])
def test_threaded_extraction_equals_one_thread(dims, lo, hi):
    """The row-parallel extraction lists exactly what the single-thread walk
    over the box lists, in the same (vertex id, local index) order, and
    respects the capacities."""
    nx, ny, nz = dims
    v = np.random.default_rng(7).random((nz, ny, nx)).astype(np.float32)
    o = oracle.order(v)
    rec, _, _ = oracle.lower_stars(o, dims, lo, hi)
    one, c1 = oracle.critical_simplices(rec, dims, lo, hi, nthreads=1)
    many, c8 = oracle.critical_simplices(rec, dims, lo, hi, nthreads=8)
    assert (c1 == c8).all()
    for d in range(4):
        assert (one[d] == many[d]).all()
        assert (np.diff(one[d]) > 0).all()
    cap = [max(int(c) // 3, 1) for c in c1]
    part, _ = oracle.critical_simplices(rec, dims, lo, hi, cap=cap, nthreads=8)
    for d in range(4):
        assert (part[d] == one[d][: cap[d]]).all()


def test_pls_batch_equals_pls_local():
    """The batched explicit-key call processes each row exactly as the
    single-star call does (random keys, some neighbours absent)."""
    rng = np.random.default_rng(11)
    m = 400
    keys = np.stack([rng.permutation(15) for _ in range(m)]).astype(np.uint8)
    keys[rng.random((m, 15)) < 0.1] = 255
    keys[:, 0] = np.where(keys[:, 0] == 255, 7, keys[:, 0])
    got = oracle.pls_batch(keys, nthreads=4)
    for r in range(m):
        k = [(-1 if x == 255 else int(x)) for x in keys[r]]
        _, want, an = oracle.pls_local(k)
        assert an == 0
        assert (got[r] == want).all(), r


@pytest.mark.parametrize("case", ["full14", "lower11"])
def test_hand_worked_star(tables, case):
    """Hand-derived ProcessLowerStars of an interior vertex with all 14
    neighbours lower (24 tets) and with 11 lower (an annulus lower link)
    (tests/golden/star_hand.md): the oracle's record of x decodes to exactly
    the hand-derived pairs and critical cells."""
    with open(os.path.join(GOLDEN, "star_hand.json")) as fh:
        g = json.load(fh)
    c = [x for x in g["cases"] if x["name"] == case][0]
    rank = g["rank_of_neighbour"]
    o = brute.hand_star_grid(rank, c["upper_ranks"], tables)
    rec, _, an = oracle.lower_stars(o, (3, 3, 3), (1, 1, 1), (2, 2, 2))
    assert an == 0
    pairs, crit = brute.record_rank_cells(rec[0], rank, tables)
    want = {(tuple(t), tuple(h)) for t, h in c["pairs"]}
    assert pairs == want
    assert crit == {tuple(x) for x in c["critical"]}
