"""Brute-force checkers for small grids, written from textbook definitions.

Nothing here shares code with the oracle's C arithmetic: the triangulation is
rebuilt from the six-tetrahedra-per-cube (Kuhn) decomposition, simplices are
compared with Python list comparison (the lexicographic comparison of Section
2.1), and homology is computed by plain union-find and mod-2 column reduction.
"""
import itertools

import numpy as np


def vid(dims, i, j, k):
    nx, ny, _ = dims
    return i + nx * (j + ny * k)


def kuhn_simplices(dims):
    """All simplices of the Kuhn triangulation of a grid (every dim >= 2).

    Each unit cube is split into the 6 tetrahedra
    {v, v+e_p0, v+e_p0+e_p1, v+(1,1,1)} over permutations p of the axes.
    Returns [set of 1-tuples, 2-tuples, 3-tuples, 4-tuples] of sorted vertex ids.
    """
    nx, ny, nz = dims
    tets = set()
    for k in range(nz - 1):
        for j in range(ny - 1):
            for i in range(nx - 1):
                for p in itertools.permutations(range(3)):
                    c = [i, j, k]
                    vs = [vid(dims, *c)]
                    for axis in p:
                        c[axis] += 1
                        vs.append(vid(dims, *c))
                    tets.add(tuple(sorted(vs)))
    out = [set(), set(), set(), tets]
    for t in tets:
        for r in (1, 2, 3):
            for f in itertools.combinations(t, r):
                out[r - 1].add(f)
    return out


def key(order, s):
    """Section 2.1: vertex orders listed decreasingly; Python compares lists
    lexicographically with a proper prefix smaller."""
    return sorted((int(order[v]) for v in s), reverse=True)


def maxv(order, s):
    return max(s, key=lambda v: order[v])


def gradient_pairs(rec, dims, tables):
    """Decodes whole-grid records into discrete vectors (tail, head).

    Returns (pairs as a list of (tail tuple, head tuple), critical set of tuples
    derived as the in-lower-star cells that are in no pair).
    """
    nx, ny, nz = dims
    nb = tables["nb"]
    et = tables["edge_tris"]
    tri = tables["tri"]
    tt = tables["tri_tets"]
    tet = tables["tet"]

    def nbid(i, j, k, e):
        return vid(dims, i + nb[e][0], j + nb[e][1], k + nb[e][2])

    pairs = []
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                x = vid(dims, i, j, k)
                w = [int(a) for a in rec[x]]
                bits = w[0] | (w[1] << 32) | (w[2] << 64) | (w[3] << 96)
                for e in range(14):
                    f = (bits >> (4 * e)) & 15
                    if f == 0:
                        continue
                    edge = tuple(sorted((x, nbid(i, j, k, e))))
                    if f == 1:
                        pairs.append(((x,), edge))
                    elif f >= 3:
                        t = et[e][f - 3]
                        a, b = tri[t]
                        tri_s = tuple(sorted((x, nbid(i, j, k, a), nbid(i, j, k, b))))
                        pairs.append((edge, tri_s))
                for t in range(36):
                    g = (bits >> (56 + 2 * t)) & 3
                    if g:
                        a, b = tri[t]
                        tri_s = tuple(sorted((x, nbid(i, j, k, a), nbid(i, j, k, b))))
                        q = tt[t][g - 1]
                        a, b, c = tet[q]
                        tet_s = tuple(sorted((x, nbid(i, j, k, a), nbid(i, j, k, b), nbid(i, j, k, c))))
                        pairs.append((tri_s, tet_s))
    return pairs


def check_matching(pairs, simplices, order):
    """Each simplex in at most one pair, pairs are facet-cofacet with the same
    max vertex.  Returns the set of unpaired simplices."""
    seen = set()
    for tail, head in pairs:
        assert len(head) == len(tail) + 1 and set(tail) < set(head), (tail, head)
        assert maxv(order, tail) == maxv(order, head), (tail, head)
        assert tail not in seen and head not in seen, (tail, head)
        seen.add(tail)
        seen.add(head)
    allc = set().union(*simplices)
    assert seen <= allc
    return allc - seen


def is_acyclic(pairs, simplices):
    """Loop-free v-paths (Section 2.3): the Hasse diagram with every arc
    pointing from a simplex to its facets, except gradient pairs whose arc is
    reversed (tail -> head), must have no directed cycle (Kahn's algorithm)."""
    allc = sorted(set().union(*simplices), key=lambda s: (len(s), s))
    idx = {s: n for n, s in enumerate(allc)}
    pair_of = {t: h for t, h in pairs}
    adj = [[] for _ in allc]
    indeg = [0] * len(allc)
    for s in allc:
        if len(s) < 2:
            continue
        for f in itertools.combinations(s, len(s) - 1):
            if pair_of.get(f) == s:
                a, b = idx[f], idx[s]
            else:
                a, b = idx[s], idx[f]
            adj[a].append(b)
            indeg[b] += 1
    stack = [n for n in range(len(allc)) if indeg[n] == 0]
    done = 0
    while stack:
        n = stack.pop()
        done += 1
        for m in adj[n]:
            indeg[m] -= 1
            if indeg[m] == 0:
                stack.append(m)
    return done == len(allc)


def union_find_d0(order, simplices):
    """Textbook D0: edges in filtration order, union-find with the elder rule.

    Returns a list of (edge tuple, dying root vertex) for every merge.
    """
    parent = {}

    def find(v):
        while parent[v] != v:
            parent[v] = parent[parent[v]]
            v = parent[v]
        return v

    for (v,) in simplices[0]:
        parent[v] = v
    merges = []
    for e in sorted(simplices[1], key=lambda s: key(order, s)):
        a, b = find(e[0]), find(e[1])
        if a == b:
            continue
        young, old = (a, b) if order[a] > order[b] else (b, a)
        merges.append((e, young))
        parent[young] = old
    return merges


def persistence_pairs(order, simplices):
    """Mod-2 boundary-matrix column reduction of the lexicographic filtration.

    Returns (pairs as list of (birth tuple, death tuple), essential set)."""
    allc = sorted(set().union(*simplices), key=lambda s: key(order, s))
    idx = {s: n for n, s in enumerate(allc)}
    low_to_col = {}
    cols = {}
    pairs = []
    for j, s in enumerate(allc):
        col = 0
        if len(s) > 1:
            for f in itertools.combinations(s, len(s) - 1):
                col |= 1 << idx[f]
        while col:
            low = col.bit_length() - 1
            if low in low_to_col:
                col ^= cols[low_to_col[low]]
            else:
                low_to_col[low] = j
                cols[j] = col
                pairs.append((allc[low], s))
                break
    paired = set()
    for b, d in pairs:
        paired.add(b)
        paired.add(d)
    return pairs, set(allc) - paired


def lower_link_betti(order, dims, tables, i, j, k):
    """Reduced Betti numbers (b~_{-1}, b~_0, b~_1, b~_2) of the lower link of
    vertex (i, j, k), from the star tables: lower neighbours, the link edges
    among them (star triangles), the link triangles (star tets)."""
    nx, ny, nz = dims
    nb = tables["nb"]
    ox = order[vid(dims, i, j, k)]
    low = []
    for e in range(14):
        a, b, c = i + nb[e][0], j + nb[e][1], k + nb[e][2]
        low.append(0 <= a < nx and 0 <= b < ny and 0 <= c < nz and order[vid(dims, a, b, c)] < ox)
    V = [e for e in range(14) if low[e]]
    E = [tuple(t) for t in tables["tri"] if low[t[0]] and low[t[1]]]
    F = [tuple(q) for q in tables["tet"] if low[q[0]] and low[q[1]] and low[q[2]]]
    if not V:
        return (1, 0, 0, 0)
    parent = {v: v for v in V}

    def find(v):
        while parent[v] != v:
            v = parent[v]
        return v

    for a, b in E:
        ra, rb = find(a), find(b)
        if ra != rb:
            parent[ra] = rb
    b0 = len({find(v) for v in V})
    b2 = 1 if len(F) == 24 else 0
    chi = len(V) - len(E) + len(F)
    b1 = b0 + b2 - chi
    return (0, b0 - 1, b1, b2)


def critical_by_dim(critset):
    out = [0, 0, 0, 0]
    for s in critset:
        out[len(s) - 1] += 1
    return out


def hand_star_grid(rank_of_neighbour, upper_ranks, tables):
    """A 3x3x3 grid order whose centre x = vertex 13 has neighbour e at rank
    rank_of_neighbour[e] among x's neighbours: ranks in upper_ranks lie above
    x, the others below; the 12 vertices that are not neighbours come last."""
    nb = tables["nb"]
    order = np.full(27, -1, np.int64)
    upper = set(upper_ranks)
    for e in range(14):
        r = int(rank_of_neighbour[e])
        order[vid((3, 3, 3), 1 + nb[e][0], 1 + nb[e][1], 1 + nb[e][2])] = 100 + r if r in upper else r
    order[13] = 50
    spare = 200
    for v in range(27):
        if order[v] < 0:
            order[v] = spare
            spare += 1
    return order.astype(np.int32).reshape(3, 3, 3)


def record_rank_cells(rec4, rank_of_neighbour, tables):
    """Pairs and critical cells of one 128-bit record, each cell as the
    descending tuple of the ranks of its lower neighbours (x implicit, () is
    x).  Returns (set of (tail, head), set of critical cells)."""
    w = [int(a) for a in rec4]
    bits = w[0] | (w[1] << 32) | (w[2] << 64) | (w[3] << 96)
    r = [int(x) for x in rank_of_neighbour]
    et, tri, tt, tet = tables["edge_tris"], tables["tri"], tables["tri_tets"], tables["tet"]

    def cell(*es):
        return tuple(sorted((r[int(e)] for e in es), reverse=True))

    ef = [(bits >> (4 * e)) & 15 for e in range(14)]
    tf = [(bits >> (56 + 2 * t)) & 3 for t in range(36)]
    pairs, paired = set(), set()
    for e in range(14):
        if ef[e] == 1:
            pairs.add(((), cell(e)))
        elif ef[e] >= 3:
            pairs.add((cell(e), cell(*tri[et[e][ef[e] - 3]])))
    for t in range(36):
        if tf[t]:
            pairs.add((cell(*tri[t]), cell(*tet[tt[t][tf[t] - 1]])))
    for a, b in pairs:
        paired |= {a, b}
    inl = [e for e in range(14) if ef[e]]
    cells = {()} | {cell(e) for e in inl}
    cells |= {cell(a, b) for a, b in tri if ef[a] and ef[b]}
    cells |= {cell(a, b, c) for a, b, c in tet if ef[a] and ef[b] and ef[c]}
    return pairs, cells - paired
