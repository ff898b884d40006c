"""CPU oracle for the discrete-gradient step of Discrete Morse Sandwich.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
library (``paper_2505_21266_amd``) never imports it and shares no code with it.

The arithmetic lives in ``dms_oracle.c`` (plain C, built with gcc); this module
only marshals numpy arrays.  What each function computes, and the passage of
the paper it follows, is stated in the C file above the function.

Functions:
  star_tables()              Kuhn star tables (Section 2.1 reading)
  order(values)              global vertex order (Section 2.1, Section 3)
  lower_stars(order, dims)   Robins' ProcessLowerStars over a box -> records
  lower_stars_sampled(...)   the same at sampled vertices, from the values
  pls_local(okey)            one lower star from 15 explicit keys
  pls_batch(keys)            many lower stars from explicit keys
  decode_record(rec)         75 cell states of one record
  critical_simplices(...)    zero-persistence skip -> 4 code lists
  d0_pairs(...)              Algorithm 1 on the extremum graph
  d0_loss_grad(...)          loss of the differentiable form and its gradient
  filtration_sort(...)       critical cells of one dimension in filtration order
  d2_pairs(...)              the dual of Algorithm 1: 2-saddle / maximum pairs
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dms_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

# cell-state codes used by the C file
ST_OUT, ST_FREE, ST_TAIL, ST_HEAD, ST_CRIT = 0, 1, 2, 3, 4
# cell numbering inside one lower star
CELL_X, CELL_EDGE0, CELL_TRI0, CELL_TET0, NCELL = 0, 1, 15, 51, 75


def build(force=True):
    """Compiles the oracle with gcc (-O3, OpenMP over vertices)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O3", "-fopenmp", "-shared", "-fPIC", "-std=c99", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    I64 = ctypes.c_int64
    I = ctypes.c_int
    lib.oracle_star_tables.argtypes = [P, P, P, P, P]
    lib.oracle_order_f32.argtypes = [P, I64, P, I]
    lib.oracle_order_f64.argtypes = [P, I64, P, I]
    lib.oracle_pls_local.argtypes = [P, I, P, P, P]
    lib.oracle_lower_stars.argtypes = [P, P, P, P, P, P, I, I, P]
    lib.oracle_lower_stars_sampled.argtypes = [P, I, P, P, I64, P, I, P]
    lib.oracle_decode_record.argtypes = [P, P]
    lib.oracle_critical_simplices.argtypes = [P, P, P, P, P, P, P, P, P, P, I]
    lib.oracle_pls_batch.argtypes = [P, I64, P, I, P]
    lib.oracle_d0_pairs.argtypes = [P, P, P, P, I64, P, P, P]
    lib.oracle_filtration_sort.argtypes = [P, P, P, I64, I, P]
    lib.oracle_d2_pairs.argtypes = [P, P, P, P, I64, P, I64, P, P, P]
    for f in (lib.oracle_star_tables, lib.oracle_order_f32, lib.oracle_order_f64,
              lib.oracle_pls_local, lib.oracle_lower_stars, lib.oracle_lower_stars_sampled,
              lib.oracle_decode_record, lib.oracle_critical_simplices, lib.oracle_d0_pairs,
              lib.oracle_filtration_sort, lib.oracle_d2_pairs, lib.oracle_pls_batch):
        f.restype = ctypes.c_int
    _lib = lib
    return lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _i64(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.int64))


def star_tables():
    """Returns dict(nb[14,3] (dx,dy,dz), tri[36,2], tet[24,3], edge_tris[14,6], tri_tets[36,2])."""
    lib = _load()
    nb = np.zeros((14, 3), np.int32)
    tri = np.zeros((36, 2), np.int32)
    tet = np.zeros((24, 3), np.int32)
    et = np.zeros((14, 6), np.int32)
    tt = np.zeros((36, 2), np.int32)
    if lib.oracle_star_tables(_p(nb), _p(tri), _p(tet), _p(et), _p(tt)) != 0:
        raise RuntimeError("oracle star tables failed")
    return dict(nb=nb, tri=tri, tet=tet, edge_tris=et, tri_tets=tt)


def order(values, nthreads=1):
    """order[v] = position of v in the ascending (value, id) sort; int32, same shape.
    nthreads: threads of the sort (1 = one qsort; 0 = all, sorted runs merged)."""
    lib = _load()
    v = np.ascontiguousarray(values)
    out = np.empty(v.shape, np.int32)
    if v.dtype == np.float32:
        rc = lib.oracle_order_f32(_p(v), v.size, _p(out), int(nthreads))
    elif v.dtype == np.float64:
        rc = lib.oracle_order_f64(_p(v), v.size, _p(out), int(nthreads))
    else:
        raise TypeError("float32 or float64 expected")
    if rc == 1:
        raise ValueError("NaN in input")
    if rc != 0:
        raise RuntimeError("oracle order failed (%d)" % rc)
    return out


def _box(dims, lo, hi):
    dims = _i64(dims)
    lo = _i64([0, 0, 0] if lo is None else lo)
    hi = _i64(dims if hi is None else hi)
    return dims, lo, hi


def lower_stars(order_arr, dims, lo=None, hi=None, literal=False, nthreads=0):
    """ProcessLowerStars over box [lo, hi) of a grid of dims (nx, ny, nz).

    order_arr is the int32 order of the whole grid (any shape, C order, x fastest).
    Returns (rec[nbox, 4] uint32, counts[4] int64, anomalies int).
    """
    lib = _load()
    dims, lo, hi = _box(dims, lo, hi)
    o = np.ascontiguousarray(order_arr, dtype=np.int32).reshape(-1)
    assert o.size == int(np.prod(dims))
    nbox = int(np.prod(hi - lo))
    rec = np.zeros((nbox, 4), np.uint32)
    counts = np.zeros(4, np.int64)
    an = np.zeros(1, np.int64)
    rc = lib.oracle_lower_stars(_p(o), _p(dims), _p(lo), _p(hi), _p(rec), _p(counts),
                                int(bool(literal)), int(nthreads), _p(an))
    if rc != 0:
        raise ValueError("bad box")
    return rec, counts, int(an[0])


def lower_stars_sampled(values, dims, vids, nthreads=0):
    """Records of the sampled vertices, computed from (value, id) comparisons."""
    lib = _load()
    v = np.ascontiguousarray(values).reshape(-1)
    dt = {np.dtype(np.float32): 0, np.dtype(np.float64): 1}[v.dtype]
    dims = _i64(dims)
    vids = _i64(vids)
    rec = np.zeros((vids.size, 4), np.uint32)
    an = np.zeros(1, np.int64)
    rc = lib.oracle_lower_stars_sampled(_p(v), dt, _p(dims), _p(vids), vids.size, _p(rec),
                                        int(nthreads), _p(an))
    if rc == 1:
        raise ValueError("NaN in input")
    if rc != 0:
        raise ValueError("bad arguments")
    if an[0]:
        raise RuntimeError("oracle anomaly count %d" % an[0])
    return rec


def pls_local(okey, literal=False):
    """One lower star from 15 keys (x, then neighbours 0..13; -1 = absent).

    Returns (states[75] int8, rec[4] uint32, anomalies).
    """
    lib = _load()
    k = _i64(okey)
    assert k.size == 15
    st = np.zeros(NCELL, np.int8)
    rec = np.zeros(4, np.uint32)
    an = np.zeros(1, np.int64)
    lib.oracle_pls_local(_p(k), int(bool(literal)), _p(st), _p(rec), _p(an))
    return st, rec, int(an[0])


def pls_batch(keys, nthreads=0):
    """Lower stars of many explicit neighbourhoods: keys is (m, 15) uint8 (x,
    then neighbours 0..13; 255 = absent).  Returns rec (m, 4) uint32."""
    lib = _load()
    k = np.ascontiguousarray(keys, dtype=np.uint8).reshape(-1, 15)
    rec = np.zeros((k.shape[0], 4), np.uint32)
    an = np.zeros(1, np.int64)
    if lib.oracle_pls_batch(_p(k), k.shape[0], _p(rec), int(nthreads), _p(an)) != 0:
        raise RuntimeError("oracle pls_batch failed")
    if an[0]:
        raise RuntimeError("oracle anomaly count %d" % an[0])
    return rec


def decode_record(rec4):
    lib = _load()
    r = np.ascontiguousarray(np.asarray(rec4, dtype=np.uint32).reshape(4))
    st = np.zeros(NCELL, np.int8)
    lib.oracle_decode_record(_p(r), _p(st))
    return st


def critical_simplices(rec, dims, lo=None, hi=None, cap=None, nthreads=1):
    """Returns ([crit0, crit1, crit2, crit3] int64 code arrays, counts[4]).
    nthreads: threads over the rows of the box (0 = all)."""
    lib = _load()
    dims, lo, hi = _box(dims, lo, hi)
    r = np.ascontiguousarray(rec, dtype=np.uint32)
    counts = np.zeros(4, np.int64)
    zero = np.zeros(4, np.int64)
    lib.oracle_critical_simplices(_p(r), _p(dims), _p(lo), _p(hi), None, None, None, None,
                                  _p(zero), _p(counts), int(nthreads))
    cap = counts.copy() if cap is None else _i64(cap)
    outs = [np.zeros(max(int(c), 1), np.int64) for c in cap]
    counts2 = np.zeros(4, np.int64)
    rc = lib.oracle_critical_simplices(_p(r), _p(dims), _p(lo), _p(hi), _p(outs[0]), _p(outs[1]),
                                       _p(outs[2]), _p(outs[3]), _p(cap), _p(counts2), int(nthreads))
    if rc != 0:
        raise ValueError("bad box")
    return [outs[d][: min(int(counts2[d]), int(cap[d]))] for d in range(4)], counts2


def d0_pairs(order_arr, rec_full, dims, crit1):
    """Algorithm 1 over the triplets of the critical edges (whole grid).

    Returns (pair_edge codes, pair_min vertex ids), in processing order.
    """
    lib = _load()
    dims = _i64(dims)
    o = np.ascontiguousarray(order_arr, dtype=np.int32).reshape(-1)
    r = np.ascontiguousarray(rec_full, dtype=np.uint32)
    c1 = _i64(crit1)
    pe = np.zeros(max(c1.size, 1), np.int64)
    pm = np.zeros(max(c1.size, 1), np.int64)
    npairs = np.zeros(1, np.int64)
    rc = lib.oracle_d0_pairs(_p(o), _p(r), _p(dims), _p(c1), c1.size, _p(pe), _p(pm), _p(npairs))
    if rc != 0:
        raise RuntimeError("oracle d0 failed (%d)" % rc)
    n = int(npairs[0])
    return pe[:n].copy(), pm[:n].copy()


def d0_loss_grad(values_f64, pair_edge, pair_min, threshold=0.05):
    """Loss of the differentiable form and its exact gradient (Section 2.5).

    Each D0 pair (sigma, t) has birth f(t) and death f(maxv(sigma)), the
    highest vertex value of each simplex; persistence = death - birth.
    L = sum over pairs with persistence < threshold of persistence^2, so
    dL/d(death) = 2 pers and dL/d(birth) = -2 pers, scattered to the two
    vertices that carry the values.
    """
    f = np.asarray(values_f64, dtype=np.float64).reshape(-1)
    dv = np.asarray(pair_edge, dtype=np.int64) >> 8
    bv = np.asarray(pair_min, dtype=np.int64)
    pers = f[dv] - f[bv]
    keep = pers < threshold
    loss = float(np.sum(pers[keep] ** 2))
    grad = np.zeros(f.size, np.float64)
    np.add.at(grad, dv[keep], 2.0 * pers[keep])
    np.add.at(grad, bv[keep], -2.0 * pers[keep])
    return loss, grad, keep


def filtration_sort(order_arr, dims, codes, dim):
    """Critical cells of dimension dim, as (maxv << 8) | local index codes,
    sorted in the filtration order of Section 2.1 (decreasing vertex-order
    lists compared lexicographically)."""
    lib = _load()
    o = np.ascontiguousarray(order_arr, dtype=np.int32).reshape(-1)
    c = _i64(codes).reshape(-1)
    out = np.zeros(max(c.size, 1), np.int64)
    rc = lib.oracle_filtration_sort(_p(o), _p(_i64(dims)), _p(c), c.size, int(dim), _p(out))
    if rc != 0:
        raise ValueError("oracle filtration sort failed (%d)" % rc)
    return out[:c.size].copy()


def d2_pairs(order_arr, rec_full, dims, crit2, crit3):
    """D2 pairs (the dual of Algorithm 1 on the tets, Section 2.6) over the
    whole grid.  Returns (pair_tri codes, pair_tet codes) in visiting order
    (decreasing triangle)."""
    lib = _load()
    o = np.ascontiguousarray(order_arr, dtype=np.int32).reshape(-1)
    r = np.ascontiguousarray(rec_full, dtype=np.uint32)
    c2 = _i64(crit2).reshape(-1)
    c3 = _i64(crit3).reshape(-1)
    pt = np.zeros(max(c2.size, 1), np.int64)
    pq = np.zeros(max(c2.size, 1), np.int64)
    npairs = np.zeros(1, np.int64)
    rc = lib.oracle_d2_pairs(_p(o), _p(r), _p(_i64(dims)), _p(c2), c2.size, _p(c3), c3.size, _p(pt), _p(pq),
                             _p(npairs))
    if rc != 0:
        raise RuntimeError("oracle d2 failed (%d)" % rc)
    n = int(npairs[0])
    return pt[:n].copy(), pq[:n].copy()
