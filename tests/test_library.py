"""Host-side checks of the HIP library (no GPU needed): it loads, exports
every symbol include/dms.h declares, its compile-time star tables equal the
oracle's, argument errors come back synchronously, and the host D0 pairing
matches the oracle's Algorithm 1."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_2505_21266_amd as dms
from paper_2505_21266_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(dms.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return dms.lib()


def _declared():
    src = open(os.path.join(ROOT, "include", "dms.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dms_[a-z0-9_]+)\s*\(", src)))


def test_exports_every_declared_symbol(L):
    names = _declared()
    assert len(names) >= 10
    for nm in names:
        assert hasattr(L, nm), nm
    assert sorted(dms.SYMBOLS) == names


def test_status_strings(L):
    for s in range(7):
        assert L.dms_status_str(s).decode().startswith("DMS_")
    assert b"gfx950" in L.dms_version()


def test_tables_match_oracle(L):
    a = dms.star_tables()
    b = oracle.star_tables()
    for k in ("nb", "tri", "tet", "edge_tris", "tri_tets"):
        assert (a[k] == b[k]).all(), k


def _a3(v):
    a = np.asarray(v, np.int64)
    return a, a.ctypes.data_as(ctypes.c_void_p)


def test_argument_errors(L):
    P = ctypes.c_void_p
    fake = P(4096)  # never dereferenced: every call below fails its checks first
    d, dp = _a3([4, 4, 4])
    l, lp = _a3([0, 0, 0])
    h, hp = _a3([4, 4, 4])
    bad, badp = _a3([0, 0, 5])
    # order
    assert L.dms_order(None, 0, 10, fake, fake, 1 << 30, fake, None) == 1
    assert L.dms_order(fake, 7, 10, fake, fake, 1 << 30, fake, None) == 1
    assert L.dms_order(fake, 0, -1, fake, fake, 1 << 30, fake, None) == 1
    assert L.dms_order(fake, 0, 1 << 31, fake, fake, 1 << 40, fake, None) == 2
    assert L.dms_order(fake, 0, 1000, fake, fake, 10, fake, None) == 3
    assert L.dms_order(fake, 0, 0, None, None, 0, None, None) == 0
    assert L.dms_order_workspace_size(1000, 0) >= 16 * 1000
    assert L.dms_order_workspace_size(1000, 1) >= 24 * 1000
    # gradient
    assert L.dms_discrete_gradient(None, dp, lp, hp, fake, None, None, 0, None) == 1
    assert L.dms_discrete_gradient(fake, dp, lp, badp, fake, None, None, 0, None) == 1
    big, bigp = _a3([2048, 2048, 1024])
    assert L.dms_discrete_gradient(fake, bigp, lp, hp, fake, None, None, 0, None) == 2
    assert L.dms_discrete_gradient(fake, dp, lp, lp, fake, None, None, 0, None) == 0  # empty box
    neg, negp = _a3([-1, 0, 0])
    assert L.dms_discrete_gradient(fake, dp, negp, hp, fake, None, None, 0, None) == 1
    need = L.dms_gradient_workspace_size(dp, lp, hp)
    assert need >= 256 + 16 * 1024
    assert L.dms_discrete_gradient(fake, dp, lp, hp, fake, None, fake, need - 1, None) == 3
    assert L.dms_gradient_workspace_size(dp, lp, badp) == 0
    # gradient from the values
    assert L.dms_discrete_gradient_values(fake, 7, dp, lp, hp, fake, None, None, 0, fake, None) == 1
    assert L.dms_discrete_gradient_values(None, 0, dp, lp, hp, fake, None, None, 0, fake, None) == 1
    assert L.dms_discrete_gradient_values(fake, 0, dp, lp, hp, fake, None, None, 0, None, None) == 1
    assert L.dms_discrete_gradient_values(fake, 1, dp, lp, badp, fake, None, None, 0, fake, None) == 1
    # no int32 order on this path: grids past 2^31 vertices are accepted, up to 2^40
    huge, hugep = _a3([1 << 21, 1 << 20, 4])
    assert L.dms_discrete_gradient_values(fake, 0, hugep, lp, hp, fake, None, None, 0, fake, None) == 2
    assert L.dms_gradient_workspace_size(bigp, lp, hp) > 0
    assert L.dms_gradient_workspace_size(hugep, lp, hp) == 0
    assert L.dms_discrete_gradient_values(fake, 0, dp, lp, hp, fake, None, fake, need - 1, fake, None) == 3
    assert L.dms_discrete_gradient_values(fake, 0, dp, lp, lp, fake, None, None, 0, fake, None) == 0
    # critical
    cap, capp = _a3([0, 0, 0, 0])
    assert L.dms_critical_simplices(fake, None, dp, lp, hp, None, None, None, None, capp, fake, fake, 0,
                                    fake, None) == 3
    ncap, ncapp = _a3([0, -1, 0, 0])
    assert L.dms_critical_simplices(fake, None, dp, lp, hp, None, None, None, None, ncapp, fake, fake,
                                    1 << 20, fake, None) == 1
    c1, c1p = _a3([0, 5, 0, 0])
    assert L.dms_critical_simplices(fake, None, dp, lp, hp, None, None, None, None, c1p, fake, fake,
                                    1 << 20, fake, None) == 1
    assert L.dms_critical_workspace_size(dp, lp, badp) == 0
    # allocation-free extraction: same argument checks, and boxes past its
    # scratch array (160 Ki tiles of 1024 records) are refused
    assert L.dms_critical_simplices_noalloc(fake, None, dp, lp, hp, None, None, None, None, ncapp, fake, fake,
                                            None) == 1
    assert L.dms_critical_simplices_noalloc(fake, None, dp, lp, hp, None, None, None, None, capp, fake, None,
                                            None) == 1
    big, bigp = _a3([1024, 1024, 161])
    assert L.dms_critical_simplices_noalloc(fake, None, bigp, lp, bigp, None, None, None, None, capp, fake, fake,
                                            None) == 2
    # backward
    need = L.dms_gradient_backward_workspace_size(3)
    assert need >= 6 * 16
    assert L.dms_gradient_backward(None, fake, fake, fake, 3, fake, 10, fake, need, None) == 1
    assert L.dms_gradient_backward(fake, fake, fake, fake, 3, None, 10, fake, need, None) == 1
    assert L.dms_gradient_backward(fake, fake, fake, fake, -1, fake, 10, fake, need, None) == 1
    assert L.dms_gradient_backward(fake, fake, fake, fake, (1 << 30) + 1, fake, 10, fake, need, None) == 1
    assert L.dms_gradient_backward(fake, fake, fake, fake, 3, fake, 10, fake, need - 1, None) == 3
    assert L.dms_gradient_backward(fake, fake, fake, fake, 3, fake, 10, None, 0, None) == 3
    assert L.dms_gradient_backward(fake, fake, fake, fake, 3, fake, 0, None, 0, None) == 0  # nothing to write
    # simplex values
    assert L.dms_simplex_values(fake, 2, 10, fake, 3, fake, None) == 1
    assert L.dms_simplex_values(None, 0, 10, fake, 3, fake, None) == 1
    assert L.dms_simplex_values(fake, 0, 10, fake, -1, fake, None) == 1
    assert L.dms_simplex_values(None, 0, 10, None, 0, None, None) == 0


def test_no_device_is_unsupported(L):
    """Without a gfx950 device (this host has none), calls whose arguments
    are valid return DMS_E_UNSUPPORTED instead of launching: dms_init, the
    gradient (which also needs dms_init), the order and the extraction."""
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    P = ctypes.c_void_p
    fake = P(4096)  # never dereferenced: the device check fails first
    d, dp = _a3([4, 4, 4])
    l, lp = _a3([0, 0, 0])
    h, hp = _a3([4, 4, 4])
    assert L.dms_init(None) == 4
    assert L.dms_discrete_gradient(fake, dp, lp, hp, fake, None, None, 0, None) == 4
    assert L.dms_discrete_gradient_values(fake, 0, dp, lp, hp, fake, None, None, 0, fake, None) == 4
    assert L.dms_order(fake, 0, 64, fake, fake, 1 << 30, fake, None) == 4
    cap, capp = _a3([0, 0, 0, 0])
    assert L.dms_critical_simplices(fake, None, dp, lp, hp, None, None, None, None, capp, fake, fake, 1 << 20,
                                    fake, None) == 4
    need = L.dms_gradient_backward_workspace_size(3)
    assert L.dms_gradient_backward(fake, fake, fake, fake, 3, fake, 10, fake, need, None) == 4
    assert L.dms_simplex_values(fake, 0, 10, fake, 3, fake, None) == 4
    assert L.dms_critical_simplices_noalloc(fake, None, dp, lp, hp, None, None, None, None, capp, fake, fake,
                                            None) == 4
    out = P()
    assert L.dms_batch_create(d.ctypes.data_as(P), 1, 0, 0, None, ctypes.byref(out)) == 4
    assert not out.value


@pytest.mark.parametrize("dims,seed", [((8, 8, 8), 1), ((13, 9, 11), 2), ((32, 32, 32), 3)])
def test_host_d0_matches_oracle(L, dims, seed):
    nx, ny, nz = dims
    rng = np.random.default_rng(seed)
    v = inputs.mixture_field((nz, ny, nx), 8, rng, 1e-3, np.float64)
    o = oracle.order(v).reshape(-1)
    rec, _, _ = oracle.lower_stars(o, dims)
    crit, _ = oracle.critical_simplices(rec, dims)
    pe0, pm0 = oracle.d0_pairs(o, rec, dims, crit[1])
    pe1, pm1 = dms.d0_pairs_host(rec, o, dims, crit[1])
    assert (pe0 == pe1).all() and (pm0 == pm1).all()


def test_host_d0_errors(L):
    dims = (4, 4, 4)
    o = np.arange(64, dtype=np.int32)
    rec = np.zeros((64, 4), np.uint32)
    with pytest.raises(dms.DmsError):
        dms.d0_pairs_host(rec, o, dims, np.array([(100 << 8) | 3], np.int64))


def test_d0_pairs_sorted_host_hand_case():
    """Algorithm 1 on three minima (orders 5, 1, 9) and three sorted triplets,
    worked by hand: edge 100 joins minima 0 and 1, the younger (0, order 5)
    dies; edge 200 joins 2 and the class of 0 (representative 1), 2 dies;
    edge 300 joins 1 and 2, already one class."""
    L = dms.lib()
    P = ctypes.c_void_p
    te = np.array([100, 200, 300], np.int64)
    t0 = np.array([0, 2, 1], np.int32)
    t1 = np.array([1, 0, 2], np.int32)
    mo = np.array([5, 1, 9], np.int32)
    pe = np.zeros(3, np.int64)
    pm = np.zeros(3, np.int32)
    npairs = np.zeros(1, np.int64)
    st = L.dms_d0_pairs_sorted_host(te.ctypes.data_as(P), t0.ctypes.data_as(P), t1.ctypes.data_as(P), 3,
                                    mo.ctypes.data_as(P), 3, pe.ctypes.data_as(P), pm.ctypes.data_as(P), 3,
                                    npairs.ctypes.data_as(P))
    assert st == 0 and int(npairs[0]) == 2
    assert pe[:2].tolist() == [100, 200] and pm[:2].tolist() == [0, 2]
    # a minimum index outside [0, n0) is an argument error
    bad = np.array([0, 7, 1], np.int32)
    assert L.dms_d0_pairs_sorted_host(te.ctypes.data_as(P), bad.ctypes.data_as(P), t1.ctypes.data_as(P), 3,
                                      mo.ctypes.data_as(P), 3, pe.ctypes.data_as(P), pm.ctypes.data_as(P),
                                      3, npairs.ctypes.data_as(P)) == 1



def test_critical_sort_argument_errors(L):
    P = ctypes.c_void_p
    fake, other = P(4096), P(8192)  # never dereferenced: every call below fails its checks first
    d, dp = _a3([4, 4, 4])
    z, zp = _a3([0, 4, 4])
    big, bigp = _a3([2048, 2048, 1024])
    ws = L.dms_critical_sort_workspace_size(100)
    assert ws >= 100 * 36
    assert L.dms_critical_sort_workspace_size(-1) == 0
    assert L.dms_critical_sort(fake, 10, 4, fake, dp, other, fake, ws, fake, None) == 1  # dim
    assert L.dms_critical_sort(fake, 10, -1, fake, dp, other, fake, ws, fake, None) == 1
    assert L.dms_critical_sort(fake, 10, 1, fake, zp, other, fake, ws, fake, None) == 1  # dims
    assert L.dms_critical_sort(fake, -1, 1, fake, dp, other, fake, ws, fake, None) == 1
    assert L.dms_critical_sort(None, 10, 1, fake, dp, other, fake, ws, fake, None) == 1
    assert L.dms_critical_sort(fake, 10, 1, fake, dp, fake, fake, ws, fake, None) == 1  # in place
    assert L.dms_critical_sort(fake, 10, 1, fake, bigp, other, fake, ws, fake, None) == 2
    assert L.dms_critical_sort(fake, 100, 1, fake, dp, other, fake, 16, fake, None) == 3
    assert L.dms_critical_sort(None, 0, 1, None, dp, None, None, 0, None, None) == 0  # empty list


def test_d2_pairs_sorted_host_hand_case():
    """The dual union-find on three maxima with ranks 4, 9, 1 and the outside
    node (index 3), triplets in decreasing triangle order, worked by hand:
    triangle 300 joins maxima 0 and 1, the lower (0, rank 4) dies; triangle
    200 joins 2 and the outside, 2 dies; triangle 100 joins 1 and the
    outside, 1 dies; every maximum is paired."""
    L = dms.lib()
    P = ctypes.c_void_p
    tc = np.array([300, 200, 100], np.int64)
    t0 = np.array([0, 2, 1], np.int32)
    t1 = np.array([1, 3, 3], np.int32)
    mr = np.array([4, 9, 1], np.int32)
    pt = np.zeros(3, np.int64)
    pm = np.zeros(3, np.int32)
    npairs = np.zeros(1, np.int64)
    st = L.dms_d2_pairs_sorted_host(tc.ctypes.data_as(P), t0.ctypes.data_as(P), t1.ctypes.data_as(P), 3,
                                    mr.ctypes.data_as(P), 3, pt.ctypes.data_as(P), pm.ctypes.data_as(P), 3,
                                    npairs.ctypes.data_as(P))
    assert st == 0 and int(npairs[0]) == 3
    assert pt.tolist() == [300, 200, 100] and pm.tolist() == [0, 2, 1]
    bad = np.array([0, 5, 1], np.int32)  # index above n3
    assert L.dms_d2_pairs_sorted_host(tc.ctypes.data_as(P), bad.ctypes.data_as(P), t1.ctypes.data_as(P), 3,
                                      mr.ctypes.data_as(P), 3, pt.ctypes.data_as(P), pm.ctypes.data_as(P),
                                      3, npairs.ctypes.data_as(P)) == 1
    fake = P(4096)
    d, dp = _a3([4, 4, 4])
    assert L.dms_d2_workspace_size(-1, 0) == 0
    assert L.dms_d2_triplets(None, fake, dp, fake, 1, fake, 1, fake, fake, fake, fake, fake, fake, 1 << 30,
                             fake, None) == 1
    assert L.dms_d2_triplets(fake, fake, dp, fake, 10, fake, 1, fake, fake, fake, fake, fake, fake, 16,
                             fake, None) == 3



def test_bindings_reject_host_tensors():
    """The pairings and the filtration sort have no CPU path: host tensors
    and wrong shapes are refused before any launch."""
    torch = pytest.importorskip("torch")
    c = torch.zeros(4, dtype=torch.int64)
    o = torch.zeros(8, dtype=torch.int32)
    r = torch.zeros((8, 4), dtype=torch.int32)
    with pytest.raises(TypeError):
        dms.critical_sort(c, 1, o, (2, 2, 2))
    with pytest.raises(TypeError):
        dms.d0_pairs(r, o, (2, 2, 2), c, c)
    with pytest.raises(TypeError):
        dms.d2_pairs(r, o, (2, 2, 2), c, c)
