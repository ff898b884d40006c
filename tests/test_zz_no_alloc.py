"""The allocation-free extraction (dms_critical_simplices_noalloc) against
the workspace form (dms_critical_simplices) on the same records: the same
lists and counts, on two calls in a row with the second box smaller, so
that nothing the first call left in the library's scratch array carries
into the second; and the size limit is refused before any launch."""
import ctypes

import numpy as np
import pytest

import oracle
import paper_2505_21266_amd as dms

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dms.lib()


def _records(dims, seed, kind):
    nx, ny, nz = dims
    rng = np.random.default_rng(seed)
    v = rng.random((nz, ny, nx), dtype=np.float32) if kind == "noise" else \
        rng.integers(0, 4, (nz, ny, nx)).astype(np.float32)
    o = dms.order(torch.from_numpy(v).cuda())
    return o, dms.discrete_gradient(o)


def test_noalloc_matches_workspace_form_twice():
    cases = [((130, 90, 70), 5, "noise", None), ((40, 33, 21), 6, "ties", ((1, 2, 1), (39, 30, 20)))]
    for dims, seed, kind, box in cases:
        o, rec = _records(dims, seed, kind)
        lo, hi = box if box else (None, None)
        if box:
            o2 = dms.discrete_gradient(o, lo, hi)
            rec = o2
        want, wcount = dms.critical_simplices(rec, dims, lo, hi)
        cap = wcount.cpu().numpy()
        flags = dms.new_flags(rec.device)
        got, gcount = dms.critical_simplices_noalloc(rec, dims, cap, lo, hi, flags=flags)
        torch.cuda.synchronize()
        assert int(flags.item()) == 0
        assert torch.equal(gcount, wcount)
        for d in range(4):
            assert torch.equal(got[d], want[d]), (dims, d)


def test_noalloc_capacity_and_limit():
    dims = (70, 50, 40)
    o, rec = _records(dims, 7, "noise")
    want, wcount = dms.critical_simplices(rec, dims)
    cap = [max(int(c) // 2, 1) for c in wcount.cpu().numpy()]
    flags = dms.new_flags(rec.device)
    got, gcount = dms.critical_simplices_noalloc(rec, dims, cap, flags=flags)
    torch.cuda.synchronize()
    assert int(flags.item()) & dms.FLAG_CAPACITY
    assert torch.equal(gcount, wcount)
    for d in range(4):
        assert torch.equal(got[d], want[d][: cap[d]])
    # a box past 160 Ki tiles of 1024 records is refused synchronously
    L = dms.lib()
    P = ctypes.c_void_p
    big = np.array([1024, 1024, 161], np.int64)
    zero = np.zeros(3, np.int64)
    capz = np.zeros(4, np.int64)
    st = L.dms_critical_simplices_noalloc(P(rec.data_ptr()), None, big.ctypes.data_as(P), zero.ctypes.data_as(P),
                                          big.ctypes.data_as(P), None, None, None, None, capz.ctypes.data_as(P),
                                          P(gcount.data_ptr()), P(flags.data_ptr()), None)
    assert st == 2
