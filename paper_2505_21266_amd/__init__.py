"""MI355X discrete-gradient library for Discrete Morse Sandwich: Python binding.

Argument marshalling only: every step runs in libdms.so (HIP kernels for
gfx950, plus the host D0 pairing).  torch provides device memory and the
current stream.  There is no CPU fallback: calls raise if the library is not
built or no GPU tensor is given.

Grids are torch tensors shaped (nz, ny, nx), x fastest; the library's dims
are (nx, ny, nz).  Boxes are half-open (x, y, z) bounds [lo, hi).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdms.so")

DMS_F32, DMS_F64 = 0, 1
FLAG_NAN, FLAG_CAPACITY, FLAG_BADCODE = 1, 2, 4
STATUS = {0: "DMS_OK", 1: "DMS_E_ARG", 2: "DMS_E_SIZE", 3: "DMS_E_WORKSPACE",
          4: "DMS_E_UNSUPPORTED", 5: "DMS_E_HIP", 6: "DMS_E_NOT_INITIALISED"}

# every symbol include/dms.h declares
SYMBOLS = ("dms_status_str", "dms_version", "dms_init", "dms_star_tables", "dms_order_workspace_size",
           "dms_order", "dms_gradient_workspace_size", "dms_discrete_gradient",
           "dms_discrete_gradient_values",
           "dms_critical_workspace_size",
           "dms_critical_simplices", "dms_critical_simplices_noalloc", "dms_simplex_values",
           "dms_gradient_backward_workspace_size",
           "dms_gradient_backward", "dms_d0_pairs_host",
           "dms_batch_create", "dms_batch_workspace_size", "dms_batch_total", "dms_batch_variant",
           "dms_batch_run", "dms_batch_destroy", "dms_d0_workspace_size", "dms_d0_triplets",
           "dms_d0_pairs_sorted_host", "dms_critical_sort_workspace_size", "dms_critical_sort",
           "dms_d2_workspace_size", "dms_d2_triplets", "dms_d2_pairs_sorted_host")

_lib = None


class DmsError(RuntimeError):
    def __init__(self, status, where):
        super().__init__("%s failed: %s" % (where, STATUS.get(status, status)))
        self.status = status


def lib():
    """Loads libdms.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libdms.so is not built: run __graft_entry__.build() "
                           "(or python paper_2505_21266_amd/build.py)")
    L = ctypes.CDLL(LIB_PATH)
    P, I64, I, SZ = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_size_t
    L.dms_status_str.argtypes = [I]
    L.dms_status_str.restype = ctypes.c_char_p
    L.dms_version.argtypes = []
    L.dms_version.restype = ctypes.c_char_p
    L.dms_init.argtypes = [P]
    L.dms_star_tables.argtypes = [P, P, P, P, P]
    L.dms_order_workspace_size.argtypes = [I64, I]
    L.dms_order_workspace_size.restype = SZ
    L.dms_order.argtypes = [P, I, I64, P, P, SZ, P, P]
    L.dms_gradient_workspace_size.argtypes = [P, P, P]
    L.dms_gradient_workspace_size.restype = SZ
    L.dms_discrete_gradient.argtypes = [P, P, P, P, P, P, P, SZ, P]
    L.dms_discrete_gradient_values.argtypes = [P, I, P, P, P, P, P, P, SZ, P, P]
    L.dms_critical_workspace_size.argtypes = [P, P, P]
    L.dms_critical_workspace_size.restype = SZ
    L.dms_critical_simplices.argtypes = [P, P, P, P, P, P, P, P, P, P, P, P, SZ, P, P]
    L.dms_critical_simplices_noalloc.argtypes = [P, P, P, P, P, P, P, P, P, P, P, P, P]
    L.dms_simplex_values.argtypes = [P, I, I64, P, I64, P, P]
    L.dms_gradient_backward_workspace_size.argtypes = [I64]
    L.dms_gradient_backward_workspace_size.restype = SZ
    L.dms_gradient_backward.argtypes = [P, P, P, P, I64, P, I64, P, SZ, P]
    L.dms_d0_pairs_host.argtypes = [P, P, P, P, I64, P, P, I64, P]
    L.dms_batch_create.argtypes = [P, I, I, I, ctypes.c_char_p, P]
    L.dms_batch_workspace_size.argtypes = [P]
    L.dms_batch_workspace_size.restype = SZ
    L.dms_batch_total.argtypes = [P]
    L.dms_batch_total.restype = I64
    L.dms_batch_variant.argtypes = [P]
    L.dms_batch_run.argtypes = [P, P, P, P, P, P, P, P, P, P, P, P, SZ, P, P]
    L.dms_batch_destroy.argtypes = [P]
    L.dms_batch_destroy.restype = None
    L.dms_d0_workspace_size.argtypes = [P, I64]
    L.dms_d0_workspace_size.restype = SZ
    L.dms_d0_triplets.argtypes = [P, P, P, P, I64, P, I64, P, P, P, P, P, P, SZ, P, P]
    L.dms_d0_pairs_sorted_host.argtypes = [P, P, P, I64, P, I64, P, P, I64, P]
    L.dms_critical_sort_workspace_size.argtypes = [I64]
    L.dms_critical_sort_workspace_size.restype = SZ
    L.dms_critical_sort.argtypes = [P, I64, ctypes.c_int, P, P, P, P, SZ, P, P]
    L.dms_d2_workspace_size.argtypes = [I64, I64]
    L.dms_d2_workspace_size.restype = SZ
    L.dms_d2_triplets.argtypes = [P, P, P, P, I64, P, I64, P, P, P, P, P, P, SZ, P, P]
    L.dms_d2_pairs_sorted_host.argtypes = [P, P, P, I64, P, I64, P, P, I64, P]
    for f in ("dms_init", "dms_critical_simplices_noalloc", "dms_simplex_values", "dms_star_tables", "dms_order", "dms_discrete_gradient", "dms_discrete_gradient_values",
              "dms_critical_simplices", "dms_d0_triplets", "dms_d0_pairs_sorted_host", "dms_critical_sort",
              "dms_d2_triplets", "dms_d2_pairs_sorted_host",
              "dms_gradient_backward", "dms_d0_pairs_host", "dms_batch_create", "dms_batch_variant",
              "dms_batch_run"):
        getattr(L, f).restype = I
    _lib = L
    return L


def _check(status, where):
    if status != 0:
        raise DmsError(status, where)


_ready = set()


def init(device=None):
    """dms_init on a device (once per device and process): checks that it is a
    gfx950 and fills the library's lower-star tables, synchronising torch's
    current stream of that device once."""
    import torch
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    idx = dev.index if dev.index is not None else torch.cuda.current_device()
    if idx in _ready:
        return
    with torch.cuda.device(idx):
        _check(lib().dms_init(ctypes.c_void_p(torch.cuda.current_stream(idx).cuda_stream)), "dms_init")
    _ready.add(idx)


def _arr3(v):
    a = np.ascontiguousarray(np.asarray(v, dtype=np.int64).reshape(3))
    return a, a.ctypes.data_as(ctypes.c_void_p)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p(0)


def _stream(t):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _require_gpu(t, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a GPU tensor (this library has no CPU path)" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)


def dims_of(t):
    """(nx, ny, nz) of a (nz, ny, nx) tensor (1-D tensors are (n, 1, 1))."""
    s = tuple(t.shape)
    if len(s) == 1:
        return (s[0], 1, 1)
    if len(s) != 3:
        raise ValueError("expected a 3-D (nz, ny, nx) tensor")
    return (s[2], s[1], s[0])


def star_tables():
    """The library's compile-time Kuhn star tables (host copies)."""
    L = lib()
    nb = np.zeros((14, 3), np.int32)
    tri = np.zeros((36, 2), np.int32)
    tet = np.zeros((24, 3), np.int32)
    et = np.zeros((14, 6), np.int32)
    tt = np.zeros((36, 2), np.int32)
    P = ctypes.c_void_p
    _check(L.dms_star_tables(nb.ctypes.data_as(P), tri.ctypes.data_as(P), tet.ctypes.data_as(P),
                             et.ctypes.data_as(P), tt.ctypes.data_as(P)), "dms_star_tables")
    return dict(nb=nb, tri=tri, tet=tet, edge_tris=et, tri_tets=tt)


class Workspace:
    """A growable device byte buffer reused across calls."""

    def __init__(self):
        self.buf = None

    def get(self, nbytes, device):
        import torch
        if self.buf is None or self.buf.numel() < nbytes or self.buf.device != device:
            self.buf = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
        return self.buf


_ws_order = Workspace()
_ws_crit = Workspace()


def new_flags(device):
    import torch
    return torch.zeros(1, dtype=torch.int32, device=device)


def check_flags(flags, allow=0):
    """Synchronises and raises if a device flag beyond `allow` is set."""
    f = int(flags.item())
    if f & ~allow & FLAG_NAN:
        raise ValueError("NaN in the input field")
    if f & ~allow & FLAG_CAPACITY:
        raise RuntimeError("critical list capacity exceeded")
    if f & ~allow & FLAG_BADCODE:
        raise ValueError("a cell code names no cell of the grid")
    return f


def _dtype_code(values):
    import torch
    if values.dtype == torch.float32:
        return DMS_F32
    if values.dtype == torch.float64:
        return DMS_F64
    raise TypeError("values must be float32 or float64")


def order(values, out=None, flags=None, check=True):
    """Global vertex order (dms_order): int32 tensor of the values' shape."""
    import torch
    _require_gpu(values, "values")
    dt = _dtype_code(values)
    L = lib()
    n = values.numel()
    if out is None:
        out = torch.empty(values.shape, dtype=torch.int32, device=values.device)
    own_flags = flags is None
    if own_flags:
        flags = new_flags(values.device)
    nbytes = L.dms_order_workspace_size(n, dt)
    ws = _ws_order.get(nbytes, values.device)
    _check(L.dms_order(_ptr(values), dt, n, _ptr(out), _ptr(ws), ws.numel(), _ptr(flags),
                       _stream(values)), "dms_order")
    if check and own_flags:
        check_flags(flags)
    return out


def _box(dims, lo, hi):
    lo = (0, 0, 0) if lo is None else tuple(int(v) for v in lo)
    hi = tuple(dims) if hi is None else tuple(int(v) for v in hi)
    return lo, hi


def gradient_workspace(order_t, lo=None, hi=None):
    """A workspace for discrete_gradient on this grid and box (uint8 tensor)."""
    import torch
    dims = dims_of(order_t)
    lo, hi = _box(dims, lo, hi)
    d, dp = _arr3(dims)
    l, lp = _arr3(lo)
    h, hp = _arr3(hi)
    return torch.empty(max(int(lib().dms_gradient_workspace_size(dp, lp, hp)), 256),
                       dtype=torch.uint8, device=order_t.device)


def critical_mask(nbox, device):
    """A critical-record mask for a box of nbox vertices: int32 tensor of
    ceil(nbox / 32) words (one bit per record)."""
    import torch
    return torch.empty(max((int(nbox) + 31) // 32, 1), dtype=torch.int32, device=device)


def _mask_ptr(mask, nbox):
    if mask is None:
        return None
    import torch
    if not mask.is_cuda or mask.dtype != torch.int32 or not mask.is_contiguous():
        raise TypeError("critical mask must be a contiguous int32 GPU tensor")
    if mask.numel() < (nbox + 31) // 32:
        raise ValueError("critical mask too small (%d < %d words)" % (mask.numel(), (nbox + 31) // 32))
    return _ptr(mask)


def discrete_gradient(order_t, lo=None, hi=None, out=None, queue=True, workspace=None, mask=None):
    """Lower-star records (dms_discrete_gradient): int32 tensor (nbox, 4)
    holding the 128-bit records (reinterpret as uint32).  queue=False passes
    no workspace (general vertices are then paired inside their tiles);
    workspace (from gradient_workspace) avoids an allocation per call;
    mask (from critical_mask) receives the bits of the records that hold a
    critical cell, for critical_simplices."""
    import torch
    _require_gpu(order_t, "order")
    if order_t.dtype != torch.int32:
        raise TypeError("order must be int32")
    dims = dims_of(order_t)
    lo, hi = _box(dims, lo, hi)
    nbox = max(0, (hi[0] - lo[0])) * max(0, (hi[1] - lo[1])) * max(0, (hi[2] - lo[2]))
    if out is None:
        out = torch.empty((nbox, 4), dtype=torch.int32, device=order_t.device)
    d, dp = _arr3(dims)
    l, lp = _arr3(lo)
    h, hp = _arr3(hi)
    init(order_t.device)
    ws, wbytes = None, 0
    if queue and nbox > 0:
        wbytes = int(lib().dms_gradient_workspace_size(dp, lp, hp))
        if workspace is not None:
            if workspace.numel() < wbytes or not workspace.is_cuda:
                raise ValueError("gradient workspace too small (%d < %d bytes)"
                                 % (workspace.numel(), wbytes))
            ws, wbytes = workspace, workspace.numel()
        else:
            ws = torch.empty(wbytes, dtype=torch.uint8, device=order_t.device)
    _check(lib().dms_discrete_gradient(_ptr(order_t), dp, lp, hp, _ptr(out), _mask_ptr(mask, nbox),
                                       _ptr(ws) if ws is not None else None, wbytes,
                                       _stream(order_t)),
           "dms_discrete_gradient")
    return out


def discrete_gradient_values(values, lo=None, hi=None, out=None, queue=True, workspace=None,
                             flags=None, check=True, mask=None):
    """Lower-star records straight from the values (dms_discrete_gradient_values):
    the same records as discrete_gradient(order(values)), without the sort.
    Raises on NaN when check (else the caller reads flags); mask as for
    discrete_gradient."""
    import torch
    _require_gpu(values, "values")
    dt = _dtype_code(values)
    dims = dims_of(values)
    lo, hi = _box(dims, lo, hi)
    nbox = max(0, (hi[0] - lo[0])) * max(0, (hi[1] - lo[1])) * max(0, (hi[2] - lo[2]))
    if out is None:
        out = torch.empty((nbox, 4), dtype=torch.int32, device=values.device)
    d, dp = _arr3(dims)
    l, lp = _arr3(lo)
    h, hp = _arr3(hi)
    own_flags = flags is None
    if own_flags:
        flags = new_flags(values.device)
    init(values.device)
    ws, wbytes = None, 0
    if queue and nbox > 0:
        wbytes = int(lib().dms_gradient_workspace_size(dp, lp, hp))
        if workspace is not None:
            if workspace.numel() < wbytes or not workspace.is_cuda:
                raise ValueError("gradient workspace too small (%d < %d bytes)"
                                 % (workspace.numel(), wbytes))
            ws, wbytes = workspace, workspace.numel()
        else:
            ws = torch.empty(wbytes, dtype=torch.uint8, device=values.device)
    _check(lib().dms_discrete_gradient_values(_ptr(values), dt, dp, lp, hp, _ptr(out),
                                              _mask_ptr(mask, nbox),
                                              _ptr(ws) if ws is not None else None, wbytes,
                                              _ptr(flags), _stream(values)),
           "dms_discrete_gradient_values")
    if check and own_flags:
        check_flags(flags)
    return out


def critical_simplices(rec, dims, lo=None, hi=None, cap=None, flags=None, counts=None, mask=None):
    """Critical cells (dms_critical_simplices) as four int64 code tensors.

    cap: per-dimension capacities; None sizes the lists exactly (one extra
    counting call and a sync).  mask: the critical mask the gradient call
    wrote with rec (only flagged records are read), or None.  Returns
    (lists, counts tensor).
    """
    import torch
    _require_gpu(rec, "rec")
    dev = rec.device
    lo, hi = _box(dims, lo, hi)
    d, dp = _arr3(dims)
    l, lp = _arr3(lo)
    h, hp = _arr3(hi)
    L = lib()
    mp = _mask_ptr(mask, max(0, hi[0] - lo[0]) * max(0, hi[1] - lo[1]) * max(0, hi[2] - lo[2]))
    nbytes = L.dms_critical_workspace_size(dp, lp, hp)
    ws = _ws_crit.get(nbytes, dev)
    if counts is None:
        counts = torch.zeros(4, dtype=torch.int64, device=dev)
    own_flags = flags is None
    if own_flags:
        flags = new_flags(dev)
    st = _stream(rec)
    if cap is None:
        zc = np.zeros(4, np.int64)
        _check(L.dms_critical_simplices(_ptr(rec), mp, dp, lp, hp, None, None, None, None,
                                        zc.ctypes.data_as(ctypes.c_void_p), _ptr(counts), _ptr(ws),
                                        ws.numel(), _ptr(flags), st), "dms_critical_simplices")
        cap = counts.cpu().numpy().copy()
        flags.zero_()
    capa = np.ascontiguousarray(np.asarray(cap, dtype=np.int64).reshape(4))
    lists = [torch.empty(int(max(c, 0)), dtype=torch.int64, device=dev) for c in capa]
    _check(L.dms_critical_simplices(_ptr(rec), mp, dp, lp, hp, _ptr(lists[0]), _ptr(lists[1]),
                                    _ptr(lists[2]), _ptr(lists[3]),
                                    capa.ctypes.data_as(ctypes.c_void_p), _ptr(counts), _ptr(ws),
                                    ws.numel(), _ptr(flags), st), "dms_critical_simplices")
    if own_flags:
        check_flags(flags)
    return lists, counts


def critical_simplices_noalloc(rec, dims, cap, lo=None, hi=None, lists=None, counts=None, flags=None,
                               mask=None):
    """The extraction with the library's own scratch array
    (dms_critical_simplices_noalloc: no workspace, nothing allocated by the
    library).  cap: per-dimension capacities; lists: four int64 tensors of
    those capacities (allocated here when None); mask as for
    critical_simplices.  Returns (lists, counts); the caller checks flags
    (DMS_FLAG_CAPACITY) after a sync."""
    import torch
    _require_gpu(rec, "rec")
    dev = rec.device
    init(dev)
    lo, hi = _box(dims, lo, hi)
    d, dp = _arr3(dims)
    l, lp = _arr3(lo)
    h, hp = _arr3(hi)
    capa = np.ascontiguousarray(np.asarray(cap, dtype=np.int64).reshape(4))
    if lists is None:
        lists = [torch.empty(int(max(c, 0)), dtype=torch.int64, device=dev) for c in capa]
    if counts is None:
        counts = torch.zeros(4, dtype=torch.int64, device=dev)
    if flags is None:
        flags = new_flags(dev)
    mp = _mask_ptr(mask, max(0, hi[0] - lo[0]) * max(0, hi[1] - lo[1]) * max(0, hi[2] - lo[2]))
    _check(lib().dms_critical_simplices_noalloc(_ptr(rec), mp, dp, lp, hp, _ptr(lists[0]), _ptr(lists[1]),
                                                _ptr(lists[2]), _ptr(lists[3]),
                                                capa.ctypes.data_as(ctypes.c_void_p), _ptr(counts),
                                                _ptr(flags), _stream(rec)),
           "dms_critical_simplices_noalloc")
    return lists, counts


def simplex_values(values, codes, out=None):
    """f of each simplex, the value of its highest vertex (dms_simplex_values):
    float64 tensor of codes' length."""
    import torch
    _require_gpu(values, "values")
    _require_gpu(codes, "codes")
    if codes.dtype != torch.int64:
        raise TypeError("codes must be int64")
    if out is None:
        out = torch.empty(codes.numel(), dtype=torch.float64, device=codes.device)
    _check(lib().dms_simplex_values(_ptr(values), _dtype_code(values), values.numel(), _ptr(codes),
                                    codes.numel(), _ptr(out), _stream(codes)), "dms_simplex_values")
    return out


def gradient_backward(birth_code, death_code, g_birth, g_death, n, out=None):
    """dL/df from dL/d(birth, death) of persistence pairs (dms_gradient_backward):
    each vertex sums its contributions in one fixed order (deterministic)."""
    import torch
    for t, nm in ((birth_code, "birth_code"), (death_code, "death_code"), (g_birth, "g_birth"),
                  (g_death, "g_death")):
        _require_gpu(t, nm)
    np_ = birth_code.numel()
    if out is None:
        out = torch.empty(int(n), dtype=torch.float64, device=birth_code.device)
    wbytes = int(lib().dms_gradient_backward_workspace_size(np_))
    ws = torch.empty(max(wbytes, 256), dtype=torch.uint8, device=birth_code.device)
    _check(lib().dms_gradient_backward(_ptr(birth_code), _ptr(death_code), _ptr(g_birth),
                                       _ptr(g_death), np_, _ptr(out), int(n), _ptr(ws), ws.numel(),
                                       _stream(out)),
           "dms_gradient_backward")
    return out


def d0_pairs_host(rec_np, order_np, dims, crit1_np):
    """Host D0 pairing (dms_d0_pairs_host) on numpy arrays of the whole grid.
    Returns (pair_edge codes, pair_min vertices) in processing order."""
    L = lib()
    P = ctypes.c_void_p
    rec_np = np.ascontiguousarray(rec_np).view(np.uint32)
    order_np = np.ascontiguousarray(order_np, dtype=np.int32)
    crit1_np = np.ascontiguousarray(crit1_np, dtype=np.int64)
    d, dp = _arr3(dims)
    cap = max(int(crit1_np.size), 1)
    pe = np.zeros(cap, np.int64)
    pm = np.zeros(cap, np.int64)
    npairs = np.zeros(1, np.int64)
    _check(L.dms_d0_pairs_host(rec_np.ctypes.data_as(P), order_np.ctypes.data_as(P), dp,
                               crit1_np.ctypes.data_as(P), crit1_np.size, pe.ctypes.data_as(P),
                               pm.ctypes.data_as(P), cap, npairs.ctypes.data_as(P)),
           "dms_d0_pairs_host")
    k = int(npairs[0])
    return pe[:k], pm[:k]


def _require_whole_grid(rec, order_t, dims, lists):
    """Arguments of the pairings: whole-grid records and order on the GPU,
    int64 critical lists on the GPU."""
    import torch
    _require_gpu(rec, "rec")
    _require_gpu(order_t, "order")
    n = int(dims[0]) * int(dims[1]) * int(dims[2])
    if rec.dtype != torch.int32 or rec.numel() != 4 * n:
        raise ValueError("rec must hold the int32 records of the whole grid (%d x 4)" % n)
    if order_t.dtype != torch.int32 or order_t.numel() != n:
        raise ValueError("order must be the int32 order of the whole grid (%d)" % n)
    for nm, t in lists:
        _require_gpu(t, nm)
        if t.dtype != torch.int64:
            raise TypeError("%s must be int64 codes" % nm)


def critical_sort(codes, dim, order_t, dims, out=None, flags=None, check=True):
    """Critical cells of dimension dim (int64 device codes, as
    critical_simplices lists them) in the filtration order of Section 2.1
    (dms_critical_sort).  Returns a new int64 tensor unless out is given."""
    import torch
    _require_gpu(codes, "codes")
    _require_gpu(order_t, "order")
    if codes.dtype != torch.int64 or order_t.dtype != torch.int32:
        raise TypeError("codes must be int64 and order int32")
    if not 0 <= int(dim) <= 3:
        raise ValueError("dim must be 0..3")
    L = lib()
    n = int(codes.numel())
    if out is None:
        out = torch.empty(n, dtype=torch.int64, device=codes.device)
    if n == 0:
        return out
    codes = codes.contiguous()
    if flags is None:
        flags = new_flags(codes.device)
    d, dp = _arr3(dims)
    ws = torch.empty(max(int(L.dms_critical_sort_workspace_size(n)), 256), dtype=torch.uint8,
                     device=codes.device)
    _check(L.dms_critical_sort(_ptr(codes), n, int(dim), _ptr(order_t), dp, _ptr(out), _ptr(ws), ws.numel(),
                               _ptr(flags), _stream(codes)), "dms_critical_sort")
    if check:
        check_flags(flags)
    return out


def d0_pairs(rec, order_t, dims, crit0, crit1):
    """D0 pairing: the extremum graph on the GPU (dms_d0_triplets: descents by
    pointer doubling, triplets sorted by edge), Algorithm 1 on the host
    (dms_d0_pairs_sorted_host).  rec/order_t/crit0/crit1 are device tensors
    of the whole grid.  Returns numpy (pair_edge codes, pair_min vertices)."""
    import torch
    _require_whole_grid(rec, order_t, dims, [("crit0", crit0), ("crit1", crit1)])
    L = lib()
    P = ctypes.c_void_p
    dev = rec.device
    n0, n1 = int(crit0.numel()), int(crit1.numel())
    d, dp = _arr3(dims)
    tri_edge = torch.empty(max(n1, 1), dtype=torch.int64, device=dev)
    tri_min0 = torch.empty(max(n1, 1), dtype=torch.int32, device=dev)
    tri_min1 = torch.empty(max(n1, 1), dtype=torch.int32, device=dev)
    min_order = torch.empty(max(n0, 1), dtype=torch.int32, device=dev)
    ntri = torch.zeros(1, dtype=torch.int64, device=dev)
    flags = new_flags(dev)
    ws = torch.empty(max(int(L.dms_d0_workspace_size(dp, n1)), 256), dtype=torch.uint8, device=dev)
    _check(L.dms_d0_triplets(_ptr(rec), _ptr(order_t), dp, _ptr(crit0), n0, _ptr(crit1), n1,
                             _ptr(tri_edge), _ptr(tri_min0), _ptr(tri_min1), _ptr(min_order),
                             _ptr(ntri), _ptr(ws), ws.numel(), _ptr(flags), _stream(rec)),
           "dms_d0_triplets")
    check_flags(flags)
    k = int(ntri.item())
    te = np.ascontiguousarray(tri_edge[:k].cpu().numpy())
    t0 = np.ascontiguousarray(tri_min0[:k].cpu().numpy())
    t1 = np.ascontiguousarray(tri_min1[:k].cpu().numpy())
    mo = np.ascontiguousarray(min_order[:n0].cpu().numpy())
    c0 = crit0.cpu().numpy()
    cap = max(k, 1)
    pe = np.zeros(cap, np.int64)
    pm = np.zeros(cap, np.int32)
    npairs = np.zeros(1, np.int64)
    _check(L.dms_d0_pairs_sorted_host(te.ctypes.data_as(P), t0.ctypes.data_as(P), t1.ctypes.data_as(P),
                                      k, mo.ctypes.data_as(P), n0, pe.ctypes.data_as(P),
                                      pm.ctypes.data_as(P), cap, npairs.ctypes.data_as(P)),
           "dms_d0_pairs_sorted_host")
    m = int(npairs[0])
    return pe[:m], (c0[pm[:m]] >> 8).astype(np.int64)


def d2_pairs(rec, order_t, dims, crit2, crit3):
    """D2 pairing: ascents on the dual complex on the GPU (dms_d2_triplets:
    triplets by decreasing triangle, maxima ranked in filtration order), the
    union-find on the host (dms_d2_pairs_sorted_host).  rec/order_t/crit2/
    crit3 are device tensors of the whole grid.  Returns numpy (pair_tri
    codes, pair_tet codes)."""
    import torch
    _require_whole_grid(rec, order_t, dims, [("crit2", crit2), ("crit3", crit3)])
    L = lib()
    P = ctypes.c_void_p
    dev = rec.device
    n2, n3 = int(crit2.numel()), int(crit3.numel())
    d, dp = _arr3(dims)
    tri_code = torch.empty(max(n2, 1), dtype=torch.int64, device=dev)
    tri_max0 = torch.empty(max(n2, 1), dtype=torch.int32, device=dev)
    tri_max1 = torch.empty(max(n2, 1), dtype=torch.int32, device=dev)
    max_rank = torch.empty(max(n3, 1), dtype=torch.int32, device=dev)
    ntri = torch.zeros(1, dtype=torch.int64, device=dev)
    flags = new_flags(dev)
    ws = torch.empty(max(int(L.dms_d2_workspace_size(n2, n3)), 256), dtype=torch.uint8, device=dev)
    _check(L.dms_d2_triplets(_ptr(rec), _ptr(order_t), dp, _ptr(crit2), n2, _ptr(crit3), n3,
                             _ptr(tri_code), _ptr(tri_max0), _ptr(tri_max1), _ptr(max_rank),
                             _ptr(ntri), _ptr(ws), ws.numel(), _ptr(flags), _stream(rec)),
           "dms_d2_triplets")
    check_flags(flags)
    k = int(ntri.item())
    tc = np.ascontiguousarray(tri_code[:k].cpu().numpy())
    t0 = np.ascontiguousarray(tri_max0[:k].cpu().numpy())
    t1 = np.ascontiguousarray(tri_max1[:k].cpu().numpy())
    mr = np.ascontiguousarray(max_rank[:n3].cpu().numpy())
    c3 = crit3.cpu().numpy()
    cap = max(k, 1)
    pt = np.zeros(cap, np.int64)
    pm = np.zeros(cap, np.int32)
    npairs = np.zeros(1, np.int64)
    _check(L.dms_d2_pairs_sorted_host(tc.ctypes.data_as(P), t0.ctypes.data_as(P), t1.ctypes.data_as(P),
                                      k, mr.ctypes.data_as(P), n3, pt.ctypes.data_as(P),
                                      pm.ctypes.data_as(P), cap, npairs.ctypes.data_as(P)),
           "dms_d2_pairs_sorted_host")
    m = int(npairs[0])
    return pt[:m], c3[pm[:m]].astype(np.int64)


def gradient_pipeline(values, lo=None, hi=None, cap=None):
    """order -> discrete gradient -> critical simplices for one field (the
    gradient marks the records holding critical cells; the extraction reads
    only those)."""
    o = order(values)
    dims = dims_of(values)
    blo, bhi = _box(dims, lo, hi)
    mask = critical_mask(max(0, bhi[0] - blo[0]) * max(0, bhi[1] - blo[1]) * max(0, bhi[2] - blo[2]),
                         values.device)
    rec = discrete_gradient(o, lo, hi, mask=mask)
    lists, counts = critical_simplices(rec, dims, lo, hi, cap=cap, mask=mask)
    return o, rec, lists, counts


class Batch:
    """Batched form (dms_batch_*): many float32 fields of uneven sides.

    sides: sequence of (nx, ny, nz).  run(values) takes the fields
    concatenated in one GPU float32 tensor and returns the concatenated
    orders and records, the four critical lists (field after field, codes
    with field-local vertex ids), per-field counts [nfields, 4] and list
    offsets [4, nfields + 1].  Keep the output buffers (reuse=True) and the
    launches replay one captured hipGraph.
    """

    def __init__(self, sides, tune=False, cache=None, device=None):
        import torch
        L = lib()
        self.sides = np.ascontiguousarray(np.asarray(sides, dtype=np.int64).reshape(-1, 3))
        self.nfields = self.sides.shape[0]
        self.ptr = ctypes.c_void_p()
        c = cache.encode() if cache else None
        _check(L.dms_batch_create(self.sides.ctypes.data_as(ctypes.c_void_p), self.nfields, DMS_F32,
                                  int(bool(tune)), c, ctypes.byref(self.ptr)), "dms_batch_create")
        sizes = self.sides.prod(axis=1)
        self.off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        self.total = int(L.dms_batch_total(self.ptr))
        self.device = device or torch.device("cuda")
        self.ws = torch.empty(max(int(L.dms_batch_workspace_size(self.ptr)), 256), dtype=torch.uint8,
                              device=self.device)
        self.bufs = None

    @property
    def variant(self):
        return int(lib().dms_batch_variant(self.ptr))

    def _alloc(self, cap):
        import torch
        dev = self.device
        return dict(order=torch.empty(self.total, dtype=torch.int32, device=dev),
                    rec=torch.empty((self.total, 4), dtype=torch.int32, device=dev),
                    lists=[torch.empty(int(max(c, 0)), dtype=torch.int64, device=dev) for c in cap],
                    cap=np.ascontiguousarray(np.asarray(cap, dtype=np.int64).reshape(4)),
                    counts=torch.zeros(4 * self.nfields, dtype=torch.int64, device=dev),
                    offsets=torch.zeros(4 * (self.nfields + 1), dtype=torch.int64, device=dev),
                    flags=new_flags(dev))

    def launch(self, values, b):
        """Enqueues one run on the current stream into the buffers b (no sync)."""
        _require_gpu(values, "values")
        if values.numel() != self.total:
            raise ValueError("values must hold all fields concatenated (%d)" % self.total)
        lists = b["lists"]
        _check(lib().dms_batch_run(self.ptr, _ptr(values), _ptr(b["order"]), _ptr(b["rec"]),
                                   _ptr(lists[0]), _ptr(lists[1]), _ptr(lists[2]), _ptr(lists[3]),
                                   b["cap"].ctypes.data_as(ctypes.c_void_p), _ptr(b["counts"]),
                                   _ptr(b["offsets"]), _ptr(self.ws), self.ws.numel(),
                                   _ptr(b["flags"]), _stream(values)), "dms_batch_run")

    def run(self, values, cap=None, reuse=True):
        if cap is None and self.bufs is not None and reuse:
            b = self.bufs
        else:
            if cap is None:
                probe = self._alloc([0, 0, 0, 0])
                self.launch(values, probe)
                cap = probe["offsets"].view(4, self.nfields + 1)[:, -1].cpu().numpy()
            b = self._alloc(cap)
            self.bufs = b
        b["flags"].zero_()
        self.launch(values, b)
        check_flags(b["flags"])
        return (b["order"], b["rec"], b["lists"], b["counts"].view(self.nfields, 4),
                b["offsets"].view(4, self.nfields + 1))

    def __del__(self):
        try:
            if self.ptr:
                lib().dms_batch_destroy(self.ptr)
                self.ptr = ctypes.c_void_p()
        except Exception:
            pass


from .autograd import PersistenceD0, PersistenceD2  # noqa: E402  (torch autograd wrapper)
