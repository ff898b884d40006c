"""GPU parity: the HIP library against the CPU oracle on the same seeded inputs.

Integer outputs (orders, 128-bit records, critical codes) must be bit-exact;
the FP64 backward must match the oracle gradient to 1e-10 relative.
"""
import sys

import numpy as np
import pytest

import oracle
import paper_2505_21266_amd as dms
from paper_2505_21266_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dms.lib()
    yield


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _field(dims, kind, seed):
    nx, ny, nz = dims
    rng = np.random.default_rng(seed)
    if kind == "noise":
        return rng.random((nz, ny, nx), dtype=np.float32)
    if kind == "ties":
        return rng.integers(0, 5, (nz, ny, nx)).astype(np.float32)
    if kind == "mixture":
        return inputs.mixture_field((nz, ny, nx), 6, rng, 1e-3, np.float32)
    if kind == "f64":
        return inputs.mixture_field((nz, ny, nx), 6, rng, 1e-4, np.float64)
    if kind.startswith("ramp"):  # tilted ramp + uniform noise of the given amplitude
        k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        amp = float(kind[4:])
        return (i + 1.37 * j + 1.91 * k + amp * rng.random((nz, ny, nx))).astype(np.float32)
    raise ValueError(kind)


# ----------------------------------------------------------------- order

# 4096 and 8192 are the tile sizes of the last pass and of the float32
# passes before it; sizes around them leave one-item and one-short tiles
@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 4095, 4096, 4097, 8191, 8192, 8193, 12289, 16385, 100003])
@pytest.mark.parametrize("kind", ["noise", "ties"])
def test_order_sizes(n, kind):
    rng = np.random.default_rng(n)
    v = rng.random(n, dtype=np.float32) if kind == "noise" else rng.integers(0, 7, n).astype(np.float32)
    _say("order", n, kind)
    got = dms.order(_dev(v)).cpu().numpy()
    assert (got == oracle.order(v)).all()


@pytest.mark.parametrize("n,kind", [(5000, "noise"), (70001, "ties"), (262144, "noise")])
def test_order_f64(n, kind):
    rng = np.random.default_rng(7 + n)
    v = rng.random(n) if kind == "noise" else rng.integers(-3, 3, n).astype(np.float64)
    _say("order f64", n, kind)
    got = dms.order(_dev(v)).cpu().numpy()
    assert (got == oracle.order(v)).all()


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_order_special_values(dtype):
    v = np.array([0.0, -0.0, np.inf, -np.inf, 1.0, -0.0, 0.0, -1e-30, 1e-30, -np.inf, 5.0],
                 dtype=dtype)
    v = np.tile(v, 900)
    got = dms.order(_dev(v)).cpu().numpy()
    assert (got == oracle.order(v)).all()


# a NaN in the first and in the second half of an 8192-key tile (the halves
# are read by different threads of a 512-thread block), at a tile's last
# element, and in the ragged last tile
@pytest.mark.parametrize("at", [17, 4321, 8191, 8999])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_order_nan_flag(dtype, at):
    v = np.random.default_rng(3).random(9000).astype(dtype)
    v[at] = np.nan
    with pytest.raises(ValueError):
        dms.order(_dev(v))


def _check_order_gpu(v, o):
    """o is the order of v iff it is a permutation of [0, n) whose inverse
    lists v in (value, id) order: that order is unique."""
    n = v.numel()
    o = o.reshape(-1)
    assert int(o.min()) >= 0 and int(o.max()) < n
    inv = torch.full((n,), -1, dtype=torch.int64, device=v.device)
    inv[o.long()] = torch.arange(n, device=v.device)
    assert bool((inv >= 0).all())
    vs = v.reshape(-1)[inv]
    assert bool((vs[1:] >= vs[:-1]).all())
    ties = vs[1:] == vs[:-1]
    assert bool((inv[1:][ties] > inv[:-1][ties]).all())


# sizes past 2^22 take the two-level inversion (coarse id buckets, then a
# fine partition inside each), the rest the one-level one
@pytest.mark.parametrize("n,kind,dtype", [(4194305, "noise", np.float32),
                                          (16777216, "ties", np.float32),
                                          (33554467, "noise", np.float32),
                                          (4194305, "ties", np.float64)])
def test_order_two_level_inversion(n, kind, dtype):
    rng = np.random.default_rng(n + 5)
    v = rng.random(n).astype(dtype) if kind == "noise" else rng.integers(0, 1000, n).astype(dtype)
    _say("order two-level", n, kind, np.dtype(dtype).name)
    got = dms.order(_dev(v))
    assert (got.cpu().numpy() == oracle.order(v)).all()


def test_order_full_block():
    """The 1026^3 float32 block of 512 Gaussians plus noise (over 2^30
    vertices, so the widest inversion window), checked by the properties that
    fix the order uniquely."""
    v, _, _ = inputs.config3()
    _say("order full block", v.shape)
    vt = _dev(v)
    del v
    o = dms.order(vt)
    _check_order_gpu(vt, o)


def test_order_config1():
    v = inputs.config1()
    got = dms.order(_dev(v)).cpu().numpy()
    assert (got == oracle.order(v)).all()


def _critical_codes_of(rec4, v):
    """Critical cells of one decoded record as (dimension, code) pairs."""
    st = oracle.decode_record(rec4)
    out = []
    for c in np.nonzero(st == oracle.ST_CRIT)[0]:
        c = int(c)
        if c == oracle.CELL_X:
            out.append((0, v << 8))
        elif c < oracle.CELL_TRI0:
            out.append((1, (v << 8) | (c - oracle.CELL_EDGE0)))
        elif c < oracle.CELL_TET0:
            out.append((2, (v << 8) | (c - oracle.CELL_TRI0)))
        else:
            out.append((3, (v << 8) | (c - oracle.CELL_TET0)))
    return out


def test_gradient_full_block_sampled():
    """The 1024^3-owned workload in the launch configuration the benchmark
    times (GPU order of the 1026^3 block, records of the owned box, the
    queue): 60000 sampled owned vertices have the oracle's records (computed
    from the values), and the critical lists restricted to the sampled
    vertices are exactly the critical cells of those records."""
    v, lo, hi = inputs.config3()
    nz, ny, nx = v.shape
    dims = (nx, ny, nz)
    w = [hi[i] - lo[i] for i in range(3)]
    rng = np.random.default_rng(31)
    m = 60000
    bx, by, bz = (rng.integers(0, w[i], m) for i in range(3))
    vids = (bx + lo[0]) + nx * ((by + lo[1]) + ny * (bz + lo[2]))
    box_idx = bx + w[0] * (by + w[1] * bz)
    want = oracle.lower_stars_sampled(v, dims, vids)
    _say("full block sampled", v.shape, m)
    vt = _dev(v)
    del v
    o = dms.order(vt)
    del vt
    rec = dms.discrete_gradient(o, lo, hi, workspace=dms.gradient_workspace(o, lo, hi))
    got = rec[_dev(box_idx)].cpu().numpy().view(np.uint32)
    assert (got == want).all()
    lists, counts = dms.critical_simplices(rec, dims, lo, hi)
    sample = set(int(x) for x in vids)
    expect = [set() for _ in range(4)]
    for r4, x in zip(want, vids):
        for d, code in _critical_codes_of(r4, int(x)):
            expect[d].add(code)
    for d in range(4):
        c = lists[d].cpu().numpy()
        mine = set(int(x) for x in c[np.isin(c >> 8, vids)])
        assert mine == expect[d], d
    assert sum(len(e) for e in expect) > 50  # the sample reaches critical cells
    del rec, o


def test_config1_exact():
    """The 64^3 white-noise workload end to end: order, every record and the
    four critical lists equal the oracle's."""
    v = inputs.config1()
    dims = (64, 64, 64)
    o = oracle.order(v)
    rec, _, _ = oracle.lower_stars(o, dims)
    crit, _ = oracle.critical_simplices(rec, dims)
    _say("config1 exact")
    og = dms.order(_dev(v))
    assert (og.cpu().numpy() == o).all()
    rg = dms.discrete_gradient(og)
    assert (rg.cpu().numpy().view(np.uint32) == rec).all()
    lists, counts = dms.critical_simplices(rg, dims)
    for d in range(4):
        assert (lists[d].cpu().numpy() == np.asarray(crit[d], np.int64)).all(), d


def test_config2_sampled():
    """The 512^3 64-Gaussian workload: the order is the unique (value, id)
    sort, 60000 sampled records equal the oracle's (from the values), the
    critical lists restricted to the sample are exactly the critical cells of
    those records, and the Euler characteristic is 1."""
    v = inputs.config2()
    nz, ny, nx = v.shape
    dims = (nx, ny, nz)
    n = nx * ny * nz
    vids = np.random.default_rng(22).integers(0, n, 60000)
    want = oracle.lower_stars_sampled(v, dims, vids)
    _say("config2 sampled")
    vt = _dev(v)
    og = dms.order(vt)
    _check_order_gpu(vt, og)
    rg = dms.discrete_gradient(og)
    assert (rg[_dev(vids)].cpu().numpy().view(np.uint32) == want).all()
    lists, counts = dms.critical_simplices(rg, dims)
    c = counts.cpu().numpy()
    assert c[0] - c[1] + c[2] - c[3] == 1
    expect = [set() for _ in range(4)]
    for r4, x in zip(want, vids):
        for d, code in _critical_codes_of(r4, int(x)):
            expect[d].add(code)
    for d in range(4):
        codes = lists[d].cpu().numpy()
        assert set(int(x) for x in codes[np.isin(codes >> 8, vids)]) == expect[d], d
    assert sum(len(e) for e in expect) > 10


# -------------------------------------------------------------- gradient

GRAD_CASES = [
    ((64, 64, 64), "noise", 1),
    ((67, 5, 9), "noise", 2),
    ((130, 3, 2), "ties", 3),
    ((33, 17, 12), "mixture", 4),
    ((70, 9, 6), "ties", 5),
    ((1, 1, 1), "noise", 6),
    ((9, 1, 1), "noise", 7),
    ((1, 7, 1), "noise", 8),
    ((1, 1, 6), "ties", 9),
    ((5, 4, 1), "noise", 10),
    ((1, 5, 6), "noise", 11),
    ((65, 66, 3), "mixture", 12),
]


@pytest.mark.parametrize("dims,kind,seed", GRAD_CASES)
def test_gradient_records(dims, kind, seed):
    """Records from the oracle's order, and from the GPU order, both equal the
    oracle's records bit for bit."""
    v = _field(dims, kind, seed)
    o = oracle.order(v)
    want, counts, an = oracle.lower_stars(o, dims)
    assert an == 0
    _say("gradient", dims, kind)
    got = dms.discrete_gradient(_dev(o)).cpu().numpy().view(np.uint32)
    assert (got == want).all()
    og = dms.order(_dev(v))
    assert (og.cpu().numpy() == o).all()
    got2 = dms.discrete_gradient(og).cpu().numpy().view(np.uint32)
    assert (got2 == want).all()


def test_gradient_queue_paths():
    """A tilted ramp plus noise (about 15% of vertices outside the tables):
    interior tiles queue their general vertices until the queue (one vertex
    in 16) overflows, later ones pair them in place, the boundary planes'
    tiles are dense and pair in place too.  With and without the queue the
    records equal the oracle's."""
    nz, ny, nx = 40, 96, 160
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    v = (i + 1.37 * j + 1.91 * k + 2.5 * np.random.default_rng(5).random((nz, ny, nx)))
    v = v.astype(np.float32)
    o = oracle.order(v)
    want, _, _ = oracle.lower_stars(o, (nx, ny, nz))
    _say("gradient queue paths")
    og = _dev(o)
    for queue in (True, False):
        got = dms.discrete_gradient(og, queue=queue).cpu().numpy().view(np.uint32)
        assert (got == want).all(), queue


# the gradient straight from the values: (value, id) comparisons instead of
# ranks must give the same records -- ties (integer fields, +-0.0) exercise
# the id tie-break
VALUE_CASES = [
    ((64, 64, 64), "noise", 41),
    ((70, 9, 6), "ties", 42),
    ((33, 17, 12), "mixture", 43),
    ((45, 37, 29), "f64", 44),
    ((160, 96, 12), "ramp2.5", 45),
    ((9, 1, 1), "ties", 46),
]


@pytest.mark.parametrize("dims,kind,seed", VALUE_CASES)
def test_gradient_from_values(dims, kind, seed):
    v = _field(dims, kind, seed)
    o = oracle.order(v)
    want, _, _ = oracle.lower_stars(o, dims)
    _say("gradient from values", dims, kind)
    got = dms.discrete_gradient_values(_dev(v)).cpu().numpy().view(np.uint32)
    assert (got == want).all()
    got2 = dms.discrete_gradient_values(_dev(v), queue=False).cpu().numpy().view(np.uint32)
    assert (got2 == want).all()


def test_gradient_from_values_signed_zero_box():
    """-0.0 and +0.0 are one value (ties by id); an owned box of a ghosted
    block reads its ghosts."""
    dims = (30, 20, 10)
    rng = np.random.default_rng(47)
    v = rng.integers(-2, 3, (10, 20, 30)).astype(np.float32)
    v[v == 0] = np.where(rng.random(int((v == 0).sum())) < 0.5, -0.0, 0.0).astype(np.float32)
    lo, hi = (1, 1, 1), (29, 19, 9)
    o = oracle.order(v)
    want, _, _ = oracle.lower_stars(o, dims, lo, hi)
    got = dms.discrete_gradient_values(_dev(v), lo, hi).cpu().numpy().view(np.uint32)
    assert (got == want).all()


def test_gradient_from_values_nan_flag():
    v = np.random.default_rng(48).random((12, 12, 12)).astype(np.float32)
    v[5, 6, 7] = np.nan
    with pytest.raises(ValueError):
        dms.discrete_gradient_values(_dev(v))


@pytest.mark.parametrize("dims,lo,hi", [((20, 18, 16), (1, 2, 1), (19, 17, 15)),
                                        ((66, 10, 7), (1, 1, 1), (65, 9, 6)),
                                        ((30, 30, 30), (0, 0, 0), (30, 1, 30)),
                                        ((30, 30, 30), (5, 5, 5), (6, 6, 6))])
def test_gradient_owned_box(dims, lo, hi):
    v = _field(dims, "noise", 13)
    o = oracle.order(v)
    want, _, _ = oracle.lower_stars(o, dims, lo, hi)
    _say("box", dims, lo, hi)
    got = dms.discrete_gradient(_dev(o), lo, hi).cpu().numpy().view(np.uint32)
    assert (got == want).all()


def test_gradient_hand_worked_cube():
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "cube2_hand.json")))
    o = np.array(g["order"], np.int32).reshape(2, 2, 2)
    want, _, _ = oracle.lower_stars(o, (2, 2, 2))
    got = dms.discrete_gradient(_dev(o)).cpu().numpy().view(np.uint32)
    assert (got == want).all()


@pytest.mark.parametrize("case", ["full14", "lower11"])
@pytest.mark.parametrize("queue", [True, False])
def test_gradient_hand_worked_stars(case, queue):
    """The GPU record of the hand-worked 14- and 11-neighbour lower stars
    (tests/golden/star_hand.md) decodes to the hand-derived pairs and
    critical cells and equals the oracle's record, both when x's tile queues
    it and when the tile pairs it in place; the whole 3x3x3 grid matches the
    oracle too."""
    import json
    import os
    import brute
    tables = oracle.star_tables()
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "star_hand.json")))
    c = [x for x in g["cases"] if x["name"] == case][0]
    o = brute.hand_star_grid(g["rank_of_neighbour"], c["upper_ranks"], tables)
    want, _, _ = oracle.lower_stars(o, (3, 3, 3))
    got = dms.discrete_gradient(_dev(o), queue=queue).cpu().numpy().view(np.uint32)
    assert (got == want).all()
    pairs, crit = brute.record_rank_cells(got[13], g["rank_of_neighbour"], tables)
    assert pairs == {(tuple(t), tuple(h)) for t, h in c["pairs"]}
    assert crit == {tuple(x) for x in c["critical"]}
    box = dms.discrete_gradient(_dev(o), (1, 1, 1), (2, 2, 2), queue=queue).cpu().numpy().view(np.uint32)
    assert (box[0] == want[13]).all()


# -------------------------------------------------------------- critical

@pytest.mark.parametrize("dims,kind,seed,box", [
    ((64, 64, 64), "noise", 1, None),
    ((40, 31, 22), "ties", 2, None),
    ((45, 37, 29), "mixture", 3, None),
    ((34, 34, 34), "noise", 4, ((1, 1, 1), (33, 33, 33))),
    ((3, 3, 3), "noise", 5, None),
    ((7, 1, 1), "noise", 6, None),
    # extraction tiles with few, about kCand and many records holding
    # critical cells (listed, listed up to the limit, re-read whole)
    ((128, 64, 24), "ramp1.2", 7, None),
    ((128, 64, 24), "ramp4.0", 8, None),
    ((128, 64, 24), "ramp6.0", 9, ((1, 1, 1), (127, 63, 23))),
])
def test_critical_lists(dims, kind, seed, box):
    v = _field(dims, kind, seed)
    lo, hi = box if box else (None, None)
    o = oracle.order(v)
    rec, counts, _ = oracle.lower_stars(o, dims, lo, hi)
    want, wcount = oracle.critical_simplices(rec, dims, lo, hi)
    _say("critical", dims, kind, box)
    _, grec, lists, gcounts = dms.gradient_pipeline(_dev(v), lo, hi)
    assert (grec.cpu().numpy().view(np.uint32) == rec).all()
    assert (gcounts.cpu().numpy() == wcount).all()
    for d in range(4):
        assert (lists[d].cpu().numpy() == want[d]).all(), d
    if box is None:
        c = wcount
        assert c[0] - c[1] + c[2] - c[3] == 1


def _mask_bits(mask, nbox):
    """The first nbox bits of a critical mask (bit r % 32 of word r / 32)."""
    b = np.unpackbits(mask.cpu().numpy().view(np.uint8), bitorder="little")
    assert not b[nbox:].any()
    return b[:nbox].astype(bool)


def _records_with_critical(lists, dims, lo, hi):
    """Box records (box order) that hold a critical cell: the max vertices
    of the oracle's critical cells."""
    nx, ny, _ = dims
    (x0, y0, z0), (x1, y1, z1) = lo, hi
    w0, w1 = x1 - x0, y1 - y0
    out = np.zeros(w0 * w1 * (z1 - z0), bool)
    for lst in lists:
        v = np.asarray(lst, np.int64) >> 8
        x, y, z = v % nx, (v // nx) % ny, v // (nx * ny)
        out[(x - x0) + w0 * ((y - y0) + w1 * (z - z0))] = True
    return out


MASK_CASES = [(c[0], c[1], c[2], None) for c in GRAD_CASES] + [
    ((34, 34, 34), "noise", 4, ((1, 1, 1), (33, 33, 33))),
    ((128, 64, 24), "ramp1.2", 7, None),
    ((128, 64, 24), "ramp6.0", 9, ((1, 1, 1), (127, 63, 23))),
    ((45, 37, 29), "f64", 44, ((2, 0, 3), (41, 37, 27))),
    ((160, 96, 12), "ramp2.5", 45, None),
]


@pytest.mark.parametrize("dims,kind,seed,box", MASK_CASES)
def test_critical_mask(dims, kind, seed, box):
    """The gradient's critical mask has exactly the bits of the records that
    hold a critical cell (from the oracle's lists), on the order path with
    and without the queue and on the values path; the extraction reading
    only flagged records gives the oracle's lists and counts."""
    v = _field(dims, kind, seed)
    lo, hi = box if box else ((0, 0, 0), dims)
    o = oracle.order(v)
    rec, _, _ = oracle.lower_stars(o, dims, lo, hi)
    want, wcount = oracle.critical_simplices(rec, dims, lo, hi)
    want_bits = _records_with_critical(want, dims, lo, hi)
    nbox = want_bits.size
    _say("critical mask", dims, kind, box)
    vt, ot = _dev(v), _dev(o)
    for path in ("order", "order-noqueue", "values"):
        mask = dms.critical_mask(nbox, vt.device)
        mask.fill_(-1)  # every word is written by the gradient call
        if path == "values":
            grec = dms.discrete_gradient_values(vt, lo, hi, mask=mask)
        else:
            grec = dms.discrete_gradient(ot, lo, hi, queue=path == "order", mask=mask)
        assert (grec.cpu().numpy().view(np.uint32) == rec).all(), path
        assert np.array_equal(_mask_bits(mask, nbox), want_bits), path
        lists, counts = dms.critical_simplices(grec, dims, lo, hi, mask=mask)
        assert (counts.cpu().numpy() == wcount).all(), path
        for d in range(4):
            assert np.array_equal(lists[d].cpu().numpy(), want[d]), (path, d)


def test_critical_mask_capacity_and_noalloc():
    """With the mask, truncated lists and the allocation-free extraction
    still equal the unmasked results."""
    dims = (40, 40, 40)
    v = _field(dims, "noise", 22)
    o = oracle.order(v)
    rec, _, _ = oracle.lower_stars(o, dims)
    want, wcount = oracle.critical_simplices(rec, dims)
    mask = dms.critical_mask(40 ** 3, torch.device("cuda"))
    grec = dms.discrete_gradient(_dev(o), mask=mask)
    cap = [max(int(c) // 2, 1) for c in wcount]
    flags = dms.new_flags(torch.device("cuda"))
    lists, counts = dms.critical_simplices(grec, dims, cap=cap, flags=flags, mask=mask)
    assert int(flags.item()) & dms.FLAG_CAPACITY
    assert (counts.cpu().numpy() == wcount).all()
    for d in range(4):
        assert (lists[d].cpu().numpy() == want[d][: cap[d]]).all()
    full = [int(c) for c in wcount]
    lists, counts = dms.critical_simplices_noalloc(grec, dims, full, mask=mask)
    torch.cuda.synchronize()
    assert (counts.cpu().numpy() == wcount).all()
    for d in range(4):
        assert (lists[d].cpu().numpy() == want[d]).all()


def test_critical_mask_too_small_is_refused():
    rec = torch.zeros((65, 4), dtype=torch.int32, device="cuda")
    with pytest.raises(ValueError):
        dms.critical_simplices(rec, (65, 1, 1), mask=dms.critical_mask(32, rec.device))


def test_critical_capacity_flag():
    dims = (40, 40, 40)
    v = _field(dims, "noise", 21)
    o = oracle.order(v)
    rec, _, _ = oracle.lower_stars(o, dims)
    want, wcount = oracle.critical_simplices(rec, dims)
    cap = [max(int(c) // 2, 1) for c in wcount]
    flags = dms.new_flags(torch.device("cuda"))
    lists, counts = dms.critical_simplices(_dev(rec.view(np.int32)), dims, cap=cap, flags=flags)
    f = int(flags.item())
    assert f & dms.FLAG_CAPACITY
    assert (counts.cpu().numpy() == wcount).all()
    for d in range(4):
        assert (lists[d].cpu().numpy() == want[d][: cap[d]]).all()


def test_critical_empty_box():
    dims = (8, 8, 8)
    rec = torch.zeros((0, 4), dtype=torch.int32, device="cuda")
    lists, counts = dms.critical_simplices(rec, dims, (2, 2, 2), (2, 5, 5))
    assert counts.cpu().numpy().tolist() == [0, 0, 0, 0]


def test_determinism_double_run():
    dims = (50, 41, 33)
    v = _dev(_field(dims, "ties", 31))
    a = dms.gradient_pipeline(v)
    b = dms.gradient_pipeline(v)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    for d in range(4):
        assert torch.equal(a[2][d], b[2][d])


# -------------------------------------------------------------- backward

@pytest.mark.parametrize("shape", [(20, 22, 24), (32, 32, 32), "config5"])
def test_backward_matches_oracle(shape):
    """Pairs, loss and gradient of the differentiable form against the
    oracle; "config5" is the full 128^3 float64 workload."""
    if shape == "config5":
        f = inputs.config5()
        shape = f.shape
    else:
        rng = np.random.default_rng(41)
        f = inputs.min_gap_pass(inputs.mixture_field(shape, 6, rng, 1e-4, np.float64))
    nz, ny, nx = shape
    dims = (nx, ny, nz)
    o = oracle.order(f)
    rec, _, _ = oracle.lower_stars(o, dims)
    crit, _ = oracle.critical_simplices(rec, dims)
    pe, pm = oracle.d0_pairs(o, rec, dims, crit[1])
    loss_o, grad_o, _ = oracle.d0_loss_grad(f, pe, pm, 0.05)
    x = _dev(f).requires_grad_(True)
    births, deaths = dms.PersistenceD0.apply(x)
    assert (births.detach().cpu().numpy() == f.reshape(-1)[pm]).all()
    assert (deaths.detach().cpu().numpy() == f.reshape(-1)[pe >> 8]).all()
    from paper_2505_21266_amd.autograd import d0_loss
    loss = d0_loss(births, deaths, 0.05)
    loss.backward()
    g = x.grad.cpu().numpy().reshape(-1)
    assert abs(float(loss.detach()) - loss_o) <= 1e-12 * max(1.0, abs(loss_o))
    scale = np.abs(grad_o).max()
    assert np.all(np.abs(g - grad_o) <= 1e-10 * np.maximum(np.abs(grad_o), 1e-300) + 1e-300)
    assert scale > 0


@pytest.mark.parametrize("shape,kind,seed", [((24, 20, 16), "noise", 61), ((32, 32, 32), "f64", 62),
                                             ((18, 30, 9), "ties", 63), ((40, 1, 7), "noise", 64)])
def test_d0_pairs_gpu_matches_oracle(shape, kind, seed):
    """GPU extremum graph + host union-find give the oracle's D0 pairs, in
    the same order (Section 2.6, Algorithm 1)."""
    nz, ny, nx = shape
    v = _field((nx, ny, nz), kind, seed)
    if kind == "f64":
        v = inputs.min_gap_pass(v)
    dims = (nx, ny, nz)
    o = oracle.order(v)
    rec, _, _ = oracle.lower_stars(o, dims)
    crit, _ = oracle.critical_simplices(rec, dims)
    pe_o, pm_o = oracle.d0_pairs(o, rec, dims, crit[1])
    _say("d0 gpu", shape, kind)
    og = dms.order(_dev(v))
    rg = dms.discrete_gradient(og)
    lists, counts = dms.critical_simplices(rg, dims)
    pe, pm = dms.d0_pairs(rg, og, dims, lists[0], lists[1])
    assert (pe == pe_o).all() and (pm == pm_o).all()
    assert len(pe) == len(crit[0]) - 1  # every minimum but one dies (one component)


@pytest.mark.parametrize("shape,kind,seed", [((24, 20, 16), "noise", 71), ((32, 32, 32), "f64", 72),
                                             ((18, 30, 9), "ties", 73), ((40, 1, 7), "noise", 74),
                                             ((33, 17, 65), "mixture", 75), ((96, 96, 96), "noise", 76)])
def test_critical_sort_matches_oracle(shape, kind, seed):
    """Critical lists of every dimension in filtration order (Section 2.1),
    from a scrambled input order, bit-exact against the oracle."""
    nz, ny, nx = shape
    v = _field((nx, ny, nz), kind, seed)
    dims = (nx, ny, nz)
    o = oracle.order(v)
    rec, _, _ = oracle.lower_stars(o, dims)
    crit, _ = oracle.critical_simplices(rec, dims)
    _say("critical sort", shape, kind, [len(c) for c in crit])
    og = dms.order(_dev(v))
    rg = dms.discrete_gradient(og)
    lists, counts = dms.critical_simplices(rg, dims)
    prng = np.random.default_rng(seed)
    for d in range(4):
        c = np.asarray(crit[d], np.int64)
        assert (lists[d].cpu().numpy() == c).all()
        p = prng.permutation(c.size)
        want = oracle.filtration_sort(o, dims, c[p], d)
        got = dms.critical_sort(lists[d][_dev(p)], d, og, dims).cpu().numpy()
        assert (got == want).all(), d


def test_critical_sort_edge_cases():
    dims = (9, 8, 7)
    v = _field(dims, "noise", 81)
    o = oracle.order(v)
    og = dms.order(_dev(v))
    empty = torch.empty(0, dtype=torch.int64, device="cuda")
    assert dms.critical_sort(empty, 2, og, dims).numel() == 0
    one = _dev(np.array([(5 << 8) | 0], np.int64))
    assert dms.critical_sort(one, 0, og, dims).cpu().tolist() == [5 << 8]
    # every vertex (a long list through all radix passes) against the oracle
    n = 9 * 8 * 7
    ids = np.random.default_rng(82).permutation(n).astype(np.int64) << 8
    got = dms.critical_sort(_dev(ids), 0, og, dims).cpu().numpy()
    assert (got == oracle.filtration_sort(o, dims, ids, 0)).all()
    # a code that names no cell: flagged, no fault
    bad = _dev(np.array([(3 << 8) | 1, (4 << 8) | 40], np.int64))
    with pytest.raises(ValueError):
        dms.critical_sort(bad, 2, og, dims)
    corner = _dev(np.array([((n - 1) << 8) | 13], np.int64))  # neighbour +(1,1,1) of the last vertex
    with pytest.raises(ValueError):
        dms.critical_sort(corner, 1, og, dims)


@pytest.mark.parametrize("shape,kind,seed", [((24, 20, 16), "noise", 91), ((32, 32, 32), "f64", 92),
                                             ((18, 30, 9), "ties", 93), ((40, 7, 1), "noise", 94),
                                             ((20, 1, 13), "noise", 95), ((48, 40, 36), "mixture", 96)])
def test_d2_pairs_gpu_matches_oracle(shape, kind, seed):
    """GPU dual ascents + host union-find give the oracle's D2 pairs, in the
    same order; every maximum is paired."""
    nz, ny, nx = shape
    v = _field((nx, ny, nz), kind, seed)
    if kind == "f64":
        v = inputs.min_gap_pass(v)
    dims = (nx, ny, nz)
    o = oracle.order(v)
    rec, _, _ = oracle.lower_stars(o, dims)
    crit, _ = oracle.critical_simplices(rec, dims)
    pt_o, pq_o = oracle.d2_pairs(o, rec, dims, crit[2], crit[3])
    _say("d2 gpu", shape, kind, len(crit[2]), len(crit[3]))
    og = dms.order(_dev(v))
    rg = dms.discrete_gradient(og)
    lists, counts = dms.critical_simplices(rg, dims)
    pt, pq = dms.d2_pairs(rg, og, dims, lists[2], lists[3])
    assert (pt == pt_o).all() and (pq == pq_o).all()
    assert len(pq) == len(crit[3])


def _densest_box(mask, side=16):
    """Corner (k, j, i) of the side^3 box holding the most True entries of a
    (nz, ny, nx) mask; ties go to the smallest corner id."""
    c = np.zeros(tuple(d + 1 for d in mask.shape), np.int64)
    c[1:, 1:, 1:] = mask.astype(np.int64).cumsum(0).cumsum(1).cumsum(2)
    s = side
    box = (c[s:, s:, s:] - c[:-s, s:, s:] - c[s:, :-s, s:] - c[s:, s:, :-s]
           + c[:-s, :-s, s:] + c[:-s, s:, :-s] + c[s:, :-s, :-s] - c[:-s, :-s, :-s])
    best = np.flatnonzero(box.reshape(-1) == box.max())[0]  # C order: smallest corner id first
    return np.unravel_index(best, box.shape), int(box.max())


def test_d0_finite_differences_config5():
    """The differentiable form on the 128^3 float64 workload against finite
    differences of the loss (Section 2.5), on the 16^3 sub-grid holding the
    most vertices with a non-zero gradient.  The step eps is a quarter of the
    smallest value gap, so the vertex order and with it every pair is
    unchanged -- checked by re-running the GPU forward at +-eps for every
    sub-grid vertex with a non-zero gradient and random others (at least
    256), whose pair lists must be identical.  Over those unchanged pairs the
    loss is an exact quadratic, and for all 4096 sub-grid vertices the
    central difference, taken term by term in exact rational arithmetic over
    the pairs the vertex enters, matches the GPU gradient to 1e-8 relative.
    The whole-loss difference (math.fsum) is checked to 1e-4 relative, the
    floor its rounding sets."""
    import math
    from fractions import Fraction
    from paper_2505_21266_amd.autograd import d0_loss
    f = inputs.config5()
    nz, ny, nx = f.shape
    dims = (nx, ny, nz)
    flat = f.reshape(-1)
    eps = float(np.diff(np.sort(flat)).min()) / 4
    assert eps > 0
    x = _dev(f).requires_grad_(True)
    births, deaths = dms.PersistenceD0.apply(x)
    d0_loss(births, deaths, 0.05).backward()
    g = x.grad.cpu().numpy().reshape(-1)

    def pairs_at(v):
        og = dms.order(_dev(v))
        rg = dms.discrete_gradient(og)
        lists, _ = dms.critical_simplices(rg, dims)
        return dms.d0_pairs(rg, og, dims, lists[0], lists[1])

    pe, pm = pairs_at(f)
    pers = flat[pe >> 8] - flat[pm]
    assert np.all(np.abs(pers - 0.05) > 2 * eps)  # the threshold set cannot change either
    (k0, j0, i0), nnz = _densest_box((g != 0).reshape(f.shape))
    k, j, i = np.meshgrid(np.arange(k0, k0 + 16), np.arange(j0, j0 + 16), np.arange(i0, i0 + 16), indexing="ij")
    sub = (i + nx * (j + ny * k)).reshape(-1)
    nonzero = sub[g[sub] != 0]
    assert nonzero.size == nnz and nnz > 0
    _say("fd config5: box", (i0, j0, k0), nnz, "non-zero vertices")
    rng = np.random.default_rng(51)
    zero = sub[g[sub] == 0]
    extra = rng.choice(zero, max(256 - nonzero.size, 32), replace=False)
    for vid in np.concatenate([nonzero, extra]):
        for sgn in (1.0, -1.0):
            vp = flat.copy()
            vp[vid] += sgn * eps
            qe, qm = pairs_at(vp.reshape(f.shape))
            assert np.array_equal(qe, pe) and np.array_equal(qm, pm), (int(vid), sgn)
    # term-wise central differences over the unchanged pairs, exactly
    death_v, birth_v = (pe >> 8).astype(np.int64), pm.astype(np.int64)
    keep = pers < 0.05
    by_vertex = {}
    for p in np.flatnonzero(keep):
        by_vertex.setdefault(int(death_v[p]), []).append(p)
        by_vertex.setdefault(int(birth_v[p]), []).append(p)
    for vid in sub:
        vid = int(vid)
        fd = Fraction(0)
        up, dn = flat[vid] + eps, flat[vid] - eps
        h = Fraction(up) - Fraction(dn)
        for p in by_vertex.get(vid, []):
            d, b = int(death_v[p]), int(birth_v[p])
            fp = {d: Fraction(flat[d]), b: Fraction(flat[b])}
            fm = dict(fp)
            fp[vid], fm[vid] = Fraction(up), Fraction(dn)
            fd += ((fp[d] - fp[b]) ** 2 - (fm[d] - fm[b]) ** 2) / h
        assert abs(float(fd) - g[vid]) <= 1e-8 * max(abs(g[vid]), 1e-6), (vid, float(fd), g[vid])
    # the whole loss, on a few of them, from the GPU forward at +-eps
    def loss_at(v):
        with torch.no_grad():
            b, d = dms.PersistenceD0.apply(_dev(v.reshape(f.shape)))
            p = (d - b).cpu().numpy()
            return math.fsum((p[p < 0.05] ** 2).tolist())

    for vid in nonzero[:24]:
        vp = flat.copy(); vp[vid] += eps
        vm = flat.copy(); vm[vid] -= eps
        fd = (loss_at(vp) - loss_at(vm)) / (vp[vid] - vm[vid])
        assert abs(fd - g[vid]) <= 1e-4 * max(abs(g[vid]), 1e-3), (int(vid), fd, g[vid])


def test_d2_backward_config5():
    """The differentiable D2 form on the 128^3 float64 workload: births and
    deaths are the highest-vertex values of the oracle's pairs, and the
    gradient of sum(pers^2) lands on those vertices exactly."""
    f = inputs.config5()
    nz, ny, nx = f.shape
    dims = (nx, ny, nz)
    o = oracle.order(f)
    rec, _, _ = oracle.lower_stars(o, dims)
    crit, _ = oracle.critical_simplices(rec, dims)
    pt, pq = oracle.d2_pairs(o, rec, dims, crit[2], crit[3])
    flat = f.reshape(-1)
    pers = flat[pq >> 8] - flat[pt >> 8]
    want = np.zeros(flat.size)
    np.add.at(want, pq >> 8, 2 * pers)
    np.add.at(want, pt >> 8, -2 * pers)
    x = _dev(f).requires_grad_(True)
    births, deaths = dms.PersistenceD2.apply(x)
    assert (births.detach().cpu().numpy() == flat[pt >> 8]).all()
    assert (deaths.detach().cpu().numpy() == flat[pq >> 8]).all()
    ((deaths - births) ** 2).sum().backward()
    g = x.grad.cpu().numpy().reshape(-1)
    # sums of at most a few terms per vertex, in another order: relative 1e-10,
    # with an absolute floor for sums that cancel
    assert np.all(np.abs(g - want) <= 1e-10 * np.abs(want) + 1e-14 * np.abs(want).max())
    assert np.abs(want).max() > 0


def test_backward_fixed_summation_order():
    """Contributions to one vertex from births and deaths of pairs listed in
    any order are summed in one fixed order -- the births by pair index,
    then the deaths by pair index -- with values for which another order
    gives another double; vertices named by no pair get zero, codes outside
    the grid are dropped."""
    bv = np.array([3, 9, 7, 1, 4, 7, 55], np.int64)   # vertex 55 is outside n = 40
    dv = np.array([7, 2, 7, 7, 9, 6, 3], np.int64)
    gb = np.array([0.5, 2.0, 1e16, -3.0, 0.25, 1.0, 8.0])
    gd = np.array([-1e16, 4.0, 1.0, 1.0, 1e-3, -2.0, 0.125])
    want = np.zeros(40)
    for v in range(40):
        acc = 0.0
        for p in range(bv.size):
            if bv[p] == v:
                acc += gb[p]
        for p in range(dv.size):
            if dv[p] == v:
                acc += gd[p]
        want[v] = acc
    assert want[7] == 2.0  # ((1e16 + 1) - 1e16) + 1 + 1 in this order; other orders differ
    got = dms.gradient_backward(_dev(bv << 8), _dev((dv << 8) | 5), _dev(gb), _dev(gd), 40).cpu().numpy()
    assert np.array_equal(got, want)


def test_d2_backward_deterministic():
    """Two runs of the D2 form on the 128^3 float64 workload give bitwise
    equal gradients (triangles and tets can share a max vertex, out of pair
    order)."""
    f = inputs.config5()
    grads = []
    for _ in range(2):
        x = _dev(f).requires_grad_(True)
        births, deaths = dms.PersistenceD2.apply(x)
        ((deaths - births) ** 2).sum().backward()
        grads.append(x.grad.cpu().numpy().copy())
    assert np.array_equal(grads[0].view(np.uint64), grads[1].view(np.uint64))


def test_backward_kernel_runs():
    # several deaths on one vertex, given adjacent: summed in pair order
    bc = _dev(np.array([5 << 8, 9 << 8, 11 << 8], np.int64))
    dc = _dev(np.array([(20 << 8) | 1, (20 << 8) | 4, (30 << 8) | 2], np.int64))
    gb = _dev(np.array([1.0, 2.0, 3.0]))
    gd = _dev(np.array([0.5, 0.25, -1.0]))
    g = dms.gradient_backward(bc, dc, gb, gd, 40).cpu().numpy()
    want = np.zeros(40)
    want[[5, 9, 11]] = [1.0, 2.0, 3.0]
    want[20] = 0.75
    want[30] = -1.0
    assert (g == want).all()
