"""GPU parity at full size: the 512^3, 1026^3 and 96-field workloads compared
with the oracle record for record and list for list.

Robins' pairing reads only a vertex's 14 neighbours (Section 2.3), so the
records of a run of z-planes follow from those planes plus one plane of
halo on each side, and a local order of that slab has the same relative
order as the global one (ties by id: a slab of whole planes keeps the ids'
order).  The oracle therefore runs slab by slab, one slab per host thread,
and every owned record and every critical cell of the GPU run is compared.
"""
import concurrent.futures
import os
import sys

import numpy as np
import pytest

import oracle
import paper_2505_21266_amd as dms
from batch_cache import pin_variant
from paper_2505_21266_amd import inputs

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
torch = pytest.importorskip("torch")

WORKERS = max(1, min(16, len(os.sched_getaffinity(0))))


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dms.lib()
    oracle.star_tables()  # build the oracle's tables before threads use them
    yield
    torch.cuda.empty_cache()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _slab_oracle(field, z0, z1, box_xy):
    """Oracle records and critical lists of owned planes [z0, z1) of field
    (nz, ny, nx), owned x/y range box_xy = ((x0, x1), (y0, y1)); vertex ids
    in the lists are the whole field's."""
    nz, ny, nx = field.shape
    s0, s1 = max(z0 - 1, 0), min(z1 + 1, nz)
    sub = np.ascontiguousarray(field[s0:s1])
    dims = (nx, ny, s1 - s0)
    (x0, x1), (y0, y1) = box_xy
    lo, hi = (x0, y0, z0 - s0), (x1, y1, z1 - s0)
    o = oracle.order(sub, nthreads=1)
    rec, _, an = oracle.lower_stars(o, dims, lo, hi, nthreads=1)
    assert an == 0
    crit, _ = oracle.critical_simplices(rec, dims, lo, hi, nthreads=1)
    shift = np.int64(s0 * nx * ny) << 8
    return rec, [c + shift for c in crit]


def _compare_slabs(field, box, rec_gpu, lists_gpu, planes, z_range=None):
    """Compares the GPU records of the owned box (rec_gpu: device (nbox, 4)
    int32, box order) and the GPU critical lists (host int64 arrays) with the
    oracle, slab by slab over owned planes z_range."""
    nz, ny, nx = field.shape
    (x0, y0, zb0), (x1, y1, zb1) = box
    w0, w1 = x1 - x0, y1 - y0
    za, zb = z_range if z_range else (zb0, zb1)
    slabs = [(z, min(z + planes, zb)) for z in range(za, zb, planes)]
    maxv = [lst >> 8 for lst in lists_gpu]
    checked = 0
    with concurrent.futures.ThreadPoolExecutor(WORKERS) as ex:
        for g in range(0, len(slabs), WORKERS):
            group = slabs[g:g + WORKERS]
            futs = [ex.submit(_slab_oracle, field, z0, z1, ((x0, x1), (y0, y1))) for z0, z1 in group]
            for (z0, z1), fut in zip(group, futs):
                want_rec, want_crit = fut.result()
                r0, r1 = (z0 - zb0) * w0 * w1, (z1 - zb0) * w0 * w1
                got = rec_gpu[r0:r1].cpu().numpy().view(np.uint32)
                assert got.shape == want_rec.shape
                bad = np.nonzero((got != want_rec).any(axis=1))[0]
                assert bad.size == 0, ("records differ", z0, z1, int(bad[0]), got[bad[0]], want_rec[bad[0]])
                v0, v1 = z0 * nx * ny, z1 * nx * ny
                for d in range(4):
                    a, b = np.searchsorted(maxv[d], [v0, v1])
                    assert np.array_equal(lists_gpu[d][a:b], want_crit[d]), ("list", d, z0, z1)
                checked += r1 - r0
            _say("  planes %d..%d exact" % (group[0][0], group[-1][1]))
    return checked


def _check_mask(mask, lists, dims, lo, hi):
    """The critical mask flags exactly the max vertices of the listed cells
    (the lists themselves are compared with the oracle's)."""
    nx, ny, _ = dims
    w0, w1 = hi[0] - lo[0], hi[1] - lo[1]
    nbox = w0 * w1 * (hi[2] - lo[2])
    want = torch.zeros(nbox, dtype=torch.bool, device=mask.device)
    for lst in lists:
        v = lst >> 8
        x, y, z = v % nx, (v // nx) % ny, v // (nx * ny)
        want[(x - lo[0]) + w0 * ((y - lo[1]) + w1 * (z - lo[2]))] = True
    bits = torch.arange(32, device=mask.device, dtype=torch.int32)
    got = ((mask.view(-1, 1) >> bits) & 1).view(-1).bool()
    assert not got[nbox:].any()
    assert torch.equal(got[:nbox], want)


# ---------------------------------------------------------------- config 2

def test_config2_exact():
    """512^3, 64 Gaussians + noise: the order equals the oracle's (threaded
    sort), and every record and every critical cell equal the oracle's."""
    v = inputs.config2()
    nz, ny, nx = v.shape
    dims = (nx, ny, nz)
    _say("config2: GPU pass")
    vt = _dev(v)
    og = dms.order(vt)
    mask = dms.critical_mask(nx * ny * nz, vt.device)
    rg = dms.discrete_gradient(og, workspace=dms.gradient_workspace(og), mask=mask)
    lists, counts = dms.critical_simplices(rg, dims, mask=mask)
    _check_mask(mask, lists, dims, (0, 0, 0), dims)
    del vt
    o = oracle.order(v, nthreads=WORKERS)
    assert np.array_equal(og.cpu().numpy(), o)
    del o
    lists = [l.cpu().numpy() for l in lists]
    c = counts.cpu().numpy()
    assert c[0] - c[1] + c[2] - c[3] == 1
    n = _compare_slabs(v, ((0, 0, 0), dims), rg, lists, 32)
    assert n == nx * ny * nz
    # nothing outside the slabs: the lists hold exactly the compared cells
    assert [len(l) for l in lists] == [int(x) for x in c]


# ---------------------------------------------------------------- config 3

@pytest.fixture(scope="module")
def config3_gpu():
    """The 1026^3 block in the benchmark's launch configuration: GPU order
    of the whole block, records of the owned 1024^3 box with the queue,
    critical lists of the box."""
    v, lo, hi = inputs.config3()
    nz, ny, nx = v.shape
    dims = (nx, ny, nz)
    _say("config3: GPU pass")
    vt = _dev(v)
    og = dms.order(vt)
    del vt
    mask = dms.critical_mask((hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2]), og.device)
    rg = dms.discrete_gradient(og, lo, hi, workspace=dms.gradient_workspace(og, lo, hi), mask=mask)
    lists, counts = dms.critical_simplices(rg, dims, lo, hi, mask=mask)
    _check_mask(mask, lists, dims, lo, hi)
    del mask
    out = dict(v=v, lo=lo, hi=hi, order=og, rec=rg, lists=[l.cpu().numpy() for l in lists],
               counts=counts.cpu().numpy())
    yield out
    del out["order"], out["rec"]
    torch.cuda.empty_cache()


def test_config3_order_exact(config3_gpu):
    """The GPU order of all 1026^3 vertices equals the oracle's (a threaded
    sort of the 1.08e9 (value, id) pairs)."""
    o = oracle.order(config3_gpu["v"], nthreads=WORKERS)
    assert np.array_equal(config3_gpu["order"].cpu().numpy(), o)


C3_PARTS = 8


@pytest.mark.parametrize("part", range(C3_PARTS))
def test_config3_exact(config3_gpu, part):
    """Every owned record and every critical cell of the 1024^3 box, an
    eighth of the owned planes per case, equal the oracle's."""
    g = config3_gpu
    lo, hi = g["lo"], g["hi"]
    span = (hi[2] - lo[2]) // C3_PARTS
    za = lo[2] + part * span
    zb = hi[2] if part == C3_PARTS - 1 else za + span
    box = (lo, hi)
    n = _compare_slabs(g["v"], box, g["rec"], g["lists"], 8, (za, zb))
    assert n == (hi[0] - lo[0]) * (hi[1] - lo[1]) * (zb - za)
    if part == C3_PARTS - 1:
        c = g["counts"]
        assert [len(l) for l in g["lists"]] == [int(x) for x in c]


# ---------------------------------------------------------------- config 4

def _field_oracle(v, s):
    o = oracle.order(v, nthreads=1).reshape(-1)
    rec, _, an = oracle.lower_stars(o, s, nthreads=1)
    assert an == 0
    crit, cnt = oracle.critical_simplices(rec, s, nthreads=1)
    return o, rec, crit, cnt


@pytest.fixture(scope="module")
def config4_oracle():
    """The 96 fields and the oracle's order, records, critical lists and
    counts of each (one field per host thread)."""
    fields, sides = inputs.config4()
    sides = [tuple(int(x) for x in s) for s in sides]
    _say("config4: oracle")
    with concurrent.futures.ThreadPoolExecutor(WORKERS) as ex:
        want = list(ex.map(_field_oracle, fields, sides))
    return fields, sides, want


@pytest.mark.parametrize("variant", [None, 0, 1, 2])
def test_config4_exact(config4_oracle, variant, tmp_path):
    """The 96-field batch (one captured graph): every field's order, every
    record, every critical list and the per-field counts and offsets equal
    the oracle's, with the autotuned tile shape (None) and with each of the
    three tile shapes forced through the tuning cache."""
    fields, sides, want = config4_oracle
    vals = _dev(np.concatenate([f.reshape(-1) for f in fields]))
    cache = None
    if variant is not None:
        cache = pin_variant(tmp_path / "tune.txt", sides, variant)
    b = dms.Batch(sides, tune=variant is None, cache=cache)
    if variant is not None:
        assert b.variant == variant
    _say("config4: variant", b.variant)
    order, rec, lists, counts, offsets = b.run(vals)
    order = order.cpu().numpy()
    rec = rec.cpu().numpy().view(np.uint32)
    L = [l.cpu().numpy() for l in lists]
    counts = counts.cpu().numpy()
    offsets = offsets.cpu().numpy()
    off = b.off
    for f, (o, wrec, crit, cnt) in enumerate(want):
        assert np.array_equal(order[off[f]:off[f + 1]], o), f
        bad = np.nonzero((rec[off[f]:off[f + 1]] != wrec).any(axis=1))[0]
        assert bad.size == 0, ("records differ", f, int(bad[0]))
        assert (counts[f] == cnt).all(), f
        for d in range(4):
            assert np.array_equal(L[d][offsets[d, f]:offsets[d, f + 1]], crit[d]), (f, d)
    for d in range(4):
        assert offsets[d, -1] == counts[:, d].sum() == L[d].size
