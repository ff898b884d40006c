"""GPU parity of the batched form: every field of a batch must equal the
single-field oracle bit for bit, graph replays must repeat the first run, and
the full 96-field workload is checked field by field on properties and on
sampled records."""
import os
import sys

import numpy as np
import pytest

import oracle
import paper_2505_21266_amd as dms
from batch_cache import pin_variant
from paper_2505_21266_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dms.lib()


def _field(side, kind, seed):
    nx, ny, nz = side
    rng = np.random.default_rng(seed)
    if kind == 0:
        return rng.random((nz, ny, nx), dtype=np.float32)
    if kind == 1:
        return rng.integers(0, 5, (nz, ny, nx)).astype(np.float32)
    return inputs.mixture_field((nz, ny, nx), 4, rng, 1e-3, np.float32)


SIDES = [(5, 7, 3), (40, 33, 9), (17, 1, 4), (64, 9, 5), (3, 3, 3), (33, 20, 11), (1, 1, 1),
         (70, 6, 4), (2, 65, 3), (31, 31, 2), (9, 9, 9), (128, 3, 2)]


def _check_fields(sides, fields, order, rec, lists, counts, offsets):
    off = np.concatenate([[0], np.cumsum([int(np.prod(s)) for s in sides])])
    order = order.cpu().numpy()
    rec = rec.cpu().numpy().view(np.uint32)
    L = [l.cpu().numpy() for l in lists]
    counts = counts.cpu().numpy()
    offsets = offsets.cpu().numpy()
    for f, (s, v) in enumerate(zip(sides, fields)):
        o = oracle.order(v).reshape(-1)
        assert (order[off[f]:off[f + 1]] == o).all(), f
        want, wc, _ = oracle.lower_stars(o, s)
        assert (rec[off[f]:off[f + 1]] == want).all(), f
        crit, cnt = oracle.critical_simplices(want, s)
        assert (counts[f] == cnt).all(), f
        for d in range(4):
            assert (L[d][offsets[d, f]:offsets[d, f + 1]] == crit[d]).all(), (f, d)


def test_batch_exact_per_field():
    fields = [_field(s, i % 3, 100 + i) for i, s in enumerate(SIDES)]
    vals = torch.from_numpy(np.concatenate([f.reshape(-1) for f in fields])).cuda()
    b = dms.Batch(SIDES)
    out = b.run(vals)
    _check_fields(SIDES, fields, *out)


@pytest.mark.parametrize("variant", [0, 1, 2])
def test_batch_exact_each_tile_shape(variant, tmp_path):
    """Each of the three tile shapes, pinned through the tuning cache, on the
    ragged fields (noise tiles pair their general vertices in place, tiles
    of the smooth and tied fields queue them) and on 300 tiny fields."""
    fields = [_field(s, i % 3, 300 + i) for i, s in enumerate(SIDES)]
    vals = torch.from_numpy(np.concatenate([f.reshape(-1) for f in fields])).cuda()
    b = dms.Batch(SIDES, cache=pin_variant(tmp_path / "tune.txt", SIDES, variant))
    assert b.variant == variant
    _check_fields(SIDES, fields, *b.run(vals))
    rng = np.random.default_rng(78)
    sides = [tuple(int(x) for x in rng.integers(1, 7, 3)) for _ in range(300)]
    fields = [_field(s, i % 3, 1900 + i) for i, s in enumerate(sides)]
    vals = torch.from_numpy(np.concatenate([f.reshape(-1) for f in fields])).cuda()
    b = dms.Batch(sides, cache=pin_variant(tmp_path / "tune300.txt", sides, variant))
    assert b.variant == variant
    _check_fields(sides, fields, *b.run(vals))


def test_batch_many_fields():
    """More fields than one byte can index: the sort must group by the whole
    field index (a second field byte), or fields f and f + 256 would mix."""
    rng = np.random.default_rng(77)
    sides = [tuple(int(x) for x in rng.integers(1, 7, 3)) for _ in range(300)]
    fields = [_field(s, i % 3, 900 + i) for i, s in enumerate(sides)]
    vals = torch.from_numpy(np.concatenate([f.reshape(-1) for f in fields])).cuda()
    b = dms.Batch(sides)
    out = b.run(vals)
    _check_fields(sides, fields, *out)


def test_batch_graph_replay():
    fields = [_field(s, (i + 1) % 3, 200 + i) for i, s in enumerate(SIDES)]
    vals = torch.from_numpy(np.concatenate([f.reshape(-1) for f in fields])).cuda()
    b = dms.Batch(SIDES)
    first = [t.clone() if not isinstance(t, list) else [x.clone() for x in t] for t in b.run(vals)]
    for rep in range(3):
        # eager work in between, then replay
        junk = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        again = b.run(vals)
        assert torch.equal(first[0], again[0]) and torch.equal(first[1], again[1]), rep
        for d in range(4):
            assert torch.equal(first[2][d], again[2][d]), (rep, d)
        assert torch.equal(first[3], again[3]) and torch.equal(first[4], again[4])
    _check_fields(SIDES, fields, *again)


def test_batch_alternating_inputs():
    """Two different batches of values through one plan and one set of
    buffers, alternating: every run equals the oracle (nothing carries over
    from the previous run, e.g. through the queue of general vertices)."""
    fa = [_field(s, i % 3, 400 + i) for i, s in enumerate(SIDES)]
    fb = [_field(s, (i + 1) % 3, 500 + i) for i, s in enumerate(SIDES)]
    va = torch.from_numpy(np.concatenate([f.reshape(-1) for f in fa])).cuda()
    vb = torch.from_numpy(np.concatenate([f.reshape(-1) for f in fb])).cuda()
    b = dms.Batch(SIDES)
    cap = [1 << 16] * 4
    bufs = b._alloc(cap)
    for rep, (vals, fields) in enumerate([(va, fa), (vb, fb), (va, fa), (vb, fb)]):
        bufs["rec"].fill_(-1)
        bufs["flags"].zero_()
        b.launch(vals, bufs)
        dms.check_flags(bufs["flags"])
        out = (bufs["order"], bufs["rec"], bufs["lists"], bufs["counts"].view(b.nfields, 4),
               bufs["offsets"].view(4, b.nfields + 1))
        _check_fields(SIDES, fields, *out)


def test_batch_autotune_cache(tmp_path):
    path = str(tmp_path / "tune.txt")
    sides = SIDES[:6]
    fields = [_field(s, i % 3, 300 + i) for i, s in enumerate(sides)]
    vals = torch.from_numpy(np.concatenate([f.reshape(-1) for f in fields])).cuda()
    b = dms.Batch(sides, tune=True, cache=path)
    out = b.run(vals)
    v = b.variant
    assert v in (0, 1, 2)
    _check_fields(sides, fields, *out)
    lines = open(path).read().split("\n")
    assert len([x for x in lines if x.strip()]) == 1
    b2 = dms.Batch(sides, tune=True, cache=path)
    assert b2.variant == v  # taken from the cache, no second tuning run
    out2 = b2.run(vals)
    _check_fields(sides, fields, *out2)
    assert len([x for x in open(path).read().split("\n") if x.strip()]) == 1


def test_batch_config4_sampled():
    """The 96-field workload: per field, the order is a permutation sorted by
    (value, id), 400 sampled records equal the oracle's, and the Euler
    characteristic of the critical counts is 1."""
    fields, sides = inputs.config4()
    sides = [tuple(int(x) for x in s) for s in sides]
    vals = torch.from_numpy(np.concatenate([f.reshape(-1) for f in fields])).cuda()
    b = dms.Batch(sides)
    order, rec, lists, counts, offsets = b.run(vals)
    order = order.cpu().numpy()
    rec = rec.cpu().numpy().view(np.uint32)
    counts = counts.cpu().numpy()
    off = b.off
    rng = np.random.default_rng(9)
    for f, (s, v) in enumerate(zip(sides, fields)):
        o = order[off[f]:off[f + 1]]
        flat = v.reshape(-1)
        inv = np.full(flat.size, -1, np.int64)
        inv[o] = np.arange(flat.size)
        assert (inv >= 0).all(), f
        vs = flat[inv]
        assert (np.diff(vs) >= 0).all(), f
        ties = np.diff(vs) == 0
        assert (np.diff(inv)[ties] > 0).all(), f
        vids = rng.integers(0, flat.size, 400)
        want = oracle.lower_stars_sampled(v, s, vids)
        assert (rec[off[f] + vids] == want).all(), f
        c = counts[f]
        assert c[0] - c[1] + c[2] - c[3] == 1, f
