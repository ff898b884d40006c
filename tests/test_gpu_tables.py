"""Every configuration of the tabulated lower stars, on the GPU, against the
oracle (Section 2.3: a record depends only on which neighbours are lower
and on their relative order).

The library looks up, instead of running Robins' loop, the records of
three families of vertices (tests/star_families.py): 645,120 regular,
322,560 with one opposite pair wholly upper and 18,063,360 with one pair
wholly lower.  Each configuration becomes the 3x3x3 block around a target
vertex of one grid (targets 3 apart, so no two blocks' stars overlap),
labelled by an injective int32 order in which the target and its 14
neighbours carry the configuration's keys; the GPU gradient of the whole
grid is then compared, at every target, with the oracle's record of the
same 15 keys -- with and without the queue of general vertices.
"""
import sys

import numpy as np
import pytest

import oracle
import paper_2505_21266_amd as dms
import star_families as sf

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
torch = pytest.importorskip("torch")

BX = BY = 256


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dms.lib()
    yield
    torch.cuda.empty_cache()


def _grid_of(keys):
    """Labels (3 BZ, 3 BY, 3 BX) int32 placing configuration c at block
    (c % BX, (c // BX) % BY, c // (BX BY)), and the targets' vertex ids."""
    m = keys.shape[0]
    bz = -(-m // (BX * BY))
    nb = oracle.star_tables()["nb"]  # (dx, dy, dz) of neighbour e
    col = {}
    for e in range(14):
        dx, dy, dz = (int(t) for t in nb[e])
        col[(dx, dy, dz)] = 1 + e
    col[(0, 0, 0)] = 0
    c = np.arange(bz * BY * BX, dtype=np.int64)
    lab = np.empty((bz, 3, BY, 3, BX, 3), np.int32)
    spare = 15
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                # padding blocks (c >= m): the position index, any injective labels do
                k = np.full(c.size, (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1), np.int64)
                if (dx, dy, dz) in col:
                    k[:m] = keys[:, col[(dx, dy, dz)]]
                else:
                    k[:m] = spare
                    spare += 1
                lab[:, dz + 1, :, dy + 1, :, dx + 1] = (c * 27 + k).reshape(bz, BY, BX)
    assert spare == 27
    lab = lab.reshape(3 * bz, 3 * BY, 3 * BX)
    nx, ny = 3 * BX, 3 * BY
    cm = c[:m]
    tx, ty, tz = 3 * (cm % BX) + 1, 3 * ((cm // BX) % BY) + 1, 3 * (cm // (BX * BY)) + 1
    return lab, tx + nx * (ty + ny * tz)


@pytest.mark.parametrize("family", sf.FAMILIES)
def test_every_table_configuration(family):
    keys = sf.family_keys(family)
    assert keys.shape[0] == sf.SIZES[family]
    want = oracle.pls_batch(keys, nthreads=0)
    lab, targets = _grid_of(keys)
    _say(family, keys.shape[0], "configurations, grid", lab.shape)
    o = torch.from_numpy(lab).cuda()
    del lab
    idx = torch.from_numpy(targets).cuda()
    for queue in (True, False):
        rec = dms.discrete_gradient(o, queue=queue)
        got = rec[idx].cpu().numpy().view(np.uint32)
        del rec
        bad = np.nonzero((got != want).any(axis=1))[0]
        assert bad.size == 0, (family, queue, int(bad.size), keys[bad[0]].tolist(), got[bad[0]], want[bad[0]])
