"""The paper's largest shape, 2048 x 1920 x 1536 (6.04e9 vertices, beyond
int32 orders), on one GPU through the path that needs no order: the gradient
from the float32 values and the extraction.  60000 sampled vertices have the
oracle's records (computed from the values), the critical lists
restricted to them are exactly the critical cells of those records, and the
critical mask flags exactly those of them that hold one (the launch
configuration of the benchmark's --large line)."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import oracle  # noqa: E402
import paper_2505_21266_amd as dms  # noqa: E402
from paper_2505_21266_amd import inputs  # noqa: E402

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_values_path_at_the_paper_largest_shape():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("generating 2048x1920x1536", flush=True)
    v = inputs.config_large()
    nz, ny, nx = v.shape
    dims = (nx, ny, nz)
    n = nx * ny * nz
    assert n > 2 ** 32  # record indices past 32 bits
    rng = np.random.default_rng(61)
    vids = rng.integers(0, n, 60000)
    vids[:8] = [0, n - 1, 2 ** 31, 2 ** 32 - 1, 2 ** 32, 2 ** 32 + 12345, n - nx, nx * ny * (nz - 1)]
    want = oracle.lower_stars_sampled(v, dims, vids)
    print("oracle sampled done", flush=True)
    vt = torch.from_numpy(v).cuda()
    del v
    mask = dms.critical_mask(n, vt.device)
    rec = dms.discrete_gradient_values(vt, check=True, mask=mask)
    lists, counts = dms.critical_simplices(rec, dims, mask=mask)
    c = counts.cpu().numpy()
    print("critical counts", c.tolist(), flush=True)
    assert c[0] - c[1] + c[2] - c[3] == 1  # Euler characteristic of the ball
    got = rec[torch.from_numpy(vids).cuda()].cpu().numpy().view(np.uint32)
    assert (got == want).all()
    expect = [set() for _ in range(4)]
    for r4, x in zip(want, vids):
        st = oracle.decode_record(r4)
        for cell in np.nonzero(st == oracle.ST_CRIT)[0]:
            cell = int(cell)
            x = int(x)
            if cell == oracle.CELL_X:
                expect[0].add(x << 8)
            elif cell < oracle.CELL_TRI0:
                expect[1].add((x << 8) | (cell - oracle.CELL_EDGE0))
            elif cell < oracle.CELL_TET0:
                expect[2].add((x << 8) | (cell - oracle.CELL_TRI0))
            else:
                expect[3].add((x << 8) | (cell - oracle.CELL_TET0))
    for d in range(4):
        codes = lists[d].cpu().numpy()
        mine = set(int(x) for x in codes[np.isin(codes >> 8, vids)])
        assert mine == expect[d], d
    assert sum(len(e) for e in expect) > 20
    # the critical mask flags exactly the sampled records that hold a critical cell
    vt_ids = torch.from_numpy(vids).cuda()
    words = mask[vt_ids >> 5].cpu().numpy().view(np.uint32)
    bits = (words >> (vids & 31).astype(np.uint32)) & 1
    has = set()
    for d in range(4):
        has |= set(c >> 8 for c in expect[d])
    assert [bool(b) for b in bits] == [int(x) in has for x in vids]
