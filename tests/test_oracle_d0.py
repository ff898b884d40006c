"""Pins of the oracle's D0 pairing (Algorithm 1 on the extremum graph,
Section 2.6) and of the differentiable form's loss gradient (Section 2.5)."""
import numpy as np
import pytest

import brute
import oracle
from paper_2505_21266_amd import inputs


def _run(v, dims):
    o = oracle.order(v)
    rec, counts, an = oracle.lower_stars(o, dims)
    assert an == 0
    crit, _ = oracle.critical_simplices(rec, dims)
    pe, pm = oracle.d0_pairs(o, rec, dims, crit[1])
    return o.reshape(-1), rec, counts, crit, pe, pm


@pytest.mark.parametrize("dims,seed", [((6, 6, 6), 1), ((9, 7, 8), 2), ((12, 12, 12), 3)])
@pytest.mark.parametrize("kind", ["noise", "mixture"])
def test_d0_equals_union_find(dims, seed, kind, tables):
    """DMS drops only zero-persistence pairs, so its D0 equals the textbook
    union-find D0 with those removed, simplex for simplex; a connected grid
    leaves exactly one minimum unpaired (the infinite class)."""
    nx, ny, nz = dims
    rng = np.random.default_rng(seed)
    if kind == "noise":
        v = rng.random((nz, ny, nx))
    else:
        v = inputs.mixture_field((nz, ny, nx), 5, rng, 1e-3, np.float64)
    o, rec, counts, crit, pe, pm = _run(v, dims)
    assert len(pe) == counts[0] - 1
    simp = brute.kuhn_simplices(dims)
    merges = brute.union_find_d0(o, simp)
    want = {(e, young) for e, young in merges if brute.maxv(o, e) != young}
    nb = tables["nb"]
    got = set()
    for code, m in zip(pe, pm):
        x, e = int(code) >> 8, int(code) & 255
        i, j, k = x % nx, (x // nx) % ny, x // (nx * ny)
        y = brute.vid(dims, i + nb[e][0], j + nb[e][1], k + nb[e][2])
        got.add((tuple(sorted((x, y))), int(m)))
    assert got == want


def test_loss_gradient_finite_differences():
    """The loss sum(pers^2 for pers < threshold) is an exact quadratic in the
    values while the order does not change, so central differences with a
    step below half the smallest value gap match the analytic gradient."""
    dims = (10, 9, 8)
    nx, ny, nz = dims
    v = inputs.min_gap_pass(np.random.default_rng(4).random((nz, ny, nx)) * 0.2)
    o, rec, counts, crit, pe, pm = _run(v, dims)
    loss, grad, keep = oracle.d0_loss_grad(v, pe, pm, threshold=0.05)
    assert keep.any()
    flat = v.reshape(-1)
    gap = np.diff(np.sort(flat)).min()
    eps = gap / 4
    idx = np.unique(np.concatenate([np.nonzero(grad)[0][:40], np.arange(0, flat.size, 37)]))
    for x in idx:
        vp = flat.copy(); vp[x] += eps
        vm = flat.copy(); vm[x] -= eps
        lp, _, _ = oracle.d0_loss_grad(vp, pe, pm, 0.05)
        lm, _, _ = oracle.d0_loss_grad(vm, pe, pm, 0.05)
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - grad[x]) <= 1e-6 * max(abs(grad[x]), 1e-3), (x, fd, grad[x])
    # the pairing itself is unchanged by the perturbation
    vp = flat.copy(); vp[idx[0]] += eps
    _, _, _, _, pe2, pm2 = _run(vp.reshape(nz, ny, nx), dims)
    assert (pe2 == pe).all() and (pm2 == pm).all()
