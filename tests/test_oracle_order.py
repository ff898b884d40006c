"""Pins of the oracle's global vertex order (Section 2.1): a sort by
(value, vertex offset), checked against numpy's stable argsort and invariants."""
import numpy as np
import pytest

import oracle
from paper_2505_21266_amd import inputs


def _stable_rank(v):
    v = np.where(v == 0, 0.0, v)  # -0.0 and +0.0 are the same value
    perm = np.argsort(v.reshape(-1), kind="stable")
    r = np.empty(perm.size, np.int64)
    r[perm] = np.arange(perm.size)
    return r


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_matches_stable_argsort(dtype):
    v = np.random.default_rng(3).random(5000).astype(dtype)
    o = oracle.order(v)
    assert (o == _stable_rank(v)).all()


def test_config1_ties():
    """The 64^3 float32 U[0,1) field has many exact ties; the order must be a
    permutation that breaks them by vertex id."""
    v = inputs.config1()
    flat = v.reshape(-1)
    n_ties = flat.size - np.unique(flat).size
    assert n_ties > 500  # ~n^2/2 * 2^-24 = 2048 expected
    o = oracle.order(v).reshape(-1)
    assert np.array_equal(np.sort(o), np.arange(flat.size))
    assert (o == _stable_rank(flat)).all()


def test_constant_field_is_identity():
    o = oracle.order(np.full((3, 4, 5), 2.5, np.float32)).reshape(-1)
    assert (o == np.arange(60)).all()


def test_signed_zero_inf():
    v = np.array([0.0, -0.0, np.inf, -np.inf, 1.0, -0.0, 0.0], np.float32)
    o = oracle.order(v)
    # -inf < the four zeros (by id) < 1 < inf
    assert o.tolist() == [1, 2, 6, 0, 5, 3, 4]


def test_nan_rejected():
    with pytest.raises(ValueError):
        oracle.order(np.array([0.0, np.nan], np.float32))


@pytest.mark.parametrize("n,threads", [(100000, 2), (100003, 3), (262144, 8), (5000, 16)])
@pytest.mark.parametrize("kind", ["noise", "ties"])
def test_threaded_sort_matches_stable_argsort(n, threads, kind):
    """The oracle's threaded sort (sorted runs, then pairwise merges that take
    the left run first on ties) gives numpy's stable argsort rank, ties by id
    included, for run counts that are and are not powers of two."""
    rng = np.random.default_rng(n + threads)
    v = rng.random(n).astype(np.float32) if kind == "noise" else rng.integers(0, 9, n).astype(np.float64)
    o = oracle.order(v, nthreads=threads)
    assert (o == _stable_rank(v)).all()
