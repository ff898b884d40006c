"""Every lower-star configuration of the three families of vertices whose
records the library looks up instead of running Robins' loop (Section 2.3:
the record of x depends only on which neighbours precede x and on their
relative order).

Neighbour e and neighbour 13 - e are opposite offsets (the 14 neighbours
form 7 opposite pairs).  The families, by which members of each pair are
lower than x:
  regular:  exactly one member of every pair (2^7 choices of the members,
            7! orders of the 7 lower neighbours);
  upper6:   one pair j has no lower member, the other six exactly one
            (7 x 2^6 x 6!);
  lower8:   one pair j has both members lower, the other six exactly one
            (7 x 2^6 x 8!).
A configuration is written as 15 keys (x, then neighbours 0..13): the
lower neighbours take keys 0..m-1 in their given order, x takes m, the
upper neighbours m+1..14 in neighbour order (their order does not enter
L(x)).  No step of the method is here; the oracle and the GPU both consume
these keys.
"""
import itertools

import numpy as np

FAMILIES = ("regular", "upper6", "lower8")
SIZES = {"regular": 128 * 5040, "upper6": 7 * 64 * 720, "lower8": 7 * 64 * 40320}


def _perms(m):
    return np.array(list(itertools.permutations(range(m))), dtype=np.uint8)


def _rows(lower, perms):
    """Key rows for one lower set (list of neighbour indices, in slot order)
    under every permutation: lower[s] gets key perms[:, s]."""
    m = len(lower)
    rows = np.empty((perms.shape[0], 15), np.uint8)
    rows[:, 0] = m
    upper = [e for e in range(14) if e not in lower]
    for s, e in enumerate(lower):
        rows[:, 1 + e] = perms[:, s]
    for u, e in enumerate(upper):
        rows[:, 1 + e] = m + 1 + u
    return rows


def lower_sets(family):
    """The lower sets of a family, each as a list of neighbour indices."""
    out = []
    if family == "regular":
        for side in range(128):
            out.append([13 - i if (side >> i) & 1 else i for i in range(7)])
        return out
    for j in range(7):
        for side6 in range(64):
            others = [i for i in range(7) if i != j]
            low = [13 - i if (side6 >> s) & 1 else i for s, i in enumerate(others)]
            if family == "lower8":
                low = low + [j, 13 - j]
            out.append(low)
    return out


def family_keys(family):
    """(SIZES[family], 15) uint8 key rows covering every configuration."""
    sets = lower_sets(family)
    perms = _perms(len(sets[0]))
    out = np.concatenate([_rows(low, perms) for low in sets])
    assert out.shape[0] == SIZES[family]
    return out
