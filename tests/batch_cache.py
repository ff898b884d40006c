"""Pinning the batched form's tile shape through its tuning cache."""
import numpy as np


def batch_signature(sides):
    """The batch plan's key for its tuning cache: FNV-1a over the fields'
    sides as little-endian int64 (x, y, z per field)."""
    h = 1469598103934665603
    for b in np.asarray(sides, dtype="<i8").tobytes():
        h ^= b
        h = (h * 1099511628211) & 0xFFFFFFFFFFFFFFFF
    return h


def pin_variant(path, sides, variant):
    """Writes a tuning cache that selects tile shape `variant` (0: 64x16,
    1: 32x32, 2: 16x64) for this batch on gfx950; returns its path."""
    with open(path, "w") as fh:
        fh.write("gfx950 %x %d\n" % (batch_signature(sides), variant))
    return str(path)
