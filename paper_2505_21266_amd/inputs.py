"""Seeded synthetic scalar fields shaped like the paper's workloads.

This module holds no step of the method: it only draws random numbers and
evaluates Gaussian mixtures, so that the GPU path and the CPU oracle can be fed
the very same arrays.  Arrays are C-ordered (nz, ny, nx), x fastest, so the
flat index of vertex (i, j, k) is i + nx*(j + ny*k).

Stand-ins for the paper's datasets (Section 6.1, which are not available here):
white noise for "Random", smooth Gaussian mixtures for the smooth
simulations (Isabel, Wavelet), mixtures plus small noise for the noisy ones.

Gaussian mixture G(B, rng) draws, in this order, centres rng.random((B, 3))
(x, y, z in the unit cube), sigma rng.uniform(0.02, 0.1, B) and amplitudes
rng.uniform(-1, 1, B); it evaluates sum_b A_b exp(-|p - c_b|^2 / (2 sigma_b^2))
in float64, separably, with per-axis normalised coordinates p_a.  Noise is
added as scale * rng.random(shape) in float64 before the cast to the output
dtype.
"""
import numpy as np

# the five workloads
CONFIG1 = dict(name="noise64", shape=(64, 64, 64), dtype="float32")
CONFIG2 = dict(name="gauss512", shape=(512, 512, 512), dtype="float32", bumps=64, seed=2)
CONFIG3 = dict(name="gauss1026_ghost", shape=(1026, 1026, 1026), dtype="float32", bumps=512,
               seed=3, owned_lo=(1, 1, 1), owned_hi=(1025, 1025, 1025))
CONFIG4 = dict(name="batch96", nfields=96, side_lo=32, side_hi=256, seed=4)
CONFIG5 = dict(name="diff128_f64", shape=(128, 128, 128), dtype="float64", bumps=16, seed=5)
# the paper's largest dataset shape (2048 x 1920 x 1536, Section 6): beyond
# int32 orders, so only the gradient from the values and the extraction run
LARGE = dict(name="mix6g", shape=(1536, 1920, 2048), dtype="float32", bumps=64, seed=6)


def _mixture_params(rng, bumps):
    centres = rng.random((bumps, 3))
    sigma = rng.uniform(0.02, 0.1, bumps)
    amp = rng.uniform(-1.0, 1.0, bumps)
    return centres, sigma, amp


def _axis_factors(coords, centre, sigma):
    # coords: (n,), centre/sigma: (B,) -> (B, n) of exp(-(p - c)^2 / (2 s^2))
    d = coords[None, :] - centre[:, None]
    return np.exp(-(d * d) / (2.0 * sigma[:, None] ** 2))


def mixture_field(shape, bumps, rng, noise, dtype, coords=None, slab=16, out=None):
    """Gaussian mixture plus noise on a grid of shape (nz, ny, nx).

    coords: optional (px, py, pz) per-axis coordinate arrays; default
    idx / (n - 1) per axis (0 for an axis of one vertex).  Evaluated and
    noised slab by slab along z, which draws the noise in exactly the order
    rng.random(shape) would.
    """
    nz, ny, nx = shape
    if coords is None:
        coords = tuple(np.arange(n, dtype=np.float64) / max(n - 1, 1) for n in (nx, ny, nz))
    px, py, pz = coords
    centres, sigma, amp = _mixture_params(rng, bumps)
    fx = _axis_factors(px, centres[:, 0], sigma)
    fy = _axis_factors(py, centres[:, 1], sigma)
    fz = _axis_factors(pz, centres[:, 2], sigma) * amp[:, None]
    if out is None:
        out = np.empty(shape, dtype=dtype)
    for k0 in range(0, nz, slab):
        k1 = min(nz, k0 + slab)
        # T[(k, j), b] = A_b fz[b, k] fy[b, j];  field[(k, j), i] = T @ fx
        t = (fz[:, k0:k1, None] * fy[:, None, :]).reshape(bumps, -1).T
        vals = (t @ fx).reshape(k1 - k0, ny, nx)
        if noise:
            vals += noise * rng.random((k1 - k0, ny, nx))
        out[k0:k1] = vals.astype(dtype)
    return out


def white_noise(shape, seed, dtype=np.float32):
    return np.random.default_rng(seed).random(shape, dtype=dtype)


def config1():
    """64^3 float32, i.i.d. U[0,1) from seed 1."""
    return white_noise((64, 64, 64), 1)


def config2(shape=(512, 512, 512)):
    """512^3 float32: 64 isotropic Gaussians (seed 2) plus 1e-3 U[0,1) noise."""
    rng = np.random.default_rng(2)
    return mixture_field(shape, 64, rng, 1e-3, np.float32)


def ghost_coords(n_owned):
    """Owned indices 1..n_owned map to [0, 1]; the ghost layer sits one step
    outside on each side."""
    return (np.arange(n_owned + 2, dtype=np.float64) - 1.0) / (n_owned - 1)


def config3(n_owned=1024, bumps=512):
    """(n_owned + 2)^3 float32 block with a one-voxel ghost layer: 512 Gaussians
    (seed 3) plus 1e-3 U[0,1).  Returns (field, owned_lo, owned_hi) with the
    owned box as half-open (x, y, z) bounds."""
    c = ghost_coords(n_owned)
    n = n_owned + 2
    rng = np.random.default_rng(3)
    f = mixture_field((n, n, n), bumps, rng, 1e-3, np.float32, coords=(c, c, c))
    return f, (1, 1, 1), (n - 1, n - 1, n - 1)


def config4_sides(nfields=96):
    """Sides (nx, ny, nz) of the batched fields, each uniform in 32..256."""
    return np.random.default_rng(4).integers(32, 257, (nfields, 3))


def config4_field(f, sides=None):
    """Field f of the batch: even f white noise U[0,1), odd f a 16-Gaussian
    mixture plus 1e-3 U[0,1); rng default_rng((4, f)); float32."""
    if sides is None:
        sides = config4_sides()
    nx, ny, nz = (int(s) for s in sides[f])
    rng = np.random.default_rng((4, f))
    if f % 2 == 0:
        return rng.random((nz, ny, nx), dtype=np.float32)
    return mixture_field((nz, ny, nx), 16, rng, 1e-3, np.float32)


def config4(nfields=96):
    sides = config4_sides(nfields)
    return [config4_field(f, sides) for f in range(nfields)], sides


def min_gap_pass(values, gap=2e-9):
    """Walks the values in (value, id) order and lifts each to at least the
    previous one plus gap, keeping the order; afterwards every pair of values
    differs by more than gap / 2."""
    v = np.asarray(values, dtype=np.float64).reshape(-1)
    perm = np.argsort(v, kind="stable")
    s = v[perm]
    # v'_r = max(s_r, v'_{r-1} + gap)  <=>  v'_r = r*gap + cummax(s_r - r*gap)
    r = np.arange(s.size, dtype=np.float64)
    lifted = np.maximum.accumulate(s - r * gap) + r * gap
    out = np.empty_like(v)
    out[perm] = lifted
    return out.reshape(np.shape(values))


def config5(shape=(128, 128, 128)):
    """128^3 float64: 16 Gaussians (seed 5) plus 1e-4 U[0,1), then the min-gap
    pass so that all value gaps exceed 1e-9."""
    rng = np.random.default_rng(5)
    f = mixture_field(shape, 16, rng, 1e-4, np.float64)
    return min_gap_pass(f)


def config_large(shape=LARGE["shape"]):
    """2048 x 1920 x 1536 float32 (6.04e9 vertices, 24 GB): 64 Gaussians
    (seed 6) plus 1e-3 U[0,1), evaluated slab by slab."""
    rng = np.random.default_rng(LARGE["seed"])
    return mixture_field(shape, LARGE["bumps"], rng, 1e-3, np.float32, slab=8)


def ramp(shape, direction, dtype=np.float64):
    """Linear field d . (x, y, z) (the Elevation case of Section 6.1)."""
    nz, ny, nx = shape
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    dx, dy, dz = direction
    return (dx * i + dy * j + dz * k).astype(dtype)
