"""Seeded synthetic inputs for the 2D and 3D diffusion problems the solver is run on.

This module holds no arithmetic of the method: it only draws coefficient fields
and right-hand sides from numpy's PCG64 generator (``default_rng(seed)``),
row-major, in float64.  Both the GPU path's tests/benchmark and the CPU oracle
take their inputs from here.

Grids are vertex grids of nx x ny points including the boundary ring; cell
fields have (ny-1) x (nx-1) entries, cell (i, j) = [x_i, x_i+1] x [y_j, y_j+1].
In 3D the arrays are [nz][ny][nx] (vertices) and [nz-1][ny-1][nx-1] (cells).
"""
import numpy as np


def cells_constant(nx, ny, value=1.0):
    return np.full((ny - 1, nx - 1), float(value))


def cells_log10_blocks(nx, ny, block=16, lo=-2.0, hi=2.0, seed=1):
    """Piecewise-constant D on block x block cell tiles, log10 D ~ U[lo, hi]."""
    rng = np.random.default_rng(seed)
    by, bx = -(-(ny - 1) // block), -(-(nx - 1) // block)
    e = rng.uniform(lo, hi, size=(by, bx))
    D = 10.0 ** np.repeat(np.repeat(e, block, axis=0), block, axis=1)
    return np.ascontiguousarray(D[: ny - 1, : nx - 1])


def cells_two_phase_blocks(nx, ny, block=64, values=(1.0, 1e-3), seed=3):
    """Random checkerboard: each block x block cell tile independently takes
    values[0] or values[1] with probability 1/2."""
    rng = np.random.default_rng(seed)
    by, bx = -(-(ny - 1) // block), -(-(nx - 1) // block)
    pick = rng.integers(0, 2, size=(by, bx))
    v = np.where(pick == 0, values[0], values[1]).astype(np.float64)
    D = np.repeat(np.repeat(v, block, axis=0), block, axis=1)
    return np.ascontiguousarray(D[: ny - 1, : nx - 1])


def cells_compensating(nx, ny, r=None):
    """The paper's workload tensor D = diag(1/r, r) per cell (section 5), as
    (Dx, Dy).  r defaults to the cell aspect ratio hy/hx of the unit square
    with nx x ny vertices, which makes the discrete operator isotropic."""
    if r is None:
        r = (nx - 1) / (ny - 1)
    shape = (ny - 1, nx - 1)
    return np.full(shape, 1.0 / r), np.full(shape, float(r))


def spacings(nx, ny):
    """Grid spacings (hx, hy) of the unit square with nx x ny vertices."""
    return 1.0 / (nx - 1), 1.0 / (ny - 1)


def cells_lognormal(nx, ny, sigma=1.0, seed=1000):
    """Per-cell i.i.d. D = exp(sigma * Z), Z ~ N(0, 1)."""
    rng = np.random.default_rng(seed)
    return np.exp(sigma * rng.standard_normal((ny - 1, nx - 1)))


def theta_box5(nx, ny, seed=3000):
    """Per-cell log-diffusivity theta: i.i.d. N(0,1) smoothed by a 5x5 mean
    filter with reflecting edges."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((ny - 1, nx - 1))
    zp = np.pad(z, 2, mode="symmetric")
    c = np.cumsum(np.cumsum(zp, axis=0), axis=1)
    c = np.pad(c, ((1, 0), (1, 0)))
    s = c[5:, 5:] - c[:-5, 5:] - c[5:, :-5] + c[:-5, :-5]
    return np.ascontiguousarray(s / 25.0)


def load_uniform(nx, ny, seed=2):
    """Load vector b = h^2 f of the vertex-centred finite-volume scheme with
    f ~ U[-1, 1] i.i.d. at interior vertices, h = 1/(n-1) per direction
    (dual-cell area hx*hy); boundary entries are zero."""
    rng = np.random.default_rng(seed)
    f = rng.uniform(-1.0, 1.0, size=(ny, nx))
    f[0, :] = 0.0
    f[-1, :] = 0.0
    f[:, 0] = 0.0
    f[:, -1] = 0.0
    hx, hy = 1.0 / (nx - 1), 1.0 / (ny - 1)
    return f * (hx * hy)


def batch_sizes(nprob=256, choices=(129, 257, 513, 1025), seed=5):
    rng = np.random.default_rng(seed)
    return [int(choices[k]) for k in rng.integers(0, len(choices), size=nprob)]


def cells3_log10_blocks(nx, ny, nz, block=8, lo=-2.0, hi=2.0, seed=11):
    """3D piecewise-constant D on block^3 cell tiles, log10 D ~ U[lo, hi]."""
    rng = np.random.default_rng(seed)
    bz, by, bx = -(-(nz - 1) // block), -(-(ny - 1) // block), -(-(nx - 1) // block)
    e = rng.uniform(lo, hi, size=(bz, by, bx))
    D = 10.0 ** np.repeat(np.repeat(np.repeat(e, block, axis=0), block, axis=1), block, axis=2)
    return np.ascontiguousarray(D[: nz - 1, : ny - 1, : nx - 1])


def cells3_lognormal(nx, ny, nz, sigma=1.0, seed=12):
    """3D per-cell i.i.d. D = exp(sigma * Z), Z ~ N(0, 1)."""
    rng = np.random.default_rng(seed)
    return np.exp(sigma * rng.standard_normal((nz - 1, ny - 1, nx - 1)))


def load3_uniform(nx, ny, nz, seed=13):
    """3D load b = h^2 f (the 7-point scheme's connections leave out the
    common factor h of the dual-face area over the edge length), f ~ U[-1, 1]
    i.i.d. at interior vertices, h the mean spacing; boundary entries zero."""
    rng = np.random.default_rng(seed)
    f = rng.uniform(-1.0, 1.0, size=(nz, ny, nx))
    f[0], f[-1] = 0.0, 0.0
    f[:, 0], f[:, -1] = 0.0, 0.0
    f[:, :, 0], f[:, :, -1] = 0.0, 0.0
    h = (1.0 / (nx - 1) + 1.0 / (ny - 1) + 1.0 / (nz - 1)) / 3.0
    return f * (h * h)
