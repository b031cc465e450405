"""Seeded synthetic particle configurations.

These generators are the only code shared by the GPU path's tests and the
oracle: they build inputs and hold none of the analysis arithmetic.  Every
configuration is drawn with ``numpy.random.default_rng(seed)`` in float64
and stored as float32 N x 3 arrays (z = 0 in 2D).  A box is the tuple
(L, tilt, dim) with tilt = (xy, xz, yz); its lattice vectors are
a1 = (Lx, 0, 0), a2 = (xy Ly, Ly, 0), a3 = (xz Lz, yz Lz, Lz), and the box is
centred on the origin.

The recipes stand in for the paper's data sets, none of which is used:
uniform ("ideal gas") points, a noisy FCC crystal, a 2D fluid with
orientations, a trajectory of uneven frames and a noisy simple-cubic
crystal.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class System:
    L: tuple
    tilt: tuple
    dim: int
    points: np.ndarray          # float32 [N, 3]
    theta: np.ndarray | None = None  # float32 [N] orientations (2D)
    quat: np.ndarray | None = None   # float32 [N, 4] unit quaternions (w, x, y, z) (3D)


def lattice_vectors(L, tilt, dim=3):
    """Columns a1, a2, a3 of the box (input construction only)."""
    Lx, Ly, Lz = L
    xy, xz, yz = tilt
    if dim == 2:
        return np.array([[Lx, xy * Ly, 0.0], [0.0, Ly, 0.0], [0.0, 0.0, 1.0]])
    return np.array([[Lx, xy * Ly, xz * Lz], [0.0, Ly, yz * Lz], [0.0, 0.0, Lz]])


def _from_fractional(s, L, tilt, dim):
    """Cartesian positions from fractional ones in [-1/2, 1/2)."""
    A = lattice_vectors(L, tilt, dim)
    r = s @ A.T
    if dim == 2:
        r[:, 2] = 0.0
    return r


def _fold(r, L, tilt, dim):
    """Fold Cartesian positions back to fractional [-1/2, 1/2) and map again."""
    A = lattice_vectors(L, tilt, dim)
    s = np.linalg.solve(A, r.T).T
    s -= np.floor(s + 0.5)
    if dim == 2:
        s[:, 2] = 0.0
    return _from_fractional(s, L, tilt, dim)


def _finish(r):
    return np.ascontiguousarray(r, dtype=np.float32)


def uniform(n, density, seed, dim=3, tilt=(0.0, 0.0, 0.0), L=None):
    """n uniform points in a periodic box at the given number density."""
    rng = np.random.default_rng(seed)
    if L is None:
        side = (n / density) ** (1.0 / dim)
        L = (side, side, side if dim == 3 else 1.0)
    s = rng.uniform(-0.5, 0.5, size=(n, 3))
    if dim == 2:
        s[:, 2] = 0.0
    return System(tuple(L), tuple(tilt), dim, _finish(_from_fractional(s, L, tilt, dim)))


def fcc(cells, a, seed=None, noise=0.0, tilt=(0.0, 0.0, 0.0)):
    """FCC crystal of cells^3 conventional cells (4 sites each) with spacing a.

    Sites are placed in fractional coordinates, so in a tilted box the
    lattice is sheared with the box and has no seam.  Gaussian noise of
    standard deviation ``noise`` (absolute) is added per Cartesian component
    and the points are folded back into the box.
    """
    basis = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]], np.float64)
    g = np.arange(cells, dtype=np.float64)
    cz, cy, cx = np.meshgrid(g, g, g, indexing="ij")
    corner = np.stack([cx.ravel(), cy.ravel(), cz.ravel()], axis=1)
    s = (corner[:, None, :] + basis[None, :, :]).reshape(-1, 3) / cells - 0.5
    L = (cells * a,) * 3
    r = _from_fractional(s, L, tilt, 3)
    if noise > 0.0:
        rng = np.random.default_rng(seed)
        r = _fold(r + rng.normal(0.0, noise, size=r.shape), L, tilt, 3)
    return System(L, tuple(tilt), 3, _finish(r))


def simple_cubic_with_vacancies(n, density, seed, noise):
    """Simple-cubic crystal with random vacancies down to exactly n points.

    m^3 sites with m = ceil(n^(1/3)) at spacing L/m in a cubic box with
    L = (n/density)^(1/3); m^3 - n sites chosen at random are removed, then
    Gaussian noise (absolute standard deviation) is added and points folded.
    """
    rng = np.random.default_rng(seed)
    side = (n / density) ** (1.0 / 3.0)
    m = int(math.ceil(n ** (1.0 / 3.0) - 1e-9))
    g = (np.arange(m, dtype=np.float64) + 0.5) / m - 0.5
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    s = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    keep = np.sort(rng.permutation(m ** 3)[:n])
    L = (side, side, side)
    r = _from_fractional(s[keep], L, (0.0, 0.0, 0.0), 3)
    r = _fold(r + rng.normal(0.0, noise, size=r.shape), L, (0.0, 0.0, 0.0), 3)
    return System(L, (0.0, 0.0, 0.0), 3, _finish(r))


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

def small_uniform(seed=1001, n=4096):
    """N = 4096 uniform points, cubic box, density 0.8 (ball r_max 3.0, RDF 100 bins)."""
    return uniform(n, 0.8, seed)


def large_fcc(seed=1002, cells=64):
    """N = 4 cells^3 noisy FCC points (a = 4^(1/3), density 1), tilts (0.5, 0.2, 0.1)."""
    a = 4.0 ** (1.0 / 3.0)
    return fcc(cells, a, seed=seed, noise=0.05 * a, tilt=(0.5, 0.2, 0.1))


def fluid_2d(seed=1003, n=262144, density=0.7):
    """2D uniform points at density 0.7 with orientations uniform in [0, 2 pi)."""
    rng = np.random.default_rng(seed)
    side = math.sqrt(n / density)
    s = rng.uniform(-0.5, 0.5, size=(n, 3))
    s[:, 2] = 0.0
    L = (side, side, 1.0)
    r = _from_fractional(s, L, (0.0, 0.0, 0.0), 2)
    theta = rng.uniform(0.0, 2.0 * math.pi, size=n)
    return System(L, (0.0, 0.0, 0.0), 2, _finish(r), np.ascontiguousarray(theta, np.float32))


def fluid_3d(seed=1007, n=262144, density=0.9, tilt=(0.0, 0.0, 0.0)):
    """3D uniform points with orientations as unit quaternions (w, x, y, z)
    uniform over rotations (normalised Gaussian 4-vectors)."""
    rng = np.random.default_rng(seed)
    side = (n / density) ** (1.0 / 3.0)
    L = (side, side, side)
    s = rng.uniform(-0.5, 0.5, size=(n, 3))
    r = _from_fractional(s, L, tilt, 3)
    g = rng.normal(size=(n, 4))
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    return System(L, tuple(tilt), 3, _finish(r), None, np.ascontiguousarray(g, np.float32))


def trajectory(seed=1004, frames=256, n_lo=1000, n_hi=200000):
    """Frames with log-uniform N in [n_lo, n_hi], density U(0.6, 1.0), tilts U(-0.3, 0.3)^3.

    Stream 0 of SeedSequence(seed).spawn(frames + 1) draws the frame sizes,
    densities and tilts; stream f + 1 draws frame f's uniform positions.
    """
    streams = np.random.SeedSequence(seed).spawn(frames + 1)
    head = np.random.default_rng(streams[0])
    ns = np.rint(np.exp(head.uniform(math.log(n_lo), math.log(n_hi), size=frames))).astype(np.int64)
    rhos = head.uniform(0.6, 1.0, size=frames)
    tilts = head.uniform(-0.3, 0.3, size=(frames, 3))
    out = []
    for f in range(frames):
        rng = np.random.default_rng(streams[f + 1])
        side = (ns[f] / rhos[f]) ** (1.0 / 3.0)
        L = (side, side, side)
        s = rng.uniform(-0.5, 0.5, size=(int(ns[f]), 3))
        out.append(System(L, tuple(float(t) for t in tilts[f]), 3,
                          _finish(_from_fractional(s, L, tuple(tilts[f]), 3))))
    return out


def smooth_target_pair(seed=1005, target_seed=1006, n=131072, density=0.9, noise=0.1):
    """(perturbed simple-cubic system, uniform target system) in the same cubic box."""
    sys_ = simple_cubic_with_vacancies(n, density, seed, noise)
    tgt = uniform(n, density, target_seed, L=sys_.L)
    return sys_, tgt
