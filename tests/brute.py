"""Independent numpy brute force used to pin the oracle.

Minimum images are found by explicit enumeration of lattice translations
(|m_k| <= 2), not by the oracle's back-substitution, so a mistake in either
shows up as a disagreement.  Only for tiny inputs.
"""
import itertools

import numpy as np

from paper_1906_06317_amd.workloads import lattice_vectors


def perpendicular_widths(L, tilt, dim=3):
    A = lattice_vectors(L, tilt, dim)
    if dim == 2:
        A2 = A[:2, :2]
        V = abs(np.linalg.det(A2))
        return np.array([V / np.linalg.norm(A2[:, 1]), V / np.linalg.norm(A2[:, 0]), np.inf])
    V = abs(np.linalg.det(A))
    a1, a2, a3 = A[:, 0], A[:, 1], A[:, 2]
    return np.array([V / np.linalg.norm(np.cross(a2, a3)),
                     V / np.linalg.norm(np.cross(a3, a1)),
                     V / np.linalg.norm(np.cross(a1, a2))])


def images(L, tilt, dim=3, reach=2):
    A = lattice_vectors(L, tilt, dim)
    rng = range(-reach, reach + 1)
    ms = [m for m in itertools.product(rng, rng, rng if dim == 3 else [0])]
    T = np.array(ms, np.float64) @ A.T
    if dim == 2:
        T[:, 2] = 0.0
    return T  # [n_images, 3]


def min_image_vectors(d, L, tilt, dim=3, reach=2):
    """Shortest image of each displacement d[n, 3] by enumeration."""
    d = np.asarray(d, np.float64).copy()
    if dim == 2:
        d[:, 2] = 0.0
    T = images(L, tilt, dim, reach)
    cand = d[:, None, :] + T[None, :, :]
    r2 = (cand ** 2).sum(-1)
    k = np.argmin(r2, axis=1)
    return cand[np.arange(d.shape[0]), k]


def pair_vectors(points, L, tilt, dim=3, query=None):
    """Minimum-image bond vectors p_j - q_i for all (i, j): [nq, n, 3]."""
    p = np.asarray(points, np.float64)
    q = p if query is None else np.asarray(query, np.float64)
    d = (p[None, :, :] - q[:, None, :]).reshape(-1, 3)
    return min_image_vectors(d, L, tilt, dim).reshape(q.shape[0], p.shape[0], 3)
