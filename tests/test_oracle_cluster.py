"""Pins for the oracle's clusters (connected components of neighbour bonds),
CPU only: a pure-Python breadth-first search over brute-force bonds, and
hand-built configurations."""
from collections import deque

import numpy as np

from paper_1906_06317_amd import workloads
from tests import brute


def _bfs_labels(adj):
    n = len(adj)
    lab = [-1] * n
    for s in range(n):
        if lab[s] >= 0:
            continue
        lab[s] = s  # s is the smallest index of its component (scan order)
        dq = deque([s])
        while dq:
            u = dq.popleft()
            for v in adj[u]:
                if lab[v] < 0:
                    lab[v] = s
                    dq.append(v)
    return np.array(lab)


def test_matches_breadth_first_search_on_brute_force_bonds(orc):
    for dim, seed in ((3, 501), (2, 502)):
        L, tilt = ((9.0, 8.0, 10.0), (0.3, -0.2, 0.1)) if dim == 3 else ((12.0, 11.0, 1.0), (0.4, 0, 0))
        rng = np.random.default_rng(seed)
        n = 250
        pts = (rng.uniform(-0.5, 0.5, (n, 3)) @ workloads.lattice_vectors(L, tilt, dim).T).astype(np.float32)
        if dim == 2:
            pts[:, 2] = 0
        r_cut = 1.1 if dim == 3 else 0.6
        v = brute.pair_vectors(pts, L, tilt, dim)
        A = ((v ** 2).sum(-1) < r_cut ** 2) & ~np.eye(n, dtype=bool)
        ref = _bfs_labels([np.nonzero(A[i])[0].tolist() for i in range(n)])
        off, idx, _ = orc.ball_query(orc.make_box(L, tilt, dim), pts, r_cut)
        labels, cidx, sizes = orc.clusters(n, off, idx)
        np.testing.assert_array_equal(labels, ref)
        roots = np.unique(ref)
        assert 5 < roots.size < n
        # cluster_idx numbers components by smallest member; sizes count them
        np.testing.assert_array_equal(cidx, np.searchsorted(roots, ref))
        np.testing.assert_array_equal(sizes, np.bincount(np.searchsorted(roots, ref)))


def test_hand_built_configurations(orc):
    """Two blobs, a chain through the periodic boundary and a lone point."""
    box = orc.make_box((10.0, 10.0, 10.0))
    pts = np.array([
        [0.0, 0.0, 0.0], [0.5, 0.0, 0.0], [0.0, 0.5, 0.0],        # blob A: 0, 1, 2
        [4.6, 3.0, 0.0], [-4.6, 3.0, 0.0], [-4.0, 3.0, 0.0],      # chain across x = +-5: 3, 4, 5
        [2.0, -3.0, 2.0],                                          # alone: 6
        [2.2, 2.0, -2.0], [2.6, 2.0, -2.0],                        # blob B: 7, 8
    ], np.float32)
    off, idx, _ = orc.ball_query(box, pts, 0.9)
    labels, cidx, sizes = orc.clusters(len(pts), off, idx)
    np.testing.assert_array_equal(labels, [0, 0, 0, 3, 3, 3, 6, 7, 7])
    np.testing.assert_array_equal(cidx, [0, 0, 0, 1, 1, 1, 2, 3, 3])
    np.testing.assert_array_equal(sizes, [3, 3, 1, 2])


def test_one_directional_lists_are_undirected_edges(orc):
    """A list holding a bond in one direction only (as a k-nearest list can)
    still joins both points."""
    off = np.array([0, 1, 1, 2, 2])
    idx = np.array([1, 1])  # 0 -> 1 and 2 -> 1; rows 1 and 3 empty
    labels, cidx, sizes = orc.clusters(4, off, idx)
    np.testing.assert_array_equal(labels, [0, 0, 0, 3])
    np.testing.assert_array_equal(sizes, [3, 1])
