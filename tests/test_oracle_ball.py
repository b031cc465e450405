"""Pins for the oracle's minimum image and ball query (CPU only)."""
import math

import numpy as np
import pytest
from scipy.spatial import cKDTree

from paper_1906_06317_amd import workloads
from tests import brute

REL = 1e-5


def random_box(rng, dim=3):
    L = rng.uniform(3.0, 7.0, size=3)
    tilt = rng.uniform(-0.5, 0.5, size=3)
    if dim == 2:
        L[2] = 1.0
        tilt[1:] = 0.0
    return tuple(L), tuple(tilt)


@pytest.mark.parametrize("dim", [2, 3])
def test_minimum_image_matches_image_search(orc, dim):
    rng = np.random.default_rng(11 + dim)
    for _ in range(20):
        L, tilt = random_box(rng, dim)
        box = orc.make_box(L, tilt, dim)
        half = 0.5 * brute.perpendicular_widths(L, tilt, dim).min()
        d = rng.uniform(-1.5, 1.5, size=(400, 3)) * np.array(L)
        if dim == 2:
            d[:, 2] = 0
        got = orc.minimum_image(box, d)
        ref = brute.min_image_vectors(d, L, tilt, dim, reach=4)
        r_ref = np.sqrt((ref ** 2).sum(1))
        inside = r_ref < half * (1 - 1e-9)
        assert inside.sum() > 10
        np.testing.assert_allclose(got[inside], ref[inside], atol=1e-9)
        # every result differs from the input by a whole lattice translation
        A = workloads.lattice_vectors(L, tilt, dim)
        m = np.linalg.solve(A, (got - np.where(dim == 2, d * [1, 1, 0], d)).T).T
        np.testing.assert_allclose(m[:, :dim], np.rint(m[:, :dim]), atol=1e-9)
        # never longer than the shortest image
        assert np.all((got ** 2).sum(1) >= (ref ** 2).sum(1) - 1e-9)


def _sets_from_csr(offsets, idx):
    return [set(idx[offsets[i]:offsets[i + 1]].tolist()) for i in range(len(offsets) - 1)]


@pytest.mark.parametrize("dim", [2, 3])
def test_ball_query_matches_image_search(orc, dim):
    rng = np.random.default_rng(21 + dim)
    for trial in range(12):
        L, tilt = random_box(rng, dim)
        n = int(rng.integers(1, 120))
        s = rng.uniform(-0.5, 0.5, size=(n, 3))
        pts = (s @ workloads.lattice_vectors(L, tilt, dim).T).astype(np.float32)
        if dim == 2:
            pts[:, 2] = 0
        # a few copies of points shifted by whole lattice vectors (same site, other image)
        half = 0.5 * brute.perpendicular_widths(L, tilt, dim).min()
        r_max = float(rng.uniform(0.3, 0.95) * half)
        box = orc.make_box(L, tilt, dim)
        off, idx, r2 = orc.ball_query(box, pts, r_max)
        v = brute.pair_vectors(pts, L, tilt, dim)
        R2 = (v ** 2).sum(-1)
        np.fill_diagonal(R2, np.inf)
        for i in range(n):
            row = idx[off[i]:off[i + 1]]
            rr = r2[off[i]:off[i + 1]]
            assert np.all(np.diff(row) > 0), "rows are in ascending point order"
            ref = set(np.nonzero(R2[i] < r_max ** 2 * (1 + REL))[0].tolist())
            assert set(row.tolist()) == ref
            np.testing.assert_allclose(rr, R2[i, row], rtol=1e-12, atol=1e-12)


def test_ball_query_with_separate_query_points(orc):
    rng = np.random.default_rng(5)
    L, tilt = (6.0, 5.0, 5.5), (0.3, -0.2, 0.4)
    A = workloads.lattice_vectors(L, tilt)
    pts = (rng.uniform(-0.5, 0.5, (90, 3)) @ A.T).astype(np.float32)
    q = (rng.uniform(-1.5, 1.5, (40, 3)) @ A.T).astype(np.float32)  # outside the box too
    box = orc.make_box(L, tilt)
    off, idx, r2 = orc.ball_query(box, pts, 2.0, query_points=q)
    v = brute.pair_vectors(pts, L, tilt, query=q)
    R2 = (v ** 2).sum(-1)
    for i in range(q.shape[0]):
        assert set(idx[off[i]:off[i + 1]].tolist()) == set(np.nonzero(R2[i] < 4.0 * (1 + REL))[0].tolist())


def test_ball_query_matches_ckdtree_cubic(orc):
    """SciPy's periodic cKDTree (orthorhombic only) as an independent reference."""
    sysm = workloads.small_uniform()
    L = sysm.L[0]
    pts = sysm.points
    r_max = 3.0
    box = orc.make_box(sysm.L, sysm.tilt)
    off, idx, r2 = orc.ball_query(box, pts, r_max)
    tree = cKDTree(np.mod(pts.astype(np.float64) + L / 2, L), boxsize=L)
    ref = tree.query_ball_point(np.mod(pts.astype(np.float64) + L / 2, L), r_max * math.sqrt(1 + REL))
    n_amb = 0
    for i in range(pts.shape[0]):
        mine = set(idx[off[i]:off[i + 1]].tolist())
        theirs = set(ref[i]) - {i}
        diff = mine ^ theirs
        # only pairs at the ambiguous band's edge may differ (cKDTree rounds differently)
        for j in diff:
            d = pts[j].astype(np.float64) - pts[i]
            d -= L * np.rint(d / L)
            assert abs((d ** 2).sum() / (r_max ** 2 * (1 + REL)) - 1) < 1e-9
            n_amb += 1
    certain = np.sum(r2 < r_max ** 2 * (1 - REL))
    # ideal-gas expectation N (N - 1) / V * 4/3 pi r^3, variance ~ 2 E (ordered pairs)
    n = pts.shape[0]
    expect = n * (n - 1) / L ** 3 * 4.0 / 3.0 * math.pi * r_max ** 3
    assert abs(int(certain) - expect) < 5 * math.sqrt(2 * expect)
    assert n_amb == 0


def _fcc_shells(m_max):
    """Multiplicities of FCC neighbour shells |r|^2 = m a^2 / 2 by enumerating
    integer vectors (h, k, l) with h + k + l even (r = a/2 (h, k, l))."""
    rng = range(-6, 7)
    counts = {}
    for h in rng:
        for k in rng:
            for l in rng:
                if (h + k + l) % 2 or (h, k, l) == (0, 0, 0):
                    continue
                m = (h * h + k * k + l * l) // 2
                if m <= m_max:
                    counts[m] = counts.get(m, 0) + 1
    return counts


def test_fcc_shell_multiplicities_enumeration():
    assert [(_fcc_shells(9))[m] for m in range(1, 10)] == [12, 6, 24, 12, 24, 8, 48, 6, 36]


def test_perfect_fcc_neighbor_counts(orc):
    a = 4.0 ** (1.0 / 3.0)
    s = workloads.fcc(6, a)  # 864 sites, box 6a
    box = orc.make_box(s.L, s.tilt)
    off, idx, r2 = orc.ball_query(box, s.points, 1.2)
    cnt = np.diff(off)
    assert np.all(cnt == 12)
    np.testing.assert_allclose(np.sqrt(r2), a / math.sqrt(2), rtol=1e-6)
    off, idx, r2 = orc.ball_query(box, s.points, 2.5)
    shells = _fcc_shells(9)
    want = sum(c for m, c in shells.items() if m * a * a / 2 < 2.5 ** 2)
    assert want == 54
    assert np.all(np.diff(off) == want)


def test_perfect_fcc_sheared_box(orc):
    """A lattice placed in fractional coordinates of a tilted box keeps its
    shell structure up to the shear: every site has the same neighbour count."""
    a = 4.0 ** (1.0 / 3.0)
    s = workloads.fcc(8, a, tilt=(0.5, 0.2, 0.1))
    box = orc.make_box(s.L, s.tilt)
    off, idx, r2 = orc.ball_query(box, s.points, 2.5)
    c = np.diff(off)
    assert np.all(c == c[0])
    # same per-site count as the 64^3 lattice, since the shear is the same
    assert c[0] == 70


def test_ball_query_symmetry(orc):
    rng = np.random.default_rng(9)
    L, tilt = (9.0, 8.0, 8.5), (0.4, -0.3, 0.2)
    A = workloads.lattice_vectors(L, tilt)
    pts = (rng.uniform(-0.5, 0.5, (500, 3)) @ A.T).astype(np.float32)
    box = orc.make_box(L, tilt)
    off, idx, r2 = orc.ball_query(box, pts, 2.7)
    rows = np.repeat(np.arange(500), np.diff(off))
    fwd = dict(zip(zip(rows.tolist(), idx.tolist()), r2.tolist()))
    for (i, j), v in fwd.items():
        assert (j, i) in fwd
        assert abs(fwd[(j, i)] - v) <= 1e-12 * max(1.0, v)


def test_lattice_translation_invariance(orc):
    rng = np.random.default_rng(3)
    L, tilt = (7.0, 6.0, 6.5), (0.2, 0.1, -0.4)
    A = workloads.lattice_vectors(L, tilt)
    pts = (rng.uniform(-0.5, 0.5, (200, 3)) @ A.T).astype(np.float64)
    shift = rng.integers(-2, 3, size=(200, 3)) @ A.T
    box = orc.make_box(L, tilt)
    o1, i1, r1 = orc.ball_query(box, pts.astype(np.float32), 2.2)
    o2, i2, r2 = orc.ball_query(box, (pts + shift).astype(np.float32), 2.2)
    for i in range(200):
        a = dict(zip(i1[o1[i]:o1[i + 1]].tolist(), r1[o1[i]:o1[i + 1]]))
        b = dict(zip(i2[o2[i]:o2[i + 1]].tolist(), r2[o2[i]:o2[i + 1]]))
        # float32 rounding of the shifted coordinates moves distances slightly
        for j in set(a) ^ set(b):
            v = a.get(j, b.get(j))
            assert abs(v / 2.2 ** 2 - 1) < 1e-4
        for j in set(a) & set(b):
            assert abs(a[j] - b[j]) < 1e-4
