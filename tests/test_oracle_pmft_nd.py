"""Pins for the oracle's 2D PMFT with relative orientation (XYT) and 3D PMFT
(XYZ) histograms (CPU only)."""
import math

import numpy as np

from paper_1906_06317_amd import workloads
from tests import brute


def _bonds(points, L, tilt, dim):
    """All ordered bonds i != j by explicit image search: vectors and rows i."""
    v = brute.pair_vectors(points, L, tilt, dim)
    n = points.shape[0]
    mask = ~np.eye(n, dtype=bool)
    return v[mask], np.repeat(np.arange(n), n - 1), np.tile(np.arange(n), n)[mask.ravel()]


def _within(lo, H, hi):
    return np.all(lo.astype(np.int64) <= H) and np.all(H <= hi.astype(np.int64))


def test_xyt_theta_zero_is_histogramdd(orc):
    """All orientations 0: (x', y') is the bond itself, so the counts summed
    over t are numpy's histogramdd of the bonds; t = 0 for every bond, which
    sits on the edge between the last and the first angle bin (both
    possible, every bond in that band)."""
    rng = np.random.default_rng(61)
    L, tilt = (9.0, 8.0, 1.0), (0.2, 0.0, 0.0)
    n = 150
    pts = (rng.uniform(-0.5, 0.5, (n, 3)) @ workloads.lattice_vectors(L, tilt, 2).T).astype(np.float32)
    pts[:, 2] = 0
    box = orc.make_box(L, tilt, 2)
    nbx, nby, nbt, xm, ym, r_max = 12, 9, 5, 2.5, 2.0, 2.8
    zero = np.zeros(n, np.float32)
    lo, hi, amb = orc.pmft_xyt_counts(box, pts, zero, None, zero, nbx, nby, nbt, xm, ym, r_max)
    d, _, _ = _bonds(pts, L, tilt, 2)
    keep = (d ** 2).sum(1) < r_max ** 2
    H, _ = np.histogramdd(d[keep, :2], bins=[nbx, nby], range=[[-xm, xm], [-ym, ym]])
    H = H.astype(np.int64)
    assert H.sum() > 500
    assert hi[:, :, 1:nbt - 1].sum() == 0
    # each bond may go to t bin 0 or nbt - 1, never both
    assert np.all(hi[:, :, 0] == hi[:, :, nbt - 1]) and lo.sum() == 0
    assert np.all(H <= hi[:, :, 0].astype(np.int64))
    assert hi[:, :, 0].sum() - H.sum() < 20


def test_xyt_marginal_over_t_is_the_2d_pmft(orc):
    """Summing over the relative orientation gives the 2D PMFT histogram."""
    s = workloads.fluid_2d(seed=62, n=600, density=0.7)
    box = orc.make_box(s.L, s.tilt, 2)
    th = s.theta
    args = (12, 12, 3.0, 3.0, 3.0)
    lo2, hi2, a2 = orc.pmft2d_counts(box, s.points, None, th, *args)
    lo, hi, a3 = orc.pmft_xyt_counts(box, s.points, th, None, th, 12, 12, 7, 3.0, 3.0, 3.0)
    assert np.all(lo.sum(2) <= lo2) and np.all(hi.sum(2) >= hi2)
    assert lo2.sum() > 3000 and lo.sum() >= lo2.sum() - 2 * a3


def test_xyt_two_particles_hand_computed(orc):
    """p0 = (0, 0), theta0 = 0 and p1 = (1.2, 0.5), theta1 = 1 in a large box;
    x_max = y_max = 2 with 4 x 4 bins of width 1, 6 angle bins of width pi/3.
      0 -> 1: d = (1.2, 0.5) unrotated: ix = floor(3.2) = 3, iy = floor(2.5) = 2;
              t = 1 - 0 = 1, 1 / (pi/3) = 0.955: it = 0.
      1 -> 0: d = (-1.2, -0.5) turned by -1 rad (cos 1 = 0.540302, sin 1 = 0.841471):
              x' = -1.2 cos1 - 0.5 sin1 = -0.648363 - 0.420735 = -1.069098: ix = 0,
              y' = 1.2 sin1 - 0.5 cos1 = 1.009765 - 0.270151 = 0.739614: iy = 2;
              t = (0 - 1) mod 2pi = 5.2832, / (pi/3) = 5.045: it = 5."""
    box = orc.make_box((20.0, 20.0, 1.0), (0.0, 0.0, 0.0), 2)
    pts = np.array([[0, 0, 0], [1.2, 0.5, 0]], np.float32)
    th = np.array([0.0, 1.0], np.float32)
    lo, hi, amb = orc.pmft_xyt_counts(box, pts, th, None, th, 4, 4, 6, 2.0, 2.0, 3.0)
    expect = np.zeros((4, 4, 6), np.int64)
    expect[3, 2, 0] = 1
    expect[0, 2, 5] = 1
    assert amb == 0
    np.testing.assert_array_equal(lo, expect)
    np.testing.assert_array_equal(hi, expect)


def test_xyt_ideal_gas_normalisation(orc):
    s = workloads.fluid_2d(seed=63, n=20000, density=0.7)
    box = orc.make_box(s.L, s.tilt, 2)
    lo, hi, amb = orc.pmft_xyt_counts(box, s.points, s.theta, None, s.theta, 6, 6, 4, 3.0, 3.0, 3.0)
    area = s.L[0] * s.L[1]
    F = orc.pmft_xyt_from_counts(lo, s.points.shape[0], s.points.shape[0], area, 3.0, 3.0)
    # bins well inside the disc r < 3: pcf = exp(-F) fluctuates around 1
    inner = np.exp(-F[1:5, 1:5, :])
    assert abs(inner.mean() - 1.0) < 0.02 and np.all(np.abs(inner - 1.0) < 0.2)


def test_xyz_identity_is_histogramdd(orc):
    rng = np.random.default_rng(64)
    L, tilt = (7.0, 6.5, 7.5), (0.2, -0.1, 0.15)
    n = 140
    pts = (rng.uniform(-0.5, 0.5, (n, 3)) @ workloads.lattice_vectors(L, tilt, 3).T).astype(np.float32)
    box = orc.make_box(L, tilt, 3)
    quat = np.tile(np.array([1, 0, 0, 0], np.float32), (n, 1))
    nb, m, r_max = (7, 6, 5), (2.0, 1.8, 2.2), 2.5
    lo, hi, amb = orc.pmft_xyz_counts(box, pts, None, quat, *nb, *m, r_max)
    d, _, _ = _bonds(pts, L, tilt, 3)
    keep = (d ** 2).sum(1) < r_max ** 2
    H, _ = np.histogramdd(d[keep], bins=list(nb), range=[[-m[0], m[0]], [-m[1], m[1]], [-m[2], m[2]]])
    H = H.astype(np.int64)
    assert H.sum() > 500 and amb < 20 and _within(lo, H, hi)
    # a quaternion is normalised first: 2.5 * identity is the identity
    lo2, hi2, _ = orc.pmft_xyz_counts(box, pts, None, 2.5 * quat, *nb, *m, r_max)
    np.testing.assert_array_equal(lo2, lo)


def test_xyz_two_particles_hand_computed(orc):
    """q = (1/2)(1, 1, 1, 1), the turn by 120 degrees about (1, 1, 1), maps
    e_x -> e_y -> e_z -> e_x; the bond in its frame is R^T d = (d_y, d_z, d_x).
    p0 = 0 with that quaternion, p1 = (0.3, -0.7, 1.2) with the identity;
    cube [-1.5, 1.5)^3 in 3 x 3 x 3 bins of width 1.
      0 -> 1: (-0.7, 1.2, 0.3): bins (floor 0.8, floor 2.7, floor 1.8) = (0, 2, 1).
      1 -> 0: (-0.3, 0.7, -1.2) unrotated: (floor 1.2, floor 2.2, floor 0.3) = (1, 2, 0)."""
    box = orc.make_box((10.0, 10.0, 10.0))
    pts = np.array([[0, 0, 0], [0.3, -0.7, 1.2]], np.float32)
    quat = np.array([[0.5, 0.5, 0.5, 0.5], [1, 0, 0, 0]], np.float32)
    lo, hi, amb = orc.pmft_xyz_counts(box, pts, None, quat, 3, 3, 3, 1.5, 1.5, 1.5, 2.0)
    expect = np.zeros((3, 3, 3), np.int64)
    expect[0, 2, 1] = 1
    expect[1, 2, 0] = 1
    assert amb == 0
    np.testing.assert_array_equal(lo, expect)
    np.testing.assert_array_equal(hi, expect)


def test_xyz_turn_about_z_is_the_2d_pmft(orc):
    """Points in the plane z = 0 of a tall 3D box, each query turned by
    theta_i about z (q = (cos theta/2, 0, 0, sin theta/2)): (x', y') are the 2D
    PMFT's and z' = 0 falls in the middle bin of an odd z binning."""
    s = workloads.fluid_2d(seed=65, n=500, density=0.7)
    box2 = orc.make_box(s.L, s.tilt, 2)
    box3 = orc.make_box((s.L[0], s.L[1], 50.0))
    th = s.theta.astype(np.float64)
    quat = np.stack([np.cos(th / 2), 0 * th, 0 * th, np.sin(th / 2)], 1).astype(np.float32)
    lo2, hi2, _ = orc.pmft2d_counts(box2, s.points, None, s.theta, 10, 10, 3.0, 3.0, 3.0)
    lo3, hi3, _ = orc.pmft_xyz_counts(box3, s.points, None, quat, 10, 10, 3, 3.0, 3.0, 3.0, 3.0)
    assert lo3[:, :, [0, 2]].sum() == 0 and lo2.sum() > 2000
    # the exact counts lie in both intervals
    assert np.all(np.maximum(lo2, lo3[:, :, 1]) <= np.minimum(hi2, hi3[:, :, 1]))


def test_xyz_ideal_gas_normalisation(orc):
    s = workloads.fluid_3d(seed=66, n=20000, density=0.9)
    box = orc.make_box(s.L, s.tilt, 3)
    lo, hi, amb = orc.pmft_xyz_counts(box, s.points, None, s.quat, 4, 4, 4, 1.6, 1.6, 1.6, 3.0)
    V = s.L[0] * s.L[1] * s.L[2]
    F = orc.pmft_xyz_from_counts(lo, s.points.shape[0], s.points.shape[0], V, 1.6, 1.6, 1.6)
    pcf = np.exp(-F)
    assert abs(pcf.mean() - 1.0) < 0.02 and np.all(np.abs(pcf - 1.0) < 0.15)
