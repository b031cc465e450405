"""GPU parity: 2D PMFT histogram against the FP64 oracle.

Every bin must lie between the oracle's lower bound (pairs certain to land
there) and upper bound (plus pairs within 1e-5 of r_max^2 or within
1e-5 x_max of a bin edge, which may land in either neighbour).
"""
import math

import numpy as np
import pytest

import oracle
from paper_1906_06317_amd import workloads
from tests.parity import check_hist

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ppa():
    import torch
    assert torch.cuda.is_available(), "a GPU is required"
    import paper_1906_06317_amd as m
    m.lib()
    return m


def _box(s):
    import paper_1906_06317_amd as m
    return m.Box(s.L, s.tilt, s.dim)


def _fluid(n, density, seed, tilt=0.0):
    rng = np.random.default_rng(seed)
    s = workloads.uniform(n, density, seed, dim=2, tilt=(tilt, 0.0, 0.0))
    theta = rng.uniform(0.0, 2 * math.pi, n).astype(np.float32)
    return s, theta


def _compare(ppa, s, theta, nbx, nby, x_max, y_max, r_max, query=None, exclude_ii=None):
    q_pts = None if query is None else query[0]
    q_th = theta if query is None else query[1]
    g = ppa.pmft2d_counts(_box(s), s.points, q_th, nbx, nby, x_max, y_max, r_max,
                          query_points=q_pts, exclude_ii=exclude_ii).cpu().numpy()
    lo, hi, amb = oracle.pmft2d_counts(oracle.make_box(s.L, s.tilt, s.dim), s.points, q_pts, q_th,
                                       nbx, nby, x_max, y_max, r_max, exclude_ii=exclude_ii)
    check_hist(g.reshape(-1).astype(np.int64), lo.reshape(-1), hi.reshape(-1))
    return g, lo, hi, amb


def test_small_fluid_square_bins(ppa):
    s, th = _fluid(6000, 0.7, 31)
    g, lo, hi, amb = _compare(ppa, s, th, 60, 60, 3.0, 3.0, 3.0)
    # the edge band (3e-5 against 0.1-wide bins, two axes) makes ~1e-3 ambiguous
    assert lo.sum() > 100000 and amb < lo.sum() * 3e-3


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_tilted_boxes_and_rectangular_ranges(ppa, seed):
    rng = np.random.default_rng(40 + seed)
    s, th = _fluid(int(rng.integers(500, 5000)), float(rng.uniform(0.3, 1.2)), seed,
                   tilt=float(rng.uniform(-0.7, 0.7)))
    r = float(rng.uniform(1.0, 3.0))
    nbx, nby = int(rng.integers(5, 90)), int(rng.integers(5, 90))
    # ranges below, at and above r_max
    x_max, y_max = r * float(rng.uniform(0.5, 1.3)), r * float(rng.uniform(0.5, 1.3))
    _compare(ppa, s, th, nbx, nby, x_max, y_max, r)


def test_zero_orientation_is_plain_bond_histogram(ppa):
    s, th = _fluid(3000, 0.7, 5)
    th[:] = 0.0
    g, lo, hi, _ = _compare(ppa, s, th, 40, 40, 2.5, 2.5, 2.5)
    # bonds i->j and j->i are opposite: with theta = 0 the histogram is
    # point-symmetric about the origin (up to ambiguous pairs)
    gs = g[::-1, ::-1]
    assert np.all(np.abs(g.astype(np.int64) - gs.astype(np.int64)) <= (hi - lo) + (hi - lo)[::-1, ::-1])


@pytest.mark.parametrize("exclude_ii", [False, True])
def test_separate_query_points(ppa, exclude_ii):
    s, th = _fluid(4000, 0.7, 8)
    rng = np.random.default_rng(9)
    q = workloads.uniform(1500, 0.7, 10, dim=2, L=s.L).points
    qth = rng.uniform(-10.0, 10.0, q.shape[0]).astype(np.float32)  # also outside [0, 2 pi)
    _compare(ppa, s, th, 50, 50, 3.0, 3.0, 3.0, query=(q, qth), exclude_ii=exclude_ii)


@pytest.mark.parametrize("nb", [256, 300, 400])
def test_large_histograms(ppa, nb):
    """256 x 256 fits the LDS only as 16-bit counters; 300 x 300 and beyond
    go to global atomics (no per-workgroup partial histograms)."""
    s, th = _fluid(3000, 0.7, 12)
    ws = ppa.pmft2d_workspace_bytes(_box(s), 3000, 0, nb, nb, 3.0, 3.0, 3.0)
    if nb >= 300:
        assert ws < 50 << 20
    else:
        assert ws > 50 << 20
    _compare(ppa, s, th, nb, nb, 3.0, 3.0, 3.0)


def test_dense_cluster_counters_hand_over(ppa):
    """6000 points in a disc of radius 0.05: one home cell makes all 36 M
    bonds, and the bins near the origin each collect far more than 2^16 of
    them inside one workgroup, so a 16-bit LDS counter must hand 2^15 at a
    time to the global count (200 x 200 bins on [-3, 3)^2, the window that
    takes two 16-bit counters per word)."""
    rng = np.random.default_rng(17)
    n = 6000
    rad = 0.05 * np.sqrt(rng.uniform(0, 1, n))
    phi = rng.uniform(0, 2 * math.pi, n)
    pts = np.zeros((n, 3), np.float32)
    pts[:, 0] = rad * np.cos(phi)
    pts[:, 1] = rad * np.sin(phi)
    s = workloads.System((10.0, 10.0, 1.0), (0.0, 0.0, 0.0), 2, pts)
    th = rng.uniform(0.0, 2 * math.pi, n).astype(np.float32)
    g, lo, hi, amb = _compare(ppa, s, th, 200, 200, 3.0, 3.0, 3.0)
    assert int(g.max()) > 1 << 17
    assert int(g.astype(np.int64).sum()) == n * (n - 1)


def test_counts_accumulate(ppa):
    s, th = _fluid(2000, 0.7, 13)
    c = ppa.pmft2d_counts(_box(s), s.points, th, 30, 30, 3.0, 3.0, 3.0)
    first = c.cpu().numpy().copy()
    ppa.pmft2d_counts(_box(s), s.points, th, 30, 30, 3.0, 3.0, 3.0, counts=c)
    np.testing.assert_array_equal(c.cpu().numpy(), 2 * first)


def test_errors(ppa):
    s, th = _fluid(100, 0.7, 14)
    with pytest.raises(ppa.PPAError) as e:
        ppa.pmft2d_counts(ppa.Box.cube(10.0), s.points, th, 10, 10, 1.0, 1.0, 1.0)
    assert e.value.code == ppa.PPA_EINVAL  # 3D box
    with pytest.raises(ppa.PPAError) as e:
        ppa.pmft2d_counts(_box(s), s.points, th, 0, 10, 1.0, 1.0, 1.0)
    assert e.value.code == ppa.PPA_EINVAL
    with pytest.raises(ppa.PPAError) as e:
        ppa.pmft2d_counts(_box(s), s.points, th, 10, 10, 1.0, 1.0,
                          0.5001 * min(_box(s).widths()[:2]))
    assert e.value.code == ppa.PPA_ERANGE


def test_fluid_2d_full_size(ppa):
    """The 2D fluid (N = 262,144, density 0.7), 200 x 200 bins on [-3, 3)^2:
    every query at once, checked on a sample of query rows against the oracle
    and in total against the ball-pair count."""
    s = workloads.fluid_2d()
    n = s.points.shape[0]
    box = _box(s)
    g = ppa.pmft2d_counts(box, s.points, s.theta, 200, 200, 3.0, 3.0, 3.0).cpu().numpy()
    nl = ppa.query_ball(box, s.points, 3.0, with_dist=False)
    total = int(g.astype(np.int64).sum())
    # every ball pair lies inside [-3, 3)^2 except bonds rounding onto the edge
    assert nl.n_pairs - 50 <= total <= nl.n_pairs
    rng = np.random.default_rng(15)
    rows = np.sort(rng.choice(n, 2000, replace=False))
    q, qth = s.points[rows], s.theta[rows]
    # the sampled rows as separate query points; their own entry (r = 0)
    # lands on the bin corner at the origin and is ambiguous there
    g_s = ppa.pmft2d_counts(box, s.points, qth, 200, 200, 3.0, 3.0, 3.0, query_points=q,
                            exclude_ii=False).cpu().numpy()
    lo, hi, amb = oracle.pmft2d_counts(oracle.make_box(s.L, s.tilt, s.dim), s.points, q, qth, 200,
                                       200, 3.0, 3.0, 3.0, exclude_ii=False)
    check_hist(g_s.reshape(-1).astype(np.int64), lo.reshape(-1), hi.reshape(-1))
    assert lo.sum() > 30000


def test_non_finite_input_is_reported(ppa):
    s, th = _fluid(500, 0.7, 16)
    pts = s.points.copy()
    pts[3, 0] = np.inf
    with pytest.raises(ppa.PPAError) as e:
        ppa.pmft2d_counts(_box(s), pts, th, 20, 20, 2.0, 2.0, 2.0)
    assert e.value.code == ppa.PPA_ENONFINITE
