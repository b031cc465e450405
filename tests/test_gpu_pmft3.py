"""GPU parity: the 2D PMFT with relative orientation (XYT) and the 3D PMFT
(XYZ) against the oracle's histogram bounds, at small sizes in full and at
the benchmark sizes on sampled query rows and exact properties."""
import ctypes
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


def _obox(s):
    return oracle.make_box(s.L, s.tilt, s.dim)


def _fluid2(n, density, seed, tilt=0.0):
    rng = np.random.default_rng(seed)
    s = workloads.uniform(n, density, seed, dim=2, tilt=(tilt, 0.0, 0.0))
    th = rng.uniform(0.0, 2 * math.pi, n).astype(np.float32)
    return s, th


def _xyt(ppa, s, th, nb, m, r_max, query=None, exclude_ii=None):
    q_pts, q_th = (None, None) if query is None else query
    g = ppa.pmft_xyt_counts(_box(s), s.points, th, *nb, *m, r_max, query_points=q_pts,
                            query_angles=q_th, exclude_ii=exclude_ii).cpu().numpy()
    lo, hi, amb = oracle.pmft_xyt_counts(_obox(s), s.points, th, q_pts,
                                         th if query is None else q_th, *nb, *m, r_max,
                                         exclude_ii=exclude_ii)
    check_hist(g.reshape(-1).astype(np.int64), lo.reshape(-1), hi.reshape(-1))
    return g, lo, hi, amb


def _xyz(ppa, s, quat, nb, m, r_max, query=None, exclude_ii=None):
    q_pts, q_quat = (None, quat) if query is None else query
    g = ppa.pmft_xyz_counts(_box(s), s.points, q_quat, *nb, *m, r_max, query_points=q_pts,
                            exclude_ii=exclude_ii).cpu().numpy()
    lo, hi, amb = oracle.pmft_xyz_counts(_obox(s), s.points, q_pts, q_quat, *nb, *m, r_max,
                                         exclude_ii=exclude_ii)
    check_hist(g.reshape(-1).astype(np.int64), lo.reshape(-1), hi.reshape(-1))
    return g, lo, hi, amb


def _quats(n, seed):
    g = np.random.default_rng(seed).normal(size=(n, 4))
    return (g / np.linalg.norm(g, axis=1, keepdims=True)).astype(np.float32)


def test_xyt_small_fluid(ppa):
    s, th = _fluid2(5000, 0.7, 71)
    g, lo, hi, amb = _xyt(ppa, s, th, (30, 30, 12), (3.0, 3.0), 3.0)
    assert lo.sum() > 80000 and amb < lo.sum() * 3e-3


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_xyt_tilted_boxes_and_ragged_bins(ppa, seed):
    rng = np.random.default_rng(80 + seed)
    s, th = _fluid2(int(rng.integers(300, 4000)), float(rng.uniform(0.3, 1.2)), 90 + seed,
                    tilt=float(rng.uniform(-0.7, 0.7)))
    r = float(rng.uniform(1.0, 3.0))
    nb = (int(rng.integers(3, 40)), int(rng.integers(3, 40)), int(rng.integers(1, 25)))
    m = (r * float(rng.uniform(0.5, 1.3)), r * float(rng.uniform(0.5, 1.3)))
    _xyt(ppa, s, th, nb, m, r)


@pytest.mark.parametrize("exclude_ii", [False, True])
def test_xyt_separate_queries_and_angles_outside_one_turn(ppa, exclude_ii):
    s, th = _fluid2(3000, 0.7, 72)
    rng = np.random.default_rng(73)
    th = rng.uniform(-20.0, 20.0, th.shape[0]).astype(np.float32)
    q = workloads.uniform(800, 0.7, 74, dim=2, L=s.L).points
    qth = rng.uniform(-20.0, 20.0, q.shape[0]).astype(np.float32)
    _xyt(ppa, s, th, (20, 20, 9), (3.0, 3.0), 3.0, query=(q, qth), exclude_ii=exclude_ii)


def test_xyt_marginal_equals_the_2d_pmft_kernel(ppa):
    s, th = _fluid2(4000, 0.7, 75)
    g3 = ppa.pmft_xyt_counts(_box(s), s.points, th, 40, 40, 16, 3.0, 3.0, 3.0).cpu().numpy()
    g2 = ppa.pmft2d_counts(_box(s), s.points, th, 40, 40, 3.0, 3.0, 3.0).cpu().numpy()
    np.testing.assert_array_equal(g3.sum(2, dtype=np.int64), g2.astype(np.int64))


def test_xyz_small_fluid(ppa):
    s = workloads.fluid_3d(seed=76, n=5000, density=0.9)
    g, lo, hi, amb = _xyz(ppa, s, s.quat, (20, 20, 20), (2.0, 2.0, 2.0), 2.0)
    assert lo.sum() > 100000 and amb < lo.sum() * 3e-3


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_xyz_triclinic_boxes_and_ragged_bins(ppa, seed):
    rng = np.random.default_rng(100 + seed)
    tilt = tuple(float(t) for t in rng.uniform(-0.4, 0.4, 3))
    s = workloads.uniform(int(rng.integers(300, 4000)), float(rng.uniform(0.3, 1.2)), 110 + seed,
                          tilt=tilt)
    quat = _quats(s.points.shape[0], 120 + seed) * float(rng.uniform(0.5, 3.0))  # not unit
    r = float(rng.uniform(1.0, 2.5))
    nb = tuple(int(v) for v in rng.integers(3, 30, 3))
    m = tuple(r * float(v) for v in rng.uniform(0.5, 1.3, 3))
    _xyz(ppa, s, quat, nb, m, r)


@pytest.mark.parametrize("exclude_ii", [False, True])
def test_xyz_separate_queries(ppa, exclude_ii):
    s = workloads.fluid_3d(seed=77, n=3000, density=0.9)
    q = workloads.uniform(700, 0.9, 78, L=s.L).points
    _xyz(ppa, s, None, (15, 15, 15), (2.0, 2.0, 2.0), 2.0, query=(q, _quats(700, 79)),
         exclude_ii=exclude_ii)


def test_xyz_identity_is_the_plain_bond_histogram_and_point_symmetric(ppa):
    s = workloads.fluid_3d(seed=81, n=3000, density=0.9)
    quat = np.tile(np.array([1, 0, 0, 0], np.float32), (3000, 1))
    g, lo, hi, _ = _xyz(ppa, s, quat, (16, 16, 16), (2.0, 2.0, 2.0), 2.0)
    # bonds i -> j and j -> i are opposite
    gs = g[::-1, ::-1, ::-1]
    tol = (hi - lo) + (hi - lo)[::-1, ::-1, ::-1]
    assert np.all(np.abs(g.astype(np.int64) - gs.astype(np.int64)) <= tol)


def test_empty_queries_and_accumulation(ppa):
    import torch
    s, th = _fluid2(2000, 0.7, 82)
    q = np.zeros((0, 3), np.float32)
    c = ppa.pmft_xyt_counts(_box(s), s.points, th, 10, 10, 4, 3.0, 3.0, 3.0, query_points=q,
                            query_angles=np.zeros(0, np.float32))
    assert int(c.sum()) == 0
    c = ppa.pmft_xyt_counts(_box(s), s.points, th, 10, 10, 4, 3.0, 3.0, 3.0)
    first = c.cpu().numpy().copy()
    ppa.pmft_xyt_counts(_box(s), s.points, th, 10, 10, 4, 3.0, 3.0, 3.0, counts=c)
    np.testing.assert_array_equal(c.cpu().numpy(), 2 * first)
    s3 = workloads.fluid_3d(seed=83, n=2000, density=0.9)
    c3 = torch.zeros((8, 8, 8), dtype=torch.uint32, device="cuda")
    ppa.pmft_xyz_counts(_box(s3), s3.points, s3.quat, 8, 8, 8, 2.0, 2.0, 2.0, 2.0, counts=c3)
    f3 = c3.cpu().numpy().copy()
    ppa.pmft_xyz_counts(_box(s3), s3.points, s3.quat, 8, 8, 8, 2.0, 2.0, 2.0, 2.0, counts=c3)
    np.testing.assert_array_equal(c3.cpu().numpy(), 2 * f3)


def test_errors(ppa):
    import torch
    s, th = _fluid2(100, 0.7, 84)
    s3 = workloads.fluid_3d(seed=85, n=200, density=0.9)
    with pytest.raises(ppa.PPAError) as e:  # XYT needs a 2D box
        ppa.pmft_xyt_counts(_box(s3), s3.points, np.zeros(200), 5, 5, 5, 1.0, 1.0, 1.0)
    assert e.value.code == ppa.PPA_EINVAL
    with pytest.raises(ppa.PPAError) as e:  # XYZ needs a 3D box
        ppa.pmft_xyz_counts(_box(s), s.points, _quats(100, 1), 5, 5, 5, 1.0, 1.0, 1.0, 1.0)
    assert e.value.code == ppa.PPA_EINVAL
    with pytest.raises(ppa.PPAError) as e:
        ppa.pmft_xyt_counts(_box(s), s.points, th, 5, 0, 5, 1.0, 1.0, 1.0)
    assert e.value.code == ppa.PPA_EINVAL
    with pytest.raises(ppa.PPAError) as e:
        ppa.pmft_xyz_counts(_box(s3), s3.points, s3.quat, 5, 5, 5, 1.0, -1.0, 1.0, 1.0)
    assert e.value.code == ppa.PPA_EINVAL
    with pytest.raises(ppa.PPAError) as e:
        ppa.pmft_xyz_counts(_box(s3), s3.points, s3.quat, 5, 5, 5, 1.0, 1.0, 1.0,
                            0.5001 * min(_box(s3).widths()))
    assert e.value.code == ppa.PPA_ERANGE
    # quaternions off 16-byte alignment are refused on the host
    box = _box(s3)
    pts = torch.as_tensor(s3.points).cuda()
    qq = torch.zeros(4 * 200 + 1, dtype=torch.float32, device="cuda")
    ws = ppa.Workspace()
    wptr, wlen = ws.get(ppa.pmft_xyz_workspace_bytes(box, 200, 0, 5, 5, 5, 1.0, 1.0, 1.0, 1.0))
    counts = torch.zeros(125, dtype=torch.uint32, device="cuda")
    rc = ppa.lib().ppa_pmft_xyz(ctypes.byref(box.c()), ctypes.c_void_p(pts.data_ptr()), 200, None,
                                ctypes.c_void_p(qq.data_ptr() + 4), 200, 5, 5, 5, 1.0, 1.0, 1.0,
                                1.0, 1, 0, wptr, wlen, ctypes.c_void_p(counts.data_ptr()),
                                ppa._stream())
    assert rc == ppa.PPA_EINVAL


def test_non_finite_orientations_are_reported(ppa):
    s, th = _fluid2(500, 0.7, 86)
    th = th.copy()
    th[7] = np.nan
    with pytest.raises(ppa.PPAError) as e:
        ppa.pmft_xyt_counts(_box(s), s.points, th, 10, 10, 4, 2.0, 2.0, 2.0)
    assert e.value.code == ppa.PPA_ENONFINITE
    s3 = workloads.fluid_3d(seed=87, n=500, density=0.9)
    quat = s3.quat.copy()
    quat[11] = 0.0
    with pytest.raises(ppa.PPAError) as e:
        ppa.pmft_xyz_counts(_box(s3), s3.points, quat, 8, 8, 8, 2.0, 2.0, 2.0, 2.0)
    assert e.value.code == ppa.PPA_ENONFINITE


def test_xyt_full_size(ppa):
    """The 2D fluid (N = 262,144, density 0.7), 100 x 100 x 36 bins: every query
    at once; the marginal over t equals the 2D PMFT kernel's histogram, and a
    sample of query rows matches the oracle."""
    s = workloads.fluid_2d()
    n = s.points.shape[0]
    box = _box(s)
    nb, m = (100, 100, 36), (3.0, 3.0)
    g = ppa.pmft_xyt_counts(box, s.points, s.theta, *nb, *m, 3.0).cpu().numpy()
    g2 = ppa.pmft2d_counts(box, s.points, s.theta, 100, 100, *m, 3.0).cpu().numpy()
    np.testing.assert_array_equal(g.sum(2, dtype=np.int64), g2.astype(np.int64))
    rng = np.random.default_rng(88)
    rows = np.sort(rng.choice(n, 1500, replace=False))
    q, qth = s.points[rows], s.theta[rows]
    g_s = ppa.pmft_xyt_counts(box, s.points, s.theta, *nb, *m, 3.0, query_points=q,
                              query_angles=qth, exclude_ii=False).cpu().numpy()
    lo, hi, amb = oracle.pmft_xyt_counts(_obox(s), s.points, s.theta, q, qth, *nb, *m, 3.0,
                                         exclude_ii=False)
    check_hist(g_s.reshape(-1).astype(np.int64), lo.reshape(-1), hi.reshape(-1))
    assert lo.sum() > 20000


def test_xyz_full_size(ppa):
    """3D fluid (N = 262,144, density 0.9, random unit quaternions), 50^3 bins
    on [-2, 2)^3, r_max = 2: every query at once (total against the ball-pair
    count), and a sample of query rows against the oracle."""
    s = workloads.fluid_3d()
    n = s.points.shape[0]
    box = _box(s)
    nb, m = (50, 50, 50), (2.0, 2.0, 2.0)
    g = ppa.pmft_xyz_counts(box, s.points, s.quat, *nb, *m, 2.0).cpu().numpy()
    nl = ppa.query_ball(box, s.points, 2.0, with_dist=False)
    total = int(g.astype(np.int64).sum())
    # every bond shorter than 2 lies in [-2, 2)^3 up to rounding onto an edge
    assert nl.n_pairs - 50 <= total <= nl.n_pairs
    rng = np.random.default_rng(89)
    rows = np.sort(rng.choice(n, 1500, replace=False))
    g_s = ppa.pmft_xyz_counts(box, s.points, s.quat[rows], *nb, *m, 2.0,
                              query_points=s.points[rows], exclude_ii=False).cpu().numpy()
    lo, hi, amb = oracle.pmft_xyz_counts(_obox(s), s.points, s.points[rows], s.quat[rows], *nb,
                                         *m, 2.0, exclude_ii=False)
    check_hist(g_s.reshape(-1).astype(np.int64), lo.reshape(-1), hi.reshape(-1))
    assert lo.sum() > 30000
