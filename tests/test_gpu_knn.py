"""GPU parity: k-nearest query against the FP64 oracle.

Rows must hold the oracle's k nearest (r^2, j) neighbours, except that a
neighbour whose r^2 lies within 1e-5 (relative) of the k-th one may be
swapped for another such neighbour; rows are sorted by distance.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1906_06317_amd import workloads
from tests.parity import REL, check_knn_rows

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


def _oracle(s, k, query_points=None, exclude_ii=None, extra=8, r_guard=0.0):
    ob = oracle.make_box(s.L, s.tilt, s.dim)
    rg = r_guard * math.sqrt(1 + REL) if r_guard > 0 else 0.0
    return oracle.knn(ob, s.points, k, query_points=query_points, exclude_ii=exclude_ii,
                      extra=extra, r_guard=rg)


def _oracle_self_rows(s, k, rows, extra=8):
    """Oracle rows of points querying themselves (own entry dropped), for a subset."""
    ob = oracle.make_box(s.L, s.tilt, s.dim)
    idx, r2, ln = oracle.knn(ob, s.points, k, query_points=s.points[rows], exclude_ii=False,
                             extra=extra + 1)
    m = k + extra
    oi = np.full((len(rows), m), -1, np.int32)
    orr = np.full((len(rows), m), np.inf)
    ol = np.zeros(len(rows), np.int32)
    for t, q in enumerate(rows):
        keep = idx[t, :ln[t]] != q
        a, b = idx[t, :ln[t]][keep][:m], r2[t, :ln[t]][keep][:m]
        oi[t, :len(a)], orr[t, :len(b)], ol[t] = a, b, len(a)
    return oi, orr, ol


def _check_csr(nl, nq, k=None):
    off = nl.offsets.cpu().numpy()
    cnt = nl.counts.cpu().numpy()
    assert off.shape == (nq + 1,) and off[0] == 0 and off[-1] == nl.n_pairs
    assert np.all(np.diff(off) == cnt)
    if k is not None:
        np.testing.assert_array_equal(off, k * np.arange(nq + 1))


@pytest.mark.parametrize("k", [1, 12, 33, 64])
def test_small_uniform(ppa, k):
    s = workloads.small_uniform()
    n = s.points.shape[0]
    nl = ppa.query_knn(_box(s), s.points, k)
    _check_csr(nl, n, k)
    idx, r2, ln = _oracle(s, k)
    n_cert, n_amb = check_knn_rows(nl, idx, r2, ln, range(n), k)
    assert n_cert >= n * k - n_amb


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_random_triclinic_boxes(ppa, dim, seed):
    rng = np.random.default_rng(500 + seed)
    n = int(rng.integers(300, 3000))
    tilt = tuple(rng.uniform(-0.6, 0.6, 3)) if dim == 3 else (float(rng.uniform(-0.6, 0.6)), 0, 0)
    s = workloads.uniform(n, float(rng.uniform(0.3, 1.5)), seed=seed, dim=dim, tilt=tilt)
    k = int(rng.integers(1, 40))
    nl = ppa.query_knn(_box(s), s.points, k)
    _check_csr(nl, n, k)
    idx, r2, ln = _oracle(s, k)
    check_knn_rows(nl, idx, r2, ln, range(n), k)


def test_perfect_fcc_twelve_at_a_over_root2(ppa):
    a = 4.0 ** (1.0 / 3.0)
    s = workloads.fcc(6, a)
    n = s.points.shape[0]
    nl = ppa.query_knn(_box(s), s.points, 12)
    _check_csr(nl, n, 12)
    d = nl.dist.cpu().numpy().reshape(n, 12)
    np.testing.assert_allclose(d, a / math.sqrt(2.0), rtol=1e-5)
    idx, r2, ln = _oracle(s, 12)
    check_knn_rows(nl, idx, r2, ln, range(n), 12)
    # k = 13 reaches the second shell (6 sites at a, tied): any one of them
    nl13 = ppa.query_knn(_box(s), s.points, 13)
    idx, r2, ln = _oracle(s, 13)
    check_knn_rows(nl13, idx, r2, ln, range(n), 13)
    np.testing.assert_allclose(nl13.dist.cpu().numpy().reshape(n, 13)[:, 12], a, rtol=1e-5)


@pytest.mark.parametrize("exclude_ii", [False, True])
def test_separate_query_points(ppa, exclude_ii):
    s = workloads.small_uniform()
    q = workloads.uniform(1500, 0.8, seed=77, L=s.L).points
    nl = ppa.query_knn(_box(s), s.points, 10, query_points=q, exclude_ii=exclude_ii)
    _check_csr(nl, q.shape[0], 10)
    idx, r2, ln = _oracle(s, 10, query_points=q, exclude_ii=exclude_ii)
    check_knn_rows(nl, idx, r2, ln, range(q.shape[0]), 10)


def test_self_included_when_not_excluded(ppa):
    s = workloads.small_uniform(n=2000)
    nl = ppa.query_knn(_box(s), s.points, 5, exclude_ii=False)
    pidx = nl.point_idx.cpu().numpy().reshape(-1, 5)
    dist = nl.dist.cpu().numpy().reshape(-1, 5)
    np.testing.assert_array_equal(pidx[:, 0], np.arange(2000))
    assert np.all(dist[:, 0] == 0.0)


def test_r_guard_short_rows(ppa):
    s = workloads.uniform(3000, 0.5, seed=9)
    k, rg = 16, 1.6
    nl = ppa.query_knn(_box(s), s.points, k, r_guard=rg)
    _check_csr(nl, 3000)
    cnt = nl.counts.cpu().numpy()
    assert cnt.min() < k and cnt.max() == k
    idx, r2, ln = _oracle(s, k, r_guard=rg, extra=12)
    check_knn_rows(nl, idx, r2, ln, range(3000), k, r_guard=rg)
    assert np.all(nl.dist.cpu().numpy() < np.float32(rg))


def test_fewer_points_than_k(ppa):
    rng = np.random.default_rng(3)
    L = 10.0
    pts = np.zeros((6, 3), np.float32)
    pts[:] = rng.normal(0.0, 0.7, size=(6, 3))  # a cluster well inside half the box
    s = workloads.System((L, L, L), (0.0, 0.0, 0.0), 3, pts)
    nl = ppa.query_knn(_box(s), pts, 12)
    _check_csr(nl, 6)
    np.testing.assert_array_equal(nl.counts.cpu().numpy(), 5)
    idx, r2, ln = _oracle(s, 12)
    check_knn_rows(nl, idx, r2, ln, range(6), 12)
    nl = ppa.query_knn(_box(s), pts, 12, exclude_ii=False)
    np.testing.assert_array_equal(nl.counts.cpu().numpy(), 6)


def test_neighbour_beyond_half_box_is_range_error(ppa):
    pts = np.array([[-4.5, 0, 0], [0, 0, 0], [3.0, 0.5, 0], [0, 4.0, 0], [1, 1, 4.2]], np.float32)
    box = ppa.Box.cube(10.0)
    with pytest.raises(ppa.PPAError) as e:
        ppa.query_knn(box, pts, 4)
    assert e.value.code == ppa.PPA_ERANGE
    # with a guard below half the box the same query is valid and rows shrink
    nl = ppa.query_knn(box, pts, 4, r_guard=4.9)
    assert int(nl.counts.cpu().numpy().min()) < 4


def test_clustered_points_use_the_shell_search(ppa):
    """A dense blob (home cells beyond the register slots) in a sparse gas
    (queries whose k-th neighbour lies past the block)."""
    rng = np.random.default_rng(11)
    L = 30.0
    blob = rng.normal(0.0, 1.0, size=(4000, 3))
    gas = rng.uniform(-L / 2, L / 2, size=(4000, 3))
    pts = np.ascontiguousarray(np.concatenate([blob, gas]), dtype=np.float32)
    s = workloads.System((L, L, L), (0.1, -0.2, 0.05), 3, pts)
    for k in (12, 40):
        nl = ppa.query_knn(_box(s), pts, k)
        _check_csr(nl, 8000, k)
        idx, r2, ln = _oracle(s, k)
        check_knn_rows(nl, idx, r2, ln, range(8000), k)


def test_coincident_points_tie_by_index(ppa):
    s = workloads.small_uniform(n=1000)
    pts = s.points.copy()
    pts[500:510] = pts[7]  # eleven points at one position
    s = workloads.System(s.L, s.tilt, 3, pts)
    nl = ppa.query_knn(_box(s), pts, 12)
    row = nl.point_idx.cpu().numpy().reshape(-1, 12)[7]
    np.testing.assert_array_equal(row[:10], np.arange(500, 510))
    # rows near the group see an 11-way exact tie, which may straddle rank k
    idx, r2, ln = _oracle(s, 12, extra=16)
    check_knn_rows(nl, idx, r2, ln, range(1000), 12)


def test_empty_inputs(ppa):
    box = ppa.Box.cube(10.0)
    import torch
    nl = ppa.query_knn(box, np.zeros((0, 3), np.float32), 4)
    assert nl.n_pairs == 0 and nl.offsets.shape[0] == 1
    q = np.random.default_rng(0).uniform(-5, 5, (7, 3)).astype(np.float32)
    nl = ppa.query_knn(box, np.zeros((0, 3), np.float32), 4, query_points=q)
    assert nl.n_pairs == 0
    np.testing.assert_array_equal(nl.offsets.cpu().numpy(), 0)
    nl = ppa.query_knn(box, q, 3, query_points=np.zeros((0, 3), np.float32))
    assert nl.n_pairs == 0 and nl.offsets.cpu().numpy().tolist() == [0]
    torch.cuda.synchronize()


def test_deterministic(ppa):
    s = workloads.uniform(5000, 0.9, seed=21, tilt=(0.2, 0.1, -0.3))
    a = ppa.query_knn(_box(s), s.points, 12)
    b = ppa.query_knn(_box(s), s.points, 12)
    assert np.array_equal(a.point_idx.cpu().numpy(), b.point_idx.cpu().numpy())
    assert np.array_equal(a.dist.cpu().numpy(), b.dist.cpu().numpy())


def test_large_fcc_sampled_rows(ppa):
    """The large noisy FCC system (N = 1,048,576, tilted box), k = 12."""
    s = workloads.large_fcc()
    n = s.points.shape[0]
    nl = ppa.query_knn(_box(s), s.points, 12)
    _check_csr(nl, n, 12)
    rng = np.random.default_rng(5)
    rows = np.sort(rng.choice(n, 200, replace=False))
    oi, orr, ol = _oracle_self_rows(s, 12, rows)
    n_cert, n_amb = check_knn_rows(nl, oi, orr, ol, rows, 12)
    assert n_cert >= 200 * 12 - n_amb
    # properties at every row: sorted, no self, all distances short
    d = nl.dist.cpu().numpy().reshape(n, 12)
    assert np.all(np.diff(d, axis=1) >= 0)
    assert float(d.max()) < 2.5
    p = nl.point_idx.cpu().numpy().reshape(n, 12)
    assert not np.any(p == np.arange(n)[:, None])


def test_non_finite_input_is_reported(ppa):
    s = workloads.small_uniform(n=500)
    pts = s.points.copy()
    pts[17, 1] = np.nan
    with pytest.raises(ppa.PPAError) as e:
        ppa.query_knn(_box(s), pts, 6)
    assert e.value.code == ppa.PPA_ENONFINITE
