"""GPU parity: k nearest selected from a stored ball NeighborList, against
the oracle's k-nearest query guarded at the list's cutoff (short rows) and
unguarded (rows holding at least k entries), with rows beyond 64 and 256
entries, ties and bad lists."""
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


def _oracle(s, k, extra=8, r_guard=0.0):
    ob = oracle.make_box(s.L, s.tilt, s.dim)
    rg = r_guard * math.sqrt(1 + REL) if r_guard > 0 else 0.0
    return oracle.knn(ob, s.points, k, extra=extra, r_guard=rg)


def _csr_ok(nl, nq):
    off = nl.offsets.cpu().numpy()
    cnt = nl.counts.cpu().numpy()
    assert off.shape == (nq + 1,) and off[0] == 0 and off[-1] == nl.n_pairs
    assert np.all(np.diff(off) == cnt)


@pytest.mark.parametrize("k,r", [(6, 1.2), (12, 1.5), (16, 1.6)])
def test_guarded_rows_from_a_ball_list(ppa, k, r):
    s = workloads.uniform(3000, 0.8, seed=700 + k, tilt=(0.2, -0.1, 0.3))
    ball = ppa.query_ball(_box(s), s.points, r)
    nl = ppa.knn_from_list(ball, k)
    _csr_ok(nl, 3000)
    idx, r2, ln = _oracle(s, k, extra=12, r_guard=r)
    check_knn_rows(nl, idx, r2, ln, range(3000), k, r_guard=r)
    d = nl.dist.cpu().numpy()
    off = nl.offsets.cpu().numpy()
    for i in range(0, 3000, 97):  # rows are sorted by distance
        assert np.all(np.diff(d[off[i]:off[i + 1]]) >= 0)


def test_long_rows_beyond_64_and_256(ppa):
    s = workloads.uniform(2500, 1.0, seed=710, dim=3)
    for r, k in ((3.0, 20), (4.2, 64)):  # about 113 and 310 entries per row
        ball = ppa.query_ball(_box(s), s.points, r)
        lens = np.diff(ball.offsets.cpu().numpy())
        assert lens.min() > k and (lens.max() > 256 or r < 4)
        nl = ppa.knn_from_list(ball, k)
        assert np.all(nl.counts.cpu().numpy() == k)
        idx, r2, ln = _oracle(s, k, extra=12)
        check_knn_rows(nl, idx, r2, ln, range(2500), k)


def test_2d_and_equal_distances(ppa):
    s = workloads.uniform(2000, 0.9, seed=720, dim=2, tilt=(0.4, 0, 0))
    ball = ppa.query_ball(_box(s), s.points, 2.0)
    nl = ppa.knn_from_list(ball, 8)
    idx, r2, ln = _oracle(s, 8, extra=12, r_guard=2.0)
    check_knn_rows(nl, idx, r2, ln, range(2000), 8, r_guard=2.0)
    # perfect FCC: the 12 at a / sqrt 2, then 2 of the 6 tied at a
    a = 4.0 ** (1.0 / 3.0)
    f = workloads.fcc(5, a)
    ball = ppa.query_ball(_box(f), f.points, 1.2 * a)
    nl = ppa.knn_from_list(ball, 14)
    idx, r2, ln = _oracle(f, 14, extra=8)
    check_knn_rows(nl, idx, r2, ln, range(f.points.shape[0]), 14)


def test_equal_to_the_query_on_the_large_fcc(ppa):
    """Every r = 2.5 row of the 1M-point noisy FCC holds more than 12 entries,
    so the selection is the unguarded 12-nearest query: sampled rows against
    the oracle, and every row against the GPU query."""
    s = workloads.large_fcc()
    n = s.points.shape[0]
    box = _box(s)
    ball = ppa.query_ball(box, s.points, 2.5)
    assert int(ball.counts.min().item()) > 12
    nl = ppa.knn_from_list(ball, 12)
    _csr_ok(nl, n)
    assert nl.n_pairs == 12 * n
    rng = np.random.default_rng(730)
    rows = np.sort(rng.choice(n, 200, replace=False))
    ob = oracle.make_box(s.L, s.tilt, 3)
    idx, r2, ln = oracle.knn(ob, s.points, 12, query_points=s.points[rows], exclude_ii=False,
                             extra=9)
    oi = np.full((200, 20), -1, np.int32)
    orr = np.full((200, 20), np.inf)
    ol = np.zeros(200, np.int32)
    for t, q in enumerate(rows):
        keep = idx[t, :ln[t]] != q
        aa, bb = idx[t, :ln[t]][keep][:20], r2[t, :ln[t]][keep][:20]
        oi[t, :len(aa)], orr[t, :len(bb)], ol[t] = aa, bb, len(aa)
    check_knn_rows(nl, oi, orr, ol, rows, 12)
    q = ppa.query_knn(box, s.points, 12)
    a_idx = nl.point_idx.cpu().numpy().reshape(n, 12)
    b_idx = q.point_idx.cpu().numpy().reshape(n, 12)
    same = (np.sort(a_idx, 1) == np.sort(b_idx, 1)).all(1)
    assert same.mean() > 0.999  # the rest differ only by near-ties at rank 12


def test_bad_lists_and_empty(ppa):
    import torch
    NL = ppa.NeighborList
    off = torch.tensor([0, 2, 5], dtype=torch.int64, device="cuda")  # 5 > capacity 3
    idx = torch.tensor([1, 0, 0], dtype=torch.int32, device="cuda")
    d = torch.tensor([0.5, 0.5, 0.7], dtype=torch.float32, device="cuda")
    with pytest.raises(ppa.PPAError) as e:
        ppa.knn_from_list(NL(off, None, idx, d, 3), 2)
    assert e.value.code == ppa.PPA_EINVAL
    off = torch.zeros(4, dtype=torch.int64, device="cuda")
    out = ppa.knn_from_list(NL(off, None, idx[:0], d[:0], 0), 3)
    assert out.n_pairs == 0
    with pytest.raises(ppa.PPAError) as e:
        ppa.knn_from_list(NL(off, None, idx[:0], d[:0], 0), 65)
    assert e.value.code == ppa.PPA_EINVAL
