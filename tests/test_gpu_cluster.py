"""GPU parity: clusters (connected components of neighbour bonds) against
the oracle, bit-exact labels, ids and sizes: on lists the oracle built (both
sides see the same bonds) and end to end through the GPU ball query where the
oracle finds no ambiguous pair; at 1M nodes on a seeded synthetic bond list
(exact) and on the GPU list of a dilute fluid (properties)."""
import numpy as np
import pytest

import oracle
from paper_1906_06317_amd import workloads

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


def _compare(ppa, n, off, idx):
    labels, cidx, sizes, k = ppa.clusters((off, idx), n)
    ol, oc, os_ = oracle.clusters(n, off, idx)
    np.testing.assert_array_equal(labels.cpu().numpy(), ol)
    np.testing.assert_array_equal(cidx.cpu().numpy(), oc)
    np.testing.assert_array_equal(sizes.cpu().numpy(), os_)
    assert k == os_.shape[0]
    return k


@pytest.mark.parametrize("dim,density,r_cut", [(3, 0.9, 0.75), (3, 0.9, 0.95), (2, 0.8, 0.8),
                                               (2, 0.8, 1.2)])
def test_oracle_lists_below_and_above_percolation(ppa, dim, density, r_cut):
    s = workloads.uniform(4000, density, seed=600 + dim, dim=dim, tilt=(0.2, -0.1, 0.15))
    off, idx, _ = oracle.ball_query(oracle.make_box(s.L, s.tilt, dim), s.points, r_cut)
    k = _compare(ppa, 4000, off, idx.astype(np.int32))
    assert k >= 1


def test_end_to_end_through_the_gpu_ball_query(ppa):
    s = workloads.uniform(6000, 1.0, seed=610, tilt=(0.3, 0.1, -0.2))
    box = _box(s)
    nl = ppa.query_ball(box, s.points, 0.8)
    labels, cidx, sizes, k = ppa.clusters(nl, 6000)
    ob = oracle.make_box(s.L, s.tilt, 3)
    off, idx, _ = oracle.ball_query(ob, s.points, 0.8)
    lo, hi, amb = oracle.rdf_counts(ob, s.points, 1, 0.8)
    ol, oc, os_ = oracle.clusters(6000, off, idx)
    if amb == 0:
        np.testing.assert_array_equal(labels.cpu().numpy(), ol)
        np.testing.assert_array_equal(sizes.cpu().numpy(), os_)
    assert 100 < k < 6000


def test_one_directional_knn_lists(ppa):
    s = workloads.uniform(3000, 0.9, seed=620)
    idx, r2, ln = oracle.knn(oracle.make_box(s.L, s.tilt, 3), s.points, 2, extra=0)
    off = np.arange(0, 2 * 3000 + 1, 2, dtype=np.int64)
    _compare(ppa, 3000, off, idx[:, :2].reshape(-1).astype(np.int32))


def test_chains_and_singletons(ppa):
    """Long chains (deep trees in the union-find) and isolated points."""
    n = 5000
    rng = np.random.default_rng(630)
    perm = rng.permutation(n)
    rows = [[] for _ in range(n)]
    # chains of 1000 points in random index order, plus 200 isolated points
    for c in range(4):
        ch = perm[c * 1000:(c + 1) * 1000]
        for a, b in zip(ch[:-1], ch[1:]):
            rows[a].append(b)
    off = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int64)
    idx = np.array([j for r in rows for j in r], np.int32)
    assert _compare(ppa, n, off, idx) == 4 + 1000


def test_bad_lists_and_empty(ppa):
    labels, cidx, sizes, k = ppa.clusters((np.zeros(6, np.int64), np.zeros(0, np.int32)), 5)
    np.testing.assert_array_equal(labels.cpu().numpy(), np.arange(5))
    assert k == 5
    with pytest.raises(ppa.PPAError) as e:
        ppa.clusters((np.array([0, 1, 1], np.int64), np.array([7], np.int32)), 2)
    assert e.value.code == ppa.PPA_EINVAL
    with pytest.raises(ppa.PPAError) as e:
        ppa.clusters((np.array([0, 3, 3], np.int64), np.array([1], np.int32)), 2)
    assert e.value.code == ppa.PPA_EINVAL
    labels, cidx, sizes, k = ppa.clusters((np.zeros(1, np.int64), np.zeros(0, np.int32)), 0)
    assert k == 0


def test_dilute_fluid_1m(ppa):
    """N = 1,048,576 uniform at density 1, bonds within 0.8 (about 2.1 per
    point, below the percolation threshold), list from the GPU ball query:
    properties that hold at any size (bonded points share a label, a label
    is the index of a member that labels itself, sizes add up)."""
    s = workloads.uniform(1 << 20, 1.0, seed=640)
    nl = ppa.query_ball(_box(s), s.points, 0.8)
    labels, cidx, sizes, k = ppa.clusters(nl, 1 << 20)
    lab = labels.cpu().numpy()
    off = nl.offsets.cpu().numpy()
    idx = nl.point_idx.cpu().numpy()
    rows = np.repeat(np.arange(1 << 20), np.diff(off))
    assert np.all(lab[rows] == lab[idx])
    assert np.all(lab <= np.arange(1 << 20)) and np.all(lab[lab] == lab)
    assert sizes.cpu().numpy().sum() == 1 << 20 and k == np.unique(lab).size
    assert 100000 < k < 1 << 20


def test_synthetic_graph_1m_against_oracle(ppa):
    """A seeded random bond list on 1,048,576 nodes (two short-range links
    per node, varied component sizes, some links one-directional), given to
    both sides: labels, ids and sizes are bit-exact."""
    n = 1 << 20
    rng = np.random.default_rng(650)
    deg = rng.integers(0, 3, n)
    off = np.concatenate([[0], np.cumsum(deg)]).astype(np.int64)
    rows = np.repeat(np.arange(n), deg)
    idx = ((rows + rng.integers(-40, 41, rows.shape[0])) % n).astype(np.int32)
    keep = rng.random(rows.shape[0]) < 0.6
    idx = np.where(keep, idx, rows).astype(np.int32)  # some self bonds (ignored)
    k = _compare(ppa, n, off, idx)
    assert 1000 < k < n


def _compare_symmetric(ppa, n, off, idx):
    """The symmetric-list path against the oracle."""
    labels, cidx, sizes, k = ppa.clusters((off, idx), n, symmetric=True)
    ol, oc, os_ = oracle.clusters(n, off, idx)
    np.testing.assert_array_equal(labels.cpu().numpy(), ol)
    np.testing.assert_array_equal(cidx.cpu().numpy(), oc)
    np.testing.assert_array_equal(sizes.cpu().numpy(), os_)
    return k


@pytest.mark.parametrize("dim,density,r_cut", [(3, 0.9, 0.75), (3, 0.9, 0.95), (3, 0.9, 1.4),
                                               (2, 0.8, 0.8), (2, 0.8, 1.2)])
def test_symmetric_flag_against_oracle(ppa, dim, density, r_cut):
    """Oracle ball lists (symmetric): below, near and above percolation, the
    sampled-rounds path gives the oracle's components."""
    s = workloads.uniform(4000, density, seed=620 + dim, dim=dim, tilt=(0.2, -0.1, 0.15))
    off, idx, _ = oracle.ball_query(oracle.make_box(s.L, s.tilt, dim), s.points, r_cut)
    assert _compare_symmetric(ppa, 4000, off, idx.astype(np.int32)) >= 1


@pytest.mark.parametrize("r_cut", [0.8, 1.2, 1.6])
def test_symmetric_flag_same_labels_1m(ppa, r_cut):
    """N = 1,048,576 uniform, GPU ball lists below and above percolation: the
    flagged call returns exactly the unflagged labels, and the labels hold the
    properties any size has (bonded points share a label, a label names a
    member that labels itself)."""
    s = workloads.uniform(1 << 20, 1.0, seed=640)
    nl = ppa.query_ball(_box(s), s.points, r_cut)
    a = ppa.clusters(nl, 1 << 20)
    b = ppa.clusters(nl, 1 << 20, symmetric=True)
    for x, y in zip(a[:3], b[:3]):
        assert np.array_equal(x.cpu().numpy(), y.cpu().numpy())
    assert a[3] == b[3]
    lab = b[0].cpu().numpy()
    off = nl.offsets.cpu().numpy()
    idx = nl.point_idx.cpu().numpy()
    rows = np.repeat(np.arange(1 << 20), np.diff(off))
    assert np.all(lab[rows] == lab[idx])
    assert np.all(lab <= np.arange(1 << 20)) and np.all(lab[lab] == lab)


def test_symmetric_flag_small_and_bad_lists(ppa):
    """The symmetric path on degenerate inputs: an empty list, a list with an
    out-of-range index and enough bonds for the hooking rounds to run
    (reported, no fault), and a long symmetric chain (one component whose
    sampled bonds form a path)."""
    labels, cidx, sizes, k = ppa.clusters((np.zeros(6, np.int64), np.zeros(0, np.int32)), 5,
                                          symmetric=True)
    np.testing.assert_array_equal(labels.cpu().numpy(), np.arange(5))
    assert k == 5
    with pytest.raises(ppa.PPAError) as e:
        ppa.clusters((np.array([0, 3, 6], np.int64), np.array([1, 7, 1, 0, 9, 0], np.int32)), 2,
                     symmetric=True)
    assert e.value.code == ppa.PPA_EINVAL
    n = 3000  # chain 0 - 1 - ... - n-1 and a separate chain of the last 500 points
    rows = []
    for i in range(n):
        nb = [j for j in (i - 1, i + 1) if 0 <= j < n and not ((i < 2500) ^ (j < 2500))]
        rows.append(nb + nb)  # listed twice: four entries, so the rounds run
    off = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int64)
    idx = np.concatenate([np.array(r, np.int32) for r in rows])
    k = _compare_symmetric(ppa, n, off, idx)
    assert k == 2
