"""GPU parity: ball query (NeighborList) and RDF against the FP64 oracle."""
import math

import numpy as np
import pytest

import oracle
from paper_1906_06317_amd import workloads
from tests import brute
from tests.parity import REL, check_hist, check_rows

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


def _oracle_rows(s, r_max, rows, query_points=None, exclude_ii=None):
    ob = oracle.make_box(s.L, s.tilt, s.dim)
    q = s.points if query_points is None else query_points
    if exclude_ii is None:
        exclude_ii = query_points is None
    # oracle over the selected query rows; exclude_ii needs true indices, so
    # pass all points and keep the wanted rows (small inputs) or recompute per row
    csr_off, csr_idx, csr_r2 = [0], [], []
    for qi in rows:
        o, i, r = oracle.ball_query(ob, s.points, r_max, query_points=q[qi:qi + 1], exclude_ii=False)
        if exclude_ii:
            keep = i != qi
            i, r = i[keep], r[keep]
        csr_idx.append(i)
        csr_r2.append(r)
        csr_off.append(csr_off[-1] + len(i))
    return (np.array(csr_off), np.concatenate(csr_idx) if csr_idx else np.zeros(0, np.int32),
            np.concatenate(csr_r2) if csr_r2 else np.zeros(0))


def _oracle_all(s, r_max, query_points=None, exclude_ii=None):
    ob = oracle.make_box(s.L, s.tilt, s.dim)
    return oracle.ball_query(ob, s.points, r_max, query_points=query_points, exclude_ii=exclude_ii)


def test_small_uniform_ball_and_rdf(ppa):
    s = workloads.small_uniform()
    box = _box(s)
    counts, nl = ppa.rdf_counts(box, s.points, 100, 3.0, neighbor_list=True)
    n = s.points.shape[0]
    ref = _oracle_all(s, 3.0)
    n_cert, n_amb = check_rows(nl, ref, range(n), 3.0)
    assert n_cert > 300000
    assert n_cert <= nl.n_pairs <= n_cert + n_amb
    off = nl.offsets.cpu().numpy()
    assert off[-1] == nl.n_pairs
    cnt = nl.counts.cpu().numpy()
    assert off[0] == 0 and np.all(np.diff(off) == cnt)
    lo, hi, amb = oracle.rdf_counts(oracle.make_box(s.L, s.tilt), s.points, 100, 3.0)
    g = counts.cpu().numpy()
    check_hist(g, lo, hi)
    # every listed pair is binned by its reported distance (a pair in the band
    # at r_max may be listed with a distance that rounds to r_max: not binned)
    assert g.sum() == int((nl.dist.cpu().numpy() < np.float32(3.0)).sum())
    # the same histogram from the stored list
    g2 = ppa.rdf_from_nlist(nl, 100, 3.0).cpu().numpy()
    np.testing.assert_array_equal(g, g2)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_random_triclinic_boxes(ppa, dim, seed):
    rng = np.random.default_rng(100 + 10 * dim + seed)
    L = rng.uniform(6.0, 14.0, 3)
    tilt = rng.uniform(-0.5, 0.5, 3)
    if dim == 2:
        L[2] = 1.0
        tilt[1:] = 0
    n = int(rng.integers(50, 3000))
    s = workloads.uniform(n, 1.0, seed=seed, dim=dim, tilt=tuple(tilt), L=tuple(L))
    half = 0.5 * brute.perpendicular_widths(tuple(L), tuple(tilt), dim)[:dim].min()
    for frac in (0.3, 0.7, 0.99):
        r_max = float(frac * half)
        box = _box(s)
        nl = ppa.query_ball(box, s.points, r_max)
        check_rows(nl, _oracle_all(s, r_max), range(n), r_max)
        bins = int(rng.integers(1, 200))
        r_min = float(rng.uniform(0, 0.5 * r_max))
        c = ppa.rdf_counts(box, s.points, bins, r_max, r_min=r_min).cpu().numpy()
        lo, hi, amb = oracle.rdf_counts(oracle.make_box(s.L, s.tilt, dim), s.points, bins, r_max,
                                        r_min)
        check_hist(c, lo, hi)
        # the same bins from the pass that also writes the list (r_min > 0
        # and r_min = 0 take different binning code there)
        for rm in (r_min, 0.0):
            c2, nl2 = ppa.rdf_counts(box, s.points, bins, r_max, r_min=rm, neighbor_list=True)
            if rm == 0.0:
                lo, hi, amb = oracle.rdf_counts(oracle.make_box(s.L, s.tilt, dim), s.points, bins,
                                                r_max, 0.0)
            check_hist(c2.cpu().numpy(), lo, hi)
            assert int(nl2.n_pairs) == int(nl.n_pairs)


def test_separate_query_points(ppa):
    rng = np.random.default_rng(7)
    s = workloads.uniform(2500, 0.9, seed=8, tilt=(0.3, -0.2, 0.1))
    A = workloads.lattice_vectors(s.L, s.tilt)
    q = (rng.uniform(-1.5, 1.5, (700, 3)) @ A.T).astype(np.float32)  # also outside the box
    box = _box(s)
    for excl in (False, True):
        nl = ppa.query_ball(box, s.points, 2.2, query_points=q, exclude_ii=excl)
        ob = oracle.make_box(s.L, s.tilt)
        ref = oracle.ball_query(ob, s.points, 2.2, query_points=q, exclude_ii=excl)
        check_rows(nl, ref, range(700), 2.2)
        c = ppa.rdf_counts(box, s.points, 50, 2.2, query_points=q, exclude_ii=excl).cpu().numpy()
        lo, hi, _ = oracle.rdf_counts(ob, s.points, 50, 2.2, query_points=q, exclude_ii=excl)
        check_hist(c, lo, hi)


@pytest.mark.parametrize("frac", [0.32, 0.62])
@pytest.mark.parametrize("dim", [2, 3])
def test_few_full_cells_split_among_wavefronts(ppa, dim, frac):
    """Few cells holding many queries each (a cutoff large against the box):
    the count and fill passes share each cell's queries among several
    wavefronts.  Self queries (the own entry found by its position in the
    home cell, beyond the first 64 too), separate query points with and
    without dropping equal indices, and the RDF of the same passes."""
    rng = np.random.default_rng(11 + dim)
    n = 3000
    s = workloads.uniform(n, 2.0, seed=12 + dim, dim=dim, tilt=(0.2, 0.1, -0.1) if dim == 3
                          else (0.2, 0.0, 0.0))
    half = 0.5 * brute.perpendicular_widths(tuple(s.L), tuple(s.tilt), dim)[:dim].min()
    # six cells per axis (candidates in register slots) or three (every
    # point a candidate, and home cells of more than 64 points)
    r_max = float(frac * half)
    box = _box(s)
    ob = oracle.make_box(s.L, s.tilt, dim)
    nl = ppa.query_ball(box, s.points, r_max)
    check_rows(nl, _oracle_all(s, r_max), range(n), r_max)
    A = workloads.lattice_vectors(s.L, s.tilt, dim)
    nq = 5000
    f = rng.uniform(-0.5, 0.5, (nq, 3))
    if dim == 2:
        f[:, 2] = 0.0
    q = (f @ A.T).astype(np.float32)
    q[:200] = s.points[:200]  # some queries coincide with points
    for excl in (False, True):
        nl = ppa.query_ball(box, s.points, r_max, query_points=q, exclude_ii=excl)
        ref = oracle.ball_query(ob, s.points, r_max, query_points=q, exclude_ii=excl)
        check_rows(nl, ref, range(nq), r_max)
        c = ppa.rdf_counts(box, s.points, 64, r_max, query_points=q, exclude_ii=excl).cpu().numpy()
        lo, hi, _ = oracle.rdf_counts(ob, s.points, 64, r_max, query_points=q, exclude_ii=excl)
        check_hist(c, lo, hi)


def test_self_pairs_and_coincident_points(ppa):
    pts = np.zeros((5, 3), np.float32)
    pts[3] = [1.0, 0, 0]
    pts[4] = [1.0, 0, 0]
    s = workloads.System((10.0, 10.0, 10.0), (0, 0, 0), 3, pts)
    box = _box(s)
    nl = ppa.query_ball(box, pts, 1.5, exclude_ii=False)
    cnt = nl.counts.cpu().numpy()
    assert cnt.tolist() == [5, 5, 5, 5, 5]
    nl = ppa.query_ball(box, pts, 1.5)
    assert nl.counts.cpu().numpy().tolist() == [4, 4, 4, 4, 4]
    nl = ppa.query_ball(box, pts, 0.5)
    assert nl.counts.cpu().numpy().tolist() == [2, 2, 2, 1, 1]


def test_empty_and_tiny_inputs(ppa):
    box = ppa.Box.cube(10.0)
    nl = ppa.query_ball(box, np.zeros((0, 3), np.float32), 2.0)
    assert nl.n_pairs == 0 and nl.offsets.cpu().numpy().tolist() == [0]
    nl = ppa.query_ball(box, np.zeros((1, 3), np.float32), 2.0)
    assert nl.n_pairs == 0
    q = np.zeros((0, 3), np.float32)
    nl = ppa.query_ball(box, np.ones((10, 3), np.float32), 2.0, query_points=q)
    assert nl.n_pairs == 0 and nl.offsets.shape[0] == 1


def test_dense_cluster_takes_streamed_path(ppa):
    """More than 1024 candidates in a stencil: the streamed path must agree."""
    rng = np.random.default_rng(5)
    pts = rng.normal(0, 0.6, (3000, 3)).astype(np.float32)
    s = workloads.System((20.0, 20.0, 20.0), (0.1, 0, 0), 3, pts)
    box = _box(s)
    counts, nl = ppa.rdf_counts(box, pts, 64, 1.9, neighbor_list=True)
    rows = list(range(0, 3000, 7))
    check_rows(nl, _oracle_rows(s, 1.9, rows), rows, 1.9)
    lo, hi, _ = oracle.rdf_counts(oracle.make_box(s.L, s.tilt), pts, 64, 1.9)
    check_hist(counts.cpu().numpy(), lo, hi)


def test_capacity_overflow_reported_then_retry(ppa):
    import torch
    s = workloads.small_uniform()
    box = _box(s)
    nl = ppa.query_ball(box, s.points, 3.0, capacity=10)  # binding retries with the exact size
    rows = list(range(0, 4096, 5))
    check_rows(nl, _oracle_rows(s, 3.0, rows), rows, 3.0)
    # raw call: capacity 1 -> PPA_ECAPACITY with the true count reported
    import ctypes
    L = ppa.lib()
    pts = torch.as_tensor(s.points).cuda()
    n = pts.shape[0]
    ws = ppa.Workspace()
    wptr, wlen = ws.get(ppa.workspace_bytes(box, n, 0, 3.0, ppa.PPA_WS_NLIST))
    off = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    cnt = torch.empty(n, dtype=torch.int32, device="cuda")
    pidx = torch.empty(1, dtype=torch.int32, device="cuda")
    npairs = torch.zeros(1, dtype=torch.int64, device="cuda")
    rc = L.ppa_query_ball(ctypes.byref(box.c()), ctypes.c_void_p(pts.data_ptr()), n, None, n, 3.0, 1,
                          0, wptr, wlen, ctypes.c_void_p(off.data_ptr()),
                          ctypes.c_void_p(cnt.data_ptr()), ctypes.c_void_p(pidx.data_ptr()), None,
                          1, ctypes.c_void_p(npairs.data_ptr()),
                          ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0
    assert ws.status() == ppa.PPA_ECAPACITY
    assert int(npairs.item()) == nl.n_pairs


def test_nonfinite_input_reported(ppa):
    s = workloads.small_uniform()
    pts = s.points.copy()
    pts[17, 1] = np.nan
    with pytest.raises(ppa.PPAError) as e:
        ppa.query_ball(_box(s), pts, 3.0)
    assert e.value.code == ppa.PPA_ENONFINITE


def test_host_errors(ppa):
    s = workloads.small_uniform()
    with pytest.raises(ppa.PPAError) as e:
        ppa.query_ball(_box(s), s.points, 9.0)
    assert e.value.code == ppa.PPA_ERANGE
    with pytest.raises(ppa.PPAError) as e:
        ppa.rdf_counts(_box(s), s.points, 0, 3.0)
    assert e.value.code == ppa.PPA_EINVAL


def test_deterministic_rows(ppa):
    s = workloads.small_uniform()
    box = _box(s)
    a = ppa.query_ball(box, s.points, 3.0)
    b = ppa.query_ball(box, s.points, 3.0)
    assert a.n_pairs == b.n_pairs
    assert np.array_equal(a.offsets.cpu().numpy(), b.offsets.cpu().numpy())
    assert np.array_equal(a.point_idx.cpu().numpy(), b.point_idx.cpu().numpy())
    assert np.array_equal(a.dist.cpu().numpy(), b.dist.cpu().numpy())


def test_large_fcc_sampled_rows_and_rdf(ppa):
    """N = 1,048,576 noisy FCC in a tilted box, in the launch configuration the
    benchmark times (one pass, list + fused RDF): sampled rows against the
    oracle, and the full histogram against properties that hold at any size."""
    import torch
    s = workloads.large_fcc()
    box = _box(s)
    n = s.points.shape[0]
    counts, nl = ppa.rdf_counts(box, s.points, 256, 2.5, neighbor_list=True)
    rng = np.random.default_rng(2)
    rows = np.unique(np.concatenate([rng.choice(n, 250, replace=False), [0, 1, n - 1, n // 2]]))
    n_cert, n_amb = check_rows(nl, _oracle_rows(s, 2.5, rows), rows, 2.5)
    assert n_cert > 60 * len(rows)
    g = counts.cpu().numpy()
    assert g.sum() == int((nl.dist.cpu().numpy() < np.float32(2.5)).sum())
    assert nl.n_pairs - g.sum() < 100
    np.testing.assert_array_equal(g, ppa.rdf_from_nlist(nl, 256, 2.5).cpu().numpy())
    cnt = nl.counts.cpu().numpy()
    assert cnt.sum() == nl.n_pairs
    assert cnt.min() >= 50 and cnt.max() <= 100
    # the histogram restricted to the sampled query rows against the oracle
    q = s.points[rows]
    sub = ppa.rdf_counts(box, s.points, 256, 2.5, query_points=q, exclude_ii=False).cpu().numpy()
    lo, hi, _ = oracle.rdf_counts(oracle.make_box(s.L, s.tilt), s.points, 256, 2.5,
                                  query_points=q, exclude_ii=False)
    # a query point sits on itself at r = 0, which falls in bin 0 for both
    check_hist(sub, lo, hi)


def test_small_cutoff_in_sparse_box_uses_exact_test(ppa):
    """Cells far larger than r_max (few points, capped cell count): the host
    rejects the expanded in/out test and the difference form runs."""
    rng = np.random.default_rng(12)
    centres = rng.uniform(-25, 25, (40, 3))
    pts = (centres[:, None, :] + rng.normal(0, 0.3, (40, 10, 3))).reshape(-1, 3).astype(np.float32)
    s = workloads.System((50.0, 50.0, 50.0), (0.1, 0.0, -0.1), 3, pts)
    box = _box(s)
    counts, nl = ppa.rdf_counts(box, pts, 20, 0.5, neighbor_list=True)
    check_rows(nl, _oracle_all(s, 0.5), range(pts.shape[0]), 0.5)
    lo, hi, _ = oracle.rdf_counts(oracle.make_box(s.L, s.tilt), pts, 20, 0.5)
    check_hist(counts.cpu().numpy(), lo, hi)
    assert nl.n_pairs > 500


def test_unaligned_output_buffers_large(ppa):
    """Row counts and offsets at addresses that are not 16-byte aligned (views
    one element into larger buffers) take the scalar path of the scan's long
    tiles (2^17 rows and more); the list must equal the one written to
    aligned buffers, and sampled rows match the oracle."""
    import ctypes
    import torch
    s = workloads.uniform(200_000, 0.8, 1011)
    box = _box(s)
    r_max = 1.6
    ref = ppa.query_ball(box, s.points, r_max)
    L = ppa.lib()
    pts = torch.as_tensor(s.points).cuda()
    n = pts.shape[0]
    ws = ppa.Workspace()
    wptr, wlen = ws.get(ppa.workspace_bytes(box, n, 0, r_max, ppa.PPA_WS_NLIST))
    off_buf = torch.zeros(n + 2, dtype=torch.int64, device="cuda")
    cnt_buf = torch.zeros(n + 1, dtype=torch.int32, device="cuda")
    off, cnt = off_buf[1:], cnt_buf[1:]
    assert off.data_ptr() % 16 != 0 and cnt.data_ptr() % 16 != 0
    P = ref.n_pairs
    pidx = torch.empty(P, dtype=torch.int32, device="cuda")
    dist = torch.empty(P, dtype=torch.float32, device="cuda")
    npairs = torch.zeros(1, dtype=torch.int64, device="cuda")
    rc = L.ppa_query_ball(ctypes.byref(box.c()), ctypes.c_void_p(pts.data_ptr()), n, None, n,
                          r_max, 1, 0, wptr, wlen, ctypes.c_void_p(off.data_ptr()),
                          ctypes.c_void_p(cnt.data_ptr()), ctypes.c_void_p(pidx.data_ptr()),
                          ctypes.c_void_p(dist.data_ptr()), P, ctypes.c_void_p(npairs.data_ptr()),
                          ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0 and ws.status() == 0
    assert int(npairs.item()) == P
    assert torch.equal(off, ref.offsets)
    assert torch.equal(cnt, (ref.offsets[1:] - ref.offsets[:-1]).to(torch.int32))
    assert torch.equal(pidx, ref.point_idx[:P]) and torch.equal(dist, ref.dist[:P])
    assert int(off_buf[0].item()) == 0 and int(cnt_buf[0].item()) == 0  # nothing written before
    rows = list(range(0, n, 997)) + [n - 1]
    check_rows(ref, _oracle_rows(s, r_max, rows), rows, r_max)


def _rows_sorted_and_same(nl_sorted, nl_plain):
    """Every row of nl_sorted is increasing in j and holds the same (j, r)
    pairs as the same row of nl_plain."""
    off = nl_plain.offsets.cpu().numpy()
    assert np.array_equal(off, nl_sorted.offsets.cpu().numpy())
    pi, pd = nl_plain.point_idx.cpu().numpy(), nl_plain.dist.cpu().numpy()
    si, sd = nl_sorted.point_idx.cpu().numpy(), nl_sorted.dist.cpu().numpy()
    n_long = 0
    for q in range(len(off) - 1):
        a, b = off[q], off[q + 1]
        if b - a > 256:
            n_long += 1
        assert np.all(np.diff(si[a:b]) > 0), f"row {q} not increasing"
        order = np.argsort(pi[a:b], kind="stable")
        assert np.array_equal(si[a:b], pi[a:b][order]), f"row {q}: different neighbours"
        assert np.array_equal(sd[a:b], pd[a:b][order]), f"row {q}: distances not moved with j"
    return n_long


def test_sort_rows_short_rows_against_oracle(ppa):
    """sort_rows: rows of about 90 entries (staged in LDS), ordered by j, the
    oracle's canonical order for the sampled rows."""
    s = workloads.small_uniform()
    box = _box(s)
    plain = ppa.query_ball(box, s.points, 3.0)
    srt = ppa.query_ball(box, s.points, 3.0, sort_rows=True)
    assert _rows_sorted_and_same(srt, plain) == 0
    rows = list(range(0, 4096, 37))
    check_rows(srt, _oracle_rows(s, 3.0, rows), rows, 3.0)
    # the oracle lists each row by increasing j: the certain part matches in order
    o_off, o_idx, o_r2 = _oracle_rows(s, 3.0, rows)
    off = srt.offsets.cpu().numpy()
    pidx = srt.point_idx.cpu().numpy()
    lo = 9.0 * (1 - REL)
    for k, q in enumerate(rows):
        oi, orr = o_idx[o_off[k]:o_off[k + 1]], o_r2[o_off[k]:o_off[k + 1]]
        certain = np.sort(oi[orr < lo])
        g = pidx[off[q]:off[q + 1]]
        assert np.array_equal(g[np.isin(g, certain)], certain)


def test_sort_rows_long_rows_bitonic(ppa):
    """Rows longer than the LDS stage (256) are sorted in place by the bitonic
    network; lengths are not powers of two.  Separate query points too."""
    s = workloads.uniform(6000, 8.0, 1012)   # r = 2.7: about 660 neighbours per point
    box = _box(s)
    plain = ppa.query_ball(box, s.points, 2.7)
    srt = ppa.query_ball(box, s.points, 2.7, sort_rows=True)
    assert _rows_sorted_and_same(srt, plain) > 1000
    q = workloads.uniform(500, 8.0, 1013, L=s.L).points
    plain = ppa.query_ball(box, s.points, 2.7, query_points=q)
    srt = ppa.query_ball(box, s.points, 2.7, query_points=q, sort_rows=True)
    assert _rows_sorted_and_same(srt, plain) > 100


def test_sort_rows_with_rdf_and_capacity_retry(ppa):
    """The RDF pass with its list sorted: the histogram is unchanged, the
    list sorted; a first attempt with too small a capacity is retried."""
    import torch
    s = workloads.small_uniform()
    box = _box(s)
    h0, plain = ppa.rdf_counts(box, s.points, 100, 3.0, neighbor_list=True)
    h1, srt = ppa.rdf_counts(box, s.points, 100, 3.0, neighbor_list=True, sort_rows=True,
                             capacity=1000)
    assert torch.equal(h0, h1)
    _rows_sorted_and_same(srt, plain)


def test_sort_rows_without_distances(ppa):
    """sort_rows with no distance output (with_dist=False): indices only,
    short rows (LDS) and long rows (bitonic) alike."""
    for s, r in ((workloads.small_uniform(), 3.0), (workloads.uniform(3000, 8.0, 1014), 2.7)):
        box = _box(s)
        plain = ppa.query_ball(box, s.points, r, with_dist=False)
        srt = ppa.query_ball(box, s.points, r, with_dist=False, sort_rows=True)
        assert srt.dist is None
        off = plain.offsets.cpu().numpy()
        pi, si = plain.point_idx.cpu().numpy(), srt.point_idx.cpu().numpy()
        for q in range(len(off) - 1):
            a, b = off[q], off[q + 1]
            assert np.array_equal(si[a:b], np.sort(pi[a:b])), f"row {q}"
