"""GPU parity: batched analysis of many frames (one cell list, one sequence
of launches) against the oracle frame by frame, against per-frame calls,
and replayed from a HIP graph."""
import numpy as np
import pytest

import oracle
from paper_1906_06317_amd import workloads
from tests.parity import check_hist, check_rows

pytestmark = pytest.mark.gpu

R_MAX, BINS = 2.5, 128


@pytest.fixture(scope="module")
def ppa():
    import torch
    assert torch.cuda.is_available(), "a GPU is required"
    import paper_1906_06317_amd as m
    m.lib()
    return m


class _FrameNL:
    """Rows of one frame cut out of the batch's NeighborList."""

    def __init__(self, nl, a, b):
        off = nl.offsets.cpu().numpy()
        lo, hi = int(off[a]), int(off[b])
        import torch
        self.offsets = torch.as_tensor(off[a:b + 1] - lo)
        self.counts = nl.counts[a:b].cpu()
        self.point_idx = nl.point_idx[lo:hi].cpu()
        self.dist = nl.dist[lo:hi].cpu()


def _frames(seed, count, n_lo, n_hi, dim=3):
    fr = workloads.trajectory(seed=seed, frames=count, n_lo=n_lo, n_hi=n_hi)
    if dim == 2:
        out = []
        for k, f in enumerate(fr):
            s = workloads.uniform(f.points.shape[0], 0.8, seed=seed * 100 + k, dim=2,
                                  tilt=(f.tilt[0], 0.0, 0.0))
            out.append(s)
        fr = out
    return fr


def _plan(ppa, frames, **kw):
    boxes = [ppa.Box(f.L, f.tilt, f.dim) for f in frames]
    sizes = [f.points.shape[0] for f in frames]
    return ppa.BatchPlan(boxes, sizes, BINS, R_MAX, **kw), np.concatenate([f.points for f in frames])


def _check_against_oracle(frames, hist, nl, pb, which=None):
    hist = hist.cpu().numpy()
    for f in (range(len(frames)) if which is None else which):
        s = frames[f]
        ob = oracle.make_box(s.L, s.tilt, s.dim)
        lo, hi, _ = oracle.rdf_counts(ob, s.points, BINS, R_MAX)
        check_hist(hist[f], lo, hi)
        ref = oracle.ball_query(ob, s.points, R_MAX)
        check_rows(_FrameNL(nl, pb[f], pb[f + 1]), ref, range(s.points.shape[0]), R_MAX)


def test_small_trajectory_against_oracle_and_per_frame_calls(ppa):
    frames = _frames(11, 12, 1500, 6000)
    plan, pts = _plan(ppa, frames)
    assert plan.config()["chosen"] == 0
    hist, nl = plan.run(pts)
    _check_against_oracle(frames, hist, nl, plan.offsets_host)
    # configuration 0 uses the per-frame grid: identical to per-frame calls
    h = hist.cpu().numpy()
    off = nl.offsets.cpu().numpy()
    pidx = nl.point_idx.cpu().numpy()
    pb = plan.offsets_host
    for f, s in enumerate(frames):
        box = ppa.Box(s.L, s.tilt, s.dim)
        c, fnl = ppa.rdf_counts(box, s.points, BINS, R_MAX, neighbor_list=True)
        np.testing.assert_array_equal(h[f], c.cpu().numpy())
        fo = fnl.offsets.cpu().numpy()
        np.testing.assert_array_equal(off[pb[f]:pb[f + 1] + 1] - off[pb[f]], fo)
        np.testing.assert_array_equal(pidx[off[pb[f]]:off[pb[f + 1]]], fnl.point_idx.cpu().numpy())


def test_cell_build_chunks_and_global_counters(ppa):
    """A batch whose frames take both cell-build paths: a frame with more
    cells than a chunk counts in LDS (global counters), a frame of several
    chunks, and small frames; every frame's rows and bins against the
    oracle, with the graph's replay equal to the run."""
    import torch
    r_max, bins = 0.6, 32
    # (points, density, tilts): the sparse frame has far more than 32768
    # cells, the dense 40000-point frame fewer, in three chunks
    specs = [(40000, 0.05, (0.1, -0.2, 0.05)), (40000, 8.0, (0.0, 0.1, 0.0)),
             (3000, 1.0, (0.2, 0.0, -0.1)), (500, 1.0, (0.0, 0.0, 0.0)),
             (17000, 0.5, (-0.1, 0.1, 0.2))]
    frames = [workloads.uniform(n, rho, seed=300 + k, tilt=t)
              for k, (n, rho, t) in enumerate(specs)]
    boxes = [ppa.Box(f.L, f.tilt, f.dim) for f in frames]
    sizes = [f.points.shape[0] for f in frames]
    plan = ppa.BatchPlan(boxes, sizes, bins, r_max)
    cells = plan.cells()
    assert cells["global_frames"] == 1, cells  # the sparse frame
    assert cells["chunks"] == 3 + 1 + 1 + 2, cells  # 40000 and 17000 points: several chunks
    pts = torch.as_tensor(np.concatenate([f.points for f in frames])).cuda()
    hist, nl = plan.run(pts)
    h = hist.cpu().numpy()
    pb = plan.offsets_host
    for f, s in enumerate(frames):
        ob = oracle.make_box(s.L, s.tilt, s.dim)
        lo, hi, _ = oracle.rdf_counts(ob, s.points, bins, r_max)
        check_hist(h[f], lo, hi)
        ref = oracle.ball_query(ob, s.points, r_max)
        check_rows(_FrameNL(nl, pb[f], pb[f + 1]), ref, range(s.points.shape[0]), r_max)
    h2 = torch.zeros_like(hist)
    launch = plan.graph(pts, h2)
    launch()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(h2.cpu().numpy(), h)


def test_every_configuration_and_the_autotuner(ppa):
    frames = _frames(12, 6, 2000, 8000)
    plan, pts = _plan(ppa, frames)
    n = plan.config()["n_configs"]
    assert n >= 4
    for c in range(n):
        plan.config(c)
        hist, nl = plan.run(pts)
        _check_against_oracle(frames, hist, nl, plan.offsets_host, which=[0, len(frames) - 1])
        h = hist.cpu().numpy()
        for f, s in enumerate(frames):
            lo, hi, _ = oracle.rdf_counts(oracle.make_box(s.L, s.tilt), s.points, BINS, R_MAX)
            check_hist(h[f], lo, hi)
    ms, cfg = plan.autotune(pts, reps=2)
    assert len(ms) == n and all(t > 0 for t in ms)
    assert cfg["chosen"] == int(np.argmin(ms))
    hist, nl = plan.run(pts)
    _check_against_oracle(frames, hist, nl, plan.offsets_host, which=[1])


def test_graph_replays(ppa):
    import torch
    frames = _frames(13, 8, 1000, 5000)
    plan, pts = _plan(ppa, frames)
    p = torch.as_tensor(pts).cuda()
    h1, nl1 = plan.run(p)
    ref_idx = nl1.point_idx.cpu().numpy().copy()
    ref_h = h1.cpu().numpy().copy()
    hist = torch.zeros((len(frames), BINS), dtype=torch.int64, device="cuda")
    launch = plan.graph(p, hist)
    for k in range(3):
        launch()
        torch.cuda.synchronize()
        assert plan.ws.status() == 0
        np.testing.assert_array_equal(hist.cpu().numpy(), (k + 1) * ref_h)
        np.testing.assert_array_equal(plan.neighbor_list().point_idx.cpu().numpy(), ref_idx)
        # eager work between replays
        plan.run(p)


def test_tiny_and_empty_frames_and_2d(ppa):
    rng = np.random.default_rng(3)
    frames = _frames(14, 5, 1000, 3000)
    L = frames[0].L
    empty = workloads.System(L, (0.0, 0.0, 0.0), 3, np.zeros((0, 3), np.float32))
    one = workloads.System(L, (0.1, 0.0, 0.0), 3, rng.uniform(-2, 2, (1, 3)).astype(np.float32))
    frames = [frames[0], empty, one, frames[1], empty, frames[2]]
    plan, pts = _plan(ppa, frames)
    hist, nl = plan.run(pts)
    _check_against_oracle(frames, hist, nl, plan.offsets_host)
    assert hist[1].sum().item() == 0 and hist[2].sum().item() == 0
    f2 = _frames(15, 4, 1500, 4000, dim=2)
    plan2, pts2 = _plan(ppa, f2)
    hist2, nl2 = plan2.run(pts2)
    _check_against_oracle(f2, hist2, nl2, plan2.offsets_host)


def test_plan_errors(ppa):
    small = ppa.Box.cube(4.0)  # half width 2 < r_max
    with pytest.raises(ppa.PPAError) as e:
        ppa.BatchPlan([ppa.Box.cube(20.0), small], [10, 10], BINS, R_MAX)
    assert e.value.code == ppa.PPA_ERANGE and "frame 1" in str(e.value)
    with pytest.raises(ppa.PPAError) as e:
        ppa.BatchPlan([ppa.Box.cube(20.0), ppa.Box.cube(20.0, dim=2)], [10, 10], BINS, R_MAX)
    assert e.value.code == ppa.PPA_EINVAL


def test_full_trajectory(ppa):
    """The 256-frame trajectory (N_f log-uniform in [1e3, 2e5], own triclinic
    boxes): autotuned batch; small frames against the oracle, the largest
    frame's sampled rows against the oracle, and every frame's histogram
    against per-frame calls."""
    import torch
    frames = workloads.trajectory()
    plan, pts = _plan(ppa, frames)
    p = torch.as_tensor(pts).cuda()
    plan.autotune(p, reps=1)
    hist, nl = plan.run(p)
    sizes = np.array([f.points.shape[0] for f in frames])
    small = list(np.argsort(sizes)[:4])
    _check_against_oracle(frames, hist, nl, plan.offsets_host, which=small)
    big = int(np.argmax(sizes))
    s = frames[big]
    pb = plan.offsets_host
    rows = np.sort(np.random.default_rng(8).choice(s.points.shape[0], 100, replace=False))
    ob = oracle.make_box(s.L, s.tilt, s.dim)
    csr_off, csr_idx, csr_r2 = [0], [], []
    for q in rows:
        o, i, r = oracle.ball_query(ob, s.points, R_MAX, query_points=s.points[q:q + 1],
                                    exclude_ii=False)
        keep = i != q
        csr_idx.append(i[keep])
        csr_r2.append(r[keep])
        csr_off.append(csr_off[-1] + int(keep.sum()))
    check_rows(_FrameNL(nl, pb[big], pb[big + 1]),
               (np.array(csr_off), np.concatenate(csr_idx), np.concatenate(csr_r2)), rows, R_MAX)
    h = hist.cpu().numpy()
    total = 0
    for f, s in enumerate(frames):
        c = ppa.rdf_counts(ppa.Box(s.L, s.tilt, s.dim), s.points, BINS, R_MAX).cpu().numpy()
        total += int(c.sum())
        # a different cell width may decide pairs in the rounding band
        # differently: at most a handful per frame
        assert np.abs(h[f] - c).sum() <= max(4, int(1e-6 * c.sum()))
    assert abs(nl.n_pairs - total) <= 256 * 4


def test_non_finite_and_capacity_are_reported(ppa):
    frames = _frames(16, 3, 1000, 2000)
    plan, pts = _plan(ppa, frames)
    bad = pts.copy()
    bad[plan.offsets_host[1] + 4, 0] = np.nan
    with pytest.raises(ppa.PPAError) as e:
        plan.run(bad)
    assert e.value.code == ppa.PPA_ENONFINITE
    # the C ABI reports the overflow (the binding's run() then grows the list
    # and runs again; test_capacity_retry_and_block_shapes covers that)
    small, pts2 = _plan(ppa, frames, capacity=1000)
    small.run(pts2, check=False)
    assert small.ws.status() == ppa.PPA_ECAPACITY
    assert int(small.n_pairs.item()) > 1000  # the true count is still reported


def test_sorted_rows_and_graph(ppa):
    """A plan with sort_rows: every row ordered by frame-local neighbour
    index, holding the unsorted run's pairs; the oracle's rows match; a graph
    replay gives the same sorted list."""
    import torch
    frames = _frames(16, 6, 1000, 6000)
    plain, pts = _plan(ppa, frames)
    srt, _ = _plan(ppa, frames, sort_rows=True)
    p = torch.as_tensor(pts).cuda()
    h0, nl0 = plain.run(p)
    h1, nl1 = srt.run(p)
    assert torch.equal(h0, h1)
    off = nl0.offsets.cpu().numpy()
    assert np.array_equal(off, nl1.offsets.cpu().numpy())
    pi, pd = nl0.point_idx.cpu().numpy(), nl0.dist.cpu().numpy()
    si, sd = nl1.point_idx.cpu().numpy(), nl1.dist.cpu().numpy()
    for q in range(len(off) - 1):
        a, b = off[q], off[q + 1]
        assert np.all(np.diff(si[a:b]) > 0), f"row {q} not increasing"
        order = np.argsort(pi[a:b], kind="stable")
        assert np.array_equal(si[a:b], pi[a:b][order]) and np.array_equal(sd[a:b], pd[a:b][order])
    _check_against_oracle(frames, h1, nl1, srt.offsets_host, which=[0, 3])
    hist = torch.zeros((len(frames), BINS), dtype=torch.int64, device="cuda")
    launch = srt.graph(p, hist)
    for _ in range(2):
        launch()
        torch.cuda.synchronize()
        assert srt.ws.status() == 0
        np.testing.assert_array_equal(srt.neighbor_list().point_idx.cpu().numpy(), si)


def test_capacity_retry_and_block_shapes(ppa):
    """A plan sized too small for its list grows it and runs again (the
    histograms counted once); every configuration reports its block shape."""
    frames = _frames(17, 5, 1500, 4000)
    plan, pts = _plan(ppa, frames, capacity=1000)
    hist, nl = plan.run(pts)
    assert plan.capacity > 1000
    _check_against_oracle(frames, hist, nl, plan.offsets_host)
    shapes = set()
    for c in range(plan.config()["n_configs"]):
        cfg = plan.config(c)
        assert cfg["cells_per_item"] >= 1 and cfg["waves_per_workgroup"] in (2, 4)
        shapes.add((cfg["cells_per_item"], cfg["waves_per_workgroup"]))
    assert len(shapes) >= 3
