"""GPU parity at the benchmark sizes, in full: the launches bench.py times,
compared element by element with expected values the FP64 oracle wrote
(tests/golden/make_golden.py, brute force over every pair).

  * the 2^20-point FCC ball query + 256-bin RDF (one ppa_rdf call writing
    the NeighborList and the histogram): every bin inside the oracle's
    [lo, hi], and every row's certain pairs (r^2 below r_max^2 (1 - 1e-5))
    present exactly once with nothing outside them but pairs of the cutoff
    band, checked by per-block pair counts and pair-hash sums;
  * its k = 12 nearest rows (ppa_query_knn): every row without a near-tie at
    rank 12 holds exactly the oracle's 12 (block hash sums); rows with a
    near-tie are checked against the oracle's stored candidates;
  * the 2D PMFT of the 262,144-point fluid (ppa_pmft2d): all 40,000 bins
    inside the oracle's bounds;
  * the 256-frame trajectory through the autotuned batch plan replayed as a
    HIP graph: every frame's 128 bins inside the bounds and every frame's
    certain pairs present exactly (per-frame hash sums).
"""
import ctypes
import json
import os
import sys

import numpy as np
import pytest

from paper_1906_06317_amd import workloads
from tests.parity import REL, check_hist

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden")
sys.path.insert(0, GOLDEN)
import pairhash  # noqa: E402

pytestmark = pytest.mark.gpu


def _golden(name):
    path = os.path.join(GOLDEN, name + ".npz")
    if not os.path.exists(path):
        pytest.fail(f"missing expected values {path}: run tests/golden/make_golden.py {name}")
    return np.load(path, allow_pickle=False)


@pytest.fixture(scope="module")
def ppa():
    import torch
    assert torch.cuda.is_available(), "a GPU is required"
    import paper_1906_06317_amd as m
    m.lib()
    return m


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _row_pairs(offsets, point_idx):
    """(row of each pair, neighbour) on the host from a CSR list."""
    off = offsets.cpu().numpy()
    idx = point_idx.cpu().numpy()
    rows = np.repeat(np.arange(len(off) - 1, dtype=np.int64), np.diff(off))
    assert rows.shape[0] == idx.shape[0]
    return rows, idx.astype(np.int64)


def _check_rows_by_hash(rows, nbrs, n_rows, block, g_count, g_hash, band_rows, band_nbrs,
                        frame=None, label=""):
    """Per block of rows: the GPU's pairs minus those of the cutoff band must
    match the oracle's certain-pair count and hash sum; every GPU pair in the
    band is allowed, each at most once."""
    assert np.all((nbrs >= 0)), f"{label}: negative neighbour index"
    h = pairhash.mix(pairhash.keys(rows, nbrs, frame))
    band_keys = pairhash.keys(band_rows, band_nbrs, frame)
    in_band = np.isin(pairhash.keys(rows, nbrs, frame), band_keys)
    # each band pair at most once
    kb = pairhash.keys(rows[in_band], nbrs[in_band], frame)
    assert np.unique(kb).shape[0] == kb.shape[0], f"{label}: a band pair listed twice"
    keep = ~in_band
    c, s = pairhash.block_sums(rows[keep], h[keep], n_rows, block)
    bad = np.nonzero((c != g_count) | (s != g_hash))[0]
    assert bad.size == 0, (f"{label}: {bad.size} row blocks differ from the oracle, first {bad[:8]} "
                           f"(counts gpu {c[bad[:4]]} oracle {g_count[bad[:4]]})")
    return int(in_band.sum())


def test_fcc1M_ball_rdf_every_row_and_bin(ppa):
    import torch
    g = _golden("fcc1M_ball_rdf")
    meta = json.loads(str(g["meta"]))
    s = workloads.large_fcc()
    n = s.points.shape[0]
    r_max, bins = meta["r_max"], meta["bins"]
    box = ppa.Box(s.L, s.tilt, s.dim)
    pts = torch.as_tensor(s.points).cuda()
    cap = int(g["block_count"].sum()) + len(g["band_rows"]) + 1024
    ws = ppa.Workspace()
    wptr, wlen = ws.get(ppa.workspace_bytes(box, n, 0, r_max, ppa.PPA_WS_NLIST))
    off = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    cnt = torch.empty(n, dtype=torch.int32, device="cuda")
    pidx = torch.empty(cap, dtype=torch.int32, device="cuda")
    dist = torch.empty(cap, dtype=torch.float32, device="cuda")
    npairs = torch.zeros(1, dtype=torch.int64, device="cuda")
    hist = torch.zeros(bins, dtype=torch.int64, device="cuda")
    L = ppa.lib()
    # the bench's headline call: self-query, list + RDF in one pass, flags 0
    rc = L.ppa_rdf(ctypes.byref(box.c()), _p(pts), n, None, n, bins, 0.0, r_max, 1, 0, wptr, wlen,
                   _p(hist), _p(off), _p(cnt), _p(pidx), _p(dist), cap, _p(npairs), _stream())
    assert rc == 0, L.ppa_last_error()
    assert ws.status() == 0
    P = int(npairs.item())
    o = off.cpu().numpy()
    assert o[0] == 0 and o[-1] == P and np.all(np.diff(o) == cnt.cpu().numpy())
    check_hist(hist.cpu().numpy(), g["hist_lo"], g["hist_hi"])
    assert int(hist.sum().item()) <= P
    rows, nbrs = _row_pairs(off, pidx[:P])
    assert np.all(nbrs < n) and not np.any(nbrs == rows), "self pair or index out of range"
    n_band = _check_rows_by_hash(rows, nbrs, n, int(g["block"]), g["block_count"],
                                 g["block_hash"], g["band_rows"], g["band_nbrs"], label="FCC ball")
    assert P == int(g["block_count"].sum()) + n_band
    # every listed distance inside the cutoff and consistent with the histogram
    d = dist[:P]
    assert float(d.max().item()) <= r_max * (1 + REL)
    assert float(d.min().item()) > 0.0


def test_fcc1M_knn12_every_row(ppa):
    import torch
    g = _golden("fcc1M_knn12")
    s = workloads.large_fcc()
    n = s.points.shape[0]
    k = int(g["k"])
    box = ppa.Box(s.L, s.tilt, s.dim)
    pts = torch.as_tensor(s.points).cuda()
    ws = ppa.Workspace()
    wptr, wlen = ws.get(ppa.knn_workspace_bytes(box, n, 0, k))
    off = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    idx = torch.empty(n * k, dtype=torch.int32, device="cuda")
    dist = torch.empty(n * k, dtype=torch.float32, device="cuda")
    npairs = torch.zeros(1, dtype=torch.int64, device="cuda")
    L = ppa.lib()
    # the bench's k-nearest call
    rc = L.ppa_query_knn(ctypes.byref(box.c()), _p(pts), n, None, n, k, 0.0, 1, 0, wptr, wlen,
                         _p(off), None, _p(idx), _p(dist), _p(npairs), _stream())
    assert rc == 0, L.ppa_last_error()
    assert ws.status() == 0 and int(npairs.item()) == n * k
    o = off.cpu().numpy()
    assert np.array_equal(o, np.arange(n + 1, dtype=np.int64) * k)
    I = idx.cpu().numpy().reshape(n, k).astype(np.int64)
    D = dist.cpu().numpy().reshape(n, k)
    assert np.all(np.diff(D, axis=1) >= 0), "rows not sorted by distance"
    tie = np.zeros(n, bool)
    tie[g["tie_rows"]] = True
    rows = np.repeat(np.arange(n, dtype=np.int64)[~tie], k)
    nb = I[~tie].ravel()
    h = pairhash.mix(pairhash.keys(rows, nb))
    c, sm = pairhash.block_sums(rows, h, n, int(g["block"]))
    bad = np.nonzero((c != g["block_count"]) | (sm != g["block_hash"]))[0]
    assert bad.size == 0, f"{bad.size} row blocks differ from the oracle's 12 nearest: {bad[:8]}"
    for t, q in enumerate(g["tie_rows"]):
        cand, r2 = g["tie_idx"][t], g["tie_r2"][t]
        r2k = r2[k - 1]
        allowed = set(cand[r2 <= r2k * (1 + REL)].tolist())
        certain = set(cand[r2 < r2k * (1 - REL)].tolist())
        got = set(I[q].tolist())
        assert len(got) == k and certain <= got <= allowed, f"row {q}"


def test_fluid2d_pmft200_every_bin(ppa):
    import torch
    g = _golden("fluid2d_pmft200")
    s = workloads.fluid_2d()
    n = s.points.shape[0]
    box = ppa.Box(s.L, s.tilt, s.dim)
    pts = torch.as_tensor(s.points).cuda()
    th = torch.as_tensor(s.theta).cuda()
    ws = ppa.Workspace()
    wptr, wlen = ws.get(ppa.pmft2d_workspace_bytes(box, n, 0, 200, 200, 3.0, 3.0, 3.0))
    counts = torch.zeros(200 * 200, dtype=torch.int32, device="cuda")
    L = ppa.lib()
    # the bench's call
    rc = L.ppa_pmft2d(ctypes.byref(box.c()), _p(pts), n, None, _p(th), n, 200, 200, 3.0, 3.0, 3.0,
                      1, 0, wptr, wlen, _p(counts), _stream())
    assert rc == 0, L.ppa_last_error()
    assert ws.status() == 0
    lo = g["lo"].astype(np.int64).reshape(-1)
    hi = lo + g["hi_minus_lo"].astype(np.int64).reshape(-1)
    check_hist(counts.cpu().numpy().astype(np.int64), lo, hi)


def test_traj256_batched_graph_every_frame(ppa):
    import torch
    g = _golden("traj256_ball_rdf")
    frames = workloads.trajectory()
    F = len(frames)
    sizes = [f.points.shape[0] for f in frames]
    boxes = [ppa.Box(f.L, f.tilt, f.dim) for f in frames]
    pts = torch.as_tensor(np.concatenate([f.points for f in frames])).cuda()
    # the bench's path: plan, autotune, graph launch
    plan = ppa.BatchPlan(boxes, sizes, 128, 2.5)
    plan.run(pts)
    plan.autotune(pts, reps=1)
    hist = torch.zeros((F, 128), dtype=torch.int64, device="cuda")
    launch = plan.graph(pts, hist)
    launch()
    torch.cuda.synchronize()
    assert plan.ws.status() == 0
    nl = plan.neighbor_list()
    h = hist.cpu().numpy()
    lo = g["hist_lo"].astype(np.int64)
    hi = lo + g["hist_hi_minus_lo"].astype(np.int64)
    for f in range(F):
        check_hist(h[f], lo[f], hi[f])
    off = nl.offsets.cpu().numpy()
    idx = nl.point_idx.cpu().numpy().astype(np.int64)
    pb = plan.offsets_host
    for f in range(F):
        a, b = off[pb[f]], off[pb[f + 1]]
        rows = np.repeat(np.arange(sizes[f], dtype=np.int64), np.diff(off[pb[f]:pb[f + 1] + 1]))
        nbrs = idx[a:b]
        assert np.all((nbrs >= 0) & (nbrs < sizes[f])) and not np.any(nbrs == rows)
        sel = g["band_frame"] == f
        _check_rows_by_hash(rows, nbrs, sizes[f], 1 << 22, g["frame_count"][f:f + 1],
                            g["frame_hash"][f:f + 1], g["band_rows"][sel], g["band_nbrs"][sel],
                            frame=f, label=f"frame {f}")
