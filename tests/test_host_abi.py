"""C ABI checks that need no GPU: the library loads, exports every function
the header declares, and its host-side validation returns the documented
codes before touching the device."""
import ctypes
import math
import os
import re
import subprocess

import numpy as np
import pytest

import paper_1906_06317_amd as ppa
from tests import brute

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(ppa_[a-z0-9_]+)\s*\(", src))
    return names


def test_library_exports_every_declared_symbol():
    L = ppa.lib()
    names = _declared()
    assert {"ppa_query_ball", "ppa_rdf", "ppa_sync_status"} <= names
    out = subprocess.run(["nm", "-D", "--defined-only", ppa._LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (ppa_[a-z0-9_]+)$", out, flags=re.M))
    assert names <= exported, names - exported
    for n in names:
        assert hasattr(L, n)


def test_version():
    assert "gfx950" in ppa.version()


@pytest.mark.parametrize("dim", [2, 3])
def test_box_widths_match_geometry(dim):
    rng = np.random.default_rng(4)
    for _ in range(10):
        L = tuple(rng.uniform(1, 10, 3))
        tilt = tuple(rng.uniform(-0.8, 0.8, 3))
        if dim == 2:
            L = (L[0], L[1], 1.0)
            tilt = (tilt[0], 0.0, 0.0)
        w = ppa.Box(L, tilt, dim).widths()
        ref = brute.perpendicular_widths(L, tilt, dim)
        np.testing.assert_allclose(w[:dim], ref[:dim], rtol=1e-12)


def test_box_from_matrix():
    m = np.array([[4.0, 1.0, 0.5], [0.0, 5.0, -1.0], [0.0, 0.0, 2.0]])
    b = ppa.Box.from_matrix(m)
    np.testing.assert_allclose(b.L, (4, 5, 2))
    np.testing.assert_allclose(b.tilt, (0.2, 0.25, -0.5))
    with pytest.raises(ppa.PPAError) as e:
        ppa.Box.from_matrix(np.array([[1.0, 0, 0], [0.3, 1, 0], [0, 0, 1]]))
    assert e.value.code == ppa.PPA_EBOX


def test_workspace_bytes_and_range_check():
    box = ppa.Box.cube(10.0)
    small = ppa.workspace_bytes(box, 1000, 0, 2.0)
    big = ppa.workspace_bytes(box, 100000, 0, 2.0)
    assert 0 < small < big
    assert ppa.workspace_bytes(box, 1000, 500, 2.0) > small
    assert ppa.workspace_bytes(box, 1000, 0, 2.0, ppa.PPA_WS_NLIST) > small
    with pytest.raises(ppa.PPAError) as e:
        ppa.workspace_bytes(box, 1000, 0, 5.0)  # = half the box width
    assert e.value.code == ppa.PPA_ERANGE
    tilted = ppa.Box((10.0, 10.0, 10.0), (0.9, 0.0, 0.0))
    w = tilted.widths()
    with pytest.raises(ppa.PPAError):
        ppa.workspace_bytes(tilted, 10, 0, 0.5 * min(w) * 1.0001)
    ppa.workspace_bytes(tilted, 10, 0, 0.5 * min(w) * 0.999)


def _call_ball(box, n=10, nq=10, qpts=None, r=1.0, flags=0, ws=1 << 8, ws_bytes=1 << 40,
               offsets=8, counts=8, pidx=8, cap=10, npairs=8):
    L = ppa.lib()
    cb = box.c() if box is not None else None
    return L.ppa_query_ball(ctypes.byref(cb) if cb is not None else None, ctypes.c_void_p(64), n,
                            qpts, nq, r, 1, flags, ctypes.c_void_p(ws), ws_bytes,
                            ctypes.c_void_p(offsets) if offsets else None,
                            ctypes.c_void_p(counts) if counts else None,
                            ctypes.c_void_p(pidx) if pidx else None, None, cap,
                            ctypes.c_void_p(npairs) if npairs else None, None)


def test_query_argument_errors_before_any_device_work():
    box = ppa.Box.cube(10.0)
    assert _call_ball(None) == ppa.PPA_EINVAL
    assert _call_ball(box, n=-1) == ppa.PPA_EINVAL
    assert _call_ball(box, nq=5) == ppa.PPA_EINVAL                 # nq != n without query points
    assert _call_ball(box, r=-1.0) == ppa.PPA_EINVAL
    assert _call_ball(box, r=float("nan")) == ppa.PPA_EINVAL
    assert _call_ball(box, flags=8) == ppa.PPA_EINVAL
    assert _call_ball(box, flags=1) == ppa.PPA_EINVAL             # a workspace flag, not a query flag
    assert _call_ball(box, flags=ppa.PPA_SORT_ROWS, r=6.0) == ppa.PPA_ERANGE  # flag accepted
    assert _call_ball(box, offsets=0) == ppa.PPA_EINVAL
    assert _call_ball(box, cap=-1) == ppa.PPA_EINVAL
    assert _call_ball(box, r=6.0) == ppa.PPA_ERANGE
    assert _call_ball(box, ws=0) == ppa.PPA_EWORKSPACE
    assert _call_ball(box, ws=(1 << 8) + 4) == ppa.PPA_EWORKSPACE   # misaligned
    assert _call_ball(box, ws_bytes=16) == ppa.PPA_EWORKSPACE
    assert b"workspace" in ppa.lib().ppa_last_error()
    bad = ppa.Box((10.0, -1.0, 10.0))
    assert _call_ball(bad) == ppa.PPA_EBOX
    bad = ppa.Box((10.0, 10.0, 10.0), (math.inf, 0, 0))
    assert _call_ball(bad) == ppa.PPA_EBOX
    bad = ppa.Box((10.0, 10.0, 10.0), (0, 0, 0), 4)
    assert _call_ball(bad) == ppa.PPA_EINVAL


def test_rdf_argument_errors():
    L = ppa.lib()
    box = ppa.Box.cube(10.0).c()
    args = lambda bins, rmin, rmax, hist: L.ppa_rdf(
        ctypes.byref(box), ctypes.c_void_p(64), 10, None, 10, bins, rmin, rmax, 1, 0,
        ctypes.c_void_p(256), 1 << 40, ctypes.c_void_p(hist) if hist else None, None, None, None,
        None, 0, None, None)
    assert args(0, 0.0, 2.0, 8) == ppa.PPA_EINVAL
    assert args(10, 2.0, 2.0, 8) == ppa.PPA_EINVAL
    assert args(10, -1.0, 2.0, 8) == ppa.PPA_EINVAL
    assert args(10, 0.0, 2.0, 0) == ppa.PPA_EINVAL
    assert L.ppa_rdf_from_nlist(None, None, 0, 10, 0.0, 1.0, None, None) == ppa.PPA_EINVAL


def test_binding_has_no_cpu_fallback():
    """The product path imports nothing from the oracle."""
    pkg = os.path.join(ROOT, "paper_1906_06317_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "from oracle" not in src, f
                assert "liboracle" not in src, f


def test_knn_workspace_and_argument_errors():
    L = ppa.lib()
    box = ppa.Box.cube(10.0)
    full = ppa.knn_workspace_bytes(box, 1000, 0, 12)
    assert full > 0
    # rows that may be short (a guard, or fewer points than k) are staged
    assert ppa.knn_workspace_bytes(box, 1000, 0, 12, r_guard=2.0) > full
    assert ppa.knn_workspace_bytes(box, 5, 0, 12) > ppa.knn_workspace_bytes(box, 5, 0, 4)
    for k in (0, 65, -3):
        with pytest.raises(ppa.PPAError) as e:
            ppa.knn_workspace_bytes(box, 1000, 0, k)
        assert e.value.code == ppa.PPA_EINVAL
    with pytest.raises(ppa.PPAError) as e:
        ppa.knn_workspace_bytes(box, 1000, 0, 12, r_guard=5.0)
    assert e.value.code == ppa.PPA_ERANGE
    with pytest.raises(ppa.PPAError) as e:
        ppa.knn_workspace_bytes(box, 1000, 0, 12, r_guard=-1.0)
    assert e.value.code == ppa.PPA_EINVAL
    cb = box.c()

    def call(k=12, n=10, nq=10, guard=0.0, flags=0, ws=256, ws_bytes=1 << 40, offsets=8, pidx=8,
             npairs=8):
        return L.ppa_query_knn(ctypes.byref(cb), ctypes.c_void_p(64), n, None, nq, k, guard, 1,
                               flags, ctypes.c_void_p(ws) if ws else None, ws_bytes,
                               ctypes.c_void_p(offsets) if offsets else None, None,
                               ctypes.c_void_p(pidx) if pidx else None, None,
                               ctypes.c_void_p(npairs) if npairs else None, None)
    assert call(k=0) == ppa.PPA_EINVAL
    assert call(k=100) == ppa.PPA_EINVAL
    assert call(nq=5) == ppa.PPA_EINVAL
    assert call(flags=2) == ppa.PPA_EINVAL
    assert call(offsets=0) == ppa.PPA_EINVAL
    assert call(pidx=0) == ppa.PPA_EINVAL
    assert call(npairs=0) == ppa.PPA_EINVAL
    assert call(guard=float("nan")) == ppa.PPA_EINVAL
    assert call(guard=7.0) == ppa.PPA_ERANGE
    assert call(ws=0) == ppa.PPA_EWORKSPACE
    assert call(ws_bytes=64) == ppa.PPA_EWORKSPACE


def test_normalisation_host_checks():
    """The normalisation calls validate their host arguments before any
    device work (the device pointers here are never dereferenced)."""
    L = ppa.lib()
    dev = ctypes.c_void_p(4096)
    b3 = ppa.Box.cube(10.0)
    b2 = ppa.Box((10.0, 10.0, 1.0), (0.0, 0.0, 0.0), 2)

    def frames(boxes, npt, nq):
        F = len(boxes)
        cb = (ppa.CBox * F)(*[b.c() for b in boxes])
        a = np.asarray(npt, np.int64)
        q = np.asarray(nq, np.int64)
        return F, cb, a, q

    def rdf(bins=10, r_min=0.0, r_max=2.0, boxes=(b3,), npt=(100,), nq=(100,), counts=dev, g=dev,
            n_frames=None):
        F, cb, a, q = frames(boxes, npt, nq)
        return L.ppa_rdf_normalize(counts, bins, r_min, r_max, F if n_frames is None else n_frames,
                                   cb, a.ctypes.data_as(ctypes.c_void_p),
                                   q.ctypes.data_as(ctypes.c_void_p), g, None, None)
    assert rdf(bins=0) == ppa.PPA_EINVAL
    assert rdf(r_min=2.0) == ppa.PPA_EINVAL
    assert rdf(r_max=float("nan")) == ppa.PPA_EINVAL
    assert rdf(counts=None) == ppa.PPA_EINVAL
    assert rdf(g=None) == ppa.PPA_EINVAL
    assert rdf(n_frames=0) == ppa.PPA_EINVAL
    assert rdf(npt=(0,)) == ppa.PPA_EINVAL          # no ideal-gas pairs to divide by
    assert rdf(nq=(-1,)) == ppa.PPA_EINVAL
    assert rdf(boxes=(b3, b2), npt=(5, 5), nq=(5, 5)) == ppa.PPA_EINVAL  # mixed dimensions
    assert rdf(boxes=(ppa.Box((10.0, -1.0, 10.0)),)) == ppa.PPA_EBOX

    def pmft2(nbx=10, nby=10, x=2.0, y=2.0, boxes=(b2,)):
        F, cb, a, q = frames(boxes, (100,), (100,))
        return L.ppa_pmft2d_normalize(dev, nbx, nby, x, y, F, cb, a.ctypes.data_as(ctypes.c_void_p),
                                      q.ctypes.data_as(ctypes.c_void_p), dev, None, None)
    assert pmft2(nbx=0) == ppa.PPA_EINVAL
    assert pmft2(y=0.0) == ppa.PPA_EINVAL
    assert pmft2(boxes=(b3,)) == ppa.PPA_EINVAL       # 2D only
    F, cb, a, q = frames((b2,), (100,), (100,))
    assert L.ppa_pmft_xyz_normalize(dev, 5, 5, 5, 1.0, 1.0, 1.0, F, cb,
                                    a.ctypes.data_as(ctypes.c_void_p),
                                    q.ctypes.data_as(ctypes.c_void_p), dev, None,
                                    None) == ppa.PPA_EINVAL  # 3D only
    assert L.ppa_pmft_xyt_normalize(dev, 5, 5, 0, 1.0, 1.0, F, cb,
                                    a.ctypes.data_as(ctypes.c_void_p),
                                    q.ctypes.data_as(ctypes.c_void_p), dev, None,
                                    None) == ppa.PPA_EINVAL
    assert L.ppa_correlation_finalize(dev, None, 10, dev, None) == ppa.PPA_EINVAL
    assert L.ppa_correlation_finalize(dev, dev, 0, dev, None) == ppa.PPA_EINVAL


def test_pmft_workspace_and_errors():
    b2 = ppa.Box((20.0, 20.0, 1.0), (0.1, 0.0, 0.0), 2)
    small = ppa.pmft2d_workspace_bytes(b2, 1000, 0, 50, 50, 3.0, 3.0, 3.0)
    assert small > 0
    assert ppa.pmft2d_workspace_bytes(b2, 1000, 500, 50, 50, 3.0, 3.0, 3.0) > small
    with pytest.raises(ppa.PPAError) as e:
        ppa.pmft2d_workspace_bytes(ppa.Box.cube(20.0), 1000, 0, 50, 50, 3.0, 3.0, 3.0)
    assert e.value.code == ppa.PPA_EINVAL
    for args in [(0, 50, 3.0, 3.0, 3.0), (50, 50, 0.0, 3.0, 3.0), (50, 50, 3.0, -1.0, 3.0),
                 (50, 50, 3.0, 3.0, float("inf"))]:
        with pytest.raises(ppa.PPAError) as e:
            ppa.pmft2d_workspace_bytes(b2, 1000, 0, *args)
        assert e.value.code == ppa.PPA_EINVAL
    with pytest.raises(ppa.PPAError) as e:
        ppa.pmft2d_workspace_bytes(b2, 1000, 0, 50, 50, 3.0, 3.0, 10.0)
    assert e.value.code == ppa.PPA_ERANGE


def test_cluster_flags_and_workspace_errors():
    L = ppa.lib()
    off = ctypes.c_void_p(256)  # never read: the host checks come first
    args = lambda flags, ws: L.ppa_cluster(off, ctypes.c_void_p(512), 10, 20, flags, ws,
                                           1 << 20, ctypes.c_void_p(1024), None, None, None,
                                           None)
    assert args(2, ctypes.c_void_p(4096)) == ppa.PPA_EINVAL          # unknown flag
    assert args(ppa.PPA_CLUSTER_SYMMETRIC, None) == ppa.PPA_EWORKSPACE  # flag accepted
    assert args(0, ctypes.c_void_p(4096 + 8)) == ppa.PPA_EWORKSPACE  # misaligned


def test_batch_cell_build_chunking():
    """The batch plan splits frames of at most 32768 cells into chunks of
    16384 points counted in LDS and leaves larger frames to global counters
    (host logic of plan creation; no device work)."""
    from paper_1906_06317_amd import workloads
    L = ppa.lib()
    specs = [(40000, 0.05), (40000, 8.0), (3000, 1.0), (0, 1.0), (500, 1.0), (17000, 0.5)]
    # (the empty frame takes the box of 1000 points)
    frames = [workloads.uniform(n or 1000, rho, seed=300 + k) for k, (n, rho) in enumerate(specs)]
    boxes = (ppa.CBox * len(frames))(*[ppa.Box(f.L, f.tilt, 3).c() for f in frames])
    off = np.concatenate([[0], np.cumsum([n for n, _ in specs])]).astype(np.int64)
    h = ctypes.c_void_p()
    assert L.ppa_batch_plan_create(len(frames), boxes, off.ctypes.data_as(ctypes.c_void_p), 32,
                                   0.0, 0.6, 1, 0, ctypes.byref(h)) == 0
    try:
        c, k, g = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        for index in (-1, 0):
            assert L.ppa_batch_config_cells(h, index, ctypes.byref(c), ctypes.byref(k),
                                            ctypes.byref(g)) == 0
            # 40000 points in 3 chunks, 3000 and 500 in one each, 17000 in 2; the
            # empty frame has none; the sparse frame has more than 32768 cells
            assert (k.value, g.value) == (7, 1)
            assert c.value > 32768
        assert L.ppa_batch_config_cells(h, 99, None, None, None) == ppa.PPA_EINVAL
    finally:
        L.ppa_batch_plan_destroy(h)


def test_batch_chunk_table_budget():
    """Chunked frames stop at a bounded partial-count array (2^27 entries):
    the frames past it count with global atomics and the plan is still made
    (host logic; no device work)."""
    L = ppa.lib()
    nf, npf = 72, 1 << 20
    # a 19^3 box at r_max 0.6: 31^3 = 29791 cells for the first configuration,
    # 64 chunks of 16384 points per frame
    boxes = (ppa.CBox * nf)(*[ppa.Box((19.0, 19.0, 19.0), (0, 0, 0), 3).c() for _ in range(nf)])
    off = (np.arange(nf + 1, dtype=np.int64) * npf)
    h = ctypes.c_void_p()
    assert L.ppa_batch_plan_create(nf, boxes, off.ctypes.data_as(ctypes.c_void_p), 32, 0.0, 0.6,
                                   1, 0, ctypes.byref(h)) == 0
    try:
        c, k, g = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        assert L.ppa_batch_config_cells(h, 0, ctypes.byref(c), ctypes.byref(k),
                                        ctypes.byref(g)) == 0
        nc = c.value // nf
        assert nc * nf == c.value and nc == 31 ** 3
        chunked = (1 << 27) // (64 * nc)
        assert (k.value, g.value) == (64 * chunked, nf - chunked)
        assert 0 < chunked < nf
    finally:
        L.ppa_batch_plan_destroy(h)
