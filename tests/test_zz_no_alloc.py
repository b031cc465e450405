"""GPU: ppa_rdf_static (the ppa_rdf call without a workspace, for callers
that cannot allocate) against ppa_rdf on the same inputs, two calls in a
row, the second smaller; outputs must be identical (same kernels, and the
static scratch keeps nothing from the first call that changes the second)."""
import ctypes

import numpy as np
import pytest

from paper_1906_06317_amd import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ppa():
    import torch
    assert torch.cuda.is_available(), "a GPU is required"
    import paper_1906_06317_amd as m
    L = m.lib()
    i32, i64, f32, P = ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_void_p
    L.ppa_rdf_static.argtypes = [ctypes.POINTER(m.CBox), P, i64, P, i64, i32, f32, f32, i32, i32,
                                 P, P, P, P, P, i64, P, P]
    L.ppa_rdf_static.restype = ctypes.c_int
    return m


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _outputs(n, cap, bins):
    import torch
    return dict(hist=torch.zeros(bins, dtype=torch.int64, device="cuda"),
                off=torch.full((n + 1,), -7, dtype=torch.int64, device="cuda"),
                cnt=torch.full((n,), -7, dtype=torch.int32, device="cuda"),
                idx=torch.full((cap,), -7, dtype=torch.int32, device="cuda"),
                dist=torch.full((cap,), -7.0, dtype=torch.float32, device="cuda"),
                np=torch.zeros(1, dtype=torch.int64, device="cuda"))


def _run(ppa, static, s, bins, r_min, r_max, query=None, sort=False):
    import torch
    n = s.points.shape[0]
    box = ppa.Box(s.L, s.tilt, s.dim)
    pts = torch.as_tensor(s.points).cuda()
    q = None if query is None else torch.as_tensor(query).cuda()
    nq = n if q is None else q.shape[0]
    excl = 1 if q is None else 0
    flags = ppa.PPA_SORT_ROWS if sort else 0
    cap = 200 * nq
    o = _outputs(nq, cap, bins)
    L = ppa.lib()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if static:
        rc = L.ppa_rdf_static(ctypes.byref(box.c()), _p(pts), n, _p(q), nq, bins, r_min, r_max,
                              excl, flags, _p(o["hist"]), _p(o["off"]), _p(o["cnt"]),
                              _p(o["idx"]), _p(o["dist"]), cap, _p(o["np"]), stream)
        assert rc == 0, L.ppa_last_error()
        assert L.ppa_sync_status(None, stream) == 0, L.ppa_last_error()
    else:
        ws = ppa.Workspace()
        wptr, wlen = ws.get(ppa.workspace_bytes(box, n, 0 if q is None else nq, r_max,
                                                ppa.PPA_WS_NLIST))
        rc = L.ppa_rdf(ctypes.byref(box.c()), _p(pts), n, _p(q), nq, bins, r_min, r_max, excl,
                       flags, wptr, wlen, _p(o["hist"]), _p(o["off"]), _p(o["cnt"]), _p(o["idx"]),
                       _p(o["dist"]), cap, _p(o["np"]), stream)
        assert rc == 0, L.ppa_last_error()
        assert ws.status() == 0
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in o.items()}


def _same(a, b):
    P = int(a["np"][0])
    assert P == int(b["np"][0]) and P > 0
    for k in ("hist", "off", "cnt"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)
    np.testing.assert_array_equal(a["idx"][:P], b["idx"][:P])
    np.testing.assert_array_equal(a["dist"][:P], b["dist"][:P])


def test_static_scratch_matches_workspace_call_twice_second_smaller(ppa):
    big = workloads.uniform(60000, 0.85, seed=91, tilt=(0.3, -0.2, 0.1))
    small = workloads.uniform(7000, 0.7, seed=92)
    r1 = _run(ppa, False, big, 64, 0.0, 2.5)
    s1 = _run(ppa, True, big, 64, 0.0, 2.5)
    _same(r1, s1)
    r2 = _run(ppa, False, small, 40, 0.5, 2.0)
    s2 = _run(ppa, True, small, 40, 0.5, 2.0)
    _same(r2, s2)
    # separate query points and sorted rows through the same scratch
    rng = np.random.default_rng(93)
    q = small.points[rng.choice(7000, 900, replace=False)] + np.float32(0.01)
    _same(_run(ppa, False, small, 16, 0.0, 1.5, query=q, sort=True),
          _run(ppa, True, small, 16, 0.0, 1.5, query=q, sort=True))


def test_static_scratch_rejects_oversized_calls(ppa):
    import torch
    L = ppa.lib()
    box = ppa.Box.cube(400.0)
    # host-side sizing refuses before any device work: the pointers are not read
    dev = ctypes.c_void_p(4096)
    rc = L.ppa_rdf_static(ctypes.byref(box.c()), dev, 4 << 20, None, 4 << 20, 10, 0.0, 2.0, 1, 0,
                          dev, dev, None, dev, None, 1, dev,
                          ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == ppa.PPA_EWORKSPACE
    assert b"static" in L.ppa_last_error()
