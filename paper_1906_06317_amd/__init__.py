"""ppa: periodic pair analysis on AMD Instinct MI355X (gfx950).

Thin Python binding of libppa.so (C ABI in include/ppa.h).  Every step of
the computation runs in the library's HIP kernels; this module only
marshals arguments.  PyTorch provides device memory and the current
stream.  There is no CPU fallback: if the library cannot be loaded, every
call raises.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libppa.so")

PPA_OK = 0
PPA_EINVAL = -1
PPA_EBOX = -2
PPA_ERANGE = -3
PPA_EWORKSPACE = -4
PPA_EDEVICE = -5
PPA_ECAPACITY = -6
PPA_ENONFINITE = -7
PPA_WS_NLIST = 1
PPA_SORT_ROWS = 2
PPA_CLUSTER_SYMMETRIC = 1

_ERRNAMES = {
    PPA_EINVAL: "PPA_EINVAL", PPA_EBOX: "PPA_EBOX", PPA_ERANGE: "PPA_ERANGE",
    PPA_EWORKSPACE: "PPA_EWORKSPACE", PPA_EDEVICE: "PPA_EDEVICE",
    PPA_ECAPACITY: "PPA_ECAPACITY", PPA_ENONFINITE: "PPA_ENONFINITE",
}


class PPAError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class CBox(ctypes.Structure):
    _fields_ = [("L", ctypes.c_double * 3), ("tilt", ctypes.c_double * 3), ("dim", ctypes.c_int32)]


@dataclass(frozen=True)
class Box:
    """Periodic box: edge lengths L, tilts (xy, xz, yz), dimension 2 or 3."""
    L: tuple
    tilt: tuple = (0.0, 0.0, 0.0)
    dim: int = 3

    @staticmethod
    def cube(L, dim=3):
        return Box((float(L),) * 3 if dim == 3 else (float(L), float(L), 1.0), (0.0, 0.0, 0.0), dim)

    @staticmethod
    def from_matrix(m, dim=3):
        """Box from a 3x3 upper-triangular matrix whose columns are the lattice vectors."""
        m = np.ascontiguousarray(m, dtype=np.float64).reshape(9)
        out = CBox()
        _check(lib().ppa_box_from_matrix(m.ctypes.data_as(ctypes.c_void_p), dim, ctypes.byref(out)))
        return Box(tuple(out.L), tuple(out.tilt), int(out.dim))

    def c(self) -> CBox:
        b = CBox()
        for k in range(3):
            b.L[k] = float(self.L[k])
            b.tilt[k] = float(self.tilt[k])
        b.dim = int(self.dim)
        return b

    @property
    def volume(self) -> float:
        return float(self.L[0] * self.L[1] * (self.L[2] if self.dim == 3 else 1.0))

    def widths(self):
        w = (ctypes.c_double * 3)()
        _check(lib().ppa_box_widths(ctypes.byref(self.c()), w))
        return tuple(w)


_lib = None


def lib():
    """Loads libppa.so (building it first if it is missing)."""
    global _lib
    if _lib is None:
        # torch first: its bundled HIP runtime then also serves libppa (same
        # soname), so torch's streams and memory are valid in the library
        import torch  # noqa: F401
        if not os.path.exists(_LIB_PATH):
            from . import build as _build
            _build.build()
        L = ctypes.CDLL(_LIB_PATH)
        P, i32, i64, f32, sz = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float,
                                ctypes.c_size_t)
        BP = ctypes.POINTER(CBox)
        sig = {
            "ppa_box_from_matrix": [P, i32, BP],
            "ppa_box_widths": [BP, P],
            "ppa_workspace_bytes": [BP, i64, i64, f32, i32, ctypes.POINTER(sz)],
            "ppa_query_ball": [BP, P, i64, P, i64, f32, i32, i32, P, sz, P, P, P, P, i64, P, P],
            "ppa_rdf": [BP, P, i64, P, i64, i32, f32, f32, i32, i32, P, sz, P, P, P, P, P, i64, P, P],
            "ppa_rdf_from_nlist": [P, P, i64, i32, f32, f32, P, P],
            "ppa_knn_workspace_bytes": [BP, i64, i64, i32, f32, ctypes.POINTER(sz)],
            "ppa_query_knn": [BP, P, i64, P, i64, i32, f32, i32, i32, P, sz, P, P, P, P, P, P],
            "ppa_pmft2d_workspace_bytes": [BP, i64, i64, i32, i32, f32, f32, f32,
                                           ctypes.POINTER(sz)],
            "ppa_pmft2d": [BP, P, i64, P, P, i64, i32, i32, f32, f32, f32, i32, i32, P, sz, P, P],
            "ppa_correlation_workspace_bytes": [BP, i64, i64, i32, f32, f32, ctypes.POINTER(sz)],
            "ppa_correlation": [BP, P, P, i64, P, P, i64, i32, f32, f32, i32, i32, P, sz, P, P, P],
            "ppa_steinhardt_workspace_bytes": [i32, i32, ctypes.POINTER(sz)],
            "ppa_steinhardt": [BP, P, i64, P, i64, P, P, i64, i32, i32, P, sz, P, P, P],
            "ppa_cluster_workspace_bytes": [i64, ctypes.POINTER(sz)],
            "ppa_knn_from_nlist_workspace_bytes": [i64, i32, ctypes.POINTER(sz)],
            "ppa_knn_from_nlist": [P, P, P, i64, i64, i32, i32, P, sz, P, P, P, P, P, P],
            "ppa_cluster": [P, P, i64, i64, i32, P, sz, P, P, P, P, P],
            "ppa_pmft_xyt_workspace_bytes": [BP, i64, i64, i32, i32, i32, f32, f32, f32,
                                             ctypes.POINTER(sz)],
            "ppa_pmft_xyt": [BP, P, P, i64, P, P, i64, i32, i32, i32, f32, f32, f32, i32, i32, P,
                             sz, P, P],
            "ppa_pmft_xyz_workspace_bytes": [BP, i64, i64, i32, i32, i32, f32, f32, f32, f32,
                                             ctypes.POINTER(sz)],
            "ppa_pmft_xyz": [BP, P, i64, P, P, i64, i32, i32, i32, f32, f32, f32, f32, i32, i32,
                             P, sz, P, P],
            "ppa_smooth_rdf_workspace_bytes": [BP, i64, i32, f32, f32, ctypes.POINTER(sz)],
            "ppa_batch_plan_create": [i32, BP, P, i32, f32, f32, i32, i32,
                                      ctypes.POINTER(ctypes.c_void_p)],
            "ppa_batch_plan_destroy": [P],
            "ppa_batch_workspace_bytes": [P, ctypes.POINTER(sz)],
            "ppa_batch_upload": [P, P, sz, P],
            "ppa_batch_run": [P, P, P, sz, P, P, P, P, P, i64, P, P],
            "ppa_batch_config": [P, i32, P, P, P, P],
            "ppa_batch_config_shape": [P, i32, P, P],
            "ppa_batch_config_cells": [P, i32, P, P, P],
            "ppa_batch_autotune": [P, P, P, sz, P, P, P, P, i64, P, i32, P, P],
            "ppa_batch_graph_create": [P, P, P, sz, P, P, P, P, P, i64, P,
                                       ctypes.POINTER(ctypes.c_void_p)],
            "ppa_batch_graph_launch": [P, P],
            "ppa_batch_graph_destroy": [P],
            "ppa_smooth_rdf_fwd": [BP, P, i64, i32, f32, f32, i32, P, sz, P, P],
            "ppa_smooth_rdf_bwd": [BP, P, i64, i32, f32, f32, P, i32, P, sz, P, P],
            "ppa_rdf_normalize": [P, i32, ctypes.c_double, ctypes.c_double, i32, BP, P, P, P, P,
                                  P],
            "ppa_rdf_bin_scale": [i32, ctypes.c_double, ctypes.c_double, i32, BP, P, P, P, P],
            "ppa_pmft2d_normalize": [P, i32, i32, ctypes.c_double, ctypes.c_double, i32, BP, P, P,
                                     P, P, P],
            "ppa_pmft_xyt_normalize": [P, i32, i32, i32, ctypes.c_double, ctypes.c_double, i32, BP,
                                       P, P, P, P, P],
            "ppa_pmft_xyz_normalize": [P, i32, i32, i32, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, i32, BP, P, P, P, P, P],
            "ppa_correlation_finalize": [P, P, i32, P, P],
            "ppa_sync_status": [P, P],
            "ppa_profile_next": [P, P, P, P],
            "ppa_probe_lds_atomics": [i32, i32, i32, P, P],
            "ppa_probe_global_atomics": [i32, i32, i32, P, P],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        L.ppa_last_error.restype = ctypes.c_char_p
        L.ppa_last_error.argtypes = []
        L.ppa_version.restype = ctypes.c_char_p
        L.ppa_version.argtypes = []
        _lib = L
    return _lib


def _check(rc):
    if rc != PPA_OK:
        raise PPAError(rc, lib().ppa_last_error().decode())
    return rc


def _torch():
    import torch
    return torch


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _points(points):
    torch = _torch()
    if not isinstance(points, torch.Tensor):
        points = torch.as_tensor(np.ascontiguousarray(points, dtype=np.float32))
    if points.device.type != "cuda":
        points = points.to("cuda")
    points = points.to(torch.float32).contiguous()
    if points.ndim != 2 or points.shape[1] != 3:
        raise ValueError("points must be an N x 3 array")
    return points


class Workspace:
    """Caller-owned device scratch memory, grown on demand (256-byte aligned)."""

    def __init__(self):
        self.buf = None
        self.ptr = 0
        self.nbytes = 0

    def get(self, nbytes):
        torch = _torch()
        if self.buf is None or self.nbytes < nbytes:
            self.buf = torch.zeros(int(nbytes) + 256, dtype=torch.uint8, device="cuda")
            base = self.buf.data_ptr()
            self.ptr = (base + 255) // 256 * 256
            self.nbytes = int(nbytes)
        return ctypes.c_void_p(self.ptr), ctypes.c_size_t(self.nbytes)

    def status(self, stream=None):
        return lib().ppa_sync_status(ctypes.c_void_p(self.ptr), _stream(stream))


_default_ws = None


def default_workspace():
    global _default_ws
    if _default_ws is None:
        _default_ws = Workspace()
    return _default_ws


def workspace_bytes(box: Box, n, nq, r_cut, flags=0):
    out = ctypes.c_size_t(0)
    _check(lib().ppa_workspace_bytes(ctypes.byref(box.c()), int(n), int(nq), float(r_cut),
                                     int(flags), ctypes.byref(out)))
    return out.value


@dataclass
class NeighborList:
    """Pairs found by a query, as CSR in query order: row q is
    point_idx[offsets[q]:offsets[q + 1]] (and dist likewise)."""
    offsets: "object"     # int64 [nq + 1]; offsets[nq] = n_pairs
    counts: "object"      # int32 [nq]
    point_idx: "object"   # int32 [n_pairs]
    dist: "object"        # float32 [n_pairs] or None
    n_pairs: int

    def query_point_indices(self):
        """Query index of every pair (length n_pairs), as in the paper's NeighborList."""
        torch = _torch()
        return torch.repeat_interleave(
            torch.arange(self.counts.shape[0], device=self.counts.device, dtype=torch.int32),
            self.counts.to(torch.int64))


def _estimate_pairs(box: Box, n, nq, r):
    rho = n / box.volume
    vball = (4.0 / 3.0) * math.pi * r ** 3 if box.dim == 3 else math.pi * r * r
    return int(nq * rho * vball * 1.25) + 4096


def _run_pairs(box, points, r_max, query_points, exclude_ii, capacity, with_dist, hist, bins,
               r_min, want_nl, ws, stream, check, sort_rows=False):
    torch = _torch()
    pts = _points(points)
    n = pts.shape[0]
    q = None if query_points is None else _points(query_points)
    nq = n if q is None else q.shape[0]
    if exclude_ii is None:
        exclude_ii = q is None
    ws = ws or default_workspace()
    need = workspace_bytes(box, n, 0 if q is None else nq, r_max, PPA_WS_NLIST if want_nl else 0)
    dev = pts.device
    if nq == 0:
        # nothing to query: an empty list and an unchanged histogram
        if not want_nl:
            return None
        return NeighborList(torch.zeros(1, dtype=torch.int64, device=dev),
                            torch.zeros(0, dtype=torch.int32, device=dev),
                            torch.zeros(0, dtype=torch.int32, device=dev),
                            torch.zeros(0, dtype=torch.float32, device=dev) if with_dist else None,
                            0)
    wptr, wlen = ws.get(need)
    cb = box.c()
    if not want_nl:
        _check(lib().ppa_rdf(ctypes.byref(cb), _ptr(pts), n, _ptr(q), nq, int(bins), float(r_min),
                             float(r_max), int(bool(exclude_ii)), 0, wptr, wlen, _ptr(hist),
                             None, None, None, None, 0, None, _stream(stream)))
        if check:
            _check(ws.status(stream))
        return None
    if capacity is None:
        capacity = _estimate_pairs(box, n, nq, r_max)
    qflags = PPA_SORT_ROWS if sort_rows else 0
    for attempt in range(2):
        offsets = torch.empty(nq + 1, dtype=torch.int64, device=dev)
        counts = torch.empty(nq, dtype=torch.int32, device=dev)
        pidx = torch.empty(max(capacity, 1), dtype=torch.int32, device=dev)
        dist = torch.empty(max(capacity, 1), dtype=torch.float32, device=dev) if with_dist else None
        npairs = torch.zeros(1, dtype=torch.int64, device=dev)
        h0 = hist.clone() if (hist is not None and attempt == 0) else None
        if hist is None:
            rc = lib().ppa_query_ball(ctypes.byref(cb), _ptr(pts), n, _ptr(q), nq, float(r_max),
                                      int(bool(exclude_ii)), qflags, wptr, wlen, _ptr(offsets),
                                      _ptr(counts), _ptr(pidx), _ptr(dist), int(capacity),
                                      _ptr(npairs), _stream(stream))
        else:
            rc = lib().ppa_rdf(ctypes.byref(cb), _ptr(pts), n, _ptr(q), nq, int(bins),
                               float(r_min), float(r_max), int(bool(exclude_ii)), qflags, wptr, wlen,
                               _ptr(hist), _ptr(offsets), _ptr(counts), _ptr(pidx), _ptr(dist),
                               int(capacity), _ptr(npairs), _stream(stream))
        _check(rc)
        st = ws.status(stream)
        if st == PPA_ECAPACITY and attempt == 0:
            capacity = int(npairs.item())
            if h0 is not None:
                hist.copy_(h0)  # the histogram was complete; it is recomputed with the list
            continue
        if check or st == PPA_ENONFINITE:
            _check(st)
        break
    np_ = int(npairs.item())
    return NeighborList(offsets, counts, pidx[:np_], None if dist is None else dist[:np_], np_)


def query_ball(box: Box, points, r_max, query_points=None, exclude_ii=None, capacity=None,
               with_dist=True, ws=None, stream=None, check=True,
               sort_rows=False) -> NeighborList:
    """All pairs (i, j) with |p_j - q_i| < r_max under periodic boundaries.

    sort_rows=True orders each row by neighbour index j."""
    return _run_pairs(box, points, r_max, query_points, exclude_ii, capacity, with_dist, None, 0,
                      0.0, True, ws, stream, check, sort_rows)


def rdf_counts(box: Box, points, bins, r_max, r_min=0.0, query_points=None, exclude_ii=None,
               counts=None, neighbor_list=False, capacity=None, ws=None, stream=None, check=True,
               sort_rows=False):
    """RDF pair histogram (int64 [bins], accumulated into `counts` when given).

    With neighbor_list=True the same pass also returns the NeighborList
    (each row ordered by neighbour index with sort_rows=True)."""
    torch = _torch()
    if counts is None:
        counts = torch.zeros(int(bins), dtype=torch.int64, device="cuda")
    nl = _run_pairs(box, points, r_max, query_points, exclude_ii, capacity, True, counts, bins,
                    r_min, neighbor_list, ws, stream, check, sort_rows)
    return (counts, nl) if neighbor_list else counts


def knn_workspace_bytes(box: Box, n, nq, k, r_guard=0.0):
    out = ctypes.c_size_t(0)
    _check(lib().ppa_knn_workspace_bytes(ctypes.byref(box.c()), int(n), int(nq), int(k),
                                         float(r_guard), ctypes.byref(out)))
    return out.value


def query_knn(box: Box, points, k, query_points=None, exclude_ii=None, r_guard=0.0,
              with_dist=True, ws=None, stream=None, check=True) -> NeighborList:
    """The k nearest points of every query point, rows sorted by (r, j).

    r_guard > 0 keeps only neighbours closer than r_guard (rows may then be
    shorter than k)."""
    torch = _torch()
    pts = _points(points)
    n = pts.shape[0]
    q = None if query_points is None else _points(query_points)
    nq = n if q is None else q.shape[0]
    if exclude_ii is None:
        exclude_ii = q is None
    ws = ws or default_workspace()
    need = knn_workspace_bytes(box, n, 0 if q is None else nq, k, r_guard)
    dev = pts.device
    if nq == 0:
        return NeighborList(torch.zeros(1, dtype=torch.int64, device=dev),
                            torch.zeros(0, dtype=torch.int32, device=dev),
                            torch.zeros(0, dtype=torch.int32, device=dev),
                            torch.zeros(0, dtype=torch.float32, device=dev) if with_dist else None,
                            0)
    wptr, wlen = ws.get(need)
    offsets = torch.empty(nq + 1, dtype=torch.int64, device=dev)
    counts = torch.empty(nq, dtype=torch.int32, device=dev)
    cap = max(nq * int(k), 1)
    pidx = torch.empty(cap, dtype=torch.int32, device=dev)
    dist = torch.empty(cap, dtype=torch.float32, device=dev) if with_dist else None
    npairs = torch.zeros(1, dtype=torch.int64, device=dev)
    _check(lib().ppa_query_knn(ctypes.byref(box.c()), _ptr(pts), n, _ptr(q), nq, int(k),
                               float(r_guard), int(bool(exclude_ii)), 0, wptr, wlen,
                               _ptr(offsets), _ptr(counts), _ptr(pidx), _ptr(dist), _ptr(npairs),
                               _stream(stream)))
    if check:
        _check(ws.status(stream))
    np_ = int(npairs.item())
    return NeighborList(offsets, counts, pidx[:np_], None if dist is None else dist[:np_], np_)


def pmft2d_workspace_bytes(box: Box, n, nq, nbx, nby, x_max, y_max, r_max):
    out = ctypes.c_size_t(0)
    _check(lib().ppa_pmft2d_workspace_bytes(ctypes.byref(box.c()), int(n), int(nq), int(nbx),
                                            int(nby), float(x_max), float(y_max), float(r_max),
                                            ctypes.byref(out)))
    return out.value


def pmft2d_counts(box: Box, points, angles, nbx, nby, x_max, y_max, r_max, query_points=None,
                  exclude_ii=None, counts=None, ws=None, stream=None, check=True):
    """2D PMFT bond histogram, uint32 [nbx, nby] (accumulated into `counts`).

    `angles` are the orientations of the query points (of `points` when
    query_points is None), in radians."""
    torch = _torch()
    pts = _points(points)
    n = pts.shape[0]
    q = None if query_points is None else _points(query_points)
    nq = n if q is None else q.shape[0]
    if exclude_ii is None:
        exclude_ii = q is None
    th = angles
    if not isinstance(th, torch.Tensor):
        th = torch.as_tensor(np.ascontiguousarray(th, dtype=np.float32))
    th = th.to(device=pts.device, dtype=torch.float32).contiguous().reshape(-1)
    if th.shape[0] != nq:
        raise ValueError("one orientation per query point is required")
    if counts is None:
        counts = torch.zeros((int(nbx), int(nby)), dtype=torch.uint32, device=pts.device)
    ws = ws or default_workspace()
    wptr, wlen = ws.get(pmft2d_workspace_bytes(box, n, 0 if q is None else nq, nbx, nby, x_max,
                                               y_max, r_max))
    _check(lib().ppa_pmft2d(ctypes.byref(box.c()), _ptr(pts), n, _ptr(q), _ptr(th), nq, int(nbx),
                            int(nby), float(x_max), float(y_max), float(r_max),
                            int(bool(exclude_ii)), 0, wptr, wlen, _ptr(counts), _stream(stream)))
    if check:
        _check(ws.status(stream))
    return counts


def _frames(boxes, n_points, n_query):
    """Per-frame host arrays for the normalisation calls: (n_frames, CBox
    array, int64 n_points, int64 n_query); scalars apply to every frame."""
    boxes = [boxes] if isinstance(boxes, Box) else list(boxes)
    F = len(boxes)
    npt = np.broadcast_to(np.asarray(n_points, np.int64), (F,)).copy()
    nq = np.broadcast_to(np.asarray(n_query, np.int64), (F,)).copy()
    return F, (CBox * F)(*[b.c() for b in boxes]), npt, nq


def _norm_outputs(counts, shape, with_log):
    torch = _torch()
    ratio = torch.empty(shape, dtype=torch.float64, device=counts.device)
    neglog = torch.empty(shape, dtype=torch.float64, device=counts.device) if with_log else None
    return ratio, neglog


def normalize_pmft2d(counts, boxes, n_points, n_query, x_max, y_max, stream=None):
    """(pair correlation, PMFT) float64 device tensors [nbx, nby] from 2D PMFT
    counts accumulated over the frames of `boxes` (a Box or one per frame;
    n_points / n_query per frame or scalars), by ppa_pmft2d_normalize."""
    F, cb, npt, nq = _frames(boxes, n_points, n_query)
    nbx, nby = counts.shape
    pcf, pmft = _norm_outputs(counts, (nbx, nby), True)
    _check(lib().ppa_pmft2d_normalize(_ptr(counts.contiguous()), int(nbx), int(nby), float(x_max),
                                      float(y_max), F, cb, npt.ctypes.data_as(ctypes.c_void_p),
                                      nq.ctypes.data_as(ctypes.c_void_p), _ptr(pcf), _ptr(pmft),
                                      _stream(stream)))
    return pcf, pmft


def _orient(v, device, rows, width, what):
    torch = _torch()
    t = v if isinstance(v, torch.Tensor) else torch.as_tensor(np.ascontiguousarray(v, np.float32))
    t = t.to(device=device, dtype=torch.float32).contiguous().reshape(-1)
    if t.shape[0] != rows * width:
        raise ValueError(f"one {what} per point is required")
    return t


def pmft_xyt_workspace_bytes(box: Box, n, nq, nbx, nby, nbt, x_max, y_max, r_max):
    out = ctypes.c_size_t(0)
    _check(lib().ppa_pmft_xyt_workspace_bytes(ctypes.byref(box.c()), int(n), int(nq), int(nbx),
                                              int(nby), int(nbt), float(x_max), float(y_max),
                                              float(r_max), ctypes.byref(out)))
    return out.value


def pmft_xyt_counts(box: Box, points, angles, nbx, nby, nbt, x_max, y_max, r_max,
                    query_points=None, query_angles=None, exclude_ii=None, counts=None, ws=None,
                    stream=None, check=True):
    """2D PMFT with relative orientation, uint32 [nbx, nby, nbt] over
    (x', y', (theta_j - theta_i) mod 2 pi), accumulated into `counts`.

    `angles` are the points' orientations; `query_angles` those of the query
    points (needed only with query_points)."""
    torch = _torch()
    pts = _points(points)
    n = pts.shape[0]
    q = None if query_points is None else _points(query_points)
    nq = n if q is None else q.shape[0]
    if exclude_ii is None:
        exclude_ii = q is None
    th = _orient(angles, pts.device, n, 1, "orientation")
    qth = None
    if q is not None:
        if query_angles is None:
            raise ValueError("query_angles are required with query_points")
        qth = _orient(query_angles, pts.device, nq, 1, "orientation")
    if counts is None:
        counts = torch.zeros((int(nbx), int(nby), int(nbt)), dtype=torch.uint32, device=pts.device)
    if nq == 0:
        return counts
    ws = ws or default_workspace()
    wptr, wlen = ws.get(pmft_xyt_workspace_bytes(box, n, 0 if q is None else nq, nbx, nby, nbt,
                                                 x_max, y_max, r_max))
    _check(lib().ppa_pmft_xyt(ctypes.byref(box.c()), _ptr(pts), _ptr(th), n, _ptr(q), _ptr(qth),
                              nq, int(nbx), int(nby), int(nbt), float(x_max), float(y_max),
                              float(r_max), int(bool(exclude_ii)), 0, wptr, wlen, _ptr(counts),
                              _stream(stream)))
    if check:
        _check(ws.status(stream))
    return counts


def normalize_pmft_xyt(counts, boxes, n_points, n_query, x_max, y_max, stream=None):
    """(pcf, PMFT) float64 device tensors [nbx, nby, nbt] from XYT counts by
    ppa_pmft_xyt_normalize (the angle bin weighted by its share of a turn)."""
    F, cb, npt, nq = _frames(boxes, n_points, n_query)
    nbx, nby, nbt = counts.shape
    pcf, pmft = _norm_outputs(counts, (nbx, nby, nbt), True)
    _check(lib().ppa_pmft_xyt_normalize(_ptr(counts.contiguous()), int(nbx), int(nby), int(nbt),
                                        float(x_max), float(y_max), F, cb,
                                        npt.ctypes.data_as(ctypes.c_void_p),
                                        nq.ctypes.data_as(ctypes.c_void_p), _ptr(pcf), _ptr(pmft),
                                        _stream(stream)))
    return pcf, pmft


def pmft_xyz_workspace_bytes(box: Box, n, nq, nbx, nby, nbz, x_max, y_max, z_max, r_max):
    out = ctypes.c_size_t(0)
    _check(lib().ppa_pmft_xyz_workspace_bytes(ctypes.byref(box.c()), int(n), int(nq), int(nbx),
                                              int(nby), int(nbz), float(x_max), float(y_max),
                                              float(z_max), float(r_max), ctypes.byref(out)))
    return out.value


def pmft_xyz_counts(box: Box, points, quats, nbx, nby, nbz, x_max, y_max, z_max, r_max,
                    query_points=None, exclude_ii=None, counts=None, ws=None, stream=None,
                    check=True):
    """3D PMFT bond histogram, uint32 [nbx, nby, nbz] of the bonds in each
    query's frame, accumulated into `counts`.

    `quats` [nq, 4] are the orientations (w, x, y, z) of the query points
    (of `points` when query_points is None)."""
    torch = _torch()
    pts = _points(points)
    n = pts.shape[0]
    q = None if query_points is None else _points(query_points)
    nq = n if q is None else q.shape[0]
    if exclude_ii is None:
        exclude_ii = q is None
    qq = _orient(quats, pts.device, nq, 4, "quaternion")
    if counts is None:
        counts = torch.zeros((int(nbx), int(nby), int(nbz)), dtype=torch.uint32, device=pts.device)
    if nq == 0:
        return counts
    ws = ws or default_workspace()
    wptr, wlen = ws.get(pmft_xyz_workspace_bytes(box, n, 0 if q is None else nq, nbx, nby, nbz,
                                                 x_max, y_max, z_max, r_max))
    _check(lib().ppa_pmft_xyz(ctypes.byref(box.c()), _ptr(pts), n, _ptr(q), _ptr(qq), nq,
                              int(nbx), int(nby), int(nbz), float(x_max), float(y_max),
                              float(z_max), float(r_max), int(bool(exclude_ii)), 0, wptr, wlen,
                              _ptr(counts), _stream(stream)))
    if check:
        _check(ws.status(stream))
    return counts


def normalize_pmft_xyz(counts, boxes, n_points, n_query, x_max, y_max, z_max, stream=None):
    """(pcf, PMFT) float64 device tensors [nbx, nby, nbz] from XYZ counts by
    ppa_pmft_xyz_normalize."""
    F, cb, npt, nq = _frames(boxes, n_points, n_query)
    nbx, nby, nbz = counts.shape
    pcf, pmft = _norm_outputs(counts, (nbx, nby, nbz), True)
    _check(lib().ppa_pmft_xyz_normalize(_ptr(counts.contiguous()), int(nbx), int(nby), int(nbz),
                                        float(x_max), float(y_max), float(z_max), F, cb,
                                        npt.ctypes.data_as(ctypes.c_void_p),
                                        nq.ctypes.data_as(ctypes.c_void_p), _ptr(pcf), _ptr(pmft),
                                        _stream(stream)))
    return pcf, pmft


def _complex_values(v, device, rows):
    """Complex (or real) per-point values as a [rows, 2] float32 device tensor."""
    torch = _torch()
    if isinstance(v, torch.Tensor):
        t = torch.view_as_real(v.to(torch.complex64)) if v.is_complex() else v
        t = t.to(device=device, dtype=torch.float32)
        if t.ndim == 1:
            t = torch.stack([t, torch.zeros_like(t)], 1)
    else:
        a = np.asarray(v)
        if np.iscomplexobj(a):
            a = np.stack([a.real, a.imag], -1)
        a = np.asarray(a, np.float32)
        if a.ndim == 1:
            a = np.stack([a, np.zeros_like(a)], 1)
        t = torch.as_tensor(np.ascontiguousarray(a)).to(device)
    t = t.contiguous().reshape(-1, 2)
    if t.shape[0] != rows:
        raise ValueError("one value per point is required")
    return t


def correlation_workspace_bytes(box: Box, n, nq, bins, r_max, r_min=0.0):
    out = ctypes.c_size_t(0)
    _check(lib().ppa_correlation_workspace_bytes(ctypes.byref(box.c()), int(n), int(nq), int(bins),
                                                 float(r_min), float(r_max), ctypes.byref(out)))
    return out.value


def correlation_sums(box: Box, points, values, bins, r_max, r_min=0.0, query_points=None,
                     query_values=None, exclude_ii=None, sums=None, counts=None, ws=None,
                     stream=None, check=True):
    """Spatial correlation sums: (sums float64 [bins, 2] = (re, im) of the sum of
    conj(f_i) g_j per bin, counts uint64 [bins]), both accumulated.  Values are
    complex or real per point; query values default to the points' values."""
    torch = _torch()
    pts = _points(points)
    n = pts.shape[0]
    q = None if query_points is None else _points(query_points)
    nq = n if q is None else q.shape[0]
    if exclude_ii is None:
        exclude_ii = q is None
    g = _complex_values(values, pts.device, n)
    f = None
    if query_values is not None:
        f = _complex_values(query_values, pts.device, nq)
    elif q is not None:
        raise ValueError("query_values are required with query_points")
    if sums is None:
        sums = torch.zeros((int(bins), 2), dtype=torch.float64, device=pts.device)
    if counts is None:
        counts = torch.zeros(int(bins), dtype=torch.uint64, device=pts.device)
    if nq == 0:
        return sums, counts
    ws = ws or default_workspace()
    wptr, wlen = ws.get(correlation_workspace_bytes(box, n, 0 if q is None else nq, bins, r_max,
                                                    r_min))
    _check(lib().ppa_correlation(ctypes.byref(box.c()), _ptr(pts), _ptr(g), n, _ptr(q), _ptr(f),
                                 nq, int(bins), float(r_min), float(r_max), int(bool(exclude_ii)),
                                 0, wptr, wlen, _ptr(sums), _ptr(counts), _stream(stream)))
    if check:
        _check(ws.status(stream))
    return sums, counts


def correlation(box: Box, points, values, bins, r_max, r_min=0.0, stream=None, **kw):
    """C(r) per bin (float64 device tensor [bins, 2] of (re, im), 0 where a bin
    holds no pair; ppa_correlation_finalize) and the pair counts."""
    torch = _torch()
    sums, counts = correlation_sums(box, points, values, bins, r_max, r_min, stream=stream, **kw)
    corr = torch.empty_like(sums)
    _check(lib().ppa_correlation_finalize(_ptr(sums), _ptr(counts), int(bins), _ptr(corr),
                                          _stream(stream)))
    return corr, counts


def steinhardt(box: Box, points, neighbors, l, query_points=None, with_w=False, ws=None,
               stream=None, check=True):
    """Steinhardt Q_l (and normalised W_l with with_w) of every query row of a
    NeighborList, float64 [nq] device tensors: (ql, wl or None).

    `neighbors` is a NeighborList (offsets, point_idx) built on these
    positions, or a tuple (offsets, point_idx) of device or host arrays."""
    torch = _torch()
    pts = _points(points)
    n = pts.shape[0]
    q = None if query_points is None else _points(query_points)
    if isinstance(neighbors, NeighborList):
        off, idx = neighbors.offsets, neighbors.point_idx
    else:
        off, idx = neighbors
    off = torch.as_tensor(np.asarray(off) if not isinstance(off, torch.Tensor) else off)
    idx = torch.as_tensor(np.asarray(idx) if not isinstance(idx, torch.Tensor) else idx)
    off = off.to(device=pts.device, dtype=torch.int64).contiguous()
    idx = idx.to(device=pts.device, dtype=torch.int32).contiguous()
    nq = off.shape[0] - 1
    if q is None and nq != n:
        raise ValueError("a list over the points needs n + 1 offsets")
    if q is not None and q.shape[0] != nq:
        raise ValueError("one offset row per query point is required")
    ql = torch.zeros(max(nq, 0), dtype=torch.float64, device=pts.device)
    wl = torch.zeros(max(nq, 0), dtype=torch.float64, device=pts.device) if with_w else None
    if nq == 0:
        return ql, wl
    need = ctypes.c_size_t(0)
    _check(lib().ppa_steinhardt_workspace_bytes(int(l), 0, ctypes.byref(need)))
    ws = ws or default_workspace()
    wptr, wlen = ws.get(need.value)
    _check(lib().ppa_steinhardt(ctypes.byref(box.c()), _ptr(pts), n, _ptr(q), nq, _ptr(off),
                                _ptr(idx) if idx.numel() else None, idx.numel(), int(l), 0, wptr,
                                wlen, _ptr(ql), _ptr(wl), _stream(stream)))
    if check:
        _check(ws.status(stream))
    return ql, wl


def clusters(neighbors, n, ws=None, stream=None, check=True, symmetric=False):
    """Connected components of a NeighborList over n points (bonds as
    undirected edges): (labels, cluster_idx, sizes, n_clusters) with labels
    the smallest index of each point's component, cluster_idx the components
    numbered by that index, sizes[:n_clusters] their point counts.

    symmetric=True declares that j is in row i exactly when i is in row j
    (a ball query of the points with themselves), which lets large
    components form faster; with a list that is not symmetric the labels
    may be wrong."""
    torch = _torch()
    if isinstance(neighbors, NeighborList):
        off, idx = neighbors.offsets, neighbors.point_idx
    else:
        off, idx = neighbors
    dev = "cuda"
    off = torch.as_tensor(np.asarray(off) if not isinstance(off, torch.Tensor) else off)
    idx = torch.as_tensor(np.asarray(idx) if not isinstance(idx, torch.Tensor) else idx)
    off = off.to(device=dev, dtype=torch.int64).contiguous()
    idx = idx.to(device=dev, dtype=torch.int32).contiguous()
    n = int(n)
    if off.shape[0] != n + 1:
        raise ValueError("the list needs n + 1 offsets (row i is point i)")
    labels = torch.empty(n, dtype=torch.int32, device=dev)
    cidx = torch.empty(n, dtype=torch.int32, device=dev)
    sizes = torch.empty(n, dtype=torch.int32, device=dev)
    nc = torch.zeros(1, dtype=torch.int64, device=dev)
    need = ctypes.c_size_t(0)
    _check(lib().ppa_cluster_workspace_bytes(n, ctypes.byref(need)))
    ws = ws or default_workspace()
    wptr, wlen = ws.get(need.value)
    _check(lib().ppa_cluster(_ptr(off), _ptr(idx) if idx.numel() else None, n, idx.numel(),
                             PPA_CLUSTER_SYMMETRIC if symmetric else 0,
                             wptr, wlen, _ptr(labels) if n else None, _ptr(cidx) if n else None,
                             _ptr(sizes) if n else None, _ptr(nc), _stream(stream)))
    if check:
        _check(ws.status(stream))
    k = int(nc.item())
    return labels, cidx, sizes[:k], k


def knn_from_list(nl: NeighborList, k, ws=None, stream=None, check=True) -> NeighborList:
    """The k entries of smallest (distance, index) of every row of a stored
    NeighborList with distances; for a ball list whose rows all hold at least
    k entries this is the k-nearest query."""
    torch = _torch()
    if nl.dist is None:
        raise ValueError("the list needs its distances")
    nq = nl.offsets.shape[0] - 1
    dev = nl.offsets.device
    need = ctypes.c_size_t(0)
    _check(lib().ppa_knn_from_nlist_workspace_bytes(nq, int(k), ctypes.byref(need)))
    ws = ws or default_workspace()
    wptr, wlen = ws.get(need.value)
    off = torch.empty(nq + 1, dtype=torch.int64, device=dev)
    counts = torch.empty(max(nq, 1), dtype=torch.int32, device=dev)
    idx = torch.empty(max(nq * int(k), 1), dtype=torch.int32, device=dev)
    dist = torch.empty(max(nq * int(k), 1), dtype=torch.float32, device=dev)
    npairs = torch.zeros(1, dtype=torch.int64, device=dev)
    cap = nl.point_idx.numel()
    _check(lib().ppa_knn_from_nlist(_ptr(nl.offsets), _ptr(nl.point_idx) if cap else None,
                                    _ptr(nl.dist) if cap else None, nq, cap, int(k), 0, wptr,
                                    wlen, _ptr(off), _ptr(counts), _ptr(idx), _ptr(dist),
                                    _ptr(npairs), _stream(stream)))
    if check:
        _check(ws.status(stream))
    np_ = int(npairs.item())
    return NeighborList(off, counts[:nq], idx[:np_], dist[:np_], np_)


def smooth_rdf_workspace_bytes(box: Box, n, bins, r_max, sigma):
    out = ctypes.c_size_t(0)
    _check(lib().ppa_smooth_rdf_workspace_bytes(ctypes.byref(box.c()), int(n), int(bins),
                                                float(r_max), float(sigma), ctypes.byref(out)))
    return out.value


def smooth_rdf_h(box: Box, points, bins, r_max, sigma, h=None, ws=None, stream=None, check=True):
    """Gaussian-smoothed RDF numerator h (float64 [bins], accumulated into `h`)."""
    torch = _torch()
    pts = _points(points)
    n = pts.shape[0]
    if h is None:
        h = torch.zeros(int(bins), dtype=torch.float64, device=pts.device)
    ws = ws or default_workspace()
    wptr, wlen = ws.get(smooth_rdf_workspace_bytes(box, n, bins, r_max, sigma))
    _check(lib().ppa_smooth_rdf_fwd(ctypes.byref(box.c()), _ptr(pts), n, int(bins), float(r_max),
                                    float(sigma), 0, wptr, wlen, _ptr(h), _stream(stream)))
    if check:
        _check(ws.status(stream))
    return h


def smooth_rdf_grad(box: Box, points, bins, r_max, sigma, grad_h, ws=None, stream=None,
                    check=True):
    """dL/dpoints (float32 [n, 3]) given dL/dh (float64 [bins]); pairs are found again."""
    torch = _torch()
    pts = _points(points)
    n = pts.shape[0]
    gh = grad_h
    if not isinstance(gh, torch.Tensor):
        gh = torch.as_tensor(np.ascontiguousarray(gh, dtype=np.float64))
    gh = gh.to(device=pts.device, dtype=torch.float64).contiguous()
    if gh.shape != (int(bins),):
        raise ValueError("grad_h must have one entry per bin")
    out = torch.empty((n, 3), dtype=torch.float32, device=pts.device)
    ws = ws or default_workspace()
    wptr, wlen = ws.get(smooth_rdf_workspace_bytes(box, n, bins, r_max, sigma))
    _check(lib().ppa_smooth_rdf_bwd(ctypes.byref(box.c()), _ptr(pts), n, int(bins), float(r_max),
                                    float(sigma), _ptr(gh), 0, wptr, wlen, _ptr(out),
                                    _stream(stream)))
    if check:
        _check(ws.status(stream))
    return out


def _smooth_function():
    torch = _torch()

    class SmoothRDF(torch.autograd.Function):
        """h = smoothed RDF numerator of `points` (float64 [bins]); its backward
        runs the library's adjoint kernel."""

        @staticmethod
        def forward(ctx, points, box, bins, r_max, sigma):
            ctx.save_for_backward(points)
            ctx.cfg = (box, int(bins), float(r_max), float(sigma))
            return smooth_rdf_h(box, points.detach(), bins, r_max, sigma)

        @staticmethod
        def backward(ctx, grad_h):
            (points,) = ctx.saved_tensors
            box, bins, r_max, sigma = ctx.cfg
            g = smooth_rdf_grad(box, points.detach(), bins, r_max, sigma, grad_h)
            return g.to(points.dtype), None, None, None, None

    return SmoothRDF


_SmoothRDF = None


def smooth_rdf(points, box: Box, bins, r_max, sigma):
    """Differentiable smoothed RDF numerator h (float64 [bins]) of a float32
    [n, 3] CUDA tensor of positions."""
    global _SmoothRDF
    if _SmoothRDF is None:
        _SmoothRDF = _smooth_function()
    return _SmoothRDF.apply(points, box, bins, r_max, sigma)


def smooth_rdf_g(h, box: Box, n_points, r_max, stream=None):
    """g_b = h_b * scale_b on the bins of [0, r_max), scale from
    ppa_rdf_bin_scale (differentiable in h)."""
    scale = rdf_bin_scale(h.shape[-1], box, n_points, n_points, 0.0, r_max, stream=stream)
    return h * scale.to(h.dtype)


class BatchPlan:
    """Batched ball query + per-frame RDF over many frames, each with its own
    box (frames are consecutive row ranges of one [N, 3] point array).

    run() returns (hist [n_frames, bins] int64, NeighborList over all rows
    with frame-local point indices); graph() captures a run in a HIP graph."""

    def __init__(self, boxes, frame_sizes, bins, r_max, r_min=0.0, exclude_ii=True,
                 capacity=None, sort_rows=False):
        torch = _torch()
        self.boxes = list(boxes)
        sizes = np.asarray(frame_sizes, dtype=np.int64)
        self.offsets_host = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        self.n_frames = len(self.boxes)
        if sizes.shape[0] != self.n_frames:
            raise ValueError("one size per box is required")
        self.n = int(self.offsets_host[-1])
        self.bins = int(bins)
        self.r_max, self.r_min = float(r_max), float(r_min)
        cboxes = (CBox * self.n_frames)(*[b.c() for b in self.boxes])
        h = ctypes.c_void_p()
        _check(lib().ppa_batch_plan_create(self.n_frames, cboxes,
                                           self.offsets_host.ctypes.data_as(ctypes.c_void_p),
                                           self.bins, self.r_min, self.r_max,
                                           int(bool(exclude_ii)),
                                           PPA_SORT_ROWS if sort_rows else 0, ctypes.byref(h)))
        self._h = h
        need = ctypes.c_size_t(0)
        _check(lib().ppa_batch_workspace_bytes(self._h, ctypes.byref(need)))
        self.ws = Workspace()
        self.wptr, self.wlen = self.ws.get(need.value)
        _check(lib().ppa_batch_upload(self._h, self.wptr, self.wlen, _stream()))
        if capacity is None:
            capacity = sum(_estimate_pairs(b, int(m), int(m), r_max) for b, m in zip(self.boxes, sizes))
        self.capacity = int(capacity)
        dev = "cuda"
        self.offsets = torch.empty(self.n + 1, dtype=torch.int64, device=dev)
        self.counts = torch.empty(self.n, dtype=torch.int32, device=dev)
        self.point_idx = torch.empty(max(self.capacity, 1), dtype=torch.int32, device=dev)
        self.dist = torch.empty(max(self.capacity, 1), dtype=torch.float32, device=dev)
        self.n_pairs = torch.zeros(1, dtype=torch.int64, device=dev)
        self._graph = None

    def __del__(self):
        try:
            if getattr(self, "_graph", None):
                lib().ppa_batch_graph_destroy(self._graph)
            if getattr(self, "_h", None):
                lib().ppa_batch_plan_destroy(self._h)
        except Exception:
            pass

    def _out(self):
        return (_ptr(self.offsets), _ptr(self.counts), _ptr(self.point_idx), _ptr(self.dist),
                self.capacity, _ptr(self.n_pairs))

    def config(self, index=-1):
        n, c, scale, cap = (ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double(),
                            ctypes.c_int32())
        _check(lib().ppa_batch_config(self._h, int(index), ctypes.byref(n), ctypes.byref(c),
                                      ctypes.byref(scale), ctypes.byref(cap)))
        run, waves = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().ppa_batch_config_shape(self._h, -1, ctypes.byref(run), ctypes.byref(waves)))
        return {"n_configs": n.value, "chosen": c.value, "cell_scale": scale.value,
                "blocks_per_cu": cap.value, "cells_per_item": run.value,
                "waves_per_workgroup": waves.value}

    def cells(self, index=-1):
        """Cell build of a configuration (-1: the chosen one): total cells,
        LDS-counted chunks, and frames counted with global atomics."""
        c, k, g = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().ppa_batch_config_cells(self._h, int(index), ctypes.byref(c), ctypes.byref(k),
                                            ctypes.byref(g)))
        return {"cells": c.value, "chunks": k.value, "global_frames": g.value}

    def autotune(self, points, reps=3, stream=None):
        """Times every launch configuration on these points and keeps the fastest."""
        pts = _points(points)
        n = self.config()["n_configs"]
        ms = (ctypes.c_float * n)()
        o = self._out()
        _check(lib().ppa_batch_autotune(self._h, _ptr(pts), self.wptr, self.wlen, o[0], o[1], o[2],
                                        o[3], o[4], o[5], int(reps), _stream(stream), ms))
        return list(ms), self.config()

    def run(self, points, hist=None, stream=None, check=True):
        torch = _torch()
        pts = _points(points)
        if pts.shape[0] != self.n:
            raise ValueError("points must hold every frame's rows")
        if hist is None:
            hist = torch.zeros((self.n_frames, self.bins), dtype=torch.int64, device=pts.device)
        hist0 = hist.clone() if check else None
        o = self._out()
        _check(lib().ppa_batch_run(self._h, _ptr(pts), self.wptr, self.wlen, _ptr(hist), *o,
                                   _stream(stream)))
        if check:
            st = self.ws.status(stream)
            if st == PPA_ECAPACITY:
                # the estimate was short: size the list from the count the run
                # reported and run again (the histograms restart from their
                # values before the call)
                self._grow(int(self.n_pairs.item()))
                hist.copy_(hist0)
                o = self._out()
                _check(lib().ppa_batch_run(self._h, _ptr(pts), self.wptr, self.wlen, _ptr(hist),
                                           *o, _stream(stream)))
                st = self.ws.status(stream)
            _check(st)
        return hist, self.neighbor_list()

    def _grow(self, pairs):
        torch = _torch()
        if self._graph:  # a captured graph points at the old buffers
            lib().ppa_batch_graph_destroy(self._graph)
            self._graph = None
        self.capacity = int(pairs) + 1024
        self.point_idx = torch.empty(self.capacity, dtype=torch.int32, device="cuda")
        self.dist = torch.empty(self.capacity, dtype=torch.float32, device="cuda")

    def neighbor_list(self):
        np_ = int(self.n_pairs.item())
        return NeighborList(self.offsets, self.counts, self.point_idx[:np_], self.dist[:np_], np_)

    def graph(self, points, hist):
        """Captures a run with these (device-resident) points and histogram; the
        returned callable replays it on a stream with one graph launch."""
        pts = _points(points)
        if self._graph:
            lib().ppa_batch_graph_destroy(self._graph)
            self._graph = None
        g = ctypes.c_void_p()
        o = self._out()
        _check(lib().ppa_batch_graph_create(self._h, _ptr(pts), self.wptr, self.wlen, _ptr(hist),
                                            *o, ctypes.byref(g)))
        self._graph = g
        self._graph_args = (pts, hist)  # keep them alive with the graph

        def launch(stream=None):
            _check(lib().ppa_batch_graph_launch(self._graph, _stream(stream)))
        return launch


def rdf_from_nlist(nl: NeighborList, bins, r_max, r_min=0.0, counts=None, stream=None):
    torch = _torch()
    if counts is None:
        counts = torch.zeros(int(bins), dtype=torch.int64, device="cuda")
    npairs = torch.tensor([nl.n_pairs], dtype=torch.int64, device=counts.device)
    _check(lib().ppa_rdf_from_nlist(_ptr(nl.dist), _ptr(npairs), int(nl.n_pairs), int(bins),
                                    float(r_min), float(r_max), _ptr(counts), _stream(stream)))
    return counts


def normalize_rdf(counts, boxes, n_points, n_query, r_min, r_max, stream=None):
    """(g, PMF = -ln g) float64 device tensors from RDF counts accumulated over
    the frames of `boxes` (a Box or one per frame; n_points / n_query per
    frame or scalars), by ppa_rdf_normalize."""
    F, cb, npt, nq = _frames(boxes, n_points, n_query)
    bins = counts.shape[-1]
    g, pmf = _norm_outputs(counts, (bins,), True)
    _check(lib().ppa_rdf_normalize(_ptr(counts.contiguous()), int(bins), float(r_min),
                                   float(r_max), F, cb, npt.ctypes.data_as(ctypes.c_void_p),
                                   nq.ctypes.data_as(ctypes.c_void_p), _ptr(g), _ptr(pmf),
                                   _stream(stream)))
    return g, pmf


def rdf_bin_scale(bins, boxes, n_points, n_query, r_min, r_max, stream=None):
    """The RDF's per-bin factor 1 / (D dV_b) (float64 device tensor [bins]),
    by ppa_rdf_bin_scale."""
    torch = _torch()
    F, cb, npt, nq = _frames(boxes, n_points, n_query)
    scale = torch.empty(int(bins), dtype=torch.float64, device="cuda")
    _check(lib().ppa_rdf_bin_scale(int(bins), float(r_min), float(r_max), F, cb,
                                   npt.ctypes.data_as(ctypes.c_void_p),
                                   nq.ctypes.data_as(ctypes.c_void_p), _ptr(scale),
                                   _stream(stream)))
    return scale


def version():
    return lib().ppa_version().decode()
