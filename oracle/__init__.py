"""FP64 reference oracle (test infrastructure only).

This package is the reference that the GPU library is checked against.  Only
the test suite, the smoke check and the CPU-baseline leg of the benchmark
import it; the GPU library never does, and the two share no code.

The compiled part (``oracle.c``) computes every result from its plain
definition: brute force over all (query, point) pairs in double precision,
starting from the same FP32 arrays the GPU receives.  The normalisation
helpers below (RDF, PMF, PMFT, smoothed RDF) are closed-form FP64 numpy.

Each function names the part of the paper it follows.  Parity status:
  * minimum image, ball query, RDF counts, k-NN, 2D PMFT counts, the 2D
    PMFT with relative orientation (XYT) and the 3D PMFT (XYZ) counts, the
    spatial correlation function, Steinhardt Q_l and W_l with the Wigner
    3j symbols, clusters, smoothed RDF and its gradient: pinned (see
    tests/test_oracle_*.py);
  * RDF / PMFT normalisation constants: the paper defines the PMF and PMFT
    only up to an additive constant, so the convention below is a reading,
    pinned statistically by the ideal-gas limit only.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

REL_BAND = 1e-5  # ambiguity band, relative in r^2, for cutoff and bin edges


class Box(ctypes.Structure):
    _fields_ = [("L", ctypes.c_double * 3), ("tilt", ctypes.c_double * 3), ("dim", ctypes.c_int32)]


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-fPIC", "-shared",
             "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, i32, f64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        BP = ctypes.POINTER(Box)
        sig = {
            "orc_minimum_image": [BP, P, i64],
            "orc_ball_count": [BP, P, i64, P, i64, f64, i32, P],
            "orc_ball_fill": [BP, P, i64, P, i64, f64, i32, P, P, P],
            "orc_rdf": [BP, P, i64, P, i64, i64, f64, f64, i32, f64, P, P, P],
            "orc_ball_rdf_rows": [BP, P, i64, P, i64, i64, f64, i32, i64, P, P, P, i64, f64, f64,
                                  f64, P, P, P],
            "orc_knn": [BP, P, i64, P, i64, i32, i32, i32, f64, P, P, P],
            "orc_pmft2d": [BP, P, i64, P, P, i64, i64, i64, f64, f64, f64, i32, f64, f64, P, P, P],
            "orc_correlation": [BP, P, P, i64, P, P, i64, i64, f64, f64, i32, f64, P, P, P, P, P],
            "orc_pmft_xyt": [BP, P, P, i64, P, P, i64, i64, i64, i64, f64, f64, f64, i32, f64,
                             f64, f64, P, P, P],
            "orc_pmft_xyz": [BP, P, i64, P, P, i64, i64, i64, i64, f64, f64, f64, f64, i32, f64,
                             f64, P, P, P],
            "orc_smooth_rdf": [BP, P, i64, i64, f64, f64, P],
            "orc_smooth_rdf_row": [BP, P, i64, i64, P, i64, f64, f64, P],
            "orc_smooth_rdf_grad": [BP, P, i64, i64, f64, f64, P, P, i64, P],
            "orc_num_threads": [],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        _lib = L
    return _lib


def num_threads() -> int:
    return int(lib().orc_num_threads())


def make_box(L, tilt=(0.0, 0.0, 0.0), dim=3) -> Box:
    L = list(L) if np.ndim(L) else [float(L)] * 3
    b = Box()
    for k in range(3):
        b.L[k] = float(L[k])
        b.tilt[k] = float(tilt[k])
    b.dim = int(dim)
    return b


def _f32(a):
    a = np.ascontiguousarray(a, dtype=np.float32)
    assert a.ndim == 2 and a.shape[1] == 3
    return a


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def minimum_image(box: Box, d):
    """Minimum image of FP64 displacements (General Utilities section)."""
    d = np.ascontiguousarray(d, dtype=np.float64).copy()
    lib().orc_minimum_image(ctypes.byref(box), _p(d), d.shape[0])
    return d


def ball_query(box: Box, points, r_max: float, query_points=None, exclude_ii=None,
               rel_band: float = REL_BAND):
    """All (i, j) with minimum-image distance below r_max (query API).

    Returns CSR (offsets int64[nq+1], idx int32[P], r2 float64[P]) that also
    holds the pairs in the band r_max^2 <= r^2 < r_max^2 (1 + rel_band), so a
    caller can tell certain pairs from ambiguous ones.
    """
    pts = _f32(points)
    if exclude_ii is None:
        exclude_ii = query_points is None
    q = pts if query_points is None else _f32(query_points)
    r2lim = float(r_max) ** 2 * (1.0 + rel_band)
    counts = np.zeros(q.shape[0], np.int64)
    lib().orc_ball_count(ctypes.byref(box), _p(pts), pts.shape[0], _p(q), q.shape[0], r2lim,
                         int(exclude_ii), _p(counts))
    offsets = np.zeros(q.shape[0] + 1, np.int64)
    np.cumsum(counts, out=offsets[1:])
    idx = np.empty(int(offsets[-1]), np.int32)
    r2 = np.empty(int(offsets[-1]), np.float64)
    lib().orc_ball_fill(ctypes.byref(box), _p(pts), pts.shape[0], _p(q), q.shape[0], r2lim,
                        int(exclude_ii), _p(offsets), _p(idx), _p(r2))
    return offsets, idx, r2


def rdf_counts(box: Box, points, bins: int, r_max: float, r_min: float = 0.0,
               query_points=None, exclude_ii=None, rel_band: float = REL_BAND):
    """RDF pair histogram bounds (lo, hi, n_ambiguous); exact counts c obey lo <= c <= hi."""
    pts = _f32(points)
    if exclude_ii is None:
        exclude_ii = query_points is None
    q = pts if query_points is None else _f32(query_points)
    lo = np.zeros(bins, np.uint64)
    hi = np.zeros(bins, np.uint64)
    amb = np.zeros(1, np.uint64)
    lib().orc_rdf(ctypes.byref(box), _p(pts), pts.shape[0], _p(q), q.shape[0], bins,
                  float(r_min), float(r_max), int(exclude_ii), rel_band, _p(lo), _p(hi), _p(amb))
    return lo, hi, int(amb[0])


def ball_rdf_rows(box: Box, points, r_max: float, bins: int, rows=None, exclude_ii=True,
                  cap: int = 256, r_min: float = 0.0, lo=None, hi=None, n_amb=None,
                  rel_band: float = REL_BAND):
    """Self-query rows [a, b) of the ball query and their RDF bounds in one sweep.

    Returns (counts int64[m], idx int32[m, cap], r2 float64[m, cap]) for the
    m = b - a rows (each row's points with r^2 < r_max^2 (1 + rel_band), in
    ascending index, padded past counts), and accumulates the rows' RDF pairs
    into lo / hi (uint64[bins]) and n_amb (uint64[1]), allocated when None and
    returned as (counts, idx, r2, lo, hi, n_amb).  A row longer than cap
    raises."""
    pts = _f32(points)
    n = pts.shape[0]
    a, b = (0, n) if rows is None else (int(rows[0]), int(rows[1]))
    q = np.ascontiguousarray(pts[a:b])
    m = b - a
    if lo is None:
        lo = np.zeros(bins, np.uint64)
        hi = np.zeros(bins, np.uint64)
        n_amb = np.zeros(1, np.uint64)
    counts = np.zeros(m, np.int64)
    idx = np.full((m, cap), -1, np.int32)
    r2 = np.full((m, cap), np.inf, np.float64)
    rc = lib().orc_ball_rdf_rows(ctypes.byref(box), _p(pts), n, _p(q), m, a,
                                 float(r_max) ** 2 * (1.0 + rel_band), int(exclude_ii), int(cap),
                                 _p(idx), _p(r2), _p(counts), int(bins), float(r_min),
                                 float(r_max), rel_band, _p(lo), _p(hi), _p(n_amb))
    if rc != 0:
        raise ValueError(f"a row holds more than cap={cap} neighbours")
    return counts, idx, r2, lo, hi, n_amb


def _complex_pairs(v, n):
    v = np.asarray(v)
    if np.iscomplexobj(v):
        out = np.stack([v.real, v.imag], -1)
    else:
        out = np.asarray(v, np.float64).reshape(n, -1)
        if out.shape[1] == 1:
            out = np.concatenate([out, np.zeros_like(out)], 1)
    return np.ascontiguousarray(out.reshape(n, 2), dtype=np.float32)


def correlation(box: Box, points, values, bins: int, r_max: float, r_min: float = 0.0,
                query_points=None, query_values=None, exclude_ii=None,
                rel_band: float = REL_BAND):
    """Spatial correlation function (density module): for ball pairs binned in
    r, S_b = sum of conj(f_i) g_j (complex128) over certain pairs, the
    ambiguity mass per bin, count bounds lo/hi and the ambiguous-pair count.
    Values are complex (or real) per point; query values default to the
    points' values."""
    pts = _f32(points)
    same = query_points is None
    if exclude_ii is None:
        exclude_ii = same
    q = pts if same else _f32(query_points)
    g = _complex_pairs(values, pts.shape[0])
    f = g if query_values is None else _complex_pairs(query_values, q.shape[0])
    s = np.zeros(2 * bins, np.float64)
    m = np.zeros(bins, np.float64)
    lo = np.zeros(bins, np.uint64)
    hi = np.zeros(bins, np.uint64)
    amb = np.zeros(1, np.uint64)
    lib().orc_correlation(ctypes.byref(box), _p(pts), _p(g), pts.shape[0], _p(q), _p(f),
                          q.shape[0], int(bins), float(r_min), float(r_max), int(exclude_ii),
                          rel_band, _p(s), _p(m), _p(lo), _p(hi), _p(amb))
    return s[0::2] + 1j * s[1::2], m, lo, hi, int(amb[0])


def knn(box: Box, points, k: int, query_points=None, exclude_ii=None, extra: int = 1,
        r_guard: float = 0.0):
    """First k + extra neighbours per query in (r^2, j) order; idx -1 pads short rows."""
    pts = _f32(points)
    if exclude_ii is None:
        exclude_ii = query_points is None
    q = pts if query_points is None else _f32(query_points)
    m = k + extra
    idx = np.empty((q.shape[0], m), np.int32)
    r2 = np.empty((q.shape[0], m), np.float64)
    ln = np.empty(q.shape[0], np.int32)
    lib().orc_knn(ctypes.byref(box), _p(pts), pts.shape[0], _p(q), q.shape[0], int(k), int(extra),
                  int(exclude_ii), float(r_guard) ** 2 if r_guard > 0 else 0.0, _p(idx), _p(r2), _p(ln))
    return idx, r2, ln


def pmft2d_counts(box: Box, points, query_points, query_theta, nbx: int, nby: int,
                  x_max: float, y_max: float, r_max: float, exclude_ii=None,
                  rel_band: float = REL_BAND, abs_band=None):
    """2D PMFT histogram bounds (lo, hi, n_ambiguous), counts[ix*nby + iy]."""
    pts = _f32(points)
    same = query_points is None
    if exclude_ii is None:
        exclude_ii = same
    q = pts if same else _f32(query_points)
    th = np.ascontiguousarray(query_theta, dtype=np.float32)
    if abs_band is None:
        abs_band = rel_band * max(x_max, y_max)
    lo = np.zeros(nbx * nby, np.uint64)
    hi = np.zeros(nbx * nby, np.uint64)
    amb = np.zeros(1, np.uint64)
    lib().orc_pmft2d(ctypes.byref(box), _p(pts), pts.shape[0], _p(q), _p(th), q.shape[0], nbx, nby,
                     float(x_max), float(y_max), float(r_max), int(exclude_ii), rel_band,
                     float(abs_band), _p(lo), _p(hi), _p(amb))
    return lo.reshape(nbx, nby), hi.reshape(nbx, nby), int(amb[0])


def pmft_xyt_counts(box: Box, points, theta, query_points, query_theta, nbx: int, nby: int,
                    nbt: int, x_max: float, y_max: float, r_max: float, exclude_ii=None,
                    rel_band: float = REL_BAND, abs_band=None, t_band=None):
    """2D PMFT with relative orientation (PMFT section): bounds (lo, hi,
    n_ambiguous) of counts[ix, iy, it] over (x', y', (theta_j - theta_i) mod 2pi)."""
    pts = _f32(points)
    same = query_points is None
    if exclude_ii is None:
        exclude_ii = same
    q = pts if same else _f32(query_points)
    th = np.ascontiguousarray(theta, dtype=np.float32)
    qth = th if same and query_theta is None else np.ascontiguousarray(query_theta, np.float32)
    if abs_band is None:
        abs_band = rel_band * max(x_max, y_max)
    if t_band is None:
        t_band = rel_band * 2.0 * math.pi
    nb = nbx * nby * nbt
    lo = np.zeros(nb, np.uint64)
    hi = np.zeros(nb, np.uint64)
    amb = np.zeros(1, np.uint64)
    lib().orc_pmft_xyt(ctypes.byref(box), _p(pts), _p(th), pts.shape[0], _p(q), _p(qth),
                       q.shape[0], nbx, nby, nbt, float(x_max), float(y_max), float(r_max),
                       int(exclude_ii), rel_band, float(abs_band), float(t_band), _p(lo), _p(hi),
                       _p(amb))
    return lo.reshape(nbx, nby, nbt), hi.reshape(nbx, nby, nbt), int(amb[0])


def pmft_xyz_counts(box: Box, points, query_points, query_quat, nbx: int, nby: int, nbz: int,
                    x_max: float, y_max: float, z_max: float, r_max: float, exclude_ii=None,
                    rel_band: float = REL_BAND, abs_band=None):
    """3D PMFT (PMFT section): bounds (lo, hi, n_ambiguous) of counts[ix, iy, iz]
    of the bonds in the frame of each query's unit quaternion (w, x, y, z)."""
    pts = _f32(points)
    same = query_points is None
    if exclude_ii is None:
        exclude_ii = same
    q = pts if same else _f32(query_points)
    qq = np.ascontiguousarray(query_quat, dtype=np.float32).reshape(-1, 4)
    if abs_band is None:
        abs_band = rel_band * max(x_max, y_max, z_max)
    nb = nbx * nby * nbz
    lo = np.zeros(nb, np.uint64)
    hi = np.zeros(nb, np.uint64)
    amb = np.zeros(1, np.uint64)
    lib().orc_pmft_xyz(ctypes.byref(box), _p(pts), pts.shape[0], _p(q), _p(qq), q.shape[0], nbx,
                       nby, nbz, float(x_max), float(y_max), float(z_max), float(r_max),
                       int(exclude_ii), rel_band, float(abs_band), _p(lo), _p(hi), _p(amb))
    return lo.reshape(nbx, nby, nbz), hi.reshape(nbx, nby, nbz), int(amb[0])


def smooth_rdf_h(box: Box, points, bins: int, r_max: float, sigma: float):
    """Smoothed RDF numerator h_b (FP64) over all ordered pairs."""
    pts = _f32(points)
    h = np.zeros(bins, np.float64)
    lib().orc_smooth_rdf(ctypes.byref(box), _p(pts), pts.shape[0], bins, float(r_max),
                         float(sigma), _p(h))
    return h


def smooth_rdf_row(box: Box, points, k: int, pk, bins: int, r_max: float, sigma: float):
    """Contribution of both ordered pairs of particle k (placed at pk) to h."""
    pts = _f32(points)
    pk = np.ascontiguousarray(pk, dtype=np.float64)
    h = np.zeros(bins, np.float64)
    lib().orc_smooth_rdf_row(ctypes.byref(box), _p(pts), pts.shape[0], int(k), _p(pk), bins,
                             float(r_max), float(sigma), _p(h))
    return h


def smooth_rdf_grad(box: Box, points, bins: int, r_max: float, sigma: float, grad_h, rows=None):
    """dL/dp for the listed rows (all when rows is None), given dL/dh."""
    pts = _f32(points)
    gh = np.ascontiguousarray(grad_h, dtype=np.float64)
    if rows is None:
        out = np.zeros((pts.shape[0], 3), np.float64)
        lib().orc_smooth_rdf_grad(ctypes.byref(box), _p(pts), pts.shape[0], bins, float(r_max),
                                  float(sigma), _p(gh), None, 0, _p(out))
    else:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        out = np.zeros((rows.shape[0], 3), np.float64)
        lib().orc_smooth_rdf_grad(ctypes.byref(box), _p(pts), pts.shape[0], bins, float(r_max),
                                  float(sigma), _p(gh), _p(rows), rows.shape[0], _p(out))
    return out


# ---------------------------------------------------------------------------
# Normalisation (closed forms, FP64).  The paper relates g(r) to the PMF by
# g = exp(-beta F) (PMFT section) and computes the PMFT as minus the log of
# the accumulated histogram; it states no normalisation, so these follow the
# usual ideal-gas one.
# ---------------------------------------------------------------------------

def wigner3j(j1: int, j2: int, j3: int, m1: int, m2: int, m3: int) -> float:
    """Wigner 3j symbol by the Racah formula, in exact rational arithmetic
    (integer j and m only)."""
    from fractions import Fraction
    from math import factorial as F, isqrt
    if m1 + m2 + m3 != 0 or abs(m1) > j1 or abs(m2) > j2 or abs(m3) > j3:
        return 0.0
    if j3 < abs(j1 - j2) or j3 > j1 + j2:
        return 0.0
    tri = Fraction(F(j1 + j2 - j3) * F(j1 - j2 + j3) * F(-j1 + j2 + j3), F(j1 + j2 + j3 + 1))
    pre = tri * F(j1 + m1) * F(j1 - m1) * F(j2 + m2) * F(j2 - m2) * F(j3 + m3) * F(j3 - m3)
    total = Fraction(0)
    for k in range(0, j1 + j2 + j3 + 1):
        args = (k, j3 - j2 + k + m1, j3 - j1 + k - m2, j1 + j2 - j3 - k, j1 - k - m1, j2 - k + m2)
        if min(args) < 0:
            continue
        den = 1
        for a in args:
            den *= F(a)
        total += Fraction((-1) ** k, den)
    sign = -1.0 if (j1 - j2 - m3) % 2 else 1.0
    return sign * math.sqrt(float(pre)) * float(total)


def steinhardt(box: Box, points, offsets, point_idx, l: int, query_points=None):
    """Steinhardt order parameters of each query row of a NeighborList (the
    paper's order-parameter features and its Q6 example on 12-neighbour
    lists; definitions after Steinhardt, Nelson and Ronchetti): with bonds
    d = minimum image of p_j - q_i (bonds of length 0 skipped) and Y_lm from
    scipy,
        q_lm(i) = mean over bonds of Y_lm(d),
        Q_l(i) = sqrt(4 pi / (2l + 1) * sum_m |q_lm|^2),
        W_l(i) = sum_{m1+m2+m3=0} (l l l; m1 m2 m3) q_lm1 q_lm2 q_lm3
                 / (sum_m |q_lm|^2)^(3/2)   (the normalised W-hat).
    Rows without bonds give 0.  Returns (Q_l, W_l) float64 [nq]."""
    from scipy.special import sph_harm_y
    pts = np.asarray(points, np.float32).astype(np.float64)
    q = pts if query_points is None else np.asarray(query_points, np.float32).astype(np.float64)
    off = np.asarray(offsets, np.int64)
    idx = np.asarray(point_idx, np.int64)[: off[-1]]
    nq = off.shape[0] - 1
    rows = np.repeat(np.arange(nq), np.diff(off))
    d = pts[idx] - q[rows]
    if box.dim == 2:
        d[:, 2] = 0.0
    d = np.ascontiguousarray(d)
    lib().orc_minimum_image(ctypes.byref(box), _p(d), d.shape[0])
    r = np.sqrt((d ** 2).sum(1))
    keep = r > 0
    rows, d, r = rows[keep], d[keep], r[keep]
    theta = np.arccos(np.clip(d[:, 2] / r, -1.0, 1.0))
    phi = np.arctan2(d[:, 1], d[:, 0])
    nb = np.bincount(rows, minlength=nq).astype(np.float64)
    qlm = np.zeros((nq, 2 * l + 1), np.complex128)
    for m in range(-l, l + 1):
        Y = sph_harm_y(l, m, theta, phi)
        qlm[:, m + l] = np.bincount(rows, weights=Y.real, minlength=nq) + \
            1j * np.bincount(rows, weights=Y.imag, minlength=nq)
    has = nb > 0
    qlm[has] /= nb[has, None]
    s2 = (np.abs(qlm) ** 2).sum(1)
    Q = np.sqrt(4 * math.pi / (2 * l + 1) * s2)
    W = np.zeros(nq, np.complex128)
    for m1 in range(-l, l + 1):
        for m2 in range(-l, l + 1):
            m3 = -m1 - m2
            if abs(m3) > l:
                continue
            w = wigner3j(l, l, l, m1, m2, m3)
            if w != 0.0:
                W += w * qlm[:, m1 + l] * qlm[:, m2 + l] * qlm[:, m3 + l]
    with np.errstate(invalid="ignore", divide="ignore"):
        Wh = np.where(s2 > 0, W.real / np.maximum(s2, 1e-300) ** 1.5, 0.0)
    return np.where(has, Q, 0.0), np.where(has, Wh, 0.0)


def clusters(n: int, offsets, point_idx):
    """Clusters of the cluster module (Analysis Modules: membership defined by
    neighbour bonds): connected components of the undirected graph on n
    points whose edges are the pairs (i, point_idx[e]) of every row i of the
    list.  Returns (labels, cluster_idx, sizes): labels[i] = smallest point
    index of i's component; cluster_idx[i] numbers the components in order
    of their smallest index; sizes[c] = points in component c."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import connected_components
    off = np.asarray(offsets, np.int64)
    idx = np.asarray(point_idx, np.int64)[: off[-1]]
    rows = np.repeat(np.arange(off.shape[0] - 1), np.diff(off))
    g = csr_matrix((np.ones(idx.shape[0]), (rows, idx)), shape=(n, n))
    nc, comp = connected_components(g, directed=True, connection="weak")
    first = np.full(nc, n, np.int64)
    np.minimum.at(first, comp, np.arange(n))
    labels = first[comp]
    order = np.argsort(first)               # components by smallest member
    rank = np.empty(nc, np.int64)
    rank[order] = np.arange(nc)
    cidx = rank[comp]
    sizes = np.bincount(cidx, minlength=nc)
    return labels.astype(np.int64), cidx.astype(np.int64), sizes.astype(np.int64)


def box_volume(L, dim=3):
    L = np.broadcast_to(np.asarray(L, np.float64), (3,))
    return float(L[0] * L[1] * (L[2] if dim == 3 else 1.0))


def shell_volumes(bins: int, r_min: float, r_max: float, dim: int = 3):
    e = r_min + np.arange(bins + 1, dtype=np.float64) * ((r_max - r_min) / bins)
    if dim == 3:
        return 4.0 / 3.0 * math.pi * (e[1:] ** 3 - e[:-1] ** 3)
    return math.pi * (e[1:] ** 2 - e[:-1] ** 2)


def rdf_normalize(counts, n_points, n_query, volume, r_min, r_max, dim=3, n_frames=1):
    """g_b = h_b / (N_q * rho * dV_b), rho = N_p / V, summed frames in the denominator."""
    counts = np.asarray(counts, np.float64)
    dv = shell_volumes(counts.shape[-1], r_min, r_max, dim)
    rho = n_points / volume
    return counts / (n_frames * n_query * rho * dv)


def pmf_from_rdf(g):
    """beta F(r) = -ln g(r); +inf where g = 0 (PMFT section's PMF relation)."""
    g = np.asarray(g, np.float64)
    with np.errstate(divide="ignore"):
        return -np.log(g)


def pmft2d_from_counts(counts, n_points, n_query, area, x_max, y_max, n_frames=1):
    """beta F(x, y) = -ln(counts / (N_q * rho * dx * dy * frames)); +inf at 0."""
    counts = np.asarray(counts, np.float64)
    nbx, nby = counts.shape
    dxdy = (2 * x_max / nbx) * (2 * y_max / nby)
    pcf = counts / (n_frames * n_query * (n_points / area) * dxdy)
    with np.errstate(divide="ignore"):
        return -np.log(pcf)


def pmft_xyt_from_counts(counts, n_points, n_query, area, x_max, y_max, n_frames=1):
    """beta F(x, y, t) = -ln(counts / (N_q rho dx dy (dt / 2 pi) frames)): the
    relative orientation is weighted by its share of the full turn, so an
    ideal gas gives F = 0; +inf at 0."""
    counts = np.asarray(counts, np.float64)
    nbx, nby, nbt = counts.shape
    w = (2 * x_max / nbx) * (2 * y_max / nby) / nbt
    pcf = counts / (n_frames * n_query * (n_points / area) * w)
    with np.errstate(divide="ignore"):
        return -np.log(pcf)


def pmft_xyz_from_counts(counts, n_points, n_query, volume, x_max, y_max, z_max, n_frames=1):
    """beta F(x, y, z) = -ln(counts / (N_q rho dx dy dz frames)); +inf at 0."""
    counts = np.asarray(counts, np.float64)
    nbx, nby, nbz = counts.shape
    w = (2 * x_max / nbx) * (2 * y_max / nby) * (2 * z_max / nbz)
    pcf = counts / (n_frames * n_query * (n_points / volume) * w)
    with np.errstate(divide="ignore"):
        return -np.log(pcf)


def smooth_rdf_g(h, n_points, volume, r_max):
    """g_b = h_b / (N * rho * dV_b) on bins of [0, r_max)."""
    return rdf_normalize(h, n_points, n_points, volume, 0.0, r_max, 3)
