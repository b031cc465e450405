"""Pins for the oracle's RDF histogram and normalisation (CPU only)."""
import math

import numpy as np
import pytest

from paper_1906_06317_amd import workloads
from tests import brute


def _np_hist(points, L, tilt, dim, bins, r_min, r_max):
    v = brute.pair_vectors(points, L, tilt, dim)
    R = np.sqrt((v ** 2).sum(-1))
    np.fill_diagonal(R, np.inf)
    R = R[np.isfinite(R)]
    h, _ = np.histogram(R[(R >= r_min) & (R < r_max)], bins=bins, range=(r_min, r_max))
    return h


@pytest.mark.parametrize("dim", [2, 3])
def test_rdf_matches_numpy_histogram(orc, dim):
    rng = np.random.default_rng(31 + dim)
    for _ in range(6):
        L = tuple(rng.uniform(5, 8, 3)) if dim == 3 else (rng.uniform(5, 8), rng.uniform(5, 8), 1.0)
        tilt = tuple(rng.uniform(-0.4, 0.4, 3)) if dim == 3 else (rng.uniform(-0.4, 0.4), 0.0, 0.0)
        n = 150
        s = rng.uniform(-0.5, 0.5, (n, 3))
        pts = (s @ workloads.lattice_vectors(L, tilt, dim).T).astype(np.float32)
        if dim == 2:
            pts[:, 2] = 0
        half = 0.5 * brute.perpendicular_widths(L, tilt, dim).min()
        r_min, r_max = 0.4, 0.9 * half
        box = orc.make_box(L, tilt, dim)
        lo, hi, amb = orc.rdf_counts(box, pts, 37, r_max, r_min)
        ref = _np_hist(pts, L, tilt, dim, 37, r_min, r_max)
        # an ambiguous pair (|r^2 - e^2| <= 1e-5 e^2) may sit on either side of e
        assert amb <= 20
        assert np.all(lo.astype(np.int64) <= ref) and np.all(ref <= hi.astype(np.int64))
        assert int((hi - lo).sum()) <= 2 * amb


def test_rdf_total_equals_ball_pairs(orc):
    s = workloads.small_uniform()
    box = orc.make_box(s.L, s.tilt)
    lo, hi, amb = orc.rdf_counts(box, s.points, 100, 3.0)
    off, idx, r2 = orc.ball_query(box, s.points, 3.0)
    certain = int(np.sum(r2 < 9.0 * (1 - 1e-5)))
    assert int(lo.sum()) <= certain <= int(hi.sum())
    assert int(hi.sum()) - int(lo.sum()) <= 2 * amb


def test_rdf_fcc_shell_counts(orc):
    """Perfect FCC: shell m sits at r^2 = m a^2 / 2 with multiplicities
    12, 6, 24, 12, 24, 8, 48, 6, 36; with bins whose edges avoid every shell,
    each shell's N * c_m pairs land in exactly one bin."""
    a = 1.0
    s = workloads.fcc(7, a)
    n = s.points.shape[0]
    box = orc.make_box(s.L, s.tilt)
    r_max = 3.0 * a * 0.5 ** 0.5 + 0.05  # covers m <= 9 (r = 3 a / sqrt 2)
    bins = 61
    lo, hi, amb = orc.rdf_counts(box, s.points, bins, r_max)
    assert amb == 0
    dr = r_max / bins
    mult = [12, 6, 24, 12, 24, 8, 48, 6, 36]
    want = np.zeros(bins, np.int64)
    for m, c in enumerate(mult, start=1):
        r = a * math.sqrt(m / 2)
        b = int(r // dr)
        assert abs(r - b * dr) > 1e-3 and abs(r - (b + 1) * dr) > 1e-3
        want[b] += n * c
    np.testing.assert_array_equal(lo.astype(np.int64), want)


def test_rdf_ideal_gas_limit(orc):
    """Uniform points: E[g_b] = (N - 1)/N with this normalisation; the mean
    over bins is checked against its binomial error and each bin's z-score
    is bounded."""
    n = 6000
    s = workloads.uniform(n, 0.8, seed=77)
    box = orc.make_box(s.L, s.tilt)
    bins, r_max = 40, 3.0
    lo, hi, amb = orc.rdf_counts(box, s.points, bins, r_max)
    V = orc.box_volume(s.L)
    g = orc.rdf_normalize(lo.astype(np.float64), n, n, V, 0.0, r_max)
    dv = orc.shell_volumes(bins, 0.0, r_max)
    expect_h = n * ((n - 1) / V) * dv
    # ordered pairs come in symmetric couples, so the variance is ~2 E[h]
    z = (lo.astype(np.float64) - expect_h) / np.sqrt(2 * expect_h)
    assert np.all(np.abs(z[5:]) < 5.0)
    w = expect_h[5:] / expect_h[5:].sum()
    assert abs(np.sum(w * g[5:]) - (n - 1) / n) < 5 * math.sqrt(2 / expect_h[5:].sum())


def test_rdf_normalisation_closed_form(orc):
    dv3 = orc.shell_volumes(3, 1.0, 4.0, 3)
    np.testing.assert_allclose(dv3, 4 / 3 * math.pi * np.array([8 - 1, 27 - 8, 64 - 27]))
    dv2 = orc.shell_volumes(2, 0.0, 2.0, 2)
    np.testing.assert_allclose(dv2, math.pi * np.array([1, 3]))
    g = orc.rdf_normalize(np.array([10.0]), 100, 50, 1000.0, 0.0, 1.0)
    np.testing.assert_allclose(g, 10.0 / (50 * 0.1 * 4 / 3 * math.pi))
    np.testing.assert_allclose(orc.pmf_from_rdf(np.array([1.0, math.e])), [0.0, -1.0])
    assert orc.pmf_from_rdf(np.array([0.0]))[0] == np.inf


def test_rdf_ambiguity_band_catches_edge_pair(orc):
    """A pair placed exactly on a bin edge is reported ambiguous and may land in
    either neighbouring bin."""
    box = orc.make_box((10.0, 10.0, 10.0))
    pts = np.array([[0, 0, 0], [1.5, 0, 0]], np.float32)  # r = 1.5 = an edge for dr = 0.5
    lo, hi, amb = orc.rdf_counts(box, pts, 6, 3.0)
    assert amb == 2
    assert lo.sum() == 0
    assert hi[2] == 2 and hi[3] == 2


def test_one_sweep_ball_rdf_rows_equal_the_separate_definitions(orc):
    """The one-sweep ball + RDF routine (used to write the full-size expected
    values) equals the ball query and the RDF computed separately, also
    when the rows are swept in pieces; and the numpy brute force pins the
    rows through image search."""
    rng = np.random.default_rng(5150)
    for trial in range(4):
        L = tuple(rng.uniform(6, 9, 3))
        tilt = tuple(rng.uniform(-0.45, 0.45, 3))
        n = 300
        s = rng.uniform(-0.5, 0.5, (n, 3))
        pts = (s @ workloads.lattice_vectors(L, tilt, 3).T).astype(np.float32)
        half = 0.5 * brute.perpendicular_widths(L, tilt, 3).min()
        r_max = 0.95 * half
        box = orc.make_box(L, tilt, 3)
        off, idx, r2 = orc.ball_query(box, pts, r_max)
        lo_ref, hi_ref, amb_ref = orc.rdf_counts(box, pts, 23, r_max)
        lo = np.zeros(23, np.uint64)
        hi = np.zeros(23, np.uint64)
        amb = np.zeros(1, np.uint64)
        cuts = [0, 77, 78, 211, n]
        for a, b in zip(cuts[:-1], cuts[1:]):
            cnt, ri, rr, lo, hi, amb = orc.ball_rdf_rows(box, pts, r_max, 23, rows=(a, b), cap=128,
                                                         lo=lo, hi=hi, n_amb=amb)
            for t, q in enumerate(range(a, b)):
                c = int(cnt[t])
                assert c == off[q + 1] - off[q]
                assert np.array_equal(ri[t, :c], idx[off[q]:off[q + 1]])
                assert np.array_equal(rr[t, :c], r2[off[q]:off[q + 1]])
                assert np.all(ri[t, c:] == -1)
        assert np.array_equal(lo, lo_ref) and np.array_equal(hi, hi_ref)
        assert int(amb[0]) == amb_ref
        # rows against the image-search brute force
        v = brute.pair_vectors(pts, L, tilt, 3)
        R2 = (v.astype(np.float64) ** 2).sum(-1)
        np.fill_diagonal(R2, np.inf)
        for q in range(0, n, 37):
            ref = np.nonzero(R2[q] < r_max ** 2 * (1 - 1e-5))[0]
            assert set(ref.tolist()) <= set(idx[off[q]:off[q + 1]].tolist())
    # a row longer than cap is reported
    with pytest.raises(ValueError):
        orc.ball_rdf_rows(box, pts, r_max, 23, cap=2)
