"""Pins for the oracle's Gaussian-smoothed RDF and its gradient (CPU only)."""
import math

import numpy as np
import pytest

from paper_1906_06317_amd import workloads
from tests import brute

BINS, R_MAX, SIGMA = 200, 3.0, 0.02


def test_sum_rule_single_pair(orc):
    """One pair at r inside [8 sigma + dr, r_max - 8 sigma - dr] carries total
    mass sum_b h_b = 2 (two ordered pairs) up to the aliasing error
    2 exp(-2 pi^2 sigma^2 / dr^2) of the periodic Gaussian sum (Poisson
    summation), here below 1e-14."""
    box = orc.make_box((20.0, 20.0, 20.0))
    dr = R_MAX / BINS
    for r in np.linspace(0.2, 2.8, 37):
        pts = np.array([[0, 0, 0], [r, 0, 0]], np.float32)
        h = orc.smooth_rdf_h(box, pts, BINS, R_MAX, SIGMA)
        assert abs(h.sum() - 2.0) < 1e-12
        # the mean of the smoothed distribution is the pair distance
        c = (np.arange(BINS) + 0.5) * dr
        assert abs((h * c).sum() / h.sum() - float(np.float32(r))) < 1e-12


def test_forward_matches_numpy_brute(orc):
    rng = np.random.default_rng(61)
    L, tilt = (7.0, 7.5, 8.0), (0.2, -0.1, 0.1)
    n = 60
    pts = (rng.uniform(-0.5, 0.5, (n, 3)) @ workloads.lattice_vectors(L, tilt).T).astype(np.float32)
    box = orc.make_box(L, tilt)
    h = orc.smooth_rdf_h(box, pts, BINS, R_MAX, SIGMA)
    v = brute.pair_vectors(pts, L, tilt)
    R = np.sqrt((v ** 2).sum(-1))[~np.eye(n, dtype=bool)]
    R = R[R < R_MAX + 8 * SIGMA]
    dr = R_MAX / BINS
    c = (np.arange(BINS) + 0.5) * dr
    u = c[None, :] - R[:, None]
    phi = np.exp(-u ** 2 / (2 * SIGMA ** 2)) / (SIGMA * math.sqrt(2 * math.pi))
    phi[np.abs(u) > 8 * SIGMA] = 0.0
    np.testing.assert_allclose(h, dr * phi.sum(0), rtol=1e-12, atol=1e-13)


def _loss_and_gh(orc, box, pts, target, n, V):
    h = orc.smooth_rdf_h(box, pts, BINS, R_MAX, SIGMA)
    scale = 1.0 / (n * (n / V) * orc.shell_volumes(BINS, 0.0, R_MAX))
    g = h * scale
    return float(((g - target) ** 2).sum()), 2.0 * (g - target) * scale, h, scale


def test_gradient_matches_richardson_fd(orc):
    """Analytic gradient against a Richardson-extrapolated central difference
    of the FP64 forward, for every coordinate of a small system; plus
    translation invariance (the gradients sum to zero)."""
    rng = np.random.default_rng(62)
    L = (6.0, 6.0, 6.0)
    n = 40
    pts = rng.uniform(-3, 3, (n, 3)).astype(np.float32)
    box = orc.make_box(L)
    V = 216.0
    tgt = orc.smooth_rdf_g(orc.smooth_rdf_h(box, rng.uniform(-3, 3, (n, 3)).astype(np.float32),
                                            BINS, R_MAX, SIGMA), n, V, R_MAX)
    L0, gh, h0, scale = _loss_and_gh(orc, box, pts, tgt, n, V)
    grad = orc.smooth_rdf_grad(box, pts, BINS, R_MAX, SIGMA, gh)
    np.testing.assert_allclose(grad.sum(0), 0.0, atol=1e-9 * np.abs(grad).max())

    def loss_at(k, pk):
        hk = h0 - orc.smooth_rdf_row(box, pts, k, pts[k].astype(np.float64), BINS, R_MAX, SIGMA) \
            + orc.smooth_rdf_row(box, pts, k, pk, BINS, R_MAX, SIGMA)
        return float(((hk * scale - tgt) ** 2).sum())

    fd = np.zeros_like(grad)
    for k in range(n):
        for a in range(3):
            def cd(e):
                p = pts[k].astype(np.float64).copy()
                p[a] += e
                fp = loss_at(k, p)
                p[a] -= 2 * e
                return (fp - loss_at(k, p)) / (2 * e)
            e = 2e-4
            fd[k, a] = (4 * cd(e / 2) - cd(e)) / 3
    err = np.abs(fd - grad).max() / np.abs(grad).max()
    assert err < 1e-6, err


def test_row_update_matches_full_recompute(orc):
    rng = np.random.default_rng(63)
    box = orc.make_box((6.0, 6.0, 6.0))
    pts = rng.uniform(-3, 3, (30, 3)).astype(np.float32)
    h0 = orc.smooth_rdf_h(box, pts, BINS, R_MAX, SIGMA)
    k = 7
    newp = np.array([0.25, -1.5, 2.0], np.float32)
    moved = pts.copy()
    moved[k] = newp
    h1 = orc.smooth_rdf_h(box, moved, BINS, R_MAX, SIGMA)
    upd = h0 - orc.smooth_rdf_row(box, pts, k, pts[k].astype(np.float64), BINS, R_MAX, SIGMA) \
        + orc.smooth_rdf_row(box, pts, k, newp.astype(np.float64), BINS, R_MAX, SIGMA)
    np.testing.assert_allclose(upd, h1, atol=1e-12)
