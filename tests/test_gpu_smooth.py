"""GPU parity: Gaussian-smoothed RDF forward and its adjoint.

Forward against the oracle's FP64 h; adjoint against the oracle's FP64
gradient for the same dL/dh and against Richardson-extrapolated central
differences of the FP64 oracle loss.  Tolerance for the float32 gradient:
relative error below 1e-4, both as ||gpu - ref||_2 / ||ref||_2 and as
max |gpu - ref| / max |ref| over the compared rows.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1906_06317_amd import workloads

pytestmark = pytest.mark.gpu

BINS, R_MAX, SIGMA = 200, 3.0, 0.02
GRAD_TOL = 1e-4


@pytest.fixture(scope="module")
def ppa():
    import torch
    assert torch.cuda.is_available(), "a GPU is required"
    import paper_1906_06317_amd as m
    m.lib()
    return m


def _obox(s):
    return oracle.make_box(s.L, s.tilt, s.dim)


def _box(s):
    import paper_1906_06317_amd as m
    return m.Box(s.L, s.tilt, s.dim)


def _volume(s):
    return oracle.box_volume(s.L, s.dim)


def _check_h(h_gpu, h_ref):
    err = np.abs(h_gpu - h_ref)
    assert np.all(err <= 2e-6 * np.abs(h_ref) + 1e-9 * np.abs(h_ref).max()), (
        f"max rel err {np.max(err / np.maximum(np.abs(h_ref), 1e-300))}")


def _check_grad(g_gpu, g_ref):
    d = g_gpu.astype(np.float64) - g_ref
    rel2 = np.linalg.norm(d) / np.linalg.norm(g_ref)
    relmax = np.abs(d).max() / np.abs(g_ref).max()
    assert rel2 < GRAD_TOL and relmax < GRAD_TOL, (rel2, relmax)
    return rel2, relmax


def _target_and_gh(s, tgt, h):
    n, V = s.points.shape[0], _volume(s)
    scale = 1.0 / (n * (n / V) * oracle.shell_volumes(BINS, 0.0, R_MAX))
    t = oracle.smooth_rdf_g(oracle.smooth_rdf_h(_obox(tgt), tgt.points, BINS, R_MAX, SIGMA), n, V,
                            R_MAX)
    return t, scale, 2.0 * (h * scale - t) * scale


@pytest.mark.parametrize("tilt", [(0.0, 0.0, 0.0), (0.3, -0.2, 0.1)])
def test_forward_small(ppa, tilt):
    s = workloads.uniform(3000, 0.9, seed=71, tilt=tilt)
    h = ppa.smooth_rdf_h(_box(s), s.points, BINS, R_MAX, SIGMA).cpu().numpy()
    _check_h(h, oracle.smooth_rdf_h(_obox(s), s.points, BINS, R_MAX, SIGMA))


def test_forward_accumulates_and_counts_pairs(ppa):
    s = workloads.uniform(2000, 0.9, seed=72)
    box = _box(s)
    h = ppa.smooth_rdf_h(box, s.points, BINS, R_MAX, SIGMA)
    first = h.cpu().numpy().copy()
    ppa.smooth_rdf_h(box, s.points, BINS, R_MAX, SIGMA, h=h)
    np.testing.assert_allclose(h.cpu().numpy(), 2 * first, rtol=1e-12)
    # each pair well inside [8 sigma, r_max - 8 sigma] carries mass 1 (sum rule)
    nl = ppa.query_ball(box, s.points, R_MAX - 8 * SIGMA - 0.05)
    inner = int(nl.n_pairs)
    assert first.sum() > inner


def test_adjoint_small_against_oracle_and_fd(ppa):
    s = workloads.uniform(1500, 0.9, seed=73, tilt=(0.1, 0.2, -0.1))
    tgt = workloads.uniform(1500, 0.9, seed=74, L=s.L, tilt=s.tilt)
    ob = _obox(s)
    h_ref = oracle.smooth_rdf_h(ob, s.points, BINS, R_MAX, SIGMA)
    t, scale, gh = _target_and_gh(s, tgt, h_ref)
    g_ref = oracle.smooth_rdf_grad(ob, s.points, BINS, R_MAX, SIGMA, gh)
    g = ppa.smooth_rdf_grad(_box(s), s.points, BINS, R_MAX, SIGMA, gh).cpu().numpy()
    _check_grad(g, g_ref)
    # central differences of the FP64 loss, Richardson-extrapolated
    rng = np.random.default_rng(5)

    def loss_at(k, pk):
        hk = h_ref - oracle.smooth_rdf_row(ob, s.points, k, s.points[k].astype(np.float64), BINS,
                                           R_MAX, SIGMA) \
            + oracle.smooth_rdf_row(ob, s.points, k, pk, BINS, R_MAX, SIGMA)
        return float(((hk * scale - t) ** 2).sum())

    for k in rng.choice(1500, 6, replace=False):
        for a in range(3):
            def cd(e):
                p = s.points[k].astype(np.float64).copy()
                p[a] += e
                lp = loss_at(k, p)
                p[a] -= 2 * e
                return (lp - loss_at(k, p)) / (2 * e)
            eps = 2e-4
            fd = (4 * cd(eps / 2) - cd(eps)) / 3
            assert abs(g[k, a] - fd) <= GRAD_TOL * np.abs(g_ref).max(), (k, a, g[k, a], fd)


def test_autograd_function(ppa):
    import torch
    s = workloads.uniform(1200, 0.9, seed=75)
    tgt = workloads.uniform(1200, 0.9, seed=76, L=s.L)
    box = _box(s)
    n, V = 1200, _volume(s)
    t = torch.as_tensor(oracle.smooth_rdf_g(oracle.smooth_rdf_h(_obox(tgt), tgt.points, BINS, R_MAX,
                                                                SIGMA), n, V, R_MAX)).cuda()
    p = torch.as_tensor(s.points).cuda().requires_grad_(True)
    g = ppa.smooth_rdf_g(ppa.smooth_rdf(p, box, BINS, R_MAX, SIGMA), box, n, R_MAX)
    loss = ((g - t) ** 2).sum()
    loss.backward()
    h_ref = oracle.smooth_rdf_h(_obox(s), s.points, BINS, R_MAX, SIGMA)
    _, _, gh = _target_and_gh(s, tgt, h_ref)
    g_ref = oracle.smooth_rdf_grad(_obox(s), s.points, BINS, R_MAX, SIGMA, gh)
    _check_grad(p.grad.cpu().numpy(), g_ref)
    np.testing.assert_allclose(p.grad.sum(0).cpu().numpy(), 0.0,
                               atol=1e-4 * float(p.grad.abs().max()) * math.sqrt(n))


def test_coincident_points_and_2d(ppa):
    s = workloads.uniform(800, 0.9, seed=77)
    pts = s.points.copy()
    pts[10] = pts[11]  # a pair at r = 0: in the forward, not in the gradient
    s = workloads.System(s.L, s.tilt, 3, pts)
    h = ppa.smooth_rdf_h(_box(s), pts, BINS, R_MAX, SIGMA).cpu().numpy()
    _check_h(h, oracle.smooth_rdf_h(_obox(s), pts, BINS, R_MAX, SIGMA))
    gh = np.random.default_rng(1).normal(size=BINS)
    g = ppa.smooth_rdf_grad(_box(s), pts, BINS, R_MAX, SIGMA, gh).cpu().numpy()
    _check_grad(g, oracle.smooth_rdf_grad(_obox(s), pts, BINS, R_MAX, SIGMA, gh))
    s2 = workloads.uniform(1500, 0.8, seed=78, dim=2, tilt=(0.2, 0, 0))
    h2 = ppa.smooth_rdf_h(_box(s2), s2.points, BINS, R_MAX, SIGMA).cpu().numpy()
    _check_h(h2, oracle.smooth_rdf_h(_obox(s2), s2.points, BINS, R_MAX, SIGMA))
    g2 = ppa.smooth_rdf_grad(_box(s2), s2.points, BINS, R_MAX, SIGMA, gh).cpu().numpy()
    _check_grad(g2[:, :2], oracle.smooth_rdf_grad(_obox(s2), s2.points, BINS, R_MAX, SIGMA, gh)[:, :2])


def test_errors(ppa):
    s = workloads.uniform(100, 0.9, seed=79)
    with pytest.raises(ppa.PPAError) as e:
        ppa.smooth_rdf_h(_box(s), s.points, 0, R_MAX, SIGMA)
    assert e.value.code == ppa.PPA_EINVAL
    with pytest.raises(ppa.PPAError) as e:
        ppa.smooth_rdf_h(_box(s), s.points, BINS, R_MAX, 0.0)
    assert e.value.code == ppa.PPA_EINVAL
    with pytest.raises(ppa.PPAError) as e:  # r_max + 8 sigma beyond half the box
        ppa.smooth_rdf_h(_box(s), s.points, BINS, 2.4, 0.02)
    assert e.value.code == ppa.PPA_ERANGE


def test_full_size_perturbed_lattice(ppa):
    """The perturbed simple-cubic system (N = 131,072, density 0.9), 200 bins
    on [0, 3), sigma 0.02; target from the uniform configuration.  Forward
    and adjoint at every bin and every particle."""
    s, tgt = workloads.smooth_target_pair()
    n = s.points.shape[0]
    box = _box(s)
    h = ppa.smooth_rdf_h(box, s.points, BINS, R_MAX, SIGMA).cpu().numpy()
    h_ref = oracle.smooth_rdf_h(_obox(s), s.points, BINS, R_MAX, SIGMA)
    _check_h(h, h_ref)
    t, scale, gh = _target_and_gh(s, tgt, h_ref)
    g = ppa.smooth_rdf_grad(box, s.points, BINS, R_MAX, SIGMA, gh).cpu().numpy()
    # every particle's gradient against the oracle's (about a minute of host
    # time); the norms are taken over all rows and over each block of 4096
    g_all = oracle.smooth_rdf_grad(_obox(s), s.points, BINS, R_MAX, SIGMA, gh)
    _check_grad(g, g_all)
    for b0 in range(0, n, 4096):
        _check_grad(g[b0:b0 + 4096], g_all[b0:b0 + 4096])
    g_ref = g_all
    # and against FP64 finite differences of the loss itself on this system:
    # moving particle k changes h only through its own pairs (both orders),
    # which smooth_rdf_row gives; Richardson-extrapolated central differences
    ob = _obox(s)

    def loss_at(k, pk):
        hk = h_ref - oracle.smooth_rdf_row(ob, s.points, k, s.points[k].astype(np.float64), BINS,
                                           R_MAX, SIGMA) \
            + oracle.smooth_rdf_row(ob, s.points, k, pk, BINS, R_MAX, SIGMA)
        return float(((hk * scale - t) ** 2).sum())

    floor = 5e-5 * np.abs(g_ref).max()
    for k in np.random.default_rng(8).choice(n, 4, replace=False):
        for a in range(3):
            def cd(e):
                p = s.points[k].astype(np.float64).copy()
                p[a] += e
                lp = loss_at(k, p)
                p[a] -= 2 * e
                return (lp - loss_at(k, p)) / (2 * e)
            eps = 2e-4
            fd = (4 * cd(eps / 2) - cd(eps)) / 3
            assert abs(g[k, a] - fd) <= GRAD_TOL * abs(fd) + floor, (k, a, g[k, a], fd)


def test_non_finite_input_is_reported(ppa):
    s = workloads.uniform(600, 0.9, seed=80)
    pts = s.points.copy()
    pts[5, 2] = np.nan
    with pytest.raises(ppa.PPAError) as e:
        ppa.smooth_rdf_h(_box(s), pts, BINS, R_MAX, SIGMA)
    assert e.value.code == ppa.PPA_ENONFINITE
    with pytest.raises(ppa.PPAError) as e:
        ppa.smooth_rdf_grad(_box(s), pts, BINS, R_MAX, SIGMA, np.ones(BINS))
    assert e.value.code == ppa.PPA_ENONFINITE
