"""Pins for the oracle's Steinhardt order parameters and Wigner 3j symbols
(CPU only): the addition theorem, closed forms, the perfect-lattice values
tabulated by Steinhardt, Nelson and Ronchetti (the paper's reference for Q_l
and W_l), rotation invariance and 3j orthogonality."""
import itertools
import math

import numpy as np
import pytest


def _one_particle(orc, bonds, l):
    """Q_l, W_l of a particle at the origin whose neighbours sit at `bonds`."""
    bonds = np.asarray(bonds, np.float64)
    box = orc.make_box((40.0, 40.0, 40.0))
    pts = bonds.astype(np.float32)
    off = np.array([0, len(bonds)])
    Q, W = orc.steinhardt(box, pts, off, np.arange(len(bonds)), l,
                          query_points=np.zeros((1, 3), np.float32))
    return Q[0], W[0]


def _fcc_bonds():
    out = set()
    for x, y in itertools.product((-1, 1), (-1, 1)):
        out |= {(x, y, 0), (x, 0, y), (0, x, y)}
    return sorted(out)


def _hcp_bonds():
    b = [(math.cos(k * math.pi / 3), math.sin(k * math.pi / 3), 0.0) for k in range(6)]
    h = math.sqrt(2.0 / 3.0)
    r = 1.0 / math.sqrt(3.0)
    for z in (h, -h):
        b += [(r * math.cos(math.pi / 6 + k * 2 * math.pi / 3),
               r * math.sin(math.pi / 6 + k * 2 * math.pi / 3), z) for k in range(3)]
    return b


def _bcc_bonds():
    return list(itertools.product((-1, 1), (-1, 1), (-1, 1)))


def _ico_bonds():
    g = (1 + math.sqrt(5)) / 2
    out = []
    for a, b in itertools.product((-1, 1), (-g, g)):
        out += [(0, a, b), (a, b, 0), (b, 0, a)]
    return out


@pytest.mark.parametrize("l", [0, 1, 2, 4, 6, 9, 12])
def test_single_bond_addition_theorem(orc, l):
    """One bond: sum_m |Y_lm|^2 = (2l + 1) / (4 pi), so Q_l = 1; and q_lm is
    Y_lm of one direction, so W-hat is (l l l; 0 0 0) (bond along +z, where
    only m = 0 survives and Y_l0 > 0)."""
    Q, W = _one_particle(orc, [(0.3, -0.2, 0.7)], l)
    assert abs(Q - 1.0) < 1e-12
    Qz, Wz = _one_particle(orc, [(0.0, 0.0, 0.9)], l)
    assert abs(Wz - orc.wigner3j(l, l, l, 0, 0, 0)) < 1e-12
    assert abs(W - Wz) < 1e-10  # rotation invariance


def test_simple_cubic_closed_forms(orc):
    sc = [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]
    assert abs(_one_particle(orc, sc, 4)[0] - math.sqrt(7 / 12)) < 1e-12
    assert abs(_one_particle(orc, sc, 6)[0] - math.sqrt(1 / 8)) < 1e-12
    assert abs(_one_particle(orc, sc, 2)[0]) < 1e-12  # cubic symmetry kills l = 2


@pytest.mark.parametrize("name,bonds,l,Q,W", [
    ("fcc", _fcc_bonds(), 4, 0.19094, -0.15932),
    ("fcc", _fcc_bonds(), 6, 0.57452, -0.01316),
    ("hcp", _hcp_bonds(), 4, 0.09722, 0.13410),
    ("hcp", _hcp_bonds(), 6, 0.48476, -0.01244),
    ("bcc", _bcc_bonds(), 6, 0.62854, 0.01316),
    ("ico", _ico_bonds(), 6, 0.66332, -0.16975),
])
def test_tabulated_lattice_values(orc, name, bonds, l, Q, W):
    q, w = _one_particle(orc, bonds, l)
    assert abs(q - Q) < 1e-5 and abs(w - W) < 1e-5


def test_icosahedron_has_no_l4_order(orc):
    # exactly 0 by symmetry; the vertices are stored as float32 points
    assert abs(_one_particle(orc, _ico_bonds(), 4)[0]) < 1e-6


def test_rotation_invariance(orc):
    rng = np.random.default_rng(7)
    A = rng.normal(size=(3, 3))
    R, _ = np.linalg.qr(A)
    bonds = np.asarray(_hcp_bonds()) * 1.3
    for l in (3, 6, 8):
        q0, w0 = _one_particle(orc, bonds, l)
        q1, w1 = _one_particle(orc, bonds @ R.T, l)
        assert abs(q0 - q1) < 1e-6 and abs(w0 - w1) < 1e-6


def test_wigner3j_orthogonality_and_values(orc):
    assert abs(orc.wigner3j(2, 2, 2, 0, 0, 0) + math.sqrt(2 / 35)) < 1e-15
    assert orc.wigner3j(1, 1, 1, 0, 0, 0) == 0.0  # odd sum of j with all m = 0
    for l in (2, 5, 8):
        for m3 in (-l, 0, 1):
            tot = sum(orc.wigner3j(l, l, l, m1, m2, m3) ** 2
                      for m1 in range(-l, l + 1) for m2 in range(-l, l + 1))
            assert abs(tot - 1.0 / (2 * l + 1)) < 1e-12


def test_rows_without_bonds_and_minimum_image(orc):
    """A row with no bonds gives 0; bonds are minimum images (a neighbour
    across the boundary counts from the near side)."""
    box = orc.make_box((10.0, 10.0, 10.0))
    pts = np.array([[4.9, 0, 0], [-4.9, 0, 0]], np.float32)  # 0.2 apart through the wall
    off = np.array([0, 1, 1])
    Q, W = orc.steinhardt(box, pts, off, np.array([1]), 2)
    assert Q[1] == 0.0 and W[1] == 0.0
    # the bond from point 0 to point 1 is +x (0.2), not -x (9.8): Y_1m picks the sign
    Q1, _ = orc.steinhardt(box, pts, off, np.array([1]), 1)
    assert abs(Q1[0] - 1.0) < 1e-12
