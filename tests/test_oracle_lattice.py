"""Pins of the oracle's lattice tables and Hermite tensors (Table I, App. C, App. D).

These compare the oracle with facts fixed by mathematics, not with itself:
Gauss-Hermite quadrature moments of N(0, c_s^2), Hermite orthogonality on the
basis marked in Table I, and NumPy's probabilists' Hermite polynomials.
"""
import math

import numpy as np
import pytest
from numpy.polynomial import hermite_e

QUAD_DEGREE = {"D2Q9": 5, "D2V17": 7, "D2V37": 9}
SIZES = {"D2Q9": (9, 1, 4), "D2V17": (17, 3, 3), "D2V37": (37, 3, 4)}
# Hermite tensor types (n_x, n_y) kept by each lattice (Table I, bottom; x <-> y symmetric)
BASIS = {
    "D2Q9": {(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2), (2, 1), (1, 2), (2, 2)},
    "D2V17": {(a, b) for a in range(4) for b in range(4) if a + b <= 3},
    "D2V37": {(a, b) for a in range(5) for b in range(5) if a + b <= 4},
}


def gauss_moment(a, s2):
    if a % 2:
        return 0.0
    return float(np.prod(np.arange(a - 1, 0, -2))) * s2 ** (a // 2) if a else 1.0


def pattern(kx, ky):
    """Index pattern with kx x's followed by ky y's."""
    return ((1 << ky) - 1) << kx


@pytest.mark.parametrize("name", ["D2Q9", "D2V17", "D2V37"])
def test_sizes_and_canonical_order(orc, name):
    lat = orc.lattice(name)
    Q, reach, n_eq = SIZES[name]
    assert lat.Q == Q and lat.reach == reach and lat.n_eq == n_eq
    keys = [(int(c[1]), int(c[0])) for c in lat.c]
    assert keys == sorted(keys) and len(set(keys)) == Q
    assert {(a, b) for a in range(5) for b in range(5) if lat.basis[a, b]} == BASIS[name]


@pytest.mark.parametrize("name", ["D2Q9", "D2V17", "D2V37"])
def test_quadrature_moments(orc, name):
    """sum_i w_i c_x^a c_y^b equals the moments of N(0, c_s^2 I) up to the
    lattice's quadrature degree (Eq. HermiteOrthoPreservation)."""
    lat = orc.lattice(name)
    cx, cy = lat.c[:, 0].astype(float), lat.c[:, 1].astype(float)
    deg = QUAD_DEGREE[name]
    for a in range(deg + 1):
        for b in range(deg + 1 - a):
            got = float(np.sum(lat.w * cx ** a * cy ** b))
            want = gauss_moment(a, lat.cs2) * gauss_moment(b, lat.cs2)
            assert got == pytest.approx(want, rel=1e-13, abs=1e-15), (a, b)


def test_d2q9_is_only_fifth_order(orc):
    lat = orc.lattice("D2Q9")
    cx = lat.c[:, 0].astype(float)
    assert abs(np.sum(lat.w * cx ** 6) - 15 * lat.cs2 ** 3) > 1e-3


def test_cs2_values(orc):
    assert orc.lattice("D2Q9").cs2 == pytest.approx(1.0 / 3.0, rel=1e-15)
    assert orc.lattice("D2V17").cs2 == pytest.approx(72.0 / (5 * (25 + math.sqrt(193))), rel=1e-15)
    assert orc.lattice("D2V37").cs2 == pytest.approx(1.0 / 1.19697977039307435897239 ** 2, rel=1e-15)


def scaled_he(n, v, cs2):
    """c_s^n He_n(v / c_s) with NumPy's probabilists' Hermite polynomials."""
    cs = math.sqrt(cs2)
    coef = np.zeros(n + 1)
    coef[n] = 1.0
    return cs ** n * hermite_e.hermeval(np.asarray(v, dtype=float) / cs, coef)


@pytest.mark.parametrize("name", ["D2Q9", "D2V17", "D2V37"])
def test_hermite_tensors_match_numpy(orc, name):
    """Every component of the oracle's rank-n tensors equals
    He_nx(c_x) He_ny(c_y) (scaled), whatever the index order (App. C)."""
    lat = orc.lattice(name)
    H = orc.hermite_table(lat)
    for n in range(5):
        for b in range(1 << n):
            ny = bin(b).count("1")
            want = scaled_he(n - ny, lat.c[:, 0], lat.cs2) * scaled_he(ny, lat.c[:, 1], lat.cs2)
            np.testing.assert_allclose(H[:, orc.toff(n, b)], want, rtol=0, atol=1e-12)


@pytest.mark.parametrize("name", ["D2Q9", "D2V17", "D2V37"])
def test_gram_matrix_on_basis(orc, name):
    """sum_i w_i H^k_i H^l_i = delta_kl k_x! k_y! c_s^(2|k|) on the basis
    (App. D orthogonality condition)."""
    lat = orc.lattice(name)
    H = orc.hermite_table(lat)
    types = sorted(BASIS[name])
    for k in types:
        for l in types:
            hk = H[:, orc.toff(sum(k), pattern(*k))]
            hl = H[:, orc.toff(sum(l), pattern(*l))]
            got = float(np.sum(lat.w * hk * hl))
            want = (math.factorial(k[0]) * math.factorial(k[1]) * lat.cs2 ** sum(k)) if k == l else 0.0
            assert got == pytest.approx(want, rel=1e-12, abs=1e-13), (k, l)


def test_excluded_tensors_break_orthogonality(orc):
    """The tensors marked as outside the basis in Table I are exactly those
    whose norm is not reproduced by the quadrature."""
    for name, bad in (("D2Q9", [(3, 0), (4, 0), (3, 1)]), ("D2V17", [(4, 0), (3, 1), (2, 2)])):
        lat = orc.lattice(name)
        H = orc.hermite_table(lat)
        for k in bad:
            h = H[:, orc.toff(sum(k), pattern(*k))]
            norm = float(np.sum(lat.w * h * h))
            want = math.factorial(k[0]) * math.factorial(k[1]) * lat.cs2 ** sum(k)
            assert abs(norm - want) > 1e-6 * want, (name, k)
