"""Pins of the 3D oracle (Table II lattices D3Q19, D3Q27, D3V39, D3Q103;
isothermal) against what the paper and the mathematics fix:

  * Gaussian quadrature: the weights reproduce the moments of N(0, c_s^2) per
    axis up to the lattice's degree (5, 5, 7, 9) and fail beyond it (D3Q103
    with the 21-digit weights and c_s printed in Table II);
  * Hermite tensors: the oracle's recursion equals the separable products of
    NumPy's probabilists' Hermite polynomials; on the Table II basis the
    weighted Gram matrix is diagonal with the Gaussian norms prod_a e_a! c_s^2e_a
    (D3Q27: the 27 tensor products, reading), except the D3Q19 pairs of
    xxy-type tensors sharing their single index (-c_s^6: the quadrature has
    degree 5); off the basis it is not;
  * the equilibrium's first three moments; the App. C 3D forms of the
    isothermal recursion (a1_xyz, a1_xxyz);
  * mass and momentum conservation of every collision, the equilibrium as a
    fixed point, RR2 = PR2, and on D3Q27 (complete basis) PR at full order =
    BGK;
  * the shear-wave decay rate nu = c_s^2 (tau - 1/2).
"""
import itertools
import math

import numpy as np
import pytest
from numpy.polynomial import hermite_e as He

from oracle import o3d

NAMES = ["D3Q19", "D3Q27", "D3V39", "D3Q103"]
DEGREE = {"D3Q19": 5, "D3Q27": 5, "D3V39": 7, "D3Q103": 9}


@pytest.fixture(scope="module")
def lats():
    return {n: o3d.lattice(n) for n in NAMES}


def gauss_moment(k, s2):
    return 0.0 if k % 2 else s2 ** (k // 2) * float(np.prod(np.arange(k - 1, 0, -2))) if k else 1.0


@pytest.mark.parametrize("name", NAMES)
def test_lattice_counts_and_weights(lats, name):
    lat = lats[name]
    assert lat.Q == {"D3Q19": 19, "D3Q27": 27, "D3V39": 39, "D3Q103": 103}[name]
    assert lat.w.sum() == pytest.approx(1.0, abs=1e-15)
    assert len({tuple(c) for c in lat.c}) == lat.Q


@pytest.mark.parametrize("name", NAMES)
def test_quadrature_moments(lats, name):
    lat = lats[name]
    deg = DEGREE[name]
    worst_in, worst_out = 0.0, 0.0
    for a, b, c in itertools.product(range(deg + 3), repeat=3):
        if a + b + c > deg + 2:
            continue
        mono = lat.c[:, 0] ** a * lat.c[:, 1] ** b * lat.c[:, 2] ** c
        lhs = float(np.sum(lat.w * mono))
        rhs = gauss_moment(a, lat.cs2) * gauss_moment(b, lat.cs2) * gauss_moment(c, lat.cs2)
        if a + b + c <= deg:
            # relative to the size of the terms summed (|c|^9 reaches 2e4 on D3Q103)
            worst_in = max(worst_in, abs(lhs - rhs) / max(1.0, float(np.sum(lat.w * np.abs(mono)))))
        elif a % 2 == 0 and b % 2 == 0 and c % 2 == 0:
            worst_out = max(worst_out, abs(lhs - rhs))
    assert worst_in <= 1e-14
    assert worst_out > 1e-6  # the degree is sharp


def tuples(n):
    return list(itertools.product(range(3), repeat=n))


def exps(t):
    return tuple(sum(1 for a in t if a == k) for k in range(3))


def he(k, x, s2):
    # probabilists' Hermite polynomial of variance s2: s^k He_k(x / s)
    s = math.sqrt(s2)
    return s ** k * He.hermeval(x / s, [0] * k + [1])


@pytest.mark.parametrize("name", NAMES)
def test_hermite_tensors_are_separable_products(lats, name):
    lat = lats[name]
    for n in range(0, 5):
        H = o3d.hermite(lat, n)
        for b, t in enumerate(tuples(n)):
            e = exps(t)
            want = he(e[0], lat.c[:, 0], lat.cs2) * he(e[1], lat.c[:, 1], lat.cs2) * he(e[2], lat.c[:, 2], lat.cs2)
            np.testing.assert_allclose(H[:, b], want, atol=1e-12)


@pytest.mark.parametrize("name", NAMES)
def test_gram_matrix_on_the_basis(lats, name):
    lat = lats[name]
    kept, dropped = [], []
    for n in range(0, 7):
        mask = o3d.basis(lat, n)
        H = o3d.hermite(lat, n)
        for b, t in enumerate(tuples(n)):
            e = exps(t)
            entry = (e, H[:, b])
            (kept if mask[b] else dropped).append(entry)
    # distinct exponent patterns
    seen = {}
    for e, h in kept:
        seen.setdefault(e, h)
    norms = {e: math.prod(math.factorial(k) * lat.cs2 ** k for k in e) for e in seen}
    pats = list(seen)

    def expected_overlap(e1, e2):
        # D3Q19 (degree 5, no velocity with three non-zero components) keeps the
        # six xxy-type tensors of Table II; two of them sharing their single
        # index (H_xxy, H_yzz) overlap by sum w x^2 y^2 z^2 - c_s^6 = -c_s^6
        if name == "D3Q19" and sum(e1) == sum(e2) == 3 and e1 != e2:
            odd1 = [a for a in range(3) if e1[a] == 1]
            odd2 = [a for a in range(3) if e2[a] == 1]
            if odd1 == odd2:
                return -lat.cs2 ** 3
        return 0.0

    for i, e1 in enumerate(pats):
        for e2 in pats[i:]:
            g = float(np.sum(lat.w * seen[e1] * seen[e2]))
            assert g == pytest.approx(norms[e1] if e1 == e2 else expected_overlap(e1, e2), abs=1e-13)
    expected = {"D3Q19": 16, "D3Q27": 27, "D3V39": 20, "D3Q103": 35}[name]
    assert len(pats) == expected
    # every dropped tensor of rank <= 4 breaks orthonormality somewhere
    for e, h in dropped:
        if sum(e) > 4:
            continue
        norm = math.prod(math.factorial(k) * lat.cs2 ** k for k in e)
        off = max(abs(float(np.sum(lat.w * h * seen[p]))) for p in pats)
        assert abs(float(np.sum(lat.w * h * h)) - norm) > 1e-8 or off > 1e-8


@pytest.mark.parametrize("name", NAMES)
def test_equilibrium_moments(lats, name):
    lat = lats[name]
    rng = np.random.default_rng(1)
    n = 20
    rho, u = rng.uniform(0.8, 1.2, n), rng.uniform(-0.1, 0.1, (3, n))
    f = o3d.equilibrium(lat, rho, *u)
    c = lat.c.astype(float)
    np.testing.assert_allclose(f.sum(0), rho, rtol=1e-14)
    for a in range(3):
        np.testing.assert_allclose((c[:, a, None] * f).sum(0), rho * u[a], atol=1e-15)
        for b in range(3):
            want = rho * (u[a] * u[b] + (lat.cs2 if a == b else 0.0))
            np.testing.assert_allclose((c[:, a, None] * c[:, b, None] * f).sum(0), want, atol=1e-14)


def noneq_node(lat, rng):
    f = o3d.equilibrium(lat, np.array([1.05]), np.array([0.04]), np.array([-0.03]), np.array([0.02]))[:, 0]
    return f * (1 + 1e-3 * rng.uniform(-1, 1, lat.Q))


@pytest.mark.parametrize("name", NAMES)
def test_app_c_3d_recursion_forms(lats, name):
    """a1_xyz = u_x a1_yz + u_y a1_xz + u_z a1_xy and the App. C form of a1_xxyz
    (theta = 1) from the oracle's general recursion."""
    lat = lats[name]
    rng = np.random.default_rng(2)
    f = noneq_node(lat, rng)
    a1 = o3d.noneq(lat, f, o3d.RR)
    r, ux, uy, uz = (float(v[0]) for v in o3d.moments(lat, f[:, None]))
    off = lambda n: (3 ** n - 1) // 2
    idx = lambda t: off(len(t)) + sum(d * 3 ** k for k, d in enumerate(t))
    X, Y, Z = 0, 1, 2
    a = lambda *t: a1[idx(t)]
    assert a(X, Y, Z) == pytest.approx(ux * a(Y, Z) + uy * a(X, Z) + uz * a(X, Y), rel=1e-12)
    if lat.nmax < 4:
        return
    want = (2 * ux * a(X, Y, Z) + uy * a(X, X, Z) + uz * a(X, X, Y)) - ux ** 2 * a(Y, Z) \
        - 2 * ux * (uy * a(X, Z) + uz * a(X, Y)) - uy * uz * a(X, X)
    assert a(X, X, Y, Z) == pytest.approx(want, rel=1e-12)


@pytest.mark.parametrize("name", NAMES)
@pytest.mark.parametrize("coll", ["RR", "PR", "BGK"])
def test_collision_conserves_and_keeps_equilibrium(lats, name, coll):
    lat = lats[name]
    cc = {"RR": o3d.RR, "PR": o3d.PR, "BGK": o3d.BGK}[coll]
    rng = np.random.default_rng(3)
    f = np.stack([noneq_node(lat, rng) for _ in range(8)], axis=1)
    g = o3d.collide(lat, f, 0.7, coll=cc)
    c = lat.c.astype(float)
    np.testing.assert_allclose(g.sum(0), f.sum(0), rtol=1e-14)
    for a in range(3):
        np.testing.assert_allclose((c[:, a, None] * g).sum(0), (c[:, a, None] * f).sum(0), atol=1e-15)
    feq = o3d.equilibrium(lat, np.array([0.9]), np.array([0.05]), np.array([0.01]), np.array([-0.07]))
    np.testing.assert_allclose(o3d.collide(lat, feq, 0.7, coll=cc), feq, atol=1e-15)


@pytest.mark.parametrize("name", NAMES)
def test_rr2_is_pr2(lats, name):
    lat = lats[name]
    rng = np.random.default_rng(4)
    f = np.stack([noneq_node(lat, rng) for _ in range(5)], axis=1)
    np.testing.assert_allclose(o3d.collide(lat, f, 0.8, o3d.RR, 2), o3d.collide(lat, f, 0.8, o3d.PR, 2), atol=1e-15)
    if lat.nmax > 2:
        assert np.abs(o3d.collide(lat, f, 0.8, o3d.RR) - o3d.collide(lat, f, 0.8, o3d.PR)).max() > 1e-9


def test_d3q27_full_pr_is_bgk(lats):
    lat = lats["D3Q27"]
    rng = np.random.default_rng(5)
    f = np.stack([noneq_node(lat, rng) for _ in range(5)], axis=1)
    np.testing.assert_allclose(o3d.collide(lat, f, 0.8, o3d.PR, 6), o3d.collide(lat, f, 0.8, o3d.BGK), atol=1e-15)


@pytest.mark.parametrize("name", NAMES)
def test_shear_wave_decay_3d(lats, name):
    lat = lats[name]
    nz, ny, nx, tau = 2, 48, 2, 0.8
    U = 1e-4 * math.sqrt(lat.cs2)
    y = (np.arange(ny) + 0.5) / ny
    ux = np.broadcast_to((U * np.sin(2 * np.pi * y))[None, :, None], (nz, ny, nx)).copy()
    z = np.zeros((nz, ny, nx))
    f = o3d.equilibrium(lat, np.ones((nz, ny, nx)), ux, z, z)
    k = 2 * np.pi / ny
    nu = lat.cs2 * (tau - 0.5)

    def amp(ff):
        _, vx, _, _ = o3d.moments(lat, ff)
        return 2.0 / ny * float(np.sum(vx[0, :, 0] * np.sin(2 * np.pi * y)))

    f = o3d.step(lat, f, tau, 20)
    a1 = amp(f)
    f = o3d.step(lat, f, tau, 300)
    a2 = amp(f)
    assert math.log(a1 / a2) / (300 * k * k) == pytest.approx(nu, rel=0.01)


# ---------------------------------------------------------- per-order relaxation

@pytest.mark.parametrize("name", NAMES)
def test_mrt_with_equal_times_is_the_single_time_operator(lats, name):
    lat = lats[name]
    rng = np.random.default_rng(8)
    f = np.stack([noneq_node(lat, rng) for _ in range(6)], axis=1)
    for coll in (o3d.RR, o3d.PR):
        np.testing.assert_array_equal(o3d.collide(lat, f, 0.7, coll, tau3=0.7, tau4=0.7), o3d.collide(lat, f, 0.7, coll))


@pytest.mark.parametrize("name", ["D3Q27", "D3V39", "D3Q103"])
@pytest.mark.parametrize("coll", ["RR", "PR"])
def test_mrt_relaxes_each_rank_with_its_own_time(lats, name, coll):
    """On a lattice whose Gram matrix is diagonal on its basis, the projection
    of f' - f^eq onto a basis tensor of rank n is k_n a1 of that tensor, with
    k_2 = 1 - 1/tau, k_3 = 1 - 1/tau3 and k_n = 1 - 1/tau4 for n >= 4."""
    lat = lats[name]
    cc = {"RR": o3d.RR, "PR": o3d.PR}[coll]
    tau, tau3, tau4 = 0.8, 0.62, 1.3
    rng = np.random.default_rng(9)
    f = noneq_node(lat, rng)
    fp = o3d.collide(lat, f[:, None], tau, cc, tau3=tau3, tau4=tau4)[:, 0]
    r, ux, uy, uz = o3d.moments(lat, f[:, None])
    feq = o3d.equilibrium(lat, r, ux, uy, uz)[:, 0]
    a1 = o3d.noneq(lat, f, cc)
    k = {2: 1 - 1 / tau, 3: 1 - 1 / tau3}
    checked = 0
    for n in range(2, lat.nmax + 1):
        H = o3d.hermite(lat, n)
        mask = o3d.basis(lat, n)
        kn = k.get(n, 1 - 1 / tau4)
        off = (3 ** n - 1) // 2
        for b in np.flatnonzero(mask):
            got = float(H[:, b] @ (fp - feq))
            assert got == pytest.approx(kn * a1[off + b], rel=1e-9, abs=1e-15)
            checked += 1
    assert checked >= {"D3Q27": 22, "D3V39": 16, "D3Q103": 30}[name] - 4


def test_mrt_shear_wave_viscosity_is_set_by_tau_alone(lats):
    lat = lats["D3V39"]
    nz, ny, nx, tau = 2, 48, 2, 0.8
    U = 1e-4 * math.sqrt(lat.cs2)
    y = (np.arange(ny) + 0.5) / ny
    ux = np.broadcast_to((U * np.sin(2 * np.pi * y))[None, :, None], (nz, ny, nx)).copy()
    z = np.zeros((nz, ny, nx))
    f = o3d.equilibrium(lat, np.ones((nz, ny, nx)), ux, z, z)
    k = 2 * np.pi / ny

    def amp(ff):
        _, vx, _, _ = o3d.moments(lat, ff)
        return 2.0 / ny * float(np.sum(vx[0, :, 0] * np.sin(2 * np.pi * y)))

    f = o3d.step(lat, f, tau, 20, tau3=0.55, tau4=1.4)
    a1 = amp(f)
    f = o3d.step(lat, f, tau, 300, tau3=0.55, tau4=1.4)
    a2 = amp(f)
    assert math.log(a1 / a2) / (300 * k * k) == pytest.approx(lat.cs2 * (tau - 0.5), rel=0.01)
