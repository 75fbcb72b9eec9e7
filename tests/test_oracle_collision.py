"""Pins of the oracle's equilibrium, non-equilibrium coefficients and collision.

Each test checks the oracle against something other than itself: the closed
form of the equilibrium coefficients (Eq. HermiteCoeffEq), Gauss-Hermite
integration of the Maxwellian (NumPy), the explicit 2D and 4-index forms of
App. C, the collision invariants (Eq. CollisionInvariant), the fixed point,
RR == PR at order 2 (Sec. II.F) and PR4 == BGK on D2Q9 (Secs. II.F, III.B).
"""
import itertools
import math

import numpy as np
import pytest
from numpy.polynomial import hermite_e

NAMES = ["D2Q9", "D2V17", "D2V37"]


def comp(orc, a, idx):
    """Component of a 31-slot tensor for an index tuple like 'xxy'."""
    b = sum(1 << j for j, ch in enumerate(idx) if ch == "y")
    return a[orc.toff(len(idx), b)]


def random_state(rng, thermal=False):
    rho = rng.uniform(0.7, 1.4)
    ux, uy = rng.uniform(-0.15, 0.15, size=2)
    theta = rng.uniform(0.8, 1.2) if thermal else 1.0
    return rho, ux, uy, theta


# ---------------------------------------------------------------- equilibrium

def closed_form_a0(idx, rho, u, sig):
    """Eq. HermiteCoeffEq with the symmetrised products written out."""
    ax = ["xy".index(ch) for ch in idx]
    n = len(ax)
    d = lambda a, b: 1.0 if a == b else 0.0
    if n == 0:
        return rho
    if n == 1:
        return rho * u[ax[0]]
    if n == 2:
        a, b = ax
        return rho * (u[a] * u[b] + sig * d(a, b))
    if n == 3:
        a, b, c = ax
        return rho * (u[a] * u[b] * u[c] + sig * (u[a] * d(b, c) + u[b] * d(a, c) + u[c] * d(a, b)))
    a, b, c, e = ax
    u2d = (u[a] * u[b] * d(c, e) + u[a] * u[c] * d(b, e) + u[a] * u[e] * d(b, c)
           + u[b] * u[c] * d(a, e) + u[b] * u[e] * d(a, c) + u[c] * u[e] * d(a, b))
    dd = d(a, b) * d(c, e) + d(a, c) * d(b, e) + d(a, e) * d(b, c)
    return rho * (u[a] * u[b] * u[c] * u[e] + sig * u2d + sig * sig * dd)


@pytest.mark.parametrize("name", NAMES)
def test_eq_coeffs_closed_form(orc, name):
    lat = orc.lattice(name)
    rng = np.random.default_rng(1)
    for _ in range(5):
        rho, ux, uy, th = random_state(rng, thermal=True)
        a0 = orc.eq_coeffs(lat, rho, ux, uy, th)
        sig = (th - 1.0) * lat.cs2
        for n in range(5):
            for idx in itertools.product("xy", repeat=n):
                want = closed_form_a0("".join(idx), rho, (ux, uy), sig)
                assert comp(orc, a0, idx) == pytest.approx(want, rel=1e-13, abs=1e-15)


def test_eq_coeffs_gauss_hermite_integral(orc):
    """a0^(n) = integral of H^(n) f^eq over velocity space (Eq. HermiteCoefficientDef),
    evaluated with a 40-point Gauss-Hermite rule per axis."""
    lat = orc.lattice("D2V37")
    z, wz = hermite_e.hermegauss(40)
    wz = wz / math.sqrt(2 * math.pi)
    cs = math.sqrt(lat.cs2)
    rng = np.random.default_rng(2)
    for _ in range(4):
        rho, ux, uy, th = random_state(rng, thermal=True)
        s = math.sqrt(lat.cs2 * th)
        X = ux + s * z[:, None]
        Y = uy + s * z[None, :]
        W = rho * wz[:, None] * wz[None, :]
        a0 = orc.eq_coeffs(lat, rho, ux, uy, th)
        for nx in range(5):
            for ny in range(5 - nx):
                cxn = np.zeros(nx + 1); cxn[nx] = 1
                cyn = np.zeros(ny + 1); cyn[ny] = 1
                Hx = cs ** nx * hermite_e.hermeval(X / cs, cxn)
                Hy = cs ** ny * hermite_e.hermeval(Y / cs, cyn)
                want = float(np.sum(W * Hx * Hy))
                got = comp(orc, a0, "x" * nx + "y" * ny)
                assert got == pytest.approx(want, rel=1e-11, abs=1e-13)


@pytest.mark.parametrize("name", NAMES)
def test_equilibrium_projects_back(orc, name):
    """sum_i H^k_i f^(0)_i = a0^k for every k of the lattice basis, and the
    moments of f^(0) are (rho, rho u, theta) (Eq. HermiteOrthoPreservation)."""
    lat = orc.lattice(name)
    H = orc.hermite_table(lat)
    rng = np.random.default_rng(3)
    for _ in range(5):
        thermal = name == "D2V37"
        rho, ux, uy, th = random_state(rng, thermal=thermal)
        f = orc.equilibrium(lat, np.array([rho]), np.array([ux]), np.array([uy]),
                            np.array([th]) if thermal else None)[:, 0]
        a0 = orc.eq_coeffs(lat, rho, ux, uy, th)
        for nx in range(5):
            for ny in range(5):
                if lat.basis[nx, ny]:
                    s = orc.toff(nx + ny, ((1 << ny) - 1) << nx)
                    assert float(H[:, s] @ f) == pytest.approx(a0[s], rel=1e-12, abs=1e-14)
        r, vx, vy, t = orc.moments(lat, f.reshape(-1, 1), thermal=thermal)
        assert (r[0], vx[0], vy[0]) == pytest.approx((rho, ux, uy), rel=1e-12, abs=1e-15)
        if thermal:
            assert t[0] == pytest.approx(th, rel=1e-12)


# ------------------------------------------------------- recursion algebra

def test_isothermal_recursion_matches_app_c_2d(orc):
    """Malaspinas' recursion (Eq. MalaspinasRecursiveRelation) against the 2D
    forms of App. C (Eq. a1Rec) at theta = 1 for arbitrary a1^(2)."""
    rng = np.random.default_rng(4)
    cs2 = 0.5
    for _ in range(10):
        rho, ux, uy, _ = random_state(rng)
        a0 = orc.eq_coeffs(orc.lattice("D2V37"), rho, ux, uy, 1.0)
        xx, xy, yy = rng.normal(size=3) * 1e-3
        a1 = np.zeros(31)
        for idx, v in (("xx", xx), ("xy", xy), ("yx", xy), ("yy", yy)):
            a1[orc.toff(2, sum(1 << j for j, ch in enumerate(idx) if ch == "y"))] = v
        out = orc.recursion(False, rho, ux, uy, 1.0, cs2, a0, a1)
        xxx = 3 * ux * xx
        xxy = 2 * ux * xy + uy * xx
        xyy = 2 * uy * xy + ux * yy
        yyy = 3 * uy * yy
        want = {
            "xxx": xxx, "xxy": xxy, "xyy": xyy, "yyy": yyy,
            "xxxx": 4 * ux * xxx - 6 * ux ** 2 * xx,
            "xxxy": 3 * ux * xxy + uy * xxx - 3 * ux ** 2 * xy - 3 * ux * uy * xx,
            "xxyy": 2 * (ux * xyy + uy * xxy) - ux ** 2 * yy - uy ** 2 * xx - 4 * ux * uy * xy,
        }
        for idx, v in want.items():
            for perm in set(itertools.permutations(idx)):
                assert comp(orc, out, perm) == pytest.approx(v, rel=1e-12, abs=1e-18), (idx, perm)
        swapped = {"yyyy": 4 * uy * yyy - 6 * uy ** 2 * yy,
                   "yyyx": 3 * uy * xyy + ux * yyy - 3 * uy ** 2 * xy - 3 * ux * uy * yy}
        for idx, v in swapped.items():
            for perm in set(itertools.permutations(idx)):
                assert comp(orc, out, perm) == pytest.approx(v, rel=1e-12, abs=1e-18)


def test_thermal_recursion_matches_four_index_form(orc):
    """The thermal recursion with a distinguished last index (Eq.
    RecursiveRelation_ThermalCase) against the symmetric 4-index form of App. C,
    for arbitrary symmetric a1^(2), a1^(3) and theta != 1; the result is a
    symmetric tensor."""
    rng = np.random.default_rng(5)
    cs2 = 1.0 / 1.19697977039307435897239 ** 2
    d = lambda a, b: 1.0 if a == b else 0.0
    for _ in range(10):
        rho, ux, uy, th = random_state(rng, thermal=True)
        u = (ux, uy)
        a0 = orc.eq_coeffs(orc.lattice("D2V37"), rho, ux, uy, th)
        s2 = rng.normal(size=3) * 1e-3
        A2 = np.array([[s2[0], s2[1]], [s2[1], s2[2]]])
        t3 = rng.normal(size=4) * 1e-3  # xxx, xxy, xyy, yyy
        A3 = np.zeros((2, 2, 2))
        for i, j, k in itertools.product(range(2), repeat=3):
            A3[i, j, k] = t3[i + j + k]
        a1 = np.zeros(31)
        for i, j in itertools.product(range(2), repeat=2):
            a1[orc.toff(2, i | j << 1)] = A2[i, j]
        for i, j, k in itertools.product(range(2), repeat=3):
            a1[orc.toff(3, i | j << 1 | k << 2)] = A3[i, j, k]
        out = orc.recursion(True, rho, ux, uy, th, cs2, a0, a1)
        sig = cs2 * (th - 1)
        for a, b, c, e in itertools.product(range(2), repeat=4):
            want = (u[a] * A3[b, c, e] + u[b] * A3[a, c, e] + u[c] * A3[a, b, e] + u[e] * A3[a, b, c]
                    + (sig * d(a, b) - u[a] * u[b]) * A2[c, e]
                    + (sig * d(a, c) - u[a] * u[c]) * A2[b, e]
                    + (sig * d(a, e) - u[a] * u[e]) * A2[b, c]
                    + (sig * d(b, c) - u[b] * u[c]) * A2[a, e]
                    + (sig * d(b, e) - u[b] * u[e]) * A2[a, c]
                    + (sig * d(c, e) - u[c] * u[e]) * A2[a, b])
            got = out[orc.toff(4, a | b << 1 | c << 2 | e << 3)]
            assert got == pytest.approx(want, rel=1e-11, abs=1e-17)


def test_ce_forms_reproduce_ce_a14(orc):
    """Chapman-Enskog a1^(2), a1^(3) built from velocity and temperature
    gradients (App. A) fed through the recursion give the CE a1^(4) of App. C,
    here checked on xxxx through the 2D form with mu c_s^2 d(theta)."""
    rng = np.random.default_rng(6)
    lat = orc.lattice("D2V37")
    cs2 = lat.cs2
    for _ in range(5):
        rho, ux, uy, th = random_state(rng, thermal=True)
        a0 = orc.eq_coeffs(lat, rho, ux, uy, th)
        G = rng.normal(size=(2, 2)) * 1e-3  # velocity gradient d_a u_b
        gth = rng.normal(size=2) * 1e-3      # temperature gradient
        tau = 0.8
        div = G[0, 0] + G[1, 1]
        A2 = np.array([[-tau * rho * cs2 * th * (G[a, b] + G[b, a] - (a == b) * div) for b in range(2)]
                       for a in range(2)])
        mu = rho * cs2 * th * tau
        d = lambda a, b: 1.0 if a == b else 0.0
        u = (ux, uy)
        A3 = np.zeros((2, 2, 2))
        for a, b, c in itertools.product(range(2), repeat=3):
            A3[a, b, c] = (u[a] * A2[b, c] + u[b] * A2[a, c] + u[c] * A2[a, b]
                           - mu * cs2 * (d(a, b) * gth[c] + d(a, c) * gth[b] + d(b, c) * gth[a]))
        a1 = np.zeros(31)
        for a, b in itertools.product(range(2), repeat=2):
            a1[orc.toff(2, a | b << 1)] = A2[a, b]
        for a, b, c in itertools.product(range(2), repeat=3):
            a1[orc.toff(3, a | b << 1 | c << 2)] = A3[a, b, c]
        out = orc.recursion(True, rho, ux, uy, th, cs2, a0, a1)
        want = 4 * ux * A3[0, 0, 0] + 6 * (cs2 * (th - 1) - ux ** 2) * A2[0, 0]
        assert out[orc.toff(4, 0)] == pytest.approx(want, rel=1e-11)


# ------------------------------------------------------------ collision

def perturbed(orc, lat, rng, n=16, thermal=False, amp=1e-3):
    rho = rng.uniform(0.8, 1.2, n)
    ux = rng.uniform(-0.1, 0.1, n)
    uy = rng.uniform(-0.1, 0.1, n)
    th = rng.uniform(0.85, 1.15, n) if thermal else None
    f = orc.equilibrium(lat, rho, ux, uy, th)
    return f * (1.0 + amp * rng.uniform(-1, 1, f.shape))


MODES = [(orc_coll, order) for orc_coll in (0, 1) for order in (2, 3, 4)] + [(2, 2)]


@pytest.mark.parametrize("name", NAMES)
@pytest.mark.parametrize("coll,order", MODES)
@pytest.mark.parametrize("thermal", [False, True])
def test_collision_invariants(orc, name, coll, order, thermal):
    """Mass and momentum (and energy, thermal) are conserved by the collision
    for arbitrary pre-collision populations (Eq. CollisionInvariant)."""
    lat = orc.lattice(name)
    if order > lat.n_eq or (thermal and name != "D2V37"):
        pytest.skip("order not supported by this lattice")
    rng = np.random.default_rng(7)
    f = perturbed(orc, lat, rng, thermal=thermal)
    out = orc.collide(lat, f, 0.6, coll=coll, order=order, thermal=thermal)
    c = lat.c.astype(float)
    for g, h in ((f, out),):
        np.testing.assert_allclose(h.sum(0), g.sum(0), rtol=1e-14)
        np.testing.assert_allclose(c[:, 0] @ h, c[:, 0] @ g, rtol=0, atol=1e-15)
        np.testing.assert_allclose(c[:, 1] @ h, c[:, 1] @ g, rtol=0, atol=1e-15)
        if thermal:
            e = (c ** 2).sum(1)
            np.testing.assert_allclose(e @ h, e @ g, rtol=1e-14)


@pytest.mark.parametrize("name", NAMES)
@pytest.mark.parametrize("coll", [0, 1, 2])
def test_equilibrium_is_fixed_point(orc, name, coll):
    lat = orc.lattice(name)
    rng = np.random.default_rng(8)
    thermal = name == "D2V37"
    rho = rng.uniform(0.8, 1.2, 8)
    ux, uy = rng.uniform(-0.1, 0.1, (2, 8))
    th = rng.uniform(0.9, 1.1, 8) if thermal else None
    f = orc.equilibrium(lat, rho, ux, uy, th)
    out = orc.collide(lat, f, 0.55, coll=coll, thermal=thermal)
    np.testing.assert_allclose(out, f, rtol=1e-13, atol=1e-16)


@pytest.mark.parametrize("name", NAMES)
@pytest.mark.parametrize("thermal", [False, True])
def test_rr2_equals_pr2(orc, name, thermal):
    lat = orc.lattice(name)
    if thermal and name != "D2V37":
        pytest.skip("thermal only on D2V37")
    rng = np.random.default_rng(9)
    f = perturbed(orc, lat, rng, thermal=thermal)
    rr = orc.collide(lat, f, 0.7, coll=0, order=2, thermal=thermal)
    pr = orc.collide(lat, f, 0.7, coll=1, order=2, thermal=thermal)
    np.testing.assert_allclose(rr, pr, rtol=0, atol=1e-15)


def test_pr4_equals_bgk_on_d2q9(orc):
    """The D2Q9 basis is complete, so projecting f - f^(0) on all of it
    changes nothing and PR at order 4 is BGK."""
    lat = orc.lattice("D2Q9")
    rng = np.random.default_rng(10)
    f = perturbed(orc, lat, rng, amp=1e-2)
    for tau in (0.51, 0.8, 1.7):
        pr = orc.collide(lat, f, tau, coll=1, order=4)
        bgk = orc.collide(lat, f, tau, coll=2)
        np.testing.assert_allclose(pr, bgk, rtol=0, atol=1e-15)
    rr = orc.collide(lat, f, 0.8, coll=0, order=4)
    assert np.abs(rr - orc.collide(lat, f, 0.8, coll=2)).max() > 1e-6


def test_pr_differs_from_bgk_on_high_order_lattices(orc):
    for name in ("D2V17", "D2V37"):
        lat = orc.lattice(name)
        f = perturbed(orc, lat, np.random.default_rng(11), amp=1e-2)
        pr = orc.collide(lat, f, 0.8, coll=1, order=lat.n_eq)
        assert np.abs(pr - orc.collide(lat, f, 0.8, coll=2)).max() > 1e-7


def test_tau_one_gives_equilibrium(orc):
    """With tau = 1 every regularized collision returns f^(0) exactly."""
    for name in NAMES:
        lat = orc.lattice(name)
        f = perturbed(orc, lat, np.random.default_rng(12), amp=1e-2)
        r, ux, uy, _ = orc.moments(lat, f)
        feq = orc.equilibrium(lat, r, ux, uy)
        for coll in (0, 1, 2):
            np.testing.assert_allclose(orc.collide(lat, f, 1.0, coll=coll), feq, rtol=0, atol=1e-15)


def test_thermal_a13_rebuild_recovers_ce_structure(orc):
    """If the third-order non-equilibrium part has exactly the CE structure
    (Eq. a1Rec) with some gradient G, the App. C rebuild (project, average the
    two estimates of G, reconstruct) returns it unchanged."""
    lat = orc.lattice("D2V37")
    H = orc.hermite_table(lat)
    rng = np.random.default_rng(13)
    d = lambda a, b: 1.0 if a == b else 0.0
    for _ in range(5):
        rho, ux, uy, th = random_state(rng, thermal=True)
        u = (ux, uy)
        a0 = orc.eq_coeffs(lat, rho, ux, uy, th)
        feq = orc.equilibrium(lat, np.array([rho]), np.array([ux]), np.array([uy]), np.array([th]))[:, 0]
        s = rng.normal(size=2) * 1e-4
        A2 = np.array([[s[0], s[1]], [s[1], -s[0]]])  # traceless: theta unchanged
        G = rng.normal(size=2) * 1e-4
        A3 = np.zeros((2, 2, 2))
        for a, b, c in itertools.product(range(2), repeat=3):
            A3[a, b, c] = (u[a] * A2[b, c] + u[b] * A2[a, c] + u[c] * A2[a, b]
                           - (d(a, b) * G[c] + d(a, c) * G[b] + d(b, c) * G[a]))
        a1 = np.zeros(31)
        for a, b in itertools.product(range(2), repeat=2):
            a1[orc.toff(2, a | b << 1)] = A2[a, b]
        for a, b, c in itertools.product(range(2), repeat=3):
            a1[orc.toff(3, a | b << 1 | c << 2)] = A3[a, b, c]
        f1 = np.zeros(lat.Q)
        for n in (2, 3):
            for b in range(1 << n):
                f1 += H[:, orc.toff(n, b)] * a1[orc.toff(n, b)] / (math.factorial(n) * lat.cs2 ** n)
        f = feq + lat.w * f1
        got = orc.noneq_coeffs(lat, f, coll=0, thermal=True)
        for a, b, c in itertools.product(range(2), repeat=3):
            assert got[orc.toff(3, a | b << 1 | c << 2)] == pytest.approx(A3[a, b, c], rel=1e-8, abs=1e-15)
        for a, b in itertools.product(range(2), repeat=2):
            assert got[orc.toff(2, a | b << 1)] == pytest.approx(A2[a, b], rel=1e-8, abs=1e-15)
        assert a0[0] == rho
