"""Dynamic pins of the oracle's full step (collide + stream, Sec. III.A).

Closed forms: the shear-wave decay rate nu k^2 with nu = c_s^2 (tau - 1/2)
(Secs. II.C and III.A), the entropy-wave decay at the same rate (Pr = 1), the
advection of a density mode at the flow speed (streaming direction),
conservation over many steps, and a uniform equilibrium as a steady state.
"""
import math

import numpy as np
import pytest

from paper_1704_04413_amd import workloads


def amplitude(field, axis_len):
    y = (np.arange(axis_len) + 0.5) / axis_len
    return 2.0 / axis_len * float(np.sum(field * np.sin(2 * np.pi * y)))


@pytest.mark.parametrize("name", ["D2Q9", "D2V17", "D2V37"])
@pytest.mark.parametrize("tau", [0.52, 0.8, 1.5])
def test_shear_wave_decay(orc, name, tau):
    lat = orc.lattice(name)
    ny, nx = 64, 4
    U = 1e-4 * math.sqrt(lat.cs2)
    y = (np.arange(ny) + 0.5) / ny
    ux = np.broadcast_to((U * np.sin(2 * np.pi * y))[:, None], (ny, nx)).copy()
    f = orc.init_populations(lat, np.ones((ny, nx)), ux, np.zeros((ny, nx)))
    nu = lat.cs2 * (tau - 0.5)
    k = 2 * np.pi / ny
    t1 = 50
    t2 = t1 + int(min(2000, 0.5 / (nu * k * k)))
    f = orc.step(lat, f, tau, t1)
    a1 = amplitude(orc.moments(lat, f)[1][:, 0], ny)
    f = orc.step(lat, f, tau, t2 - t1)
    a2 = amplitude(orc.moments(lat, f)[1][:, 0], ny)
    nu_meas = math.log(a1 / a2) / ((t2 - t1) * k * k)
    assert nu_meas == pytest.approx(nu, rel=0.01)


def test_entropy_wave_decays_at_thermal_diffusivity(orc):
    """Isobaric temperature mode on D2V37 (thermal): decays at
    chi k^2 with chi = c_s^2 theta (tau - 1/2), i.e. Pr = 1."""
    lat = orc.lattice("D2V37")
    ny, nx, tau, eps = 64, 4, 0.8, 1e-4
    y = (np.arange(ny) + 0.5) / ny
    th = np.broadcast_to((1.0 + eps * np.sin(2 * np.pi * y))[:, None], (ny, nx)).copy()
    rho = 1.0 / th
    z = np.zeros((ny, nx))
    f = orc.init_populations(lat, rho, z, z, th)
    k = 2 * np.pi / ny
    chi = lat.cs2 * (tau - 0.5)
    t1, t2 = 200, 1200
    f = orc.step(lat, f, tau, t1, thermal=True)
    a1 = amplitude(orc.moments(lat, f, thermal=True)[3][:, 0] - 1.0, ny)
    f = orc.step(lat, f, tau, t2 - t1, thermal=True)
    a2 = amplitude(orc.moments(lat, f, thermal=True)[3][:, 0] - 1.0, ny)
    chi_meas = math.log(a1 / a2) / ((t2 - t1) * k * k)
    assert chi_meas == pytest.approx(chi, rel=0.03)


def test_density_mode_advects_with_the_flow(orc):
    """Streaming moves f_i along +c_i: the phase of a density Fourier mode in
    a uniform flow u turns by -k u t (the acoustic part only rescales it)."""
    lat = orc.lattice("D2Q9")
    nx, ny, u, t = 64, 4, 0.05, 10
    x = (np.arange(nx) + 0.5) / nx
    rho = np.broadcast_to(1.0 + 1e-4 * np.cos(2 * np.pi * x)[None, :], (ny, nx)).copy()
    f = orc.init_populations(lat, rho, np.full((ny, nx), u), np.zeros((ny, nx)))
    k = 2 * np.pi / nx

    def phase(ff):
        r = orc.moments(lat, ff)[0][0]
        return np.angle(np.sum((r - r.mean()) * np.exp(-1j * 2 * np.pi * x)))

    p0 = phase(f)
    p1 = phase(orc.step(lat, f, 0.8, t))
    assert (p1 - p0) == pytest.approx(-k * u * t, rel=0.05)


@pytest.mark.parametrize("name,thermal", [("D2Q9", False), ("D2V17", False), ("D2V37", False),
                                          ("D2V37", True)])
def test_conservation_over_run(orc, name, thermal):
    lat = orc.lattice(name)
    n = 32
    u0, tau = workloads.shear_layer_params(lat.cs2, n, 1e4)
    rho, ux, uy = workloads.shear_layer_fields(n, n, u0)
    th = np.ones((n, n)) if thermal else None
    noise = workloads.uniform_noise(0, lat.Q, n, n)
    f = orc.init_populations(lat, rho, ux, uy, th, noise, 1e-8, eq_order=2 if not thermal else None)
    c = lat.c.astype(float)

    def totals(ff):
        m = ff.sum()
        jx = float(np.einsum("i,iyx->", c[:, 0], ff))
        jy = float(np.einsum("i,iyx->", c[:, 1], ff))
        e = float(np.einsum("i,iyx->", (c ** 2).sum(1), ff))
        return m, jx, jy, e

    m0, jx0, jy0, e0 = totals(f)
    f = orc.step(lat, f, tau, 100, thermal=thermal)
    m1, jx1, jy1, e1 = totals(f)
    assert abs(m1 - m0) <= 1e-13 * abs(m0)
    scale = float(np.sum(np.abs(ux * rho))) + float(np.sum(np.abs(uy * rho)))
    assert abs(jx1 - jx0) <= 1e-13 * scale and abs(jy1 - jy0) <= 1e-13 * scale
    if thermal:
        assert abs(e1 - e0) <= 1e-13 * abs(e0)


@pytest.mark.parametrize("name", ["D2Q9", "D2V17", "D2V37"])
def test_uniform_equilibrium_is_steady(orc, name):
    lat = orc.lattice(name)
    n = 8
    f = orc.init_populations(lat, np.full((n, n), 1.1), np.full((n, n), 0.05), np.full((n, n), -0.03))
    g = orc.step(lat, f, 0.6, 10)
    np.testing.assert_allclose(g, f, rtol=1e-13, atol=0)


def entropy_wave_chi(orc, tau, tau3, coll):
    lat = orc.lattice("D2V37")
    ny, nx, eps = 64, 4, 1e-4
    y = (np.arange(ny) + 0.5) / ny
    th = np.broadcast_to((1.0 + eps * np.sin(2 * np.pi * y))[:, None], (ny, nx)).copy()
    z = np.zeros((ny, nx))
    f = orc.init_populations(lat, 1.0 / th, z, z, th)
    k = 2 * np.pi / ny
    t1, t2 = 200, 1200
    f = orc.step(lat, f, tau, t1, coll=coll, thermal=True, tau3=tau3)
    a1 = amplitude(orc.moments(lat, f, thermal=True)[3][:, 0] - 1.0, ny)
    f = orc.step(lat, f, tau, t2 - t1, coll=coll, thermal=True, tau3=tau3)
    a2 = amplitude(orc.moments(lat, f, thermal=True)[3][:, 0] - 1.0, ny)
    return math.log(a1 / a2) / ((t2 - t1) * k * k), lat.cs2


@pytest.mark.parametrize("coll", ["RR", "PR"])
@pytest.mark.parametrize("tau,tau3", [(0.8, 0.6), (0.6, 0.9)])
def test_entropy_wave_decays_with_the_rank3_time(orc, coll, tau, tau3):
    """Per-order relaxation (Eq. GenRegCollision with one time per rank): the
    heat flux is carried by the rank-3 coefficients, so an isobaric
    temperature mode decays at chi = c_s^2 theta (tau_3 - 1/2) while the
    viscosity keeps tau_2 = tau: Pr = (tau - 1/2) / (tau_3 - 1/2)."""
    chi, cs2 = entropy_wave_chi(orc, tau, tau3, orc.RR if coll == "RR" else orc.PR)
    assert chi == pytest.approx(cs2 * (tau3 - 0.5), rel=0.05)
    assert abs(chi - cs2 * (tau - 0.5)) > 0.5 * cs2 * abs(tau3 - tau)


@pytest.mark.parametrize("name", ["D2Q9", "D2V37"])
def test_shear_wave_ignores_rank3_and_rank4_times(orc, name):
    lat = orc.lattice(name)
    ny, nx, tau = 64, 4, 0.8
    U = 1e-4 * math.sqrt(lat.cs2)
    y = (np.arange(ny) + 0.5) / ny
    ux = np.broadcast_to((U * np.sin(2 * np.pi * y))[:, None], (ny, nx)).copy()
    f = orc.init_populations(lat, np.ones((ny, nx)), ux, np.zeros((ny, nx)))
    k = 2 * np.pi / ny
    f = orc.step(lat, f, tau, 50, tau3=0.6, tau4=1.1)
    a1 = amplitude(orc.moments(lat, f)[1][:, 0], ny)
    f = orc.step(lat, f, tau, 1000, tau3=0.6, tau4=1.1)
    a2 = amplitude(orc.moments(lat, f)[1][:, 0], ny)
    assert math.log(a1 / a2) / (1000 * k * k) == pytest.approx(lat.cs2 * (tau - 0.5), rel=0.01)


def test_per_order_times_equal_to_tau_are_the_single_time_operator(orc):
    lat = orc.lattice("D2V37")
    rng = np.random.default_rng(4)
    f = orc.equilibrium(lat, rng.uniform(0.9, 1.1, 30), rng.uniform(-0.1, 0.1, 30), rng.uniform(-0.1, 0.1, 30))
    f = f * (1 + 1e-3 * rng.uniform(-1, 1, f.shape))
    for coll in (orc.RR, orc.PR):
        assert np.array_equal(orc.collide(lat, f, 0.7, coll=coll, tau3=0.7, tau4=0.7), orc.collide(lat, f, 0.7, coll=coll))
        assert not np.array_equal(orc.collide(lat, f, 0.7, coll=coll, tau3=0.9), orc.collide(lat, f, 0.7, coll=coll))
