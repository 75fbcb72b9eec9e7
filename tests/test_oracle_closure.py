"""Pins of the closure's CPU reference: network gradients against central
finite differences, GELU's derivative, Adam against its first-step closed
form, bfloat16 rounding against torch's, and the closure collision's
invariants (zero residual = plain RR, conservation under any residual)."""
import numpy as np
import pytest

from oracle import mlp


def test_gelu_prime_matches_finite_difference():
    z = np.linspace(-6, 6, 101)
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    np.testing.assert_allclose(mlp.gelu_prime(z), fd, rtol=1e-7, atol=1e-9)
    assert mlp.gelu(0.0) == 0.0 and abs(mlp.gelu(10.0) - 10.0) < 1e-12


def test_gradients_match_central_differences():
    rng = np.random.default_rng(0)
    theta = mlp.init_params(1)
    theta[mlp.NIN * mlp.NH:mlp.NIN * mlp.NH + mlp.NH] = rng.normal(0, 0.1, mlp.NH)  # nonzero b1
    X = rng.normal(size=(32, mlp.NIN))
    X[:, -1] = 1.0
    T = rng.normal(size=(32, mlp.NOUT))
    _, g = mlp.loss_and_grad(theta, X, T, emulate_bf16=False)
    idx = np.concatenate([rng.choice(mlp.NPARAM - 16, 40, replace=False), [mlp.NPARAM - 16 + 3]])
    # central differences: truncation ~h^2, rounding ~1e-16/h of a loss of order 1
    h = 1e-5
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (mlp.loss_and_grad(tp, X, T, False)[0] - mlp.loss_and_grad(tm, X, T, False)[0]) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-5, abs=1e-9), i
    # padding outputs receive no gradient
    p = mlp.unpack(g)
    assert np.all(p["W3"][:, mlp.NOUT:] == 0) and np.all(p["b3"][mlp.NOUT:] == 0)


def test_adam_first_step_is_signed_lr():
    """After one step from zero moments Adam moves each parameter by lr*sign(g)
    (up to eps)."""
    th = np.zeros(5)
    g = np.array([1.0, -2.0, 3e-3, -4e-2, 0.5])
    new, m, v = mlp.adam(th, g, np.zeros(5), np.zeros(5), 1, 1e-3)
    np.testing.assert_allclose(new, -1e-3 * np.sign(g), rtol=1e-5)


def test_bf16_rounding_matches_torch():
    import torch

    x = np.random.default_rng(3).normal(size=10000) * 10 ** np.random.default_rng(4).uniform(-8, 8, 10000)
    want = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.bf16(x), want)


def test_closure_collision_invariants(orc):
    lat = orc.lattice("D2V37")
    rng = np.random.default_rng(5)
    n = 64
    rho = rng.uniform(0.9, 1.1, n)
    ux, uy = rng.uniform(-0.08, 0.08, (2, n))
    f = orc.equilibrium(lat, rho, ux, uy) * (1 + 1e-3 * rng.uniform(-1, 1, (lat.Q, n)))
    tau = 0.52
    plain = orc.collide(lat, f, tau)
    zero = orc.collide_closure(lat, f, tau, np.zeros((9, n)))
    np.testing.assert_allclose(zero, plain, rtol=0, atol=1e-16)
    resid = rng.normal(size=(9, n)) * 1e-3
    out = orc.collide_closure(lat, f, tau, resid)
    c = lat.c.astype(float)
    np.testing.assert_allclose(out.sum(0), f.sum(0), rtol=1e-14)
    np.testing.assert_allclose(c[:, 0] @ out, c[:, 0] @ f, atol=1e-15)
    np.testing.assert_allclose(c[:, 1] @ out, c[:, 1] @ f, atol=1e-15)
    assert np.abs(out - plain).max() > 1e-6


def test_closure_inputs_are_the_rr_coefficients(orc):
    """The exported plain-RR a_hat^(3..4) equal (1 - 1/2tau) times the oracle's
    own non-equilibrium coefficients, and the features match the moments."""
    lat = orc.lattice("D2V37")
    rng = np.random.default_rng(6)
    n = 16
    f = orc.equilibrium(lat, rng.uniform(0.9, 1.1, n), rng.uniform(-0.05, 0.05, n), rng.uniform(-0.05, 0.05, n))
    f = f * (1 + 1e-3 * rng.uniform(-1, 1, f.shape))
    tau = 0.6
    feat, rr = orc.closure_inputs(lat, f, tau)
    s = 1 - 0.5 / tau
    for k in range(n):
        a1 = orc.noneq_coeffs(lat, f[:, k])
        assert feat[4, k] == pytest.approx(s * a1[orc.toff(2, 0)], rel=1e-12)
        assert feat[5, k] == pytest.approx(s * a1[orc.toff(2, 2)], rel=1e-12)
        assert rr[0, k] == pytest.approx(s * a1[orc.toff(3, 0)], rel=1e-12)
        assert rr[8, k] == pytest.approx(s * a1[orc.toff(4, 15)], rel=1e-12)
    r, vx, vy, _ = orc.moments(lat, f)
    np.testing.assert_allclose(feat[0], r - 1, rtol=1e-12)
    np.testing.assert_allclose(feat[1], vx, rtol=1e-12)
    np.testing.assert_allclose(feat[2], vy, rtol=1e-12)
    np.testing.assert_allclose(feat[3], (vx ** 2 + vy ** 2) / lat.cs2, rtol=1e-12)
