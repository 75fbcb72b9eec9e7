"""Pins of the oracle's harness pieces that are not part of the step: the
periodic fourth-order centred first derivative and the vorticity built from
it (Sec. III.B computes the enstrophy with that stencil), the kinetic-energy
and enstrophy statistics, and the closure reference's GELU and Adam.

Each check is an independent fact, not the formula typed again:
  - the derivative against the analytic derivative of a Fourier mode, with
    the error falling as h^4 (a second-order stencil falls as h^2), and
    against the stencil's Fourier symbol (8 sin t - sin 2t) / 6 at t = k h
    (a property of any periodic centred five-point stencil with these
    weights, derived by summing the shifted exponentials);
  - vorticity sign and axes on fields that vary along one axis only;
  - the statistics on a sine field, whose discrete means over a full period
    are known in closed form (mean of sin^2 = 1/2, of sin^4 = 3/8);
  - GELU and its derivative against torch's own tanh-form GELU and autograd;
  - Adam over several steps against torch.optim.Adam, and against moment
    sums written as weighted series (exact rational arithmetic) instead of
    the recursive update.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import mlp


def mode(n, m, axis, phase=0.3):
    """sin(2 pi m (i + 1/2) / n + phase) along `axis` of an n x n grid."""
    i = (np.arange(n) + 0.5) / n
    s = np.sin(2 * np.pi * m * i + phase)
    return np.broadcast_to(s[:, None] if axis == 0 else s[None, :], (n, n)).copy()


def dmode(n, m, axis, phase=0.3):
    """Analytic derivative of mode() with respect to the grid index."""
    i = (np.arange(n) + 0.5) / n
    k = 2 * np.pi * m / n
    d = k * np.cos(2 * np.pi * m * i + phase)
    return np.broadcast_to(d[:, None] if axis == 0 else d[None, :], (n, n)).copy()


@pytest.mark.parametrize("axis", [0, 1])
def test_ddx4_is_fourth_order(axis):
    errs = []
    for n in (64, 128, 256):
        got = oracle.ddx4(mode(n, 3, axis), axis)
        k = 2 * np.pi * 3 / n
        errs.append(float(np.abs(got - dmode(n, 3, axis)).max()) / k)  # relative to |f'| max
        # no derivative along the other axis of a field constant there
        assert np.abs(oracle.ddx4(mode(n, 3, axis), 1 - axis)).max() < 1e-15
    # leading relative error (k h)^4 / 30: halving h divides it by 16
    for a, b in zip(errs, errs[1:]):
        assert 15.0 < a / b < 16.5, errs
    k = 2 * np.pi * 3 / 256
    assert errs[-1] == pytest.approx(k ** 4 / 30, rel=0.01)


@pytest.mark.parametrize("m", [1, 5, 13])
def test_ddx4_fourier_symbol(m):
    n = 64
    t = 2 * np.pi * m / n
    sym = (8 * math.sin(t) - math.sin(2 * t)) / 6.0
    for axis in (0, 1):
        f = mode(n, m, axis)
        want = dmode(n, m, axis) * (sym / t)
        np.testing.assert_allclose(oracle.ddx4(f, axis), want, rtol=0, atol=1e-14)


def test_vorticity_sign_and_axes():
    n = 48
    t = 2 * np.pi / n
    sym = (8 * math.sin(t) - math.sin(2 * t)) / 6.0
    # shear u_x = sin(2 pi y): omega = -d u_x / dy
    ux, uy = mode(n, 1, 0, 0.0), np.zeros((n, n))
    np.testing.assert_allclose(oracle.vorticity(ux, uy), -dmode(n, 1, 0, 0.0) * sym / t, atol=1e-15)
    # u_y = sin(2 pi x): omega = +d u_y / dx
    ux, uy = np.zeros((n, n)), mode(n, 1, 1, 0.0)
    np.testing.assert_allclose(oracle.vorticity(ux, uy), dmode(n, 1, 1, 0.0) * sym / t, atol=1e-15)
    # a counter-clockwise eddy at the centre: u = (-(y - c), x - c) locally
    i = np.arange(n) - (n - 1) / 2
    X, Y = np.meshgrid(i, i)  # [y, x]
    env = np.exp(-(X ** 2 + Y ** 2) / 50.0)
    w = oracle.vorticity(-Y * env, X * env)
    assert w[n // 2, n // 2] == pytest.approx(2.0, rel=0.05)


def test_flow_stats_closed_forms():
    n, U, u0 = 64, 0.03, 0.05
    ux, uy = mode(n, 1, 0, 0.0) * U, np.zeros((n, n))
    st = oracle.flow_stats(ux, uy, u0, n)
    # KE = (U^2 / 2 u0^2) sin^2: mean (1/2), mean of the square (3/8)
    a = U * U / (2 * u0 * u0)
    assert st["ke_mean"] == pytest.approx(a / 2, rel=1e-13)
    assert st["ke_std"] == pytest.approx(a * math.sqrt(3 / 8 - 1 / 4), rel=1e-12)
    # omega = -U D cos, D the stencil's symbol; enstrophy 0.5 omega^2 (L/u0)^2
    t = 2 * np.pi / n
    D = (8 * math.sin(t) - math.sin(2 * t)) / 6.0
    b = 0.5 * (U * D) ** 2 * (n / u0) ** 2
    assert st["ens_mean"] == pytest.approx(b / 2, rel=1e-12)
    assert st["ens_std"] == pytest.approx(b * math.sqrt(3 / 8 - 1 / 4), rel=1e-11)
    # the continuum enstrophy of the shear, (2 pi U / u0)^2 / 4, within O(h^4)
    assert st["ens_mean"] == pytest.approx((2 * np.pi * U / u0) ** 2 / 4, rel=t ** 4 / 15 + 1e-12)
    # a uniform flow carries no enstrophy and no spatial spread
    st = oracle.flow_stats(np.full((n, n), U), np.full((n, n), -U), u0, n)
    assert st["ke_mean"] == pytest.approx(U * U / (u0 * u0), rel=1e-14)
    assert st["ke_std"] < 1e-14 and st["ens_mean"] == 0.0 and st["ens_std"] == 0.0


def test_gelu_against_torch():
    import torch
    import torch.nn.functional as F

    z = np.linspace(-8, 8, 4001)
    zt = torch.tensor(z, dtype=torch.float64, requires_grad=True)
    y = F.gelu(zt, approximate="tanh")
    np.testing.assert_allclose(mlp.gelu(z), y.detach().numpy(), rtol=1e-14, atol=1e-15)
    (g,) = torch.autograd.grad(y.sum(), zt)
    np.testing.assert_allclose(mlp.gelu_prime(z), g.numpy(), rtol=1e-13, atol=1e-14)
    # the tanh form stays within 1e-3 of the exact (erf) GELU
    exact = F.gelu(torch.tensor(z, dtype=torch.float64)).numpy()
    assert np.abs(mlp.gelu(z) - exact).max() < 1e-3
    assert mlp.gelu(1.0) == pytest.approx(0.8411919906, abs=1e-10)


def adam_series(gs, t, lr, b1, b2, eps):
    """Parameter after t Adam steps from 0, with m_t and v_t written as
    weighted sums of the gradients (exact rationals) rather than updated
    recursively."""
    th = 0.0
    B1, B2 = Fraction(b1), Fraction(b2)
    for s in range(1, t + 1):
        m = sum((1 - B1) * B1 ** (s - r) * Fraction(gs[r - 1]) for r in range(1, s + 1))
        v = sum((1 - B2) * B2 ** (s - r) * Fraction(gs[r - 1]) ** 2 for r in range(1, s + 1))
        mh, vh = m / (1 - B1 ** s), v / (1 - B2 ** s)
        th -= lr * float(mh) / (math.sqrt(float(vh)) + eps)
    return th


def test_adam_multi_step_series():
    gs = [1.0, -1.0, 2.0, 0.25, -3.0]
    lr, b1, b2, eps = 0.1, 0.8, 0.95, 1e-8
    th, m, v = np.zeros(1), np.zeros(1), np.zeros(1)
    for t in range(1, len(gs) + 1):
        th, m, v = mlp.adam(th, np.array([gs[t - 1]]), m, v, t, lr, b1, b2, eps)
        assert th[0] == pytest.approx(adam_series(gs, t, lr, b1, b2, eps), rel=1e-13, abs=1e-16), t
    # the same sequence with the betas swapped ends elsewhere
    assert abs(th[0] - adam_series(gs, len(gs), lr, b2, b1, eps)) > 1e-3


def test_adam_against_torch():
    import torch

    rng = np.random.default_rng(11)
    p0 = rng.normal(size=257)
    grads = rng.normal(size=(6, 257)) * np.array([1.0, 0.1, 3.0, 0.01, 1.0, 0.5])[:, None]
    for betas in ((0.9, 0.999), (0.7, 0.9)):
        p = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
        opt = torch.optim.Adam([p], lr=2e-3, betas=betas, eps=1e-8)
        th, m, v = p0.copy(), np.zeros_like(p0), np.zeros_like(p0)
        for t, g in enumerate(grads, start=1):
            p.grad = torch.tensor(g, dtype=torch.float64)
            opt.step()
            th, m, v = mlp.adam(th, g, m, v, t, 2e-3, betas[0], betas[1], 1e-8)
            np.testing.assert_allclose(th, p.detach().numpy(), rtol=1e-13, atol=1e-15)


# ---- the pins above catch plausible mistakes (planted in the oracle, on the CPU)

def _fails(fn, *a):
    try:
        fn(*a)
    except AssertionError:
        return True
    return False


def test_planted_mistakes_fail_the_pins(monkeypatch):
    good_ddx4, good_adam, good_gelu = oracle.ddx4, mlp.adam, mlp.gelu

    def flipped(g, axis):  # sign error
        return -good_ddx4(g, axis)

    def second_order(g, axis):  # the plain centred difference
        return (np.roll(g, -1, axis) - np.roll(g, 1, axis)) / 2.0

    def swapped_axes(ux, uy):  # transposed operands
        return good_ddx4(uy, 0) - good_ddx4(ux, 1)

    for bad in (flipped, second_order):
        monkeypatch.setattr(oracle, "ddx4", bad)
        assert _fails(test_ddx4_is_fourth_order, 0) and _fails(test_vorticity_sign_and_axes)
    monkeypatch.setattr(oracle, "ddx4", good_ddx4)
    monkeypatch.setattr(oracle, "vorticity", swapped_axes)
    assert _fails(test_vorticity_sign_and_axes) and _fails(test_flow_stats_closed_forms)
    monkeypatch.undo()

    def no_half(ux, uy, u0, L):  # KE / enstrophy without the 1/2
        ke = (ux * ux + uy * uy) / (u0 * u0)
        w = oracle.vorticity(ux, uy)
        en = w * w * (L / u0) ** 2
        return dict(ke_mean=float(ke.mean()), ke_std=float(ke.std()), ens_mean=float(en.mean()),
                    ens_std=float(en.std()))

    monkeypatch.setattr(oracle, "flow_stats", no_half)
    assert _fails(test_flow_stats_closed_forms)
    monkeypatch.undo()

    def adam_swapped(theta, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        return good_adam(theta, grad, m, v, t, lr, beta2, beta1, eps)

    def adam_no_bias_correction(theta, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        m = beta1 * m + (1 - beta1) * grad
        v = beta2 * v + (1 - beta2) * grad * grad
        return theta - lr * m / (np.sqrt(v) + eps), m, v

    for bad in (adam_swapped, adam_no_bias_correction):
        monkeypatch.setattr(mlp, "adam", bad)
        assert _fails(test_adam_multi_step_series) and _fails(test_adam_against_torch)
    monkeypatch.undo()

    for c, a in ((np.sqrt(np.pi / 2), 0.044715), (np.sqrt(2 / np.pi), 0.0447)):
        monkeypatch.setattr(mlp, "GELU_C", c)
        monkeypatch.setattr(mlp, "GELU_A", a)
        assert _fails(test_gelu_against_torch)
    monkeypatch.undo()
    assert mlp.gelu is good_gelu and oracle.ddx4 is good_ddx4
