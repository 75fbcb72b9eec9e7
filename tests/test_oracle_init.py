"""The f^(0) + f^(1) initial state of the oracle (Sec. III.B: f^(1) from the
analytic velocity gradients, expanded over the same Hermite terms as f^(0)).

Pins: f^(1) carries no mass or momentum; and it is the Chapman-Enskog state.
A shear wave started from f^(0) + f^(1) decays as exp(-nu k^2 t) from the
first step (nu = c_s^2 (tau - 1/2)), while one started from f^(0) alone
lags by its start-up transient.  A wave along y exercises the xy component;
a diagonal wave (div u = 0) the xx and yy components as well.  A wrong sign,
a missing factor tau or a transposed gradient index each leave a deficit of
the f^(0) kind (~1e-3).
"""
import numpy as np
import pytest

LATTICES = ["D2Q9", "D2V17", "D2V37"]


@pytest.mark.parametrize("name", LATTICES)
def test_noneq_init_carries_no_mass_or_momentum(orc, name):
    lat = orc.lattice(name)
    rng = np.random.default_rng(3)
    n = 50
    rho = rng.uniform(0.9, 1.1, n)
    ux, uy = rng.uniform(-0.1, 0.1, n), rng.uniform(-0.1, 0.1, n)
    g = rng.uniform(-1e-2, 1e-2, (4, n))
    f1 = orc.noneq_init(lat, rho, ux, uy, g, 0.7)
    assert np.abs(f1.sum(axis=0)).max() <= 1e-15
    for d in range(2):
        assert np.abs((lat.c[:, d][:, None] * f1).sum(axis=0)).max() <= 1e-15
    # the rank-2 projection returns -rho c_s^2 tau S, S = grad u + grad u^T
    hxy = ((lat.c[:, 0] * lat.c[:, 1])[:, None] * f1).sum(axis=0)
    np.testing.assert_allclose(hxy, -rho * lat.cs2 * 0.7 * (g[1] + g[2]), rtol=1e-12, atol=1e-17)


def wave_decay(orc, lat, tau, diagonal, with_f1, n=64, amp=1e-3, steps=10):
    k = 2 * np.pi / n
    x, y = np.meshgrid(np.arange(n) + 0.5, np.arange(n) + 0.5)
    if diagonal:
        s, c = np.sin(k * (x + y)), np.cos(k * (x + y))
        ux, uy = amp * s / np.sqrt(2), -amp * s / np.sqrt(2)
        g = np.stack([amp * k * c / np.sqrt(2)] * 2 + [-amp * k * c / np.sqrt(2)] * 2)
        kmag, mode = k * np.sqrt(2), s
    else:
        s, c = np.sin(k * y), np.cos(k * y)
        ux, uy = amp * s, 0 * s
        g = np.stack([0 * s, amp * k * c, 0 * s, 0 * s])
        kmag, mode = k, s
    rho = np.ones((n, n))
    f0 = orc.init_populations(lat, rho, ux, uy, grad=g if with_f1 else None, tau=tau)
    nu = lat.cs2 * (tau - 0.5)
    f = orc.collide(lat, f0, tau)
    dev = []
    for t in range(1, steps + 1):
        f = orc.collide(lat, orc.stream(lat, f), tau)
        _, vx, vy, _ = orc.moments(lat, f)
        along = (vx - vy) / np.sqrt(2) if diagonal else vx
        a = np.sum(along * mode) / np.sum(mode * mode)
        dev.append(a / amp / np.exp(-nu * kmag ** 2 * t) - 1.0)
    return np.abs(np.array(dev)).max()


@pytest.mark.parametrize("name", LATTICES)
@pytest.mark.parametrize("diagonal", [False, True])
def test_noneq_init_is_the_chapman_enskog_state(orc, name, diagonal):
    lat = orc.lattice(name)
    tau = 0.8
    with_f1 = wave_decay(orc, lat, tau, diagonal, True)
    without = wave_decay(orc, lat, tau, diagonal, False)
    print(f"[pin] {name} {'diagonal' if diagonal else 'shear'} wave: |A/A_CE - 1| <= {with_f1:.2e} "
          f"from f0+f1, {without:.2e} from f0")
    assert with_f1 <= 5e-5
    assert without >= 20 * with_f1
