"""The moment representation (LBM_STORE_MOMENTS: six FP64 values per node)
against the FP64 oracle and against the population form of the library.

For the isothermal recursive regularization the post-collision populations
are a function of (rho, u, a1^(2)), so lbm_populations rebuilt from the
moments must equal the oracle's C(f^n) element by element: both sides in
double, a few ulps of |f| <= 1 per step, bound 1e-12 as for the population
form.  Grids narrower than the staged tile take the modulo wrap path."""
import numpy as np
import pytest

from paper_1704_04413_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def b():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1704_04413_amd import binding

    binding.lib()
    return binding


def check(got, want, atol, what="f"):
    err = float(np.abs(np.asarray(got) - np.asarray(want)).max())
    print(f"[parity] moments {what}: max |gpu - oracle| = {err:.3e} (bound {atol:.0e})", flush=True)
    assert err <= atol, err


def case(orc, name, nx, ny, re=1e4, k=20.0, grad=False):
    lat = orc.lattice(name)
    u0, tau = wl.shear_layer_params(lat.cs2, max(nx, ny), re)
    rho, ux, uy = wl.shear_layer_fields(nx, ny, u0, k=k)
    g = wl.shear_layer_gradients(nx, ny, u0, k=k) if grad else None
    noise = wl.uniform_noise(7, lat.Q, ny, nx)
    f0 = orc.init_populations(lat, rho, ux, uy, None, noise, 1e-8, grad=g, tau=tau)
    return lat, tau, (rho, ux, uy, g, noise), f0


def sim_of(b, name, nx, ny, tau, fields, flags, order=None):
    rho, ux, uy, g, noise = fields
    return b.Simulation(name, nx, ny, tau, rho, ux, uy, noise=noise, noise_amp=1e-8, grad=g, flags=flags,
                        reg_order=order)


@pytest.mark.parametrize("name,order", [("D2Q9", 2), ("D2Q9", 3), ("D2Q9", 4), ("D2V17", 2), ("D2V17", 3),
                                        ("D2V37", 2), ("D2V37", 3), ("D2V37", 4)])
def test_moments_against_oracle(orc, b, name, order):
    nx, ny = 70, 45
    print(f"[case] moments {name} RR{order} {nx}x{ny}", flush=True)
    lat, tau, fields, f0 = case(orc, name, nx, ny)
    sim = sim_of(b, name, nx, ny, tau, fields, b.LBM_STORE_MOMENTS, order)
    done = 0
    for steps in (0, 1, 7):
        sim.step(steps - done)
        done = steps
        got = sim.populations().cpu().numpy()
        want = orc.collide(lat, orc.step(lat, f0, tau, steps, order=order), tau, order=order)
        check(got, want, 1e-12)
    sim.close()


@pytest.mark.parametrize("name,nx,ny", [("D2Q9", 1, 1), ("D2Q9", 2, 3), ("D2V17", 3, 4), ("D2V37", 3, 5),
                                        ("D2V37", 65, 3), ("D2V37", 5, 70), ("D2V37", 130, 9)])
def test_moments_small_and_ragged_grids(orc, b, name, nx, ny):
    print(f"[case] moments {name} {nx}x{ny}", flush=True)
    lat, tau, fields, f0 = case(orc, name, nx, ny, re=3e3, k=8.0)
    sim = sim_of(b, name, nx, ny, tau, fields, b.LBM_STORE_MOMENTS)
    sim.step(5)
    got = sim.populations().cpu().numpy()
    sim.close()
    check(got, orc.collide(lat, orc.step(lat, f0, tau, 5), tau), 1e-12)


@pytest.mark.parametrize("name", ["D2Q9", "D2V37"])
def test_moments_follow_the_population_form(orc, b, name):
    """200 steps of the shear layer with the f^(0) + f^(1) start: populations
    and diagnostics of both representations agree."""
    nx, ny = 128, 96
    print(f"[case] moments vs populations {name} {nx}x{ny} x 200", flush=True)
    lat, tau, fields, _ = case(orc, name, nx, ny, re=3e4, k=40.0, grad=True)
    a = sim_of(b, name, nx, ny, tau, fields, b.LBM_STORE_MOMENTS)
    p = sim_of(b, name, nx, ny, tau, fields, 0)
    a.step(200)
    p.step(200)
    fa, fp = a.populations().cpu().numpy(), p.populations().cpu().numpy()
    ma, mp = a.moments(), p.moments()
    check(fa, fp, 1e-11, "populations vs population form")
    for key in ("rho", "ux", "uy", "vort"):
        check(ma[key].cpu().numpy(), mp[key].cpu().numpy(), 1e-11, key)
    sa, sp = np.asarray(ma["sums"]), np.asarray(mp["sums"])
    # the net momentum sums are ~0: absolute bound of 1e-12 per node
    print(f"[parity] moments sums max |diff| {np.abs(sa - sp)[:8].max():.3e}", flush=True)
    np.testing.assert_allclose(sa[:8], sp[:8], rtol=1e-10, atol=1e-12 * nx * ny)
    assert sa[8] == sp[8] == 0
    a.close()
    p.close()


def test_moments_rejected_where_populations_are_needed(orc, b):
    import torch

    lat, tau, fields, _ = case(orc, "D2V37", 16, 16)
    sim = sim_of(b, "D2V37", 16, 16, tau, fields, b.LBM_STORE_MOMENTS)
    with pytest.raises(b.LbmError):
        b.lbm_batch_create([sim.ctx], 64, 4)
    theta = torch.zeros(b.LBM_MLP_NPARAM, dtype=torch.float32, device="cuda")
    norm = torch.ones(b.LBM_MLP_NNORM, dtype=torch.float32, device="cuda")
    with pytest.raises(b.LbmError):
        b.lbm_closure_set(sim.ctx, theta, norm)
    sim.close()


@pytest.mark.parametrize("name,n", [("D2V37", 1024), ("D2V17", 1024), ("D2V37", 2048)])
def test_moments_full_size_sampled(orc, b, name, n):
    """The moment form at the benchmark's grid sizes (its launch shape:
    16-row blocks of 64 - 2R output columns, ragged at the right edge): init
    + 2 steps, the rebuilt post-collision populations checked at 512 sampled
    nodes (edges included) that the oracle evaluates one by one (gather the
    neighbours' post-collision values, collide)."""
    import torch

    print(f"[case] moments {name} {n}x{n} sampled nodes", flush=True)
    steps = 2
    lat = orc.lattice(name)
    u0, tau = wl.shear_layer_params(lat.cs2, n, 1e5)
    rho, ux, uy = wl.shear_layer_fields(n, n, u0)
    noise = wl.uniform_noise(3, lat.Q, n, n)
    sim = b.Simulation(name, n, n, tau, rho, ux, uy, noise=noise, noise_amp=1e-8, flags=b.LBM_STORE_MOMENTS)
    sim.step(steps)
    f = sim.populations()
    rng = np.random.default_rng(11)
    ys = np.concatenate([[0, n - 1, 15, 16, 0], rng.integers(0, n, 507)])
    xs = np.concatenate([[0, n - 1, 57, 58, n - 3], rng.integers(0, n, 507)])
    got = f[:, torch.as_tensor(ys, device=f.device), torch.as_tensor(xs, device=f.device)].cpu().numpy()
    sim.close()
    del f

    def post(ys_, xs_, t):
        if t == 0:
            f0 = orc.init_populations(lat, rho[ys_, xs_], ux[ys_, xs_], uy[ys_, xs_], None,
                                      noise[:, ys_, xs_], 1e-8)
            return orc.collide(lat, f0, tau)
        pre = np.empty((lat.Q, len(ys_)))
        for i, (cx, cy) in enumerate(lat.c):
            pre[i] = post((ys_ - cy) % n, (xs_ - cx) % n, t - 1)[i]
        return orc.collide(lat, pre, tau)

    check(got, post(ys, xs, steps), 1e-13)


# ------------------------------------------------------------ thermal form


@pytest.mark.parametrize("a13", [False, True])
def test_thermal_moments_sod_against_oracle(orc, b, a13):
    """Thermal D2V37 (App. C) in the moment representation (rho, u, theta,
    a1^(2), a1^(3) per node): the Sod tube of the population-form test (400 x 4, tau 0.6,
    40 steps; 4 rows take the modulo wrap of the staged block), populations
    rebuilt from the moments against the oracle, same bound (1e-11 for
    |f| <= 3.3), and theta against the oracle's."""
    print(f"[case] thermal moments sod a13_projected={a13}", flush=True)
    lat = orc.lattice("D2V37")
    nx, ny, tau, steps = 400, 4, 0.6, 40
    rho, ux, uy, th = wl.sod_fields(nx, ny)
    f0 = orc.init_populations(lat, rho, ux, uy, th)
    flags = b.LBM_STORE_MOMENTS | b.LBM_THERMAL | (b.LBM_A13_PROJECTED if a13 else 0)
    sim = b.Simulation("D2V37", nx, ny, tau, rho, ux, uy, theta=th, flags=flags)
    assert b.lbm_buffer_elems("D2V37", nx, ny, flags) == 11 * nx * ny
    sim.step(steps)
    got = sim.populations().cpu().numpy()
    m = sim.moments()
    sim.close()
    want = orc.collide(lat, orc.step(lat, f0, tau, steps, thermal=True, a13_raw=a13), tau, thermal=True,
                       a13_raw=a13)
    check(got, want, 1e-11)
    _, _, _, t = orc.moments(lat, want, thermal=True)
    np.testing.assert_allclose(m["theta"].cpu().numpy(), t, rtol=0, atol=2e-9)


def test_thermal_moments_shear_with_noise(orc, b):
    """Thermal shear layer with a temperature perturbation and seeded noise on
    a ragged 70 x 45 grid, RR at order 3 and 4."""
    lat = orc.lattice("D2V37")
    nx, ny = 70, 45
    u0, tau = wl.shear_layer_params(lat.cs2, nx, 3e3)
    rho, ux, uy = wl.shear_layer_fields(nx, ny, u0, k=20.0)
    th = 1.0 + 0.05 * np.cos(2 * np.pi * (np.arange(ny)[:, None] + 0.5) / ny) * np.ones((1, nx))
    noise = wl.uniform_noise(4, lat.Q, ny, nx)
    f0 = orc.init_populations(lat, rho, ux, uy, th, noise, 1e-8)
    for order in (3, 4):
        print(f"[case] thermal moments shear RR{order} {nx}x{ny}", flush=True)
        sim = b.Simulation("D2V37", nx, ny, tau, rho, ux, uy, theta=th, noise=noise, noise_amp=1e-8,
                           flags=b.LBM_STORE_MOMENTS | b.LBM_THERMAL, reg_order=order)
        sim.step(9)
        got = sim.populations().cpu().numpy()
        sim.close()
        want = orc.collide(lat, orc.step(lat, f0, tau, 9, thermal=True, order=order), tau, thermal=True,
                           order=order)
        check(got, want, 1e-12)


def test_thermal_moments_per_order_relaxation(orc, b):
    """Pr = 0.5 on the Sod tube: rank 3 relaxed with its own time; the state is
    the pre-collision moments, so every rebuild uses the times in force."""
    print("[case] thermal moments per-order relaxation", flush=True)
    lat = orc.lattice("D2V37")
    nx, ny, tau, tau3 = 400, 4, 0.6, 0.7
    rho, ux, uy, th = wl.sod_fields(nx, ny)
    sim = b.Simulation("D2V37", nx, ny, tau, rho, ux, uy, theta=th, flags=b.LBM_STORE_MOMENTS | b.LBM_THERMAL)
    sim.set_relaxation(tau3, tau)
    sim.step(30)
    got = sim.populations().cpu().numpy()
    sim.close()
    f0 = orc.init_populations(lat, rho, ux, uy, th)
    g = orc.step(lat, f0, tau, 30, thermal=True, tau3=tau3, tau4=tau)
    check(got, orc.collide(lat, g, tau, thermal=True, tau3=tau3, tau4=tau), 1e-11)


def test_thermal_moments_follow_the_population_form(orc, b):
    """100 steps of the Sod tube on 800 x 20: fields and diagnostics of both
    representations agree.  The two sum in different orders, so they differ
    by rounding each step; the oracle run from an f^0 perturbed by 1e-16
    relative moves by 4.8e-13 at step 100 (|f| <= 3.3) and by 2.3e-8 at step
    200, after the waves of the two interfaces have met, hence 100 steps and
    a bound of 1e-11."""
    print("[case] thermal moments vs populations 800x20 x 100", flush=True)
    nx, ny, tau = 800, 20, 0.6
    rho, ux, uy, th = wl.sod_fields(nx, ny)
    a = b.Simulation("D2V37", nx, ny, tau, rho, ux, uy, theta=th, flags=b.LBM_STORE_MOMENTS | b.LBM_THERMAL)
    p = b.Simulation("D2V37", nx, ny, tau, rho, ux, uy, theta=th, flags=b.LBM_THERMAL)
    a.step(100)
    p.step(100)
    check(a.populations().cpu().numpy(), p.populations().cpu().numpy(), 1e-11, "populations vs population form")
    ma, mp = a.moments(), p.moments()
    for key in ("rho", "ux", "uy", "theta"):
        check(ma[key].cpu().numpy(), mp[key].cpu().numpy(), 1e-10, key)
    sa, sp = np.asarray(ma["sums"]), np.asarray(mp["sums"])
    np.testing.assert_allclose(sa[[0, 3]], sp[[0, 3]], rtol=1e-12)
    assert sa[8] == sp[8] == 0
    a.close()
    p.close()
