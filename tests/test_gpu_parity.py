"""GPU parity: the HIP library (through its C-ABI) against the FP64 oracle.

The library keeps the post-collision state, so after n steps its populations
are C(f^n), which the oracle produces as collide(step(f^0, n)).  Tolerances
for FP64 storage: both sides compute in double with different association
orders; one step rounds each population to a few ulps of |f| <= 1, so the
absolute difference after n <= 50 steps is bounded by ~n * 1e-15 and tested
at 1e-12.
"""
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


def say(msg):
    print(f"[case] {msg}", flush=True)


def check(got, want, atol):
    err = float(np.abs(np.asarray(got) - np.asarray(want)).max())
    print(f"[parity] max |gpu - oracle| = {err:.3e} (bound {atol:.0e})", flush=True)
    assert err <= atol, err


def shear_case(orc, name, nx, ny, re=1e4, seed=0, eq_order=None):
    lat = orc.lattice(name)
    u0, tau = wl.shear_layer_params(lat.cs2, max(nx, ny), re)
    rho, ux, uy = wl.shear_layer_fields(nx, ny, u0)
    noise = wl.uniform_noise(seed, lat.Q, ny, nx)
    f0 = orc.init_populations(lat, rho, ux, uy, None, noise, 1e-8, eq_order=eq_order)
    return lat, u0, tau, (rho, ux, uy, None, noise), f0


def run_gpu(b, name, nx, ny, tau, fields, steps, flags=0, order=None):
    rho, ux, uy, th, noise = fields
    sim = b.Simulation(name, nx, ny, tau, rho, ux, uy, theta=th, noise=noise,
                       noise_amp=1e-8 if noise is not None else 0.0, flags=flags, reg_order=order)
    sim.step(steps)
    f = sim.populations().cpu().numpy()
    mom = sim.moments()
    out = dict(f=f, rho=mom["rho"].cpu().numpy(), ux=mom["ux"].cpu().numpy(), uy=mom["uy"].cpu().numpy(),
               theta=mom["theta"].cpu().numpy(), vort=mom["vort"].cpu().numpy(), sums=mom["sums"],
               steps=sim.steps)
    sim.close()
    return out


@pytest.mark.parametrize("name", ["D2Q9", "D2V17", "D2V37"])
@pytest.mark.parametrize("nx,ny,steps", [(70, 45, 30), (64, 64, 5)])
def test_fp64_rr_populations(orc, b, name, nx, ny, steps):
    say(f"fp64 RR {name} {nx}x{ny} steps={steps}")
    eq = 2 if name == "D2Q9" else None
    lat, u0, tau, fields, f0 = shear_case(orc, name, nx, ny, eq_order=eq)
    got = run_gpu(b, name, nx, ny, tau, fields, steps,
                  flags=b.LBM_EQ_INIT_ORDER2 if eq == 2 else 0)
    want = orc.collide(lat, orc.step(lat, f0, tau, steps), tau)
    assert got["steps"] == steps
    check(got["f"], want, 1e-12)


@pytest.mark.parametrize("name,order", [("D2Q9", 2), ("D2Q9", 3), ("D2V17", 2), ("D2V37", 3)])
def test_fp64_lower_orders(orc, b, name, order):
    say(f"fp64 RR order {order} {name}")
    lat, u0, tau, fields, f0 = shear_case(orc, name, 40, 37)
    got = run_gpu(b, name, 40, 37, tau, fields, 10, order=order)
    want = orc.collide(lat, orc.step(lat, f0, tau, 10, order=order), tau, order=order)
    check(got["f"], want, 1e-12)


@pytest.mark.parametrize("name,coll,order", [("D2Q9", "PR", 4), ("D2Q9", "BGK", 2), ("D2V17", "PR", 3),
                                             ("D2V37", "PR", 4), ("D2V37", "BGK", 2)])
def test_fp64_pr_bgk(orc, b, name, coll, order):
    say(f"fp64 {coll}{order} {name}")
    lat, u0, tau, fields, f0 = shear_case(orc, name, 40, 36, re=3e3)
    c = orc.PR if coll == "PR" else orc.BGK
    flags = b.LBM_COLL_PR if coll == "PR" else b.LBM_COLL_BGK
    got = run_gpu(b, name, 40, 36, tau, fields, 10, flags=flags, order=order)
    want = orc.collide(lat, orc.step(lat, f0, tau, 10, coll=c, order=order), tau, coll=c, order=order)
    check(got["f"], want, 1e-12)


@pytest.mark.parametrize("name,coll", [("D2Q9", "rr"), ("D2V17", "rr"), ("D2V37", "rr"), ("D2V37", "pr"),
                                       ("D2Q9", "bgk")])
def test_fp64_noneq_initial_state(orc, b, name, coll):
    """f^(0) + f^(1) start from the analytic shear-layer gradients (Sec. III.B)
    on a ragged grid, then 7 steps."""
    nx, ny = 70, 45
    say(f"f0+f1 start {name} {coll} {nx}x{ny}")
    lat = orc.lattice(name)
    u0, tau = wl.shear_layer_params(lat.cs2, max(nx, ny), 1e4)
    rho, ux, uy = wl.shear_layer_fields(nx, ny, u0, k=20.0)
    g = wl.shear_layer_gradients(nx, ny, u0, k=20.0)
    noise = wl.uniform_noise(5, lat.Q, ny, nx)
    flags = {"rr": 0, "pr": b.LBM_COLL_PR, "bgk": b.LBM_COLL_BGK}[coll]
    ocoll = {"rr": orc.RR, "pr": orc.PR, "bgk": orc.BGK}[coll]
    order = lat.n_eq if coll != "bgk" else 2
    f0 = orc.init_populations(lat, rho, ux, uy, None, noise, 1e-8, grad=g, tau=tau)
    assert np.abs(f0 - orc.init_populations(lat, rho, ux, uy, None, noise, 1e-8)).max() > 1e-6
    for steps in (0, 7):
        sim = b.Simulation(name, nx, ny, tau, rho, ux, uy, noise=noise, noise_amp=1e-8, grad=g, flags=flags,
                           reg_order=order)
        sim.step(steps)
        got = sim.populations().cpu().numpy()
        sim.close()
        want = orc.collide(lat, orc.step(lat, f0, tau, steps, coll=ocoll, order=order), tau, coll=ocoll,
                           order=order)
        check(got, want, 1e-12)


@pytest.mark.parametrize("a13", [False, True])
def test_fp64_thermal_sod(orc, b, a13):
    say(f"fp64 thermal D2V37 sod a13_projected={a13}")
    lat = orc.lattice("D2V37")
    # 400 cells keep the two periodic interfaces' waves apart over 40 steps;
    # there a 1e-16 relative perturbation of f^0 moves the oracle's result by
    # < 1e-13 (|f| <= 3.3), so 1e-11 leaves room for the GPU's rounding
    nx, ny, tau, steps = 400, 4, 0.6, 40
    rho, ux, uy, th = wl.sod_fields(nx, ny)
    f0 = orc.init_populations(lat, rho, ux, uy, th)
    flags = b.LBM_THERMAL | (b.LBM_A13_PROJECTED if a13 else 0)
    got = run_gpu(b, "D2V37", nx, ny, tau, (rho, ux, uy, th, None), steps, flags=flags)
    want = orc.collide(lat, orc.step(lat, f0, tau, steps, thermal=True, a13_raw=a13), tau, thermal=True,
                       a13_raw=a13)
    check(got["f"], want, 1e-11)
    r, vx, vy, t = orc.moments(lat, want, thermal=True)
    # theta = (sum f|c|^2 - rho u^2) / (2 rho c_s^2) moves by at most
    # sum_i |c_i|^2 |df_i| / (2 rho c_s^2) <= 1e-11 * 200 / 1.4 for |df| <= 1e-11
    np.testing.assert_allclose(got["theta"], t, rtol=0, atol=2e-9)


def test_fp64_thermal_shear_pr(orc, b):
    say("fp64 thermal D2V37 PR4 shear layer")
    lat, u0, tau, fields, f0 = shear_case(orc, "D2V37", 33, 31, re=3e3)
    rho, ux, uy, _, noise = fields
    th = 1.0 + 0.05 * np.cos(2 * np.pi * np.arange(33) / 33)[None, :] * np.ones((31, 1))
    f0 = orc.init_populations(lat, rho, ux, uy, th, noise, 1e-8)
    got = run_gpu(b, "D2V37", 33, 31, tau, (rho, ux, uy, th, noise), 8, flags=b.LBM_THERMAL | b.LBM_COLL_PR)
    want = orc.collide(lat, orc.step(lat, f0, tau, 8, coll=orc.PR, thermal=True), tau, coll=orc.PR,
                       thermal=True)
    check(got["f"], want, 1e-12)


@pytest.mark.parametrize("name,nx,ny", [("D2Q9", 1, 1), ("D2Q9", 1, 7), ("D2V17", 3, 3), ("D2V37", 3, 5),
                                        ("D2V37", 65, 3)])
def test_fp64_minimum_grids(orc, b, name, nx, ny):
    """Grids as small as the stencil reach: every periodic wrap aliases."""
    say(f"fp64 minimum grid {name} {nx}x{ny}")
    lat = orc.lattice(name)
    rng = np.random.default_rng(nx * 100 + ny)
    rho = rng.uniform(0.9, 1.1, (ny, nx))
    ux, uy = rng.uniform(-0.05, 0.05, (2, ny, nx))
    noise = wl.uniform_noise(3, lat.Q, ny, nx)
    f0 = orc.init_populations(lat, rho, ux, uy, None, noise, 1e-3)
    got = run_gpu(b, name, nx, ny, 0.7, (rho, ux, uy, None, noise * (1e-3 / 1e-8)), 7)
    want = orc.collide(lat, orc.step(lat, f0, 0.7, 7), 0.7)
    check(got["f"], want, 1e-12)
    # the +-2 vorticity stencil wraps more than once on axes shorter than 2
    _, vx, vy, _ = orc.moments(lat, want)
    w = orc.vorticity(vx, vy)
    np.testing.assert_allclose(got["vort"], w, rtol=0, atol=1e-11)
    assert got["sums"][6] == pytest.approx(float(np.sum(w * w)), rel=1e-9, abs=1e-20)


def test_zero_steps_and_uniform_steady_state(orc, b):
    say("fp64 zero steps / uniform equilibrium")
    lat = orc.lattice("D2V37")
    n = 19
    rho, ux, uy = np.full((n, n), 1.1), np.full((n, n), 0.05), np.full((n, n), -0.03)
    f0 = orc.init_populations(lat, rho, ux, uy)
    g0 = run_gpu(b, "D2V37", n, n, 0.6, (rho, ux, uy, None, None), 0)
    # the collision rebuilds f from O(1) coefficients: a few ulps of 1
    check(g0["f"], f0, 5e-15)
    g = run_gpu(b, "D2V37", n, n, 0.6, (rho, ux, uy, None, None), 25)
    check(g["f"], f0, 5e-14)


def test_moments_and_diagnostics(orc, b):
    say("fp64 moments / vorticity / sums D2V17")
    lat, u0, tau, fields, f0 = shear_case(orc, "D2V17", 48, 40)
    got = run_gpu(b, "D2V17", 48, 40, tau, fields, 12)
    want = orc.collide(lat, orc.step(lat, f0, tau, 12), tau)
    # moments of populations that agree to 1e-12 agree to Q * 3 * 1e-12
    # (|c| <= 3); the fourth-order difference adds a factor 3
    check(got["f"], want, 1e-12)
    r, vx, vy, _ = orc.moments(lat, want)
    np.testing.assert_allclose(got["rho"], r, rtol=0, atol=2e-11)
    np.testing.assert_allclose(got["ux"], vx, rtol=0, atol=6e-11)
    np.testing.assert_allclose(got["uy"], vy, rtol=0, atol=6e-11)
    np.testing.assert_allclose(got["vort"], orc.vorticity(vx, vy), rtol=0, atol=2e-10)
    s = got["sums"]
    assert s[0] == pytest.approx(r.sum(), rel=1e-13)
    assert s[1] == pytest.approx(float((r * vx).sum()), abs=1e-12)
    assert s[4] == pytest.approx(float((vx ** 2 + vy ** 2).sum()), rel=1e-8)
    assert s[6] == pytest.approx(float((orc.vorticity(vx, vy) ** 2).sum()), rel=1e-8)
    assert s[8] == 0


def test_fp64_conservation_long_run(orc, b):
    say("fp64 conservation D2V37 96x96 x 400 steps")
    lat, u0, tau, fields, f0 = shear_case(orc, "D2V37", 96, 96, re=1e5)
    rho, ux, uy, _, noise = fields
    sim = b.Simulation("D2V37", 96, 96, tau, rho, ux, uy, noise=noise, noise_amp=1e-8)
    s0 = sim.moments()["sums"]
    sim.step(400)
    s1 = sim.moments()["sums"]
    sim.close()
    assert abs(s1[0] - s0[0]) <= 1e-13 * s0[0]
    scale = float(np.abs(rho * ux).sum())
    assert abs(s1[1] - s0[1]) <= 1e-13 * scale and abs(s1[2] - s0[2]) <= 1e-13 * scale


def test_fp64_d2v37_full_size_sampled(orc, b):
    """D2V37, 1024 x 1024, FP64, the benchmark's launch configuration: one
    init + 2 steps, checked at 512 sampled nodes the oracle evaluates one by
    one (gather the neighbours' post-collision values, collide)."""
    say("fp64 D2V37 1024^2 sampled nodes")
    import torch

    name, n, steps = "D2V37", 1024, 2
    lat = orc.lattice(name)
    u0, tau = wl.shear_layer_params(lat.cs2, n, 1e5)
    rho, ux, uy = wl.shear_layer_fields(n, n, u0)
    noise = wl.uniform_noise(1, lat.Q, n, n)
    sim = b.Simulation(name, n, n, tau, rho, ux, uy, noise=noise, noise_amp=1e-8)
    sim.step(steps)
    f = sim.populations()
    rng = np.random.default_rng(5)
    ys = np.concatenate([[0, n - 1, 3], rng.integers(0, n, 509)])
    xs = np.concatenate([[0, n - 1, n - 2], rng.integers(0, n, 509)])
    got = f[:, torch.as_tensor(ys, device=f.device), torch.as_tensor(xs, device=f.device)].cpu().numpy()
    sums = sim.moments()["sums"]
    sim.close()
    del f

    def post(ys_, xs_, t):
        """post-collision populations C(f^t) at the given nodes (t <= 2)."""
        if t == 0:
            f0 = orc.init_populations(lat, rho[ys_, xs_], ux[ys_, xs_], uy[ys_, xs_], None,
                                      noise[:, ys_, xs_], 1e-8)
            return orc.collide(lat, f0, tau)
        pre = np.empty((lat.Q, len(ys_)))
        for i, (cx, cy) in enumerate(lat.c):
            src = post((ys_ - cy) % n, (xs_ - cx) % n, t - 1)
            pre[i] = src[i]
        return orc.collide(lat, pre, tau)

    want = post(ys, xs, steps)
    check(got, want, 1e-13)
    assert sums[8] == 0
    mass0 = float(rho.sum()) + 1e-8 * float(lat.w @ noise.reshape(lat.Q, -1).sum(1))
    assert sums[0] == pytest.approx(mass0, rel=1e-13)


@pytest.mark.parametrize("name,coll,flags", [("D2Q9", "rr", 0), ("D2V17", "rr", 0), ("D2V37", "rr", 0),
                                             ("D2V37", "pr", 0), ("D2V37", "rr", "moments"),
                                             ("D2V17", "rr", "moments")])
def test_fp64_per_order_relaxation(orc, b, name, coll, flags):
    """Ranks 3 and 4 relaxed with their own times (lbm_set_relaxation)."""
    nx, ny, tau3, tau4 = 40, 36, 0.62, 0.9
    say(f"per-order relaxation {name} {coll} {flags or 'populations'}")
    lat, u0, tau, fields, f0 = shear_case(orc, name, nx, ny, re=3e3)
    rho, ux, uy, th, noise = fields
    fl = (b.LBM_COLL_PR if coll == "pr" else 0) | (b.LBM_STORE_MOMENTS if flags == "moments" else 0)
    sim = b.Simulation(name, nx, ny, tau, rho, ux, uy, noise=noise, noise_amp=1e-8, flags=fl)
    sim.set_relaxation(tau3, tau4)
    sim.step(10)
    got = sim.populations().cpu().numpy()
    sim.close()
    c = orc.PR if coll == "pr" else orc.RR
    if flags == "moments":
        # the state is the pre-collision moments: every rebuild, the first one
        # included, uses the times in force
        g = orc.step(lat, f0, tau, 10, coll=c, tau3=tau3, tau4=tau4)
    else:
        # the stored initial state is C(f0) with the single time (set_relaxation
        # comes after lbm_init)
        g = orc.stream(lat, orc.collide(lat, f0, tau, coll=c))
        g = orc.step(lat, g, tau, 9, coll=c, tau3=tau3, tau4=tau4)
    want = orc.collide(lat, g, tau, coll=c, tau3=tau3, tau4=tau4)
    check(got, want, 1e-12)
    assert np.abs(want - orc.collide(lat, orc.step(lat, f0, tau, 10, coll=c), tau, coll=c)).max() > 1e-10


def test_fp64_thermal_per_order_relaxation(orc, b):
    """Thermal D2V37 Sod with Pr = (tau - 1/2)/(tau3 - 1/2) = 0.5."""
    say("thermal per-order relaxation")
    lat = orc.lattice("D2V37")
    nx, ny, tau, tau3 = 400, 4, 0.6, 0.7
    rho, ux, uy, th = wl.sod_fields(nx, ny)
    sim = b.Simulation("D2V37", nx, ny, tau, rho, ux, uy, theta=th, flags=b.LBM_THERMAL)
    sim.set_relaxation(tau3, tau)
    sim.step(30)
    got = sim.populations().cpu().numpy()
    sim.close()
    f0 = orc.init_populations(lat, rho, ux, uy, th)
    g = orc.stream(lat, orc.collide(lat, f0, tau, thermal=True))
    g = orc.step(lat, g, tau, 29, thermal=True, tau3=tau3, tau4=tau)
    want = orc.collide(lat, g, tau, thermal=True, tau3=tau3, tau4=tau)
    check(got, want, 1e-11)


@pytest.mark.parametrize("name,flags", [("D2V37", 0), ("D2Q9", 0), ("D2V37", 0x2), ("D2V37", 0x4),
                                        ("D2V37", 0x1)])
def test_cache_policy_and_tile_order_do_not_change_results(orc, b, name, flags, monkeypatch):
    """The three cache policies of the 2D step (ordinary loads with
    non-temporal stores; ordinary loads and stores with the tile order
    reversed every other step; non-temporal loads with ordinary stores) give
    bitwise the same states: each node's update is independent of launch
    order, and the BF16 dither is keyed by node and step only."""
    say(f"cache policy / tile order {name} flags={flags:#x}")
    lat = orc.lattice(name)
    u0, tau = wl.shear_layer_params(lat.cs2, 96, 1e4)
    rho, ux, uy = wl.shear_layer_fields(96, 70, u0)
    noise = wl.uniform_noise(5, lat.Q, 70, 96)
    th = np.ones_like(rho) if flags & b.LBM_THERMAL else None
    out = []
    for pol in ("0", "1", "2"):
        monkeypatch.setenv("RRLBM_CACHE_POLICY", pol)
        sim = b.Simulation(name, 96, 70, tau, rho, ux, uy, theta=th, noise=noise, noise_amp=1e-8, flags=flags)
        sim.step(7)
        out.append(sim.populations().cpu().numpy())
        sim.close()
    np.testing.assert_array_equal(out[0], out[1])
    np.testing.assert_array_equal(out[0], out[2])
