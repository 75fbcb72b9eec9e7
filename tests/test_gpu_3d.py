"""GPU parity of the 3D lattices (Table II: D3Q19, D3Q27, D3V39, D3Q103) against the
FP64 3D oracle, through the C-ABI.

As in 2D the library keeps the post-collision state, so after n steps its
populations equal the oracle's collide(step(f^0, n)).  Grids span two 64-wide
x blocks with a ragged tail and a row count (ny * nz) that is not a multiple
of the 4-row tile.  Both sides compute in double in different association
orders; one step moves each population by a few ulps of |f| <= 1, tested at
1e-12 after at most 12 steps.
"""
import math

import numpy as np
import pytest

from paper_1704_04413_amd import workloads as wl

pytestmark = pytest.mark.gpu

NAMES = ["D3Q19", "D3Q27", "D3V39", "D3Q103"]


@pytest.fixture(scope="module")
def b():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1704_04413_amd import binding

    binding.lib()
    return binding


@pytest.fixture(scope="module")
def o3d():
    from oracle import o3d as m

    m.build()
    return m


def say(msg):
    print(f"[case] {msg}", flush=True)


def check(got, want, atol):
    err = float(np.abs(np.asarray(got) - np.asarray(want)).max())
    print(f"[parity] max |gpu - oracle| = {err:.3e} (bound {atol:.0e})", flush=True)
    assert err <= atol, err


def case(o3d, name, nx, ny, nz, seed=0, amp=1e-6, mach=0.1):
    lat = o3d.lattice(name)
    u0 = mach * math.sqrt(lat.cs2)
    rho, ux, uy, uz = wl.shear_layer_fields_3d(nx, ny, nz, u0, k=20.0, delta=0.1)
    noise = wl.uniform_noise_3d(seed, lat.Q, nz, ny, nx)
    f0 = o3d.equilibrium(lat, rho, ux, uy, uz) + amp * lat.w[:, None, None, None] * noise
    return lat, (rho, ux, uy, uz, noise), f0


def run_gpu(b, name, dims, tau, fields, steps, flags=0, order=None, amp=1e-6):
    nx, ny, nz = dims
    rho, ux, uy, uz, noise = fields
    sim = b.Simulation3D(name, nx, ny, nz, tau, rho, ux, uy, uz, noise=noise, noise_amp=amp, flags=flags,
                         reg_order=order)
    sim.step(steps)
    f = sim.populations().cpu().numpy()
    mom = sim.moments()
    out = dict(f=f, steps=sim.steps, sums=mom["sums"],
               **{k: mom[k].cpu().numpy() for k in ("rho", "ux", "uy", "uz")})
    sim.close()
    return out


COLLS = {"RR": (0, 0), "PR": (1, 0x10), "BGK": (2, 0x20)}


@pytest.mark.parametrize("name", NAMES)
@pytest.mark.parametrize("coll", ["RR", "PR", "BGK"])
def test_3d_populations(o3d, b, name, coll):
    dims, steps, tau = (70, 5, 3), 8, 0.52
    say(f"3D {coll} {name} {dims} steps={steps}")
    lat, fields, f0 = case(o3d, name, *dims)
    ocoll, flags = COLLS[coll]
    got = run_gpu(b, name, dims, tau, fields, steps, flags=flags)
    want = o3d.collide(lat, o3d.step(lat, f0, tau, steps, coll=ocoll), tau, coll=ocoll)
    assert got["steps"] == steps
    check(got["f"], want, 1e-12)


@pytest.mark.parametrize("name,order", [("D3Q19", 2), ("D3Q27", 2), ("D3Q27", 3), ("D3Q27", 4), ("D3Q27", 5),
                                        ("D3V39", 2), ("D3Q103", 2), ("D3Q103", 3)])
def test_3d_lower_orders(o3d, b, name, order):
    dims, steps, tau = (66, 4, 4), 6, 0.6
    say(f"3D RR order {order} {name} {dims}")
    lat, fields, f0 = case(o3d, name, *dims, seed=1)
    got = run_gpu(b, name, dims, tau, fields, steps, order=order)
    want = o3d.collide(lat, o3d.step(lat, f0, tau, steps, order=order), tau, order=order)
    check(got["f"], want, 1e-12)


@pytest.mark.parametrize("name", NAMES)
def test_3d_moments_and_sums(o3d, b, name):
    dims, steps, tau = (64, 4, 5), 5, 0.55
    say(f"3D moments {name} {dims}")
    lat, fields, f0 = case(o3d, name, *dims, seed=2)
    got = run_gpu(b, name, dims, tau, fields, steps)
    want = o3d.collide(lat, o3d.step(lat, f0, tau, steps), tau)
    r, ux, uy, uz = o3d.moments(lat, want)
    for k, v in (("rho", r), ("ux", ux), ("uy", uy), ("uz", uz)):
        check(got[k], v, 1e-13)
    c = lat.c.astype(float)
    n = r.size
    s = got["sums"]
    assert s[0] == pytest.approx(r.sum(), rel=1e-13)
    for a, u in enumerate((ux, uy, uz)):
        assert s[1 + a] == pytest.approx(float((r * u).sum()), abs=1e-13 * n)
    e = 0.5 * float(np.sum((c ** 2).sum(1)[:, None, None, None] * want))
    assert s[4] == pytest.approx(e, rel=1e-13)
    u2 = ux ** 2 + uy ** 2 + uz ** 2
    assert s[5] == pytest.approx(float(u2.sum()), rel=1e-12)
    assert s[6] == pytest.approx(float((u2 ** 2).sum()), rel=1e-12)
    assert s[7] == 0
    # mass and momentum are collision and streaming invariants
    assert s[0] == pytest.approx(float(f0.sum()), rel=1e-14)


@pytest.mark.parametrize("name", NAMES)
def test_3d_second_order_start(o3d, b, name):
    """LBM_EQ_INIT_ORDER2: f^(0) truncated at rank 2, w_i rho (1 + c.u/c_s^2
    + (c.u)^2/(2 c_s^4) - u^2/(2 c_s^2)), written here from the lattice
    tables; the library's state after init is its collision."""
    dims = (65, 3, 3)
    say(f"3D order-2 start {name} {dims}")
    lat, fields, _ = case(o3d, name, *dims, seed=3)
    rho, ux, uy, uz, noise = fields
    c = lat.c.astype(float)
    cu = c[:, 0, None, None, None] * ux + c[:, 1, None, None, None] * uy + c[:, 2, None, None, None] * uz
    u2 = ux ** 2 + uy ** 2 + uz ** 2
    cs2 = lat.cs2
    f0 = lat.w[:, None, None, None] * rho * (1 + cu / cs2 + cu ** 2 / (2 * cs2 ** 2) - u2 / (2 * cs2))
    f0 = f0 + 1e-6 * lat.w[:, None, None, None] * noise
    got = run_gpu(b, name, dims, 0.7, fields, 3, flags=b.LBM_EQ_INIT_ORDER2)
    want = o3d.collide(lat, o3d.step(lat, f0, 0.7, 3), 0.7)
    check(got["f"], want, 1e-12)


@pytest.mark.parametrize("name", NAMES)
def test_3d_minimum_grid(o3d, b, name):
    """Every dimension at the lattice reach (the pull wraps once per axis)."""
    lat = o3d.lattice(name)
    reach = int(np.abs(lat.c).max())
    dims = (reach, reach, reach)
    say(f"3D minimum grid {name} {dims}")
    lat, fields, f0 = case(o3d, name, *dims, seed=4)
    got = run_gpu(b, name, dims, 0.8, fields, 7)
    want = o3d.collide(lat, o3d.step(lat, f0, 0.8, 7), 0.8)
    check(got["f"], want, 1e-12)


def test_3d_contexts_reject_2d_calls(b):
    say("3D context rejects 2D-only calls")
    n = 4 * 4 * 4
    z = np.zeros((4, 4, 4))
    sim = b.Simulation3D("D3Q19", 4, 4, 4, 0.7, np.ones((4, 4, 4)), z, z, z)
    with pytest.raises(b.LbmError):
        b.lbm_moments(sim.ctx)
    with pytest.raises(b.LbmError):
        b.lbm_batch_create([sim.ctx])
    sim.step(2)
    assert sim.steps == 2
    m = sim.moments()
    assert m["sums"][0] == pytest.approx(n, rel=1e-14)
    sim.close()


@pytest.mark.parametrize("name", NAMES)
def test_3d_shear_wave_decay_full_size(b, name):
    """At 128^3 (the size the 3D benchmark lines time): a shear wave
    u_x = U sin(2 pi y / ny) decays at nu = c_s^2 (tau - 1/2), a property of
    the method that holds at any size (the oracle is not run here)."""
    n, tau = 128, 0.8
    say(f"3D shear wave {name} {n}^3")
    _, _, _, cs2 = b.lbm_lattice_info(name)
    U = 1e-4 * math.sqrt(cs2)
    y = (np.arange(n) + 0.5) / n
    ux = np.broadcast_to((U * np.sin(2 * np.pi * y))[None, :, None], (n, n, n)).copy()
    z = np.zeros((n, n, n))
    sim = b.Simulation3D(name, n, n, n, tau, np.ones((n, n, n)), ux, z, z)
    wave = np.sin(2 * np.pi * y)

    def amp():
        vx = sim.moments(sums=False)["ux"].cpu().numpy()
        return 2.0 / n * float(np.mean(vx, axis=(0, 2)) @ wave)

    sim.step(50)
    a1 = amp()
    sim.step(400)
    a2 = amp()
    sim.close()
    k = 2 * np.pi / n
    nu = math.log(a1 / a2) / (400 * k * k)
    assert nu == pytest.approx(cs2 * (tau - 0.5), rel=0.01)


@pytest.mark.parametrize("name,flags", [("D3Q19", 0), ("D3V39", 0), ("D3Q19", 0x20), ("D3Q27", 0x20)])
def test_3d_cache_policies_give_the_same_states(o3d, b, name, flags, monkeypatch):
    """The three cache policies of the RR and BGK steps (streaming; ordinary
    loads and stores with the tile order reversed every other step;
    non-temporal loads with ordinary stores) give bitwise the same
    populations."""
    dims = (66, 6, 5)
    say(f"3D cache policies {name} flags={flags:#x} {dims}")
    lat, fields, _ = case(o3d, name, *dims, seed=7)
    out = []
    for pol in ("0", "1", "2"):
        monkeypatch.setenv("RRLBM_CACHE_POLICY", pol)
        out.append(run_gpu(b, name, dims, 0.6, fields, 5, flags=flags)["f"])
    np.testing.assert_array_equal(out[0], out[1])
    np.testing.assert_array_equal(out[0], out[2])


@pytest.mark.parametrize("name,coll,order", [("D3Q27", "RR", 6), ("D3Q27", "RR", 4), ("D3V39", "RR", 3),
                                             ("D3Q103", "RR", 4), ("D3Q27", "PR", 6), ("D3Q19", "RR", 3)])
def test_3d_per_order_relaxation(o3d, b, name, coll, order):
    """lbm_set_relaxation on a 3D context: rank 3 relaxes with tau3, every rank
    >= 4 with tau4 (oracle: o3_step_mrt), from the next step on."""
    dims, tau, tau3, tau4, steps = (66, 5, 3), 0.8, 0.62, 1.3, 6
    say(f"3D per-order relaxation {coll} {name} order {order}")
    lat, fields, f0 = case(o3d, name, *dims, seed=8)
    ocoll, flags = COLLS[coll]
    rho, ux, uy, uz, noise = fields
    sim = b.Simulation3D(name, *dims, tau, rho, ux, uy, uz, noise=noise, noise_amp=1e-6, flags=flags,
                         reg_order=order)
    sim.set_relaxation(tau3, tau4)
    sim.step(steps)
    got = sim.populations().cpu().numpy()
    sim.close()
    # the initial state is collided with the single time (the times are set
    # after init); every step then streams and collides with the per-order
    # times: S_n = C'(stream(C'(... stream(S_0)))) = C'(step'(stream(S_0), n - 1))
    s0 = o3d.collide(lat, f0, tau, ocoll, order)
    streamed = np.empty_like(s0)
    for i in range(lat.Q):  # push streaming: f_i(x + c_i) = s0_i(x)
        streamed[i] = np.roll(s0[i], shift=(int(lat.c[i, 2]), int(lat.c[i, 1]), int(lat.c[i, 0])), axis=(0, 1, 2))
    want = o3d.collide(lat, o3d.step(lat, streamed, tau, steps - 1, ocoll, order, tau3=tau3, tau4=tau4), tau, ocoll,
                       order, tau3=tau3, tau4=tau4)
    check(got, want, 1e-12)
