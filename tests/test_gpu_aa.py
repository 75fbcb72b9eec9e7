"""The single-buffer scheme (LBM_SCHEME_AA) through the C-ABI.

It computes the same explicit step of Sec. III.A as the two-buffer pull
step, only with each post-collision value kept in another slot of one
buffer (the slot depends on the parity of the step count), so:
  - FP64 states after even and odd step counts agree with the FP64 oracle to
    the pull step's bound (1e-12 after <= 50 steps, see test_gpu_parity);
  - for every storage, collision and the thermal form, the populations, the
    fields and the sums equal those of the pull step bit for bit (same
    arithmetic, same node keys and step numbers for the BF16 dither), with
    every cache policy, on ragged grids and on grids as small as the
    stencil reach (where the periodic wraps alias);
  - checkpoints taken after even and odd step counts resume bit for bit;
  - the same on the 3D lattices of Table II (RR, PR and BGK).
"""
import math

import numpy as np
import pytest

from paper_1704_04413_amd import workloads as wl

pytestmark = pytest.mark.gpu

AA = 0x800


@pytest.fixture(scope="module")
def b():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1704_04413_amd import binding

    binding.lib()
    assert binding.LBM_SCHEME_AA == AA
    return binding


def say(msg):
    print(f"[case] {msg}", flush=True)


def fields_for(b, name, nx, ny, flags, re=1e4, seed=0):
    q, _, _, cs2 = b.lbm_lattice_info(name)
    u0, tau = wl.shear_layer_params(cs2, max(nx, ny), re)
    rho, ux, uy = wl.shear_layer_fields(nx, ny, u0)
    th = None
    if flags & b.LBM_THERMAL:
        th = 1.0 + 0.05 * np.cos(2 * np.pi * np.arange(nx) / nx)[None, :] * np.ones((ny, 1))
    noise = wl.uniform_noise(seed, q, ny, nx)
    return tau, (rho, ux, uy, th, noise)


def run(b, name, nx, ny, tau, fields, flags, steps, relax=None, order=None):
    rho, ux, uy, th, noise = fields
    sim = b.Simulation(name, nx, ny, tau, rho, ux, uy, theta=th, noise=noise, noise_amp=1e-8, flags=flags,
                       reg_order=order)
    assert len(sim.bufs) == (1 if flags & AA else 2)
    if relax:
        sim.set_relaxation(*relax)
    sim.step(steps)
    mom = sim.moments()
    out = dict(f=sim.populations().cpu().numpy(), sums=np.asarray(mom["sums"]),
               **{k: mom[k].cpu().numpy() for k in ("rho", "ux", "uy", "theta", "vort")})
    assert sim.steps == steps
    sim.close()
    return out


def assert_same(got, want):
    for k in ("f", "rho", "ux", "uy", "theta", "vort"):
        np.testing.assert_array_equal(got[k], want[k], err_msg=k)
    np.testing.assert_array_equal(got["sums"], want["sums"])


@pytest.mark.parametrize("name", ["D2Q9", "D2V17", "D2V37"])
@pytest.mark.parametrize("steps", [0, 1, 6, 7])
def test_aa_fp64_matches_oracle(orc, b, name, steps):
    """150 x 37: three 64-wide tile columns (the last ragged) and a ragged
    last row of tiles."""
    nx, ny = 150, 37
    say(f"AA fp64 {name} {nx}x{ny} steps={steps} against the oracle")
    lat = orc.lattice(name)
    eq = 2 if name == "D2Q9" else None
    u0, tau = wl.shear_layer_params(lat.cs2, nx, 1e4)
    rho, ux, uy = wl.shear_layer_fields(nx, ny, u0)
    noise = wl.uniform_noise(0, lat.Q, ny, nx)
    f0 = orc.init_populations(lat, rho, ux, uy, None, noise, 1e-8, eq_order=eq)
    flags = AA | (b.LBM_EQ_INIT_ORDER2 if eq == 2 else 0)
    got = run(b, name, nx, ny, tau, (rho, ux, uy, None, noise), flags, steps)
    want = orc.collide(lat, orc.step(lat, f0, tau, steps), tau)
    err = float(np.abs(got["f"] - want).max())
    print(f"[parity] max |gpu - oracle| = {err:.3e} (bound 1e-12)", flush=True)
    assert err <= 1e-12, err
    r, vx, vy, _ = orc.moments(lat, want)
    np.testing.assert_allclose(got["rho"], r, rtol=0, atol=1e-11)
    np.testing.assert_allclose(got["ux"], vx, rtol=0, atol=1e-11)
    np.testing.assert_allclose(got["uy"], vy, rtol=0, atol=1e-11)


SCHEME_CASES = [
    ("D2V37", 0), ("D2V37", 0x2), ("D2V37", 0x4), ("D2V37", 0x2 | 0x400),
    ("D2V37", 0x1), ("D2V37", 0x1 | 0x200), ("D2V37", 0x1 | 0x10), ("D2V37", 0x1 | 0x20),
    ("D2V37", 0x10), ("D2V37", 0x20), ("D2Q9", 0x2), ("D2Q9", 0x4), ("D2V17", 0), ("D2V17", 0x4),
]


@pytest.mark.parametrize("name,flags", SCHEME_CASES)
@pytest.mark.parametrize("policy", ["0", "1", "2"])
def test_aa_equals_pull_bitwise(b, name, flags, policy, monkeypatch):
    nx, ny, steps = 97, 70, 5
    say(f"AA vs pull {name} flags={flags:#x} policy={policy} {nx}x{ny}")
    tau, fields = fields_for(b, name, nx, ny, flags)
    relax = (0.61, 0.7) if not flags & b.LBM_COLL_BGK else None
    monkeypatch.setenv("RRLBM_CACHE_POLICY", policy)
    for s in (steps - 1, steps):  # both placements of the state
        want = run(b, name, nx, ny, tau, fields, flags, s, relax=relax)
        got = run(b, name, nx, ny, tau, fields, flags | AA, s, relax=relax)
        assert_same(got, want)


@pytest.mark.parametrize("name,nx,ny", [("D2Q9", 1, 1), ("D2Q9", 2, 7), ("D2V17", 3, 3), ("D2V37", 3, 5),
                                        ("D2V37", 65, 3)])
def test_aa_minimum_grids(b, name, nx, ny):
    """Grids as small as the reach: x + c_i and x - c_i wrap onto the same
    nodes for several i, and a node may read and write its own slots through
    the wrap; each slot still belongs to one thread."""
    say(f"AA minimum grid {name} {nx}x{ny}")
    tau, fields = fields_for(b, name, nx, ny, 0)
    for s in (6, 7):
        assert_same(run(b, name, nx, ny, tau, fields, AA, s), run(b, name, nx, ny, tau, fields, 0, s))


@pytest.mark.parametrize("name,n,flags", [("D2V37", 768, 0), ("D2V37", 1024, 0), ("D2V37", 1024, 0x2),
                                          ("D2V17", 1024, 0)])
def test_aa_full_size_bitwise(b, name, n, flags):
    """Sizes where one buffer fits the memory-side cache and where it does
    not (D2V37 FP64 1024^2, 296 MiB), compared whole on the GPU."""
    import torch

    say(f"AA vs pull full size {name} {n}x{n} flags={flags:#x}")
    tau, (rho, ux, uy, _, noise) = fields_for(b, name, n, n, 0, re=3e4)
    res = []
    for fl in (flags, flags | AA):
        sim = b.Simulation(name, n, n, tau, rho, ux, uy, noise=noise, noise_amp=1e-8, flags=fl)
        sim.step(3)
        res.append(sim.populations())
        sim.close()
    assert torch.equal(res[0], res[1])


@pytest.mark.parametrize("flags", [0, 0x4, 0x1])
@pytest.mark.parametrize("k", [3, 4])
def test_aa_checkpoint_resume(b, flags, k):
    import torch

    name, n, total = "D2V37", 70, 9
    say(f"AA checkpoint D2V37 flags={flags:#x} {k}+{total - k} steps")
    tau, fields = fields_for(b, name, n, n, flags)
    want = run(b, name, n, n, tau, fields, flags | AA, total)
    rho, ux, uy, th, noise = fields
    first = b.Simulation(name, n, n, tau, rho, ux, uy, theta=th, noise=noise, noise_amp=1e-8, flags=flags | AA)
    first.step(k)
    host = first.save()
    dev = torch.empty(b.lbm_checkpoint_bytes(first.ctx), dtype=torch.uint8, device="cuda")
    b.lbm_save(first.ctx, dev)
    first.close()
    for buf in (host, dev):
        second = b.Simulation(name, n, n, tau, rho, ux, uy, theta=th, noise=noise * 2, noise_amp=1e-8,
                              flags=flags | AA)
        second.load(buf)
        assert second.steps == k
        second.step(total - k)
        np.testing.assert_array_equal(second.populations().cpu().numpy(), want["f"])
        second.close()
    # the slots differ from the two-buffer state's: another scheme rejects it
    other = b.Simulation(name, n, n, tau, rho, ux, uy, theta=th, noise=noise, noise_amp=1e-8, flags=flags)
    with pytest.raises(b.LbmError) as e:
        other.load(host)
    assert e.value.code == b.LBM_EINVAL
    other.close()


def test_aa_rejected_by_batches_and_closure(b):
    say("AA contexts in a batch / with the closure")
    tau, (rho, ux, uy, _, noise) = fields_for(b, "D2V37", 64, 64, 0)
    sim = b.Simulation("D2V37", 64, 64, tau, rho, ux, uy, noise=noise, noise_amp=1e-8, flags=AA)
    with pytest.raises(b.LbmError) as e:
        b.lbm_batch_create([sim.ctx])
    assert e.value.code == b.LBM_EINVAL
    import torch

    x = torch.zeros(1 << 16, dtype=torch.float32, device="cuda")
    with pytest.raises(b.LbmError) as e:
        b.lbm_closure_samples(sim.ctx, 2, x, x)
    assert e.value.code == b.LBM_EINVAL
    sim.close()


# ---------------------------------------------------------------- 3D lattices

NAMES_3D = ["D3Q19", "D3Q27", "D3V39", "D3Q103"]
COLLS_3D = {"RR": (0, 0), "PR": (1, 0x10), "BGK": (2, 0x20)}


def fields_3d(b, name, dims, seed=0, mach=0.1):
    nx, ny, nz = dims
    q, _, _, cs2 = b.lbm_lattice_info(name)
    rho, ux, uy, uz = wl.shear_layer_fields_3d(nx, ny, nz, mach * math.sqrt(cs2), k=20.0, delta=0.1)
    return rho, ux, uy, uz, wl.uniform_noise_3d(seed, q, nz, ny, nx)


def run_3d(b, name, dims, tau, fields, flags, steps, relax=None, order=None):
    rho, ux, uy, uz, noise = fields
    sim = b.Simulation3D(name, *dims, tau, rho, ux, uy, uz, noise=noise, noise_amp=1e-6, flags=flags,
                         reg_order=order)
    assert len(sim.bufs) == (1 if flags & AA else 2)
    if relax:
        sim.set_relaxation(*relax)
    sim.step(steps)
    mom = sim.moments()
    out = dict(f=sim.populations().cpu().numpy(), sums=np.asarray(mom["sums"]),
               **{k: mom[k].cpu().numpy() for k in ("rho", "ux", "uy", "uz")})
    assert sim.steps == steps
    sim.close()
    return out


def assert_same_3d(got, want):
    for k in ("f", "rho", "ux", "uy", "uz", "sums"):
        np.testing.assert_array_equal(got[k], want[k], err_msg=k)


@pytest.mark.parametrize("name", NAMES_3D)
@pytest.mark.parametrize("steps", [5, 6])
def test_aa_3d_matches_oracle(b, name, steps):
    """70 x 5 x 3: two 64-wide x blocks with a ragged tail, 15 rows (not a
    multiple of the 4-row tile)."""
    from oracle import o3d

    o3d.build()
    dims, tau = (70, 5, 3), 0.52
    say(f"AA 3D RR {name} {dims} steps={steps} against the oracle")
    lat = o3d.lattice(name)
    rho, ux, uy, uz, noise = fields_3d(b, name, dims)
    f0 = o3d.equilibrium(lat, rho, ux, uy, uz) + 1e-6 * lat.w[:, None, None, None] * noise
    got = run_3d(b, name, dims, tau, (rho, ux, uy, uz, noise), AA, steps)
    want = o3d.collide(lat, o3d.step(lat, f0, tau, steps), tau)
    err = float(np.abs(got["f"] - want).max())
    print(f"[parity] max |gpu - oracle| = {err:.3e} (bound 1e-12)", flush=True)
    assert err <= 1e-12, err


@pytest.mark.parametrize("name", NAMES_3D)
@pytest.mark.parametrize("coll", ["RR", "PR", "BGK"])
def test_aa_3d_equals_pull_bitwise(b, name, coll):
    dims = (66, 6, 5)
    say(f"AA vs pull 3D {name} {coll} {dims}")
    fields = fields_3d(b, name, dims, seed=3)
    flags = COLLS_3D[coll][1]
    relax = (0.62, 0.9) if coll != "BGK" else None
    for s in (4, 5):
        assert_same_3d(run_3d(b, name, dims, 0.6, fields, flags | AA, s, relax=relax),
                       run_3d(b, name, dims, 0.6, fields, flags, s, relax=relax))


F32D = 0x2 | 0x400


@pytest.mark.parametrize("name", NAMES_3D)
@pytest.mark.parametrize("storage", ["fp64", "fp32d"])
@pytest.mark.parametrize("policy", ["0", "1", "2"])
def test_aa_3d_policies(b, name, storage, policy, monkeypatch):
    """Ordinary stores (1), non-temporal ones (0), non-temporal ones in the
    steps that write a node's own slots only (2): the same states as the
    pull step, bit for bit."""
    dims = (66, 6, 5)
    say(f"AA 3D {name} {storage} policy {policy}")
    fields = fields_3d(b, name, dims, seed=4)
    flags = F32D if storage == "fp32d" else 0
    want = run_3d(b, name, dims, 0.6, fields, flags, 7)
    monkeypatch.setenv("RRLBM_CACHE_POLICY", policy)
    assert_same_3d(run_3d(b, name, dims, 0.6, fields, flags | AA, 7), want)


@pytest.mark.parametrize("coll", ["PR", "BGK"])
def test_aa_3d_nontemporal_other_collisions(b, coll, monkeypatch):
    dims = (66, 6, 5)
    say(f"AA 3D D3Q19 {coll} policy 0")
    fields = fields_3d(b, "D3Q19", dims, seed=8)
    flags = COLLS_3D[coll][1]
    want = run_3d(b, "D3Q19", dims, 0.6, fields, flags, 5)
    monkeypatch.setenv("RRLBM_CACHE_POLICY", "0")
    assert_same_3d(run_3d(b, "D3Q19", dims, 0.6, fields, flags | AA, 5), want)


@pytest.mark.parametrize("name,storage", [("D3V39", "fp64"), ("D3Q103", "fp64"), ("D3Q103", "fp32d"),
                                          ("D3V39", "fp32d")])
def test_aa_3d_full_size_bitwise(b, name, storage):
    """128^3, the size the 3D lines of the benchmark time, with the default
    policy: non-temporal stores for the buffers above 512 MiB (D3V39 FP64,
    624 MiB; D3Q103 1648 and 824 MiB), ordinary ones below (D3V39 FP32,
    312 MiB).  Three in-place steps against three pull steps, every value and
    the FP64 sums compared on the GPU."""
    import torch

    n = 128
    flags = F32D if storage == "fp32d" else 0
    say(f"AA vs pull 3D full size {name} {storage} {n}^3")
    q, _, _, cs2 = b.lbm_lattice_info(name)
    rho, ux, uy, uz = wl.shear_layer_fields_3d(n, n, n, 0.1 * math.sqrt(cs2))
    out = []
    for fl in (flags | AA, flags):
        sim = b.Simulation3D(name, n, n, n, 0.51, rho, ux, uy, uz, flags=fl)
        sim.step(3)
        out.append((sim.populations(), np.asarray(sim.moments()["sums"])))
        sim.close()
    assert torch.equal(out[0][0], out[1][0])
    np.testing.assert_array_equal(out[0][1], out[1][1])
    assert out[0][1][7] == 0  # no non-finite node


@pytest.mark.parametrize("name,dims", [("D3Q19", (1, 1, 1)), ("D3Q27", (2, 1, 3)), ("D3V39", (3, 3, 3)),
                                       ("D3Q103", (3, 4, 3))])
def test_aa_3d_minimum_grids(b, name, dims):
    say(f"AA 3D minimum grid {name} {dims}")
    fields = fields_3d(b, name, dims, seed=5)
    for s in (6, 7):
        assert_same_3d(run_3d(b, name, dims, 0.7, fields, AA, s), run_3d(b, name, dims, 0.7, fields, 0, s))


@pytest.mark.parametrize("k", [2, 3])
def test_aa_3d_checkpoint_resume(b, k):
    name, dims, total = "D3Q19", (12, 12, 12), 5
    say(f"AA 3D checkpoint {name} {k}+{total - k} steps")
    fields = fields_3d(b, name, dims, seed=6)
    rho, ux, uy, uz, noise = fields
    want = run_3d(b, name, dims, 0.7, fields, AA, total)["f"]
    first = b.Simulation3D(name, *dims, 0.7, rho, ux, uy, uz, noise=noise, noise_amp=1e-6, flags=AA)
    first.step(k)
    buf = first.save()
    first.close()
    second = b.Simulation3D(name, *dims, 0.7, rho, ux, uy, uz, flags=AA)
    second.load(buf)
    assert second.steps == k
    second.step(total - k)
    np.testing.assert_array_equal(second.populations().cpu().numpy(), want)
    second.close()


@pytest.mark.parametrize("steps", [4, 5])
def test_aa_noalloc_moments(b, steps):
    """The allocation-free diagnostics read the single-buffer state through
    the same placement as lbm_moments, at both parities."""
    import torch

    name, n = "D2V37", 90
    say(f"AA noalloc moments {name} {n}x{n} steps={steps}")
    tau, (rho, ux, uy, _, noise) = fields_for(b, name, n, n, 0)
    sim = b.Simulation(name, n, n, tau, rho, ux, uy, noise=noise, noise_amp=1e-8, flags=AA)
    sim.step(steps)
    mk = lambda: torch.empty((n, n), dtype=torch.float64, device="cuda")
    want, got = [mk() for _ in range(5)], [mk() for _ in range(5)]
    s_want = b.lbm_moments(sim.ctx, *want, sums=True)
    s_got = b.lbm_moments_noalloc(sim.ctx, *got, sums=True)
    for w, g in zip(want, got):
        assert torch.equal(w, g)
    np.testing.assert_array_equal(s_got, s_want)
    sim.close()
