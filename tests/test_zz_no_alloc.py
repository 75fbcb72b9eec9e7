"""The allocation-free diagnostics entry point (lbm_moments_noalloc) through
the C-ABI against lbm_moments on the same state: fields and sums bit for bit,
on two calls in a row (the second on a smaller grid, so the shared scratch
holds stale partial sums beyond the new grid), for population and moment
storage; and its argument and size checks."""
import numpy as np
import pytest

from paper_1704_04413_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1704_04413_amd import binding

    binding.lib()
    return binding, torch


def shear(b, lattice, nx, ny, flags, steps):
    q, _, _, cs2 = b.lbm_lattice_info(lattice)
    u0, tau = wl.shear_layer_params(cs2, max(nx, ny), 3e4)
    rho, ux, uy = wl.shear_layer_fields(nx, ny, u0)
    theta = np.ones_like(rho) if flags & b.LBM_THERMAL else None
    sim = b.Simulation(lattice, nx, ny, tau, rho, ux, uy, theta=theta, noise=wl.uniform_noise(1, q, ny, nx),
                       noise_amp=1e-8, flags=flags)
    sim.step(steps)
    return sim


def both(b, torch, sim):
    mk = lambda: torch.full((sim.ny, sim.nx), np.nan, dtype=torch.float64, device="cuda")
    want = [mk() for _ in range(5)]
    s_want = b.lbm_moments(sim.ctx, *want, sums=True)
    got = [mk() for _ in range(5)]
    s_got = b.lbm_moments_noalloc(sim.ctx, *got, sums=True)
    for g, w in zip(got, want):
        assert torch.equal(g, w)
    assert np.array_equal(s_got, s_want), (s_got, s_want)
    return s_got


@pytest.mark.parametrize("lattice,flags", [("D2V37", 0), ("D2V37", 0x1), ("D2Q9", 0x2), ("D2V17", 0x8)])
def test_noalloc_matches_moments_twice(env, lattice, flags):
    b, torch = env
    print(f"[case] noalloc {lattice} flags={flags:#x} 300x260 then 70x45", flush=True)
    big = shear(b, lattice, 300, 260, flags, 6)
    s1 = both(b, torch, big)
    assert s1[8] == 0 and s1[0] > 0
    big.close()
    small = shear(b, lattice, 70, 45, flags, 3)
    both(b, torch, small)
    # fields only, no sums and no vorticity: ux, uy may be omitted
    r = torch.empty((45, 70), dtype=torch.float64, device="cuda")
    b.lbm_moments_noalloc(small.ctx, rho=r)
    r2 = torch.empty_like(r)
    b.lbm_moments(small.ctx, rho=r2)
    assert torch.equal(r, r2)
    small.close()


def test_noalloc_rejections(env):
    b, torch = env
    print("[case] noalloc argument and size checks", flush=True)
    s = shear(b, "D2Q9", 32, 32, 0, 1)
    with pytest.raises(b.LbmError):
        b.lbm_moments_noalloc(s.ctx, sums=True)  # sums need ux, uy
    s.close()
    n = 4100  # 4100^2 > LBM_NOALLOC_MAX_NODES
    assert n * n > b.LBM_NOALLOC_MAX_NODES
    big = shear(b, "D2Q9", n, n, b.LBM_STORE_BF16, 0)
    ux = torch.empty((n, n), dtype=torch.float64, device="cuda")
    uy = torch.empty_like(ux)
    with pytest.raises(b.LbmError, match="allocation-free limit"):
        b.lbm_moments_noalloc(big.ctx, ux=ux, uy=uy, sums=True)
    big.close()
