"""CPU-side checks of the C-ABI library: it loads, exports every symbol the
header declares, reports the same lattice constants as the oracle (two
independent tables of Table I), and rejects invalid arguments before touching
the GPU."""
import os
import re

import numpy as np
import pytest

from paper_1704_04413_amd import binding as b

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "rrlbm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = b.lib()
    syms = declared_symbols()
    assert syms, "no declarations parsed"
    assert sorted(syms) == sorted(b.EXPORTS)
    for s in syms:
        assert hasattr(L, s), s


@pytest.mark.parametrize("name", ["D2Q9", "D2V17", "D2V37"])
def test_lattice_tables_agree_with_oracle(orc, name):
    lat = orc.lattice(name)
    q, reach, n_eq, cs2 = b.lbm_lattice_info(name)
    assert (q, reach, n_eq) == (lat.Q, lat.reach, lat.n_eq)
    assert cs2 == pytest.approx(lat.cs2, rel=2e-16)
    cx, cy, w = b.lbm_lattice_velocities(name)
    np.testing.assert_array_equal(np.stack([cx, cy], 1), lat.c)
    # D2V17's closed-form weights lose a few ulps to cancellation when the
    # oracle evaluates them in double; the library holds 25-digit decimals
    np.testing.assert_allclose(w, lat.w, rtol=1e-14, atol=0)


def test_buffer_elems_cover_the_grid():
    for name in ("D2Q9", "D2V17", "D2V37"):
        q = b.lbm_lattice_info(name)[0]
        for nx, ny in ((1, 1), (3, 3), (128, 128), (1000, 7), (1024, 1024)):
            assert b.lbm_buffer_elems(name, nx, ny) >= q * nx * ny
            assert b.lbm_buffer_elems(name, nx, ny, b.LBM_STORE_MOMENTS) == 6 * nx * ny
    # thermal moment state: rho, u, theta, a1^(2), a1^(3)
    assert b.lbm_buffer_elems("D2V37", 9, 5, b.LBM_STORE_MOMENTS | b.LBM_THERMAL) == 11 * 9 * 5
    with pytest.raises(b.LbmError):
        b.lbm_buffer_elems(7, 4, 4)
    with pytest.raises(b.LbmError):
        b.lbm_buffer_elems("D2Q9", 0, 4)


class FakePtr:
    """Non-null pointer stand-in: validation fails before anything is dereferenced."""

    def __init__(self, v):
        self.v = v

    def data_ptr(self):
        return self.v


@pytest.mark.parametrize("args,code", [
    (dict(lattice=9), b.LBM_EINVAL),
    (dict(lattice=b.LBM_D3Q19), b.LBM_EINVAL),      # 3D lattices go through lbm_init_3d
    (dict(nx=2), b.LBM_EINVAL),                     # below the D2V37 reach
    (dict(ny=0), b.LBM_EINVAL),
    (dict(tau=0.5), b.LBM_ETAU),
    (dict(tau=float("nan")), b.LBM_ETAU),
    (dict(reg_order=5), b.LBM_EINVAL),
    (dict(reg_order=1), b.LBM_EINVAL),
    (dict(flags=b.LBM_STORE_FP32 | b.LBM_STORE_BF16), b.LBM_EINVAL),
    (dict(flags=b.LBM_COLL_PR | b.LBM_COLL_BGK), b.LBM_EINVAL),
    (dict(flags=1 << 20), b.LBM_EINVAL),
    (dict(lattice=0, flags=b.LBM_THERMAL), b.LBM_EINVAL),  # thermal needs D2V37
    (dict(lattice=1, reg_order=4), b.LBM_EINVAL),          # D2V17 stops at rank 3
    (dict(same_buffers=True), b.LBM_EINVAL),
    (dict(no_rho=True), b.LBM_EINVAL),
    (dict(flags=b.LBM_THERMAL, grad=True), b.LBM_EINVAL),  # the f^(1) start is isothermal
    (dict(flags=b.LBM_STORE_MOMENTS | b.LBM_STORE_FP32), b.LBM_EINVAL),
    (dict(flags=b.LBM_STORE_MOMENTS | b.LBM_COLL_PR), b.LBM_EINVAL),  # moments: RR only
    (dict(flags=b.LBM_STORE_MOMENTS | b.LBM_COLL_BGK), b.LBM_EINVAL),
    (dict(lattice=0, flags=b.LBM_STORE_MOMENTS | b.LBM_THERMAL), b.LBM_EINVAL),  # thermal needs D2V37
    (dict(flags=b.LBM_SCHEME_AA), b.LBM_EINVAL),                     # one buffer: f_b must be NULL
    (dict(flags=b.LBM_SCHEME_AA, no_fb=True, no_fa=True), b.LBM_EINVAL),
    (dict(flags=b.LBM_SCHEME_AA | b.LBM_STORE_MOMENTS, no_fb=True), b.LBM_EINVAL),  # populations only
    (dict(no_fb=True), b.LBM_EINVAL),                                # two buffers without the flag
])
def test_init_rejects_invalid_arguments(args, code):
    p = dict(lattice=2, nx=8, ny=8, tau=0.6, reg_order=4, flags=0)
    p.update({k: v for k, v in args.items() if k in p})
    fa, fb = FakePtr(0x1000), FakePtr(0x2000)
    if args.get("same_buffers"):
        fb = fa
    if args.get("no_fb"):
        fb = None
    if args.get("no_fa"):
        fa = None
    rho = None if args.get("no_rho") else FakePtr(0x3000)
    with pytest.raises(b.LbmError) as e:
        b.lbm_init(p["lattice"], p["nx"], p["ny"], p["tau"], p["reg_order"], p["flags"], fa, fb, rho,
                   FakePtr(0x4000), FakePtr(0x5000), grad=FakePtr(0x6000) if args.get("grad") else None)
    assert e.value.code == code
    assert b.lbm_last_error()


def test_null_context_is_rejected():
    for fn in (lambda: b.lbm_step(None, 1), lambda: b.lbm_moments(None), lambda: b.lbm_populations(None, None),
               lambda: b.lbm_set_relaxation(None, 0.7, 0.7)):
        with pytest.raises(b.LbmError):
            fn()
    b.lbm_destroy(None)
    assert b.lbm_step_count(None) == -1


def test_batch_rejects_invalid_arguments():
    for args in (([], 64, 4), ([None], 64, 4), ([None], 32, 4), ([None], 64, 0), ([None], 64, 17)):
        with pytest.raises(b.LbmError) as e:
            b.lbm_batch_create(*args)
        assert e.value.code == b.LBM_EINVAL
    for fn in (lambda: b.lbm_batch_step(None, 1), lambda: b.lbm_batch_config(None),
               lambda: b.lbm_batch_autotune(None, 4)):
        with pytest.raises(b.LbmError):
            fn()
    b.lbm_batch_destroy(None)


# ---------------------------------------------------------------- 3D

@pytest.mark.parametrize("name", ["D3Q19", "D3Q27", "D3V39", "D3Q103"])
def test_3d_lattice_tables_agree_with_oracle(name):
    from oracle import o3d

    lat = o3d.lattice(name)
    q, reach, n_eq, cs2 = b.lbm_lattice_info(name)
    assert (q, n_eq) == (lat.Q, lat.nmax)
    assert reach == int(np.abs(lat.c).max())
    assert cs2 == pytest.approx(lat.cs2, rel=2e-16)
    cx, cy, cz, w = b.lbm_lattice_velocities_3d(name)
    np.testing.assert_array_equal(np.stack([cx, cy, cz], 1), lat.c)
    np.testing.assert_allclose(w, lat.w, rtol=1e-15, atol=0)
    with pytest.raises(b.LbmError):
        b.lbm_lattice_velocities(name)
    with pytest.raises(b.LbmError):
        b.lbm_lattice_velocities_3d("D2Q9")


def test_3d_buffer_elems():
    for name in ("D3Q19", "D3Q27", "D3V39", "D3Q103"):
        q = b.lbm_lattice_info(name)[0]
        for nx, ny, nz in ((1, 1, 1), (3, 5, 7), (64, 64, 64), (128, 128, 128)):
            n = b.lbm_buffer_elems_3d(name, nx, ny, nz)
            assert n >= q * nx * ny * nz
            assert n == q * nx * (-(-(ny * nz) // 4) * 4)
        # FP32 storage (with double arithmetic) holds the same number of elements
        assert b.lbm_buffer_elems_3d(name, 4, 4, 4, b.LBM_STORE_FP32 | b.LBM_MATH_FP64) == \
            b.lbm_buffer_elems_3d(name, 4, 4, 4)
        for fl in (b.LBM_STORE_BF16, b.LBM_STORE_MOMENTS):
            with pytest.raises(b.LbmError):
                b.lbm_buffer_elems_3d(name, 4, 4, 4, fl)
        with pytest.raises(b.LbmError):
            b.lbm_buffer_elems(name, 4, 4)
    with pytest.raises(b.LbmError):
        b.lbm_buffer_elems_3d("D2V37", 4, 4, 4)
    with pytest.raises(b.LbmError):
        b.lbm_buffer_elems_3d("D3Q19", 4, 0, 4)


@pytest.mark.parametrize("args,code", [
    (dict(lattice=b.LBM_D2V37), b.LBM_EINVAL),
    (dict(lattice=9), b.LBM_EINVAL),
    (dict(nz=2), b.LBM_EINVAL),                       # below the D3V39 reach
    (dict(nx=0), b.LBM_EINVAL),
    (dict(nx=1 << 14, ny=1 << 14, nz=4), b.LBM_EINVAL),  # layout beyond 2^31 elements
    (dict(tau=0.5), b.LBM_ETAU),
    (dict(reg_order=4), b.LBM_EINVAL),                # D3V39 stops at rank 3
    (dict(reg_order=1), b.LBM_EINVAL),
    (dict(flags=b.LBM_STORE_FP32), b.LBM_EINVAL),                    # FP32 storage computes in double
    (dict(flags=b.LBM_MATH_FP64), b.LBM_EINVAL),
    (dict(flags=b.LBM_STORE_BF16 | b.LBM_MATH_FP64), b.LBM_EINVAL),
    (dict(flags=b.LBM_THERMAL), b.LBM_EINVAL),
    (dict(flags=b.LBM_COLL_PR | b.LBM_COLL_BGK), b.LBM_EINVAL),
    (dict(same_buffers=True), b.LBM_EINVAL),
    (dict(no_uz=True), b.LBM_EINVAL),
    (dict(flags=b.LBM_SCHEME_AA), b.LBM_EINVAL),                      # one buffer: f_b must be NULL
    (dict(flags=b.LBM_SCHEME_AA, no_fb=True, no_fa=True), b.LBM_EINVAL),
    (dict(no_fb=True), b.LBM_EINVAL),                                 # two buffers without the flag
])
def test_init_3d_rejects_invalid_arguments(args, code):
    p = dict(lattice=b.LBM_D3V39, nx=8, ny=8, nz=8, tau=0.6, reg_order=3, flags=0)
    p.update({k: v for k, v in args.items() if k in p})
    fa, fb = FakePtr(0x1000), FakePtr(0x2000)
    if args.get("same_buffers"):
        fb = fa
    if args.get("no_fb"):
        fb = None
    if args.get("no_fa"):
        fa = None
    uz = None if args.get("no_uz") else FakePtr(0x6000)
    with pytest.raises(b.LbmError) as e:
        b.lbm_init_3d(p["lattice"], p["nx"], p["ny"], p["nz"], p["tau"], p["reg_order"], p["flags"], fa, fb,
                      FakePtr(0x3000), FakePtr(0x4000), FakePtr(0x5000), uz)
    assert e.value.code == code
    assert b.lbm_last_error()


def test_3d_calls_reject_null_context():
    with pytest.raises(b.LbmError):
        b.lbm_moments_3d(None)
