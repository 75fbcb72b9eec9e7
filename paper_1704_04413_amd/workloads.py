"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds no arithmetic of the lattice Boltzmann method: it only
builds the macroscopic initial fields of the paper's two test cases (the
doubly periodic shear layer of Sec. III.B, Eqs. MB_InitialState_ux/uy, and the
Sod tube of Sec. III.C) and seeded uniform noise.  Lattice constants (c_s^2)
are always supplied by the caller, so each side of a comparison uses its own.
"""
from __future__ import annotations

import numpy as np


def cell_centres(n: int) -> np.ndarray:
    """Dimensionless cell-centre coordinates (i + 1/2)/n, i = 0..n-1."""
    return (np.arange(n, dtype=np.float64) + 0.5) / n


def shear_layer_fields(nx: int, ny: int, u0: float, k: float = 80.0, delta: float = 0.05,
                       phase: float = 0.0):
    """Doubly periodic shear layer: rho = 1, two tanh shear layers at y = 1/4
    and 3/4 of width 1/k, transverse perturbation of relative amplitude delta.
    `phase` shifts the perturbation, sin(2 pi (x + 1/4 + phase)).
    Returns rho, ux, uy as float64 arrays indexed [y, x]."""
    x = cell_centres(nx)[None, :]
    y = cell_centres(ny)[:, None]
    ux = np.where(y <= 0.5, u0 * np.tanh(k * (y - 0.25)), u0 * np.tanh(k * (0.75 - y)))
    ux = np.broadcast_to(ux, (ny, nx)).copy()
    uy = np.broadcast_to(u0 * delta * np.sin(2.0 * np.pi * (x + 0.25 + phase)), (ny, nx)).copy()
    rho = np.ones((ny, nx))
    return rho, ux, uy


def shear_layer_gradients(nx: int, ny: int, u0: float, k: float = 80.0, delta: float = 0.05,
                          phase: float = 0.0):
    """Analytic velocity gradients of `shear_layer_fields` in lattice units
    (per node spacing): array [4, ny, nx] = (dux/dx, dux/dy, duy/dx, duy/dy)."""
    x = cell_centres(nx)[None, :]
    y = cell_centres(ny)[:, None]
    dux_dy = np.where(y <= 0.5, u0 * k / np.cosh(k * (y - 0.25)) ** 2, -u0 * k / np.cosh(k * (0.75 - y)) ** 2) / ny
    duy_dx = u0 * delta * 2.0 * np.pi * np.cos(2.0 * np.pi * (x + 0.25 + phase)) / nx
    g = np.zeros((4, ny, nx))
    g[1] = np.broadcast_to(dux_dy, (ny, nx))
    g[2] = np.broadcast_to(duy_dx, (ny, nx))
    return g


def shear_layer_params(cs2: float, n: int, re: float, mach: float = 0.1):
    """Characteristic speed u0 = Mach * c_s and the discrete relaxation time
    giving Re = u0 n / nu with nu = c_s^2 (tau - 1/2) (isothermal)."""
    u0 = mach * np.sqrt(cs2)
    nu = u0 * n / re
    return float(u0), float(0.5 + nu / cs2)


def sod_fields(nx: int, ny: int, rho_l=8.0, p_l=10.0, rho_r=1.0, p_r=1.0, x_split=None,
               theta_left=0.5):
    """Sod tube along x, periodic in y.  Cells i < x_split hold the left state,
    the rest the right state; u = 0.  Temperatures are scaled so the left
    state has theta = theta_left (0.5 makes the left adiabatic sound speed
    sqrt(gamma theta) c_s equal c_s for gamma = 2); the right state keeps the
    physical ratio T_R / T_L = (p_r / rho_r) / (p_l / rho_l).
    Returns rho, ux, uy, theta [y, x]."""
    x_split = nx // 2 if x_split is None else x_split
    theta_r = theta_left * (p_r / rho_r) / (p_l / rho_l)
    left = (np.arange(nx) < x_split)[None, :]
    rho = np.broadcast_to(np.where(left, rho_l, rho_r), (ny, nx)).astype(np.float64).copy()
    theta = np.broadcast_to(np.where(left, theta_left, theta_r), (ny, nx)).astype(np.float64).copy()
    zeros = np.zeros((ny, nx))
    return rho, zeros.copy(), zeros.copy(), theta


def uniform_noise(seed: int, q: int, ny: int, nx: int) -> np.ndarray:
    """U(-1, 1) samples of shape (q, ny, nx) from NumPy's PCG64 with `seed`."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-1.0, 1.0, size=(q, ny, nx))


def shear_layer_fields_3d(nx: int, ny: int, nz: int, u0: float, k: float = 80.0, delta: float = 0.05):
    """The doubly periodic shear layer extruded along z, with a second
    perturbation u_z = u0 delta sin(2 pi (z + x)) so that the flow is
    three-dimensional.  Returns rho, ux, uy, uz as float64 arrays [z, y, x]."""
    rho2, ux2, uy2 = shear_layer_fields(nx, ny, u0, k, delta)
    x = cell_centres(nx)[None, None, :]
    z = cell_centres(nz)[:, None, None]
    shape = (nz, ny, nx)
    ux = np.broadcast_to(ux2[None], shape).copy()
    uy = np.broadcast_to(uy2[None], shape).copy()
    uz = np.broadcast_to(u0 * delta * np.sin(2.0 * np.pi * (z + x)), shape).copy()
    return np.ones(shape), ux, uy, uz


def uniform_noise_3d(seed: int, q: int, nz: int, ny: int, nx: int) -> np.ndarray:
    """U(-1, 1) samples of shape (q, nz, ny, nx) from NumPy's PCG64 with `seed`."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-1.0, 1.0, size=(q, nz, ny, nx))


def batch_instances(seed: int = 0, count: int = 64):
    """The mixed batch workload: `count` shear-layer instances (lattice name,
    side, Re) with side uniform in {128, ..., 1024}, lattices D2Q9/D2V17/D2V37
    with probabilities 0.5/0.3/0.2 and Re log-uniform in [1e4, 1e6] (NumPy
    PCG64 with `seed`)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sides = np.array([128, 192, 256, 384, 512, 768, 1024])
    out = []
    for _ in range(count):
        n = int(rng.choice(sides))
        lat = str(rng.choice(["D2Q9", "D2V17", "D2V37"], p=[0.5, 0.3, 0.2]))
        re = float(10 ** rng.uniform(4, 6))
        out.append((lat, n, re))
    return out
