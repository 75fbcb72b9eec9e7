"""CPU reference ("oracle") for the recursive-regularized LBM step.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this package; the product library never does.

The arithmetic of the method lives in ``rr_oracle.c`` (plain C, FP64, no
FMA contraction); this module loads it through ctypes and adds the pieces of
the harness that are not part of the step: the flow diagnostics of Sec. III.B
(kinetic energy, enstrophy from a fourth-order centred difference, the
stability criterion) and the exact Riemann solution used for the Sod tube of
Sec. III.C.  It shares no code with the HIP library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rr_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

D2Q9, D2V17, D2V37 = 0, 1, 2
RR, PR, BGK = 0, 1, 2
LATTICES = {"D2Q9": D2Q9, "D2V17": D2V17, "D2V37": D2V37}


def build(force: bool = False) -> str:
    """Compile rr_oracle.c into liboracle.so with gcc (FP64, no contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        i64 = ctypes.c_int64
        L.orc_lattice.argtypes = [ctypes.c_int, ip, ip, dp, ip, ip, dp]
        L.orc_basis.argtypes = [ctypes.c_int, ip]
        L.orc_hermite_table.argtypes = [ctypes.c_int, dp]
        L.orc_eq_coeffs.argtypes = [ctypes.c_int] + [ctypes.c_double] * 4 + [dp]
        L.orc_noneq_coeffs.argtypes = [ctypes.c_int] * 4 + [dp, dp]
        L.orc_recursion.argtypes = [ctypes.c_int] + [ctypes.c_double] * 5 + [dp, dp]
        L.orc_equilibrium.argtypes = [ctypes.c_int, ctypes.c_int, i64, dp, dp, dp, dp, dp]
        L.orc_noneq_init.argtypes = [ctypes.c_int, ctypes.c_int, i64, dp, dp, dp, dp, ctypes.c_double, dp]
        L.orc_collide.argtypes = [ctypes.c_int] * 5 + [ctypes.c_double, i64, dp, dp]
        L.orc_step.argtypes = [ctypes.c_int] * 5 + [ctypes.c_double] + [ctypes.c_int] * 3 + [dp, dp]
        L.orc_collide_mrt.argtypes = [ctypes.c_int] * 5 + [ctypes.c_double] * 3 + [i64, dp, dp]
        L.orc_step_mrt.argtypes = [ctypes.c_int] * 5 + [ctypes.c_double] * 3 + [ctypes.c_int] * 3 + [dp, dp]
        L.orc_moments.argtypes = [ctypes.c_int, ctypes.c_int, i64, dp, dp, dp, dp]
        L.orc_threads.argtypes = []
        L.orc_closure_inputs.argtypes = [ctypes.c_int, ctypes.c_double, i64, dp, dp, dp]
        L.orc_collide_closure.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, i64, dp, dp, dp]
        L.orc_noneq_projected.argtypes = [ctypes.c_int, i64, dp, dp]
        _lib = L
    return _lib


def threads() -> int:
    """Host threads the oracle's parallel loops use."""
    return int(lib().orc_threads())


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


@dataclass(frozen=True)
class Lattice:
    id: int
    name: str
    Q: int
    n_eq: int
    cs2: float
    c: np.ndarray  # (Q, 2) integer velocities, canonical order (ascending c_y, then c_x)
    w: np.ndarray  # (Q,) weights
    basis: np.ndarray  # (5, 5) basis[nx, ny]

    @property
    def reach(self) -> int:
        return int(np.abs(self.c).max())


def lattice(name_or_id) -> Lattice:
    lid = LATTICES[name_or_id] if isinstance(name_or_id, str) else int(name_or_id)
    Q, n_eq, cs2 = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
    cx = (ctypes.c_int * 37)()
    cy = (ctypes.c_int * 37)()
    w = (ctypes.c_double * 37)()
    _check(lib().orc_lattice(lid, ctypes.byref(Q), ctypes.byref(n_eq), ctypes.byref(cs2), cx, cy, w),
           "lattice")
    q = Q.value
    bas = (ctypes.c_int * 25)()
    _check(lib().orc_basis(lid, bas), "basis")
    name = {v: k for k, v in LATTICES.items()}[lid]
    return Lattice(lid, name, q, n_eq.value, cs2.value,
                   np.array([[cx[i], cy[i]] for i in range(q)], dtype=np.int64),
                   np.array([w[i] for i in range(q)]),
                   np.array(list(bas), dtype=np.int64).reshape(5, 5))


def toff(n: int, b: int) -> int:
    """Slot of the rank-n tensor component whose index pattern is b (bit j = y)."""
    return (1 << n) - 1 + b


def hermite_table(lat: Lattice) -> np.ndarray:
    H = np.zeros(lat.Q * 31)
    _check(lib().orc_hermite_table(lat.id, _p(H)), "hermite_table")
    return H.reshape(lat.Q, 31)


def eq_coeffs(lat: Lattice, rho, ux, uy, theta=1.0) -> np.ndarray:
    a0 = np.zeros(31)
    _check(lib().orc_eq_coeffs(lat.id, rho, ux, uy, theta, _p(a0)), "eq_coeffs")
    return a0


def noneq_coeffs(lat: Lattice, f, coll=RR, thermal=False, a13_raw=False) -> np.ndarray:
    f = np.ascontiguousarray(f, dtype=np.float64)
    a1 = np.zeros(31)
    _check(lib().orc_noneq_coeffs(lat.id, coll, int(thermal), int(a13_raw), _p(f), _p(a1)),
           "noneq_coeffs")
    return a1


def recursion(thermal, rho, ux, uy, theta, cs2, a0, a1_in) -> np.ndarray:
    a0 = np.ascontiguousarray(a0, dtype=np.float64)
    a1 = np.array(a1_in, dtype=np.float64)
    _check(lib().orc_recursion(int(thermal), rho, ux, uy, theta, cs2, _p(a0), _p(a1)), "recursion")
    return a1


def equilibrium(lat: Lattice, rho, ux, uy, theta=None, order=None) -> np.ndarray:
    """Equilibrium populations, shape (Q,) + rho.shape, truncated at `order`
    (default: the lattice's full order)."""
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    shape = rho.shape
    ux = np.ascontiguousarray(np.broadcast_to(ux, shape), dtype=np.float64)
    uy = np.ascontiguousarray(np.broadcast_to(uy, shape), dtype=np.float64)
    th = None if theta is None else np.ascontiguousarray(np.broadcast_to(theta, shape), dtype=np.float64)
    n = rho.size
    out = np.zeros((lat.Q, n))
    order = lat.n_eq if order is None else order
    _check(lib().orc_equilibrium(lat.id, order, n, _p(rho.reshape(-1)), _p(ux.reshape(-1)),
                                 _p(uy.reshape(-1)), None if th is None else _p(th.reshape(-1)),
                                 _p(out)), "equilibrium")
    return out.reshape((lat.Q,) + shape)


def collide(lat: Lattice, f, tau, coll=RR, order=None, thermal=False, a13_raw=False, tau3=None,
            tau4=None) -> np.ndarray:
    """Post-collision populations; tau3, tau4 relax ranks 3 and 4 on their own
    (default tau)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    n = f.size // lat.Q
    out = np.zeros_like(f)
    order = lat.n_eq if order is None else order
    t3, t4 = (tau if tau3 is None else tau3), (tau if tau4 is None else tau4)
    _check(lib().orc_collide_mrt(lat.id, coll, order, int(thermal), int(a13_raw), tau, t3, t4, n, _p(f),
                                 _p(out)), "collide")
    return out


def noneq_init(lat: Lattice, rho, ux, uy, grad, tau, order=None) -> np.ndarray:
    """f^(1) of the isothermal initial state from velocity gradients
    grad[4, ...] = (dux/dx, dux/dy, duy/dx, duy/dy) (Sec. III.B, App. C)."""
    order = lat.n_eq if order is None else order
    rho, ux, uy = (np.ascontiguousarray(a, dtype=np.float64) for a in (rho, ux, uy))
    g = np.ascontiguousarray(grad, dtype=np.float64).reshape(4, -1)
    n = rho.size
    f1 = np.zeros((lat.Q, n))
    _check(lib().orc_noneq_init(lat.id, order, n, _p(rho), _p(ux), _p(uy), _p(g), tau, _p(f1)), "noneq_init")
    return f1.reshape((lat.Q,) + rho.shape)


def init_populations(lat: Lattice, rho, ux, uy, theta=None, noise=None, noise_amp=0.0,
                     eq_order=None, grad=None, tau=None) -> np.ndarray:
    """f = f^(0) (truncated at eq_order) [+ f^(1) from the velocity gradients
    `grad` at relaxation time `tau`, same truncation] + noise_amp * w_i * noise_i."""
    f = equilibrium(lat, rho, ux, uy, theta, eq_order)
    if grad is not None:
        if theta is not None:
            raise ValueError("the f^(1) initial state is isothermal")
        f = f + noneq_init(lat, rho, ux, uy, grad, tau, eq_order)
    if noise is not None:
        f = f + noise_amp * lat.w.reshape((-1,) + (1,) * (f.ndim - 1)) * noise
    return np.ascontiguousarray(f)


def step(lat: Lattice, f, tau, nsteps, coll=RR, order=None, thermal=False, a13_raw=False, tau3=None,
         tau4=None) -> np.ndarray:
    """nsteps of collide + periodic push stream; f has shape (Q, ny, nx);
    tau3, tau4 relax ranks 3 and 4 on their own (default tau)."""
    f = np.array(f, dtype=np.float64, order="C", copy=True)
    _, ny, nx = f.shape
    tmp = np.empty_like(f)
    order = lat.n_eq if order is None else order
    t3, t4 = (tau if tau3 is None else tau3), (tau if tau4 is None else tau4)
    _check(lib().orc_step_mrt(lat.id, coll, order, int(thermal), int(a13_raw), tau, t3, t4, nx, ny, nsteps,
                              _p(f), _p(tmp)), "step")
    return f


def moments(lat: Lattice, f, thermal=False):
    f = np.ascontiguousarray(f, dtype=np.float64)
    shape = f.shape[1:]
    n = f.size // lat.Q
    rho, ux, uy, th = (np.zeros(n) for _ in range(4))
    _check(lib().orc_moments(lat.id, int(thermal), n, _p(f), _p(rho), _p(ux), _p(uy), _p(th)),
           "moments")
    r = [a.reshape(shape) for a in (rho, ux, uy, th)]
    return r[0], r[1], r[2], r[3]


def closure_inputs(lat: Lattice, f, tau):
    """(feat[7, n], rr[9, n]) of pre-collision populations f (Q, ...):
    feat = (rho-1, ux, uy, |u|^2/cs2, ahat_xx, ahat_xy, ahat_yy), rr = ahat of
    the plain recursive a1^(3..4) in the order 30,21,12,03,40,31,22,13,04."""
    f = np.ascontiguousarray(f, dtype=np.float64).reshape(lat.Q, -1)
    n = f.shape[1]
    feat, rr = np.zeros((7, n)), np.zeros((9, n))
    _check(lib().orc_closure_inputs(lat.id, tau, n, _p(f), _p(feat), _p(rr)), "closure_inputs")
    return feat, rr


def noneq_projected(lat: Lattice, f) -> np.ndarray:
    """a1 by projection, (12, n): xx, xy, yy, 30, 21, 12, 03, 40, 31, 22, 13, 04."""
    f = np.ascontiguousarray(f, dtype=np.float64).reshape(lat.Q, -1)
    out = np.zeros((12, f.shape[1]))
    _check(lib().orc_noneq_projected(lat.id, f.shape[1], _p(f), _p(out)), "noneq_projected")
    return out


def stream(lat: Lattice, g) -> np.ndarray:
    """Periodic push streaming of (Q, ny, nx) populations: f_i(x + c_i) = g_i(x)."""
    return np.stack([np.roll(g[i], shift=(int(lat.c[i, 1]), int(lat.c[i, 0])), axis=(0, 1))
                     for i in range(lat.Q)])


def collide_closure(lat: Lattice, f, tau, resid, order=None) -> np.ndarray:
    """Isothermal RR collision with a residual resid[9, n] (a_hat scaling)
    added to a1^(3..4)."""
    shape = f.shape
    f = np.ascontiguousarray(f, dtype=np.float64).reshape(lat.Q, -1)
    n = f.shape[1]
    resid = np.ascontiguousarray(resid, dtype=np.float64).reshape(9, n)
    out = np.zeros_like(f)
    order = lat.n_eq if order is None else order
    _check(lib().orc_collide_closure(lat.id, order, tau, n, _p(f), _p(resid), _p(out)), "collide_closure")
    return out.reshape(shape)


# ---- diagnostics of Sec. III.B ---------------------------------------------

def ddx4(g, axis):
    """Periodic fourth-order centred first derivative (grid spacing 1)."""
    return (-np.roll(g, -2, axis) + 8.0 * np.roll(g, -1, axis)
            - 8.0 * np.roll(g, 1, axis) + np.roll(g, 2, axis)) / 12.0


def vorticity(ux, uy):
    """omega = d(uy)/dx - d(ux)/dy on arrays indexed [y, x]."""
    return ddx4(uy, 1) - ddx4(ux, 0)


def flow_stats(ux, uy, u0, L):
    """Kinetic energy 0.5|u|^2/u0^2 and enstrophy 0.5 omega^2 (L/u0)^2:
    spatial mean and standard deviation of each."""
    ke = 0.5 * (ux * ux + uy * uy) / (u0 * u0)
    w = vorticity(ux, uy)
    en = 0.5 * w * w * (L / u0) ** 2
    return dict(ke_mean=float(ke.mean()), ke_std=float(ke.std()),
                ens_mean=float(en.mean()), ens_std=float(en.std()))


# ---- exact Riemann solution (Sod tube, Sec. III.C) ------------------------

def riemann_exact(rhoL, pL, uL, rhoR, pR, uR, gamma, xi):
    """Exact solution of the 1D Euler Riemann problem at similarity
    coordinates xi = (x - x0)/t, for an ideal gas with ratio gamma.
    Star pressure by Newton iteration on the pressure function (shock:
    Rankine-Hugoniot branch, rarefaction: isentropic branch).
    Returns rho, u, p arrays."""
    g = gamma
    cL, cR = np.sqrt(g * pL / rhoL), np.sqrt(g * pR / rhoR)

    def fK(p, rhoK, pK, cK):
        if p > pK:
            A = 2.0 / ((g + 1.0) * rhoK)
            B = (g - 1.0) / (g + 1.0) * pK
            s = np.sqrt(A / (p + B))
            return (p - pK) * s, s * (1.0 - 0.5 * (p - pK) / (p + B))
        r = p / pK
        return (2.0 * cK / (g - 1.0) * (r ** ((g - 1.0) / (2.0 * g)) - 1.0),
                1.0 / (rhoK * cK) * r ** (-(g + 1.0) / (2.0 * g)))

    p = max(1e-8, 0.5 * (pL + pR))
    for _ in range(100):
        f1, d1 = fK(p, rhoL, pL, cL)
        f2, d2 = fK(p, rhoR, pR, cR)
        dp = (f1 + f2 + (uR - uL)) / (d1 + d2)
        pn = max(1e-12, p - dp)
        if abs(pn - p) < 1e-14 * (pn + p):
            p = pn
            break
        p = pn
    f1, _ = fK(p, rhoL, pL, cL)
    f2, _ = fK(p, rhoR, pR, cR)
    us = 0.5 * (uL + uR) + 0.5 * (f2 - f1)
    ps = p

    xi = np.asarray(xi, dtype=np.float64)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    pr = np.empty_like(xi)
    gm = (g - 1.0) / (g + 1.0)
    for k, s in np.ndenumerate(xi):
        if s <= us:  # left of the contact
            if ps > pL:
                SL = uL - cL * np.sqrt((g + 1.0) / (2 * g) * ps / pL + (g - 1.0) / (2 * g))
                if s <= SL:
                    rho[k], u[k], pr[k] = rhoL, uL, pL
                else:
                    rho[k] = rhoL * (ps / pL + gm) / (gm * ps / pL + 1.0)
                    u[k], pr[k] = us, ps
            else:
                csL = cL * (ps / pL) ** ((g - 1.0) / (2 * g))
                SH, ST = uL - cL, us - csL
                if s <= SH:
                    rho[k], u[k], pr[k] = rhoL, uL, pL
                elif s >= ST:
                    rho[k] = rhoL * (ps / pL) ** (1.0 / g)
                    u[k], pr[k] = us, ps
                else:
                    c = 2.0 / (g + 1.0) * (cL + (g - 1.0) / 2.0 * (uL - s))
                    u[k] = 2.0 / (g + 1.0) * (cL + (g - 1.0) / 2.0 * uL + s)
                    rho[k] = rhoL * (c / cL) ** (2.0 / (g - 1.0))
                    pr[k] = pL * (c / cL) ** (2.0 * g / (g - 1.0))
        else:  # right of the contact
            if ps > pR:
                SR = uR + cR * np.sqrt((g + 1.0) / (2 * g) * ps / pR + (g - 1.0) / (2 * g))
                if s >= SR:
                    rho[k], u[k], pr[k] = rhoR, uR, pR
                else:
                    rho[k] = rhoR * (ps / pR + gm) / (gm * ps / pR + 1.0)
                    u[k], pr[k] = us, ps
            else:
                csR = cR * (ps / pR) ** ((g - 1.0) / (2 * g))
                SH, ST = uR + cR, us + csR
                if s >= SH:
                    rho[k], u[k], pr[k] = rhoR, uR, pR
                elif s <= ST:
                    rho[k] = rhoR * (ps / pR) ** (1.0 / g)
                    u[k], pr[k] = us, ps
                else:
                    c = 2.0 / (g + 1.0) * (cR - (g - 1.0) / 2.0 * (uR - s))
                    u[k] = 2.0 / (g + 1.0) * (-cR + (g - 1.0) / 2.0 * uR + s)
                    rho[k] = rhoR * (c / cR) ** (2.0 / (g - 1.0))
                    pr[k] = pR * (c / cR) ** (2.0 * g / (g - 1.0))
    return rho, u, pr, ps, us
