"""3D part of the CPU reference (Table II lattices D3Q19, D3Q27, D3V39,
D3Q103, isothermal): ctypes access to ``rr_oracle3d.c``.

TEST INFRASTRUCTURE ONLY, like the rest of this package.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rr_oracle3d.c")
_LIB = os.path.join(_HERE, "liboracle3d.so")

LATTICES = {"D3Q19": 0, "D3Q27": 1, "D3V39": 2, "D3Q103": 3}
RR, PR, BGK = 0, 1, 2


def build(force: bool = False) -> str:
    """Compile rr_oracle3d.c into liboracle3d.so with gcc (FP64, no contraction)."""
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
        build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        i64 = ctypes.c_int64
        L.o3_lattice.argtypes = [ctypes.c_int, ip, ip, dp, ip, ip, ip, dp]
        L.o3_basis.argtypes = [ctypes.c_int, ctypes.c_int, ip]
        L.o3_hermite.argtypes = [ctypes.c_int, ctypes.c_int, dp]
        L.o3_equilibrium.argtypes = [ctypes.c_int, i64, dp, dp, dp, dp, dp]
        L.o3_noneq.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp]
        L.o3_collide.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, i64, dp, dp]
        L.o3_step.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double] + [ctypes.c_int] * 4 + [dp, dp]
        d = ctypes.c_double
        L.o3_collide_mrt.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, d, d, d, i64, dp, dp]
        L.o3_step_mrt.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, d, d, d] + [ctypes.c_int] * 4 + [dp, dp]
        L.o3_moments.argtypes = [ctypes.c_int, i64, dp, dp, dp, dp, dp]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle3d {what} failed ({rc})")


@dataclass
class Lattice3:
    name: str
    id: int
    Q: int
    nmax: int
    cs2: float
    c: np.ndarray  # (Q, 3) integers
    w: np.ndarray


def lattice(name: str) -> Lattice3:
    lid = LATTICES[name]
    Q, nmax = ctypes.c_int(), ctypes.c_int()
    cs2 = ctypes.c_double()
    cx, cy, cz = (np.zeros(103, dtype=np.int32) for _ in range(3))
    w = np.zeros(103)
    ip = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
    _check(lib().o3_lattice(lid, ctypes.byref(Q), ctypes.byref(nmax), ctypes.byref(cs2), ip(cx), ip(cy), ip(cz),
                            _p(w)), "lattice")
    q = Q.value
    c = np.stack([cx[:q], cy[:q], cz[:q]], axis=1).astype(np.int64)
    return Lattice3(name, lid, q, nmax.value, cs2.value, c, w[:q].copy())


def basis(lat: Lattice3, n: int) -> np.ndarray:
    """Mask over the rank-n tuples (base 3, digit k = index k, 0 x 1 y 2 z)."""
    m = np.zeros(3 ** n, dtype=np.int32)
    _check(lib().o3_basis(lat.id, n, m.ctypes.data_as(ctypes.POINTER(ctypes.c_int))), "basis")
    return m.astype(bool)


def hermite(lat: Lattice3, n: int) -> np.ndarray:
    H = np.zeros((lat.Q, 3 ** n))
    _check(lib().o3_hermite(lat.id, n, _p(H)), "hermite")
    return H


def equilibrium(lat: Lattice3, rho, ux, uy, uz) -> np.ndarray:
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    shape = rho.shape
    ux, uy, uz = (np.ascontiguousarray(np.broadcast_to(a, shape), dtype=np.float64) for a in (ux, uy, uz))
    out = np.zeros((lat.Q, rho.size))
    _check(lib().o3_equilibrium(lat.id, rho.size, _p(rho.reshape(-1)), _p(ux.reshape(-1)), _p(uy.reshape(-1)),
                                _p(uz.reshape(-1)), _p(out)), "equilibrium")
    return out.reshape((lat.Q,) + shape)


def noneq(lat: Lattice3, f_node, coll=RR) -> np.ndarray:
    """Non-equilibrium coefficients of one node, all ranks on full tuples
    (flat, rank n from offset (3^n - 1) / 2)."""
    f = np.ascontiguousarray(f_node, dtype=np.float64)
    a1 = np.zeros(1093)
    _check(lib().o3_noneq(lat.id, coll, _p(f), _p(a1)), "noneq")
    return a1


def collide(lat: Lattice3, f, tau, coll=RR, order=None, tau3=None, tau4=None) -> np.ndarray:
    """One collision; tau3 (rank 3) and tau4 (ranks >= 4) default to tau."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros_like(f)
    order = lat.nmax if order is None else order
    t3 = tau if tau3 is None else tau3
    t4 = tau if tau4 is None else tau4
    _check(lib().o3_collide_mrt(lat.id, coll, order, tau, t3, t4, f.size // lat.Q, _p(f), _p(out)), "collide")
    return out


def step(lat: Lattice3, f, tau, nsteps, coll=RR, order=None, tau3=None, tau4=None) -> np.ndarray:
    """nsteps of collide + periodic push stream; f has shape (Q, nz, ny, nx)."""
    f = np.array(f, dtype=np.float64, order="C", copy=True)
    _, nz, ny, nx = f.shape
    tmp = np.empty_like(f)
    order = lat.nmax if order is None else order
    t3 = tau if tau3 is None else tau3
    t4 = tau if tau4 is None else tau4
    _check(lib().o3_step_mrt(lat.id, coll, order, tau, t3, t4, nx, ny, nz, nsteps, _p(f), _p(tmp)), "step")
    return f


def moments(lat: Lattice3, f):
    f = np.ascontiguousarray(f, dtype=np.float64)
    shape = f.shape[1:]
    n = f.size // lat.Q
    r, ux, uy, uz = (np.zeros(n) for _ in range(4))
    _check(lib().o3_moments(lat.id, n, _p(f), _p(r), _p(ux), _p(uy), _p(uz)), "moments")
    return tuple(a.reshape(shape) for a in (r, ux, uy, uz))
