"""ctypes binding of librrlbm.so (the C-ABI of include/rrlbm.h).

Functions keep the C names and only marshal arguments: device arrays are
torch tensors on the GPU (passed by data pointer), streams are torch streams.
Every step of the method runs in the HIP library; there is no fallback, and
loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

LIB_PATH = os.environ.get("RRLBM_LIB") or os.path.join(os.path.dirname(os.path.abspath(__file__)), "librrlbm.so")

LBM_D2Q9, LBM_D2V17, LBM_D2V37 = 0, 1, 2
LBM_D3Q19, LBM_D3Q27, LBM_D3V39, LBM_D3Q103 = 3, 4, 5, 6
LATTICES = {"D2Q9": LBM_D2Q9, "D2V17": LBM_D2V17, "D2V37": LBM_D2V37,
            "D3Q19": LBM_D3Q19, "D3Q27": LBM_D3Q27, "D3V39": LBM_D3V39, "D3Q103": LBM_D3Q103}
LBM_THERMAL = 0x1
LBM_STORE_FP32 = 0x2
LBM_STORE_BF16 = 0x4
LBM_STORE_MOMENTS = 0x8
LBM_COLL_PR = 0x10
LBM_COLL_BGK = 0x20
LBM_EQ_INIT_ORDER2 = 0x100
LBM_A13_PROJECTED = 0x200
LBM_MATH_FP64 = 0x400
LBM_SCHEME_AA = 0x800
LBM_NSUMS = 10
LBM_NSUMS_3D = 8

LBM_OK, LBM_EINVAL, LBM_ETAU, LBM_EDEVICE, LBM_ENOMEM = 0, -1, -2, -3, -4

# every symbol declared in include/rrlbm.h
EXPORTS = ["lbm_lattice_info", "lbm_lattice_velocities", "lbm_buffer_elems", "lbm_init", "lbm_step",
           "lbm_step_count", "lbm_set_relaxation", "lbm_moments", "lbm_populations", "lbm_destroy", "lbm_last_error",
           "lbm_batch_create", "lbm_batch_step", "lbm_batch_autotune", "lbm_batch_config", "lbm_batch_destroy",
           "lbm_closure_samples", "lbm_mlp_stats", "lbm_mlp_normalize", "lbm_mlp_create", "lbm_mlp_forward",
           "lbm_mlp_step", "lbm_mlp_destroy", "lbm_closure_set", "lbm_closure_fallbacks",
           "lbm_lattice_velocities_3d", "lbm_buffer_elems_3d", "lbm_init_3d", "lbm_moments_3d",
           "lbm_checkpoint_bytes", "lbm_save", "lbm_load", "lbm_moments_noalloc"]
LBM_NOALLOC_MAX_NODES = 1 << 24
LBM_MLP_NPARAM = 5776
LBM_MLP_NNORM = 96


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"librrlbm error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load librrlbm.so (raises if it is missing: there is no other path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
        L = ctypes.CDLL(LIB_PATH)
        vp, dp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)
        L.lbm_lattice_info.argtypes = [ctypes.c_int, ip, ip, ip, dp]
        L.lbm_lattice_velocities.argtypes = [ctypes.c_int, ip, ip, dp]
        L.lbm_buffer_elems.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint32]
        L.lbm_buffer_elems.restype = ctypes.c_int64
        L.lbm_init.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                               ctypes.c_int, ctypes.c_uint32, vp, vp, vp, vp, vp, vp, vp, vp, ctypes.c_double, vp]
        L.lbm_step.argtypes = [vp, ctypes.c_int]
        L.lbm_set_relaxation.argtypes = [vp, ctypes.c_double, ctypes.c_double]
        L.lbm_step_count.argtypes = [vp]
        L.lbm_step_count.restype = ctypes.c_int64
        L.lbm_moments.argtypes = [vp, vp, vp, vp, vp, vp, dp]
        L.lbm_moments_noalloc.argtypes = [vp, vp, vp, vp, vp, vp, dp]
        L.lbm_populations.argtypes = [vp, vp]
        L.lbm_destroy.argtypes = [vp]
        L.lbm_destroy.restype = None
        L.lbm_last_error.argtypes = []
        L.lbm_last_error.restype = ctypes.c_char_p
        L.lbm_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int]
        L.lbm_batch_step.argtypes = [vp, ctypes.c_int]
        L.lbm_batch_autotune.argtypes = [vp, ctypes.c_int, ctypes.c_char_p, ctypes.c_int]
        L.lbm_batch_config.argtypes = [vp, ip, ip]
        L.lbm_batch_destroy.argtypes = [vp]
        L.lbm_batch_destroy.restype = None
        i64 = ctypes.c_int64
        L.lbm_closure_samples.argtypes = [vp, ctypes.c_int, vp, vp]
        L.lbm_mlp_stats.argtypes = [vp, vp, i64, vp, vp]
        L.lbm_mlp_normalize.argtypes = [vp, vp, i64, vp, vp]
        L.lbm_mlp_create.argtypes = [ctypes.POINTER(vp), vp, i64, vp]
        L.lbm_mlp_forward.argtypes = [vp, vp, i64, vp]
        L.lbm_mlp_step.argtypes = [vp, vp, vp, vp, i64, ctypes.c_float, vp, ctypes.POINTER(ctypes.c_double)]
        L.lbm_mlp_destroy.argtypes = [vp]
        L.lbm_mlp_destroy.restype = None
        L.lbm_closure_set.argtypes = [vp, vp, vp]
        L.lbm_closure_fallbacks.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
        ci = ctypes.c_int
        L.lbm_lattice_velocities_3d.argtypes = [ci, ip, ip, ip, dp]
        L.lbm_buffer_elems_3d.argtypes = [ci, ci, ci, ci, ctypes.c_uint32]
        L.lbm_buffer_elems_3d.restype = ctypes.c_int64
        L.lbm_init_3d.argtypes = [ctypes.POINTER(vp), ci, ci, ci, ci, ctypes.c_double, ci, ctypes.c_uint32,
                                  vp, vp, vp, vp, vp, vp, vp, ctypes.c_double, vp]
        L.lbm_moments_3d.argtypes = [vp, vp, vp, vp, vp, dp]
        L.lbm_checkpoint_bytes.argtypes = [vp]
        L.lbm_checkpoint_bytes.restype = ctypes.c_int64
        L.lbm_save.argtypes = [vp, vp, ctypes.c_int64]
        L.lbm_load.argtypes = [vp, vp, ctypes.c_int64]
        _lib = L
    return _lib


def _check(rc):
    if rc != LBM_OK:
        raise LbmError(rc, lbm_last_error())
    return rc


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def lattice_id(lattice) -> int:
    return LATTICES[lattice] if isinstance(lattice, str) else int(lattice)


def lbm_last_error() -> str:
    return lib().lbm_last_error().decode()


def lbm_lattice_info(lattice):
    q, r, n, cs2 = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
    _check(lib().lbm_lattice_info(lattice_id(lattice), ctypes.byref(q), ctypes.byref(r), ctypes.byref(n),
                                  ctypes.byref(cs2)))
    return q.value, r.value, n.value, cs2.value


def lbm_lattice_velocities(lattice):
    q = lbm_lattice_info(lattice)[0]
    cx, cy, w = (ctypes.c_int * q)(), (ctypes.c_int * q)(), (ctypes.c_double * q)()
    _check(lib().lbm_lattice_velocities(lattice_id(lattice), cx, cy, w))
    return np.array(list(cx)), np.array(list(cy)), np.array(list(w))


def lbm_buffer_elems(lattice, nx, ny, flags=0) -> int:
    n = lib().lbm_buffer_elems(lattice_id(lattice), nx, ny, flags)
    if n < 0:
        raise LbmError(int(n), lbm_last_error())
    return int(n)


def lbm_init(lattice, nx, ny, tau, reg_order, flags, f_a, f_b, rho, ux, uy, theta=None, grad=None, noise=None,
             noise_amp=0.0, stream=None):
    """Returns the context handle (an integer)."""
    ctx = ctypes.c_void_p()
    s = ctypes.c_void_p(stream.cuda_stream if stream is not None else 0)
    _check(lib().lbm_init(ctypes.byref(ctx), lattice_id(lattice), nx, ny, tau, reg_order, flags, _ptr(f_a),
                          _ptr(f_b), _ptr(rho), _ptr(ux), _ptr(uy), _ptr(theta), _ptr(grad), _ptr(noise),
                          noise_amp, s))
    return ctx.value


def lbm_step(ctx, nsteps: int):
    _check(lib().lbm_step(ctypes.c_void_p(ctx), nsteps))


def lbm_set_relaxation(ctx, tau3: float, tau4: float):
    _check(lib().lbm_set_relaxation(ctypes.c_void_p(ctx), tau3, tau4))


def lbm_step_count(ctx) -> int:
    return int(lib().lbm_step_count(ctypes.c_void_p(ctx)))


def lbm_moments(ctx, rho=None, ux=None, uy=None, theta=None, vort=None, sums=False):
    out = (ctypes.c_double * LBM_NSUMS)() if sums else None
    _check(lib().lbm_moments(ctypes.c_void_p(ctx), _ptr(rho), _ptr(ux), _ptr(uy), _ptr(theta), _ptr(vort),
                             out))
    return np.array(list(out)) if sums else None


def lbm_moments_noalloc(ctx, rho=None, ux=None, uy=None, theta=None, vort=None, sums=False):
    out = (ctypes.c_double * LBM_NSUMS)() if sums else None
    _check(lib().lbm_moments_noalloc(ctypes.c_void_p(ctx), _ptr(rho), _ptr(ux), _ptr(uy), _ptr(theta), _ptr(vort),
                                     out))
    return np.array(list(out)) if sums else None


def lbm_populations(ctx, f_out):
    _check(lib().lbm_populations(ctypes.c_void_p(ctx), _ptr(f_out)))


def lbm_destroy(ctx):
    lib().lbm_destroy(ctypes.c_void_p(ctx))


LBM_CHECKPOINT_HEADER_BYTES = 64


def lbm_checkpoint_bytes(ctx) -> int:
    n = lib().lbm_checkpoint_bytes(ctypes.c_void_p(ctx))
    if n < 0:
        raise LbmError(int(n), lbm_last_error())
    return int(n)


def _addr(buf):
    """Address of a numpy array (host) or torch tensor (host or device)."""
    if isinstance(buf, np.ndarray):
        assert buf.flags["C_CONTIGUOUS"]
        return ctypes.c_void_p(buf.ctypes.data), buf.nbytes
    return ctypes.c_void_p(buf.data_ptr()), buf.numel() * buf.element_size()


def lbm_save(ctx, dst):
    p, n = _addr(dst)
    _check(lib().lbm_save(ctypes.c_void_p(ctx), p, n))


def lbm_load(ctx, src):
    p, n = _addr(src)
    _check(lib().lbm_load(ctypes.c_void_p(ctx), p, n))


def lbm_lattice_velocities_3d(lattice):
    q = lbm_lattice_info(lattice)[0]
    cx, cy, cz, w = (ctypes.c_int * q)(), (ctypes.c_int * q)(), (ctypes.c_int * q)(), (ctypes.c_double * q)()
    _check(lib().lbm_lattice_velocities_3d(lattice_id(lattice), cx, cy, cz, w))
    return np.array(list(cx)), np.array(list(cy)), np.array(list(cz)), np.array(list(w))


def lbm_buffer_elems_3d(lattice, nx, ny, nz, flags=0) -> int:
    n = lib().lbm_buffer_elems_3d(lattice_id(lattice), nx, ny, nz, flags)
    if n < 0:
        raise LbmError(int(n), lbm_last_error())
    return int(n)


def lbm_init_3d(lattice, nx, ny, nz, tau, reg_order, flags, f_a, f_b, rho, ux, uy, uz, noise=None,
                noise_amp=0.0, stream=None):
    """Returns the context handle (an integer)."""
    ctx = ctypes.c_void_p()
    s = ctypes.c_void_p(stream.cuda_stream if stream is not None else 0)
    _check(lib().lbm_init_3d(ctypes.byref(ctx), lattice_id(lattice), nx, ny, nz, tau, reg_order, flags, _ptr(f_a),
                             _ptr(f_b), _ptr(rho), _ptr(ux), _ptr(uy), _ptr(uz), _ptr(noise), noise_amp, s))
    return ctx.value


def lbm_moments_3d(ctx, rho=None, ux=None, uy=None, uz=None, sums=False):
    out = (ctypes.c_double * LBM_NSUMS_3D)() if sums else None
    _check(lib().lbm_moments_3d(ctypes.c_void_p(ctx), _ptr(rho), _ptr(ux), _ptr(uy), _ptr(uz), out))
    return np.array(list(out)) if sums else None


def lbm_batch_create(ctxs, tile_x=64, blocks_per_cu=4):
    """ctxs: context handles (integers).  Returns the batch handle."""
    arr = (ctypes.c_void_p * len(ctxs))(*[ctypes.c_void_p(c) for c in ctxs])
    out = ctypes.c_void_p()
    _check(lib().lbm_batch_create(ctypes.byref(out), arr, len(ctxs), tile_x, blocks_per_cu))
    return out.value


def lbm_batch_step(batch, nsteps: int):
    _check(lib().lbm_batch_step(ctypes.c_void_p(batch), nsteps))


def lbm_batch_autotune(batch, steps_per_trial: int = 10) -> list:
    """Returns [(tile_x, blocks_per_cu, ms_per_step), ...] for every candidate."""
    buf = ctypes.create_string_buffer(4096)
    _check(lib().lbm_batch_autotune(ctypes.c_void_p(batch), steps_per_trial, buf, len(buf)))
    rows = []
    for line in buf.value.decode().splitlines():
        t, b, ms = line.split()
        rows.append((int(t), int(b), float(ms)))
    return rows


def lbm_batch_config(batch):
    t, b = ctypes.c_int(), ctypes.c_int()
    _check(lib().lbm_batch_config(ctypes.c_void_p(batch), ctypes.byref(t), ctypes.byref(b)))
    return t.value, b.value


def lbm_batch_destroy(batch):
    lib().lbm_batch_destroy(ctypes.c_void_p(batch))


def _stream(stream):
    return ctypes.c_void_p(stream.cuda_stream if stream is not None else 0)


def lbm_closure_samples(ctx, factor, x, r):
    _check(lib().lbm_closure_samples(ctypes.c_void_p(ctx), factor, _ptr(x), _ptr(r)))


def lbm_mlp_stats(x, r, n, norm, stream=None):
    _check(lib().lbm_mlp_stats(_ptr(x), _ptr(r), n, _ptr(norm), _stream(stream)))


def lbm_mlp_normalize(x, r, n, norm, stream=None):
    _check(lib().lbm_mlp_normalize(_ptr(x), _ptr(r), n, _ptr(norm), _stream(stream)))


def lbm_mlp_create(theta, max_batch, stream=None):
    out = ctypes.c_void_p()
    _check(lib().lbm_mlp_create(ctypes.byref(out), _ptr(theta), max_batch, _stream(stream)))
    return out.value


def lbm_mlp_forward(m, x, n, y):
    _check(lib().lbm_mlp_forward(ctypes.c_void_p(m), _ptr(x), n, _ptr(y)))


def lbm_mlp_step(m, x, t, idx, batch, lr, grad=None, want_loss=False):
    loss = ctypes.c_double()
    _check(lib().lbm_mlp_step(ctypes.c_void_p(m), _ptr(x), _ptr(t), _ptr(idx), batch, lr, _ptr(grad),
                              ctypes.byref(loss) if want_loss else None))
    return loss.value if want_loss else None


def lbm_mlp_destroy(m):
    lib().lbm_mlp_destroy(ctypes.c_void_p(m))


def lbm_closure_set(ctx, theta, norm):
    _check(lib().lbm_closure_set(ctypes.c_void_p(ctx), _ptr(theta), _ptr(norm)))


def lbm_closure_fallbacks(ctx) -> int:
    n = ctypes.c_int64()
    _check(lib().lbm_closure_fallbacks(ctypes.c_void_p(ctx), ctypes.byref(n)))
    return int(n.value)


# ---------------------------------------------------------------- helper

class Simulation:
    """Owns the population buffers (torch tensors: two, or one with
    LBM_SCHEME_AA) and one context."""

    def __init__(self, lattice, nx, ny, tau, rho, ux, uy, theta=None, noise=None, noise_amp=0.0,
                 reg_order=None, flags=0, device="cuda:0", stream=None, grad=None):
        import torch

        self.torch = torch
        self.lattice = lattice_id(lattice)
        self.q, self.reach, self.n_eq, self.cs2 = lbm_lattice_info(self.lattice)
        self.nx, self.ny, self.tau, self.flags = nx, ny, tau, flags
        self.reg_order = self.n_eq if reg_order is None else reg_order
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        dtype = (torch.float32 if flags & LBM_STORE_FP32 else
                 torch.bfloat16 if flags & LBM_STORE_BF16 else torch.float64)
        n = lbm_buffer_elems(self.lattice, nx, ny, flags)
        self.bufs = [torch.empty(n, dtype=dtype, device=self.device) for _ in range(1 if flags & LBM_SCHEME_AA else 2)]

        def dev(a):
            if a is None:
                return None
            t = torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)) if isinstance(a, np.ndarray) else a
            return t.to(self.device, torch.float64).contiguous()

        fields = [dev(a) for a in (rho, ux, uy, theta, grad, noise)]
        f_b = self.bufs[1] if len(self.bufs) > 1 else None
        self.ctx = lbm_init(self.lattice, nx, ny, tau, self.reg_order, flags, self.bufs[0], f_b,
                            *fields, noise_amp=noise_amp, stream=self.stream)
        self._keep = fields  # inputs must outlive the asynchronous init

    @property
    def steps(self) -> int:
        return lbm_step_count(self.ctx)

    def step(self, n: int = 1):
        lbm_step(self.ctx, n)

    def set_relaxation(self, tau3: float, tau4: float):
        lbm_set_relaxation(self.ctx, tau3, tau4)

    def populations(self):
        t = self.torch.empty((self.q, self.ny, self.nx), dtype=self.torch.float64, device=self.device)
        lbm_populations(self.ctx, t)
        return t

    def save(self) -> np.ndarray:
        """Checkpoint of the current step (host bytes)."""
        buf = np.empty(lbm_checkpoint_bytes(self.ctx), dtype=np.uint8)
        lbm_save(self.ctx, buf)
        return buf

    def load(self, buf):
        lbm_load(self.ctx, buf)

    def moments(self, sums=True, vorticity=True):
        torch = self.torch
        mk = lambda: torch.empty((self.ny, self.nx), dtype=torch.float64, device=self.device)
        rho, ux, uy, th = mk(), mk(), mk(), mk()
        vort = mk() if vorticity else None
        s = lbm_moments(self.ctx, rho, ux, uy, th, vort, sums=sums)
        return dict(rho=rho, ux=ux, uy=uy, theta=th, vort=vort, sums=s)

    def close(self):
        if self.ctx:
            self.stream.synchronize()
            lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Simulation3D(Simulation):
    """A 3D context (Table II lattices, FP64 populations or FP32 with
    LBM_STORE_FP32 | LBM_MATH_FP64) and its buffers (two, or one with
    LBM_SCHEME_AA); fields are [z][y][x] arrays."""

    def __init__(self, lattice, nx, ny, nz, tau, rho, ux, uy, uz, noise=None, noise_amp=0.0, reg_order=None,
                 flags=0, device="cuda:0", stream=None):
        import torch

        self.torch = torch
        self.lattice = lattice_id(lattice)
        self.q, self.reach, self.n_eq, self.cs2 = lbm_lattice_info(self.lattice)
        self.nx, self.ny, self.nz, self.tau, self.flags = nx, ny, nz, tau, flags
        self.reg_order = self.n_eq if reg_order is None else reg_order
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        n = lbm_buffer_elems_3d(self.lattice, nx, ny, nz, flags)
        dtype = torch.float32 if flags & LBM_STORE_FP32 else torch.float64
        self.bufs = [torch.empty(n, dtype=dtype, device=self.device)
                     for _ in range(1 if flags & LBM_SCHEME_AA else 2)]

        def dev(a):
            if a is None:
                return None
            t = torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)) if isinstance(a, np.ndarray) else a
            return t.to(self.device, torch.float64).contiguous()

        fields = [dev(a) for a in (rho, ux, uy, uz, noise)]
        f_b = self.bufs[1] if len(self.bufs) > 1 else None
        self.ctx = lbm_init_3d(self.lattice, nx, ny, nz, tau, self.reg_order, flags, self.bufs[0], f_b,
                               *fields, noise_amp=noise_amp, stream=self.stream)
        self._keep = fields

    def populations(self):
        t = self.torch.empty((self.q, self.nz, self.ny, self.nx), dtype=self.torch.float64, device=self.device)
        lbm_populations(self.ctx, t)
        return t

    def moments(self, sums=True):
        torch = self.torch
        mk = lambda: torch.empty((self.nz, self.ny, self.nx), dtype=torch.float64, device=self.device)
        rho, ux, uy, uz = mk(), mk(), mk(), mk()
        s = lbm_moments_3d(self.ctx, rho, ux, uy, uz, sums=sums)
        return dict(rho=rho, ux=ux, uy=uy, uz=uz, sums=s)
