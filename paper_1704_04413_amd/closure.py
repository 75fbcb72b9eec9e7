"""Learned-closure workflow on the GPU (the network itself lives in the HIP
library, see include/rrlbm.h): training samples from fine runs of the plain
method restricted to a coarse grid, training with the library's gradient and
Adam kernels, and evaluation against the restricted fine reference.

Shear layers follow the paper's doubly periodic case (Sec. III.B); fine and
coarse grids share Re and Mach (acoustic scaling), so coarse step k matches
fine step factor*k.  A seed draws the layer's steepness k in [60, 100], the
perturbation amplitude delta in [0.03, 0.08] and its phase (a phase alone
would only translate the same flow), so held-out seeds are different flows.
"""
from __future__ import annotations

import time

import numpy as np

from . import binding as b
from . import workloads as wl

NPARAM = b.LBM_MLP_NPARAM


def flow_of(seed: int) -> dict:
    """Shear-layer parameters of one seed: steepness k, amplitude delta, phase."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return dict(k=float(rng.uniform(60.0, 100.0)), delta=float(rng.uniform(0.03, 0.08)), phase=float(rng.uniform()))


def grid_params(n_coarse: int, factor: int, re: float, mach: float = 0.1):
    """(u0, tau_fine, tau_coarse) of the D2V37 shear layer."""
    cs2 = b.lbm_lattice_info("D2V37")[3]
    u0, tau_c = wl.shear_layer_params(cs2, n_coarse, re, mach)
    _, tau_f = wl.shear_layer_params(cs2, n_coarse * factor, re, mach)
    return u0, tau_f, tau_c


def init_theta(seed: int) -> np.ndarray:
    """He-normal initial weights, zero biases, padded outputs zero."""
    rng = np.random.Generator(np.random.PCG64(seed))
    th = np.zeros(NPARAM, dtype=np.float32)
    th[0:512] = rng.normal(0, np.sqrt(2.0 / 8), 512)
    th[576:4672] = rng.normal(0, np.sqrt(2.0 / 64), 4096)
    w3 = np.zeros((64, 16), dtype=np.float32)
    w3[:, :9] = rng.normal(0, np.sqrt(1.0 / 64), (64, 9))
    th[4736:5760] = w3.reshape(-1)
    return th


def _stats(sums, n, u0):
    """Mean kinetic energy |u|^2 / (2 u0^2) and mean enstrophy omega^2 (n/u0)^2 / 2
    from the library's sums (Sec. III.B diagnostics)."""
    return 0.5 * sums[4] / (n * n) / u0 ** 2, 0.5 * (n / u0) ** 2 * sums[6] / (n * n)


def generate_samples(torch, seeds, n_coarse=256, factor=4, re=3e4, snaps=tuple(range(150, 1501, 150)), mach=0.1):
    """Runs the plain method on the fine grid for each seed and restricts it
    at coarse steps `snaps`.  Returns raw x [N, 8], r [N, 16] (device
    float32), the per-snapshot restricted velocities with the fine run's
    mean kinetic energy and enstrophy, and timing."""
    u0, tau_f, _ = grid_params(n_coarse, factor, re, mach)
    nf, nc = n_coarse * factor, n_coarse * n_coarse
    xs, rs, ref = [], [], {}
    t0 = time.perf_counter()
    dropped = []
    for seed in seeds:
        rho, ux, uy = wl.shear_layer_fields(nf, nf, u0, **flow_of(seed))
        sim = b.Simulation("D2V37", nf, nf, tau_f, rho, ux, uy)
        for k in snaps:
            sim.step(factor * k - sim.steps)
            sums = sim.moments(vorticity=True)["sums"]
            if sums[8] > 0:  # the fine run blew up: no samples from here on
                dropped.append((seed, k))
                break
            x = torch.empty((nc, 8), dtype=torch.float32, device=sim.device)
            r = torch.empty((nc, 16), dtype=torch.float32, device=sim.device)
            b.lbm_closure_samples(sim.ctx, factor, x, r)
            xs.append(x)
            rs.append(r)
            ke, ens = _stats(sums, nf, u0)
            ref[(seed, k)] = (x[:, 1].reshape(n_coarse, n_coarse).double().cpu().numpy(),
                              x[:, 2].reshape(n_coarse, n_coarse).double().cpu().numpy(), ke, ens)
        sim.close()
    torch.cuda.synchronize()
    ref["dropped"] = dropped
    return torch.cat(xs), torch.cat(rs), ref, time.perf_counter() - t0


def train(torch, x, r, steps=4000, batch=16384, lr=2e-3, seed=0, log_every=500):
    """Normalises (in place) and trains; returns theta, norm and the loss log."""
    n = x.shape[0]
    norm = torch.empty(b.LBM_MLP_NNORM, dtype=torch.float32, device=x.device)
    b.lbm_mlp_stats(x, r, n, norm)
    b.lbm_mlp_normalize(x, r, n, norm)
    theta = torch.as_tensor(init_theta(seed)).to(x.device)
    m = b.lbm_mlp_create(theta, batch)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    perm = torch.as_tensor(rng.permutation(n).astype(np.int32)).to(x.device)
    pos, log = 0, []
    t0 = time.perf_counter()
    for s in range(steps):
        if pos + batch > n:
            perm = torch.as_tensor(rng.permutation(n).astype(np.int32)).to(x.device)
            pos = 0
        cur = lr * (0.05 + 0.95 * 0.5 * (1.0 + np.cos(np.pi * s / steps)))  # cosine decay to lr/20
        want = (s % log_every == 0) or s == steps - 1
        loss = b.lbm_mlp_step(m, x, r, perm[pos:pos + batch], batch, float(cur), None, want_loss=want)
        if want:
            log.append((s, loss))
        pos += batch
    torch.cuda.synchronize()
    b.lbm_mlp_destroy(m)
    return theta, norm, log, time.perf_counter() - t0


def a_priori(torch, theta, norm, x_raw, r_raw):
    """Residual prediction on samples the network has not seen, in the
    a_hat units of the targets.  The plain recursion predicts a zero
    residual; the closure predicts the network's output where the sample is
    inside the training range and zero elsewhere."""
    x, r = x_raw.clone(), r_raw.clone()
    n = x.shape[0]
    b.lbm_mlp_normalize(x, r, n, norm)
    y = torch.empty((n, 16), dtype=torch.float32, device=x.device)
    m = b.lbm_mlp_create(theta, 1)
    b.lbm_mlp_forward(m, x, n, y)
    b.lbm_mlp_destroy(m)
    nv = norm.double().cpu().numpy()
    z = x[:, :7].double().cpu().numpy()
    yy = y[:, :9].double().cpu().numpy()
    target = r_raw[:, :9].double().cpu().numpy()
    inside = np.all((z >= nv[16:23]) & (z <= nv[24:31]), axis=1) & \
        np.all((yy >= nv[64:73]) & (yy <= nv[80:89]), axis=1)
    pred = (yy * nv[48:57] + nv[32:41]) * inside[:, None]
    mse_plain = np.mean(target ** 2, axis=0)
    mse_cl = np.mean((target - pred) ** 2, axis=0)
    return dict(mse_plain=mse_plain.tolist(), mse_closure=mse_cl.tolist(),
                gain=float(1.0 - mse_cl.sum() / mse_plain.sum()),
                gain_per_component=(1.0 - mse_cl / mse_plain).tolist(),
                fallback_fraction=float(1.0 - inside.mean()))


def coarse_run(torch, seed, snaps, n_coarse=256, factor=4, re=3e4, theta=None, norm=None, mach=0.1):
    """Coarse plain (theta None) or closure run; velocities, non-finite count,
    mean kinetic energy and enstrophy at `snaps`."""
    u0, tau_f, tau_c = grid_params(n_coarse, factor, re, mach)
    rho, ux, uy = wl.shear_layer_fields(n_coarse, n_coarse, u0, **flow_of(seed))
    sim = b.Simulation("D2V37", n_coarse, n_coarse, tau_c, rho, ux, uy)
    if theta is not None:
        b.lbm_closure_set(sim.ctx, theta, norm)
    out = {}
    for k in snaps:
        sim.step(k - sim.steps)
        mo = sim.moments(vorticity=True)
        out[k] = (mo["ux"].cpu().numpy(), mo["uy"].cpu().numpy(), int(mo["sums"][8])) + \
            _stats(mo["sums"], n_coarse, u0)
    fb = b.lbm_closure_fallbacks(sim.ctx) if theta is not None else 0
    sim.close()
    return out, fb


def velocity_error(run, ref, seed, k):
    ux, uy = run[k][:2]
    rx, ry = ref[(seed, k)][:2]
    return float(np.sqrt(np.sum((ux - rx) ** 2 + (uy - ry) ** 2) / np.sum(rx ** 2 + ry ** 2)))


def step_rate(torch, n, steps=200, theta=None, norm=None, re=3e4):
    """MLUPS of the D2V37 FP64 step at n x n, plain or with the closure."""
    cs2 = b.lbm_lattice_info("D2V37")[3]
    u0, tau = wl.shear_layer_params(cs2, n, re)
    rho, ux, uy = wl.shear_layer_fields(n, n, u0)
    sim = b.Simulation("D2V37", n, n, tau, rho, ux, uy)
    if theta is not None:
        b.lbm_closure_set(sim.ctx, theta, norm)
    sim.step(10)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record(sim.stream)
    sim.step(steps)
    e.record(sim.stream)
    torch.cuda.synchronize()
    sim.close()
    return n * n * steps / (s.elapsed_time(e) * 1e-3) / 1e6


def experiment(torch, train_seeds=range(16), test_seeds=range(16, 20), n_coarse=256, factor=4, re=3e4,
               snaps=tuple(range(150, 1501, 150)), steps=4000, batch=16384, mach=0.1):
    """The whole closure study; returns a JSON-ready dict.  A posteriori, per
    held-out seed and evaluation step: the coarse velocity's relative L2
    distance to the restricted fine run (plain and closure) and the signed
    gain 1 - err_closure / err_plain; the relative errors of the mean
    kinetic energy and enstrophy against the fine run's own."""
    x, r, ref_train, t_gen = generate_samples(torch, list(train_seeds), n_coarse, factor, re, snaps, mach)
    xh, rh, ref, t_gen2 = generate_samples(torch, list(test_seeds), n_coarse, factor, re, snaps, mach)
    n_train = int(x.shape[0])
    theta, norm, log, t_train = train(torch, x, r, steps, batch)
    del x, r
    ap = a_priori(torch, theta, norm, xh, rh)
    post = []
    for seed in test_seeds:
        plain, _ = coarse_run(torch, seed, snaps, n_coarse, factor, re, mach=mach)
        clos, fb = coarse_run(torch, seed, snaps, n_coarse, factor, re, theta, norm, mach=mach)
        for k in (snaps[len(snaps) // 2], snaps[-1]):
            if (seed, k) not in ref:
                continue
            ep, ec = velocity_error(plain, ref, seed, k), velocity_error(clos, ref, seed, k)
            ke_f, ens_f = ref[(seed, k)][2:]
            post.append(dict(seed=seed, step=k, err_plain=ep, err_closure=ec, gain=1.0 - ec / ep,
                             ke_err_plain=abs(plain[k][3] / ke_f - 1), ke_err_closure=abs(clos[k][3] / ke_f - 1),
                             ens_err_plain=abs(plain[k][4] / ens_f - 1), ens_err_closure=abs(clos[k][4] / ens_f - 1),
                             nonfinite=plain[k][2] + clos[k][2]))
        post[-1]["fallback_nodes"] = fb
        post[-1]["fallback_fraction"] = fb / float(n_coarse * n_coarse * snaps[-1])
    rates = {f"{n}": dict(plain=round(step_rate(torch, n), 1),
                          closure=round(step_rate(torch, n, theta=theta, norm=norm), 1))
             for n in sorted({n_coarse, n_coarse * factor, 2048})}
    return dict(train_seeds=list(train_seeds), test_seeds=list(test_seeds), n_coarse=n_coarse, factor=factor,
                re=re, mach=mach, train_samples=n_train, test_samples=int(xh.shape[0]),
                fine_runs_blown_up=dict(train=ref_train["dropped"], test=ref["dropped"]),
                mean_gain=float(np.mean([p["gain"] for p in post])),
                seconds=dict(fine_runs=round(t_gen + t_gen2, 2), training=round(t_train, 2)),
                loss_log=log, a_priori=ap, a_posteriori=post, MLUPS=rates)
