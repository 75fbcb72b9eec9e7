"""Workload studies on the GPU: reduced-precision storage against the FP64
plain form on the paper's shear layer (Sec. III.B), and the thermal D2V37
Sod tube (Sec. III.C).  Every step runs in the HIP library; these functions
only set up seeded inputs, step, and reduce the library's diagnostics.

Stability follows the paper's criterion (Sec. III.B): a run is unstable once
<|u|^2> exceeds its initial value (checked every `every` steps, within two
convective times t_c = N/u0) or a non-finite node appears.
"""
from __future__ import annotations

import time

import numpy as np

from . import binding as b
from . import workloads as wl

STORE = {"fp64": 0, "fp32": b.LBM_STORE_FP32, "bf16": b.LBM_STORE_BF16,
         "fp32d": b.LBM_STORE_FP32 | b.LBM_MATH_FP64}


def _flow_stats(s, n, u0):
    """KE and enstrophy mean/std from the library's sums (KE = |u|^2/2/u0^2,
    enstrophy = omega^2/2 (n/u0)^2)."""
    nodes = n * n
    ke_m = 0.5 * s[4] / nodes / u0 ** 2
    ke_s = np.sqrt(max(0.0, 0.25 * s[5] / nodes / u0 ** 4 - ke_m ** 2))
    en_scale = 0.5 * (n / u0) ** 2
    en_m = en_scale * s[6] / nodes
    en_s = np.sqrt(max(0.0, en_scale ** 2 * s[7] / nodes - en_m ** 2))
    return ke_m, ke_s, en_m, en_s


def shear_run(torch, lattice, n, re, storage, steps, every, keep_fields_at=()):
    """Shear layer at Mach 0.1; returns the diagnostic history, the blow-up
    step (None if stable) and velocity fields at the requested steps."""
    q, _, _, cs2 = b.lbm_lattice_info(lattice)
    u0, tau = wl.shear_layer_params(cs2, n, re)
    rho, ux, uy = wl.shear_layer_fields(n, n, u0)
    noise = wl.uniform_noise(0, q, n, n)
    sim = b.Simulation(lattice, n, n, tau, rho, ux, uy, noise=noise, noise_amp=1e-8, flags=STORE[storage])
    tc = n / u0
    hist, fields, blow = [], {}, None
    u2_0 = None
    while sim.steps <= steps:
        m = sim.moments()
        s = m["sums"]
        u2 = s[4] / (n * n)
        u2_0 = u2 if u2_0 is None else u2_0
        hist.append((sim.steps,) + tuple(float(v) for v in _flow_stats(s, n, u0)))
        if sim.steps in keep_fields_at:
            fields[sim.steps] = (m["ux"].clone(), m["uy"].clone())
        if blow is None and (s[8] > 0 or (sim.steps <= 2 * tc and u2 > u2_0 * (1 + 1e-12))):
            blow = sim.steps
        if s[8] > 0 or sim.steps == steps:
            break
        sim.step(min(every, steps - sim.steps))
    sim.close()
    return dict(history=hist, blow_up_step=blow, tau=tau, u0=u0), fields


def precision_study(torch, lattices=("D2V17", "D2V37"), sizes=(512, 1024), res=(3e4, 1e5, 1e6), steps=10000,
                    every=500, storages=("fp32", "fp32d", "bf16")):
    """Weight-shifted storage (FP32 with float or double arithmetic, BF16)
    against the FP64 plain form: blow-up steps, velocity relative L2 error at
    the last common checkpoint, largest relative deviation of the KE /
    enstrophy means."""
    out = []
    t0 = time.perf_counter()
    for lat in lattices:
        for n in sizes:
            for re in res:
                ref, fref = shear_run(torch, lat, n, re, "fp64", steps, every, keep_fields_at=range(0, steps + 1, every))
                row = dict(lattice=lat, n=n, re=re, tau=ref["tau"], blow_up_fp64=ref["blow_up_step"])
                for st in storages:
                    r, f = shear_run(torch, lat, n, re, st, steps, every, keep_fields_at=range(0, steps + 1, every))
                    common = sorted(set(fref) & set(f))
                    k = common[-1]
                    ux, uy = f[k]
                    rx, ry = fref[k]
                    err = float(torch.sqrt(((ux - rx) ** 2 + (uy - ry) ** 2).sum() / (rx ** 2 + ry ** 2).sum()))
                    h, hr = np.array(r["history"]), np.array(ref["history"])
                    m = min(len(h), len(hr))
                    dke = float(np.max(np.abs(h[:m, 1] - hr[:m, 1]) / np.abs(hr[:m, 1])))
                    den = float(np.max(np.abs(h[:m, 3] - hr[:m, 3]) / np.abs(hr[:m, 3])))
                    row[st] = dict(blow_up_step=r["blow_up_step"], compared_at=k, velocity_rel_l2=err,
                                   ke_mean_rel_dev=dke, enstrophy_mean_rel_dev=den)
                del fref
                out.append(row)
    return dict(rows=out, steps=steps, seconds=round(time.perf_counter() - t0, 1))


def sod_run(torch, tau, storage="fp64", nx=2000, ny=4, steps=800, snap=None, theta_left=0.5, every=50,
            rho_l=8.0, p_l=10.0):
    """Thermal D2V37 Sod tube (rho, p)_L = (rho_l, p_l), (1, 1)_R, u = 0,
    interface at nx/2, periodic.  Returns the blow-up step (first check with a
    non-finite node or theta <= 0) and y-averaged rho, u, theta at `snap`."""
    q, _, _, cs2 = b.lbm_lattice_info("D2V37")
    rho, ux, uy, th = wl.sod_fields(nx, ny, rho_l=rho_l, p_l=p_l, theta_left=theta_left)
    sim = b.Simulation("D2V37", nx, ny, tau, rho, ux, uy, theta=th, flags=b.LBM_THERMAL | STORE[storage])
    blow, prof = None, None
    marks = sorted(set(range(0, steps + 1, every)) | ({snap} if snap else set()))
    for k in marks:
        sim.step(k - sim.steps)
        m = sim.moments(vorticity=False)
        if k == snap:
            prof = {key: m[key].mean(0).double().cpu().numpy() for key in ("rho", "ux", "theta")}
        if blow is None and (m["sums"][8] > 0 or float(m["theta"].min()) <= 0.0):
            blow = k
            break
    sim.close()
    return dict(blow_up_step=blow, profile=prof, cs2=cs2)


# The paper's two Sod cases (Sec. III.C, Fig. 6): left state, tau, time of
# the comparison in t_c = L_x / c_R, left temperature of the lattice scaling.
SOD_CASES = {
    "P10_rho8": dict(rho_l=8.0, p_l=10.0, tau=0.595, t_over_tc=0.2, theta_left=0.5),
    "P10_rho2": dict(rho_l=2.0, p_l=10.0, tau=0.760, t_over_tc=0.1, theta_left=1.0),
}


def sod_profiles(torch, case, storage="fp64", nx=2000, ny=4, exact=None):
    """One of the paper's Sod cases at t = t_over_tc * L_x / c_R, L_x = nx / 2
    (before the waves of the two interfaces meet).  Returns the step, the
    blow-up step and the y-averaged profiles; with `exact` (a callable
    (rho_l, p_l, u_l, rho_r, p_r, u_r, gamma, xi) -> (rho, u, p, ...), the
    exact Riemann solution) also L1 errors over the cells [nx/4, 3nx/4) of rho
    and p (relative to the mean exact value) and of u (relative to the
    largest exact |u|)."""
    c = SOD_CASES[case]
    cs2 = b.lbm_lattice_info("D2V37")[3]
    th_r = c["theta_left"] * c["rho_l"] / c["p_l"]
    c_r = np.sqrt(2.0 * th_r * cs2)
    t = int(round(c["t_over_tc"] * (nx / 2) / c_r))
    r = sod_run(torch, c["tau"], storage, nx=nx, ny=ny, steps=t, snap=t, theta_left=c["theta_left"],
                rho_l=c["rho_l"], p_l=c["p_l"])
    out = dict(case=case, storage=storage, tau=c["tau"], theta_left=c["theta_left"], theta_right=th_r, step=t,
               blow_up_step=r["blow_up_step"])
    if r["blow_up_step"] is not None:
        return out
    pr = out["profile"] = r["profile"]
    if exact is not None:
        x = np.arange(nx) + 0.5
        rho_e, u_e, p_e = exact(c["rho_l"], c["rho_l"] * cs2 * c["theta_left"], 0.0, 1.0, cs2 * th_r, 0.0, 2.0,
                                (x - nx / 2) / t)[:3]
        w = slice(nx // 4, 3 * nx // 4)
        p = pr["rho"] * cs2 * pr["theta"]
        l1 = lambda a, e: float(np.abs(a[w] - e[w]).mean() / np.abs(e[w]).mean())
        out.update(l1_rho=l1(pr["rho"], rho_e), l1_p=l1(p, p_e),
                   l1_u=float(np.abs(pr["ux"][w] - u_e[w]).mean() / np.abs(u_e[w]).max()))
    return out


def sod_study(torch, taus=(0.5005, 0.51, 0.55, 0.595), steps=800):
    """Blow-up steps of the (8, 10) case over `steps` at each tau, FP64 and
    FP32 storage, and both paper cases at their comparison time (blow-up,
    FP32 against FP64)."""
    rows = []
    for tau in taus:
        row = dict(tau=tau)
        for st in ("fp64", "fp32"):
            t0 = time.perf_counter()
            r = sod_run(torch, tau, st, steps=steps)
            row[st] = dict(blow_up_step=r["blow_up_step"], seconds=round(time.perf_counter() - t0, 2))
        rows.append(row)
    cases = []
    for case in SOD_CASES:
        r64 = sod_profiles(torch, case, "fp64")
        r32 = sod_profiles(torch, case, "fp32")
        row = {k: v for k, v in r64.items() if k not in ("profile", "storage")}
        row["fp32_blow_up_step"] = r32["blow_up_step"]
        if "profile" in r64 and "profile" in r32:
            row["fp32_vs_fp64_max_rel_rho"] = float(np.abs(r32["profile"]["rho"] - r64["profile"]["rho"]).max()
                                                    / r64["profile"]["rho"].max())
        cases.append(row)
    return dict(blow_up=rows, paper_cases=cases)


def shear_stable(torch, lattice, n, re, mach, flags, order, every=25, noneq_start=True):
    """The paper's stability criterion for the doubly periodic shear layer
    (Sec. III.B): stable if <|u|^2>(t) < <|u|^2>(0) for every t <= 2 t_c,
    t_c = n / (M0 c_s), and no node turns non-finite (checked every `every`
    steps).  The run starts from f^(0) + f^(1) with the analytic velocity
    gradients, as in the paper (from f^(0) alone if not `noneq_start`)."""
    q, _, _, cs2 = b.lbm_lattice_info(lattice)
    u0, tau = wl.shear_layer_params(cs2, n, re, mach)
    rho, ux, uy = wl.shear_layer_fields(n, n, u0)
    grad = wl.shear_layer_gradients(n, n, u0) if noneq_start else None
    sim = b.Simulation(lattice, n, n, tau, rho, ux, uy, noise=wl.uniform_noise(0, q, n, n), noise_amp=1e-8,
                       reg_order=order, flags=flags, grad=grad)
    horizon = int(np.ceil(2.0 * n / u0))
    u2_0 = None
    ok = True
    while True:
        s = sim.moments(vorticity=False)["sums"]
        u2 = s[4]
        u2_0 = u2 if u2_0 is None else u2_0
        if s[8] > 0 or not np.isfinite(u2) or (sim.steps > 0 and u2 >= u2_0):
            ok = False
            break
        if sim.steps >= horizon:
            break
        sim.step(min(every, horizon - sim.steps))
    sim.close()
    return ok


COLLISIONS = {"BGK": b.LBM_COLL_BGK, "PR": b.LBM_COLL_PR, "RR": 0}


def max_stable_mach(torch, lattice, coll, order, re, n=128, lo=0.05, hi=1.6, tol=0.01, noneq_start=True):
    """Largest M0 (to `tol`, Fig. 5 uses 0.01) for which the shear layer at
    Re on n^2 nodes stays stable, by bisection between `lo` and `hi`.
    Returns (M0max, runs); M0max = 0 if `lo` already fails, `hi` if it holds."""
    flags, runs = COLLISIONS[coll], 0

    def stable(m):
        nonlocal runs
        runs += 1
        return shear_stable(torch, lattice, n, re, m, flags, order, noneq_start=noneq_start)

    if not stable(lo):
        return 0.0, runs
    if stable(hi):
        return hi, runs
    while hi - lo > tol + 1e-9:
        mid = round(0.5 * (lo + hi), 4)
        if stable(mid):
            lo = mid
        else:
            hi = mid
    return round(lo, 4), runs


def stability_range(torch, res=(1e4, 3e4, 1e5, 3e5, 1e6), n=128, noneq_start=True):
    """M0max against Re for BGK, PR at the lattice's full order and RR at every
    order 2..N_eq, on D2Q9, D2V17 and D2V37 (the study of Fig. 5)."""
    variants = []
    for lat in ("D2Q9", "D2V17", "D2V37"):
        n_eq = b.lbm_lattice_info(lat)[2]
        variants.append((lat, "BGK", 2))
        variants.append((lat, "PR", n_eq))
        variants += [(lat, "RR", k) for k in range(2, n_eq + 1)]
    rows = []
    t0 = time.perf_counter()
    for lat, coll, order in variants:
        row = dict(lattice=lat, collision=coll, order=order, m0_max={})
        for re in res:
            m, runs = max_stable_mach(torch, lat, coll, order, re, n, noneq_start=noneq_start)
            row["m0_max"][f"{re:.0e}"] = m
        rows.append(row)
    return dict(n=n, criterion="<u^2>(t) < <u^2>(0) for t <= 2 n/(M0 c_s), no non-finite node",
                start="f0+f1" if noneq_start else "f0", resolution=0.01, rows=rows,
                seconds=round(time.perf_counter() - t0, 1))


# ---- the Re = 3e4 comparison of Sec. III.B (Figs. 2-4) ---------------------

PAPER_MACH = {"D2Q9": 0.2, "D2V17": 0.35, "D2V37": 0.57}


def shear_history(torch, lattice, n, re, mach, coll, order, samples_per_tc=40, horizon_tc=2.0, noise_seed=0):
    """One run of the doubly periodic shear layer started from f^(0) + f^(1)
    (analytic gradients, Sec. III.B): the spatial mean and standard deviation
    of the kinetic energy and of the enstrophy at t = k t_c / samples_per_tc
    (nearest step), k = 0 .. horizon_tc * samples_per_tc, t_c = n / u0; the
    first sample where the paper's stability criterion fails (<|u|^2>(t) >=
    <|u|^2>(0), or a non-finite node), and the first where the run has
    blown up (a non-finite node, or <|u|^2> above twice its initial value).
    The run continues past a failed criterion until it blows up."""
    q, _, _, cs2 = b.lbm_lattice_info(lattice)
    u0, tau = wl.shear_layer_params(cs2, n, re, mach)
    rho, ux, uy = wl.shear_layer_fields(n, n, u0)
    grad = wl.shear_layer_gradients(n, n, u0)
    sim = b.Simulation(lattice, n, n, tau, rho, ux, uy, noise=wl.uniform_noise(noise_seed, q, n, n),
                       noise_amp=1e-8, reg_order=order, flags=COLLISIONS[coll], grad=grad)
    tc = n / u0
    nsamp = int(round(horizon_tc * samples_per_tc))
    marks = [int(round(k * tc / samples_per_tc)) for k in range(nsamp + 1)]
    hist, fail, blow, u2_0, u2max = [], None, None, None, 0.0
    for k, step in enumerate(marks):
        sim.step(step - sim.steps)
        s = sim.moments(vorticity=True)["sums"]
        u2 = s[4]
        u2_0 = u2 if u2_0 is None else u2_0
        if s[8] > 0 or not np.isfinite(u2) or u2 > 2.0 * u2_0:
            blow = k
            fail = k if fail is None else fail
            break
        if fail is None and k > 0 and u2 >= u2_0:
            fail = k
        u2max = max(u2max, u2 / u2_0)
        hist.append(_flow_stats(s, n, u0))
    sim.close()
    return dict(t_over_tc=[k / samples_per_tc for k in range(len(hist))], stats=np.array(hist),
                samples_per_tc=samples_per_tc, unstable_at=None if fail is None else fail / samples_per_tc,
                blow_up_at=None if blow is None else blow / samples_per_tc, max_u2_ratio=u2max, tau=tau, u0=u0)


def _history_error(run, ref):
    """max_t |X - X_ref| / max_t |X_ref| for X = KE mean, KE std, enstrophy
    mean, enstrophy std, over the samples both runs reached before either
    failed the stability criterion."""
    m = min(len(run["stats"]), len(ref["stats"]))
    for r in (run, ref):
        if r["unstable_at"] is not None:
            m = min(m, int(round(r["unstable_at"] * r["samples_per_tc"])))
    if m == 0:
        return None
    a, r = run["stats"][:m], ref["stats"][:m]
    scale = np.abs(ref["stats"]).max(axis=0)
    e = np.abs(a - r).max(axis=0) / scale
    return dict(zip(("ke_mean", "ke_std", "ens_mean", "ens_std"), (round(float(x), 5) for x in e)))


def comparison_study(torch, re=3e4, sizes=(128, 256), ref_n=2048, convergence=(512, 1024), samples_per_tc=40):
    """The Re = 3e4 study of Figs. 2-4: BGK, PR and RR at every order 2..N_eq
    on D2Q9 (M0 0.2), D2V17 (0.35) and D2V37 (0.57), on L^2 grids for L in
    `sizes`, against a BGK reference on ref_n^2 (per lattice; RR at full order
    on the same grid where BGK blows up before 2 t_c), up to 2 t_c;
    plus the mesh convergence of RR at full order.  Reports, per run, where
    the stability criterion failed (t/t_c) and the largest deviation of the
    four statistics from the reference over the common samples, relative to
    the reference's largest value."""
    out = []
    t0 = time.perf_counter()
    for lat, mach in PAPER_MACH.items():
        n_eq = b.lbm_lattice_info(lat)[2]
        ref = shear_history(torch, lat, ref_n, re, mach, "BGK", 2, samples_per_tc)
        ref_coll, bgk_ref_blow = "BGK", ref["blow_up_at"]
        if ref["blow_up_at"] is not None:
            # the BGK reference did not last 2 t_c: RR at full order on the same grid instead
            ref = shear_history(torch, lat, ref_n, re, mach, "RR", n_eq, samples_per_tc)
            ref_coll = f"RR{n_eq}"
        rows = []
        variants = [("BGK", 2)] + [("PR", k) for k in range(2, n_eq + 1)] + [("RR", k) for k in range(2, n_eq + 1)]
        for n in sizes:
            for coll, order in variants:
                run = shear_history(torch, lat, n, re, mach, coll, order, samples_per_tc)
                rows.append(dict(n=n, collision=coll, order=order if coll != "BGK" else None,
                                 tau=run["tau"], unstable_at_t_over_tc=run["unstable_at"],
                                 blow_up_at_t_over_tc=run["blow_up_at"],
                                 max_u2_over_initial=round(run["max_u2_ratio"], 6),
                                 error_vs_ref=_history_error(run, ref)))
        conv = []
        for n in tuple(sizes) + tuple(convergence):
            run = shear_history(torch, lat, n, re, mach, "RR", n_eq, samples_per_tc)
            conv.append(dict(n=n, unstable_at_t_over_tc=run["unstable_at"], blow_up_at_t_over_tc=run["blow_up_at"],
                             max_u2_over_initial=round(run["max_u2_ratio"], 6), error_vs_ref=_history_error(run, ref)))
        samples = list(range(0, 2 * samples_per_tc + 1, samples_per_tc // 4))
        out.append(dict(lattice=lat, mach=mach, re=re, reference=dict(
            n=ref_n, collision=ref_coll, bgk_blow_up_at_t_over_tc=bgk_ref_blow,
            unstable_at_t_over_tc=ref["unstable_at"], blow_up_at_t_over_tc=ref["blow_up_at"],
            max_u2_over_initial=round(ref["max_u2_ratio"], 6),
            at_t_over_tc=[ref["t_over_tc"][k] for k in samples if k < len(ref["stats"])],
            ke_mean=[round(float(ref["stats"][k, 0]), 6) for k in samples if k < len(ref["stats"])],
            ke_std=[round(float(ref["stats"][k, 1]), 6) for k in samples if k < len(ref["stats"])],
            ens_mean=[round(float(ref["stats"][k, 2]), 4) for k in samples if k < len(ref["stats"])],
            ens_std=[round(float(ref["stats"][k, 3]), 4) for k in samples if k < len(ref["stats"])]),
            runs=rows, rr_convergence=conv))
    return dict(criterion="<u^2>(t) < <u^2>(0) for t <= 2 t_c, no non-finite node",
                blow_up="a non-finite node or <u^2>(t) > 2 <u^2>(0); runs continue past the criterion until then",
                start="f0 + f1 (analytic gradients), f0 at the lattice's full order", samples_per_tc=samples_per_tc,
                error="max_t |X - X_ref| / max_t |X_ref| over the samples both runs reached", lattices=out,
                seconds=round(time.perf_counter() - t0, 1))


def stability_scan(torch, lattice, variants, re, machs, n=128, every=1):
    """Stable or not (Sec. III.B criterion, checked every `every` steps) for
    each M0 of a grid, and the t/t_c where a run fails: shows whether the
    stable set is an interval [0, M0max] as bisection assumes."""
    rows = []
    for coll, order in variants:
        res, blows, peaks = [], [], []
        for m in machs:
            q, _, _, cs2 = b.lbm_lattice_info(lattice)
            u0, tau = wl.shear_layer_params(cs2, n, re, m)
            rho, ux, uy = wl.shear_layer_fields(n, n, u0)
            sim = b.Simulation(lattice, n, n, tau, rho, ux, uy, noise=wl.uniform_noise(0, q, n, n), noise_amp=1e-8,
                               reg_order=order, flags=COLLISIONS[coll], grad=wl.shear_layer_gradients(n, n, u0))
            horizon = int(np.ceil(2.0 * n / u0))
            u2_0, fail, blow, u2max = None, None, None, 0.0
            while True:
                s = sim.moments(vorticity=False)["sums"]
                u2 = s[4]
                u2_0 = u2 if u2_0 is None else u2_0
                if s[8] > 0 or not np.isfinite(u2) or u2 > 2.0 * u2_0:
                    blow = sim.steps
                    fail = sim.steps if fail is None else fail
                    break
                if fail is None and sim.steps > 0 and u2 >= u2_0:
                    fail = sim.steps
                u2max = max(u2max, u2 / u2_0)
                if sim.steps >= horizon:
                    break
                sim.step(min(every, horizon - sim.steps))
            sim.close()
            res.append(None if fail is None else round(fail * u0 / n, 4))
            blows.append(None if blow is None else round(blow * u0 / n, 4))
            peaks.append(round(u2max, 6))
        rows.append(dict(collision=coll, order=order, unstable_at_t_over_tc=res, blow_up_at_t_over_tc=blows,
                         max_u2_over_initial=peaks))
    return dict(lattice=lattice, re=re, n=n, every=every, machs=[round(m, 4) for m in machs], rows=rows,
                blow_up="a non-finite node or <u^2>(t) > 2 <u^2>(0) before 2 t_c")
