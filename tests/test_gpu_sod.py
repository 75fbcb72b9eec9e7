"""Thermal D2V37 Sod tube (Sec. III.C) on the GPU against the exact Riemann
solution of the oracle (gamma = 2): (rho, p)_L = (8, 10), (1, 1)_R, theta_L
= 1/2 so the left adiabatic sound speed is c_s, 2000 x 4 periodic tube,
interface at x = 1000.  Compared at t/t_c = 0.2 with t_c = L_x/c_R and L_x =
1000 (half the periodic tube), before the waves of the two interfaces meet,
over cells [500, 1500).  tau = 0.595 is the paper's value for this case;
the lower values of the workload (0.5005, 0.51, 0.55) blow up within about
100 steps, in the oracle as on the GPU, and are reported by bench.py."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1704_04413_amd import binding, studies

    binding.lib()
    return torch, studies


def exact(orc, cs2, t, nx=2000):
    th_l, th_r = 0.5, 0.4
    x = np.arange(nx) + 0.5
    xi = (x - nx / 2) / t
    rho, u, p, _, _ = orc.riemann_exact(8.0, 8.0 * cs2 * th_l, 0.0, 1.0, cs2 * th_r, 0.0, 2.0, xi)
    return rho, u, p


@pytest.mark.parametrize("tau", [0.595, 0.7])
def test_sod_profiles_against_exact_solution(orc, env, tau):
    torch, st = env
    cs2 = orc.lattice("D2V37").cs2
    c_r = np.sqrt(2.0 * 0.4 * cs2)
    t = int(round(0.2 * 1000 / c_r))
    print(f"[case] sod tau={tau} t={t}", flush=True)
    r64 = st.sod_run(torch, tau, "fp64", steps=t, snap=t)
    r32 = st.sod_run(torch, tau, "fp32", steps=t, snap=t)
    assert r64["blow_up_step"] is None and r32["blow_up_step"] is None
    rho_e, u_e, p_e = exact(orc, cs2, t)
    w = slice(500, 1500)
    pr = r64["profile"]
    p_lbm = pr["rho"] * cs2 * pr["theta"]
    l1 = lambda a, b: float(np.abs(a[w] - b[w]).mean() / np.abs(b[w]).mean())
    e_rho, e_p = l1(pr["rho"], rho_e), l1(p_lbm, p_e)
    e_u = float(np.abs(pr["ux"][w] - u_e[w]).mean() / np.abs(u_e[w]).max())
    d32 = float(np.abs(r32["profile"]["rho"] - pr["rho"]).max() / pr["rho"].max())
    print(f"[sod] tau {tau}: L1 rel rho {e_rho:.4f} p {e_p:.4f} u {e_u:.4f}; fp32 vs fp64 max rho {d32:.2e}",
          flush=True)
    assert e_rho <= 0.03 and e_p <= 0.03 and e_u <= 0.03
    assert d32 <= 1e-4


@pytest.mark.parametrize("case", ["P10_rho8", "P10_rho2"])
def test_sod_paper_cases(orc, env, case):
    """Both Sod cases of the paper at their own tau and comparison time (Fig. 6:
    (10, 8) at tau 0.595, t/t_c = 0.2; (10, 2) at tau 0.760, t/t_c = 0.1), on
    the 2000 x 4 tube (L_x = 1000), against the exact solution."""
    torch, st = env
    print(f"[case] sod paper case {case}", flush=True)
    r64 = st.sod_profiles(torch, case, "fp64", exact=orc.riemann_exact)
    r32 = st.sod_profiles(torch, case, "fp32", exact=orc.riemann_exact)
    assert r64["blow_up_step"] is None and r32["blow_up_step"] is None
    d32 = float(np.abs(r32["profile"]["rho"] - r64["profile"]["rho"]).max() / r64["profile"]["rho"].max())
    print(f"[sod] {case}: step {r64['step']}, theta L/R {r64['theta_left']}/{r64['theta_right']:.2f}: L1 rel rho "
          f"{r64['l1_rho']:.4f} p {r64['l1_p']:.4f} u {r64['l1_u']:.4f}; FP32 L1 rho {r32['l1_rho']:.4f}; "
          f"fp32 vs fp64 max rho {d32:.2e}", flush=True)
    assert r64["l1_rho"] <= 0.03 and r64["l1_p"] <= 0.03 and r64["l1_u"] <= 0.03
    assert d32 <= 1e-4
