"""The Re = 3e4 double shear layer of Sec. III.B (Figs. 2-4) on the GPU:
the statements the paper makes about it, checked on the runs themselves.

  * PR at the full order of D2Q9 (N = 4) and BGK are the same operator
    (Sec. II.F): their kinetic-energy and enstrophy histories coincide.
  * On the under-resolved grid (L = 128) BGK fails the stability criterion
    before 2 t_c, while RR at order 3 and 4 stays stable (D2Q9, M0 = 0.2).
  * RR is more stable than PR on D2V17 (M0 = 0.35, L = 256: PR3 fails, RR3
    does not).
  * RR at full order converges to a fine run as L grows: the enstrophy
    error against L = 1024 falls by more than 3x from L = 128 to 256.
Histories are the library's own diagnostics (FD4 vorticity, Sec. III.B)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def st():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1704_04413_amd import binding, studies

    binding.lib()
    return studies, torch


def test_pr4_equals_bgk_and_rr_outlasts_both_on_d2q9(st):
    studies, torch = st
    print("[case] Re 3e4 D2Q9 M0 0.2 L 128: BGK, PR4, RR3, RR4", flush=True)
    runs = {k: studies.shear_history(torch, "D2Q9", 128, 3e4, 0.2, c, o, samples_per_tc=20)
            for k, (c, o) in {"BGK": ("BGK", 2), "PR4": ("PR", 4), "RR3": ("RR", 3), "RR4": ("RR", 4)}.items()}
    a, p = runs["BGK"]["stats"], runs["PR4"]["stats"]
    m = min(len(a), len(p), int(round(runs["BGK"]["unstable_at"] * 20)))  # up to BGK's failure
    assert m > 5
    np.testing.assert_allclose(p[:m], a[:m], rtol=1e-6)
    assert runs["BGK"]["unstable_at"] is not None and runs["BGK"]["unstable_at"] < 2.0
    assert runs["RR3"]["unstable_at"] is None and runs["RR4"]["unstable_at"] is None
    print(f"[comparison] BGK fails at t/t_c {runs['BGK']['unstable_at']}, RR3/RR4 stable to 2 t_c", flush=True)


def test_rr3_more_stable_than_pr3_on_d2v17(st):
    studies, torch = st
    print("[case] Re 3e4 D2V17 M0 0.35 L 256: PR3, RR3", flush=True)
    pr = studies.shear_history(torch, "D2V17", 256, 3e4, 0.35, "PR", 3, samples_per_tc=20)
    rr = studies.shear_history(torch, "D2V17", 256, 3e4, 0.35, "RR", 3, samples_per_tc=20)
    print(f"[comparison] PR3 fails at {pr['unstable_at']}, RR3 at {rr['unstable_at']}", flush=True)
    assert pr["unstable_at"] is not None
    assert rr["unstable_at"] is None


def test_rr4_converges_on_d2q9(st):
    studies, torch = st
    print("[case] Re 3e4 D2Q9 M0 0.2 RR4: L 128, 256 against L 1024", flush=True)
    ref = studies.shear_history(torch, "D2Q9", 1024, 3e4, 0.2, "RR", 4, samples_per_tc=20)
    assert ref["unstable_at"] is None
    errs = []
    for n in (128, 256):
        run = studies.shear_history(torch, "D2Q9", n, 3e4, 0.2, "RR", 4, samples_per_tc=20)
        errs.append(studies._history_error(run, ref))
    print(f"[comparison] RR4 errors against L 1024: {errs}", flush=True)
    assert errs[0]["ke_mean"] < 2e-3 and errs[1]["ke_mean"] < errs[0]["ke_mean"]
    assert errs[1]["ens_mean"] * 3 < errs[0]["ens_mean"]
    assert errs[1]["ens_std"] * 3 < errs[0]["ens_std"]
