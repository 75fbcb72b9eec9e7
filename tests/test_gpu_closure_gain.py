"""What the trained closure gains over the plain recursion, at reduced scale
(coarse 64^2 D2V37, fine 256^2, Re 3e4, six training and two held-out
seeds, each a different shear layer: steepness, amplitude and phase of the
perturbation), trained on the GPU by the library's kernels.

A priori (held-out flows) the network removes most of the plain recursion's
squared error in a_hat^(3..4) against the restricted fine run: that is the
gain this test asserts.  A posteriori the coarse run with the closure must
stay finite and keep mass and momentum; its velocity distance to the
restricted fine run is reported with its sign and is not claimed to improve:
the coarse error is dominated by the under-resolved rank-2 dynamics, which the
closure does not touch, and at Mach 0.1 the rank-3/4 terms barely act (the
full-size study at the paper's D2V37 Mach 0.57 changes the velocity error by
-4% .. +1% and the late-time enstrophy error by -2% .. -5%)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_closure_gain_small():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1704_04413_amd import closure as cl

    print("[case] closure gain 64^2 / 256^2", flush=True)
    res = cl.experiment(torch, range(6), range(6, 8), 64, 4, 3e4, tuple(range(50, 401, 50)), 1500, 8192)
    ap = res["a_priori"]
    print(f"[closure] a priori gain {ap['gain']:.3f}, fallback {ap['fallback_fraction']:.4f}; "
          f"loss {res['loss_log'][0][1]:.3f} -> {res['loss_log'][-1][1]:.3f}", flush=True)
    for p in res["a_posteriori"]:
        print(f"[closure] seed {p['seed']} step {p['step']}: velocity error plain {p['err_plain']:.6f} "
              f"closure {p['err_closure']:.6f} (signed gain {p['gain']:+.5f})", flush=True)
    assert ap["gain"] >= 0.5
    assert all(g > 0 for g in ap["gain_per_component"])
    assert ap["fallback_fraction"] < 0.01
    for p in res["a_posteriori"]:
        assert p["nonfinite"] == 0
        assert abs(p["gain"]) < 0.05  # no claim of a gain; the closure must not derail the run either
    assert res["loss_log"][-1][1] < 0.2 * res["loss_log"][0][1]
