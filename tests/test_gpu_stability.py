"""Stability range of the doubly periodic shear layer on 128^2 nodes (the
study of Fig. 5), run through the library: M0max to 0.01 by bisection,
stable meaning <|u|^2>(t) < <|u|^2>(0) up to t = 2 t_c and no non-finite
node, starting from f^(0) + f^(1) as the paper does.

Checked here, as the paper states them: on D2Q9 the fourth-order PR and
BGK are the same operator (identical M0max); the recursive regularization
reaches a higher M0max than the projection on D2Q9 and D2V17 (Re 3e4 and
1e5, the most stable RR order against PR at full order)."""
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


def test_d2q9_pr4_is_bgk(env):
    torch, st = env
    print("[case] stability D2Q9 PR4 vs BGK, Re 1e4", flush=True)
    m_pr, _ = st.max_stable_mach(torch, "D2Q9", "PR", 4, 1e4)
    m_bgk, _ = st.max_stable_mach(torch, "D2Q9", "BGK", 2, 1e4)
    print(f"[stability] D2Q9 Re 1e4: PR4 {m_pr}, BGK {m_bgk}", flush=True)
    assert m_pr == m_bgk > 0.3


@pytest.mark.parametrize("name,n_eq", [("D2Q9", 4), ("D2V17", 3)])
@pytest.mark.parametrize("re", [3e4, 1e5])
def test_rr_more_stable_than_pr(env, name, n_eq, re):
    torch, st = env
    print(f"[case] stability {name} Re {re:.0e}", flush=True)
    m_pr, _ = st.max_stable_mach(torch, name, "PR", n_eq, re)
    m_rr = max(st.max_stable_mach(torch, name, "RR", k, re)[0] for k in range(2, n_eq + 1))
    print(f"[stability] {name} Re {re:.0e}: PR{n_eq} {m_pr}, best RR {m_rr}", flush=True)
    assert m_rr > m_pr + 0.02
