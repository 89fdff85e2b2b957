"""GPU parity of the SARA dictionary against the FP64 oracle."""
import numpy as np
import pytest
import torch

from oracle import wavelets as wv
from gpu_util import DEV, purimi, rel_l2, say, to_dev

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "f64": 1e-12}


@pytest.fixture(scope="module")
def P():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return purimi()


def _rdt(prec):
    return torch.float32 if prec == "f32" else torch.float64


def test_filters_agree_with_the_oracle_derivation(P):
    say("psi filters")
    plan = P.PsiPlan(16, 2, 0x1FF, P.PR_F64, DEV)
    for k in range(1, 9):
        got = np.array(P.pr_psi_filter(plan.handle, k))
        assert np.max(np.abs(got - wv.daubechies_lowpass(k))) < 1e-14


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("n,levels,mask", [
    (64, 3, 0x1FF), (32, 4, 0x1FF), (256, 4, 0x1FF), (16, 3, 0b110), (8, 2, 0x1), (128, 1, 0x180),
])
def test_analysis_and_synthesis_parity(P, prec, n, levels, mask):
    say(f"psi parity {prec} n={n} L={levels} mask={mask:#x}")
    plan = P.PsiPlan(n, levels, mask, P.PR_F32 if prec == "f32" else P.PR_F64, DEV)
    S = wv.Sara(n, levels, mask)
    assert plan.nb == S.nb
    rng = np.random.default_rng(n * 10 + levels)
    x = rng.standard_normal((n, n))
    a_gpu = plan.adjoint(to_dev(x, _rdt(prec))).cpu().numpy()
    a_ref = S.adjoint(x)
    for b in range(S.nb):
        assert rel_l2(a_gpu[b], a_ref[b]) <= TOL[prec], S.bases[b]
    alpha = rng.standard_normal((S.nb, n, n))
    x_gpu = plan.apply(to_dev(alpha, _rdt(prec))).cpu().numpy()
    assert rel_l2(x_gpu, S.forward(alpha)) <= TOL[prec]


def test_tight_frame_on_gpu(P):
    n = 128
    say("psi tight frame")
    plan = P.PsiPlan(n, 4, 0x1FF, P.PR_F64, DEV)
    x = torch.randn((n, n), dtype=torch.float64, device=DEV)
    back = plan.apply(plan.adjoint(x))
    assert torch.max(torch.abs(back - x)).item() < 1e-12
