"""Tile autotuner and the two-launch form of the gridding stage.

The autotuner must return an admissible tile side whose plan gives the same
operator as the oracle; gridding run as patches-then-merge must equal the
one-call gridding bit for bit.
"""
import numpy as np
import pytest
import torch

from oracle import measurement as ms
from gpu_util import DEV, problem, purimi, rel_l2, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return purimi()


@pytest.mark.parametrize("n,M,J", [(64, 30000, 4), (128, 200000, 4), (64, 5000, 6)])
def test_tuned_plan_matches_oracle(P, n, M, J):
    say(f"tune n={n} M={M} J={J}")
    x, uv, _, spec = problem(n, M, J=J, seed=7)
    uv_d = to_dev(uv, torch.float32)
    T = P.tune_tile(n, uv_d, J=J)
    assert T in (8, 16, 32)
    plan = P.PhiPlan(n, uv_d, None, J=J, D=2000, tile=T)
    assert plan.desc.tile == T
    y = plan.apply(to_dev(x, torch.float32))
    perm = plan.perm().cpu().numpy()
    y_ref = ms.phi(x, uv.astype(np.float64), None, spec)
    assert rel_l2(y.cpu().numpy(), y_ref[perm]) <= 1e-5


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_patches_then_merge_equals_gridding(P, prec):
    say(f"grid parts {prec}")
    rdt = torch.float32 if prec == "f32" else torch.float64
    x, uv, w, spec = problem(64, 40000, seed=9, prec=prec, weights=True)
    plan = P.PhiPlan(64, to_dev(uv, rdt), to_dev(w, rdt), J=4, D=2000)
    y = plan.apply(to_dev(x, rdt))
    a = torch.empty((64, 64), dtype=rdt, device=DEV)
    b = torch.empty_like(a)
    P.pr_phi_gw_adjoint(plan.handle, y)
    P.pr_phi_fzs_adjoint(plan.handle, a)
    P.pr_phi_grid_patches(plan.handle, y)
    P.pr_phi_grid_merge(plan.handle)
    P.pr_phi_fzs_adjoint(plan.handle, b)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
