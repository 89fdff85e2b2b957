"""First-order (linear) kernel lookup on the GPU against the oracle's
first-order mode: Phi and Phi^dagger element by element over J, tiles and
ragged counts, FP32 <= 1e-5 and FP64 <= 1e-12 relative; the solver path
(fused degridding / gridding of Algorithm 1) for three FP64 iterations.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import admm, measurement as ms, wavelets as wv
from gpu_util import DEV, problem, purimi, rel_l2, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return purimi()


def lin_plan(P, n, uv, w, J, D, prec, tile=0):
    rdt = torch.float32 if prec == "f32" else torch.float64
    plan = P.PhiPlan(n, to_dev(uv, rdt), None if w is None else to_dev(w, rdt), J=J, D=D, tile=tile,
                     prec=P.PR_F32 if prec == "f32" else P.PR_F64, interp=1)
    return plan, plan.perm().cpu().numpy()


@pytest.mark.parametrize("prec,tol", [("f32", 1e-5), ("f64", 1e-12)])
@pytest.mark.parametrize("n,M,J,tile", [(64, 12345, 4, 0), (64, 3001, 6, 0), (32, 999, 2, 8),
                                        (64, 40000, 4, 8), (32, 5000, 8, 8)])
def test_linear_phi_and_adjoint_match_oracle(P, prec, tol, n, M, J, tile):
    say(f"linear phi {prec} n={n} M={M} J={J} tile={tile}")
    x, uv, w, _ = problem(n, M, J=J, seed=M + J, prec=prec, weights=True)
    spec = ms.PhiSpec(n, 2 * n, J, 2000, "linear")
    uv64 = uv.astype(np.float64)
    plan, perm = lin_plan(P, n, uv, w, J, 2000, prec, tile)
    rdt = torch.float32 if prec == "f32" else torch.float64
    cdt = torch.complex64 if prec == "f32" else torch.complex128
    y = plan.apply(to_dev(x, rdt)).cpu().numpy()
    y_ref = ms.phi(x, uv64, w.astype(np.float64), spec)[perm]
    assert rel_l2(y, y_ref) <= tol
    v = np.random.default_rng(M).standard_normal(M) + 1j * np.random.default_rng(M + 1).standard_normal(M)
    xa = plan.adjoint(to_dev(v, cdt)).cpu().numpy()
    xa_ref = ms.phi_adjoint(v[np.argsort(perm)], uv64, w.astype(np.float64), spec)
    assert rel_l2(xa, xa_ref) <= tol


def test_linear_admm_fp64_matches_oracle(P):
    say("linear admm fp64")
    n, M, J = 64, 8192, 4
    rng = np.random.default_rng(77)
    x_true = W.gaussian_sky(n, 20, rng)
    uv = W.uv_gaussian(M, rng).astype(np.float64)
    spec = ms.PhiSpec(n, 2 * n, J, 2000, "linear")
    y0 = ms.phi(x_true, uv, None, spec)
    y, _, eps = W.add_noise(y0, W.unit_complex_noise(M, rng), 30.0)
    nrm = ms.power_method(uv, None, spec, iters=50)
    phi = lambda v: ms.phi(v, uv, None, spec) / nrm
    phi_adj = lambda v: ms.phi_adjoint(v, uv, None, spec) / nrm
    S = wv.Sara(n, 3)
    gamma = admm.default_gamma(y, phi_adj, S.adjoint)
    x_ref, _, _, _ = admm.admm(y, phi, phi_adj, S.forward, S.adjoint, eps, admm.AdmmParams(gamma=gamma, iters=3),
                               np.zeros((n, n)))
    plan, perm = lin_plan(P, n, uv, None, J, 2000, "f64")
    psi = P.PsiPlan(n, 3, 0x1FF, P.PR_F64, DEV)
    nrm_gpu = plan.norm(50)
    assert nrm_gpu == pytest.approx(nrm, rel=1e-12)
    xg, rep = P.admm_solve(plan, psi, to_dev(y[perm], torch.complex128),
                           P.admm_params(eps, gamma, iters=3, op_norm=nrm_gpu))
    assert rep.nonfinite == 0
    assert rel_l2(xg.cpu().numpy(), x_ref) <= 1e-10
