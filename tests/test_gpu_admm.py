"""GPU parity of Algorithm 1 (Dual Forward-Backward ADMM) against the oracle.

The workload is the 64^2 image / 8192-visibility configuration with J = 4,
D = 2000, SARA (Dirac + db1..db8) at 3 levels, 30 dB noise. Each side computes
its own operator norm by the power method; gamma and epsilon are inputs.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import admm, measurement as ms, wavelets as wv
from gpu_util import DEV, make_plan, purimi, rel_l2, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return purimi()


def c0_problem(iters):
    w = W.CONFIGS["admm64"]
    rng = W.rng_for(w.index)
    x_true = W.make_sky(w, rng)
    uv = W.make_uv(w, rng)                        # float32 baselines
    spec = ms.PhiSpec(w.n, w.K, w.J, w.D)
    uv64 = uv.astype(np.float64)
    y0 = ms.phi(x_true, uv64, None, spec)
    y, sigma, eps = W.add_noise(y0, W.unit_complex_noise(w.M, rng), w.snr_db)
    return w, x_true, uv, uv64, spec, y, eps


def oracle_run(w, uv64, spec, y, eps, iters, norm_iters=100):
    nrm = ms.power_method(uv64, None, spec, iters=norm_iters)
    phi = lambda x: ms.phi(x, uv64, None, spec) / nrm
    phi_adj = lambda v: ms.phi_adjoint(v, uv64, None, spec) / nrm
    S = wv.Sara(w.n, w.levels)
    gamma = admm.default_gamma(y, phi_adj, S.adjoint)
    p = admm.AdmmParams(gamma=gamma, iters=iters)
    x, s, d, rep = admm.admm(y, phi, phi_adj, S.forward, S.adjoint, eps, p, np.zeros((w.n, w.n)))
    return x, rep, gamma, nrm


@pytest.mark.parametrize("prec,tol,iters", [("f64", 1e-10, 50), ("f32", 1e-4, 50), ("f64", 1e-10, 3)])
def test_admm_parity_admm64(P, prec, tol, iters):
    say(f"admm admm64 {prec} iters={iters}")
    w, x_true, uv, uv64, spec, y, eps = c0_problem(iters)
    x_ref, rep_ref, gamma, nrm_ref = oracle_run(w, uv64, spec, y, eps, iters)
    uv_dev = uv if prec == "f32" else uv64
    plan, perm = make_plan(P, w.n, uv_dev, None, w.J, w.D, prec)
    pprec = P.PR_F32 if prec == "f32" else P.PR_F64
    psi = P.PsiPlan(w.n, w.levels, 0x1FF, pprec, DEV)
    nrm = plan.norm(100)
    assert nrm == pytest.approx(nrm_ref, rel=1e-5 if prec == "f32" else 1e-12)
    cdt = torch.complex64 if prec == "f32" else torch.complex128
    y_plan = to_dev(y[perm], cdt)
    prm = P.admm_params(eps, gamma, iters=iters, op_norm=nrm)
    x, rep = P.admm_solve(plan, psi, y_plan, prm)
    xg = x.cpu().numpy()
    assert rep.iters_done == iters and rep.nonfinite == 0
    assert rel_l2(xg, x_ref) <= tol
    assert rep.resid_norm == pytest.approx(rep_ref.resid[-1], rel=max(tol, 1e-9) * 10)
    assert rep.rel_var == pytest.approx(rep_ref.rel_var[-1], rel=0.05 if prec == "f32" else 1e-6)
    assert rep.l1_norm == pytest.approx(rep_ref.l1[-1], rel=max(tol, 1e-9) * 10)
    assert np.all(xg >= 0)


def test_admm_is_bitwise_reproducible(P):
    say("admm determinism")
    w, x_true, uv, uv64, spec, y, eps = c0_problem(5)
    plan, perm = make_plan(P, w.n, uv, None, w.J, w.D, "f32")
    psi = P.PsiPlan(w.n, w.levels, 0x1FF, P.PR_F32, DEV)
    y_plan = to_dev(y[perm], torch.complex64)
    prm = P.admm_params(eps, 0.3, iters=5, op_norm=plan.norm(20))
    a, ra = P.admm_solve(plan, psi, y_plan, prm)
    b, rb = P.admm_solve(plan, psi, y_plan, prm)
    assert torch.equal(a, b)
    assert ra.resid_norm == rb.resid_norm and ra.l1_norm == rb.l1_norm
