"""GPU parity of the Primal-Dual algorithm against the oracle.

Workload: the 64^2 image / 8192-visibility configuration (D = 2000, SARA at
3 levels, 30 dB noise), both misfits (the l2 ball of Algorithm 1's
constrained problem and the MAP least-squares term), the gridding walk
(J = 4) and the J-lane gridding (J = 6).
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import admm, measurement as ms, primal_dual as pd, wavelets as wv
from gpu_util import DEV, make_plan, purimi, rel_l2, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return purimi()


def c0_data(J=None, interp="nearest"):
    w = W.CONFIGS["admm64"]
    rng = W.rng_for(w.index)
    x_true = W.make_sky(w, rng)
    uv = W.make_uv(w, rng)
    J = w.J if J is None else J
    spec = ms.PhiSpec(w.n, w.K, J, w.D, interp)
    uv64 = uv.astype(np.float64)
    y0 = ms.phi(x_true, uv64, None, spec)
    y, _, eps = W.add_noise(y0, W.unit_complex_noise(w.M, rng), w.snr_db)
    return w, J, uv, uv64, spec, y, eps


def oracle_pd(w, uv64, spec, y, eps, misfit, iters, tau, sigma, theta, inner=1):
    nrm = ms.power_method(uv64, None, spec, iters=100)
    phi = lambda x: ms.phi(x, uv64, None, spec) / nrm
    phi_adj = lambda v: ms.phi_adjoint(v, uv64, None, spec) / nrm
    S = wv.Sara(w.n, w.levels)
    gamma = admm.default_gamma(y, phi_adj, S.adjoint)
    x, z, d, rep = pd.primal_dual(y, phi, phi_adj, S.forward, S.adjoint, gamma, tau, sigma, theta, iters,
                                  np.zeros((w.n, w.n)), misfit=misfit, eps=eps, inner_iters=inner)
    return x, rep, gamma, nrm


def run_gpu(P, w, J, uv, uv64, y, prec, prm, interp=0):
    plan, perm = make_plan(P, w.n, uv if prec == "f32" else uv64, None, J, w.D, prec, interp=interp)
    psi = P.PsiPlan(w.n, w.levels, 0x1FF, P.PR_F32 if prec == "f32" else P.PR_F64, DEV)
    y_plan = to_dev(y[perm], torch.complex64 if prec == "f32" else torch.complex128)
    return P.pd_solve(plan, psi, y_plan, prm)


@pytest.mark.parametrize("misfit,prec,tol,iters,theta,inner,J", [
    ("ball", "f64", 1e-10, 50, 1.0, 1, 4),
    ("ball", "f32", 1e-4, 50, 1.0, 1, 4),
    ("l2", "f64", 1e-10, 50, 1.0, 1, 4),
    ("l2", "f32", 1e-4, 50, 1.0, 1, 4),
    ("ball", "f64", 1e-10, 10, 0.0, 3, 4),
    ("l2", "f64", 1e-10, 10, 0.5, 1, 6),
    ("ball", "f64", 1e-10, 10, 1.0, 1, 6),
])
def test_pd_parity_admm64(P, misfit, prec, tol, iters, theta, inner, J):
    say(f"pd admm64 {misfit} {prec} iters={iters} theta={theta} inner={inner} J={J}")
    w, J, uv, uv64, spec, y, eps = c0_data(J)
    tau, sigma = 0.5, 1.0
    x_ref, rep_ref, gamma, nrm = oracle_pd(w, uv64, spec, y, eps, misfit, iters, tau, sigma, theta, inner)
    mis = P.PR_PD_BALL if misfit == "ball" else P.PR_PD_L2
    x, rep = run_gpu(P, w, J, uv, uv64, y, prec,
                     P.pd_params(gamma, tau, sigma, theta, iters=iters, misfit=mis, eps=eps, inner_iters=inner,
                                 op_norm=nrm))
    xg = x.cpu().numpy()
    assert rep.iters_done == iters and rep.nonfinite == 0
    assert rel_l2(xg, x_ref) <= tol
    assert np.all(xg >= 0)
    assert rep.resid_norm == pytest.approx(rep_ref.resid[-1], rel=max(tol, 1e-9) * 10)
    assert rep.l1_norm == pytest.approx(rep_ref.l1[-1], rel=max(tol, 1e-9) * 10)
    assert rep.rel_var == pytest.approx(rep_ref.rel_var[-1], rel=0.05 if prec == "f32" else 1e-6)


def test_pd_device_norm_and_gamma(P):
    say("pd admm64 f64 device norm and gamma")
    w, J, uv, uv64, spec, y, eps = c0_data()
    x_ref, _, gamma, nrm = oracle_pd(w, uv64, spec, y, eps, "ball", 20, 0.5, 1.0, 1.0)
    x, rep = run_gpu(P, w, J, uv, uv64, y, "f64",
                     P.pd_params(0.0, 0.5, 1.0, 1.0, iters=20, eps=eps, gamma_factor=1e-3, norm_iters=100))
    assert rep.op_norm == pytest.approx(nrm, rel=1e-12)
    assert rel_l2(x.cpu().numpy(), x_ref) <= 1e-9


def test_pd_parameter_checks_and_determinism(P):
    say("pd parameter checks, determinism")
    w, J, uv, uv64, spec, y, eps = c0_data()
    plan, perm = make_plan(P, w.n, uv, None, J, w.D, "f32")
    psi = P.PsiPlan(w.n, w.levels, 0x1FF, P.PR_F32, DEV)
    y_plan = to_dev(y[perm], torch.complex64)
    nrm = plan.norm(20)
    for bad in (dict(theta=1.5), dict(tau=0.0), dict(misfit=7), dict(eps=-1.0)):
        kw = dict(iters=2, eps=eps, op_norm=nrm)
        kw.update(bad)
        with pytest.raises(P.PrError) as e:
            P.pd_solve(plan, psi, y_plan, P.pd_params(0.01, **kw))
        assert e.value.code == P.PR_EINVAL
    prm = P.pd_params(0.01, iters=7, eps=eps, op_norm=nrm)
    a, _ = P.pd_solve(plan, psi, y_plan, prm)
    b, _ = P.pd_solve(plan, psi, y_plan, prm)
    assert torch.equal(a, b)


@pytest.mark.parametrize("misfit", ["ball", "l2"])
def test_pd_first_order_lookup(P, misfit):
    say(f"pd admm64 first-order lookup {misfit} f64")
    w, J, uv, uv64, spec, y, eps = c0_data(interp="linear")
    x_ref, _, gamma, nrm = oracle_pd(w, uv64, spec, y, eps, misfit, 10, 0.5, 1.0, 1.0)
    mis = P.PR_PD_BALL if misfit == "ball" else P.PR_PD_L2
    x, rep = run_gpu(P, w, J, uv, uv64, y, "f64",
                     P.pd_params(gamma, 0.5, 1.0, 1.0, iters=10, misfit=mis, eps=eps, op_norm=nrm), interp=1)
    assert rep.nonfinite == 0
    assert rel_l2(x.cpu().numpy(), x_ref) <= 1e-10
