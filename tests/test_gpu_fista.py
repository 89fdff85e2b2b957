"""GPU parity of FISTA (Algorithm "FISTA", MAP problem) against the oracle.

Workload: the 64^2 image / 8192-visibility configuration (J = 4, D = 2000,
SARA at 3 levels, 30 dB noise). The prox of gamma lambda g is the DualFB of
Algorithm 1 on both sides, with the dual variable carried over.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import admm, fista, measurement as ms, wavelets as wv
from gpu_util import DEV, make_plan, purimi, rel_l2, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return purimi()


def c0_data(interp="nearest"):
    w = W.CONFIGS["admm64"]
    rng = W.rng_for(w.index)
    x_true = W.make_sky(w, rng)
    uv = W.make_uv(w, rng)
    spec = ms.PhiSpec(w.n, w.K, w.J, w.D, interp)
    uv64 = uv.astype(np.float64)
    y0 = ms.phi(x_true, uv64, None, spec)
    y, _, _ = W.add_noise(y0, W.unit_complex_noise(w.M, rng), w.snr_db)
    return w, uv, uv64, spec, y


def oracle_fista(w, uv64, spec, y, iters, lam, inner_iters=1, norm_iters=100):
    nrm = ms.power_method(uv64, None, spec, iters=norm_iters)
    phi = lambda x: ms.phi(x, uv64, None, spec) / nrm
    phi_adj = lambda v: ms.phi_adjoint(v, uv64, None, spec) / nrm
    S = wv.Sara(w.n, w.levels)
    gamma = admm.default_gamma(y, phi_adj, S.adjoint)
    x, d, rep = fista.fista(y, phi, phi_adj, S.forward, S.adjoint, gamma, lam, iters,
                            np.zeros((w.n, w.n)), inner_iters=inner_iters)
    obj = fista.objective(x, y, phi, S.adjoint, gamma)
    return x, rep, gamma, nrm, obj


def run_gpu(P, w, uv, uv64, y, prec, prm, interp=0):
    plan, perm = make_plan(P, w.n, uv if prec == "f32" else uv64, None, w.J, w.D, prec, interp=interp)
    psi = P.PsiPlan(w.n, w.levels, 0x1FF, P.PR_F32 if prec == "f32" else P.PR_F64, DEV)
    cdt = torch.complex64 if prec == "f32" else torch.complex128
    y_plan = to_dev(y[perm], cdt)
    return plan, P.fista_solve(plan, psi, y_plan, prm)


@pytest.mark.parametrize("prec,tol,iters,inner", [
    ("f64", 1e-10, 50, 1), ("f32", 1e-4, 50, 1), ("f64", 1e-10, 10, 3), ("f64", 1e-10, 1, 1)])
def test_fista_parity_admm64(P, prec, tol, iters, inner):
    say(f"fista admm64 {prec} iters={iters} inner={inner}")
    w, uv, uv64, spec, y = c0_data()
    lam = 1.0
    x_ref, rep_ref, gamma, nrm, _ = oracle_fista(w, uv64, spec, y, iters, lam, inner)
    plan, (x, rep) = run_gpu(P, w, uv, uv64, y, prec,
                             P.fista_params(gamma, lam, iters=iters, inner_iters=inner, op_norm=nrm))
    xg = x.cpu().numpy()
    assert rep.iters_done == iters and rep.nonfinite == 0
    assert rel_l2(xg, x_ref) <= tol
    assert np.all(xg >= 0)
    assert rep.resid_norm == pytest.approx(rep_ref.resid[-1], rel=max(tol, 1e-9) * 10)
    assert rep.l1_norm == pytest.approx(rep_ref.l1[-1], rel=max(tol, 1e-9) * 10)


def test_fista_device_norm_and_gamma(P):
    say("fista admm64 f64 device norm and gamma")
    w, uv, uv64, spec, y = c0_data()
    x_ref, rep_ref, gamma, nrm, _ = oracle_fista(w, uv64, spec, y, 20, 0.9)
    _, (x, rep) = run_gpu(P, w, uv, uv64, y, "f64",
                          P.fista_params(0.0, 0.9, iters=20, gamma_factor=1e-3, norm_iters=100))
    assert rep.op_norm == pytest.approx(nrm, rel=1e-12)
    assert rel_l2(x.cpu().numpy(), x_ref) <= 1e-9


def test_fista_reaches_the_oracle_objective(P):
    say("fista admm64 f32 objective")
    w, uv, uv64, spec, y = c0_data()
    x_ref, _, gamma, nrm, obj_ref = oracle_fista(w, uv64, spec, y, 100, 1.0)
    _, (x, _) = run_gpu(P, w, uv, uv64, y, "f32", P.fista_params(gamma, 1.0, iters=100, op_norm=nrm))
    phi = lambda v: ms.phi(v, uv64, None, spec) / nrm
    S = wv.Sara(w.n, w.levels)
    obj = fista.objective(x.cpu().numpy().astype(np.float64), y, phi, S.adjoint, gamma)
    assert obj == pytest.approx(obj_ref, rel=1e-4)


def test_fista_zero_iterations_and_determinism(P):
    say("fista zero iterations, determinism")
    w, uv, uv64, spec, y = c0_data()
    plan, perm = make_plan(P, w.n, uv, None, w.J, w.D, "f32")
    psi = P.PsiPlan(w.n, w.levels, 0x1FF, P.PR_F32, DEV)
    y_plan = to_dev(y[perm], torch.complex64)
    x0 = torch.rand((w.n, w.n), dtype=torch.float32, device=DEV)
    x, rep = P.fista_solve(plan, psi, y_plan, P.fista_params(0.01, 1.0, iters=0, op_norm=plan.norm(20)), x0)
    assert rep.iters_done == 0 and torch.equal(x, x0)
    prm = P.fista_params(0.01, 1.0, iters=7, op_norm=plan.norm(20))
    a, _ = P.fista_solve(plan, psi, y_plan, prm)
    b, _ = P.fista_solve(plan, psi, y_plan, prm)
    assert torch.equal(a, b)


@pytest.mark.parametrize("prec,tol", [("f64", 1e-10), ("f32", 1e-4)])
def test_fista_first_order_lookup(P, prec, tol):
    say(f"fista admm64 first-order lookup {prec}")
    w, uv, uv64, spec, y = c0_data("linear")
    x_ref, _, gamma, nrm, _ = oracle_fista(w, uv64, spec, y, 20, 1.0)
    _, (x, rep) = run_gpu(P, w, uv, uv64, y, prec, P.fista_params(gamma, 1.0, iters=20, op_norm=nrm), interp=1)
    assert rep.nonfinite == 0
    assert rel_l2(x.cpu().numpy(), x_ref) <= tol
