"""GPU parity of the reweighted analysis l1 (SARA reweighting around
Algorithm 1) against the oracle, on the 64^2 image / 8192-visibility
workload: round 0 unweighted, then rounds with w = delta / (delta + |Psi^dagger x|)."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import admm, measurement as ms, reweight as rw, wavelets as wv
from gpu_util import DEV, make_plan, purimi, rel_l2, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return purimi()


def c0_data():
    w = W.CONFIGS["admm64"]
    rng = W.rng_for(w.index)
    x_true = W.make_sky(w, rng)
    uv = W.make_uv(w, rng)
    spec = ms.PhiSpec(w.n, w.K, w.J, w.D)
    uv64 = uv.astype(np.float64)
    y0 = ms.phi(x_true, uv64, None, spec)
    y, _, eps = W.add_noise(y0, W.unit_complex_noise(w.M, rng), w.snr_db)
    return w, uv, uv64, spec, y, eps


def oracle_rw(w, uv64, spec, y, eps, iters, rounds, delta0, beta):
    nrm = ms.power_method(uv64, None, spec, iters=100)
    phi = lambda x: ms.phi(x, uv64, None, spec) / nrm
    phi_adj = lambda v: ms.phi_adjoint(v, uv64, None, spec) / nrm
    S = wv.Sara(w.n, w.levels)
    gamma = admm.default_gamma(y, phi_adj, S.adjoint)
    x, wts, reps = rw.sara_reweighted(y, phi, phi_adj, S.forward, S.adjoint, eps, admm.AdmmParams(gamma=gamma, iters=iters),
                                      rounds, delta0, beta, np.zeros((w.n, w.n)))
    return x, reps, gamma, nrm


def run_gpu(P, w, uv, uv64, y, prec, prm, rounds, delta0, beta):
    plan, perm = make_plan(P, w.n, uv if prec == "f32" else uv64, None, w.J, w.D, prec)
    psi = P.PsiPlan(w.n, w.levels, 0x1FF, P.PR_F32 if prec == "f32" else P.PR_F64, DEV)
    y_plan = to_dev(y[perm], torch.complex64 if prec == "f32" else torch.complex128)
    return P.admm_reweighted_solve(plan, psi, y_plan, prm, rounds, delta0, beta)


@pytest.mark.parametrize("prec,tol,iters,rounds", [("f64", 1e-10, 20, 2), ("f32", 1e-4, 20, 2), ("f64", 1e-10, 5, 0)])
def test_reweighted_parity_admm64(P, prec, tol, iters, rounds):
    say(f"reweighted admm64 {prec} iters={iters} rounds={rounds}")
    w, uv, uv64, spec, y, eps = c0_data()
    delta0, beta = 1e-3, 0.5
    x_ref, reps, gamma, nrm = oracle_rw(w, uv64, spec, y, eps, iters, rounds, delta0, beta)
    x, rep = run_gpu(P, w, uv, uv64, y, prec, P.admm_params(eps, gamma, iters=iters, op_norm=nrm), rounds, delta0, beta)
    xg = x.cpu().numpy()
    assert rep.iters_done == iters * (rounds + 1) and rep.nonfinite == 0
    assert rel_l2(xg, x_ref) <= tol
    assert np.all(xg >= 0)
    assert rep.resid_norm == pytest.approx(reps[-1].resid[-1], rel=max(tol, 1e-9) * 10)
    assert rep.l1_norm == pytest.approx(reps[-1].l1[-1], rel=max(tol, 1e-9) * 10)


def test_reweighted_device_gamma_and_checks(P):
    say("reweighted device norm and gamma, parameter checks")
    w, uv, uv64, spec, y, eps = c0_data()
    x_ref, _, gamma, nrm = oracle_rw(w, uv64, spec, y, eps, 10, 1, 1e-3, 1.0)
    x, rep = run_gpu(P, w, uv, uv64, y, "f64", P.admm_params(eps, 0.0, iters=10, gamma_factor=1e-3, norm_iters=100),
                     1, 1e-3, 1.0)
    assert rel_l2(x.cpu().numpy(), x_ref) <= 1e-9
    for bad in ((1, 0.0, 0.5), (1, 1e-3, 1.5), (-1, 1e-3, 0.5)):
        with pytest.raises(P.PrError) as e:
            run_gpu(P, w, uv, uv64, y, "f32", P.admm_params(eps, 0.01, iters=2, op_norm=1.0), *bad)
        assert e.value.code == P.PR_EINVAL
