"""GPU parity at the sizes the benchmark times.

256^2 image / 10^6 visibilities (J = 4 and 6, SARA at 4 levels): Phi and
Phi^dagger element by element, and three iterations of Algorithm 1 in the
plan and launch configuration `bench.py` times. At this size the wavelet
levels of 256 and 128 run in the per-level kernels with the DualFB update fused
into the analysis stores, and the gridding work items span several staged
chunks, which the 64^2 workload never reaches.

128^2 image / 4*10^4 visibilities, SARA at 3 levels: FISTA, Primal-Dual,
local l2 balls (8 baseline-length sections) and reweighting.

The oracle's operator norm (power method, a few steps) is the op_norm of both
sides, so both solve the same normalised problem; gamma and epsilon follow the
data generation of the workloads.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import admm, fista, measurement as ms, primal_dual as pd, reweight as rw, wavelets as wv
from gpu_util import DEV, make_plan, max_rel, purimi, rel_l2, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return purimi()


class Data:
    """Seeded inputs of a workload and the oracle's normalised operators."""

    def __init__(self, key, J=None, norm_iters=8):
        w = W.CONFIGS[key]
        rng = W.rng_for(w.index)
        self.w = w
        self.J = w.J if J is None else J
        self.x_true = W.make_sky(w, rng)
        self.uv = W.make_uv(w, rng)
        self.uv64 = self.uv.astype(np.float64)
        self.spec = ms.PhiSpec(w.n, w.K, self.J, w.D)
        y0 = ms.phi(self.x_true, self.uv64, None, self.spec)
        self.y, self.sigma, self.eps = W.add_noise(y0, W.unit_complex_noise(w.M, rng), w.snr_db)
        self.nrm = ms.power_method(self.uv64, None, self.spec, iters=norm_iters)
        self.S = wv.Sara(w.n, w.levels)
        self.gamma = admm.default_gamma(self.y, self.phi_adj, self.S.adjoint)

    def phi(self, x):
        return ms.phi(x, self.uv64, None, self.spec) / self.nrm

    def phi_adj(self, v):
        return ms.phi_adjoint(v, self.uv64, None, self.spec) / self.nrm

    def gpu(self, P, prec):
        plan, perm = make_plan(P, self.w.n, self.uv if prec == "f32" else self.uv64, None, self.J, self.w.D, prec)
        psi = P.PsiPlan(self.w.n, self.w.levels, 0x1FF, P.PR_F32 if prec == "f32" else P.PR_F64, DEV)
        y_plan = to_dev(self.y[perm], torch.complex64 if prec == "f32" else torch.complex128)
        return plan, perm, psi, y_plan


@pytest.fixture(scope="module")
def op256():
    return Data("op256")


@pytest.fixture(scope="module")
def mid128():
    return Data("mid128", norm_iters=20)


# ---------------------------------------------------------------------------
# operators at 256^2 / 10^6
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("prec,J", [("f32", 4), ("f64", 4), ("f32", 6)])
def test_phi_elementwise_op256(P, prec, J):
    say(f"phi elementwise 256^2/1e6 {prec} J={J}")
    w = W.CONFIGS["op256"]
    rng = W.rng_for(w.index)
    x = W.make_sky(w, rng)
    uv = W.make_uv(w, rng)
    uv64 = uv.astype(np.float64)
    spec = ms.PhiSpec(w.n, w.K, J, w.D)
    plan, perm = make_plan(P, w.n, uv if prec == "f32" else uv64, None, J, w.D, prec)
    rdt = torch.float32 if prec == "f32" else torch.float64
    cdt = torch.complex64 if prec == "f32" else torch.complex128
    y_gpu = plan.apply(to_dev(x, rdt)).cpu().numpy()
    y_ref = ms.phi(x, uv64, None, spec)[perm]
    tol_l2, tol_max = (1e-5, 1e-4) if prec == "f32" else (1e-12, 1e-11)
    assert rel_l2(y_gpu, y_ref) <= tol_l2
    assert max_rel(y_gpu, y_ref) <= tol_max
    # the adjoint on data visibilities (the dirty map) and on random ones
    for yy in (y_ref, (lambda g: g.standard_normal(w.M) + 1j * g.standard_normal(w.M))(np.random.default_rng(11))):
        x_gpu = plan.adjoint(to_dev(yy, cdt)).cpu().numpy()
        inv = np.empty_like(perm)
        inv[perm] = np.arange(perm.size)
        x_ref = ms.phi_adjoint(yy[inv], uv64, None, spec)
        assert rel_l2(x_gpu, x_ref) <= tol_l2
        assert max_rel(x_gpu, x_ref) <= tol_max


# ---------------------------------------------------------------------------
# Algorithm 1 at 256^2 / 10^6, SARA 4 levels
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def admm_op256_ref(op256):
    d = op256
    x, s, dd, rep = admm.admm(d.y, d.phi, d.phi_adj, d.S.forward, d.S.adjoint, d.eps,
                              admm.AdmmParams(gamma=d.gamma, iters=3), np.zeros((d.w.n, d.w.n)))
    return x, rep


@pytest.mark.parametrize("prec,tol", [("f64", 1e-10), ("f32", 1e-4)])
def test_admm_op256(P, op256, admm_op256_ref, prec, tol):
    say(f"admm 256^2/1e6 SARA-4 3 iterations {prec}")
    d = op256
    x_ref, rep_ref = admm_op256_ref
    plan, perm, psi, y_plan = d.gpu(P, prec)
    x, rep = P.admm_solve(plan, psi, y_plan, P.admm_params(d.eps, d.gamma, iters=3, op_norm=d.nrm))
    xg = x.cpu().numpy()
    assert rep.iters_done == 3 and rep.nonfinite == 0
    assert rel_l2(xg, x_ref) <= tol
    assert max_rel(xg, x_ref) <= 10 * tol
    assert np.all(xg >= 0)
    assert rep.resid_norm == pytest.approx(rep_ref.resid[-1], rel=max(tol, 1e-9) * 10)
    assert rep.l1_norm == pytest.approx(rep_ref.l1[-1], rel=max(tol, 1e-9) * 10)


def test_admm_op256_one_iteration_fp32(P, op256):
    """One iteration in FP32: the error of a single DualFB step at this size."""
    say("admm 256^2/1e6 one iteration f32")
    d = op256
    x_ref, _, _, _ = admm.admm(d.y, d.phi, d.phi_adj, d.S.forward, d.S.adjoint, d.eps,
                               admm.AdmmParams(gamma=d.gamma, iters=1), np.zeros((d.w.n, d.w.n)))
    plan, perm, psi, y_plan = d.gpu(P, "f32")
    x, rep = P.admm_solve(plan, psi, y_plan, P.admm_params(d.eps, d.gamma, iters=1, op_norm=d.nrm))
    assert rel_l2(x.cpu().numpy(), x_ref) <= 1e-5


# ---------------------------------------------------------------------------
# the other solvers at 128^2 / 4*10^4, SARA 3 levels
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("prec,tol", [("f64", 1e-10), ("f32", 1e-4)])
def test_fista_mid128(P, mid128, prec, tol):
    say(f"fista 128^2/4e4 {prec}")
    d = mid128
    iters = 20
    x_ref, _, rep_ref = fista.fista(d.y, d.phi, d.phi_adj, d.S.forward, d.S.adjoint, d.gamma, 1.0, iters,
                                    np.zeros((d.w.n, d.w.n)))
    plan, perm, psi, y_plan = d.gpu(P, prec)
    x, rep = P.fista_solve(plan, psi, y_plan, P.fista_params(d.gamma, 1.0, iters=iters, op_norm=d.nrm))
    assert rep.iters_done == iters and rep.nonfinite == 0
    assert rel_l2(x.cpu().numpy(), x_ref) <= tol
    assert rep.resid_norm == pytest.approx(rep_ref.resid[-1], rel=max(tol, 1e-9) * 10)


@pytest.mark.parametrize("misfit,prec,tol", [("ball", "f64", 1e-10), ("ball", "f32", 1e-4), ("l2", "f64", 1e-10)])
def test_primal_dual_mid128(P, mid128, misfit, prec, tol):
    say(f"primal-dual 128^2/4e4 {misfit} {prec}")
    d = mid128
    iters, tau, sigma, theta = 20, 0.5, 1.0, 1.0
    x_ref, _, _, rep_ref = pd.primal_dual(d.y, d.phi, d.phi_adj, d.S.forward, d.S.adjoint, d.gamma, tau, sigma,
                                          theta, iters, np.zeros((d.w.n, d.w.n)), misfit=misfit, eps=d.eps)
    plan, perm, psi, y_plan = d.gpu(P, prec)
    mis = P.PR_PD_BALL if misfit == "ball" else P.PR_PD_L2
    x, rep = P.pd_solve(plan, psi, y_plan, P.pd_params(d.gamma, tau, sigma, theta, iters=iters, misfit=mis,
                                                       eps=d.eps, op_norm=d.nrm))
    assert rep.iters_done == iters and rep.nonfinite == 0
    assert rel_l2(x.cpu().numpy(), x_ref) <= tol
    assert rep.resid_norm == pytest.approx(rep_ref.resid[-1], rel=max(tol, 1e-9) * 10)


@pytest.mark.parametrize("prec,tol", [("f64", 1e-10), ("f32", 1e-4)])
def test_local_balls_mid128(P, mid128, prec, tol):
    say(f"local balls 128^2/4e4 8 sections {prec}")
    d = mid128
    nsec, iters = 8, 20
    order = np.argsort(np.hypot(d.uv64[:, 0], d.uv64[:, 1]), kind="stable")
    sec = np.empty(d.w.M, dtype=np.int32)
    for j, part in enumerate(np.array_split(order, nsec)):
        sec[part] = j
    m = np.bincount(sec, minlength=nsec).astype(np.float64)
    eps_j = d.sigma * np.sqrt(m + 2.0 * np.sqrt(m))
    x_ref, _, _, rep_ref = admm.admm(d.y, d.phi, d.phi_adj, d.S.forward, d.S.adjoint, eps_j,
                                     admm.AdmmParams(gamma=d.gamma, iters=iters), np.zeros((d.w.n, d.w.n)),
                                     sections=sec)
    plan, perm, psi, y_plan = d.gpu(P, prec)
    balls = P.Balls(plan, torch.as_tensor(sec[perm]).to(DEV), nsec)
    x, rep = P.admm_local_solve(plan, psi, balls, y_plan, P.admm_params(0.0, d.gamma, iters=iters, op_norm=d.nrm),
                                eps_j)
    assert rep.iters_done == iters and rep.nonfinite == 0
    assert rel_l2(x.cpu().numpy(), x_ref) <= tol
    assert rep.resid_norm == pytest.approx(rep_ref.resid[-1], rel=max(tol, 1e-9) * 10)


@pytest.mark.parametrize("prec,tol", [("f64", 1e-10), ("f32", 1e-4)])
def test_reweighted_mid128(P, mid128, prec, tol):
    say(f"reweighting 128^2/4e4 2 rounds {prec}")
    d = mid128
    iters, rounds, delta0, beta = 10, 2, 1e-3, 0.5
    x_ref, _, reps = rw.sara_reweighted(d.y, d.phi, d.phi_adj, d.S.forward, d.S.adjoint, d.eps,
                                        admm.AdmmParams(gamma=d.gamma, iters=iters), rounds, delta0, beta,
                                        np.zeros((d.w.n, d.w.n)))
    plan, perm, psi, y_plan = d.gpu(P, prec)
    x, rep = P.admm_reweighted_solve(plan, psi, y_plan, P.admm_params(d.eps, d.gamma, iters=iters, op_norm=d.nrm),
                                     rounds, delta0, beta)
    assert rep.iters_done == iters * (rounds + 1) and rep.nonfinite == 0
    assert rel_l2(x.cpu().numpy(), x_ref) <= tol
    assert rep.l1_norm == pytest.approx(reps[-1].l1[-1], rel=max(tol, 1e-9) * 10)
