"""Plans with many small gridding items: a large grid sparsely covered, so
that most tiles hold a few visibilities. Their items of at most 64
visibilities are gridded by the small-item kernel (one wave per item)
instead of the segment walk (J <= 4) or the J-lane gridding (J = 6).
Parity of Phi and Phi^dagger and of ADMM
iterations (whose gridding runs the ball projection and multiplier update in
the same kernel) against the oracle, and bitwise repeatability.
"""
import functools

import numpy as np
import pytest
import torch

from oracle import admm, measurement as ms, primal_dual as pd, wavelets as wv
from gpu_util import DEV, make_plan, purimi, rel_l2, say, to_dev
import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "f64": 1e-12}
N, M = 512, 20000          # K = 1024: 4096 tiles of 16 (16384 of 8), about 5 (1) visibilities each


@pytest.fixture(scope="module")
def P():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return purimi()


def sparse_problem(prec, seed):
    rng = np.random.default_rng(seed)
    x = W.gaussian_sky(N, W.n_sources_for(N), rng)
    dt = np.float32 if prec == "f32" else np.float64
    uv = rng.uniform(-3.1, 3.1, (M, 2)).astype(dt)   # uniform over the grid
    return x, uv


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("J", [2, 4, 6])
def test_phi_parity_with_small_items(P, prec, J):
    say(f"small items phi prec={prec} J={J}")
    x, uv = sparse_problem(prec, 11 + J)
    spec = ms.PhiSpec(N, 2 * N, J, 2000)
    plan, perm = make_plan(P, N, uv, None, J, 2000, prec)
    rdt = torch.float32 if prec == "f32" else torch.float64
    cdt = torch.complex64 if prec == "f32" else torch.complex128
    uv64 = uv.astype(np.float64)
    y_gpu = plan.apply(to_dev(x, rdt)).cpu().numpy()
    y_ref = ms.phi(x, uv64, None, spec)[perm]
    assert rel_l2(y_gpu, y_ref) <= TOL[prec]
    rng = np.random.default_rng(J)
    yy = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    xa = plan.adjoint(to_dev(yy[perm], cdt)).cpu().numpy()
    xa_ref = ms.phi_adjoint(yy, uv64, None, spec)
    assert rel_l2(xa, xa_ref) <= TOL[prec]
    # bitwise repeatable
    xb = plan.adjoint(to_dev(yy[perm], cdt)).cpu().numpy()
    assert np.array_equal(xa, xb)


@pytest.mark.parametrize("prec,tol,J", [("f64", 1e-10, 4), ("f32", 1e-4, 4), ("f64", 1e-10, 6)])
def test_admm_parity_with_small_items(P, prec, tol, J):
    """Three ADMM iterations with the same operator scale (the oracle's power
    method, 20 steps) and gamma on both sides: the small-item kernel's ADMM
    prologue."""
    say(f"small items admm prec={prec} J={J}")
    x_true, uv = sparse_problem(prec, 5)
    spec = ms.PhiSpec(N, 2 * N, J, 2000)
    uv64 = uv.astype(np.float64)
    rng = np.random.default_rng(6)
    y0 = ms.phi(x_true, uv64, None, spec)
    y, sigma, eps = W.add_noise(y0, W.unit_complex_noise(M, rng), 30.0)
    nrm = ms.power_method(uv64, None, spec, iters=20)
    gamma, iters, levels = 1e-3, 3, 3
    phi = lambda v: ms.phi(v, uv64, None, spec) / nrm
    phi_adj = lambda v: ms.phi_adjoint(v, uv64, None, spec) / nrm
    S = wv.Sara(N, levels)
    x_ref, _, _, rep_ref = admm.admm(y, phi, phi_adj, S.forward, S.adjoint, eps,
                                     admm.AdmmParams(gamma=gamma, iters=iters), np.zeros((N, N)))
    plan, perm = make_plan(P, N, uv, None, J, 2000, prec)
    pprec = P.PR_F32 if prec == "f32" else P.PR_F64
    psi = P.PsiPlan(N, levels, 0x1FF, pprec, DEV)
    cdt = torch.complex64 if prec == "f32" else torch.complex128
    prm = P.admm_params(eps, gamma, iters=iters, op_norm=nrm)
    x, rep = P.admm_solve(plan, psi, to_dev(y[perm], cdt), prm)
    assert rep.iters_done == iters and rep.nonfinite == 0
    assert rel_l2(x.cpu().numpy(), x_ref) <= tol
    x2, _ = P.admm_solve(plan, psi, to_dev(y[perm], cdt), prm)
    assert torch.equal(x, x2)


@functools.lru_cache(maxsize=None)
def _sparse_admm(J):
    """The sparse problem with noise, the oracle's operator scale and gamma."""
    x_true, uv = sparse_problem("f32", 8)      # FP32 baselines: both precisions see the same values
    spec = ms.PhiSpec(N, 2 * N, J, 2000)
    uv64 = uv.astype(np.float64)
    rng = np.random.default_rng(9)
    y0 = ms.phi(x_true, uv64, None, spec)
    y, sigma, eps = W.add_noise(y0, W.unit_complex_noise(M, rng), 30.0)
    nrm = ms.power_method(uv64, None, spec, iters=20)
    phi = lambda v: ms.phi(v, uv64, None, spec) / nrm
    phi_adj = lambda v: ms.phi_adjoint(v, uv64, None, spec) / nrm
    return dict(uv=uv, uv64=uv64, y=y, sigma=sigma, eps=eps, nrm=nrm, phi=phi, phi_adj=phi_adj,
                S=wv.Sara(N, 3), gamma=1e-3, J=J)


@pytest.fixture(scope="module")
def sparse_admm():
    return _sparse_admm(4)


def _gpu(P, d, prec):
    uv = d["uv"] if prec == "f32" else d["uv64"]
    plan, perm = make_plan(P, N, uv, None, d["J"], 2000, prec)
    psi = P.PsiPlan(N, 3, 0x1FF, P.PR_F32 if prec == "f32" else P.PR_F64, DEV)
    cdt = torch.complex64 if prec == "f32" else torch.complex128
    return plan, perm, psi, to_dev(d["y"][perm], cdt)


@pytest.mark.parametrize("prec,tol,J", [("f64", 1e-10, 4), ("f32", 1e-4, 4), ("f64", 1e-10, 6)])
def test_local_balls_with_small_items(P, prec, tol, J):
    """Four baseline-length sections: the small-item kernel's section-ball
    prologue (after the segment walk at J = 4, after the J-lane gridding at
    J = 6)."""
    say(f"small items local balls prec={prec} J={J}")
    d = _sparse_admm(J)
    nsec, iters = 4, 3
    order = np.argsort(np.hypot(d["uv64"][:, 0], d["uv64"][:, 1]), kind="stable")
    sec = np.empty(M, dtype=np.int32)
    for j, part in enumerate(np.array_split(order, nsec)):
        sec[part] = j
    m = np.bincount(sec, minlength=nsec).astype(np.float64)
    eps_j = d["sigma"] * np.sqrt(m + 2.0 * np.sqrt(m))
    x_ref, _, _, _ = admm.admm(d["y"], d["phi"], d["phi_adj"], d["S"].forward, d["S"].adjoint, eps_j,
                               admm.AdmmParams(gamma=d["gamma"], iters=iters), np.zeros((N, N)), sections=sec)
    plan, perm, psi, y_plan = _gpu(P, d, prec)
    balls = P.Balls(plan, torch.as_tensor(sec[perm]).to(DEV), nsec)
    x, rep = P.admm_local_solve(plan, psi, balls, y_plan,
                                P.admm_params(0.0, d["gamma"], iters=iters, op_norm=d["nrm"]), eps_j)
    assert rep.iters_done == iters and rep.nonfinite == 0
    assert rel_l2(x.cpu().numpy(), x_ref) <= tol


@pytest.mark.parametrize("prec,tol", [("f64", 1e-10), ("f32", 1e-4)])
def test_primal_dual_with_small_items(P, sparse_admm, prec, tol):
    """Primal-Dual with the ball: the gridding prologue without the
    multiplier term."""
    say(f"small items primal-dual prec={prec}")
    d = sparse_admm
    iters, tau, sigma, theta = 3, 0.5, 1.0, 1.0
    x_ref, _, _, _ = pd.primal_dual(d["y"], d["phi"], d["phi_adj"], d["S"].forward, d["S"].adjoint, d["gamma"],
                                    tau, sigma, theta, iters, np.zeros((N, N)), misfit="ball", eps=d["eps"])
    plan, perm, psi, y_plan = _gpu(P, d, prec)
    x, rep = P.pd_solve(plan, psi, y_plan, P.pd_params(d["gamma"], tau, sigma, theta, iters=iters,
                                                       misfit=P.PR_PD_BALL, eps=d["eps"], op_norm=d["nrm"]))
    assert rep.iters_done == iters and rep.nonfinite == 0
    assert rel_l2(x.cpu().numpy(), x_ref) <= tol


def test_fused_batch_with_small_item_members(P):
    """A fused batch whose members split their small items (sparse 512^2
    plans) or do not (a dense 64^2 plan): one walk, one small-item and one
    degridding launch over all of them give each member's own results
    bitwise."""
    say("small items fused batch")
    chs = []
    for i, (n, m, sparse) in enumerate([(512, 20000, True), (64, 8192, False), (512, 12000, True)]):
        rng = np.random.default_rng(40 + i)
        x = W.gaussian_sky(n, W.n_sources_for(n), rng)
        uv = (rng.uniform(-3.1, 3.1, (m, 2)) if sparse else W.uv_gaussian(m, rng)).astype(np.float32)
        plan, _ = make_plan(P, n, uv, None, 4, 2000, "f32", 16)
        psi = P.PsiPlan(n, 3, 0x1FF, P.PR_F32, DEV)
        chs.append(dict(n=n, M=m, x=to_dev(x, torch.float32), plan=plan, psi=psi))
    b = P.Batch(max_members=4, nstreams=2)
    for ch in chs:
        b.add(ch["plan"], ch["psi"], torch.zeros(ch["M"], dtype=torch.complex64, device=DEV),
              P.admm_params(1.0, 1e-3, iters=1, op_norm=1.0))
    b.fuse()
    xs_in = [ch["x"] for ch in chs]
    ys = [torch.empty(ch["M"], dtype=torch.complex64, device=DEV) for ch in chs]
    xs = [torch.empty_like(ch["x"]) for ch in chs]
    P.pr_batch_phi_apply(b.handle, xs_in, ys)
    P.pr_batch_phi_adjoint(b.handle, ys, xs)
    torch.cuda.synchronize()
    for ch, yb, xb in zip(chs, ys, xs):
        assert torch.equal(yb, ch["plan"].apply(ch["x"])), (ch["n"], ch["M"])
        assert torch.equal(xb, ch["plan"].adjoint(yb)), (ch["n"], ch["M"])


def test_degridding_blocks_without_scheduled_items(P):
    """One dense tile among thousands of sparse ones: the plan has a single
    item of more than 64 visibilities, so all degridding blocks but one
    have no scheduled item and go straight to the small items after copying
    the kernel table into LDS (which they must wait for). Phi against the
    oracle, then repeated applications bitwise equal."""
    say("degridding blocks without scheduled items")
    n, m_sparse, m_dense = 512, 12000, 100
    rng = np.random.default_rng(77)
    x = W.gaussian_sky(n, W.n_sources_for(n), rng)
    cell = 2 * np.pi / (2 * n)                       # one grid cell in radians per pixel
    dense = 1.0 + rng.uniform(0.0, 4 * cell, (m_dense, 2))
    uv = np.concatenate([rng.uniform(-3.1, 3.1, (m_sparse, 2)), dense]).astype(np.float32)
    spec = ms.PhiSpec(n, 2 * n, 4, 2000)
    plan, perm = make_plan(P, n, uv, None, 4, 2000, "f32")
    xd = to_dev(x, torch.float32)
    y = plan.apply(xd)
    assert rel_l2(y.cpu().numpy(), ms.phi(x, uv.astype(np.float64), None, spec)[perm]) <= TOL["f32"]
    for _ in range(20):
        assert torch.equal(plan.apply(xd), y)
