"""Checkpoint and resume of Algorithm 1 at the boundary, and the power
method's stopping tolerance.

solve(k) then export, import into a fresh workspace and resume(m) must give
bitwise the iterate of an uninterrupted solve(k + m): the state of the
iteration (x, the multiplier s, the DualFB dual d, 1 / ||Phi||, gamma and the
count) is all that carries over between outer iterations of Algorithm 1.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import measurement as ms
from gpu_util import DEV, make_plan, purimi, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return purimi()


def c0(P, prec):
    w = W.CONFIGS["admm64"]
    rng = W.rng_for(w.index)
    x_true = W.make_sky(w, rng)
    uv = W.make_uv(w, rng)
    uv64 = uv.astype(np.float64)
    spec = ms.PhiSpec(w.n, w.K, w.J, w.D)
    y0 = ms.phi(x_true, uv64, None, spec)
    y, _, eps = W.add_noise(y0, W.unit_complex_noise(w.M, rng), w.snr_db)
    plan, perm = make_plan(P, w.n, uv if prec == "f32" else uv64, None, w.J, w.D, prec)
    pprec = P.PR_F32 if prec == "f32" else P.PR_F64
    psi = P.PsiPlan(w.n, w.levels, 0x1FF, pprec, DEV)
    y_plan = to_dev(y[perm], torch.complex64 if prec == "f32" else torch.complex128)
    return w, plan, psi, y_plan, eps


@pytest.mark.parametrize("prec,where,gamma", [("f32", "device", 0.0), ("f64", "host", 0.0), ("f32", "host", 0.02)])
def test_resume_after_export_import_is_bitwise(P, prec, where, gamma):
    say(f"checkpoint {prec} state on {where} gamma={gamma}")
    w, plan, psi, y, eps = c0(P, prec)
    k, m = 4, 3
    # device-side norm and gamma (gamma <= 0) or a fixed gamma
    prm = lambda it: P.admm_params(eps, gamma, iters=it, gamma_factor=1e-3, norm_iters=50)
    x_full, rep_full = P.admm_solve(plan, psi, y, prm(k + m))

    nbytes = P.pr_admm_workspace_size(plan.handle, psi.handle)
    ws_a = P._workspace(nbytes, DEV)
    x = torch.zeros((w.n, w.n), dtype=plan.rdtype, device=DEV)
    rep_a = P.pr_admm_solve(plan.handle, psi.handle, y, prm(k), x, ws_a)
    assert rep_a.iters_done == k
    sb = P.pr_admm_state_bytes(plan.handle, psi.handle)
    dev = torch.device(DEV) if where == "device" else torch.device("cpu")
    state = torch.empty(sb, dtype=torch.uint8, device=dev)
    P.pr_admm_state_export(plan.handle, psi.handle, ws_a, x, state)
    del ws_a
    # a fresh workspace and image, garbage first
    ws_b = torch.full((max(nbytes, 256),), 0x7F, dtype=torch.uint8, device=DEV)
    x_b = torch.full((w.n, w.n), 3.0, dtype=plan.rdtype, device=DEV)
    P.pr_admm_state_import(plan.handle, psi.handle, state, ws_b, x_b)
    rep_b = P.pr_admm_resume(plan.handle, psi.handle, y, prm(m), x_b, ws_b)
    assert rep_b.iters_done == k + m and rep_full.iters_done == k + m
    assert torch.equal(x_b, x_full)
    assert rep_b.resid_norm == rep_full.resid_norm and rep_b.l1_norm == rep_full.l1_norm
    assert rep_b.op_norm == rep_full.op_norm
    # resuming on the same workspace continues the count as well
    rep_c = P.pr_admm_resume(plan.handle, psi.handle, y, prm(0), x_b, ws_b)
    assert rep_c.iters_done == k + m


def test_import_refuses_other_plans(P):
    say("checkpoint refused for other plans")
    w, plan, psi, y, eps = c0(P, "f32")
    ws = P._workspace(P.pr_admm_workspace_size(plan.handle, psi.handle), DEV)
    x = torch.zeros((w.n, w.n), dtype=torch.float32, device=DEV)
    P.pr_admm_solve(plan.handle, psi.handle, y, P.admm_params(eps, 0.02, iters=1, op_norm=1.0), x, ws)
    state = torch.empty(P.pr_admm_state_bytes(plan.handle, psi.handle), dtype=torch.uint8)
    P.pr_admm_state_export(plan.handle, psi.handle, ws, x, state)
    psi2 = P.PsiPlan(w.n, 2, 0x1FF, P.PR_F32, DEV)
    ws2 = P._workspace(P.pr_admm_workspace_size(plan.handle, psi2.handle), DEV)
    with pytest.raises(P.PrError) as e:
        P.pr_admm_state_import(plan.handle, psi2.handle, state, ws2, x)
    assert e.value.code == P.PR_EINVAL
    junk = torch.zeros_like(state)
    with pytest.raises(P.PrError) as e:
        P.pr_admm_state_import(plan.handle, psi.handle, junk, ws, x)
    assert e.value.code == P.PR_EINVAL


def test_power_method_tolerance(P):
    say("power method rtol")
    w = W.CONFIGS["admm64"]
    rng = W.rng_for(w.index)
    W.make_sky(w, rng)
    uv64 = W.make_uv(w, rng).astype(np.float64)
    spec = ms.PhiSpec(w.n, w.K, w.J, w.D)
    ref = ms.power_method(uv64, None, spec, iters=300)
    plan, _ = make_plan(P, w.n, uv64, None, w.J, w.D, "f64")
    fixed = plan.norm(300)
    tol = plan.norm(300, rtol=1e-12)
    assert fixed == pytest.approx(ref, rel=1e-12)
    assert tol == pytest.approx(ref, rel=1e-9)
    # a loose tolerance stops at the same step as the oracle's rule (the change
    # of ||A x|| from one step to the next); the estimate is a lower bound
    loose = plan.norm(300, rtol=1e-3)
    assert loose == pytest.approx(ms.power_method(uv64, None, spec, iters=300, rtol=1e-3), rel=1e-9)
    assert loose < fixed * (1 + 1e-12)
