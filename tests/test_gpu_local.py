"""GPU parity of Algorithm 1 with local l2-ball constraints (one ball per
visibility section, Section "Local Fidelity Constraint ADMM") against the
oracle, on the 64^2 image / 8192-visibility workload.

Sections follow the paper's split: visibilities ordered by baseline length
and cut into equal-count sections; radii eps_j = sigma sqrt(M_j + 2 sqrt(M_j))
(the global rule applied per section). Also: random interleaved sections with
an empty one, a single section against the global-ball solver, the two
section-norm paths (8 sections, 9 with an empty one) against each other, bad ids.
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


def c0_data(J=None):
    w = W.CONFIGS["admm64"]
    rng = W.rng_for(w.index)
    x_true = W.make_sky(w, rng)
    uv = W.make_uv(w, rng)
    spec = ms.PhiSpec(w.n, w.K, w.J if J is None else J, w.D)
    uv64 = uv.astype(np.float64)
    y0 = ms.phi(x_true, uv64, None, spec)
    y, sigma, eps = W.add_noise(y0, W.unit_complex_noise(w.M, rng), w.snr_db)
    return w, uv, uv64, spec, y, sigma, eps


def length_sections(uv64, nsec):
    order = np.argsort(np.hypot(uv64[:, 0], uv64[:, 1]), kind="stable")
    sec = np.empty(len(order), dtype=np.int32)
    for j, part in enumerate(np.array_split(order, nsec)):
        sec[part] = j
    return sec


def radii(sec, nsec, sigma):
    m = np.bincount(sec, minlength=nsec).astype(np.float64)
    return sigma * np.sqrt(m + 2.0 * np.sqrt(m))


def oracle_local(w, uv64, spec, y, sec, eps_j, iters):
    nrm = ms.power_method(uv64, None, spec, iters=100)
    phi = lambda x: ms.phi(x, uv64, None, spec) / nrm
    phi_adj = lambda v: ms.phi_adjoint(v, uv64, None, spec) / nrm
    S = wv.Sara(w.n, w.levels)
    gamma = admm.default_gamma(y, phi_adj, S.adjoint)
    p = admm.AdmmParams(gamma=gamma, iters=iters)
    x, s, d, rep = admm.admm(y, phi, phi_adj, S.forward, S.adjoint, eps_j, p, np.zeros((w.n, w.n)), sections=sec)
    return x, rep, gamma, nrm


def gpu_local(P, w, uv, uv64, y, sec, nsec, eps_j, prec, prm, J=None):
    plan, perm = make_plan(P, w.n, uv if prec == "f32" else uv64, None, w.J if J is None else J, w.D, prec)
    psi = P.PsiPlan(w.n, w.levels, 0x1FF, P.PR_F32 if prec == "f32" else P.PR_F64, DEV)
    y_plan = to_dev(y[perm], torch.complex64 if prec == "f32" else torch.complex128)
    balls = P.Balls(plan, torch.as_tensor(sec[perm]).to(DEV), nsec)
    x, rep = P.admm_local_solve(plan, psi, balls, y_plan, prm, eps_j)
    return x, rep, balls, plan, psi, y_plan


# up to 8 sections the norms come from the degridding partials, above 8 from
# the section-sorted pieces: both paths in both precisions, and the largest
# section count of the first path
@pytest.mark.parametrize("prec,tol,iters,nsec", [("f64", 1e-10, 50, 4), ("f32", 1e-4, 50, 4), ("f64", 1e-10, 10, 8),
                                                 ("f64", 1e-10, 10, 16), ("f32", 1e-4, 20, 16)])
def test_local_balls_parity_admm64(P, prec, tol, iters, nsec):
    say(f"local balls admm64 {prec} iters={iters} nsec={nsec}")
    w, uv, uv64, spec, y, sigma, _ = c0_data()
    sec = length_sections(uv64, nsec)
    eps_j = radii(sec, nsec, sigma)
    x_ref, rep_ref, gamma, nrm = oracle_local(w, uv64, spec, y, sec, eps_j, iters)
    x, rep, balls, *_ = gpu_local(P, w, uv, uv64, y, sec, nsec, eps_j, prec,
                                  P.admm_params(0.0, gamma, iters=iters, op_norm=nrm))
    xg = x.cpu().numpy()
    assert rep.iters_done == iters and rep.nonfinite == 0
    assert rel_l2(xg, x_ref) <= tol
    assert np.all(xg >= 0)
    assert rep.resid_norm == pytest.approx(rep_ref.resid[-1], rel=max(tol, 1e-9) * 10)
    assert rep.l1_norm == pytest.approx(rep_ref.l1[-1], rel=max(tol, 1e-9) * 10)
    nj = balls.norms()
    assert nj.shape == (nsec,) and np.all(np.isfinite(nj)) and np.all(nj >= 0)


def test_interleaved_sections_with_an_empty_one(P):
    say("local balls random sections, one empty")
    w, uv, uv64, spec, y, sigma, _ = c0_data()
    rng = np.random.default_rng(31)
    nsec = 8
    sec = rng.integers(0, nsec - 1, w.M).astype(np.int32)     # section 7 stays empty
    eps_j = radii(sec, nsec, sigma)
    x_ref, _, gamma, nrm = oracle_local(w, uv64, spec, y, sec, eps_j, 10)
    x, rep, balls, *_ = gpu_local(P, w, uv, uv64, y, sec, nsec, eps_j, "f64",
                                  P.admm_params(0.0, gamma, iters=10, op_norm=nrm))
    assert rel_l2(x.cpu().numpy(), x_ref) <= 1e-10
    assert balls.norms()[7] == 0.0


def test_partials_path_matches_the_piece_path(P):
    # up to 8 sections the norms come from the degridding partials, above 8 from
    # the section-sorted pieces: 8 length sections, then the same ids with a 9th
    # (empty, eps 0 -> kappa 1) section, must give the same iterate
    say("local balls 8 sections (partials) vs 9 with an empty one (pieces)")
    w, uv, uv64, spec, y, sigma, _ = c0_data()
    sec = length_sections(uv64, 8)
    prm = P.admm_params(0.0, 0.05, iters=10, op_norm=1.0)
    e8 = radii(sec, 8, sigma)
    x8, _, b8, *_ = gpu_local(P, w, uv, uv64, y, sec, 8, e8, "f64", prm)
    x9, _, b9, *_ = gpu_local(P, w, uv, uv64, y, sec, 9, np.append(e8, 0.0), "f64", prm)
    assert rel_l2(x9.cpu().numpy(), x8.cpu().numpy()) <= 1e-12
    n8, n9 = b8.norms(), b9.norms()
    assert n9[8] == 0.0
    np.testing.assert_allclose(n9[:8], n8, rtol=1e-12)


def test_one_section_matches_the_global_ball_solver(P):
    say("local balls single section vs global")
    w, uv, uv64, spec, y, sigma, eps = c0_data()
    sec = np.zeros(w.M, dtype=np.int32)
    prm = P.admm_params(eps, 0.05, iters=20, op_norm=1.0)
    x, _, _, plan, psi, y_plan = gpu_local(P, w, uv, uv64, y, sec, 1, [eps], "f64", prm)
    xg, _ = P.admm_solve(plan, psi, y_plan, prm)
    assert rel_l2(x.cpu().numpy(), xg.cpu().numpy()) <= 1e-12


def test_bad_section_ids_are_refused_and_solves_repeat(P):
    say("local balls bad ids, determinism")
    w, uv, uv64, spec, y, sigma, _ = c0_data()
    plan, perm = make_plan(P, w.n, uv, None, w.J, w.D, "f32")
    bad = torch.zeros(w.M, dtype=torch.int32, device=DEV)
    bad[17] = 5
    with pytest.raises(P.PrError) as e:
        P.Balls(plan, bad, 5)
    assert e.value.code == P.PR_EINVAL
    sec = length_sections(uv64, 4)
    balls = P.Balls(plan, torch.as_tensor(sec[perm]).to(DEV), 4)
    psi = P.PsiPlan(w.n, w.levels, 0x1FF, P.PR_F32, DEV)
    y_plan = to_dev(y[perm], torch.complex64)
    prm = P.admm_params(0.0, 0.05, iters=6, op_norm=plan.norm(20))
    a, _ = P.admm_local_solve(plan, psi, balls, y_plan, prm, radii(sec, 4, sigma))
    b, _ = P.admm_local_solve(plan, psi, balls, y_plan, prm, radii(sec, 4, sigma))
    assert torch.equal(a, b)


def test_local_balls_with_the_j_lane_gridding(P):
    say("local balls admm64 J=6 f64")
    w, uv, uv64, spec, y, sigma, _ = c0_data(J=6)
    sec = length_sections(uv64, 4)
    eps_j = radii(sec, 4, sigma)
    x_ref, _, gamma, nrm = oracle_local(w, uv64, spec, y, sec, eps_j, 10)
    x, rep, *_ = gpu_local(P, w, uv, uv64, y, sec, 4, eps_j, "f64", P.admm_params(0.0, gamma, iters=10, op_norm=nrm),
                           J=6)
    assert rep.nonfinite == 0
    assert rel_l2(x.cpu().numpy(), x_ref) <= 1e-10
