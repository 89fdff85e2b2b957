"""Serving loop on the GPU: continuous batching of imaging solves.

A job's result must not depend on what else is running: the same request
served alone, in a mix admitted while others run, under an arena that admits
only two jobs at a time, and through pr_admm_solve, gives the same image bit
for bit. One FP64 job of the 64^2 / 8192-visibility workload is checked
against the FP64 oracle run of Algorithm 1.
"""
import time

import numpy as np
import pytest
import torch

import workloads as W
from oracle import admm, measurement as ms, wavelets as wv
from gpu_util import DEV, make_plan, problem, purimi, rel_l2, say, to_dev

pytestmark = pytest.mark.gpu

# (n, M, seed)
JOBS = [(64, 8192, 21), (32, 3000, 22), (128, 40000, 23), (64, 20000, 24), (32, 500, 25)]


@pytest.fixture(scope="module")
def P():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return purimi()


def request(P, n, M, seed, prec="f32", iters=6, norm_iters=30):
    rdt = torch.float32 if prec == "f32" else torch.float64
    cdt = torch.complex64 if prec == "f32" else torch.complex128
    x, uv, _, spec = problem(n, M, seed=seed, prec=prec)
    y0 = ms.phi(x, uv.astype(np.float64), None, spec)
    rng = np.random.default_rng(200 + seed)
    y, _, eps = W.add_noise(y0, W.unit_complex_noise(M, rng), 30.0)
    uv_d, y_d = to_dev(uv, rdt), to_dev(y, cdt)
    prm = P.admm_params(eps, 0.0, iters=iters, gamma_factor=1e-3, norm_iters=norm_iters)
    desc = P.job_desc(n, uv_d, y_d, prm, levels=3)
    return dict(n=n, M=M, uv=uv, y=y, uv_d=uv_d, y_d=y_d, prm=prm, desc=desc, rdt=rdt)


def drain(srv, jids, limit_s=60.0, on_tick=None, max_running=None):
    t0 = time.time()
    ticks = 0
    while True:
        q, r, f = srv.tick()
        ticks += 1
        if max_running is not None:
            assert r <= max_running
        if on_tick:
            on_tick(ticks)
        if all(srv.state(j) == 2 for j in jids):
            return ticks
        assert time.time() - t0 < limit_s, "serving loop did not finish"


def test_served_alone_equals_mix_and_solver(P):
    say("serve alone vs mix")
    reqs = [request(P, *j) for j in JOBS]
    a = reqs[0]
    srv = P.Server(1 << 30, max_active=8, nstreams=4)
    ja = srv.submit(a["desc"], keep=(a["uv_d"], a["y_d"]))
    drain(srv, [ja])
    x_alone, rep_alone = srv.fetch(ja, a["n"])
    assert rep_alone.iters_done == 6 and rep_alone.nonfinite == 0

    srv2 = P.Server(1 << 30, max_active=8, nstreams=4)
    ids = {}
    for i in (1, 2):
        ids[i] = srv2.submit(reqs[i]["desc"], keep=(reqs[i]["uv_d"], reqs[i]["y_d"]))

    def arrivals(tick):
        if tick == 3:
            ids[0] = srv2.submit(a["desc"], keep=(a["uv_d"], a["y_d"]))
        if tick == 5:
            for i in (3, 4):
                ids[i] = srv2.submit(reqs[i]["desc"], keep=(reqs[i]["uv_d"], reqs[i]["y_d"]))

    for _ in range(6):
        srv2.tick()
        arrivals(_ + 1)
    drain(srv2, list(ids.values()))
    x_mix, rep_mix = srv2.fetch(ids[0], a["n"])
    assert torch.equal(x_mix, x_alone)
    assert rep_mix.resid_norm == rep_alone.resid_norm and rep_mix.op_norm == rep_alone.op_norm

    # the same request through the solver entry point
    plan, perm = make_plan(P, a["n"], a["uv"], None, 4, 2000, "f32")
    psi = P.PsiPlan(a["n"], 3, 0x1FF, P.PR_F32, DEV)
    y_plan = to_dev(a["y"][perm], torch.complex64)
    x_solve, rep_solve = P.admm_solve(plan, psi, y_plan, a["prm"])
    assert torch.equal(x_solve, x_alone)
    assert rep_solve.l1_norm == rep_alone.l1_norm

    # the others against their own lone solves
    for i in (1, 2, 3, 4):
        r = reqs[i]
        x_i, _ = srv2.fetch(ids[i], r["n"])
        plan, perm = make_plan(P, r["n"], r["uv"], None, 4, 2000, "f32")
        psi = P.PsiPlan(r["n"], 3, 0x1FF, P.PR_F32, DEV)
        x_s, _ = P.admm_solve(plan, psi, to_dev(r["y"][perm], torch.complex64), r["prm"])
        assert torch.equal(x_i, x_s), f"job n={r['n']} M={r['M']}"


def test_admission_by_footprint(P):
    say("serve admission by footprint")
    reqs = [request(P, 64, 8192, 30 + i, iters=4) for i in range(5)]
    need = max(P.pr_server_job_bytes(r["desc"]) for r in reqs)
    srv = P.Server(2 * need + 4096, max_active=16, nstreams=4)
    ids = [srv.submit(r["desc"], keep=(r["uv_d"], r["y_d"])) for r in reqs]
    done_first = {}
    t0 = time.time()
    while True:
        q, r, f = srv.tick()
        assert r <= 2
        # fetch finished jobs so that their memory is returned
        for j in ids:
            if j not in done_first and srv.state(j) == 2:
                done_first[j] = srv.fetch(j, 64)[0]
        if len(done_first) == len(ids):
            break
        assert time.time() - t0 < 60
    for r, j in zip(reqs, ids):
        plan, perm = make_plan(P, 64, r["uv"], None, 4, 2000, "f32")
        psi = P.PsiPlan(64, 3, 0x1FF, P.PR_F32, DEV)
        x_s, _ = P.admm_solve(plan, psi, to_dev(r["y"][perm], torch.complex64), r["prm"])
        assert torch.equal(done_first[j], x_s)
    free, largest = P.pr_server_free_bytes(srv.handle)
    assert free == largest >= 2 * need


def test_oversize_request_is_refused(P):
    say("serve oversize")
    r = request(P, 64, 8192, 40)
    need = P.pr_server_job_bytes(r["desc"])
    srv = P.Server(need // 2, max_active=4, nstreams=1)
    with pytest.raises(P.PrError) as e:
        srv.submit(r["desc"])
    assert e.value.code == P.PR_EWORKSPACE


def test_served_fp64_job_matches_oracle(P):
    say("serve admm64 fp64 vs oracle")
    w = W.CONFIGS["admm64"]
    rng = W.rng_for(w.index)
    x_true = W.make_sky(w, rng)
    uv = W.make_uv(w, rng)
    spec = ms.PhiSpec(w.n, w.K, w.J, w.D)
    uv64 = uv.astype(np.float64)
    y0 = ms.phi(x_true, uv64, None, spec)
    y, sigma, eps = W.add_noise(y0, W.unit_complex_noise(w.M, rng), w.snr_db)
    nrm = ms.power_method(uv64, None, spec, iters=100)
    phi = lambda x: ms.phi(x, uv64, None, spec) / nrm
    phi_adj = lambda v: ms.phi_adjoint(v, uv64, None, spec) / nrm
    S = wv.Sara(w.n, w.levels)
    gamma = admm.default_gamma(y, phi_adj, S.adjoint)
    x_ref, _, _, _ = admm.admm(y, phi, phi_adj, S.forward, S.adjoint, eps, admm.AdmmParams(gamma=gamma, iters=w.iters),
                               np.zeros((w.n, w.n)))
    uv_d, y_d = to_dev(uv64, torch.float64), to_dev(y, torch.complex128)
    prm = P.admm_params(eps, 0.0, iters=w.iters, gamma_factor=1e-3, norm_iters=100)
    srv = P.Server(1 << 28, max_active=2, nstreams=2)
    j = srv.submit(P.job_desc(w.n, uv_d, y_d, prm, levels=w.levels), keep=(uv_d, y_d))
    drain(srv, [j])
    x, rep = srv.fetch(j, w.n, dtype=torch.float64)
    assert rep.op_norm == pytest.approx(nrm, rel=1e-12)
    assert rel_l2(x.cpu().numpy(), x_ref) <= 1e-10


def test_cancel_queued_and_running_jobs(P):
    """A queued job leaves the queue, a running one is stopped and its arena
    memory released; the other jobs still give their solo results bitwise."""
    say("serve cancel")
    reqs = [request(P, *j) for j in (JOBS[2], JOBS[0], JOBS[1])]    # largest first
    # solo results
    solo = []
    for r in reqs:
        s1 = P.Server(1 << 30, max_active=4, nstreams=2)
        j = s1.submit(r["desc"], keep=(r["uv_d"], r["y_d"]))
        drain(s1, [j])
        solo.append(s1.fetch(j, r["n"])[0])
    need = [P.pr_server_job_bytes(r["desc"]) for r in reqs]
    # the first (largest) job fits; what it leaves is less than the smallest job
    srv = P.Server(need[0] + (min(need) // 2 & ~255), max_active=4, nstreams=2)
    total, _ = P.pr_server_free_bytes(srv.handle)
    ids = [srv.submit(r["desc"], keep=(r["uv_d"], r["y_d"])) for r in reqs]
    srv.tick()
    assert [srv.state(j) for j in ids] == [1, 0, 0]
    srv.cancel(ids[1])                                  # queued
    with pytest.raises(P.PrError):
        srv.state(ids[1])
    srv.cancel(ids[0])                                  # running
    with pytest.raises(P.PrError):
        srv.state(ids[0])
    assert P.pr_server_free_bytes(srv.handle)[0] == total
    drain(srv, [ids[2]])
    x, rep = srv.fetch(ids[2], reqs[2]["n"])
    assert torch.equal(x, solo[2]) and rep.nonfinite == 0
    with pytest.raises(P.PrError):
        srv.cancel(ids[2])                              # fetched: unknown


@pytest.mark.parametrize("bad", [float("nan"), float("inf")])
def test_nonfinite_data_is_flagged(P, bad):
    """A NaN or an infinity in the observed visibilities reaches the FP64
    diagnostics: the report says so instead of returning a silent image."""
    say(f"nonfinite flag {bad}")
    x, uv, _, spec = problem(32, 3000, seed=7, prec="f32")
    plan, perm = make_plan(P, 32, uv, None, 4, 2000, "f32")
    psi = P.PsiPlan(32, 3, 0x1FF, P.PR_F32, DEV)
    y = plan.apply(to_dev(x, torch.float32))
    prm = P.admm_params(0.1 * float(torch.linalg.vector_norm(y).item()), 1e-3, iters=3, op_norm=1.0)
    _, rep = P.admm_solve(plan, psi, y, prm)
    assert rep.nonfinite == 0
    y_bad = y.clone()
    y_bad[1234] = complex(bad, 0.0)
    _, rep = P.admm_solve(plan, psi, y_bad, prm)
    assert rep.nonfinite != 0


def test_data_may_change_once_the_job_runs(P):
    """uv, w and y must stay valid only until the job is running: the server
    has read them by then. Overwriting y right after admission leaves the
    served image unchanged."""
    say("serve: y overwritten once running")
    a = request(P, *JOBS[0])
    srv = P.Server(1 << 30, max_active=8, nstreams=4)
    ja = srv.submit(a["desc"], keep=(a["uv_d"], a["y_d"]))
    drain(srv, [ja])
    x_ref, _ = srv.fetch(ja, a["n"])
    y_tmp = a["y_d"].clone()
    uv_tmp = a["uv_d"].clone()
    desc = P.job_desc(a["n"], uv_tmp, y_tmp, a["prm"], levels=3)
    jb = srv.submit(desc, keep=(uv_tmp, y_tmp))
    while srv.state(jb) < 1:
        srv.tick()
    y_tmp.fill_(float("nan"))
    uv_tmp.fill_(float("nan"))
    drain(srv, [jb])
    x_b, rep_b = srv.fetch(jb, a["n"])
    assert rep_b.nonfinite == 0
    assert torch.equal(x_b, x_ref)
