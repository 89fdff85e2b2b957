"""Batched solves on the GPU: channels of different n and M stepped together.

Every member has its own plans and workspace and runs the kernels of a solve
alone, so the batched results must be bitwise equal to per-channel calls, for
the operators (batched Phi on stacked channels = per-channel Phi) and for the
solver, with and without graph replay.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import measurement as ms
from gpu_util import DEV, make_plan, problem, purimi, say, to_dev

pytestmark = pytest.mark.gpu

# (n, M, seed): uneven image sizes and visibility counts, one ragged tiny channel
CHANNELS = [(32, 3000, 1), (64, 20000, 2), (128, 60000, 3), (64, 700, 4), (32, 12000, 5)]


@pytest.fixture(scope="module")
def P():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return purimi()


def make_channels(P, prec):
    rdt = torch.float32 if prec == "f32" else torch.float64
    cdt = torch.complex64 if prec == "f32" else torch.complex128
    pprec = P.PR_F32 if prec == "f32" else P.PR_F64
    out = []
    for n, M, seed in CHANNELS:
        x, uv, _, spec = problem(n, M, seed=seed, prec=prec)
        y0 = ms.phi(x, uv.astype(np.float64), None, spec)
        rng = np.random.default_rng(100 + seed)
        y, _, eps = W.add_noise(y0, W.unit_complex_noise(M, rng), 30.0)
        plan, perm = make_plan(P, n, uv, None, 4, 2000, prec)
        psi = P.PsiPlan(n, 3, 0x1FF, pprec, DEV)
        out.append(dict(n=n, M=M, x=to_dev(x, rdt), plan=plan, psi=psi, y=to_dev(y[perm], cdt), eps=eps))
    return out


def params(P, ch, iters):
    return P.admm_params(ch["eps"], 0.0, iters=iters, gamma_factor=1e-3, norm_iters=30)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_batched_phi_equals_per_channel(P, prec):
    say(f"batch phi {prec}")
    chs = make_channels(P, prec)
    b = P.Batch(max_members=8, nstreams=3)
    for ch in chs:
        b.add(ch["plan"], ch["psi"], ch["y"], params(P, ch, 1))
    ys = [torch.empty(ch["M"], dtype=ch["y"].dtype, device=DEV) for ch in chs]
    P.pr_batch_phi_apply(b.handle, [ch["x"] for ch in chs], ys)
    xs = [torch.empty_like(ch["x"]) for ch in chs]
    P.pr_batch_phi_adjoint(b.handle, ys, xs)
    torch.cuda.synchronize()
    for ch, yb, xb in zip(chs, ys, xs):
        assert torch.equal(yb, ch["plan"].apply(ch["x"]))
        assert torch.equal(xb, ch["plan"].adjoint(yb))


@pytest.mark.parametrize("use_graph", [True, False])
def test_batched_admm_equals_alone(P, use_graph):
    say(f"batch admm graph={use_graph}")
    chs = make_channels(P, "f32")
    b = P.Batch(max_members=8, nstreams=4)
    slots = [b.add(ch["plan"], ch["psi"], ch["y"], params(P, ch, 1)) for ch in chs]
    for k in range(1, 4):
        b.step(1, use_graph=use_graph)
        torch.cuda.synchronize()
        # eager work of the program itself between graph replays
        junk = torch.randn(1 << 20, device=DEV)
        junk.mul_(2.0).sum().item()
        for ch, slot in zip(chs, slots):
            alone, rep = P.admm_solve(ch["plan"], ch["psi"], ch["y"], params(P, ch, k))
            assert torch.equal(b.x(slot), alone), f"channel n={ch['n']} M={ch['M']} step {k}"
    rep_b = b.report(slots[2])
    _, rep_a = P.admm_solve(chs[2]["plan"], chs[2]["psi"], chs[2]["y"], params(P, chs[2], 3))
    assert rep_b.iters_done == 3
    assert rep_b.resid_norm == rep_a.resid_norm and rep_b.l1_norm == rep_a.l1_norm
    assert rep_b.op_norm == rep_a.op_norm


def test_membership_change_recaptures(P):
    say("batch membership change")
    chs = make_channels(P, "f32")
    b = P.Batch(max_members=8, nstreams=2)
    slots = [b.add(ch["plan"], ch["psi"], ch["y"], params(P, ch, 1)) for ch in chs]
    b.step(2, use_graph=True)
    b.remove(slots[1])
    assert P.pr_batch_members(b.handle) == len(chs) - 1
    b.step(1, use_graph=True)
    torch.cuda.synchronize()
    for i, (ch, slot) in enumerate(zip(chs, slots)):
        if i == 1:
            continue
        alone, _ = P.admm_solve(ch["plan"], ch["psi"], ch["y"], params(P, ch, 3))
        assert torch.equal(b.x(slot), alone)


def test_batch_rejects_shared_plans(P):
    say("batch shared plan")
    chs = make_channels(P, "f32")[:1]
    b = P.Batch(max_members=4, nstreams=1)
    b.add(chs[0]["plan"], chs[0]["psi"], chs[0]["y"], params(P, chs[0], 1))
    with pytest.raises(P.PrError):
        b.add(chs[0]["plan"], chs[0]["psi"], chs[0]["y"], params(P, chs[0], 1))


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_fused_phi_equals_per_channel(P, prec):
    """pr_batch_fuse: one launch per stage over all members, bitwise equal to
    each member's own Phi and Phi^dagger (also after new vectors are passed)."""
    say(f"fused batch phi {prec}")
    chs = make_channels(P, prec)
    b = P.Batch(max_members=8, nstreams=3)
    for ch in chs:
        b.add(ch["plan"], ch["psi"], ch["y"], params(P, ch, 1))
    b.fuse()
    for rnd in range(3):
        xin = [ch["x"] * (1.0 + 0.5 * rnd) for ch in chs]          # new tensors each round
        ys = [torch.empty(ch["M"], dtype=ch["y"].dtype, device=DEV) for ch in chs]
        P.pr_batch_phi_apply(b.handle, xin, ys)
        xs = [torch.empty_like(ch["x"]) for ch in chs]
        P.pr_batch_phi_adjoint(b.handle, ys, xs)
        torch.cuda.synchronize()
        for ch, xi, yb, xb in zip(chs, xin, ys, xs):
            assert torch.equal(yb, ch["plan"].apply(xi)), (rnd, ch["n"], ch["M"])
            assert torch.equal(xb, ch["plan"].adjoint(yb)), (rnd, ch["n"], ch["M"])


def test_fused_many_channels_and_membership_change(P):
    """Twenty channels of four image sizes (several FFT size classes, many work
    items per block); removing a member drops the fused form (the calls launch
    per member), fusing again restores it."""
    say("fused batch, 20 channels")
    rng = np.random.default_rng(9)
    chans = [(int(rng.choice([32, 64, 128, 256])), int(rng.integers(500, 80000))) for _ in range(20)]
    b = P.Batch(max_members=32, nstreams=4)
    chs = []
    for i, (n, M) in enumerate(chans):
        x, uv, _, spec = problem(n, M, seed=300 + i, prec="f32")
        plan, perm = make_plan(P, n, uv, None, 4, 2000, "f32")
        psi = P.PsiPlan(n, 3, 0x1FF, P.PR_F32, DEV)
        y = torch.zeros(M, dtype=torch.complex64, device=DEV)
        chs.append(dict(n=n, M=M, x=to_dev(x, torch.float32), plan=plan, psi=psi, slot=None))
        chs[-1]["slot"] = b.add(plan, psi, y, P.admm_params(1.0, 1e-3, iters=1, op_norm=1.0))
    b.fuse()

    def check(active):
        xs_in = [None] * 32
        ys = [None] * 32
        xs = [None] * 32
        for ch in active:
            xs_in[ch["slot"]] = ch["x"]
            ys[ch["slot"]] = torch.empty(ch["M"], dtype=torch.complex64, device=DEV)
            xs[ch["slot"]] = torch.empty_like(ch["x"])
        P.pr_batch_phi_apply(b.handle, xs_in, ys)
        P.pr_batch_phi_adjoint(b.handle, ys, xs)
        torch.cuda.synchronize()
        for ch in active:
            assert torch.equal(ys[ch["slot"]], ch["plan"].apply(ch["x"])), (ch["n"], ch["M"])
            assert torch.equal(xs[ch["slot"]], ch["plan"].adjoint(ys[ch["slot"]])), (ch["n"], ch["M"])

    check(chs)
    b.remove(chs[3]["slot"])
    rest = chs[:3] + chs[4:]
    check(rest)            # per-member launches
    b.fuse()
    check(rest)            # fused again


def test_fuse_rejects_mixed_kernels_and_small_workspace(P):
    say("fused batch errors")
    x, uv, _, spec = problem(32, 2000, seed=1, prec="f32")
    mk = lambda **kw: P.PhiPlan(32, to_dev(uv, torch.float32), None, **kw)
    psi = lambda: P.PsiPlan(32, 3, 0x1FF, P.PR_F32, DEV)
    y = torch.zeros(2000, dtype=torch.complex64, device=DEV)
    prm = P.admm_params(1.0, 1e-3, iters=1, op_norm=1.0)
    for other in (dict(tile=8), dict(J=6), dict(interp=1)):
        b = P.Batch(max_members=4, nstreams=1)
        b.add(mk(), psi(), y, prm)
        b.add(mk(**other), psi(), y, prm)
        with pytest.raises(P.PrError) as e:
            P.pr_batch_fuse_bytes(b.handle)
        assert e.value.code == P.PR_EUNSUPPORTED, other
    b = P.Batch(max_members=4, nstreams=1)
    b.add(mk(), psi(), y, prm)
    need = P.pr_batch_fuse_bytes(b.handle)
    small = torch.empty(max(256, need - 256), dtype=torch.uint8, device=DEV)
    with pytest.raises(P.PrError) as e:
        P.pr_batch_fuse(b.handle, small)
    assert e.value.code == P.PR_EWORKSPACE
