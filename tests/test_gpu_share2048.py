"""The 2048^2 / 5e8-visibility workload at full size, in the launch
configuration the benchmark times (default tile, FP32 storage).

The oracle cannot run Phi^dagger over 5e8 visibilities, so: Phi is checked
on a sample of visibilities the oracle computes one by one (its full 4096^2
FFT, then the sampled degridding); Phi^dagger through the adjoint identity
with FP64 inner products; two ADMM iterations through invariants (finite
FP64 diagnostics, a non-negative iterate, bitwise repeatability).
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import measurement as ms
from gpu_util import DEV, purimi, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return purimi()


@pytest.fixture(scope="module")
def big(P):
    wl = W.CONFIGS["share2048"]
    say("big full size: generating 5e8 baselines on the device")
    gen = W.torch_generator(wl.index, DEV)
    uv = W.uv_ring_core_torch(wl.M, gen, DEV)
    x = W.make_sky(wl, W.rng_for(wl.index))
    say("big full size: plan")
    plan = P.PhiPlan(wl.n, uv, None, J=wl.J, D=wl.D)
    return dict(wl=wl, uv=uv, x=x, plan=plan, gen=gen)


def inner_f64(a, b, chunk=1 << 26):
    """Re sum conj(a) b in FP64, chunked (complex inputs)."""
    acc = 0.0
    for i in range(0, a.numel(), chunk):
        acc += float((a[i:i + chunk].to(torch.complex128).conj() * b[i:i + chunk].to(torch.complex128)).sum().real)
    return acc


def test_share2048_phi_sampled_vs_oracle(P, big):
    wl, plan = big["wl"], big["plan"]
    say("big phi")
    y = plan.apply(torch.as_tensor(big["x"], dtype=torch.float32, device=DEV))
    perm = plan.perm()
    # 20000 visibilities spread over the plan order (every tile region), plus
    # the ends; integer arithmetic (a float32 linspace rounds M - 1 up to M)
    pos = torch.cat([torch.arange(20000, dtype=torch.int64) * (wl.M - 1) // 19999,
                     torch.tensor([0, 1, wl.M - 2, wl.M - 1], dtype=torch.int64)])
    assert int(pos.min()) >= 0 and int(pos.max()) < wl.M
    pos = pos.to(DEV)
    idx = perm[pos]
    uv_s = big["uv"][idx].double().cpu().numpy()
    spec = ms.PhiSpec(wl.n, wl.K, wl.J, wl.D)
    y_ref = ms.phi(big["x"], uv_s, None, spec)
    y_gpu = y[pos].cpu().numpy().astype(np.complex128)
    err = np.linalg.norm(y_gpu - y_ref) / np.linalg.norm(y_ref)
    say(f"big phi sampled rel err {err:.3e}")
    assert err <= 1e-5


def test_share2048_adjoint_identity(P, big):
    wl, plan = big["wl"], big["plan"]
    say("big adjoint identity")
    g = torch.Generator(device=DEV)
    g.manual_seed(77)
    x = torch.rand((wl.n, wl.n), generator=g, device=DEV)
    v = torch.complex(torch.randn(wl.M, generator=g, device=DEV), torch.randn(wl.M, generator=g, device=DEV))
    ax = plan.apply(x)
    av = plan.adjoint(v)
    lhs = inner_f64(ax, v)
    rhs = float((x.double() * av.double()).sum())
    say(f"big <Phi x, v> = {lhs:.9e}, <x, Phi^H v> = {rhs:.9e}")
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


def test_share2048_admm_invariants(P, big):
    wl, plan = big["wl"], big["plan"]
    say("big admm 2 iterations")
    psi = P.PsiPlan(wl.n, wl.levels, 0x1FF, P.PR_F32, DEV)
    y = plan.apply(torch.as_tensor(big["x"], dtype=torch.float32, device=DEV))
    y, _, eps = W.add_noise_torch(y, W.unit_complex_noise_torch(wl.M, big["gen"], DEV), wl.snr_db)
    prm = P.admm_params(eps, 0.0, iters=2, gamma_factor=1e-3, norm_iters=10)
    a, ra = P.admm_solve(plan, psi, y, prm)
    b, rb = P.admm_solve(plan, psi, y, prm)
    assert ra.nonfinite == 0 and np.isfinite(ra.resid_norm) and ra.op_norm > 0
    assert bool((a >= 0).all())
    assert torch.equal(a, b) and ra.resid_norm == rb.resid_norm
