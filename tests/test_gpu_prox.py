"""GPU parity of the proximal operators against the FP64 oracle."""
import numpy as np
import pytest
import torch

from oracle import prox
from gpu_util import DEV, purimi, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return purimi()


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64, torch.complex64, torch.complex128])
@pytest.mark.parametrize("length", [1, 1000, 300001])
def test_soft_threshold(P, dtype, length):
    say(f"prox_l1 {dtype} {length}")
    rng = np.random.default_rng(length)
    x = rng.standard_normal(length)
    if dtype.is_complex:
        x = x + 1j * rng.standard_normal(length)
    lam = 0.8
    x[0] = lam if not dtype.is_complex else lam * (0.6 + 0.8j)   # the tie |x| = lambda gives 0
    xd = to_dev(x, dtype)
    out = torch.empty_like(xd)
    P.pr_prox_l1(xd, out, lam)
    ref = prox.soft_threshold(np.asarray(xd.cpu().numpy(), dtype=np.complex128 if dtype.is_complex else np.float64), lam)
    got = out.cpu().numpy()
    tol = 1e-6 if dtype in (torch.float32, torch.complex64) else 1e-15
    assert np.max(np.abs(got - ref)) <= tol * max(1.0, np.max(np.abs(ref)))
    assert got[0] == 0
    P.pr_prox_l1(xd, xd, lam)          # in place
    assert torch.equal(xd, out)


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
@pytest.mark.parametrize("eps_scale", [0.3, 1.0, 3.0])
def test_l2ball_projection(P, dtype, eps_scale):
    say(f"proj_l2ball {dtype} {eps_scale}")
    rng = np.random.default_rng(11)
    M = 123457
    z = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    x = z + 0.01 * (rng.standard_normal(M) + 1j * rng.standard_normal(M))
    xd, zd = to_dev(x, dtype), to_dev(z, dtype)
    x64 = xd.cpu().numpy().astype(np.complex128)
    z64 = zd.cpu().numpy().astype(np.complex128)
    dist = prox.l2_distance(x64, z64)
    eps = eps_scale * dist
    out = torch.empty_like(xd)
    scratch = torch.empty(P.pr_proj_l2ball_scratch_bytes(M), dtype=torch.uint8, device=DEV)
    d = P.pr_proj_l2ball(xd, zd, out, eps, scratch, want_dist=True)
    assert d == pytest.approx(dist, rel=1e-12)
    ref = prox.proj_l2ball(x64, z64, eps)
    tol = 1e-6 if dtype == torch.complex64 else 1e-14
    assert np.max(np.abs(out.cpu().numpy() - ref)) <= tol * np.max(np.abs(ref))
    if eps_scale == 1.0:
        pass  # boundary case: within rounding of the boundary either branch is the same point


def test_l2ball_is_bitwise_reproducible(P):
    say("proj_l2ball determinism")
    M = 1 << 20
    x = torch.randn(M, dtype=torch.complex64, device=DEV)
    z = torch.randn(M, dtype=torch.complex64, device=DEV)
    scratch = torch.empty(P.pr_proj_l2ball_scratch_bytes(M), dtype=torch.uint8, device=DEV)
    a, b = torch.empty_like(x), torch.empty_like(x)
    da = P.pr_proj_l2ball(x, z, a, 10.0, scratch, want_dist=True)
    db = P.pr_proj_l2ball(x, z, b, 10.0, scratch, want_dist=True)
    assert da == db and torch.equal(a, b)
