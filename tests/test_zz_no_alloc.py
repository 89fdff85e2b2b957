"""The allocation-free l2-ball projection against the one with a caller
scratch: the same kernels in the same order, so the results must agree bit for
bit; two calls in a row, the second on a shorter input (the static scratch
keeps the first call's partial sums, which the second must not see)."""
import ctypes as C

import numpy as np
import pytest
import torch

from gpu_util import DEV, purimi

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return purimi()


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
def test_noalloc_projection_matches_scratch_form(P, dtype):
    rng = np.random.default_rng(77)
    lens = (1_000_003, 4099)           # second call shorter (several reduction blocks, ragged)
    scratch = torch.empty(P.pr_proj_l2ball_scratch_bytes(lens[0]), dtype=torch.uint8, device=DEV)
    for n in lens:
        x = torch.as_tensor(rng.standard_normal(n) + 1j * rng.standard_normal(n)).to(DEV, dtype)
        c = torch.as_tensor(rng.standard_normal(n) + 1j * rng.standard_normal(n)).to(DEV, dtype)
        dist = float(torch.linalg.vector_norm(x.to(torch.complex128) - c.to(torch.complex128)).item())
        for eps in (0.5 * dist, 2.0 * dist):          # projected, and left unchanged
            ref = torch.empty_like(x)
            got = torch.empty_like(x)
            d_ref = P.pr_proj_l2ball(x, c, ref, eps, scratch, want_dist=True)
            d_got = P.pr_proj_l2ball_noalloc(x, c, got, eps, want_dist=True)
            torch.cuda.synchronize()
            assert torch.equal(got, ref)
            assert d_got == d_ref
            assert d_got == pytest.approx(dist, rel=1e-12)


def test_noalloc_projection_argument_errors(P):
    L = P.lib()
    x = torch.zeros(16, dtype=torch.complex64, device=DEV)
    assert L.pr_proj_l2ball_noalloc(None, None, None, -1, 0, 1.0, None, None) == P.PR_EINVAL
    assert L.pr_proj_l2ball_noalloc(C.c_void_p(x.data_ptr()), None, C.c_void_p(x.data_ptr()), 16, 0, 1.0,
                                    None, None) == P.PR_EINVAL
    assert L.pr_proj_l2ball_noalloc(C.c_void_p(x.data_ptr()), C.c_void_p(x.data_ptr()),
                                    C.c_void_p(x.data_ptr()), 16, 5, 1.0, None, None) == P.PR_EINVAL
    assert L.pr_proj_l2ball_noalloc(C.c_void_p(x.data_ptr()), C.c_void_p(x.data_ptr()),
                                    C.c_void_p(x.data_ptr()), 16, 0, -1.0, None, None) == P.PR_EINVAL
