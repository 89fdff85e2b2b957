"""Host read-backs refuse a stream under graph capture (a captured copy to
host memory would replay into whatever that address holds later), and the
refusal leaves the stream and the library usable."""
import numpy as np
import pytest
import torch

import workloads as W
from gpu_util import DEV, make_plan, problem, purimi, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return purimi()


def test_host_readbacks_refuse_capture(P):
    say("host read-backs under capture")
    x, uv, _, spec = problem(32, 3000, seed=5, prec="f32")
    plan, _ = make_plan(P, 32, uv, None, 4, 2000, "f32")
    v = torch.randn(1000, dtype=torch.complex64, device=DEV)
    c = torch.zeros_like(v)
    out = torch.empty_like(v)
    scratch = torch.empty(P.pr_proj_l2ball_scratch_bytes(1000), dtype=torch.uint8, device=DEV)
    junk = torch.zeros(16, device=DEV)
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    codes = []
    with torch.cuda.stream(s):
        g.capture_begin()
        try:
            junk.add_(1.0)                       # the graph is not empty
            for call in (lambda: plan.norm(3),
                         lambda: P.pr_proj_l2ball(v, c, out, 1.0, scratch, want_dist=True),
                         lambda: P.pr_proj_l2ball_noalloc(v, c, out, 1.0, want_dist=True)):
                try:
                    call()
                    codes.append(0)
                except P.PrError as e:
                    codes.append(e.code)
        finally:
            g.capture_end()
    assert codes == [P.PR_EINVAL] * 3
    g.replay()
    torch.cuda.synchronize()
    assert float(junk[0].item()) == 1.0          # recorded by the capture, run by the replay
    # the same calls work outside the capture
    assert plan.norm(3) > 0
    d = P.pr_proj_l2ball(v, c, out, 1.0, scratch, want_dist=True)
    assert d == pytest.approx(float(torch.linalg.vector_norm(v.to(torch.complex128)).item()), rel=1e-12)
