"""GPU parity of the measurement operator against the FP64 oracle.

Every array the oracle sees is the GPU's input widened to FP64; visibility
vectors are compared in plan order (y_plan[k] = y_user[perm[k]]).
"""
import numpy as np
import pytest
import torch

from oracle import measurement as ms
from gpu_util import DEV, cell_keys, make_plan, problem, purimi, rel_l2, say, to_dev

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "f64": 1e-12}


@pytest.fixture(scope="module")
def P():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return purimi()


def _rdt(prec):
    return torch.float32 if prec == "f32" else torch.float64


def _cdt(prec):
    return torch.complex64 if prec == "f32" else torch.complex128


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_phi_parity_at_the_largest_image(P, prec):
    """n = 4096 (K = 8192), the largest image a plan accepts: every FFT pass
    holds one line of 8192 points per block (2048 radix-4 butterflies per
    stage), in both precisions."""
    n, M, J = 4096, 3000, 4
    say(f"phi parity largest image prec={prec}")
    x, uv, w, spec = problem(n, M, J, 2000, seed=4096, prec=prec, weights=False)
    plan, perm = make_plan(P, n, uv, w, J, 2000, prec, 0)
    y_gpu = plan.apply(to_dev(x, _rdt(prec))).cpu().numpy()
    uv64 = uv.astype(np.float64)
    y_ref = ms.phi(x, uv64, None, spec)[perm]
    assert rel_l2(y_gpu, y_ref) <= TOL[prec]
    rng = np.random.default_rng(7)
    yy = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    x_gpu = plan.adjoint(to_dev(yy[perm], _cdt(prec))).cpu().numpy()
    x_ref = ms.phi_adjoint(yy, uv64, None, spec)
    assert rel_l2(x_gpu, x_ref) <= TOL[prec]


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("n,M,J,tile,weights", [
    (64, 8192, 4, 0, False),      # the 64^2 / 8192-visibility workload
    (64, 12345, 4, 8, True),      # ragged M, weights
    (32, 3001, 6, 8, True),
    (32, 999, 2, 16, False),
    (32, 2048, 8, 8, True),
    (128, 40000, 4, 16, False),
    (16, 1, 4, 8, False),         # a single visibility
])
def test_phi_and_adjoint_parity(P, prec, n, M, J, tile, weights):
    say(f"phi parity prec={prec} n={n} M={M} J={J} tile={tile} w={weights}")
    x, uv, w, spec = problem(n, M, J, 2000, seed=n + M + J, prec=prec, weights=weights)
    plan, perm = make_plan(P, n, uv, w, J, 2000, prec, tile)
    assert sorted(perm.tolist()) == list(range(M))
    y_gpu = plan.apply(to_dev(x, _rdt(prec))).cpu().numpy()
    uv64 = uv.astype(np.float64)
    w64 = None if w is None else w.astype(np.float64)
    y_ref = ms.phi(x, uv64, w64, spec)[perm]
    assert rel_l2(y_gpu, y_ref) <= TOL[prec]
    # adjoint on random data
    rng = np.random.default_rng(M)
    yy = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    yy_plan = yy[perm]
    x_gpu = plan.adjoint(to_dev(yy_plan, _cdt(prec))).cpu().numpy()
    x_ref = ms.phi_adjoint(yy, uv64, w64, spec)
    assert rel_l2(x_gpu, x_ref) <= TOL[prec]


@pytest.mark.parametrize("J,tile", [(4, 8), (4, 16), (2, 32)])
def test_plan_order_is_the_stable_cell_sort(P, J, tile):
    n, M = 64, 20000
    say(f"plan order J={J} tile={tile}")
    x, uv, w, spec = problem(n, M, J, 2000, seed=tile)
    plan, perm = make_plan(P, n, uv, None, J, 2000, "f32", tile)
    keys = cell_keys(uv.astype(np.float64), spec, tile)
    ks = keys[perm]
    assert np.all(np.diff(ks) >= 0)
    # stable: equal keys keep the user order
    same = np.diff(ks) == 0
    assert np.all(np.diff(perm)[same] > 0)


@pytest.mark.parametrize("prec,J,tile,M", [("f32", 2, 32, 40000), ("f32", 6, 16, 40000), ("f64", 6, 8, 30000),
                                           ("f64", 8, 8, 30000), ("f32", 4, 8, 600000), ("f64", 4, 16, 50000)])
def test_tile_and_support_variants(P, prec, J, tile, M):
    # includes a dense case (~37 visibilities per grid cell) where runs span many segments
    n = 64 if M > 100000 else 128
    say(f"phi variants {prec} J={J} tile={tile} M={M}")
    x, uv, w, spec = problem(n, M, J, 2000, seed=77 + J, prec=prec, weights=True)
    plan, perm = make_plan(P, n, uv, w, J, 2000, prec, tile)
    uv64, w64 = uv.astype(np.float64), w.astype(np.float64)
    y_gpu = plan.apply(to_dev(x, _rdt(prec))).cpu().numpy()
    assert rel_l2(y_gpu, ms.phi(x, uv64, w64, spec)[perm]) <= TOL[prec]
    rng = np.random.default_rng(3)
    yy = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    x_gpu = plan.adjoint(to_dev(yy[perm], _cdt(prec))).cpu().numpy()
    assert rel_l2(x_gpu, ms.phi_adjoint(yy, uv64, w64, spec)) <= TOL[prec]


def test_empty_visibility_set(P):
    say("phi M=0")
    n = 16
    uv = np.zeros((0, 2), dtype=np.float32)
    plan, perm = make_plan(P, n, uv, None, 4, 2000)
    assert plan.items == 0
    x = plan.adjoint(torch.zeros(0, dtype=torch.complex64, device=DEV))
    assert torch.count_nonzero(x).item() == 0
    y = plan.apply(torch.ones((n, n), dtype=torch.float32, device=DEV))
    assert y.numel() == 0


@pytest.mark.parametrize("prec,tol", [("f32", 2e-6), ("f64", 1e-12)])
def test_adjoint_identity_on_gpu(P, prec, tol):
    n, M = 64, 30000
    say(f"adjoint identity {prec}")
    x, uv, w, spec = problem(n, M, 4, 2000, seed=5, prec=prec, weights=True)
    plan, perm = make_plan(P, n, uv, w, 4, 2000, prec)
    rng = np.random.default_rng(1)
    xr = rng.standard_normal((n, n))
    yr = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    phix = plan.apply(to_dev(xr, _rdt(prec))).cpu().numpy().astype(np.complex128)
    phiy = plan.adjoint(to_dev(yr, _cdt(prec))).cpu().numpy().astype(np.float64)
    lhs = np.real(np.vdot(yr, phix))
    rhs = np.sum(xr * phiy)
    assert abs(lhs - rhs) <= tol * np.linalg.norm(yr) * np.linalg.norm(phix)


def test_gridding_is_bitwise_deterministic(P):
    n, M = 128, 200000
    say("gridding determinism")
    x, uv, w, spec = problem(n, M, 4, 2000, seed=9, weights=True)
    plan, perm = make_plan(P, n, uv, w, 4, 2000)
    rng = np.random.default_rng(2)
    y = to_dev(rng.standard_normal(M) + 1j * rng.standard_normal(M), torch.complex64)
    a = plan.adjoint(y).clone()
    b = plan.adjoint(y).clone()
    assert torch.equal(a, b)
    # a second plan over the same baselines gives the same order and the same bits
    plan2, perm2 = make_plan(P, n, uv, w, 4, 2000)
    assert np.array_equal(perm, perm2)
    assert torch.equal(plan2.adjoint(y), a)


@pytest.mark.parametrize("prec,tol", [("f32", 1e-5), ("f64", 1e-11)])
def test_power_method_parity(P, prec, tol):
    n, M = 32, 4000
    say(f"power method {prec}")
    x, uv, w, spec = problem(n, M, 4, 2000, seed=3, prec=prec)
    plan, perm = make_plan(P, n, uv, None, 4, 2000, prec)
    g = plan.norm(60)
    r = ms.power_method(uv.astype(np.float64), None, spec, iters=60)
    assert g == pytest.approx(r, rel=tol)


@pytest.mark.parametrize("J", [4, 6])
def test_phi_parity_at_the_single_operator_size(P, J):
    # 256^2 image, 512^2 grid, 1e6 visibilities: complex64 GPU against the FP64 oracle
    n, M = 256, 1_000_000
    say(f"phi parity 256^2 M=1e6 J={J}")
    x, uv, w, spec = problem(n, M, J, 2000, seed=1001)
    plan, perm = make_plan(P, n, uv, None, J, 2000)
    uv64 = uv.astype(np.float64)
    y_gpu = plan.apply(to_dev(x, torch.float32)).cpu().numpy()
    y_ref = ms.phi(x, uv64, None, spec)[perm]
    assert rel_l2(y_gpu, y_ref) <= 1e-5
    x_gpu = plan.adjoint(to_dev(y_ref, torch.complex64)).cpu().numpy()
    x_ref = ms.phi_adjoint(y_ref[np.argsort(perm)], uv64, None, spec)
    assert rel_l2(x_gpu, x_ref) <= 1e-5


@pytest.mark.parametrize("n,M,J,tile,weights", [
    (64, 12345, 4, 16, True),
    (64, 12345, 4, 8, False),
    (32, 3001, 6, 8, True),       # J > 4: the J-lane gridding kernel
    (32, 999, 2, 16, False),
    (32, 2048, 8, 8, True),
    (128, 200000, 4, 16, True),   # multi-chunk walk items
])
def test_stored_taps_equal_recomputed_taps(P, n, M, J, tile, weights):
    """FP32 plans store each visibility's nearest-sample taps (interp 0); the
    same plan with interp 2 recomputes them from (u, v) at every launch. Both
    pick the same samples, so Phi, Phi^dagger and the fused ADMM stages agree
    bit for bit."""
    say(f"stored vs recomputed taps n={n} M={M} J={J} tile={tile} w={weights}")
    x, uv, w, spec = problem(n, M, J, 2000, seed=7 * n + M + J, prec="f32", weights=weights)
    uv_d = torch.as_tensor(uv).to(DEV)
    w_d = None if w is None else torch.as_tensor(w).to(DEV)
    a = P.PhiPlan(n, uv_d, w_d, J=J, D=2000, tile=tile, interp=0)
    b = P.PhiPlan(n, uv_d, w_d, J=J, D=2000, tile=tile, interp=2)
    assert a.persistent.numel() < b.persistent.numel()     # (tap word, w) pairs vs (u, v, w)
    assert torch.equal(a.perm(), b.perm())
    xd = to_dev(x, torch.float32)
    ya, yb = a.apply(xd), b.apply(xd)
    assert torch.equal(ya, yb)
    rng = np.random.default_rng(M + 1)
    yy = to_dev(rng.standard_normal(M) + 1j * rng.standard_normal(M), torch.complex64)
    assert torch.equal(a.adjoint(yy), b.adjoint(yy))
    # the fused ADMM degridding epilogue and gridding prologue
    psi = P.PsiPlan(n, 3, 0x1FF, P.PR_F32, DEV)
    prm = P.admm_params(0.5 * float(torch.linalg.vector_norm(ya).item()), 1e-3, iters=3, op_norm=1.0)
    xa, ra = P.admm_solve(a, psi, ya, prm)
    xb, rb = P.admm_solve(b, psi, ya, prm)
    assert torch.equal(xa, xb)
    assert ra.resid_norm == rb.resid_norm and ra.l1_norm == rb.l1_norm
