"""Pins of the reweighted-l1 oracle (weighted DualFB, weighted ADMM and the
reweighting loop)."""
import numpy as np
import pytest

from oracle import admm, reweight as rw


def _bisect_tau_weighted(y, w, eps):
    # x = max(y - tau w, 0) with ||x - y|| = eps
    lo, hi = 0.0, float(np.max(y / w)) + 1.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if np.linalg.norm(np.maximum(y - mid * w, 0.0) - y) > eps:
            hi = mid
        else:
            lo = mid
    return lo


def test_weighted_dualfb_dirac_is_the_weighted_shift():
    rng = np.random.default_rng(41)
    z = rng.standard_normal((8, 8))
    w = rng.uniform(0.2, 2.0, (1, 8, 8))
    zbar, _ = admm.dual_fb(z, np.zeros((1, 8, 8)), 0.3, 1.0, lambda a: a[0], lambda x: x[None], 200, weights=w)
    assert np.allclose(zbar, np.maximum(z - 0.3 * w[0], 0.0), atol=1e-12)


def test_weighted_admm_identity_operator_closed_form():
    # min sum w_i |x_i| s.t. ||x - y|| <= eps, x >= 0  ->  x = max(y - tau w, 0)
    rng = np.random.default_rng(42)
    N = 48
    y = rng.uniform(0.2, 2.0, N)
    w = rng.uniform(0.3, 1.5, N)
    eps = 1.2
    xstar = np.maximum(y - _bisect_tau_weighted(y, w, eps) * w, 0.0)
    p = admm.AdmmParams(gamma=0.1, iters=800)
    x, _, _, _ = admm.admm(y.astype(complex), lambda v: v.astype(complex), np.real, lambda a: a[0],
                           lambda v: v[None], eps, p, np.zeros(N), weights=w[None])
    assert np.max(np.abs(x - xstar)) < 1e-6


def test_unit_weights_reproduce_the_unweighted_solver():
    rng = np.random.default_rng(43)
    M, N = 20, 6
    A = rng.standard_normal((M, N)) + 1j * rng.standard_normal((M, N))
    A /= np.linalg.norm(A, 2)
    y = A @ np.abs(rng.standard_normal(N))
    ident = lambda v: np.array(v, dtype=np.float64)
    p = admm.AdmmParams(gamma=0.01, iters=30)
    a = admm.admm(y, lambda v: A @ v, lambda r: np.real(A.conj().T @ r), ident, ident, 0.1, p, np.zeros(N))[0]
    b = admm.admm(y, lambda v: A @ v, lambda r: np.real(A.conj().T @ r), ident, ident, 0.1, p, np.zeros(N),
                  weights=np.ones(N))[0]
    assert np.array_equal(a, b)


def test_reweighting_rounds_follow_the_closed_form():
    rng = np.random.default_rng(44)
    N = 40
    y = rng.uniform(0.2, 2.0, N)
    eps, delta0, beta = 1.0, 0.5, 0.5
    p = admm.AdmmParams(gamma=0.1, iters=1500)
    x, w, reps = rw.sara_reweighted(y.astype(complex), lambda v: v.astype(complex), np.real, lambda a: a[0],
                                    lambda v: v[None], eps, p, 2, delta0, beta, np.zeros(N))
    # by hand: round 0 unweighted, then two weighted rounds with delta0 and delta0 beta
    xr = np.maximum(y - _bisect_tau_weighted(y, np.ones(N), eps), 0.0)
    for delta in (delta0, delta0 * beta):
        wr = delta / (delta + np.abs(xr))
        xr = np.maximum(y - _bisect_tau_weighted(y, wr, eps) * wr, 0.0)
    assert np.max(np.abs(x - xr)) < 1e-5
    # the returned weights are those of the last round
    assert np.max(np.abs(w[0] - wr)) < 1e-5
    assert len(reps) == 3
