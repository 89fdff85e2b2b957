"""Pins of the Primal-Dual oracle (Algorithm "Primal-Dual Algorithm").

The full SARA problem has no closed form ("parity unpinned" beyond its parts);
these cases fix the iteration by hand-computed steps, closed-form limits,
brute-force minima, the direct prox of the conjugates and the saddle-point
optimality condition.
"""
import itertools

import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import primal_dual as pd
from oracle import wavelets as wv

ident = lambda v: np.array(v, dtype=np.float64)


def _bisect_tau(y, eps):
    lo, hi = 0.0, float(np.max(y)) + 1.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if np.linalg.norm(np.maximum(y - mid, 0.0) - y) > eps:
            hi = mid
        else:
            lo = mid
    return lo


@pytest.mark.parametrize("misfit,z_exp,x_exp", [
    # y = 2, sigma = 1, tau = 0.5, theta = 1, gamma = 0.2, by hand:
    # l2:   z1 = (0 - 2) / 2 = -1, x1 = 0.5 - 0.1 = 0.4, xh1 = 0.8;
    #       z2 = (-1 + 0.8 - 2) / 2 = -1.1, x2 = 0.4 + 0.55 - 0.1 = 0.85
    ("l2", [-1.0, -1.1], [0.4, 0.85]),
    # ball (eps = 0.5): z1 = 0 - P_B(0) = -1.5, x1 = 0.75 - 0.1 = 0.65, xh1 = 1.3;
    #       z2 = -0.2 - P_B(-0.2) = -0.2 - 1.5 = -1.7, x2 = 0.65 + 0.85 - 0.1 = 1.4
    ("ball", [-1.5, -1.7], [0.65, 1.4]),
])
def test_two_iterations_by_hand(misfit, z_exp, x_exp):
    one = lambda v: np.array([complex(np.ravel(v)[0])])
    one_adj = lambda r: np.array([np.real(r[0])])
    y = np.array([2.0 + 0j])
    for k in (1, 2):
        x, z, _, _ = pd.primal_dual(y, one, one_adj, ident, ident, 0.2, 0.5, 1.0, 1.0, k, np.zeros(1),
                                    misfit=misfit, eps=0.5)
        assert z[0] == pytest.approx(z_exp[k - 1], abs=1e-15)
        assert x[0] == pytest.approx(x_exp[k - 1], abs=1e-15)


def test_l2_identity_operator_dirac_closed_form():
    # min gamma ||x||_1 + 1/2 ||y - x||^2, x >= 0  ->  x = max(y - gamma, 0)
    rng = np.random.default_rng(11)
    n = 8
    y = rng.standard_normal((n, n))
    S = wv.Sara(n, 1, mask=0x1)
    x, z, _, _ = pd.primal_dual(y, lambda v: v.astype(np.complex128), np.real, S.forward, S.adjoint,
                                0.3, 0.5, 1.0, 1.0, 400, np.zeros((n, n)), misfit="l2", inner_iters=5)
    assert np.max(np.abs(x - np.maximum(y - 0.3, 0.0))) < 1e-8
    # optimality of the saddle point: z = grad f(L x) = L x - y
    assert np.max(np.abs(z - (x - y))) < 1e-8


def test_ball_identity_operator_dirac_closed_form():
    # min ||x||_1 s.t. ||x - y|| <= eps, x >= 0  ->  x = max(y - t, 0) with ||x - y|| = eps
    rng = np.random.default_rng(12)
    N = 64
    y = rng.uniform(0.2, 2.0, N)
    eps = 1.5
    xstar = np.maximum(y - _bisect_tau(y, eps), 0.0)
    x, _, _, _ = pd.primal_dual(y.astype(complex), lambda v: v.astype(complex), np.real,
                                lambda a: a[0], lambda v: v[None], 0.1, 0.5, 1.0, 1.0, 600, np.zeros(N),
                                misfit="ball", eps=eps)
    assert np.max(np.abs(x - xstar)) < 1e-6
    assert np.linalg.norm(x - y) == pytest.approx(eps, rel=1e-6)


def test_tiny_map_problem_matches_brute_force_minimum():
    rng = np.random.default_rng(9)
    A = rng.standard_normal((3, 2)) + 1j * rng.standard_normal((3, 2))
    A /= np.linalg.norm(A, 2)
    y = A @ np.array([0.7, 0.0]) + 0.05 * (rng.standard_normal(3) + 1j * rng.standard_normal(3))
    gamma = 0.05
    x, z, _, _ = pd.primal_dual(y, lambda v: A @ np.ravel(v), lambda r: np.real(A.conj().T @ r), ident, ident,
                                gamma, 0.7, 1.0, 1.0, 4000, np.zeros(2), misfit="l2", inner_iters=20)
    obj = lambda v: gamma * np.sum(np.abs(v)) + 0.5 * np.sum(np.abs(A @ v - y) ** 2)
    g = np.linspace(0.0, 1.5, 1501)
    best = min((obj(np.array([a, b])), a, b) for a, b in itertools.product(g[::10], g[::10]))
    a0, b0 = best[1], best[2]
    fine = [(obj(np.array([a, b])), a, b)
            for a in g[max(0, int(a0 * 1000) - 20):int(a0 * 1000) + 21]
            for b in g[max(0, int(b0 * 1000) - 20):int(b0 * 1000) + 21]]
    fmin, am, bm = min(fine)
    assert obj(x) <= fmin + 1e-9
    assert abs(x[0] - am) <= 2e-3 and abs(x[1] - bm) <= 2e-3
    assert np.max(np.abs(z - (A @ x - y))) < 1e-8


@pytest.mark.parametrize("misfit", ["l2", "ball"])
def test_moreau_step_equals_the_direct_prox_of_the_conjugate(misfit):
    # f* of the ball indicator is the support function Re<z, y> + eps ||z||;
    # f* of 1/2 ||. - y||^2 is 1/2 ||z||^2 + Re<z, y>. The prox is minimised numerically.
    rng = np.random.default_rng(13)
    M, sigma, eps = 4, 0.7, 0.8
    y = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    for scale in (0.3, 3.0):
        u = scale * (rng.standard_normal(M) + 1j * rng.standard_normal(M))
        if misfit == "ball":
            fstar = lambda z: np.real(np.vdot(y, z)) + eps * np.linalg.norm(z)
        else:
            fstar = lambda z: 0.5 * np.linalg.norm(z) ** 2 + np.real(np.vdot(y, z))
        c = lambda p: p[:M] + 1j * p[M:]
        obj = lambda p: sigma * fstar(c(p)) + 0.5 * np.linalg.norm(c(p) - u) ** 2
        p0 = np.concatenate([u.real, u.imag])
        r = minimize(obj, p0, method="Powell", options={"xtol": 1e-11, "ftol": 1e-14, "maxiter": 200000})
        z_num = c(r.x)
        z_or = pd.prox_conjugate(u, y, sigma, misfit, eps)
        assert obj(np.concatenate([z_or.real, z_or.imag])) <= r.fun + 1e-10
        assert np.max(np.abs(z_or - z_num)) < 1e-4
