"""Pins of the FISTA oracle (Algorithm "FISTA" for the MAP problem)."""
import itertools

import numpy as np
import pytest

from oracle import fista as fs
from oracle import wavelets as wv


def test_identity_operator_dirac_closed_form():
    # min gamma ||x||_1 + 1/2 ||y - x||^2, x >= 0  ->  x = max(y - gamma, 0)
    rng = np.random.default_rng(4)
    n = 8
    y = rng.standard_normal((n, n))
    gamma = 0.3
    ident = lambda v: v.astype(np.complex128)
    real = lambda v: np.real(v)
    S = wv.Sara(n, 1, mask=0x1)            # Dirac only (scale 1)
    x, _, _ = fs.fista(y, ident, real, S.forward, S.adjoint, gamma, 0.5, 400, np.zeros((n, n)),
                       inner_iters=5)
    assert np.max(np.abs(x - np.maximum(y - gamma, 0.0))) < 1e-8


def test_tiny_problem_matches_brute_force_minimum():
    # N = 2 real unknowns, M = 3 complex visibilities, Dirac dictionary with positivity
    rng = np.random.default_rng(9)
    A = rng.standard_normal((3, 2)) + 1j * rng.standard_normal((3, 2))
    A /= np.linalg.norm(A, 2)                  # ||Phi|| = 1
    x_true = np.array([0.7, 0.0])
    y = A @ x_true + 0.05 * (rng.standard_normal(3) + 1j * rng.standard_normal(3))
    gamma = 0.05
    phi = lambda v: A @ np.ravel(v)
    phi_adj = lambda r: np.real(A.conj().T @ r)
    ident = lambda v: np.array(v, dtype=np.float64)
    x, _, _ = fs.fista(y, phi, phi_adj, ident, ident, gamma, 1.0, 3000, np.zeros(2), inner_iters=20)
    obj = lambda v: gamma * np.sum(np.abs(v)) + 0.5 * np.sum(np.abs(A @ v - y) ** 2)
    g = np.linspace(0.0, 1.5, 1501)              # x >= 0, step 1e-3
    best = min((obj(np.array([a, b])), a, b) for a, b in itertools.product(g[::10], g[::10]))
    # refine around the coarse minimum
    a0, b0 = best[1], best[2]
    fine = [(obj(np.array([a, b])), a, b)
            for a in g[max(0, int(a0 * 1000) - 20):int(a0 * 1000) + 21]
            for b in g[max(0, int(b0 * 1000) - 20):int(b0 * 1000) + 21]]
    fmin, am, bm = min(fine)
    assert obj(x) <= fmin + 1e-9
    assert abs(x[0] - am) <= 2e-3 and abs(x[1] - bm) <= 2e-3
    assert np.all(x >= 0)


def test_fixed_point_of_the_forward_backward_map():
    # Dirac dictionary with positivity: the DualFB prox is exact after one
    # iteration, so the limit is a fixed point of x -> prox(x - lam grad f(x))
    rng = np.random.default_rng(10)
    n, M = 8, 40
    A = rng.standard_normal((M, n * n)) + 1j * rng.standard_normal((M, n * n))
    A /= np.linalg.norm(A, 2)
    y = A @ np.abs(rng.standard_normal(n * n)) + 0.01 * rng.standard_normal(M)
    phi = lambda v: A @ np.ravel(v)
    phi_adj = lambda r: np.real(A.conj().T @ r).reshape(n, n)
    ident = lambda v: np.array(v, dtype=np.float64)
    gamma, lam = 0.02, 1.0
    x, d, _ = fs.fista(y, phi, phi_adj, ident, ident, gamma, lam, 3000, np.zeros((n, n)), inner_iters=2)
    z = x - lam * phi_adj(phi(x) - y)
    xp = np.maximum(z - gamma * lam, 0.0)          # the exact prox for this dictionary
    assert np.linalg.norm(xp - x) <= 1e-9 * np.linalg.norm(x)
