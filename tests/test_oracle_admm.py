"""Pins of the oracle's DualFB and ADMM (CPU only).

The full SARA problem has no closed form ("parity unpinned" beyond its parts);
these special cases reduce it to closed forms, and the 64^2 / 8192-visibility run is checked
against invariants of the method.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import admm, measurement as ms, prox, wavelets as wv


def _bisect_tau(y, eps):
    lo, hi = 0.0, float(np.max(y)) + 1.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if np.linalg.norm(np.maximum(y - mid, 0.0) - y) > eps:
            hi = mid
        else:
            lo = mid
    return lo


def test_admm_identity_operator_dirac_closed_form():
    rng = np.random.default_rng(0)
    N = 64
    y = rng.uniform(0.2, 2.0, N)
    eps = 1.5
    xstar = np.maximum(y - _bisect_tau(y, eps), 0.0)
    ident = lambda x: x.astype(complex)
    p = admm.AdmmParams(gamma=0.1, iters=400, inner_iters=1)
    x, s, d, rep = admm.admm(y.astype(complex), ident, np.real, lambda a: a[0], lambda x: x[None],
                             eps, p, np.zeros(N))
    assert np.max(np.abs(x - xstar)) < 1e-6
    assert np.linalg.norm(x - y) == pytest.approx(eps, rel=1e-6)


def test_dualfb_dirac_is_shifted_positive_part():
    rng = np.random.default_rng(1)
    z = rng.standard_normal((8, 8))
    gamma = 0.3
    zbar, _ = admm.dual_fb(z, np.zeros((1, 8, 8)), gamma, 1.0, lambda a: a[0], lambda x: x[None], 200)
    assert np.allclose(zbar, np.maximum(z - gamma, 0.0), atol=1e-10)


@pytest.mark.parametrize("N", [1, 4])
def test_dualfb_orthonormal_basis_without_positivity(N):
    # prox of gamma ||W .||_1 for orthonormal W is W^T S_gamma(W z) (semi-orthogonal prox property)
    n, L = 16, 2
    h = wv.daubechies_lowpass(N)
    Wf = lambda x: wv.dwt2(x[0] if x.ndim == 3 else x, h, L)[None]
    Wt = lambda a: wv.idwt2(a[0], h, L)
    rng = np.random.default_rng(2)
    z = rng.standard_normal((n, n))
    gamma = 0.4
    zbar, _ = admm.dual_fb(z, np.zeros((1, n, n)), gamma, 1.0, Wt, Wf, 300, positivity=False)
    ref = wv.idwt2(prox.soft_threshold(wv.dwt2(z, h, L), gamma), h, L)
    assert np.allclose(zbar, ref, atol=1e-10)


def test_local_balls_imply_global_ball():
    rng = np.random.default_rng(3)
    sizes = [5, 17, 9, 30]
    eps_j = rng.uniform(0.5, 2.0, len(sizes))
    y = [rng.standard_normal(m) + 1j * rng.standard_normal(m) for m in sizes]
    v = [yj + 3 * (rng.standard_normal(m) + 1j * rng.standard_normal(m)) for yj, m in zip(y, sizes)]
    r = [prox.proj_l2ball(vj, yj, e) for vj, yj, e in zip(v, y, eps_j)]
    glob = prox.l2_distance(np.concatenate(r), np.concatenate(y))
    assert glob <= math.sqrt(np.sum(eps_j ** 2)) * (1 + 1e-14)


def test_c0_sized_run_invariants():
    w = W.CONFIGS["admm64"]
    rng = W.rng_for(w.index)
    x_true = W.make_sky(w, rng)
    uv = W.make_uv(w, rng).astype(np.float64)
    spec = ms.PhiSpec(w.n, w.K, w.J, w.D)
    y0 = ms.phi(x_true, uv, None, spec)
    y, sigma, eps = W.add_noise(y0, W.unit_complex_noise(w.M, rng), w.snr_db)
    nrm = ms.power_method(uv, None, spec, iters=50)
    phi = lambda x: ms.phi(x, uv, None, spec) / nrm
    phi_adj = lambda v: ms.phi_adjoint(v, uv, None, spec) / nrm
    S = wv.Sara(w.n, w.levels)
    gamma = admm.default_gamma(y, phi_adj, S.adjoint)
    p = admm.AdmmParams(gamma=gamma, iters=w.iters)
    x, s, d, rep = admm.admm(y, phi, phi_adj, S.forward, S.adjoint, eps, p, np.zeros((w.n, w.n)))
    assert np.all(x >= 0) and np.all(np.isfinite(x))
    # the residual falls into the ball's neighbourhood and the iterates settle
    assert rep.resid[-1] < 0.2 * rep.resid[0]
    assert rep.resid[-1] <= 1.05 * eps
    assert rep.rel_var[-1] < 0.05
    # the reconstruction (in physical units x / ||Phi||) is closer to the sky than the zero image
    err = np.linalg.norm(x / nrm - x_true) / np.linalg.norm(x_true)
    assert err < 0.5


def test_local_ball_projection_is_the_nearest_point_of_the_product_of_balls():
    rng = np.random.default_rng(21)
    M, nsec = 40, 4
    sec = rng.integers(0, nsec, M)
    eps_j = rng.uniform(0.3, 1.5, nsec)
    z = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    x = z + 2.0 * (rng.standard_normal(M) + 1j * rng.standard_normal(M))
    p = prox.proj_l2balls_local(x, z, eps_j, sec)
    for j in range(nsec):
        idx = sec == j
        assert np.linalg.norm(p[idx] - z[idx]) <= eps_j[j] * (1 + 1e-14)
    # brute force: no sampled point of the product set is closer to x
    best = np.linalg.norm(p - x)
    for _ in range(2000):
        q = z.copy()
        for j in range(nsec):
            idx = np.nonzero(sec == j)[0]
            d = rng.standard_normal(idx.size) + 1j * rng.standard_normal(idx.size)
            q[idx] = z[idx] + d * (eps_j[j] * rng.uniform() ** (1.0 / (2 * idx.size)) / np.linalg.norm(d))
        assert np.linalg.norm(q - x) >= best - 1e-12


def test_admm_local_balls_identity_operator_closed_form():
    # min ||x||_1 s.t. ||x_j - y_j|| <= eps_j per section, x >= 0: separable,
    # x_j = max(y_j - tau_j, 0) with ||x_j - y_j|| = eps_j
    rng = np.random.default_rng(22)
    N, nsec = 64, 3
    y = rng.uniform(0.2, 2.0, N)
    sec = rng.integers(0, nsec, N)
    eps_j = np.array([0.6, 1.0, 0.8])
    xstar = np.zeros(N)
    for j in range(nsec):
        idx = sec == j
        xstar[idx] = np.maximum(y[idx] - _bisect_tau(y[idx], eps_j[j]), 0.0)
    ident = lambda x: x.astype(complex)
    p = admm.AdmmParams(gamma=0.1, iters=600, inner_iters=1)
    x, s, d, rep = admm.admm(y.astype(complex), ident, np.real, lambda a: a[0], lambda x: x[None],
                             eps_j, p, np.zeros(N), sections=sec)
    assert np.max(np.abs(x - xstar)) < 1e-6
    for j in range(nsec):
        assert np.linalg.norm((x - y)[sec == j]) == pytest.approx(eps_j[j], rel=1e-6)


def test_admm_local_balls_are_invariant_to_the_visibility_order():
    rng = np.random.default_rng(23)
    M, N, nsec = 30, 6, 3
    A = rng.standard_normal((M, N)) + 1j * rng.standard_normal((M, N))
    A /= np.linalg.norm(A, 2)
    y = A @ np.abs(rng.standard_normal(N)) + 0.05 * (rng.standard_normal(M) + 1j * rng.standard_normal(M))
    sec = rng.integers(0, nsec, M)
    eps_j = np.array([0.05, 0.1, 0.08])
    ident = lambda v: np.array(v, dtype=np.float64)
    p = admm.AdmmParams(gamma=0.01, iters=40)

    def run(perm):
        Ap = A[perm]
        return admm.admm(y[perm], lambda v: Ap @ v, lambda r: np.real(Ap.conj().T @ r), ident, ident,
                         eps_j, p, np.zeros(N), sections=sec[perm])[0]

    x0 = run(np.arange(M))
    x1 = run(rng.permutation(M))
    assert np.max(np.abs(x0 - x1)) < 1e-12
    # one section equals the global ball
    xg = admm.admm(y, lambda v: A @ v, lambda r: np.real(A.conj().T @ r), ident, ident, 0.1, p, np.zeros(N))[0]
    xl = admm.admm(y, lambda v: A @ v, lambda r: np.real(A.conj().T @ r), ident, ident, [0.1], p, np.zeros(N),
                   sections=np.zeros(M, dtype=int))[0]
    assert np.array_equal(xg, xl)
