"""Pins of the oracle's measurement operator (CPU only)."""
import math
from fractions import Fraction

import numpy as np
import pytest

import workloads as W
from oracle import kaiser_bessel as kb
from oracle import measurement as ms
from oracle.nudft import nudft


def naive_dft2(g):
    K = g.shape[0]
    k = np.arange(K)
    E = np.exp(-2j * np.pi * np.outer(k, k) / K)
    out = np.zeros((K, K), dtype=complex)
    for ky in range(K):
        for kx in range(K):
            out[ky, kx] = np.sum(g * np.outer(E[ky], E[kx]))
    return out


@pytest.mark.parametrize("n,K", [(4, 8), (8, 16)])
def test_szf_against_naive_dft(n, K):
    spec = ms.PhiSpec(n, K, 4, 200)
    rng = np.random.default_rng(0)
    x = rng.standard_normal((n, n))
    g0 = np.zeros((K, K))
    for iy in range(n):
        for ix in range(n):
            py, px = iy - n // 2, ix - n // 2
            g0[py % K, px % K] = x[iy, ix] * spec.corr[ix] * spec.corr[iy]
    ref = naive_dft2(g0)
    got = ms.szf(x, spec)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_fft_parseval_and_delta():
    K = 32
    rng = np.random.default_rng(1)
    g = rng.standard_normal((K, K)) + 1j * rng.standard_normal((K, K))
    G = np.fft.fft2(g)
    assert np.sum(np.abs(G) ** 2) == pytest.approx(K * K * np.sum(np.abs(g) ** 2), rel=1e-13)
    d = np.zeros((K, K)); d[0, 0] = 1.0
    assert np.allclose(np.fft.fft2(d), 1.0, atol=1e-15)


def _exact_taps(s_float, J, D):
    """Nearest samples from exact rational arithmetic on the FP64 coordinate."""
    s = Fraction(s_float)
    j0 = math.floor(s) - J // 2 + 1
    out = []
    for a in range(J):
        x = abs(s - (j0 + a)) * D            # exact distance in table samples
        lo = math.floor(x)
        out.append(lo + 1 if x - lo >= Fraction(1, 2) else lo)   # ties: larger distance
    return j0, out


@pytest.mark.parametrize("J,D", [(4, 2000), (6, 2000), (4, 4), (8, 16)])
def test_nearest_sample_rule_brute_force(J, D):
    K = 128
    rng = np.random.default_rng(11)
    u = np.concatenate([rng.uniform(-math.pi, math.pi, 300),
                        [-math.pi, 0.0, 2 * math.pi / K, -2 * math.pi / K, math.pi - 1e-7]])
    u = u.astype(np.float32).astype(np.float64)
    j0, idx = ms.taps_1d(u, K, J, D)
    s = ms.grid_coordinate(u, K)
    for k in range(u.size):
        ej0, eidx = _exact_taps(float(s[k]), J, D)
        assert j0[k] == ej0
        assert list(idx[k]) == eidx
    assert idx.min() >= 0 and idx.max() <= J * D // 2


def test_tie_breaks_toward_larger_distance():
    # D = 4 and a fractional part of 1/8 put every tap distance on a half sample
    J, D = 4, 4
    j0, idx = ms.taps_from_coordinate(np.array([3.125, -0.875]), J, D)
    assert list(j0) == [2, -2]
    # distances 1.125, 0.125, 0.875, 1.875 -> 4.5, 0.5, 3.5, 7.5 samples -> 5, 1, 4, 8
    assert list(idx[0]) == [5, 1, 4, 8]
    assert list(idx[1]) == [5, 1, 4, 8]


# Relative error of Phi against the direct NUDFT of eq. (meas_eq) on this
# problem: J = 4: 7.1e-4 (D = 2000) and 6.6e-4 (D = 2e5, the kernel's own
# error); J = 6: 2.0e-4 (D = 2000, the table's error dominates) and 7.0e-6
# (D = 2e5). Each bound is twice the measured value: a wrong shape parameter,
# correction or tap offset moves the error by orders of magnitude.
@pytest.mark.parametrize("J,D,tol", [(4, 2000, 1.4e-3), (4, 200_000, 1.4e-3), (6, 2000, 4e-4),
                                     (6, 200_000, 1.5e-5)])
def test_phi_approximates_nudft(J, D, tol):
    n, K = 32, 64
    spec = ms.PhiSpec(n, K, J, D)
    rng = np.random.default_rng(5)
    x = W.gaussian_sky(n, 20, rng)
    uv = W.uv_gaussian(400, rng).astype(np.float64)
    w = rng.uniform(0.5, 1.5, 400)
    y = ms.phi(x, uv, w, spec)
    y0 = nudft(x, uv, w)
    assert np.linalg.norm(y - y0) / np.linalg.norm(y0) < tol


def test_phi_approximates_nudft_near_band_edge():
    # baselines next to +-pi wrap their taps around the grid
    n, K = 16, 32
    spec = ms.PhiSpec(n, K, 6, 20000)
    rng = np.random.default_rng(9)
    x = rng.uniform(0, 1, (n, n))
    uv = np.array([[-math.pi, 0.1], [math.pi - 1e-3, -math.pi], [3.0, 3.1], [-3.1, -2.9]])
    y = ms.phi(x, uv, None, spec)
    y0 = nudft(x, uv)
    assert np.max(np.abs(y - y0)) / np.max(np.abs(y0)) < 2e-3


def _random_problem(n=16, K=32, M=300, J=4, seed=2):
    spec = ms.PhiSpec(n, K, J, 2000)
    rng = np.random.default_rng(seed)
    uv = W.uv_gaussian(M, rng).astype(np.float64)
    w = rng.uniform(0.5, 1.5, M)
    return spec, rng, uv, w


def test_adjoint_identity_real_and_complex():
    spec, rng, uv, w = _random_problem()
    n, M = spec.n, uv.shape[0]
    x = rng.standard_normal((n, n))
    y = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    lhs = np.real(np.vdot(y, ms.phi(x, uv, w, spec)))
    rhs = np.sum(x * ms.phi_adjoint(y, uv, w, spec))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    xc = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    phix = ms.gw(ms.szf(xc, spec), uv, w, spec)
    lhs = np.vdot(y, phix)
    rhs = np.vdot(ms.phi_adjoint_complex(y, uv, w, spec), xc)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_dense_matrices_are_conjugate_transposes():
    spec, rng, uv, w = _random_problem(n=8, K=16, M=20)
    n, M = spec.n, uv.shape[0]
    N = n * n
    A = np.zeros((M, N), dtype=complex)
    for j in range(N):
        e = np.zeros(N, dtype=complex); e[j] = 1
        A[:, j] = ms.gw(ms.szf(e.reshape(n, n), spec), uv, w, spec)
    B = np.zeros((N, M), dtype=complex)
    for k in range(M):
        e = np.zeros(M, dtype=complex); e[k] = 1
        B[:, k] = ms.phi_adjoint_complex(e, uv, w, spec).reshape(-1)
    assert np.max(np.abs(B - A.conj().T)) <= 1e-13 * np.max(np.abs(A))
    # each row has exactly the J^2-tap structure: column j of F sampled by the taps
    # equals the NUDFT row up to the kernel error, so A is not degenerate
    assert np.linalg.matrix_rank(A) == min(M, N)


def test_power_method_matches_dense_two_norm():
    spec, rng, uv, w = _random_problem(n=8, K=16, M=60)
    n, M = spec.n, uv.shape[0]
    N = n * n
    A = np.zeros((M, N), dtype=complex)
    for j in range(N):
        e = np.zeros(N); e[j] = 1
        A[:, j] = ms.phi(e.reshape(n, n), uv, w, spec)
    real_map = np.vstack([A.real, A.imag])            # R^N -> R^{2M}
    ref = np.linalg.norm(real_map, 2)
    got = ms.power_method(uv, w, spec, iters=2000)
    assert got == pytest.approx(ref, rel=1e-8)
    # the stopping rule: a tight rtol reaches the same norm well before 2000
    # steps; every estimate ||A x|| of a unit x is a lower bound of ||A||
    assert ms.power_method(uv, w, spec, iters=2000, rtol=1e-15) == pytest.approx(ref, rel=1e-7)
    for rtol in (1e-2, 1e-3, 1e-6):
        est = ms.power_method(uv, w, spec, iters=2000, rtol=rtol)
        assert est <= ref * (1 + 1e-12)
    # a loose rtol stops after the first step that changes by <= rtol: the same
    # value as a fixed count equal to that step
    loose = ms.power_method(uv, w, spec, iters=2000, rtol=1e-2)
    steps = next(k for k in range(1, 2000)
                 if ms.power_method(uv, w, spec, iters=k) == loose)
    assert steps < 2000


def test_visibility_order_is_irrelevant():
    spec, rng, uv, w = _random_problem()
    x = rng.standard_normal((spec.n, spec.n))
    perm = rng.permutation(uv.shape[0])
    y = ms.phi(x, uv, w, spec)
    yp = ms.phi(x, uv[perm], w[perm], spec)
    assert np.array_equal(y[perm], yp)
