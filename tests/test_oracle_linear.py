"""First-order (linear) lookup of the pre-sampled kernel (Section "Kernel
Pre-Sampling" weighs zeroth- against first-order interpolation).

Pins: the lower sample index and fraction against exact rational arithmetic
on the FP64 coordinate; the interpolation error against the exact kernel
within the textbook bound max|g''| / (8 D^2); agreement with the nearest rule
on sample points; Phi against the direct non-uniform DFT (first order reaches
the exact-kernel NUFFT error at D = 2000, far below the nearest rule); the
adjoint identity.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import workloads as W
from oracle import kaiser_bessel as kb, measurement as ms
from oracle.nudft import nudft


def _exact_linear(s_float, J, D):
    s = Fraction(s_float)
    j0 = math.floor(s) - J // 2 + 1
    out = []
    for a in range(J):
        x = abs(s - (j0 + a)) * D
        lo = math.floor(x)
        out.append((lo, x - lo))
    return j0, out


@pytest.mark.parametrize("J,D", [(4, 2000), (6, 2000), (4, 4), (8, 16)])
def test_linear_rule_brute_force(J, D):
    K = 128
    rng = np.random.default_rng(12)
    u = np.concatenate([rng.uniform(-math.pi, math.pi, 300),
                        [-math.pi, 0.0, 2 * math.pi / K, -2 * math.pi / K, math.pi - 1e-7]])
    u = u.astype(np.float32).astype(np.float64)
    s = ms.grid_coordinate(u, K)
    j0, i, ph = ms.linear_taps_from_coordinate(s, J, D)
    for k in range(u.size):
        ej0, ex = _exact_linear(float(s[k]), J, D)
        assert j0[k] == ej0
        for a in range(J):
            assert i[k, a] == ex[a][0]
            assert ph[k, a] == pytest.approx(float(ex[a][1]), abs=1e-9)
    assert i.min() >= 0 and i.max() <= J * D // 2 and ph.min() >= 0 and ph.max() < 1


@pytest.mark.parametrize("J,D", [(4, 16), (4, 100), (6, 100), (4, 2000)])
def test_linear_error_within_second_derivative_bound(J, D):
    beta = kb.kb_beta(J, 2.0)
    table = kb.kb_table(J, D, beta)
    # max |g''| on [0, J/2) by central differences on a fine grid
    h = 1e-4
    tt = np.linspace(h, J / 2 - h, 20001)
    g2 = (kb.kb_kernel(tt + h, J, beta) - 2 * kb.kb_kernel(tt, J, beta) + kb.kb_kernel(tt - h, J, beta)) / h ** 2
    bound = np.max(np.abs(g2)) / (8.0 * D * D)
    rng = np.random.default_rng(3)
    t = rng.uniform(0, J / 2 - 1e-9, 20000)
    x = t * D
    i = np.floor(x).astype(np.int64)
    ph = x - i
    err = np.max(np.abs(ms.linear_weights(table, i, ph) - kb.kb_kernel(t, J, beta)))
    assert err <= bound * 1.01 + 1e-15
    # and the nearest rule is much worse at the same density
    near = np.max(np.abs(table[np.floor(x + 0.5).astype(np.int64)] - kb.kb_kernel(t, J, beta)))
    assert err < near / 5


def test_linear_equals_nearest_on_sample_points():
    J, D, K = 4, 8, 64
    # s with fractional part k / D: every tap distance is a whole number of samples
    s = np.array([3.0, 3.125, -2.5, 10.875, 0.0])
    j0, i, ph = ms.linear_taps_from_coordinate(s, J, D)
    j0n, idx = ms.taps_from_coordinate(s, J, D)
    assert np.all(j0 == j0n)
    assert np.all(ph == 0.0)
    assert np.all(i == idx)


@pytest.mark.parametrize("J", [4, 6])
def test_linear_phi_reaches_exact_kernel_accuracy(J):
    n, K = 32, 64
    rng = np.random.default_rng(5)
    x = W.gaussian_sky(n, 20, rng)
    uv = W.uv_gaussian(400, rng).astype(np.float64)
    w = rng.uniform(0.5, 1.5, 400)
    y0 = nudft(x, uv, w)
    e_lin = np.linalg.norm(ms.phi(x, uv, w, ms.PhiSpec(n, K, J, 2000, "linear")) - y0) / np.linalg.norm(y0)
    e_near = np.linalg.norm(ms.phi(x, uv, w, ms.PhiSpec(n, K, J, 2000)) - y0) / np.linalg.norm(y0)
    # the exact-kernel NUFFT error at this size is 5.6e-4 (J = 4) and 5.3e-6 (J = 6)
    limit = {4: 1.2e-3, 6: 1.2e-5}[J]
    assert e_lin < limit
    if J == 6:
        assert e_lin < e_near / 10


def test_linear_adjoint_identity():
    n, K, J = 16, 32, 4
    spec = ms.PhiSpec(n, K, J, 100, "linear")
    rng = np.random.default_rng(8)
    uv = W.uv_gaussian(300, rng).astype(np.float64)
    w = rng.uniform(0.5, 1.5, 300)
    x = rng.standard_normal((n, n))
    y = rng.standard_normal(300) + 1j * rng.standard_normal(300)
    lhs = np.vdot(ms.phi(x, uv, w, spec), y).real
    rhs = float(np.sum(x * ms.phi_adjoint(y, uv, w, spec)))
    assert lhs == pytest.approx(rhs, rel=1e-12)
