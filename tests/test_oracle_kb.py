"""Pins of the oracle's Kaiser-Bessel kernel, table and correction (CPU only)."""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate, special

from oracle import kaiser_bessel as kb

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_i0_matches_scipy():
    x = np.linspace(0.0, 40.0, 2001)
    assert np.max(np.abs(kb.i0(x) / special.i0(x) - 1.0)) < 1e-14


@pytest.mark.parametrize("J", [2, 4, 6, 8])
def test_kernel_shape(J):
    beta = kb.kb_beta(J)
    assert kb.kb_kernel(0.0, J, beta) == pytest.approx(1.0, abs=1e-15)
    # edge value is 1/I0(beta), zero outside, symmetric, monotone on [0, J/2]
    assert kb.kb_kernel(J / 2, J, beta) == pytest.approx(1.0 / special.i0(beta), rel=1e-13)
    assert kb.kb_kernel(J / 2 + 1e-9, J, beta) == 0.0
    t = np.linspace(0, J / 2, 1001)
    g = kb.kb_kernel(t, J, beta)
    assert np.all(np.diff(g) < 0)
    assert np.allclose(kb.kb_kernel(-t, J, beta), g, rtol=0, atol=0)


@pytest.mark.parametrize("J", [4, 6])
def test_fourier_transform_against_quadrature(J):
    beta = kb.kb_beta(J)
    for f in [0.0, 0.05, 0.13, 0.25, 0.4, 0.9]:
        val, _ = integrate.quad(lambda t: kb.kb_kernel(t, J, beta) * math.cos(2 * math.pi * f * t),
                                -J / 2, J / 2, epsabs=1e-14, epsrel=1e-13, limit=200)
        assert kb.kb_fourier(f, J, beta) == pytest.approx(val, rel=1e-10, abs=1e-13)


def _max_abs_derivative(J, beta):
    t = np.linspace(0, J / 2, 200001)
    g = kb.kb_kernel(t, J, beta)
    return float(np.max(np.abs(np.diff(g) / np.diff(t))))


@pytest.mark.parametrize("J,D", [(4, 2000), (6, 2000), (4, 50)])
def test_table_nearest_sample_error_bound(J, D):
    beta = kb.kb_beta(J)
    T = kb.kb_table(J, D, beta)
    assert T.size == J * D // 2 + 1
    rng = np.random.default_rng(7)
    t = rng.uniform(0, J / 2, 20000)
    idx = np.floor(t * D + 0.5).astype(int)
    err = np.abs(T[idx] - kb.kb_kernel(t, J, beta))
    bound = _max_abs_derivative(J, beta) / (2 * D)
    assert err.max() <= bound * (1 + 1e-6) + 1e-15
    # and the bound is essentially reached, so the check is not vacuous
    assert err.max() > 0.5 * bound


def test_paper_presampling_accuracy_claim():
    fx = json.load(open(os.path.join(GOLDEN, "presampling_accuracy.json")))
    J, D = fx["J"], fx["samples_per_pixel"]
    beta = kb.kb_beta(J)
    T = kb.kb_table(J, D, beta)
    # the table covers 0 <= t <= J/2: J/2 * D samples (plus the t = 0 end point)
    assert T.size - 1 == fx["samples_for_half_support"]
    rng = np.random.default_rng(3)
    t = rng.uniform(0, J / 2, 200000)
    idx = np.floor(t * D + 0.5).astype(int)
    assert np.max(np.abs(T[idx] - kb.kb_kernel(t, J, beta))) <= fx["max_abs_error"]


def test_correction_is_reciprocal_transform():
    n, K, J = 16, 32, 4
    beta = kb.kb_beta(J)
    c = kb.correction(n, K, J, beta)
    assert c.size == n
    # centre pixel: 1/ghat(0) = I0(beta) beta / (J sinh beta)
    assert c[n // 2] == pytest.approx(special.i0(beta) * beta / (J * math.sinh(beta)), rel=1e-13)
    # symmetric in p (c[p] = c[-p]) and growing towards the edge
    assert np.allclose(c[1:], c[1:][::-1], rtol=1e-14)
    assert np.all(np.diff(c[n // 2:]) > 0)
