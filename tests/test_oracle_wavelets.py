"""Pins of the oracle's Daubechies filters, DWT and SARA dictionary (CPU only)."""
import json
import math
import os

import numpy as np
import pytest

from oracle import wavelets as wv

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _closed(expr):
    return eval(expr, {"sqrt": math.sqrt})


@pytest.mark.parametrize("N", range(1, 9))
def test_filter_identities(N):
    h = wv.daubechies_lowpass(N)
    g = wv.highpass_from_lowpass(h)
    assert h.size == 2 * N
    assert h.sum() == pytest.approx(math.sqrt(2), abs=1e-14)
    for m in range(N):                                   # double-shift orthonormality
        ip = np.dot(h[: h.size - 2 * m], h[2 * m:])
        assert ip == pytest.approx(1.0 if m == 0 else 0.0, abs=1e-13)
    k = np.arange(2 * N, dtype=float)
    for p in range(N):                                   # vanishing moments of g
        mom = np.sum(k ** p * g)
        assert abs(mom) <= 1e-10 * max(1.0, np.sum(np.abs(k ** p * g)))
    # power complementarity |H(w)|^2 + |H(w + pi)|^2 = 2
    w = np.linspace(0, math.pi, 97)
    H = lambda om: np.polyval(h[::-1], np.exp(-1j * om))
    assert np.allclose(np.abs(H(w)) ** 2 + np.abs(H(w + math.pi)) ** 2, 2.0, atol=1e-12)


@pytest.mark.parametrize("N", range(2, 9))
def test_filters_are_minimum_phase(N):
    # z^(2N-1) H(z) = (z + 1)^N Q(z); every zero of Q lies strictly inside the unit circle
    h = wv.daubechies_lowpass(N)
    binom = np.array([math.comb(N, k) for k in range(N + 1)], dtype=float)
    q, rem = np.polydiv(h, binom)
    assert np.max(np.abs(rem)) < 1e-12
    assert np.all(np.abs(np.roots(q)) < 1)


def test_db1_db2_closed_forms():
    fx = json.load(open(os.path.join(GOLDEN, "daubechies_closed_forms.json")))
    for name, N in (("db1", 1), ("db2", 2)):
        ref = np.array([_closed(e) for e in fx[name]])
        assert np.allclose(wv.daubechies_lowpass(N), ref, rtol=0, atol=1e-15)


def test_haar_2x2_by_hand():
    a, b, c, d = 1.0, 2.0, 4.0, 8.0
    x = np.array([[a, b], [c, d]])
    out = wv.dwt2(x, wv.daubechies_lowpass(1), 1)
    ref = np.array([[(a + b + c + d) / 2, (a - b + c - d) / 2],
                    [(a + b - c - d) / 2, (a - b - c + d) / 2]])
    assert np.allclose(out, ref, atol=1e-15)


@pytest.mark.parametrize("N", [1, 2, 5, 8])
@pytest.mark.parametrize("n,levels", [(16, 3), (32, 2), (8, 3)])
def test_perfect_reconstruction_and_energy(N, n, levels):
    h = wv.daubechies_lowpass(N)
    rng = np.random.default_rng(N * 100 + n)
    x = rng.standard_normal((n, n))
    c = wv.dwt2(x, h, levels)
    assert np.sum(c * c) == pytest.approx(np.sum(x * x), rel=1e-13)
    assert np.allclose(wv.idwt2(c, h, levels), x, atol=1e-12)
    assert np.allclose(wv.dwt2(wv.idwt2(x, h, levels), h, levels), x, atol=1e-12)


def test_periodic_shift_equivariance_one_level():
    h = wv.daubechies_lowpass(4)
    rng = np.random.default_rng(0)
    x = rng.standard_normal((16, 16))
    c = wv.dwt2(x, h, 1)
    cs = wv.dwt2(np.roll(x, -2, axis=1), h, 1)
    # a shift of two pixels shifts each subband by one coefficient
    assert np.allclose(cs[:, :8], np.roll(c[:, :8], -1, axis=1), atol=1e-13)
    assert np.allclose(cs[:, 8:], np.roll(c[:, 8:], -1, axis=1), atol=1e-13)


def test_sara_tight_frame_and_adjoint():
    n, L = 32, 3
    S = wv.Sara(n, L)
    assert S.nb == 9
    rng = np.random.default_rng(4)
    x = rng.standard_normal((n, n))
    alpha = rng.standard_normal((9, n, n))
    assert np.allclose(S.forward(S.adjoint(x)), x, atol=1e-12)
    assert np.sum(S.adjoint(x) * alpha) == pytest.approx(np.sum(x * S.forward(alpha)), rel=1e-12)
    # the Dirac block is x / 3
    assert np.allclose(S.adjoint(x)[0], x / 3, atol=0)


def test_basis_mask_selection():
    S = wv.Sara(16, 2, mask=0b110)        # db1, db2
    assert S.bases == ["db1", "db2"]
    assert S.scale == pytest.approx(1 / math.sqrt(2))
