"""Pre-sampled Kaiser-Bessel gridding kernel (oracle, FP64).

Test infrastructure only (see the package header).

Paper passages: the kernel is the Kaiser-Bessel interpolation kernel with
support J (Section "Benchmark Timings"); it is pre-sampled on 0 <= |u| <= J/2
using the symmetry g(u) = g(-u) and looked up by zeroth-order (nearest sample)
interpolation (Section "Kernel Pre-Sampling"). The gridding correction S of
eq. (matrix_equation) divides each pixel by the kernel's Fourier transform.

Readings where the paper is silent:
  * shape parameter beta = pi sqrt((J/alpha)^2 (alpha - 1/2)^2 - 0.8), the
    formula of Beatty et al. (the work the paper cites for pre-sampling), with
    oversampling alpha = 2;
  * the correction is 1 / ghat(p/K) with ghat the closed-form Fourier transform
    of the continuous kernel.

Pins (tests/test_oracle_kb.py): I0 against scipy.special.i0; ghat against
numerical quadrature of g; table error against the derivative bound
max|g'| / (2D); the paper's accuracy claim for 2e5 samples per pixel.
"""
from __future__ import annotations

import math

import numpy as np


def i0(x):
    """Modified Bessel function of the first kind, order 0, by its power series.

    I0(x) = sum_k (x/2)^(2k) / (k!)^2. All terms are positive, so summing until
    the term drops below 1e-18 of the partial sum is accurate to rounding.
    """
    x = np.asarray(x, dtype=np.float64)
    q = (x * 0.5) ** 2
    term = np.ones_like(x)
    total = np.ones_like(x)
    k = 0
    while True:
        k += 1
        term = term * q / (k * k)
        total = total + term
        if np.all(term <= 1e-18 * total):
            break
    return total


def kb_beta(J: int, alpha: float = 2.0) -> float:
    return math.pi * math.sqrt((J / alpha) ** 2 * (alpha - 0.5) ** 2 - 0.8)


def kb_kernel(t, J: int, beta: float):
    """g(t) = I0(beta sqrt(1 - (2t/J)^2)) / I0(beta) on |t| <= J/2, else 0."""
    t = np.asarray(t, dtype=np.float64)
    arg = 1.0 - (2.0 * t / J) ** 2
    inside = arg >= 0.0
    val = i0(beta * np.sqrt(np.where(inside, arg, 0.0))) / i0(beta)
    return np.where(inside, val, 0.0)


def kb_table(J: int, D: int, beta: float) -> np.ndarray:
    """Samples T[i] = g(i / D) for i = 0 .. floor(J D / 2)."""
    i = np.arange(J * D // 2 + 1, dtype=np.float64)
    return kb_kernel(i / D, J, beta)


def kb_fourier(f, J: int, beta: float):
    """Closed-form Fourier transform of the kernel, ghat(f) = int g(t) e^{-2 pi i f t} dt.

    ghat(f) = J sinh(sqrt(beta^2 - (pi J f)^2)) / (sqrt(beta^2 - (pi J f)^2) I0(beta)),
    continued analytically (sinh -> sin) where (pi J f)^2 > beta^2.
    """
    f = np.asarray(f, dtype=np.float64)
    z2 = beta * beta - (math.pi * J * f) ** 2
    out = np.empty_like(f)
    pos = z2 > 0
    neg = z2 < 0
    zero = ~(pos | neg)
    zp = np.sqrt(np.where(pos, z2, 1.0))
    zn = np.sqrt(np.where(neg, -z2, 1.0))
    out = np.where(pos, np.sinh(zp) / zp, out)
    out = np.where(neg, np.sin(zn) / zn, out)
    out = np.where(zero, 1.0, out)
    return J * out / i0(beta)


def correction(n: int, K: int, J: int, beta: float) -> np.ndarray:
    """c[p + n/2] = 1 / ghat(p / K) for centred pixel offsets p = -n/2 .. n/2-1."""
    p = np.arange(-(n // 2), n - n // 2, dtype=np.float64)
    return 1.0 / kb_fourier(p / K, J, beta)
