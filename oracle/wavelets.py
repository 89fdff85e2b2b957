"""Daubechies wavelets and the SARA dictionary (oracle, FP64).

Test infrastructure only (see the package header).

Paper passages: the dictionary is a concatenation of n_w = 9 bases, a Dirac
basis and the 2-D separable (product of 1-D) Daubechies wavelets 1 to 8,
applied to a fixed number of levels (Section "MPI Wavelet Operator
Benchmarks"); x = Psi alpha with alpha the stacked coefficients of all bases
(Section "Distributed Wavelet Operator"); the analysis form of the problem
uses Psi^dagger x (Section "Analysis and Synthesis").

Readings where the paper is silent:
  * dbN low-pass filter (2N taps) from spectral factorisation of
    P(y) = sum_{k<N} C(N-1+k, k) y^k with y = sin^2(w/2), keeping the zeros
    inside the unit circle (minimum phase), normalised to sum h = sqrt(2),
    ordered as the coefficients of z^0, z^-1, ...; high-pass
    g_k = (-1)^k h_{2N-1-k};
  * periodic boundaries; one level filters the rows then the columns of the
    current low-low block, keeping the low half first (Mallat layout);
    analysis lo[m] = sum_k h[k] a[(2m + k) mod L], hi[m] likewise with g;
    synthesis is the transpose (equal to the inverse, the transform being
    orthonormal);
  * the dictionary is scaled by 1/sqrt(n_bases) so that Psi Psi^dagger = I.

Pins (tests/test_oracle_wavelets.py): filter identities (sum, double-shift
orthogonality, vanishing moments), db1 = Haar and the closed form of db2,
perfect reconstruction and the tight-frame identity, a 2x2 Haar block by hand.
"""
from __future__ import annotations

import math

import numpy as np


def daubechies_lowpass(N: int) -> np.ndarray:
    """Minimum-phase Daubechies low-pass filter with N vanishing moments."""
    if N < 1:
        raise ValueError("N >= 1")
    p = [math.comb(N - 1 + k, k) for k in range(N)]       # ascending powers of y
    zeros = []
    if N > 1:
        for yr in np.roots(p[::-1]):
            b = 2.0 - 4.0 * yr                              # z + 1/z = 2 - 4 y
            disc = np.sqrt(b * b - 4.0 + 0j)
            z1, z2 = (b + disc) / 2.0, (b - disc) / 2.0
            zeros.append(z1 if abs(z1) < 1.0 else z2)
    poly = np.array([1.0 + 0j])
    for _ in range(N):
        poly = np.convolve(poly, [1.0, 1.0])
    for z in zeros:
        poly = np.convolve(poly, [1.0, -z])
    h = poly.real.copy()
    return h * (math.sqrt(2.0) / h.sum())


def highpass_from_lowpass(h: np.ndarray) -> np.ndarray:
    L = h.size
    return np.array([(-1) ** k * h[L - 1 - k] for k in range(L)])


def analysis_1d(a: np.ndarray, h: np.ndarray, g: np.ndarray, axis: int):
    a = np.moveaxis(np.asarray(a, dtype=np.float64), axis, 0)
    L = a.shape[0]
    m2 = 2 * np.arange(L // 2)
    lo = np.zeros((L // 2,) + a.shape[1:])
    hi = np.zeros((L // 2,) + a.shape[1:])
    for k in range(h.size):
        take = a[(m2 + k) % L]
        lo += h[k] * take
        hi += g[k] * take
    return np.moveaxis(np.concatenate([lo, hi], axis=0), 0, axis)


def synthesis_1d(c: np.ndarray, h: np.ndarray, g: np.ndarray, axis: int):
    """Transpose of analysis_1d: scatter each coefficient back along its filter taps."""
    c = np.moveaxis(np.asarray(c, dtype=np.float64), axis, 0)
    L = c.shape[0]
    lo, hi = c[: L // 2], c[L // 2:]
    out = np.zeros_like(c)
    m2 = 2 * np.arange(L // 2)
    for k in range(h.size):
        idx = (m2 + k) % L                     # distinct for fixed k
        out[idx] += h[k] * lo + g[k] * hi
    return np.moveaxis(out, 0, axis)


def dwt2(x: np.ndarray, h: np.ndarray, levels: int) -> np.ndarray:
    g = highpass_from_lowpass(h)
    c = np.array(x, dtype=np.float64, copy=True)
    L = c.shape[0]
    for _ in range(levels):
        blk = analysis_1d(c[:L, :L], h, g, axis=1)   # rows
        blk = analysis_1d(blk, h, g, axis=0)         # columns
        c[:L, :L] = blk
        L //= 2
    return c


def idwt2(c: np.ndarray, h: np.ndarray, levels: int) -> np.ndarray:
    g = highpass_from_lowpass(h)
    x = np.array(c, dtype=np.float64, copy=True)
    L = x.shape[0] >> (levels - 1)
    for _ in range(levels):
        blk = synthesis_1d(x[:L, :L], h, g, axis=0)  # columns (transpose order)
        blk = synthesis_1d(blk, h, g, axis=1)        # rows
        x[:L, :L] = blk
        L *= 2
    return x


SARA_BASES = ("dirac",) + tuple(f"db{k}" for k in range(1, 9))


def basis_list(mask: int = 0x1FF):
    """Bases selected by bit mask: bit 0 Dirac, bit k (1..8) dbk."""
    return [SARA_BASES[i] for i in range(9) if mask >> i & 1]


class Sara:
    """Psi^dagger x = [x; W_1 x; ...] / sqrt(nb), Psi alpha = (alpha_0 + sum W_i^T alpha_i) / sqrt(nb)."""

    def __init__(self, n: int, levels: int, mask: int = 0x1FF):
        if n % (1 << levels):
            raise ValueError("n must be divisible by 2^levels")
        self.n, self.levels = n, levels
        self.bases = basis_list(mask)
        self.filters = {b: daubechies_lowpass(int(b[2:])) for b in self.bases if b != "dirac"}
        self.scale = 1.0 / math.sqrt(len(self.bases))

    @property
    def nb(self) -> int:
        return len(self.bases)

    def adjoint(self, x: np.ndarray) -> np.ndarray:
        x = np.asarray(x, dtype=np.float64).reshape(self.n, self.n)
        out = np.empty((self.nb, self.n, self.n))
        for i, b in enumerate(self.bases):
            out[i] = x if b == "dirac" else dwt2(x, self.filters[b], self.levels)
        return out * self.scale

    def forward(self, alpha: np.ndarray) -> np.ndarray:
        alpha = np.asarray(alpha, dtype=np.float64).reshape(self.nb, self.n, self.n)
        x = np.zeros((self.n, self.n))
        for i, b in enumerate(self.bases):
            x += alpha[i] if b == "dirac" else idwt2(alpha[i], self.filters[b], self.levels)
        return x * self.scale
