"""Measurement operator Phi = W G F Z S and its adjoint (oracle, FP64).

Test infrastructure only (see the package header).

Paper passages: eq. (meas_eq) gives the Fourier relation with the sign
e^{-2 pi i (lu + mv)}; eq. (matrix_equation) factors the discrete operator as
y = W G F Z S x with S the gridding correction, Z zero padding, F an FFT, G the
convolutional interpolation off the grid and W noise weights; the adjoint
applies the adjoints in reverse order (S^H Z^H F^H G^H W^H). The pre-sampled
kernel is looked up by nearest sample (zeroth order) or interpolated linearly
between the two samples that bracket the tap distance (first order), the two
options the paper weighs in Section "Kernel Pre-Sampling". The operator is
normalised by its norm from the power method (Section "Distributed Images").

Conventions (readings where the paper is silent; every one is a parameter the
GPU library follows too):
  * image x[iy, ix], centred pixel p = (ix - n/2, iy - n/2); u pairs with the
    column offset p_x, v with the row offset p_y;
  * grid side K = oversample * n; pixel p is placed at grid index p mod K, so
    no fftshift phase is needed; F is the unnormalised DFT with sign e^{-};
  * u, v are in radians per pixel; the continuous grid coordinate is
    s = u * (K / 2 pi) computed in FP64;
  * the J taps of one axis are the cells j_a = floor(s) - J/2 + 1 + a,
    a = 0..J-1 (J even), each taken mod K;
  * nearest-sample rule: with fr = s - floor(s) and f = fr * D (both FP64),
    tap a at distance t_a = |s - j_a| uses sample round(t_a D) with ties toward
    the larger distance; written with m = J/2 - 1 - a this is
    m D + round_half_up(f) for m >= 0 and |m| D - round_half_down(f) for m < 0;
  * first-order rule: the distance in samples x_a = t_a D is formed as
    m D + f (m >= 0) or |m| D - f (m < 0) from the same FP64 f; with
    i = floor(x_a) and phi = x_a - i the weight is (1 - phi) T[i] + phi T[i+1]
    (for m >= 0: i = m D + floor(f), phi = f - floor(f); for m < 0 and f not an
    integer: i = |m| D - floor(f) - 1, phi = 1 - (f - floor(f)); for m < 0 and
    f an integer: i = |m| D - f, phi = 0);
  * weights W are real.

Parity: Phi, Phi^H are exact linear maps once the table is fixed, pinned by the
adjoint identity, by explicit dense matrices, by the direct non-uniform DFT
within the NUFFT error, and by F against a naive DFT (tests/test_oracle_phi.py).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import kaiser_bessel as kb


@dataclass
class PhiSpec:
    n: int
    K: int
    J: int = 4
    D: int = 2000
    interp: str = "nearest"     # "nearest" (zeroth order) or "linear" (first order)

    def __post_init__(self):
        if self.J % 2:
            raise ValueError("J must be even")
        if self.interp not in ("nearest", "linear"):
            raise ValueError("interp must be 'nearest' or 'linear'")
        self.beta = kb.kb_beta(self.J, self.K / self.n)
        self.table = kb.kb_table(self.J, self.D, self.beta)
        self.corr = kb.correction(self.n, self.K, self.J, self.beta)


# --------------------------------------------------------------------------
# interpolation taps
# --------------------------------------------------------------------------
def grid_coordinate(u, K: int):
    """s = u K / (2 pi) in FP64 (u widened exactly from its storage type)."""
    return np.asarray(u, dtype=np.float64) * (K / (2.0 * math.pi))


def taps_from_coordinate(s, J: int, D: int):
    """First tap cell and table indices for continuous grid coordinates s (FP64).

    Returns (j0, idx): j0 = floor(s) - J/2 + 1 (not yet reduced mod K) and idx
    of shape (M, J) with the nearest table sample for each tap.
    """
    s = np.asarray(s, dtype=np.float64).reshape(-1)
    fl = np.floor(s)
    fr = s - fl
    f = fr * D
    ff = np.floor(f)
    r = f - ff
    up = ff + (r >= 0.5)          # round half up of f
    dn = ff + (r > 0.5)           # round half down of f
    idx = np.empty((s.size, J), dtype=np.int64)
    for a in range(J):
        m = J // 2 - 1 - a
        if m >= 0:
            idx[:, a] = (m * D + up).astype(np.int64)
        else:
            idx[:, a] = ((-m) * D - dn).astype(np.int64)
    j0 = fl.astype(np.int64) - J // 2 + 1
    return j0, idx


def taps_1d(u, K: int, J: int, D: int):
    """Taps of one axis for coordinates u in radians per pixel."""
    return taps_from_coordinate(grid_coordinate(u, K), J, D)


def linear_taps_from_coordinate(s, J: int, D: int):
    """First tap cell, lower sample index and fraction for first-order lookup.

    Returns (j0, i, phi): i and phi of shape (M, J) such that the tap weight
    is (1 - phi) T[i] + phi T[i + 1], the straight line between the two
    samples bracketing the tap distance x = t D (see the module header).
    """
    s = np.asarray(s, dtype=np.float64).reshape(-1)
    fl = np.floor(s)
    fr = s - fl
    f = fr * D
    ff = np.floor(f)
    r = f - ff
    i = np.empty((s.size, J), dtype=np.int64)
    ph = np.empty((s.size, J), dtype=np.float64)
    for a in range(J):
        m = J // 2 - 1 - a
        if m >= 0:                       # x = m D + f
            i[:, a] = (m * D + ff).astype(np.int64)
            ph[:, a] = r
        else:                            # x = |m| D - f
            frac = r > 0
            i[:, a] = ((-m) * D - ff - frac).astype(np.int64)
            ph[:, a] = np.where(frac, 1.0 - r, 0.0)
    j0 = fl.astype(np.int64) - J // 2 + 1
    return j0, i, ph


def linear_weights(table, i, ph):
    """(1 - phi) T[i] + phi T[i + 1]; with phi = 0 only T[i] is used."""
    i1 = np.minimum(i + 1, table.size - 1)
    return (1.0 - ph) * table[i] + ph * table[i1]


def tap_weights(uv, spec: PhiSpec):
    """Per-visibility first cells and kernel weights on both axes."""
    if spec.interp == "linear":
        su = grid_coordinate(uv[:, 0], spec.K)
        sv = grid_coordinate(uv[:, 1], spec.K)
        ju, iu, pu = linear_taps_from_coordinate(su, spec.J, spec.D)
        jv, iv, pv = linear_taps_from_coordinate(sv, spec.J, spec.D)
        return ju, linear_weights(spec.table, iu, pu), jv, linear_weights(spec.table, iv, pv)
    ju, iu = taps_1d(uv[:, 0], spec.K, spec.J, spec.D)
    jv, iv = taps_1d(uv[:, 1], spec.K, spec.J, spec.D)
    return ju, spec.table[iu], jv, spec.table[iv]


# --------------------------------------------------------------------------
# S Z F and its adjoint
# --------------------------------------------------------------------------
def _grid_index(n: int, K: int):
    p = np.arange(-(n // 2), n - n // 2)
    return np.mod(p, K)


def szf(x, spec: PhiSpec):
    """F Z S x: corrected image placed at p mod K, then the unnormalised 2-D DFT.

    x may be real or complex (the complex case is used by the adjoint tests).
    """
    n, K = spec.n, spec.K
    x = np.asarray(x)
    x = x.astype(np.complex128 if np.iscomplexobj(x) else np.float64).reshape(n, n)
    g0 = np.zeros((K, K), dtype=np.complex128)
    gi = _grid_index(n, K)
    g0[np.ix_(gi, gi)] = x * spec.corr[None, :] * spec.corr[:, None]
    return np.fft.fft2(g0)


def szf_adjoint(grid, spec: PhiSpec):
    """S^H Z^H F^H grid: unnormalised inverse DFT (sign e^{+}), crop, correct. Complex."""
    n, K = spec.n, spec.K
    full = np.fft.ifft2(grid) * (K * K)
    gi = _grid_index(n, K)
    return full[np.ix_(gi, gi)] * spec.corr[None, :] * spec.corr[:, None]


# --------------------------------------------------------------------------
# G W and its adjoint
# --------------------------------------------------------------------------
def gw(X, uv, w, spec: PhiSpec, chunk: int = 1 << 18):
    """y_k = w_k sum_{a,b} g_a(u_k) g_b(v_k) X[(jv_k + b) mod K, (ju_k + a) mod K]."""
    K, J = spec.K, spec.J
    M = uv.shape[0]
    y = np.empty(M, dtype=np.complex128)
    w = np.ones(M) if w is None else np.asarray(w, dtype=np.float64)
    for s0 in range(0, M, chunk):
        sl = slice(s0, min(M, s0 + chunk))
        ju, wu, jv, wv = tap_weights(uv[sl], spec)
        acc = np.zeros(ju.size, dtype=np.complex128)
        for b in range(J):
            row = np.mod(jv + b, K)
            for a in range(J):
                col = np.mod(ju + a, K)
                acc += wv[:, b] * wu[:, a] * X[row, col]
        y[sl] = w[sl] * acc
    return y


def gw_adjoint(y, uv, w, spec: PhiSpec, chunk: int = 1 << 18):
    """grid[(jv + b) mod K, (ju + a) mod K] += g_a g_b w_k y_k (the transpose of gw)."""
    K, J = spec.K, spec.J
    M = uv.shape[0]
    y = np.asarray(y, dtype=np.complex128)
    w = np.ones(M) if w is None else np.asarray(w, dtype=np.float64)
    re = np.zeros(K * K)
    im = np.zeros(K * K)
    for s0 in range(0, M, chunk):
        sl = slice(s0, min(M, s0 + chunk))
        ju, wu, jv, wv = tap_weights(uv[sl], spec)
        yw = w[sl] * y[sl]
        for b in range(J):
            row = np.mod(jv + b, K)
            for a in range(J):
                col = np.mod(ju + a, K)
                val = wv[:, b] * wu[:, a] * yw
                flat = row * K + col
                re += np.bincount(flat, weights=val.real, minlength=K * K)
                im += np.bincount(flat, weights=val.imag, minlength=K * K)
    return (re + 1j * im).reshape(K, K)


# --------------------------------------------------------------------------
# Phi, Phi^H and the operator norm
# --------------------------------------------------------------------------
def phi(x, uv, w, spec: PhiSpec):
    """y = W G F Z S x."""
    return gw(szf(x, spec), uv, w, spec)


def phi_adjoint_complex(y, uv, w, spec: PhiSpec):
    """Phi^H y as a complex image (adjoint of Phi acting on complex images)."""
    return szf_adjoint(gw_adjoint(y, uv, w, spec), spec)


def phi_adjoint(y, uv, w, spec: PhiSpec):
    """Re(Phi^H y): the adjoint of Phi restricted to real images (dirty map)."""
    return phi_adjoint_complex(y, uv, w, spec).real


def power_method(uv, w, spec: PhiSpec, iters: int = 100, rtol: float = 0.0):
    """Largest eigenvalue of Re Phi^H Phi by power iteration; returns ||Phi||.

    Starts from the constant image of unit norm; each step x <- A x / ||A x||;
    the estimate after the last step is ||A x|| and ||Phi|| = sqrt of it.
    With rtol > 0 the iteration also stops after the first step whose estimate
    changed by at most rtol times itself from the step before (Section
    "Distributed Images" normalises Phi by this power-method estimate).
    """
    n = spec.n
    x = np.full((n, n), 1.0 / n)
    lam = 0.0
    lam_prev = -1.0
    for _ in range(iters):
        ax = phi_adjoint(phi(x, uv, w, spec), uv, w, spec)
        lam = float(np.sqrt(np.sum(ax * ax)))
        x = ax / lam
        if rtol > 0 and lam_prev >= 0 and abs(lam - lam_prev) <= rtol * lam:
            break
        lam_prev = lam
    return math.sqrt(lam)
