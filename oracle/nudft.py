"""Direct non-uniform DFT (oracle, FP64, small sizes only).

Test infrastructure only (see the package header).

This is the discrete form of eq. (meas_eq) with a(l, m) = 1: each visibility is
y_k = w_k sum_p x[p] exp(-i (u_k p_x + v_k p_y)) over centred pixels p. The
NUFFT of eq. (matrix_equation) approximates it; the gap is the interpolation
error of the kernel, which tests bound (pin of Phi, not of this function, which
is its own definition written out).
"""
from __future__ import annotations

import numpy as np


def nudft(x, uv, w=None):
    n = x.shape[0]
    p = np.arange(-(n // 2), n - n // 2, dtype=np.float64)
    u = np.asarray(uv[:, 0], dtype=np.float64)
    v = np.asarray(uv[:, 1], dtype=np.float64)
    ex = np.exp(-1j * np.outer(u, p))        # (M, n) over p_x
    ey = np.exp(-1j * np.outer(v, p))        # (M, n) over p_y
    y = np.einsum("ky,yx,kx->k", ey, np.asarray(x, dtype=np.float64), ex)
    if w is not None:
        y = y * np.asarray(w, dtype=np.float64)
    return y
