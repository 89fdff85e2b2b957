"""Dual Forward-Backward ADMM (oracle, FP64).

Test infrastructure only (see the package header).

Paper passage: Algorithm 1 (Section "Sparse Regularization using Dual
Forward-Backward ADMM") for the constrained analysis problem
min ||Psi^dagger x||_1 + iota_C(x) + iota_B(Phi x), C = R_+^N,
B = {z : ||z - y|| <= epsilon}. One outer iteration:
  v = Phi x; r = P_B(v + s); s <- s + varrho (v - r);
  xt = x - rho Phi^dagger (v - r + s)    (uses the updated s);
  x = DualFB(xt, gamma).
DualFB starts from zbar = P_C(z) and repeats
  d <- (1/eta) (I - S_gamma)(eta d + Psi^dagger zbar); zbar = P_C(z - Psi d),
returning zbar. d is carried over between outer iterations (warm start).

Local variant (Section "Local Fidelity Constraint ADMM", eq. proj-L2-local):
the visibilities are split into sections y_j with radii epsilon_j and the r
step projects each section onto its own ball; the rest is unchanged.

Readings: the DualFB update of zbar subtracts Psi d from the fixed input z
(the distributed versions, Algorithms 2 and 3, write plain z there); initial
x = 0, s = 0, d = 0; the objective line of the distributed prox section is
read as prox of gamma (||Psi^dagger .||_1 + iota_R+). Diagnostics follow the
convergence criteria of Section "Distributed Convergence".

Parity: an iteration, so no closed form in general ("parity unpinned" for the
full SARA problem beyond its parts); special cases are pinned in
tests/test_oracle_admm.py (Phi = I with a Dirac dictionary has the closed-form
solution max(y - tau, 0); a single orthonormal basis reduces DualFB to
W^T S_gamma W).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .prox import clip_magnitude, proj_l2ball, proj_l2balls_local, proj_positive, l2_distance


@dataclass
class AdmmParams:
    gamma: float
    iters: int = 50
    inner_iters: int = 1
    rho: float = 0.5
    varrho: float = 1.0
    eta: float = 1.0


@dataclass
class AdmmReport:
    rel_var: list = field(default_factory=list)
    resid: list = field(default_factory=list)
    l1: list = field(default_factory=list)


def dual_fb(z, d, gamma: float, eta: float, psi, psi_adj, inner_iters: int,
            positivity: bool = True, weights=None):
    """DualFB of Algorithm 1; ``positivity=False`` drops P_C (used by a pin only).
    ``weights`` (coefficient-shaped) turn the l1 norm into the weighted
    sum_i w_i |[Psi^dagger x]_i|: the threshold of coefficient i is gamma w_i."""
    proj = proj_positive if positivity else (lambda v: np.real(v))
    thr = gamma if weights is None else gamma * np.asarray(weights, dtype=np.float64)
    zbar = proj(z)
    for _ in range(inner_iters):
        d = (1.0 / eta) * clip_magnitude(eta * d + psi_adj(zbar), thr)
        zbar = proj(z - psi(d))
    return zbar, d


def admm(y, phi, phi_adj, psi, psi_adj, eps, p: AdmmParams, x0, d0=None, sections=None, weights=None):
    """Run ``p.iters`` outer iterations; returns (x, s, d, report).

    phi / phi_adj are the (normalised) measurement operator and its real-image
    adjoint; psi / psi_adj the dictionary synthesis and analysis. With
    ``sections`` (the section of each visibility) ``eps`` holds one radius per
    section and r is the independent projection onto each section's ball
    (Section "Local Fidelity Constraint ADMM"); otherwise one global ball.
    """
    x = np.array(x0, dtype=np.float64, copy=True)
    y = np.asarray(y, dtype=np.complex128)
    s = np.zeros_like(y)
    d = np.zeros_like(psi_adj(x)) if d0 is None else np.array(d0, dtype=np.float64)
    rep = AdmmReport()
    for _ in range(p.iters):
        v = phi(x)
        r = proj_l2ball(v + s, y, eps) if sections is None else proj_l2balls_local(v + s, y, eps, sections)
        s = s + p.varrho * (v - r)
        xt = x - p.rho * phi_adj(v - r + s)
        x_new, d = dual_fb(xt, d, p.gamma, p.eta, psi, psi_adj, p.inner_iters, weights=weights)
        nx = float(np.sqrt(np.sum(x_new * x_new)))
        rep.rel_var.append(l2_distance(x_new, x) / nx if nx > 0 else math.inf)
        rep.resid.append(l2_distance(v, y))
        rep.l1.append(float(np.sum(np.abs(psi_adj(x_new)))))
        x = x_new
    return x, s, d, rep


def default_gamma(y, phi_adj, psi_adj, factor: float = 1e-3) -> float:
    """gamma = factor * max |Psi^dagger Phi^dagger y|."""
    return factor * float(np.max(np.abs(psi_adj(phi_adj(y)))))
