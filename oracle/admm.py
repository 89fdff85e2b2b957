"""Dual Forward-Backward ADMM (oracle, FP64).

Test infrastructure only (see the package header).

Method (Section "Sparse Regularization using Dual Forward-Backward ADMM",
Algorithm 1): the constrained analysis problem (eq. global-min-problem-admm)
    min_x  ||Psi^dagger x||_1 + iota_C(x) + iota_B(Phi x),
    C = R_+^N,  B = {z : ||z - y||_2 <= epsilon},
takes a slack r = Phi x with multiplier s, and ADMM alternates the two
subproblems of its Lagrangian:
  * r-subproblem (eq. admm-basic-min-steps-r): the prox of iota_B at Phi x + s,
    i.e. the projection onto the ball (eq. l2ball_prox);
  * the multiplier moves by the constraint residual Phi x - r, scaled by varrho;
  * x-subproblem (eq. admm-basic-min-steps-x): not solved exactly but by one
    forward-backward step: a gradient step of size rho on the quadratic
    coupling term (gradient Re Phi^dagger (Phi x - r + s), taken with the
    updated multiplier), then the prox of gamma ||Psi^dagger .||_1 + iota_C;
  * that prox has no closed form for a non-orthogonal Psi; it is computed by
    forward-backward on its dual: Moreau's decomposition (eq.
    Moreau_decomposition) turns the prox of the l1 term into a projection of
    the dual variable onto the l_inf ball of radius gamma, the clip operator
    I - S_gamma of the soft threshold, and the positivity projection acts on
    the primal estimate; the dual variable is carried from one outer
    iteration to the next.

Local variant (Section "Local Fidelity Constraint ADMM", eq. proj-L2-local):
B is the product of per-section balls, so the r-subproblem projects each
section of visibilities onto its own ball.

Readings: the primal estimate of the dual forward-backward subtracts Psi d
from the fixed input of the prox (as the distributed Algorithms 2 and 3
write it); x, s and d start at 0; the objective written for the distributed
prox is read as the prox of gamma (||Psi^dagger .||_1 + iota_R+).
Diagnostics follow Section "Distributed Convergence".

Parity: an iteration, so no closed form in general ("parity unpinned" for the
full SARA problem beyond its parts); special cases are pinned in
tests/test_oracle_admm.py (Phi = I with a Dirac dictionary has the closed-form
solution max(y - tau, 0); a single orthonormal basis reduces the prox to
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
    """prox of f = gamma ||Psi^dagger .||_1 (+ iota_C) at z by dual forward-backward.

    The dual variable d (coefficient-shaped, warm start given) takes
    forward-backward steps of size eta on the dual problem: a gradient step
    along Psi^dagger of the current primal estimate, then the projection onto
    the l_inf ball of radius gamma (clip_magnitude = I - S_gamma, from Moreau's
    identity). The primal estimate is the projection of z - Psi d onto C.
    ``positivity=False`` drops P_C (a pin uses it); ``weights`` (coefficient-
    shaped) give the weighted norm sum_i w_i |[Psi^dagger x]_i|, radius gamma w_i.
    Returns (primal estimate, dual variable)."""
    proj = proj_positive if positivity else (lambda v: np.real(v))
    thr = gamma if weights is None else gamma * np.asarray(weights, dtype=np.float64)
    primal = proj(z)
    for _ in range(inner_iters):
        d = (1.0 / eta) * clip_magnitude(eta * d + psi_adj(primal), thr)
        primal = proj(z - psi(d))
    return primal, d


def _data_prox(u, y, eps, sections):
    """r-subproblem: the prox of iota_B at u, the projection onto the data ball
    (one global ball, or one ball per section)."""
    return proj_l2ball(u, y, eps) if sections is None else proj_l2balls_local(u, y, eps, sections)


def admm(y, phi, phi_adj, psi, psi_adj, eps, p: AdmmParams, x0, d0=None, sections=None, weights=None):
    """Run ``p.iters`` outer iterations; returns (x, s, d, report).

    phi / phi_adj are the (normalised) measurement operator and its real-image
    adjoint; psi / psi_adj the dictionary synthesis and analysis. With
    ``sections`` (the section of each visibility) ``eps`` holds one radius per
    section (Section "Local Fidelity Constraint ADMM"); otherwise one global
    ball.
    """
    x = np.array(x0, dtype=np.float64, copy=True)
    y = np.asarray(y, dtype=np.complex128)
    s = np.zeros_like(y)                      # multiplier of the slack r = Phi x
    d = np.zeros_like(psi_adj(x)) if d0 is None else np.array(d0, dtype=np.float64)
    rep = AdmmReport()
    for _ in range(p.iters):
        phix = phi(x)
        r = _data_prox(phix + s, y, eps, sections)
        residual = phix - r                   # constraint residual Phi x - r
        s = s + p.varrho * residual
        grad = phi_adj(residual + s)          # coupling-term gradient with the updated multiplier
        x_new, d = dual_fb(x - p.rho * grad, d, p.gamma, p.eta, psi, psi_adj, p.inner_iters, weights=weights)
        nx = float(np.sqrt(np.sum(x_new * x_new)))
        rep.rel_var.append(l2_distance(x_new, x) / nx if nx > 0 else math.inf)
        rep.resid.append(l2_distance(phix, y))
        rep.l1.append(float(np.sum(np.abs(psi_adj(x_new)))))
        x = x_new
    return x, s, d, rep


def default_gamma(y, phi_adj, psi_adj, factor: float = 1e-3) -> float:
    """gamma = factor * max |Psi^dagger Phi^dagger y|."""
    return factor * float(np.max(np.abs(psi_adj(phi_adj(y)))))
