"""Primal-Dual splitting (oracle, FP64).

Test infrastructure only (see the package header).

Paper passage: Section "Primal-Dual Splitting" and Algorithm "Primal-Dual
Algorithm" for min_x f(L x) + g(x), written as a saddle-point problem:
  z_{k+1} = prox_{sigma f*}(z_k + sigma L xh_k),
  x_{k+1} = prox_{tau g}(x_k - tau L^dagger z_{k+1}),
  xh_{k+1} = x_{k+1} + theta (x_{k+1} - x_k),
with prox_{sigma f*} obtained from prox of f by Moreau's decomposition as the
section states: prox_{sigma f*}(u) = u - sigma prox_{f / sigma}(u / sigma).

Readings: L = Phi (normalised); g = gamma ||Psi^dagger .||_1 + iota_R+, whose
prox with weight tau is the DualFB of Algorithm 1 with threshold tau gamma
and the dual variable d carried between iterations (as for the other
solvers); two choices of f:
  "ball": f = iota of {v : ||v - y|| <= epsilon} (the constrained problem,
          prox_{f / sigma} = P_B for any sigma),
  "l2":   f = 1/2 ||v - y||^2 (the MAP problem,
          prox_{f / sigma}(w) = (y + sigma w) / (1 + sigma)).
x_0 = xh_0 given, z_0 = 0, d_0 = 0.

Parity: an iteration; pinned in tests/test_oracle_primal_dual.py by closed
forms (Phi = I, Dirac dictionary, both misfits), brute-force minimisation of
the MAP objective, the direct prox of the conjugates by numerical
minimisation (the Moreau step) and the optimality condition of the saddle
point.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .admm import dual_fb
from .prox import proj_l2ball


@dataclass
class PdReport:
    resid: list = field(default_factory=list)      # ||L xh_k - y||
    l1: list = field(default_factory=list)         # ||Psi^dagger x_{k+1}||_1
    rel_var: list = field(default_factory=list)    # ||x_{k+1} - x_k|| / ||x_{k+1}||


def prox_f(w, y, sigma_inv: float, misfit: str, eps: float = 0.0):
    """prox of (sigma_inv * f) at w for the two misfits."""
    if misfit == "ball":
        return proj_l2ball(w, y, eps)
    if misfit == "l2":
        # argmin_v sigma_inv/2 ||v - y||^2 + 1/2 ||v - w||^2
        return (sigma_inv * y + w) / (sigma_inv + 1.0)
    raise ValueError(misfit)


def prox_conjugate(u, y, sigma: float, misfit: str, eps: float = 0.0):
    """prox_{sigma f*}(u) by Moreau's decomposition."""
    return u - sigma * prox_f(u / sigma, y, 1.0 / sigma, misfit, eps)


def primal_dual(y, phi, phi_adj, psi, psi_adj, gamma: float, tau: float, sigma: float, theta: float,
                iters: int, x0, misfit: str = "ball", eps: float = 0.0, inner_iters: int = 1,
                eta: float = 1.0, positivity: bool = True):
    """Run ``iters`` iterations; returns (x, z, d, report)."""
    x = np.array(x0, dtype=np.float64, copy=True)
    xh = x.copy()
    y = np.asarray(y, dtype=np.complex128)
    z = np.zeros_like(y)
    d = np.zeros_like(psi_adj(x))
    rep = PdReport()
    for _ in range(iters):
        v = phi(xh)
        z = prox_conjugate(z + sigma * v, y, sigma, misfit, eps)
        x_new, d = dual_fb(x - tau * phi_adj(z), d, tau * gamma, eta, psi, psi_adj, inner_iters, positivity)
        xh = x_new + theta * (x_new - x)
        nx = float(np.linalg.norm(x_new))
        rep.resid.append(float(np.linalg.norm(v - y)))
        rep.l1.append(float(np.sum(np.abs(psi_adj(x_new)))))
        rep.rel_var.append(float(np.linalg.norm(x_new - x)) / nx if nx > 0 else float("inf"))
        x = x_new
    return x, z, d, rep
