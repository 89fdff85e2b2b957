"""FISTA for the unconstrained (MAP) imaging problem (oracle, FP64).

Test infrastructure only (see the package header).

Paper passages: the MAP estimate of Section "Sparse Regularization" (gamma g
plus the data misfit), the Forward-Backward step of Section "Forward-Backward
Splitting" and Algorithm "FISTA":
  x_{k+1} = prox_{lambda gamma g}(xh_k - lambda grad f(xh_k)),
  theta_{k+1} = (1 + sqrt(1 + 4 theta_k^2)) / 2,
  xh_{k+1} = x_{k+1} + (theta_k - 1) / theta_{k+1} (x_{k+1} - x_k),
starting from x_0 = xh_0, theta_0 = 1.

Readings: the misfit is f(x) = 1/2 ||y - Phi x||^2 (the square and the 1/2 fix
the gradient grad f(x) = Re Phi^dagger (Phi x - y), whose Lipschitz constant is
||Phi||^2 = 1 for the normalised operator); g = ||Psi^dagger .||_1 + iota_R+
as in the constrained problem; the prox of lambda gamma g is approximated by
the DualFB iterations of Algorithm 1 with the dual variable d carried over
between outer iterations, as the paper does for the same prox.

Parity: an iteration; pinned in tests/test_oracle_fista.py by closed forms
(Phi = I with a Dirac dictionary converges to max(y - gamma, 0)) and by
brute-force minimisation of the objective on tiny problems.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .admm import dual_fb


@dataclass
class FistaReport:
    resid: list = field(default_factory=list)      # ||Phi xh_k - y|| at each gradient
    l1: list = field(default_factory=list)         # ||Psi^dagger x_{k+1}||_1


def objective(x, y, phi, psi_adj, gamma: float) -> float:
    r = phi(x) - y
    return gamma * float(np.sum(np.abs(psi_adj(x)))) + 0.5 * float(np.vdot(r, r).real)


def fista(y, phi, phi_adj, psi, psi_adj, gamma: float, lam: float, iters: int, x0,
          inner_iters: int = 1, eta: float = 1.0, positivity: bool = True):
    """Run ``iters`` FISTA iterations; returns (x, d, report)."""
    x = np.array(x0, dtype=np.float64, copy=True)
    xh = x.copy()
    y = np.asarray(y, dtype=np.complex128)
    d = np.zeros_like(psi_adj(x))
    theta = 1.0
    rep = FistaReport()
    for _ in range(iters):
        r = phi(xh) - y
        z = xh - lam * phi_adj(r)
        x_new, d = dual_fb(z, d, gamma * lam, eta, psi, psi_adj, inner_iters, positivity)
        theta_new = (1.0 + math.sqrt(1.0 + 4.0 * theta * theta)) / 2.0
        xh = x_new + ((theta - 1.0) / theta_new) * (x_new - x)
        rep.resid.append(float(np.sqrt(np.vdot(r, r).real)))
        rep.l1.append(float(np.sum(np.abs(psi_adj(x_new)))))
        x, theta = x_new, theta_new
    return x, d, rep
