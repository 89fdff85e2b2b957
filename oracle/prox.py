"""Closed-form proximal operators (oracle, FP64).

Test infrastructure only (see the package header).

Paper passages (Section "Proximal Operators"): the projection onto a closed
convex set is the proximal operator of its indicator function (subsection
"Indicator Function"); the l2 ball centred at z of radius epsilon projects
x to x if ||x - z|| <= epsilon and to z + epsilon (x - z)/||x - z|| otherwise
(subsection "Fidelity Constraint", eq. l2ball_prox); the prox of the l1 norm is
soft thresholding, S_lambda(x_i) = 0 for |x_i| <= lambda and
x_i (|x_i| - lambda)/|x_i| otherwise (subsection "Promoting Sparsity").

Readings: ties |x_i| = lambda give 0 and ||x - z|| = epsilon leaves x
unchanged (the ball is closed); C = R_+^N projects by max(Re x, 0); norms in FP64.

Pins (tests/test_oracle_prox.py): brute-force minimisation of the proximal
objective on small grids, and the Moreau identity for the l1 case.
"""
from __future__ import annotations

import numpy as np


def soft_threshold(x, lam: float):
    x = np.asarray(x)
    mag = np.abs(x)
    keep = mag > lam
    safe = np.where(keep, mag, 1.0)
    return np.where(keep, x * ((mag - lam) / safe), 0.0 * x)


def clip_magnitude(x, lam: float):
    """(I - S_lambda)(x): the part soft thresholding removes."""
    return np.asarray(x) - soft_threshold(x, lam)


def proj_positive(x):
    return np.maximum(np.real(np.asarray(x)), 0.0)


def l2_distance(x, z) -> float:
    d = np.asarray(x) - np.asarray(z)
    return float(np.sqrt(np.sum(np.abs(d) ** 2)))


def proj_l2ball(x, z, eps: float):
    x = np.asarray(x)
    z = np.asarray(z)
    dist = l2_distance(x, z)
    if dist <= eps:
        return x.copy()
    return z + (eps / dist) * (x - z)


def proj_l2balls_local(x, z, eps_j, sections):
    """Independent projections onto the balls ||x_j - z_j|| <= eps_j of the
    sections j (eq. proj-L2-local, Section "Local Fidelity Constraint ADMM");
    ``sections[k]`` is the section of element k."""
    x = np.asarray(x)
    z = np.asarray(z)
    sections = np.asarray(sections)
    out = x.copy()
    for j, e in enumerate(np.asarray(eps_j, dtype=np.float64)):
        idx = np.nonzero(sections == j)[0]
        if idx.size:
            out[idx] = proj_l2ball(x[idx], z[idx], float(e))
    return out
