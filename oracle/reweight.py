"""Reweighted analysis l1 (SARA reweighting) around Algorithm 1 (oracle, FP64).

Test infrastructure only (see the package header).

Paper passage: Section "Sparse Regularization" states that the analysis
problem with the over-complete SARA frame is solved several times, the l1
norm being reweighted between solves. The paper gives no weight rule.

Readings: the weighted problem replaces ||Psi^dagger x||_1 by
sum_i w_i |[Psi^dagger x]_i| (the DualFB threshold of coefficient i becomes
gamma w_i); the weights after a solve are w_i = delta / (delta + |[Psi^dagger x]_i|)
with delta = delta0 beta^(r-1) for the r-th reweighting (the usual
log-penalty majorisation); round 0 is unweighted; every round restarts
Algorithm 1 from the previous x with s = 0 and d = 0.

Parity: an iteration; pinned in tests/test_oracle_reweight.py by closed forms
(Phi = I with a Dirac dictionary: every round is max(y - tau w, 0) on the
ball) and by unit weights reproducing the unweighted solver.
"""
from __future__ import annotations

import numpy as np

from .admm import AdmmParams, admm


def weights_from(alpha, delta: float):
    """w_i = delta / (delta + |alpha_i|)."""
    return delta / (delta + np.abs(np.asarray(alpha, dtype=np.float64)))


def sara_reweighted(y, phi, phi_adj, psi, psi_adj, eps, p: AdmmParams, rounds: int, delta0: float, beta: float,
                    x0):
    """Round 0 unweighted, then ``rounds`` reweighted solves; returns (x, weights, reports)."""
    x, _, _, rep = admm(y, phi, phi_adj, psi, psi_adj, eps, p, x0)
    reps = [rep]
    w = None
    delta = delta0
    for _ in range(rounds):
        w = weights_from(psi_adj(x), delta)
        x, _, _, rep = admm(y, phi, phi_adj, psi, psi_adj, eps, p, x, weights=w)
        reps.append(rep)
        delta *= beta
    return x, w, reps
