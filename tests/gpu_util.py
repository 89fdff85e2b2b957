"""Helpers shared by the GPU parity tests: seeded problems, plan order, norms."""
from __future__ import annotations

import math
import sys

import numpy as np
import torch

import workloads as W
from oracle import measurement as ms

DEV = "cuda:0"


def say(msg: str):
    """Name the case before each GPU step (flushed, so a fault still shows it)."""
    print(msg, flush=True)
    sys.stdout.flush()


def purimi():
    from paper_1903_04502_amd import purimi as P
    P.lib()
    return P


def rel_l2(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    den = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / (den if den > 0 else 1.0))


def max_rel(a, b) -> float:
    """Largest element-wise error over the largest reference magnitude."""
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    den = float(np.max(np.abs(b))) if b.size else 0.0
    return float(np.max(np.abs(a - b)) / (den if den > 0 else 1.0)) if b.size else 0.0


def to_dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device=DEV, dtype=dtype)


def problem(n, M, J=4, D=2000, seed=0, prec="f32", weights=False, uv_law="gaussian"):
    """Seeded image, baselines (rounded to the storage precision) and weights."""
    rng = np.random.default_rng(seed)
    x = W.gaussian_sky(n, W.n_sources_for(n), rng)
    dt = np.float32 if prec == "f32" else np.float64
    uv = (W.uv_ring_core(M, rng, dtype=dt) if uv_law == "ringcore" else W.uv_gaussian(M, rng, dtype=dt))
    w = rng.uniform(0.5, 1.5, M).astype(dt) if weights else None
    spec = ms.PhiSpec(n, 2 * n, J, D)
    return x, uv, w, spec


def make_plan(P, n, uv, w, J, D, prec="f32", tile=0, interp=0):
    rdt = torch.float32 if prec == "f32" else torch.float64
    uv_d = to_dev(uv, rdt)
    w_d = None if w is None else to_dev(w, rdt)
    plan = P.PhiPlan(n, uv_d, w_d, J=J, D=D, tile=tile, prec=P.PR_F32 if prec == "f32" else P.PR_F64, interp=interp)
    perm = plan.perm().cpu().numpy() if uv.shape[0] else np.zeros(0, dtype=np.int64)
    return plan, perm


def cell_keys(uv, spec, T):
    """Tile-major base-cell key of each visibility from the oracle's tap rule."""
    K, J, D = spec.K, spec.J, spec.D
    ju, _ = ms.taps_1d(uv[:, 0], K, J, D)
    jv, _ = ms.taps_1d(uv[:, 1], K, J, D)
    bu, bv = np.mod(ju, K), np.mod(jv, K)
    nT = K // T
    tile = (bv // T) * nT + bu // T
    return tile * T * T + (bv % T) * T + bu % T
