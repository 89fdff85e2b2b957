#!/usr/bin/env python3
"""Throughput of the ADMM imaging path on one MI355X.

Workload (default): 256 x 256 image, 512 x 512 grid, M = 1e6 visibilities
(Gaussian baselines, sigma = pi/3, inside [-pi, pi)), Kaiser-Bessel J = 4 at
D = 2000 samples per cell, SARA (Dirac + db1..db8) at 4 levels, 30 dB noise,
all seeded and synthetic. Inputs are resident in HBM before timing starts.

Timed, after W warm-up passes, on torch's current stream with HIP events:
  * K pairs (Phi, Phi^dagger), each stage bracketed by events:
    value = M / (t_Phi + t_Phi^dagger) in visibilities/s (FP32);
  * K ADMM iterations (Algorithm 1, one DualFB iteration each) in one
    solve call: ms_per_step = its time / K (FP32);
  * the same two figures in FP64 (reported beside, not as `value`).
`roofline` is the degridding kernel (one launch per Phi): 20 algorithmic
bytes per visibility (u, v, w, y in FP32) over its event-timed duration,
against the 8 TB/s HBM peak. `cpu_baseline` times the FP64 oracle's Phi and
Phi^dagger on the same full input on this host.

Prints ONE JSON line. `--gpus` above 1 is not supported (one GPU per box).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("Φ+Φ† visibilities/s and ADMM iter time, FP32 vs FP64; "
          "solves/s + p99 latency")
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c1", choices=["c1", "c1j6"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import workloads as W
    from paper_1903_04502_amd import purimi as P

    P.lib()
    assert torch.cuda.is_available(), "bench needs a GPU"
    dev = torch.device("cuda:0")
    wl = W.CONFIGS[args.workload]
    n, M, J, D, L = wl.n, wl.M, wl.J, wl.D, wl.levels
    rng = W.rng_for(wl.index)
    log(f"workload {wl.name}: generating inputs")
    x_true = W.make_sky(wl, rng)
    uv32 = W.make_uv(wl, rng)
    noise = W.unit_complex_noise(M, rng)
    K_steps, W_steps = args.steps, args.warmup
    out = {}

    def run_prec(prec):
        rdt = torch.float32 if prec == P.PR_F32 else torch.float64
        uv = torch.as_tensor(uv32.astype(np.float64) if prec == P.PR_F64 else uv32).to(dev)
        plan = P.PhiPlan(n, uv, None, J=J, D=D, prec=prec)
        psi = P.PsiPlan(n, L, 0x1FF, prec, dev)
        perm = plan.perm()
        x = torch.as_tensor(x_true).to(dev, rdt)
        y0 = plan.apply(x)
        # noisy data at 30 dB in plan order (noise draws are indexed by user order)
        y0_user = torch.empty_like(y0)
        y0_user[perm] = y0
        y_user, sigma, eps = W.add_noise(y0_user.cpu().numpy().astype(np.complex128), noise, wl.snr_db)
        y = torch.as_tensor(y_user).to(dev, plan.cdtype)[perm].contiguous()
        op_norm = plan.norm(100)
        dirty = plan.adjoint(y) / op_norm
        gamma = 1e-3 * float(psi.adjoint(dirty).abs().max().item())
        xg = torch.empty((n, n), dtype=rdt, device=dev)
        yv = torch.empty_like(y)
        stream = torch.cuda.current_stream(dev)
        h = plan.handle
        # ---- Phi, Phi^dagger pairs
        for _ in range(W_steps):
            P.pr_phi_apply(h, x, yv)
            P.pr_phi_adjoint(h, y, xg)
        torch.cuda.synchronize()
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(K_steps)]
        for k in range(K_steps):
            e = ev[k]
            e[0].record(stream)
            P.pr_phi_fzs(h, x)
            e[1].record(stream)
            P.pr_phi_gw(h, yv)
            e[2].record(stream)
            P.pr_phi_gw_adjoint(h, y)
            e[3].record(stream)
            P.pr_phi_fzs_adjoint(h, xg)
            e[4].record(stream)
        torch.cuda.synchronize()
        t = np.array([[ev[k][i].elapsed_time(ev[k][i + 1]) for i in range(4)] for k in range(K_steps)])
        t_fzs, t_gw, t_gwa, t_fzsa = t.mean(axis=0)
        t_phi, t_adj = t_fzs + t_gw, t_gwa + t_fzsa
        # ---- ADMM iterations
        prm = P.admm_params(eps, gamma, iters=W_steps, op_norm=op_norm)
        ws = torch.empty(P.pr_admm_workspace_size(h, psi.handle), dtype=torch.uint8, device=dev)
        xa = torch.zeros((n, n), dtype=rdt, device=dev)
        P.pr_admm_solve(h, psi.handle, y, prm, xa, ws, want_report=False)
        torch.cuda.synchronize()
        prm = P.admm_params(eps, gamma, iters=K_steps, op_norm=op_norm)
        xa.zero_()
        torch.cuda.synchronize()
        a0, a1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a0.record(stream)
        P.pr_admm_solve(h, psi.handle, y, prm, xa, ws, want_report=False)
        a1.record(stream)
        torch.cuda.synchronize()
        t_admm = a0.elapsed_time(a1) / K_steps
        rep = P.pr_admm_solve(h, psi.handle, y, P.admm_params(eps, gamma, iters=K_steps, op_norm=op_norm),
                              torch.zeros((n, n), dtype=rdt, device=dev), ws, want_report=True)
        return dict(t_fzs=t_fzs, t_gw=t_gw, t_gwa=t_gwa, t_fzsa=t_fzsa, t_phi=t_phi, t_adj=t_adj,
                    t_admm=t_admm, items=plan.items, tile=plan.desc.tile, op_norm=op_norm, gamma=gamma,
                    eps=eps, resid=rep.resid_norm, nonfinite=rep.nonfinite, y_plan=yv, perm=perm,
                    plan=plan, x=x)

    log("FP32 runs")
    r32 = run_prec(P.PR_F32)
    log(f"FP32: phi {r32['t_phi']:.3f} ms, adj {r32['t_adj']:.3f} ms, admm {r32['t_admm']:.3f} ms")
    r64 = None
    if not args.no_fp64:
        log("FP64 runs")
        r64 = run_prec(P.PR_F64)
        log(f"FP64: phi {r64['t_phi']:.3f} ms, adj {r64['t_adj']:.3f} ms, admm {r64['t_admm']:.3f} ms")

    value = M / ((r32["t_phi"] + r32["t_adj"]) * 1e-3)
    deg_bytes = 20.0 * M
    achieved = deg_bytes / (r32["t_gw"] * 1e-3) / 1e9
    res = {
        "metric": METRIC,
        "value": value,
        "unit": "visibilities/s",
        "n_gpus": 1,
        "steps": K_steps,
        "warmup": W_steps,
        "ms_per_step": r32["t_admm"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded sky of Gaussian sources, Gaussian baselines, 30 dB noise)",
        "config": {"workload": wl.name, "image": n, "grid": 2 * n, "visibilities": M, "J": J,
                   "table_samples_per_cell": D, "sara_levels": L, "dualfb_iters": 1,
                   "step": "one ADMM iteration (ms_per_step); value from (Phi, Phi^dagger) pairs"},
        "phi_ms": r32["t_phi"], "phi_adjoint_ms": r32["t_adj"],
        "stage_ms": {"fzs": r32["t_fzs"], "gw": r32["t_gw"], "gw_adjoint": r32["t_gwa"],
                     "fzs_adjoint": r32["t_fzsa"]},
        "admm_iter_ms_fp32": r32["t_admm"],
        "roofline": {"bound": "hbm", "kernel": "degrid_kernel (pr_phi_gw)", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None, "algorithmic_bytes_per_launch": deg_bytes},
        "work_items": r32["items"],
    }
    if r64 is not None:
        res["fp64"] = {"value": M / ((r64["t_phi"] + r64["t_adj"]) * 1e-3), "phi_ms": r64["t_phi"],
                       "phi_adjoint_ms": r64["t_adj"], "admm_iter_ms": r64["t_admm"],
                       "stage_ms": {"fzs": r64["t_fzs"], "gw": r64["t_gw"], "gw_adjoint": r64["t_gwa"],
                                    "fzs_adjoint": r64["t_fzsa"]}}
    if not args.no_cpu_baseline:
        log("CPU baseline: oracle Phi and Phi^dagger on the full input")
        from oracle import measurement as ms
        spec = ms.PhiSpec(n, 2 * n, J, D)
        uv64 = uv32.astype(np.float64)
        t0 = time.perf_counter()
        y_ref = ms.phi(x_true, uv64, None, spec)
        t1 = time.perf_counter()
        ms.phi_adjoint(y_ref, uv64, None, spec)
        t2 = time.perf_counter()
        res["cpu_baseline"] = {"value": M / (t2 - t0), "unit": "visibilities/s", "cores": 1, "kind": "oracle",
                               "sample": f"one Phi ({t1 - t0:.1f} s) and one Phi^dagger ({t2 - t1:.1f} s) of the "
                                         f"FP64 NumPy oracle on the full {M}-visibility input (single thread)",
                               "host_cpus": os.cpu_count()}
        perm = r32["perm"].cpu().numpy()
        y32 = r32["y_plan"].cpu().numpy().astype(np.complex128)
        # the last Phi of the timed loop was applied to the sky: compare in plan order
        err = float(np.linalg.norm(y32 - y_ref[perm]) / np.linalg.norm(y_ref))
        res["phi_rel_err_fp32_vs_oracle"] = err
        if r64 is not None:
            y64 = r64["y_plan"].cpu().numpy()
            perm64 = r64["perm"].cpu().numpy()
            res["fp64"]["phi_rel_err_vs_oracle"] = float(np.linalg.norm(y64 - y_ref[perm64]) / np.linalg.norm(y_ref))
    print(json.dumps(res))


if __name__ == "__main__":
    main()
