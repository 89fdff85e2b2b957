#!/usr/bin/env python3
"""Throughput of the ADMM imaging path on one MI355X.

Workload of `value` (default): 256 x 256 image, 512 x 512 grid, M = 1e6
visibilities (Gaussian baselines, sigma = pi/3, inside [-pi, pi)),
Kaiser-Bessel J = 4 at D = 2000 samples per cell, SARA (Dirac + db1..db8) at
4 levels, 30 dB noise, all seeded and synthetic. Inputs are resident in HBM
before timing starts.

Timed, after W warm-up passes, on torch's current stream with HIP events:
  * K pairs (Phi, Phi^dagger) between two events: value = M / t_pair in
    visibilities/s (FP32); then K more pairs with every launch bracketed by
    events for the per-stage times and the roofline kernel's duration;
  * K ADMM iterations (Algorithm 1, one DualFB iteration each) in one
    solve call: ms_per_step = its time / K (FP32);
  * the same two figures in FP64 (reported beside, not as `value`);
  * `batch`: 64 channels (n in {128..1024}, M log-uniform in [1e4, 5e6],
    all planned with one tile: of the tiles the per-channel autotuner chose,
    the one whose fused pair is faster) as one batch: batched (Phi,
    Phi^dagger) per member and fused, graph-replayed ADMM steps, errors
    against the FP64 operator and the oracle;
  * `serving`: Poisson arrivals (20 req/s) of 30-iteration solves drawn from
    the channel law plus 5% 2048^2 / 5e7-visibility jobs through the
    continuous-batching server, FP32 and FP64: solves/s, p50/p99 latency and
    the final image error against the true sky.
  * `large_workload`: the 2048^2 image / 4096^2 grid / 5e8 ring-plus-core
    visibility workload (FP32, 5 timed steps) run by this script in a child
    process (`--workload share2048`), its pair rate, stage times, solver iteration
    times and roofline; `--no-large` skips it.
`roofline` is the slower of the two single-launch visibility kernels
(gridding patches or degridding): 20 algorithmic bytes per visibility (u, v,
w, y in FP32) over its event-timed duration, against the 8 TB/s HBM peak;
`traffic` comes from the committed rocprofv3 counter summary while the
kernel source is unchanged. `cpu_baseline` times the FP64 oracle's Phi and
Phi^dagger on the same full input on this host.

Prints ONE JSON line. `--gpus` above 1 is not supported (one GPU per box).
"""
from __future__ import annotations

import argparse
import hashlib
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


def kernel_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or None.

    The summary profiles/<kernel>_<workload>_pmc.md records FETCH_SIZE and
    WRITE_SIZE scaled by a copy-kernel calibration and the sha256 of the
    kernel's source file; a changed source makes the figure stale (None).
    """
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_pmc.md")
    src = os.path.join(ROOT, "paper_1903_04502_amd", "csrc", "gridding.hip")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        line = line.strip().lstrip("-* ").strip()
        if ":" in line:
            k, v = line.split(":", 1)
            fields[k.strip().strip("`")] = v.strip().strip("`")
    try:
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
        if fields.get("source_sha256") != digest:
            return None
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError, OSError):
        return None


def copy_bandwidth(dev, nbytes=1 << 31, reps=5):
    """Device-to-device copy rate (read + write bytes / time), the practical
    HBM ceiling the visibility kernels are also compared against."""
    import torch
    src = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / reps * 1e-3
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * nbytes / t / 1e9


def side_pair_ms(P, plan, x, y, xg, K_steps, windows=3):
    """ms per (Phi, Phi^dagger) pair of a side configuration: the median of a
    few windows of K pairs, each between two events (one host stall inside a
    single window would otherwise decide the figure)."""
    import torch
    ts = []
    for _ in range(windows):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(K_steps):
            P.pr_phi_apply(plan.handle, x, y)
            P.pr_phi_adjoint(plan.handle, y, xg)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1) / K_steps)
    return float(np.median(ts))


def run_linear(P, dev, n, J, D, uv32, x_true, K_steps, W_steps, with_oracle):
    """The same workload with first-order (linear) kernel lookup, FP32."""
    import torch
    plan = P.PhiPlan(n, torch.as_tensor(uv32).to(dev), None, J=J, D=D, interp=1)
    x = torch.as_tensor(x_true, dtype=torch.float32, device=dev)
    y = torch.empty(plan.M, dtype=torch.complex64, device=dev)
    xg = torch.empty_like(x)
    for _ in range(W_steps):
        P.pr_phi_apply(plan.handle, x, y)
        P.pr_phi_adjoint(plan.handle, y, xg)
    torch.cuda.synchronize()
    t = side_pair_ms(P, plan, x, y, xg, K_steps)
    out = {"interp": "linear (first order)", "phi_pair_ms": t, "vis_per_s": plan.M / (t * 1e-3)}
    if with_oracle:
        from oracle import measurement as ms
        P.pr_phi_apply(plan.handle, x, y)
        y_ref = ms.phi(x_true, uv32.astype(np.float64), None, ms.PhiSpec(n, 2 * n, J, D, "linear"))
        perm = plan.perm().cpu().numpy()
        out["phi_rel_err_vs_oracle"] = float(np.linalg.norm(y.cpu().numpy() - y_ref[perm]) / np.linalg.norm(y_ref))
    return out


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _cpu_gw(task):
    """Worker: the oracle's degridding of one chunk of visibilities."""
    from oracle import measurement as ms
    X, uv, spec = task
    return ms.gw(X, uv, None, spec)


def _cpu_gw_adjoint(task):
    """Worker: the oracle's gridding of one chunk of visibilities (a partial grid)."""
    from oracle import measurement as ms
    y, uv, spec = task
    return ms.gw_adjoint(y, uv, None, spec)


def cpu_pair_parallel(x, uv64, spec, workers):
    """The oracle's Phi and Phi^dagger with the visibility work split into
    `workers` chunks on as many spawned processes (none of them touches the
    GPU): S Z and F and their adjoints once in this process, the degridding and
    gridding of each chunk in a worker, partial grids added in chunk order."""
    import multiprocessing as mp
    from oracle import measurement as ms
    M = uv64.shape[0]
    bounds = np.linspace(0, M, workers + 1).astype(np.int64)
    with mp.get_context("spawn").Pool(workers) as pool:
        pool.map(_cpu_gw, [(np.zeros((spec.K, spec.K), complex), uv64[:8], spec)] * workers)   # start-up
        t0 = time.perf_counter()
        X = ms.szf(x, spec)
        y = np.concatenate(pool.map(_cpu_gw, [(X, uv64[a:b], spec) for a, b in zip(bounds[:-1], bounds[1:])]))
        t1 = time.perf_counter()
        grids = pool.map(_cpu_gw_adjoint, [(y[a:b], uv64[a:b], spec) for a, b in zip(bounds[:-1], bounds[1:])])
        g = grids[0]
        for q in grids[1:]:
            g = g + q
        ms.szf_adjoint(g, spec).real
        t2 = time.perf_counter()
    return {"workers": workers, "phi_s": t1 - t0, "adj_s": t2 - t1, "pair_s": t2 - t0}


def run_j6(P, dev, n, D, L, uv32, x_true, K_steps, W_steps, with_oracle):
    """The same workload with the J = 6 kernel (the wider support the
    benchmark configuration names), FP32: (Phi, Phi^dagger) pairs and one
    ADMM iteration."""
    import torch
    plan = P.PhiPlan(n, torch.as_tensor(uv32).to(dev), None, J=6, D=D)
    psi = P.PsiPlan(n, L, 0x1FF, P.PR_F32, dev)
    x = torch.as_tensor(x_true, dtype=torch.float32, device=dev)
    y = torch.empty(plan.M, dtype=torch.complex64, device=dev)
    xg = torch.empty_like(x)
    for _ in range(W_steps):
        P.pr_phi_apply(plan.handle, x, y)
        P.pr_phi_adjoint(plan.handle, y, xg)
    torch.cuda.synchronize()
    t = side_pair_ms(P, plan, x, y, xg, K_steps)
    op_norm = plan.norm(100)
    gamma = 1e-3 * float(psi.adjoint(plan.adjoint(y) / op_norm).abs().max().item())
    eps = 0.05 * float(torch.linalg.vector_norm(y).item()) / op_norm
    ws = torch.empty(P.pr_admm_workspace_size(plan.handle, psi.handle), dtype=torch.uint8, device=dev)
    xa = torch.zeros_like(x)
    P.pr_admm_solve(plan.handle, psi.handle, y, P.admm_params(eps, gamma, iters=W_steps, op_norm=op_norm), xa, ws,
                    want_report=False)
    xa.zero_()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    P.pr_admm_solve(plan.handle, psi.handle, y, P.admm_params(eps, gamma, iters=K_steps, op_norm=op_norm), xa, ws,
                    want_report=False)
    e1.record()
    torch.cuda.synchronize()
    out = {"workload": "op-256sq-M1e6-J6", "J": 6, "phi_pair_ms": t, "vis_per_s": plan.M / (t * 1e-3),
           "admm_iter_ms_fp32": e0.elapsed_time(e1) / K_steps, "tile": plan.desc.tile}
    if with_oracle:
        from oracle import measurement as ms
        P.pr_phi_apply(plan.handle, x, y)
        y_ref = ms.phi(x_true, uv32.astype(np.float64), None, ms.PhiSpec(n, 2 * n, 6, D))
        perm = plan.perm().cpu().numpy()
        out["phi_rel_err_vs_oracle"] = float(np.linalg.norm(y.cpu().numpy() - y_ref[perm]) / np.linalg.norm(y_ref))
    return out


def run_batch(P, dev, args):
    """64 channels of uneven n and M stepped together. The autotuner measures
    each channel's tile alone; the fused launches need one kernel shape, so
    each tile the autotuner chose is tried for all channels (fused pairs
    timed) and the faster one is used."""
    import torch
    import workloads as W
    rng = W.rng_for(3)
    chans = W.batch_channels(64, rng)
    gen = W.torch_generator(3, dev)
    members, tiles, errs64 = [], {}, []
    t0 = time.perf_counter()
    drawn = []
    for n, M in chans:
        x = W.gaussian_sky(n, W.n_sources_for(n), rng)
        uv = W.uv_gaussian(M, rng)
        T = P.tune_tile(n, torch.as_tensor(uv).to(dev))
        tiles[T] = tiles.get(T, 0) + 1
        drawn.append((x, uv))
    trial = {}
    # the default tile always has the fused launch; a tuned tile whose walk
    # does not fit in LDS (32 at J = 4) is skipped
    for Tc in sorted(set(tiles) | {16}):
        bb = P.Batch(max_members=len(chans), nstreams=4)
        xs_c, ys_c, xo_c = [], [], []
        for (n, M), (x, uv) in zip(chans, drawn):
            pl = P.PhiPlan(n, torch.as_tensor(uv).to(dev), None, J=4, D=2000, tile=Tc)
            ps = P.PsiPlan(n, 3, 0x1FF, P.PR_F32, dev)
            xd = torch.as_tensor(x, dtype=torch.float32, device=dev)
            yd = torch.zeros(M, dtype=torch.complex64, device=dev)
            bb.add(pl, ps, yd, P.admm_params(1.0, 1e-3, iters=1, op_norm=1.0))
            xs_c.append(xd)
            ys_c.append(torch.empty_like(yd))
            xo_c.append(torch.empty_like(xd))
        try:
            bb.fuse(dev)
            for _ in range(3):
                P.pr_batch_phi_apply(bb.handle, xs_c, ys_c)
                P.pr_batch_phi_adjoint(bb.handle, ys_c, xo_c)
        except P.PrError as e:
            if e.code != P.PR_EUNSUPPORTED:
                raise
            del bb, xs_c, ys_c, xo_c
            torch.cuda.empty_cache()
            continue
        torch.cuda.synchronize()
        t0c = time.perf_counter()
        for _ in range(5):
            P.pr_batch_phi_apply(bb.handle, xs_c, ys_c)
            P.pr_batch_phi_adjoint(bb.handle, ys_c, xo_c)
        torch.cuda.synchronize()
        trial[Tc] = (time.perf_counter() - t0c) / 5 * 1e3
        del bb, xs_c, ys_c, xo_c
        torch.cuda.empty_cache()
    T = min(trial, key=trial.get)
    for (n, M), (x, uv) in zip(chans, drawn):
        uv_d = torch.as_tensor(uv).to(dev)
        plan = P.PhiPlan(n, uv_d, None, J=4, D=2000, tile=T)
        psi = P.PsiPlan(n, 3, 0x1FF, P.PR_F32, dev)
        x_d = torch.as_tensor(x, dtype=torch.float32, device=dev)
        y0 = plan.apply(x_d)
        y, _, eps = W.add_noise_torch(y0, W.unit_complex_noise_torch(M, gen, dev))
        # FP32 operator error against the FP64 operator on the same baselines (user order)
        plan64 = P.PhiPlan(n, uv_d.double(), None, J=4, D=2000, prec=P.PR_F64)
        y64 = plan64.apply(x_d.double())
        u32 = torch.empty_like(y0)
        u32[plan.perm()] = y0
        u64 = torch.empty_like(y64)
        u64[plan64.perm()] = y64
        errs64.append(float((u32.to(torch.complex128) - u64).norm() / u64.norm()))
        del plan64, y64, u64
        members.append(dict(n=n, M=M, x=x, uv=uv, x_d=x_d, y=y, eps=eps, plan=plan, psi=psi, y_user=u32))
    t_setup = time.perf_counter() - t0
    # oracle check on the three smallest channels
    from oracle import measurement as ms
    errs_or = []
    for m in sorted(members, key=lambda m: m["M"])[:3]:
        spec = ms.PhiSpec(m["n"], 2 * m["n"], 4, 2000)
        yr = ms.phi(m["x"], m["uv"].astype(np.float64), None, spec)
        errs_or.append(float(np.linalg.norm(m["y_user"].cpu().numpy() - yr) / np.linalg.norm(yr)))
    b = P.Batch(max_members=len(members), nstreams=4)
    for m in members:
        m["slot"] = b.add(m["plan"], m["psi"], m["y"],
                          P.admm_params(m["eps"], 0.0, iters=1, gamma_factor=1e-3, norm_iters=100))
    xs = [m["x_d"] for m in members]
    ys = [torch.empty(m["M"], dtype=torch.complex64, device=dev) for m in members]
    xo = [torch.empty_like(m["x_d"]) for m in members]
    stream = torch.cuda.current_stream(dev)
    K, Wm = args.steps, args.warmup
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def time_pairs():
        for _ in range(Wm):
            P.pr_batch_phi_apply(b.handle, xs, ys)
            P.pr_batch_phi_adjoint(b.handle, ys, xo)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(K):
            P.pr_batch_phi_apply(b.handle, xs, ys)
            P.pr_batch_phi_adjoint(b.handle, ys, xo)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / K

    t_pair_members = time_pairs()          # one launch sequence per member, over the streams
    y_members = [v.clone() for v in ys]
    x_members = [v.clone() for v in xo]
    b.fuse(dev)                            # one launch per stage for all members
    t_pair = time_pairs()
    fused_bitwise = all(torch.equal(a_, c_) for a_, c_ in zip(ys, y_members)) and \
        all(torch.equal(a_, c_) for a_, c_ in zip(xo, x_members))
    out = {}
    for use_graph in (True, False):
        b.step(Wm, use_graph=use_graph)
        torch.cuda.synchronize()
        e0.record(stream)
        b.step(K, use_graph=use_graph)
        e1.record(stream)
        torch.cuda.synchronize()
        out["graph" if use_graph else "streams"] = e0.elapsed_time(e1) / K
    rep = [b.report(m["slot"]) for m in members[:4]]
    sum_m = int(sum(m["M"] for m in members))
    # algorithmic bytes of one batched (Phi, Phi^dagger): 40 B per visibility
    # (u, v, w and y read or written by the degridding and by the gridding) plus
    # the pruned transforms of each channel, 4n^2 + 16nK + 8K^2 each way
    fft_b = sum(2 * (4 * m["n"] ** 2 + 16 * m["n"] * 2 * m["n"] + 8 * (2 * m["n"]) ** 2) for m in members)
    pair_bytes = 40.0 * sum_m + fft_b
    ach = pair_bytes / (t_pair * 1e-3) / 1e9
    return {"workload": "channels-64ch-n128..1024-M1e4..5e6-J4-sara3", "channels": len(members), "visibilities": sum_m,
            "tiles_from_autotuner": {str(k): v for k, v in sorted(tiles.items())}, "tile_used": T,
            "fused_pair_ms_by_tile": {str(k): v for k, v in sorted(trial.items())},
            "phi_pair_ms": t_pair, "vis_per_s": sum_m / (t_pair * 1e-3),
            "phi_pair_ms_per_member_launches": t_pair_members, "fused_bitwise_equal_to_per_member": fused_bitwise,
            "roofline": {"bound": "hbm", "kernel": "fused batched (Phi, Phi^dagger), all launches", "achieved": ach,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS, "traffic": None,
                         "algorithmic_bytes_per_pair": pair_bytes},
            "admm_step_ms_graph": out["graph"], "admm_step_ms_streams": out["streams"],
            "admm_vis_per_s": sum_m / (out["graph"] * 1e-3),
            "max_rel_err_fp32_vs_fp64": max(errs64), "median_rel_err_fp32_vs_fp64": float(np.median(errs64)),
            "rel_err_vs_oracle_smallest3": errs_or, "nonfinite": int(sum(r.nonfinite for r in rep)),
            "setup_s": t_setup}


_SERVE_POOL = {}


def serve_pool(n_small=24):
    """Host data of the request pool: channel-law jobs plus two 2048^2 / 5e7 jobs."""
    import workloads as W
    if "pool" in _SERVE_POOL:
        return _SERVE_POOL["pool"]
    rng = W.rng_for(4)
    shapes = W.batch_channels(n_small, rng) + [(2048, 50_000_000)] * 2
    pool = []
    for n, M in shapes:
        pool.append(dict(n=n, M=M, x=W.gaussian_sky(n, W.n_sources_for(n), rng), uv=W.uv_gaussian(M, rng)))
    _SERVE_POOL["pool"] = pool
    return pool


def run_serve(P, dev, args, prec, rate=None, nreq=None):
    """Poisson arrivals of imaging solves through the continuous-batching server."""
    import torch
    import workloads as W
    pool = serve_pool()
    rdt = torch.float32 if prec == P.PR_F32 else torch.float64
    gen = W.torch_generator(4, dev)
    data = []
    for d in pool:
        uv_d = torch.as_tensor(d["uv"]).to(dev, rdt)
        x_d = torch.as_tensor(d["x"]).to(dev, rdt)
        plan = P.PhiPlan(d["n"], uv_d, None, J=4, D=2000, prec=prec)
        y0 = plan.apply(x_d)
        y_user = torch.empty_like(y0)
        y_user[plan.perm()] = y0
        del plan
        y, _, eps = W.add_noise_torch(y_user, W.unit_complex_noise_torch(d["M"], gen, dev, y_user.dtype))
        data.append(dict(n=d["n"], M=d["M"], uv=uv_d, y=y, x=x_d, eps=eps))
    torch.cuda.synchronize()
    rate = args.serve_rate if rate is None else rate
    nreq = args.serve_requests if nreq is None else nreq
    rng = np.random.default_rng(1004)   # same arrivals and job mix for both precisions
    total = args.serve_warmup + nreq
    arrivals = np.cumsum(rng.exponential(1.0 / rate, total))
    big = rng.uniform(size=total) < 0.05
    pick = np.where(big, len(data) - 2 + rng.integers(0, 2, total), rng.integers(0, len(data) - 2, total))
    arena = (48 << 30) if prec == P.PR_F32 else (96 << 30)
    srv = P.Server(arena, max_active=64, nstreams=4, device=dev)
    info, lat, errs = {}, {}, {}
    t0 = time.perf_counter()
    i_next, done, limit = 0, 0, 600.0
    while done < total:
        now = time.perf_counter() - t0
        while i_next < total and arrivals[i_next] <= now:
            d = data[pick[i_next]]
            prm = P.admm_params(d["eps"], 0.0, iters=30, gamma_factor=1e-3, norm_iters=100)
            jid = srv.submit(P.job_desc(d["n"], d["uv"], d["y"], prm, levels=3), keep=(d["uv"], d["y"]))
            info[jid] = (i_next, d)
            i_next += 1
        q, r, f = srv.tick()
        if f:
            for jid in [j for j in info if j not in lat and srv.state(j) == 2]:
                t_done = time.perf_counter() - t0
                i, d = info[jid]
                lat[jid] = (i, t_done - arrivals[i], t_done)
                x, rep = srv.fetch(jid, d["n"], dtype=rdt)
                errs[jid] = float((x / rep.op_norm - d["x"]).norm() / d["x"].norm())
                done += 1
                if done % 50 == 0:
                    log(f"  served {done}/{total} at {time.perf_counter() - t0:.1f} s")
        if q == 0 and r == 0 and i_next < total:
            time.sleep(max(0.0, min(0.01, arrivals[i_next] - (time.perf_counter() - t0))))
        else:
            time.sleep(0.0002)
        if time.perf_counter() - t0 > limit:
            break
    timed = [v for v in lat.values() if v[0] >= args.serve_warmup]
    l_ms = np.array([v[1] for v in timed]) * 1e3
    first = arrivals[args.serve_warmup] if total > args.serve_warmup else 0.0
    last = max(v[2] for v in timed) if timed else 0.0
    e = np.array([errs[j] for j in lat if lat[j][0] >= args.serve_warmup])
    nbig = int(big[args.serve_warmup:].sum())
    return {"workload": "serving-poisson-channel-law+5pct-2048sq-M5e7-30iters", "rate_req_s": rate,
            "requests": len(timed), "warmup_requests": args.serve_warmup, "big_jobs": nbig,
            "solves_per_s": len(timed) / (last - first) if timed else 0.0,
            "p50_ms": float(np.percentile(l_ms, 50)) if timed else None,
            "p99_ms": float(np.percentile(l_ms, 99)) if timed else None,
            "mean_ms": float(l_ms.mean()) if timed else None,
            "img_err_median": float(np.median(e)) if e.size else None,
            "completed_all": done == total}


def pmc_probe(P, dev, workload="op256"):
    """The kernels the counter passes read: the workload's gridding and
    degridding (256^2 / 1e6 by default, or the 2048^2 / 5e8 share), and a
    plain 512 MiB device copy whose FETCH_SIZE / WRITE_SIZE calibrate bytes."""
    import torch
    import workloads as W
    wl = W.CONFIGS[workload]
    rng = W.rng_for(wl.index)
    x = W.make_sky(wl, rng)
    if workload == "share2048":
        uv_d = W.uv_ring_core_torch(wl.M, W.torch_generator(wl.index, dev), dev)
    else:
        uv_d = torch.as_tensor(W.make_uv(wl, rng)).to(dev)
    plan = P.PhiPlan(wl.n, uv_d, None, J=wl.J, D=wl.D)
    del uv_d
    xd = torch.as_tensor(x, dtype=torch.float32, device=dev)
    y = plan.apply(xd)
    for _ in range(5):
        P.pr_phi_gw(plan.handle, y)
        P.pr_phi_grid_patches(plan.handle, y)
        P.pr_phi_grid_merge(plan.handle)
    src = torch.ones(1 << 27, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"pmc_probe": "done", "copy_bytes": src.numel() * 4, "visibilities": wl.M}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="op256", choices=["op256", "op256j6", "share2048"],
                    help="share2048: 2048^2 image, 5e8 ring-plus-core visibilities, FP32 (FP64 scalars) only")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=1000, help="timed requests (FP32)")
    ap.add_argument("--serve-requests-fp64", type=int, default=200,
                    help="timed requests in FP64 (it saturates below 20 req/s, so the queue only grows)")
    ap.add_argument("--serve-warmup", type=int, default=50)
    ap.add_argument("--serve-sweep", default="", help="comma-separated arrival rates (req/s): FP32 load sweep")
    ap.add_argument("--serve-rate", type=float, default=20.0, help="Poisson arrival rate, requests/s")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the 2048^2 / 5e8-visibility sub-run reported under `large_workload`")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="only run the kernels counted by the rocprofv3 --pmc passes (see profiles/)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import workloads as W
    from paper_1903_04502_amd import purimi as P

    P.lib()
    assert torch.cuda.is_available(), "bench needs a GPU"
    dev = torch.device("cuda:0")
    if args.pmc_probe:
        pmc_probe(P, dev, args.workload if args.workload != "op256j6" else "op256")
        return
    wl = W.CONFIGS[args.workload]
    n, M, J, D, L = wl.n, wl.M, wl.J, wl.D, wl.levels
    rng = W.rng_for(wl.index)
    log(f"workload {wl.name}: generating inputs")
    x_true = W.make_sky(wl, rng)
    big = args.workload == "share2048"
    if big:
        # 5e8 baselines and noise drawn on the device (seeded torch generator)
        args.no_fp64 = True
        args.no_batch = args.no_serve = True
        gen = W.torch_generator(wl.index, dev)
        uv_dev = W.uv_ring_core_torch(M, gen, dev)
        uv32 = None
    else:
        uv32 = W.make_uv(wl, rng)
        noise = W.unit_complex_noise(M, rng)
    K_steps, W_steps = args.steps, args.warmup
    out = {}

    def run_prec(prec):
        rdt = torch.float32 if prec == P.PR_F32 else torch.float64
        if big:
            uv = uv_dev
        else:
            uv = torch.as_tensor(uv32.astype(np.float64) if prec == P.PR_F64 else uv32).to(dev)
        plan = P.PhiPlan(n, uv, None, J=J, D=D, prec=prec)
        psi = P.PsiPlan(n, L, 0x1FF, prec, dev)
        perm = plan.perm()
        x = torch.as_tensor(x_true).to(dev, rdt)
        y0 = plan.apply(x)
        if big:
            # noise is iid: drawn directly in plan order on the device
            y, sigma, eps = W.add_noise_torch(y0, W.unit_complex_noise_torch(M, gen, dev), wl.snr_db)
            del y0
        else:
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
        # ---- Phi, Phi^dagger pairs: whole pairs between two events (value) ...
        for _ in range(W_steps):
            P.pr_phi_apply(h, x, yv)
            P.pr_phi_adjoint(h, y, xg)
        torch.cuda.synchronize()
        p0, p1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        p0.record(stream)
        for _ in range(K_steps):
            P.pr_phi_apply(h, x, yv)
            P.pr_phi_adjoint(h, y, xg)
        p1.record(stream)
        torch.cuda.synchronize()
        t_pair = p0.elapsed_time(p1) / K_steps
        # ... and each launch bracketed by events (stage times, roofline)
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(K_steps)]
        for k in range(K_steps):
            e = ev[k]
            e[0].record(stream)
            P.pr_phi_fzs(h, x)
            e[1].record(stream)
            P.pr_phi_gw(h, yv)                 # one launch: degrid_kernel
            e[2].record(stream)
            P.pr_phi_grid_patches(h, y)        # one launch: grid_walk_kernel (J <= 4)
            e[3].record(stream)
            P.pr_phi_grid_merge(h)             # one launch: merge_patches_kernel
            e[4].record(stream)
            P.pr_phi_fzs_adjoint(h, xg)
            e[5].record(stream)
        torch.cuda.synchronize()
        t = np.array([[ev[k][i].elapsed_time(ev[k][i + 1]) for i in range(5)] for k in range(K_steps)])
        t_fzs, t_gw, t_patch, t_merge, t_fzsa = t.mean(axis=0)
        t_gwa = t_patch + t_merge
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
        # one iteration from x = 0 (compared with the oracle's first iteration)
        x_it1 = torch.zeros((n, n), dtype=rdt, device=dev)
        P.pr_admm_solve(h, psi.handle, y, P.admm_params(eps, gamma, iters=1, op_norm=op_norm), x_it1, ws,
                        want_report=False)
        del ws
        # ---- FISTA iterations (MAP problem, the same gamma, unit step)
        fws = torch.empty(P.pr_fista_workspace_size(h, psi.handle), dtype=torch.uint8, device=dev)
        xf = torch.zeros((n, n), dtype=rdt, device=dev)
        P.pr_fista_solve(h, psi.handle, y, P.fista_params(gamma, 1.0, iters=W_steps, op_norm=op_norm), xf, fws,
                         want_report=False)
        xf.zero_()
        torch.cuda.synchronize()
        f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        f0.record(stream)
        P.pr_fista_solve(h, psi.handle, y, P.fista_params(gamma, 1.0, iters=K_steps, op_norm=op_norm), xf, fws,
                         want_report=False)
        f1.record(stream)
        torch.cuda.synchronize()
        t_fista = f0.elapsed_time(f1) / K_steps
        del fws
        # ---- Primal-Dual iterations (the constrained problem: the same eps and gamma)
        pws = torch.empty(P.pr_pd_workspace_size(h, psi.handle), dtype=torch.uint8, device=dev)
        xp = torch.zeros((n, n), dtype=rdt, device=dev)
        P.pr_pd_solve(h, psi.handle, y, P.pd_params(gamma, iters=W_steps, eps=eps, op_norm=op_norm), xp, pws,
                      want_report=False)
        xp.zero_()
        torch.cuda.synchronize()
        f0.record(stream)
        P.pr_pd_solve(h, psi.handle, y, P.pd_params(gamma, iters=K_steps, eps=eps, op_norm=op_norm), xp, pws,
                      want_report=False)
        f1.record(stream)
        torch.cuda.synchronize()
        t_pd = f0.elapsed_time(f1) / K_steps
        del pws
        # ---- local l2 balls: 4 equal-count baseline-length sections, eps_j = sigma sqrt(M_j + 2 sqrt(M_j))
        nsec = 4
        r_len = torch.hypot(uv[:, 0].float(), uv[:, 1].float())
        cuts = torch.sort(r_len).values[[(M * j) // nsec for j in range(1, nsec)]]
        sec_user = torch.bucketize(r_len, cuts, right=True).to(torch.int32)
        del r_len
        sec_plan = sec_user[perm.long()].contiguous()
        cnt = torch.bincount(sec_user, minlength=nsec).double().cpu().numpy()
        del sec_user
        eps_j = sigma * np.sqrt(cnt + 2.0 * np.sqrt(cnt))
        balls = P.Balls(plan, sec_plan, nsec)
        del sec_plan
        lws = torch.empty(P.pr_admm_workspace_size(h, psi.handle), dtype=torch.uint8, device=dev)
        xl = torch.zeros((n, n), dtype=rdt, device=dev)
        P.pr_admm_local_solve(h, psi.handle, balls.handle, y, P.admm_params(0.0, gamma, iters=W_steps, op_norm=op_norm),
                              eps_j, xl, lws, want_report=False)
        xl.zero_()
        torch.cuda.synchronize()
        lprm = P.admm_params(0.0, gamma, iters=K_steps, op_norm=op_norm)
        f0.record(stream)
        # (the call copies the radii and synchronises once before its first kernel)
        P.pr_admm_local_solve(h, psi.handle, balls.handle, y, lprm, eps_j, xl, lws, want_report=False)
        f1.record(stream)
        torch.cuda.synchronize()
        t_local = f0.elapsed_time(f1) / K_steps
        del lws, balls
        return dict(t_fzs=t_fzs, t_gw=t_gw, t_gwa=t_gwa, t_patch=t_patch, t_merge=t_merge, t_fzsa=t_fzsa,
                    t_phi=t_phi, t_adj=t_adj, t_pair=t_pair,
                    t_admm=t_admm, t_fista=t_fista, t_pd=t_pd, t_local=t_local, items=plan.items, tile=plan.desc.tile, op_norm=op_norm, gamma=gamma,
                    eps=eps, resid=rep.resid_norm, nonfinite=rep.nonfinite, y_plan=yv, perm=perm,
                    plan=plan, x=x, y_data=y, x_adj=xg, x_it1=x_it1)

    log("FP32 runs")
    r32 = run_prec(P.PR_F32)
    log(f"FP32: phi {r32['t_phi']:.3f} ms, adj {r32['t_adj']:.3f} ms, admm {r32['t_admm']:.3f} ms")
    r64 = None
    if not args.no_fp64:
        log("FP64 runs")
        r64 = run_prec(P.PR_F64)
        log(f"FP64: phi {r64['t_phi']:.3f} ms, adj {r64['t_adj']:.3f} ms, admm {r64['t_admm']:.3f} ms")

    value = M / (r32["t_pair"] * 1e-3)
    copy_gbs = copy_bandwidth(dev)
    # dominant single-kernel stage of the operator pair: gridding patches or degridding
    vis_bytes = 20.0 * M            # u, v, w, y in FP32 per visibility, once per launch
    kernels = {"grid_walk_kernel": r32["t_patch"], "degrid_kernel": r32["t_gw"]}
    dom = max(kernels, key=kernels.get)
    roof = {}
    for kname, t_ms in kernels.items():
        ach = vis_bytes / (t_ms * 1e-3) / 1e9
        roof[kname] = {"bound": "hbm", "kernel": kname, "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": ach / HBM_PEAK_GBS, "traffic": kernel_traffic(kname, wl.name),
                       "algorithmic_bytes_per_launch": vis_bytes, "launch_ms": t_ms,
                       "frac_of_copy": ach / copy_gbs}
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
        "phi_pair_ms": r32["t_pair"], "phi_ms": r32["t_phi"], "phi_adjoint_ms": r32["t_adj"],
        "stage_ms": {"fzs": r32["t_fzs"], "gw": r32["t_gw"], "grid_patches": r32["t_patch"],
                     "grid_merge": r32["t_merge"], "fzs_adjoint": r32["t_fzsa"]},
        "admm_iter_ms_fp32": r32["t_admm"],
        "fista_iter_ms_fp32": r32["t_fista"],
        "primal_dual_iter_ms_fp32": r32["t_pd"],
        "admm_local_balls_iter_ms_fp32": r32["t_local"],
        "roofline": roof[dom],
        "copy_gbs": copy_gbs,
        "roofline_other": [v for k, v in roof.items() if k != dom],
        "work_items": r32["items"],
    }
    if r64 is not None:
        res["fp64"] = {"value": M / (r64["t_pair"] * 1e-3), "phi_ms": r64["t_phi"],
                       "phi_adjoint_ms": r64["t_adj"], "admm_iter_ms": r64["t_admm"],
                       "fista_iter_ms": r64["t_fista"], "primal_dual_iter_ms": r64["t_pd"],
                       "admm_local_balls_iter_ms": r64["t_local"],
                       "stage_ms": {"fzs": r64["t_fzs"], "gw": r64["t_gw"], "grid_patches": r64["t_patch"],
                                    "grid_merge": r64["t_merge"], "fzs_adjoint": r64["t_fzsa"]}}
    if not args.no_cpu_baseline and big:
        log("CPU baseline: oracle Phi and Phi^dagger on a 2e6-visibility sample of the 5e8")
        from oracle import measurement as ms
        spec = ms.PhiSpec(n, 2 * n, J, D)
        Ms = 2_000_000
        uv_s = uv_dev[:Ms].double().cpu().numpy()
        t0 = time.perf_counter()
        y_s = ms.phi(x_true, uv_s, None, spec)
        t1 = time.perf_counter()
        ms.phi_adjoint(y_s, uv_s, None, spec)
        t2 = time.perf_counter()
        res["cpu_baseline"] = {"value": Ms / (t2 - t0), "unit": "visibilities/s", "cores": 1, "kind": "oracle",
                               "sample": f"one Phi ({t1 - t0:.1f} s) and one Phi^dagger ({t2 - t1:.1f} s) of the "
                                         f"FP64 NumPy oracle on the full 2048^2 image and the first {Ms} of the "
                                         f"5e8 baselines (single thread; the 4096^2 FFTs are not amortised)",
                               "host_cpus": os.cpu_count()}
        # sampled parity of the timed Phi: the sample's visibilities in plan order
        perm = r32["perm"]
        pos = torch.nonzero(perm < Ms).squeeze(1)
        y_gpu = r32["y_plan"][pos].cpu().numpy().astype(np.complex128)
        y_or = y_s[perm[pos].cpu().numpy()]
        res["phi_rel_err_fp32_vs_oracle_sample"] = float(np.linalg.norm(y_gpu - y_or) / np.linalg.norm(y_or))
    elif not args.no_cpu_baseline:
        log("CPU baseline: oracle Phi and Phi^dagger on the full input (one thread, then all host cores)")
        from oracle import admm as oadmm, measurement as ms, wavelets as owv
        spec = ms.PhiSpec(n, 2 * n, J, D)
        uv64 = uv32.astype(np.float64)
        t0 = time.perf_counter()
        y_ref = ms.phi(x_true, uv64, None, spec)
        t1 = time.perf_counter()
        ms.phi_adjoint(y_ref, uv64, None, spec)
        t2 = time.perf_counter()
        workers = min(16, os.cpu_count() or 1)
        tp = cpu_pair_parallel(x_true, uv64, spec, workers)
        res["cpu_baseline"] = {"value": M / tp["pair_s"], "unit": "visibilities/s", "cores": tp["workers"],
                               "kind": "oracle",
                               "sample": f"one Phi ({tp['phi_s']:.2f} s) and one Phi^dagger ({tp['adj_s']:.2f} s) of "
                                         f"the FP64 NumPy oracle on the full {M}-visibility input, the visibilities "
                                         f"split over {tp['workers']} worker processes (the oracle's own degridding "
                                         f"and gridding per chunk, partial grids added in chunk order)",
                               "single_thread": {"value": M / (t2 - t0), "phi_s": t1 - t0, "adj_s": t2 - t1},
                               "host_cpus": os.cpu_count(), "cpu_model": cpu_model()}
        # the oracle's first ADMM iteration with the GPU's operator norm and gamma (one thread)
        perm = r32["perm"].cpu().numpy()
        inv = np.empty_like(perm)
        inv[perm] = np.arange(perm.size)
        y_user = r32["y_data"].cpu().numpy().astype(np.complex128)[inv]
        nrm = r32["op_norm"]
        S = owv.Sara(n, L)
        t0 = time.perf_counter()
        x1_ref, _, _, _ = oadmm.admm(y_user, lambda v: ms.phi(v, uv64, None, spec) / nrm,
                                     lambda v: ms.phi_adjoint(v, uv64, None, spec) / nrm, S.forward, S.adjoint,
                                     r32["eps"], oadmm.AdmmParams(gamma=r32["gamma"], iters=1), np.zeros((n, n)))
        res["cpu_baseline"]["admm_iter_s_single_thread"] = time.perf_counter() - t0
        rel = lambda g, r: float(np.linalg.norm(g - r) / np.linalg.norm(r))
        y32 = r32["y_plan"].cpu().numpy().astype(np.complex128)
        # the last Phi of the timed loop was applied to the sky: compare in plan order
        res["phi_rel_err_fp32_vs_oracle"] = rel(y32, y_ref[perm])
        xadj_ref = ms.phi_adjoint(y_user, uv64, None, spec)
        res["phi_adjoint_rel_err_fp32_vs_oracle"] = rel(r32["x_adj"].cpu().numpy(), xadj_ref)
        res["admm_iter_rel_err_fp32_vs_oracle"] = rel(r32["x_it1"].cpu().numpy(), x1_ref)
        if r64 is not None:
            y64 = r64["y_plan"].cpu().numpy()
            perm64 = r64["perm"].cpu().numpy()
            res["fp64"]["phi_rel_err_vs_oracle"] = rel(y64, y_ref[perm64])
            inv64 = np.empty_like(perm64)
            inv64[perm64] = np.arange(perm64.size)
            yu64 = r64["y_data"].cpu().numpy()[inv64]
            res["fp64"]["phi_adjoint_rel_err_vs_oracle"] = rel(r64["x_adj"].cpu().numpy(),
                                                             ms.phi_adjoint(yu64, uv64, None, spec))
    del r32, r64
    torch.cuda.empty_cache()
    if not big:
        log("first-order kernel lookup")
        res["linear_lookup"] = run_linear(P, dev, n, J, D, uv32, x_true, K_steps, W_steps, not args.no_cpu_baseline)
        log("J = 6")
        res["j6"] = run_j6(P, dev, n, D, L, uv32, x_true, K_steps, W_steps, not args.no_cpu_baseline)
    if not args.no_batch:
        log("batched channels")
        res["batch"] = run_batch(P, dev, args)
    if not args.no_serve:
        for prec in (P.PR_F32, P.PR_F64):
            tag = "fp32" if prec == P.PR_F32 else "fp64"
            log(f"serving {tag}")
            nreq = args.serve_requests if prec == P.PR_F32 else args.serve_requests_fp64
            res.setdefault("serving", {})[tag] = run_serve(P, dev, args, prec, nreq=nreq)
            torch.cuda.empty_cache()
        s32, s64 = res["serving"]["fp32"], res["serving"]["fp64"]
        s32["img_err_gap_vs_fp64"] = abs(s32["img_err_median"] - s64["img_err_median"])
        for rate in [float(r) for r in args.serve_sweep.split(",") if r.strip()]:
            log(f"serving sweep fp32 at {rate} req/s")
            r = run_serve(P, dev, args, P.PR_F32, rate=rate, nreq=max(100, int(10 * rate)))
            res.setdefault("serving_sweep_fp32", []).append(
                {k: r[k] for k in ("rate_req_s", "requests", "solves_per_s", "p50_ms", "p99_ms", "completed_all")})
            torch.cuda.empty_cache()
    if not big and not args.no_large:
        res["large_workload"] = run_large(args)
    print(json.dumps(res))


def run_large(args):
    """The 2048^2 / 5e8-visibility workload (one GPU's share of the paper's
    largest run), measured by this script in a child process after the
    device memory of the main run is released: its own JSON line is kept."""
    import subprocess
    import torch
    torch.cuda.empty_cache()
    log("large workload: 2048^2 image, 5e8 visibilities (child process)")
    cmd = [sys.executable, os.path.abspath(__file__), "--workload", "share2048", "--steps", "20", "--warmup", "2"]
    if args.no_cpu_baseline:
        cmd.append("--no-cpu-baseline")
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
    sys.stderr.write(r.stderr[-2000:])
    lines = [l for l in r.stdout.splitlines() if l.startswith("{")]
    if r.returncode != 0 or not lines:
        return {"error": f"child exited with {r.returncode}"}
    child = json.loads(lines[-1])
    keep = ("value", "unit", "ms_per_step", "phi_pair_ms", "phi_ms", "phi_adjoint_ms", "stage_ms",
            "admm_iter_ms_fp32", "fista_iter_ms_fp32", "primal_dual_iter_ms_fp32",
            "admm_local_balls_iter_ms_fp32", "roofline", "roofline_other", "copy_gbs", "config", "roofline_admm",
            "cpu_baseline", "phi_rel_err_fp32_vs_oracle_sample", "steps", "warmup")
    return {k: child[k] for k in keep if k in child}


if __name__ == "__main__":
    main()
