"""Thin Python binding of the gfx950 library (include/purimi.h).

Functions named ``pr_*`` mirror the C entry points one to one and only
marshal arguments: device tensors become pointers, and the stream is torch's
current stream on the tensors' device. The plan classes at the bottom hold the
caller-owned workspaces as torch tensors (torch is the device allocator).

Nothing here computes any part of the method; if ``libpurimi.so`` is missing
every call raises (there is no fallback).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpurimi.so")

PR_OK, PR_EINVAL, PR_EWORKSPACE, PR_EHIP, PR_EUNSUPPORTED = 0, 1, 2, 3, 4
PR_F32, PR_F64 = 0, 1
PR_PD_BALL, PR_PD_L2 = 0, 1


class PrError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"purimi error {code}: {msg}")
        self.code = code


class pr_phi_desc(C.Structure):
    _fields_ = [("n", C.c_int32), ("oversample", C.c_int32), ("J", C.c_int32), ("D", C.c_int32),
                ("M", C.c_int64), ("prec", C.c_int32), ("tile", C.c_int32), ("interp", C.c_int32)]


class pr_admm_params(C.Structure):
    _fields_ = [("iters", C.c_int32), ("inner_iters", C.c_int32), ("eps", C.c_double),
                ("gamma", C.c_double), ("rho", C.c_double), ("varrho", C.c_double),
                ("eta", C.c_double), ("rel_tol", C.c_double), ("op_norm", C.c_double),
                ("gamma_factor", C.c_double), ("norm_iters", C.c_int32)]


class pr_fista_params(C.Structure):
    _fields_ = [("iters", C.c_int32), ("inner_iters", C.c_int32), ("gamma", C.c_double),
                ("lambda_", C.c_double), ("eta", C.c_double), ("op_norm", C.c_double),
                ("gamma_factor", C.c_double), ("norm_iters", C.c_int32)]


class pr_pd_params(C.Structure):
    _fields_ = [("iters", C.c_int32), ("inner_iters", C.c_int32), ("misfit", C.c_int32), ("eps", C.c_double),
                ("gamma", C.c_double), ("tau", C.c_double), ("sigma", C.c_double), ("theta", C.c_double),
                ("eta", C.c_double), ("op_norm", C.c_double), ("gamma_factor", C.c_double),
                ("norm_iters", C.c_int32)]


class pr_reweight_params(C.Structure):
    _fields_ = [("rounds", C.c_int32), ("delta0", C.c_double), ("beta", C.c_double)]


class pr_admm_report(C.Structure):
    _fields_ = [("iters_done", C.c_int32), ("rel_var", C.c_double), ("resid_norm", C.c_double),
                ("l1_norm", C.c_double), ("op_norm", C.c_double), ("nonfinite", C.c_int32)]


class pr_job_desc(C.Structure):
    _fields_ = [("n", C.c_int32), ("J", C.c_int32), ("D", C.c_int32), ("tile", C.c_int32),
                ("levels", C.c_int32), ("basis_mask", C.c_uint32), ("prec", C.c_int32), ("M", C.c_int64),
                ("uv", C.c_void_p), ("w", C.c_void_p), ("y", C.c_void_p), ("params", pr_admm_params),
                ("interp", C.c_int32)]


_VP, _I32, _I64, _U32, _D, _SZ = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_double, C.c_size_t
_SIGS = {
    "pr_last_error": (C.c_char_p, []),
    "pr_version": (C.c_int, []),
    "pr_phi_plan_sizes": (C.c_int, [C.POINTER(pr_phi_desc), C.POINTER(_SZ), C.POINTER(_SZ)]),
    "pr_phi_plan_create": (C.c_int, [C.POINTER(pr_phi_desc), _VP, _VP, _VP, _VP, _VP, C.POINTER(_VP)]),
    "pr_phi_plan_destroy": (C.c_int, [_VP]),
    "pr_phi_plan_perm": (C.c_int, [_VP, C.POINTER(_VP)]),
    "pr_phi_plan_perm_copy": (C.c_int, [_VP, _VP, _VP]),
    "pr_phi_plan_items": (C.c_int, [_VP, C.POINTER(_I64)]),
    "pr_phi_apply": (C.c_int, [_VP, _VP, _VP, _VP]),
    "pr_phi_adjoint": (C.c_int, [_VP, _VP, _VP, _VP]),
    "pr_phi_fzs": (C.c_int, [_VP, _VP, _VP]),
    "pr_phi_gw": (C.c_int, [_VP, _VP, _VP]),
    "pr_phi_gw_adjoint": (C.c_int, [_VP, _VP, _VP]),
    "pr_phi_fzs_adjoint": (C.c_int, [_VP, _VP, _VP]),
    "pr_phi_grid_patches": (C.c_int, [_VP, _VP, _VP]),
    "pr_phi_grid_merge": (C.c_int, [_VP, _VP]),
    "pr_phi_norm": (C.c_int, [_VP, _I32, _D, _VP, C.POINTER(_D), _VP]),
    "pr_psi_plan_sizes": (C.c_int, [_I32, _I32, _U32, _I32, C.POINTER(_SZ), C.POINTER(_SZ)]),
    "pr_psi_plan_create": (C.c_int, [_I32, _I32, _U32, _I32, _VP, _VP, _VP, C.POINTER(_VP)]),
    "pr_psi_plan_destroy": (C.c_int, [_VP]),
    "pr_psi_plan_bases": (C.c_int, [_VP, C.POINTER(_I32)]),
    "pr_psi_filter": (C.c_int, [_VP, _I32, C.POINTER(_D)]),
    "pr_psi_apply": (C.c_int, [_VP, _VP, _VP, _VP]),
    "pr_psi_adjoint": (C.c_int, [_VP, _VP, _VP, _VP]),
    "pr_prox_l1": (C.c_int, [_VP, _VP, _I64, _I32, _I32, _D, _VP]),
    "pr_proj_l2ball_scratch_bytes": (_SZ, [_I64]),
    "pr_proj_l2ball": (C.c_int, [_VP, _VP, _VP, _I64, _I32, _D, _VP, C.POINTER(_D), _VP]),
    "pr_proj_l2ball_noalloc": (C.c_int, [_VP, _VP, _VP, _I64, _I32, _D, C.POINTER(_D), _VP]),
    "pr_admm_workspace_size": (C.c_int, [_VP, _VP, C.POINTER(_SZ)]),
    "pr_admm_solve": (C.c_int, [_VP, _VP, _VP, C.POINTER(pr_admm_params), _VP, _VP,
                                C.POINTER(pr_admm_report), _VP]),
    "pr_admm_resume": (C.c_int, [_VP, _VP, _VP, C.POINTER(pr_admm_params), _VP, _VP,
                                 C.POINTER(pr_admm_report), _VP]),
    "pr_admm_state_bytes": (C.c_int, [_VP, _VP, C.POINTER(_SZ)]),
    "pr_admm_state_export": (C.c_int, [_VP, _VP, _VP, _VP, _VP, _VP]),
    "pr_admm_state_import": (C.c_int, [_VP, _VP, _VP, _VP, _VP, _VP]),
    "pr_fista_workspace_size": (C.c_int, [_VP, _VP, C.POINTER(_SZ)]),
    "pr_fista_solve": (C.c_int, [_VP, _VP, _VP, C.POINTER(pr_fista_params), _VP, _VP,
                                 C.POINTER(pr_admm_report), _VP]),
    "pr_pd_workspace_size": (C.c_int, [_VP, _VP, C.POINTER(_SZ)]),
    "pr_pd_solve": (C.c_int, [_VP, _VP, _VP, C.POINTER(pr_pd_params), _VP, _VP, C.POINTER(pr_admm_report), _VP]),
    "pr_balls_sizes": (C.c_int, [C.c_int64, _I32, C.POINTER(_SZ), C.POINTER(_SZ)]),
    "pr_balls_create": (C.c_int, [C.c_int64, _I32, _VP, _VP, _SZ, _VP, _SZ, _VP, C.POINTER(_VP)]),
    "pr_balls_destroy": (C.c_int, [_VP]),
    "pr_balls_norms": (C.c_int, [_VP, C.POINTER(_D), _VP]),
    "pr_admm_local_solve": (C.c_int, [_VP, _VP, _VP, _VP, C.POINTER(pr_admm_params), C.POINTER(_D), _VP, _VP,
                                      C.POINTER(pr_admm_report), _VP]),
    "pr_reweight_workspace_size": (C.c_int, [_VP, _VP, C.POINTER(_SZ)]),
    "pr_admm_reweighted_solve": (C.c_int, [_VP, _VP, _VP, C.POINTER(pr_admm_params), C.POINTER(pr_reweight_params),
                                           _VP, _VP, C.POINTER(pr_admm_report), _VP]),
    "pr_phi_tune": (C.c_int, [C.POINTER(pr_phi_desc), _VP, _VP, _VP, _VP, _VP, _I32, _VP, C.POINTER(_I32),
                              C.POINTER(_D)]),
    "pr_batch_create": (C.c_int, [_I32, _I32, C.POINTER(_VP)]),
    "pr_batch_destroy": (C.c_int, [_VP]),
    "pr_batch_add": (C.c_int, [_VP, _VP, _VP, _VP, _VP, C.POINTER(pr_admm_params), _VP, _VP, C.POINTER(_I32)]),
    "pr_batch_remove": (C.c_int, [_VP, _I32]),
    "pr_batch_members": (C.c_int, [_VP, C.POINTER(_I32)]),
    "pr_batch_step": (C.c_int, [_VP, _I32, _I32, _VP]),
    "pr_batch_phi_apply": (C.c_int, [_VP, C.POINTER(_VP), C.POINTER(_VP), _VP]),
    "pr_batch_phi_adjoint": (C.c_int, [_VP, C.POINTER(_VP), C.POINTER(_VP), _VP]),
    "pr_batch_report": (C.c_int, [_VP, _I32, C.POINTER(pr_admm_report), _VP]),
    "pr_batch_fuse_bytes": (C.c_int, [_VP, C.POINTER(_SZ)]),
    "pr_batch_fuse": (C.c_int, [_VP, _VP, _SZ, _VP]),
    "pr_server_job_bytes": (C.c_int, [C.POINTER(pr_job_desc), C.POINTER(_SZ)]),
    "pr_server_create": (C.c_int, [_VP, _SZ, _I32, _I32, C.POINTER(_VP)]),
    "pr_server_destroy": (C.c_int, [_VP]),
    "pr_server_submit": (C.c_int, [_VP, C.POINTER(pr_job_desc), C.POINTER(_I64)]),
    "pr_server_tick": (C.c_int, [_VP, C.POINTER(_I32), C.POINTER(_I32), C.POINTER(_I32)]),
    "pr_server_job_state": (C.c_int, [_VP, _I64, C.POINTER(_I32), C.POINTER(_I32)]),
    "pr_server_fetch": (C.c_int, [_VP, _I64, _VP, C.POINTER(pr_admm_report), _VP]),
    "pr_server_cancel": (C.c_int, [_VP, C.c_int64]),
    "pr_server_free_bytes": (C.c_int, [_VP, C.POINTER(_SZ), C.POINTER(_SZ)]),
}

_lib = None


def lib() -> C.CDLL:
    """Load libpurimi.so (built in place by ``build()``); raise if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run paper_1903_04502_amd.build.build()")
        h = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(h, name)
            f.restype = res
            f.argtypes = args
        _lib = h
    return _lib


def exported_symbols():
    return list(_SIGS)


def _check(rc: int):
    if rc != PR_OK:
        raise PrError(rc, lib().pr_last_error().decode())


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(device=None):
    return torch.cuda.current_stream(device).cuda_stream


def _prec_of(dtype) -> int:
    if dtype in (torch.float32, torch.complex64):
        return PR_F32
    if dtype in (torch.float64, torch.complex128):
        return PR_F64
    raise TypeError(f"unsupported dtype {dtype}")


# --------------------------------------------------------------------------
# one-to-one wrappers (same names as the C symbols)
# --------------------------------------------------------------------------
def pr_last_error() -> str:
    return lib().pr_last_error().decode()


def pr_version() -> int:
    return lib().pr_version()


def pr_phi_plan_sizes(desc: pr_phi_desc):
    p, s = _SZ(), _SZ()
    _check(lib().pr_phi_plan_sizes(C.byref(desc), C.byref(p), C.byref(s)))
    return p.value, s.value


def pr_phi_plan_create(desc, uv, w, persistent, scratch, stream=None):
    h = _VP()
    _check(lib().pr_phi_plan_create(C.byref(desc), _ptr(uv), _ptr(w), _ptr(persistent), _ptr(scratch),
                                    stream if stream is not None else _stream(), C.byref(h)))
    return h.value


def pr_phi_plan_destroy(plan):
    _check(lib().pr_phi_plan_destroy(plan))


def pr_phi_plan_perm(plan) -> int:
    p = _VP()
    _check(lib().pr_phi_plan_perm(plan, C.byref(p)))
    return p.value


def pr_phi_plan_perm_copy(plan, dst, stream=None):
    _check(lib().pr_phi_plan_perm_copy(plan, _ptr(dst), stream if stream is not None else _stream()))


def pr_phi_plan_items(plan) -> int:
    v = _I64()
    _check(lib().pr_phi_plan_items(plan, C.byref(v)))
    return v.value


def pr_phi_apply(plan, x, y, stream=None):
    _check(lib().pr_phi_apply(plan, _ptr(x), _ptr(y), stream if stream is not None else _stream()))


def pr_phi_adjoint(plan, y, x, stream=None):
    _check(lib().pr_phi_adjoint(plan, _ptr(y), _ptr(x), stream if stream is not None else _stream()))


def pr_phi_fzs(plan, x, stream=None):
    _check(lib().pr_phi_fzs(plan, _ptr(x), stream if stream is not None else _stream()))


def pr_phi_gw(plan, y, stream=None):
    _check(lib().pr_phi_gw(plan, _ptr(y), stream if stream is not None else _stream()))


def pr_phi_gw_adjoint(plan, y, stream=None):
    _check(lib().pr_phi_gw_adjoint(plan, _ptr(y), stream if stream is not None else _stream()))


def pr_phi_fzs_adjoint(plan, x, stream=None):
    _check(lib().pr_phi_fzs_adjoint(plan, _ptr(x), stream if stream is not None else _stream()))


def pr_phi_grid_patches(plan, y, stream=None):
    _check(lib().pr_phi_grid_patches(plan, _ptr(y), stream if stream is not None else _stream()))


def pr_phi_grid_merge(plan, stream=None):
    _check(lib().pr_phi_grid_merge(plan, stream if stream is not None else _stream()))


def pr_phi_norm(plan, iters, rtol, vis_ws, stream=None) -> float:
    v = _D()
    _check(lib().pr_phi_norm(plan, iters, float(rtol), _ptr(vis_ws), C.byref(v),
                             stream if stream is not None else _stream()))
    return v.value


def pr_psi_plan_sizes(n, levels, mask, prec):
    p, s = _SZ(), _SZ()
    _check(lib().pr_psi_plan_sizes(n, levels, mask, prec, C.byref(p), C.byref(s)))
    return p.value, s.value


def pr_psi_plan_create(n, levels, mask, prec, persistent, scratch, stream=None):
    h = _VP()
    _check(lib().pr_psi_plan_create(n, levels, mask, prec, _ptr(persistent), _ptr(scratch),
                                    stream if stream is not None else _stream(), C.byref(h)))
    return h.value


def pr_psi_plan_destroy(plan):
    _check(lib().pr_psi_plan_destroy(plan))


def pr_psi_plan_bases(plan) -> int:
    v = _I32()
    _check(lib().pr_psi_plan_bases(plan, C.byref(v)))
    return v.value


def pr_psi_filter(plan, k):
    buf = (_D * (2 * k))()
    _check(lib().pr_psi_filter(plan, k, buf))
    return list(buf)


def pr_psi_apply(plan, alpha, x, stream=None):
    _check(lib().pr_psi_apply(plan, _ptr(alpha), _ptr(x), stream if stream is not None else _stream()))


def pr_psi_adjoint(plan, x, alpha, stream=None):
    _check(lib().pr_psi_adjoint(plan, _ptr(x), _ptr(alpha), stream if stream is not None else _stream()))


def pr_prox_l1(inp, out, lam, stream=None):
    is_c = 1 if inp.is_complex() else 0
    _check(lib().pr_prox_l1(_ptr(inp), _ptr(out), inp.numel(), is_c, _prec_of(inp.dtype), float(lam),
                            stream if stream is not None else _stream()))


def pr_proj_l2ball_scratch_bytes(length: int) -> int:
    return lib().pr_proj_l2ball_scratch_bytes(length)


def pr_proj_l2ball(inp, center, out, eps, scratch, want_dist=False, stream=None):
    d = _D()
    _check(lib().pr_proj_l2ball(_ptr(inp), _ptr(center), _ptr(out), inp.numel(), _prec_of(inp.dtype), float(eps),
                                _ptr(scratch), C.byref(d) if want_dist else None,
                                stream if stream is not None else _stream()))
    return d.value if want_dist else None


def pr_proj_l2ball_noalloc(inp, center, out, eps, want_dist=False, stream=None):
    """pr_proj_l2ball with the library's static scratch (allocates nothing)."""
    d = _D()
    _check(lib().pr_proj_l2ball_noalloc(_ptr(inp), _ptr(center), _ptr(out), inp.numel(), _prec_of(inp.dtype),
                                        float(eps), C.byref(d) if want_dist else None,
                                        stream if stream is not None else _stream()))
    return d.value if want_dist else None


def pr_admm_workspace_size(phi, psi) -> int:
    v = _SZ()
    _check(lib().pr_admm_workspace_size(phi, psi, C.byref(v)))
    return v.value


def pr_admm_solve(phi, psi, y, params: pr_admm_params, x, workspace, want_report=True, stream=None):
    rep = pr_admm_report()
    _check(lib().pr_admm_solve(phi, psi, _ptr(y), C.byref(params), _ptr(x), _ptr(workspace),
                               C.byref(rep) if want_report else None, stream if stream is not None else _stream()))
    return rep if want_report else None


def pr_admm_resume(phi, psi, y, params: pr_admm_params, x, workspace, want_report=True, stream=None):
    rep = pr_admm_report()
    _check(lib().pr_admm_resume(phi, psi, _ptr(y), C.byref(params), _ptr(x), _ptr(workspace),
                                C.byref(rep) if want_report else None, stream if stream is not None else _stream()))
    return rep if want_report else None


def pr_admm_state_bytes(phi, psi) -> int:
    v = _SZ()
    _check(lib().pr_admm_state_bytes(phi, psi, C.byref(v)))
    return v.value


def pr_admm_state_export(phi, psi, workspace, x, state, stream=None):
    _check(lib().pr_admm_state_export(phi, psi, _ptr(workspace), _ptr(x), _ptr(state),
                                      stream if stream is not None else _stream()))


def pr_admm_state_import(phi, psi, state, workspace, x, stream=None):
    _check(lib().pr_admm_state_import(phi, psi, _ptr(state), _ptr(workspace), _ptr(x),
                                      stream if stream is not None else _stream()))


def pr_phi_tune(desc: pr_phi_desc, uv, w, persistent, scratch, vis_ws, reps=3, stream=None):
    t, ms = _I32(), _D()
    _check(lib().pr_phi_tune(C.byref(desc), _ptr(uv), _ptr(w), _ptr(persistent), _ptr(scratch), _ptr(vis_ws),
                             reps, stream if stream is not None else _stream(), C.byref(t), C.byref(ms)))
    return t.value, ms.value


def pr_batch_create(max_members: int, nstreams: int):
    h = _VP()
    _check(lib().pr_batch_create(max_members, nstreams, C.byref(h)))
    return h.value


def pr_batch_destroy(b):
    _check(lib().pr_batch_destroy(b))


def pr_batch_add(b, phi, psi, y, x, params: pr_admm_params, workspace, stream=None) -> int:
    slot = _I32()
    _check(lib().pr_batch_add(b, phi, psi, _ptr(y), _ptr(x), C.byref(params), _ptr(workspace),
                              stream if stream is not None else _stream(), C.byref(slot)))
    return slot.value


def pr_batch_remove(b, slot: int):
    _check(lib().pr_batch_remove(b, slot))


def pr_batch_members(b) -> int:
    c = _I32()
    _check(lib().pr_batch_members(b, C.byref(c)))
    return c.value


def pr_batch_step(b, iters: int, use_graph: bool = True, stream=None):
    _check(lib().pr_batch_step(b, iters, 1 if use_graph else 0, stream if stream is not None else _stream()))


def _ptr_array(ts, n):
    arr = (_VP * n)()
    for i, t in enumerate(ts):
        arr[i] = _ptr(t)
    return arr


def pr_batch_phi_apply(b, xs, ys, stream=None):
    n = max(len(xs), len(ys))
    _check(lib().pr_batch_phi_apply(b, _ptr_array(xs, n), _ptr_array(ys, n),
                                    stream if stream is not None else _stream()))


def pr_batch_phi_adjoint(b, ys, xs, stream=None):
    n = max(len(xs), len(ys))
    _check(lib().pr_batch_phi_adjoint(b, _ptr_array(ys, n), _ptr_array(xs, n),
                                      stream if stream is not None else _stream()))


def pr_batch_report(b, slot: int, stream=None) -> pr_admm_report:
    rep = pr_admm_report()
    _check(lib().pr_batch_report(b, slot, C.byref(rep), stream if stream is not None else _stream()))
    return rep


def pr_batch_fuse_bytes(b) -> int:
    v = _SZ()
    _check(lib().pr_batch_fuse_bytes(b, C.byref(v)))
    return v.value


def pr_batch_fuse(b, workspace, stream=None):
    _check(lib().pr_batch_fuse(b, _ptr(workspace), workspace.numel() * workspace.element_size(),
                               stream if stream is not None else _stream()))


def pr_server_job_bytes(desc: pr_job_desc) -> int:
    v = _SZ()
    _check(lib().pr_server_job_bytes(C.byref(desc), C.byref(v)))
    return v.value


def pr_server_create(arena, arena_bytes: int, max_active: int, nstreams: int):
    h = _VP()
    _check(lib().pr_server_create(_ptr(arena), arena_bytes, max_active, nstreams, C.byref(h)))
    return h.value


def pr_server_destroy(srv):
    _check(lib().pr_server_destroy(srv))


def pr_server_submit(srv, desc: pr_job_desc) -> int:
    jid = _I64()
    _check(lib().pr_server_submit(srv, C.byref(desc), C.byref(jid)))
    return jid.value


def pr_server_tick(srv):
    q, r, f = _I32(), _I32(), _I32()
    _check(lib().pr_server_tick(srv, C.byref(q), C.byref(r), C.byref(f)))
    return q.value, r.value, f.value


def pr_server_job_state(srv, job_id: int):
    st, it = _I32(), _I32()
    _check(lib().pr_server_job_state(srv, job_id, C.byref(st), C.byref(it)))
    return st.value, it.value


def pr_server_fetch(srv, job_id: int, x_out=None, want_report=True, stream=None):
    rep = pr_admm_report()
    _check(lib().pr_server_fetch(srv, job_id, _ptr(x_out), C.byref(rep) if want_report else None,
                                 stream if stream is not None else _stream()))
    return rep if want_report else None


def pr_server_cancel(srv, job_id: int):
    _check(lib().pr_server_cancel(srv, int(job_id)))


def pr_server_free_bytes(srv):
    f, l = _SZ(), _SZ()
    _check(lib().pr_server_free_bytes(srv, C.byref(f), C.byref(l)))
    return f.value, l.value


# --------------------------------------------------------------------------
# plan holders: workspaces are torch tensors on the plan's device
# --------------------------------------------------------------------------
def _workspace(nbytes: int, device) -> torch.Tensor:
    # torch's caching allocator returns blocks aligned to at least 512 bytes
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def tune_tile(n, uv, w=None, J=4, D=2000, oversample=2, prec=None, reps=3, interp=0) -> int:
    """Fastest tile side for these baselines, measured by pr_phi_tune."""
    dev = uv.device
    prec = _prec_of(uv.dtype) if prec is None else prec
    M = uv.shape[0]
    pb = sb = 0
    for T in (8, 16, 32):
        try:
            p, s_ = pr_phi_plan_sizes(pr_phi_desc(n, oversample, J, D, M, prec, T, interp))
        except PrError:
            continue
        pb, sb = max(pb, p), max(sb, s_)
    cdt = torch.complex64 if prec == PR_F32 else torch.complex128
    vis = torch.empty(max(M, 1), dtype=cdt, device=dev)
    t, _ = pr_phi_tune(pr_phi_desc(n, oversample, J, D, M, prec, 0, interp), uv.contiguous(),
                       None if w is None else w.contiguous(), _workspace(pb, dev), _workspace(sb, dev), vis, reps,
                       _stream(dev))
    return t


class PhiPlan:
    """Measurement operator plan for one set of baselines (see pr_phi_plan_create).
    tile: 0 = the library default, "auto" = measured by the autotuner.
    interp: 0 = nearest table sample (FP32 plans with tiles <= 16 and D <= 2047
    store each visibility's taps, evaluated once), 1 = first-order (linear)
    lookup, 2 = nearest table sample with the taps recomputed from the stored
    (u, v) at every launch (the same samples as 0)."""

    def __init__(self, n, uv, w=None, J=4, D=2000, oversample=2, tile=0, prec=None, interp=0):
        dev = uv.device
        self.prec = _prec_of(uv.dtype) if prec is None else prec
        self.rdtype = torch.float32 if self.prec == PR_F32 else torch.float64
        self.cdtype = torch.complex64 if self.prec == PR_F32 else torch.complex128
        M = uv.shape[0]
        if tile == "auto":
            tile = tune_tile(n, uv, w, J, D, oversample, self.prec, interp=interp)
        self.desc = pr_phi_desc(n, oversample, J, D, M, self.prec, tile, interp)
        self.n, self.M, self.device = n, M, dev
        pb, sb = pr_phi_plan_sizes(self.desc)
        self.persistent = _workspace(pb, dev)
        self.scratch = _workspace(sb, dev)
        uv = uv.contiguous()
        w = None if w is None else w.contiguous()
        self.handle = pr_phi_plan_create(self.desc, uv, w, self.persistent, self.scratch, _stream(dev))
        self.items = pr_phi_plan_items(self.handle)

    def perm(self) -> torch.Tensor:
        """plan position -> user index (int64 device tensor)."""
        out = torch.empty(self.M, dtype=torch.int32, device=self.device)
        pr_phi_plan_perm_copy(self.handle, out, _stream(self.device))
        return out.to(torch.int64)

    def apply(self, x, y=None):
        y = torch.empty(self.M, dtype=self.cdtype, device=self.device) if y is None else y
        pr_phi_apply(self.handle, x, y)
        return y

    def adjoint(self, y, x=None):
        x = torch.empty((self.n, self.n), dtype=self.rdtype, device=self.device) if x is None else x
        pr_phi_adjoint(self.handle, y, x)
        return x

    def norm(self, iters=100, rtol=0.0):
        vis = torch.empty(max(self.M, 1), dtype=self.cdtype, device=self.device)
        return pr_phi_norm(self.handle, iters, rtol, vis)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            _lib.pr_phi_plan_destroy(h)
            self.handle = None


class PsiPlan:
    """SARA dictionary plan (see pr_psi_plan_create)."""

    def __init__(self, n, levels, mask=0x1FF, prec=PR_F32, device="cuda"):
        self.n, self.levels, self.mask, self.prec = n, levels, mask, prec
        self.rdtype = torch.float32 if prec == PR_F32 else torch.float64
        pb, sb = pr_psi_plan_sizes(n, levels, mask, prec)
        self.device = torch.device(device)
        self.persistent = _workspace(pb, self.device)
        self.scratch = _workspace(sb, self.device)
        self.handle = pr_psi_plan_create(n, levels, mask, prec, self.persistent, self.scratch, _stream(self.device))
        self.nb = pr_psi_plan_bases(self.handle)

    def adjoint(self, x, alpha=None):
        alpha = torch.empty((self.nb, self.n, self.n), dtype=self.rdtype, device=self.device) if alpha is None else alpha
        pr_psi_adjoint(self.handle, x, alpha)
        return alpha

    def apply(self, alpha, x=None):
        x = torch.empty((self.n, self.n), dtype=self.rdtype, device=self.device) if x is None else x
        pr_psi_apply(self.handle, alpha, x)
        return x

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            _lib.pr_psi_plan_destroy(h)
            self.handle = None


def pr_fista_workspace_size(phi, psi) -> int:
    v = _SZ()
    _check(lib().pr_fista_workspace_size(phi, psi, C.byref(v)))
    return v.value


def pr_fista_solve(phi, psi, y, params: "pr_fista_params", x, workspace, want_report=True, stream=None):
    rep = pr_admm_report()
    _check(lib().pr_fista_solve(phi, psi, _ptr(y), C.byref(params), _ptr(x), _ptr(workspace),
                                C.byref(rep) if want_report else None, stream if stream is not None else _stream()))
    return rep if want_report else None


def pr_pd_workspace_size(phi, psi) -> int:
    v = _SZ()
    _check(lib().pr_pd_workspace_size(phi, psi, C.byref(v)))
    return v.value


def pr_pd_solve(phi, psi, y, params: "pr_pd_params", x, workspace, want_report=True, stream=None):
    rep = pr_admm_report()
    _check(lib().pr_pd_solve(phi, psi, _ptr(y), C.byref(params), _ptr(x), _ptr(workspace),
                             C.byref(rep) if want_report else None, stream if stream is not None else _stream()))
    return rep if want_report else None


def admm_params(eps, gamma, iters=50, inner_iters=1, rho=0.5, varrho=1.0, eta=1.0, rel_tol=0.0, op_norm=0.0,
                gamma_factor=0.0, norm_iters=0):
    return pr_admm_params(iters, inner_iters, eps, gamma, rho, varrho, eta, rel_tol, op_norm, gamma_factor,
                          norm_iters)


def admm_solve(phi: PhiPlan, psi: PsiPlan, y, params: pr_admm_params, x0=None, want_report=True):
    """Run Algorithm 1; returns (x, report). x is in normalised-operator units."""
    ws = _workspace(pr_admm_workspace_size(phi.handle, psi.handle), phi.device)
    x = torch.zeros((phi.n, phi.n), dtype=phi.rdtype, device=phi.device) if x0 is None else x0.clone()
    rep = pr_admm_solve(phi.handle, psi.handle, y, params, x, ws, want_report)
    return x, rep


def fista_params(gamma, lam, iters=50, inner_iters=1, eta=1.0, op_norm=0.0, gamma_factor=0.0, norm_iters=0):
    return pr_fista_params(iters, inner_iters, gamma, lam, eta, op_norm, gamma_factor, norm_iters)


def fista_solve(phi: PhiPlan, psi: PsiPlan, y, params: pr_fista_params, x0=None, want_report=True):
    """Run FISTA for the MAP problem; returns (x, report). x is in normalised-operator units."""
    ws = _workspace(pr_fista_workspace_size(phi.handle, psi.handle), phi.device)
    x = torch.zeros((phi.n, phi.n), dtype=phi.rdtype, device=phi.device) if x0 is None else x0.clone()
    rep = pr_fista_solve(phi.handle, psi.handle, y, params, x, ws, want_report)
    return x, rep


def pd_params(gamma, tau=0.5, sigma=1.0, theta=1.0, iters=50, misfit=None, eps=0.0, inner_iters=1, eta=1.0,
              op_norm=0.0, gamma_factor=0.0, norm_iters=0):
    """misfit: PR_PD_BALL (default) or PR_PD_L2."""
    return pr_pd_params(iters, inner_iters, PR_PD_BALL if misfit is None else misfit, eps, gamma, tau, sigma, theta,
                        eta, op_norm, gamma_factor, norm_iters)


def pd_solve(phi: PhiPlan, psi: PsiPlan, y, params: pr_pd_params, x0=None, want_report=True):
    """Run the Primal-Dual algorithm; returns (x, report). x is in normalised-operator units."""
    ws = _workspace(pr_pd_workspace_size(phi.handle, psi.handle), phi.device)
    x = torch.zeros((phi.n, phi.n), dtype=phi.rdtype, device=phi.device) if x0 is None else x0.clone()
    rep = pr_pd_solve(phi.handle, psi.handle, y, params, x, ws, want_report)
    return x, rep


def pr_reweight_workspace_size(phi, psi) -> int:
    v = _SZ()
    _check(lib().pr_reweight_workspace_size(phi, psi, C.byref(v)))
    return v.value


def pr_admm_reweighted_solve(phi, psi, y, params: pr_admm_params, rw: pr_reweight_params, x, workspace,
                             want_report=True, stream=None):
    rep = pr_admm_report()
    _check(lib().pr_admm_reweighted_solve(phi, psi, _ptr(y), C.byref(params), C.byref(rw), _ptr(x), _ptr(workspace),
                                          C.byref(rep) if want_report else None,
                                          stream if stream is not None else _stream()))
    return rep if want_report else None


def admm_reweighted_solve(phi: PhiPlan, psi: PsiPlan, y, params: pr_admm_params, rounds: int, delta0: float,
                          beta: float, x0=None, want_report=True):
    """Reweighted analysis l1 around Algorithm 1; returns (x, report of the last round)."""
    ws = _workspace(pr_reweight_workspace_size(phi.handle, psi.handle), phi.device)
    x = torch.zeros((phi.n, phi.n), dtype=phi.rdtype, device=phi.device) if x0 is None else x0.clone()
    rep = pr_admm_reweighted_solve(phi.handle, psi.handle, y, params, pr_reweight_params(rounds, delta0, beta), x, ws,
                                   want_report)
    return x, rep


class Balls:
    """Sections of a plan's visibilities for the local l2-ball constraints.
    section: int32 device tensor [M] in plan order (copied by the library)."""

    def __init__(self, phi: PhiPlan, section, nsec: int):
        L = lib()
        assert section.dtype == torch.int32 and section.numel() == phi.M and section.is_contiguous()
        pb, sb = _SZ(), _SZ()
        _check(L.pr_balls_sizes(phi.M, nsec, C.byref(pb), C.byref(sb)))
        self.persistent = _workspace(pb.value, phi.device)
        scratch = _workspace(sb.value, phi.device)
        self.nsec, self.M = nsec, phi.M
        h = _VP()
        _check(L.pr_balls_create(phi.M, nsec, _ptr(section), _ptr(self.persistent), pb.value, _ptr(scratch),
                                 sb.value, _stream(), C.byref(h)))
        self.handle = h.value

    def norms(self):
        out = (_D * self.nsec)()
        _check(lib().pr_balls_norms(self.handle, out, _stream()))
        return np.array(out[:], dtype=np.float64)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            _lib.pr_balls_destroy(h)
            self.handle = None


def pr_admm_local_solve(phi, psi, balls, y, params: pr_admm_params, eps, x, workspace, want_report=True,
                        stream=None):
    e = np.ascontiguousarray(eps, dtype=np.float64)
    rep = pr_admm_report()
    _check(lib().pr_admm_local_solve(phi, psi, balls, _ptr(y), C.byref(params), e.ctypes.data_as(C.POINTER(_D)),
                                     _ptr(x), _ptr(workspace), C.byref(rep) if want_report else None,
                                     stream if stream is not None else _stream()))
    return rep if want_report else None


def admm_local_solve(phi: PhiPlan, psi: PsiPlan, balls: Balls, y, params: pr_admm_params, eps, x0=None,
                     want_report=True):
    """Algorithm 1 with one l2 ball per section (radii ``eps``, one per section); returns (x, report)."""
    ws = _workspace(pr_admm_workspace_size(phi.handle, psi.handle), phi.device)
    x = torch.zeros((phi.n, phi.n), dtype=phi.rdtype, device=phi.device) if x0 is None else x0.clone()
    assert np.size(eps) == balls.nsec
    rep = pr_admm_local_solve(phi.handle, psi.handle, balls.handle, y, params, eps, x, ws, want_report)
    return x, rep


class Batch:
    """Independent solves stepped together (see pr_batch_create). Keeps the
    members' plans, data and workspaces alive while they are members."""

    def __init__(self, max_members=64, nstreams=4):
        self.handle = pr_batch_create(max_members, nstreams)
        self.max_members = max_members
        self._keep = {}

    def add(self, phi: PhiPlan, psi: PsiPlan, y, params: pr_admm_params, x0=None) -> int:
        ws = _workspace(pr_admm_workspace_size(phi.handle, psi.handle), phi.device)
        x = torch.zeros((phi.n, phi.n), dtype=phi.rdtype, device=phi.device) if x0 is None else x0.clone()
        slot = pr_batch_add(self.handle, phi.handle, psi.handle, y, x, params, ws)
        self._keep[slot] = (phi, psi, y, x, ws)
        return slot

    def x(self, slot: int):
        return self._keep[slot][3]

    def remove(self, slot: int):
        pr_batch_remove(self.handle, slot)
        self._keep.pop(slot, None)

    def step(self, iters=1, use_graph=True):
        pr_batch_step(self.handle, iters, use_graph)

    def fuse(self, device="cuda"):
        """One launch per operator stage for pr_batch_phi_apply / _adjoint over
        the current members (the workspace is kept by this object)."""
        self._fuse_ws = _workspace(max(256, pr_batch_fuse_bytes(self.handle)), torch.device(device))
        pr_batch_fuse(self.handle, self._fuse_ws)

    def report(self, slot: int) -> pr_admm_report:
        return pr_batch_report(self.handle, slot)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            _lib.pr_batch_destroy(h)
            self.handle = None


def job_desc(n, uv, y, params: pr_admm_params, w=None, J=4, D=2000, levels=3, mask=0x1FF, tile=0,
             interp=0) -> pr_job_desc:
    prec = _prec_of(uv.dtype)
    return pr_job_desc(n, J, D, tile, levels, mask, prec, uv.shape[0], _ptr(uv), _ptr(w), _ptr(y), params, interp)


class Server:
    """Continuous-batching request loop (see pr_server_create); the arena is
    one device tensor owned by this object."""

    def __init__(self, arena_bytes, max_active=64, nstreams=4, device="cuda"):
        self.arena = _workspace(arena_bytes, torch.device(device))
        self.handle = pr_server_create(self.arena, int(arena_bytes), max_active, nstreams)
        self._inputs = {}

    def submit(self, desc: pr_job_desc, keep=()) -> int:
        jid = pr_server_submit(self.handle, desc)
        self._inputs[jid] = keep          # uv / w / y tensors, alive until admission
        return jid

    def tick(self):
        q, r, f = pr_server_tick(self.handle)
        for jid in [j for j in self._inputs if pr_server_job_state(self.handle, j)[0] >= 1]:
            self._inputs.pop(jid)
        return q, r, f

    def state(self, jid: int) -> int:
        return pr_server_job_state(self.handle, jid)[0]

    def fetch(self, jid: int, n: int, dtype=torch.float32, want_report=True):
        x = torch.empty((n, n), dtype=dtype, device=self.arena.device)
        rep = pr_server_fetch(self.handle, jid, x, want_report)
        return x, rep

    def cancel(self, jid: int):
        pr_server_cancel(self.handle, jid)
        self._inputs.pop(jid, None)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            _lib.pr_server_destroy(h)
            self.handle = None
