"""The C ABI library loads, exports every declared symbol, and rejects bad
arguments with the documented codes before touching a GPU (CPU only)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "purimi.h")


@pytest.fixture(scope="module")
def P():
    from paper_1903_04502_amd import purimi
    if not os.path.exists(purimi.LIB_PATH):
        from paper_1903_04502_amd import build
        build.build(verbose=False)
    purimi.lib()
    return purimi


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pr_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported_and_bound(P):
    names = declared_functions()
    assert len(names) >= 20
    h = C.CDLL(P.LIB_PATH)
    for name in names:
        assert hasattr(h, name), name
    assert sorted(P.exported_symbols()) == names


def test_version_and_error_text(P):
    assert P.pr_version() >= 10000
    with pytest.raises(P.PrError) as e:
        P.pr_phi_plan_sizes(P.pr_phi_desc(100, 2, 4, 2000, 10, 0, 0))
    assert e.value.code == P.PR_EINVAL
    assert "power of two" in P.pr_last_error()


@pytest.mark.parametrize("field,value,code", [
    ("n", 4, 1), ("n", 8192, 1), ("oversample", 3, 4), ("J", 5, 1), ("J", 10, 1),
    ("D", 0, 1), ("M", -1, 1), ("M", 1 << 31, 1), ("M", (1 << 31) - (1 << 20) + 1, 1), ("prec", 2, 1),
    ("tile", 12, 1),
])
def test_phi_descriptor_validation(P, field, value, code):
    d = P.pr_phi_desc(64, 2, 4, 2000, 1000, 0, 0)
    setattr(d, field, value)
    with pytest.raises(P.PrError) as e:
        P.pr_phi_plan_sizes(d)
    assert e.value.code == code


def test_tiles_that_do_not_fit_lds_are_refused(P):
    with pytest.raises(P.PrError) as e:
        P.pr_phi_plan_sizes(P.pr_phi_desc(256, 2, 4, 2000, 1000, 1, 32))
    assert e.value.code == P.PR_EUNSUPPORTED
    with pytest.raises(P.PrError) as e:
        P.pr_phi_plan_sizes(P.pr_phi_desc(256, 2, 6, 2000, 1000, 0, 32))
    assert e.value.code == P.PR_EUNSUPPORTED
    assert P.pr_phi_plan_sizes(P.pr_phi_desc(256, 2, 2, 2000, 1000, 0, 32))[0] > 0
    assert P.pr_phi_plan_sizes(P.pr_phi_desc(256, 2, 8, 2000, 1000, 1, 8))[0] > 0


def test_phi_sizes_scale_with_the_problem(P):
    small = P.pr_phi_plan_sizes(P.pr_phi_desc(64, 2, 4, 2000, 8192, 0, 0))
    big = P.pr_phi_plan_sizes(P.pr_phi_desc(64, 2, 4, 2000, 81920, 0, 0))
    f64 = P.pr_phi_plan_sizes(P.pr_phi_desc(64, 2, 4, 2000, 8192, 1, 0))
    assert all(v > 0 and v % 256 == 0 for v in small + big + f64)
    assert big[0] > small[0] and f64[0] > small[0]
    # persistent part holds at least the stored taps (or uv), w and the
    # permutation: 12 B per visibility in FP32 with stored taps, else 16 B
    assert big[0] >= 12 * 81920
    assert P.pr_phi_plan_sizes(P.pr_phi_desc(64, 2, 4, 2000, 81920, 0, 0, 2))[0] >= 16 * 81920


def test_workspace_and_null_checks(P):
    L = P.lib()
    d = P.pr_phi_desc(64, 2, 4, 2000, 10, 0, 0)
    h = C.c_void_p()
    assert L.pr_phi_plan_create(C.byref(d), 256, None, None, 256, None, C.byref(h)) == P.PR_EWORKSPACE
    assert L.pr_phi_plan_create(C.byref(d), 256, None, 256 + 8, 512, None, C.byref(h)) == P.PR_EWORKSPACE
    assert L.pr_phi_plan_create(C.byref(d), None, None, 256, 512, None, C.byref(h)) == P.PR_EINVAL
    assert L.pr_phi_apply(None, 256, 256, None) == P.PR_EINVAL
    assert L.pr_phi_adjoint(None, 256, 256, None) == P.PR_EINVAL
    assert L.pr_phi_norm(None, 10, 0.0, 256, None, None) == P.PR_EINVAL


def test_prox_argument_checks(P):
    L = P.lib()
    assert L.pr_prox_l1(256, 256, -1, 0, 0, 0.1, None) == P.PR_EINVAL
    assert L.pr_prox_l1(256, 256, 10, 0, 7, 0.1, None) == P.PR_EINVAL
    assert L.pr_prox_l1(256, 256, 10, 0, 0, -0.1, None) == P.PR_EINVAL
    assert L.pr_prox_l1(None, None, 10, 0, 0, 0.1, None) == P.PR_EINVAL
    assert L.pr_proj_l2ball(256, 256, 256, 10, 0, 1.0, 256 + 4, None, None) == P.PR_EWORKSPACE
    assert L.pr_proj_l2ball(256, 256, 256, 10, 0, -1.0, 256, None, None) == P.PR_EINVAL
    assert P.pr_proj_l2ball_scratch_bytes(1000) >= 8 * 1024


def test_psi_and_admm_checks(P):
    L = P.lib()
    with pytest.raises(P.PrError):
        P.pr_psi_plan_sizes(96, 3, 0x1FF, 0)
    with pytest.raises(P.PrError):
        P.pr_psi_plan_sizes(64, 7, 0x1FF, 0)
    with pytest.raises(P.PrError):
        P.pr_psi_plan_sizes(64, 3, 0x200, 0)
    pb, sb = P.pr_psi_plan_sizes(64, 3, 0x1FF, 0)
    assert pb > 0 and sb >= 8 * 64 * 64 * 4
    prm = P.admm_params(1.0, 0.1)
    rep = P.pr_admm_report()
    assert L.pr_admm_solve(None, None, None, C.byref(prm), None, None, C.byref(rep), None) == P.PR_EINVAL
    assert L.pr_psi_apply(None, 256, 256, None) == P.PR_EINVAL


def test_interp_mode_is_validated(P):
    assert P.pr_phi_plan_sizes(P.pr_phi_desc(64, 2, 4, 2000, 1000, 0, 0, 1))[0] > 0
    assert P.pr_phi_plan_sizes(P.pr_phi_desc(64, 2, 4, 2000, 1000, 0, 0, 2))[0] > 0
    for bad in (-1, 3):
        with pytest.raises(P.PrError) as e:
            P.pr_phi_plan_sizes(P.pr_phi_desc(64, 2, 4, 2000, 1000, 0, 0, bad))
        assert e.value.code == P.PR_EINVAL


def test_visibility_storage_follows_the_lookup(P):
    """Nearest-sample FP32 plans with tiles <= 16 and D <= 2047 keep 8 bytes
    per visibility (tap word, w) instead of the 12-byte (u, v, w) triple; every
    other plan keeps the triples (interp 2 asks for them explicitly)."""
    M = 100000
    size = lambda prec=0, tile=0, interp=0, D=2000: P.pr_phi_plan_sizes(
        P.pr_phi_desc(256, 2, 4, D, M, prec, tile, interp))[0]
    words, triples = size(), size(interp=2)
    assert triples - words == pytest.approx(4 * M, abs=4096)
    assert size(tile=8) < size(tile=8, interp=2)
    assert size(tile=32) - size(tile=32, interp=2) == 0           # tile 32: triples
    assert size(interp=1) == size(interp=2)                       # first order: triples
    assert size(D=2048) - size(D=2048, interp=2) == 0             # 12-bit sample field
    assert size(D=2047) < size(D=2047, interp=2)
    assert size(prec=1) == size(prec=1, interp=2)                 # FP64: triples


def test_fista_argument_checks(P):
    L = P.lib()
    rep = P.pr_admm_report()
    good = P.fista_params(0.1, 1.0)
    assert L.pr_fista_solve(None, None, None, C.byref(good), None, None, C.byref(rep), None) == P.PR_EINVAL
    sz = C.c_size_t()
    assert L.pr_fista_workspace_size(None, None, C.byref(sz)) == P.PR_EINVAL
    assert P.pr_fista_params._fields_[3][0] == "lambda_"


def test_balls_argument_checks(P):
    L = P.lib()
    pb, sb = C.c_size_t(), C.c_size_t()
    assert L.pr_balls_sizes(1000, 0, C.byref(pb), C.byref(sb)) == P.PR_EINVAL
    assert L.pr_balls_sizes(-1, 4, C.byref(pb), C.byref(sb)) == P.PR_EINVAL
    assert L.pr_balls_sizes(1 << 31, 4, C.byref(pb), C.byref(sb)) == P.PR_EINVAL
    assert L.pr_balls_sizes((1 << 31) - (1 << 20) + 1, 4, C.byref(pb), C.byref(sb)) == P.PR_EINVAL
    assert L.pr_balls_sizes(1000, 4, C.byref(pb), C.byref(sb)) == P.PR_OK
    assert pb.value >= 8 * 1000 and sb.value >= 16 * 1000
    h = C.c_void_p()
    assert L.pr_balls_create(1000, 4, 256, None, pb.value, 256, sb.value, None, C.byref(h)) == P.PR_EWORKSPACE
    assert L.pr_balls_create(1000, 4, 256, 256, pb.value - 256, 256, sb.value, None, C.byref(h)) == P.PR_EWORKSPACE
    assert L.pr_balls_create(1000, 4, None, 256, pb.value, 256, sb.value, None, C.byref(h)) == P.PR_EINVAL
    rep = P.pr_admm_report()
    assert L.pr_admm_local_solve(None, None, None, None, None, None, None, None, C.byref(rep), None) == P.PR_EINVAL


def test_largest_visibility_count_is_accepted(P):
    """The bound is 2^31 - 2^20 visibilities: positions plus any per-item
    offset stay below 2^31, and products with positions are 64-bit."""
    big = (1 << 31) - (1 << 20)
    pb, sb = P.pr_phi_plan_sizes(P.pr_phi_desc(2048, 2, 4, 2000, big, 0, 0))
    assert pb >= 12 * big   # stored taps (4 B), w (4 B), permutation (4 B) per visibility
    L = P.lib()
    p2, s2 = C.c_size_t(), C.c_size_t()
    assert L.pr_balls_sizes(big, 4, C.byref(p2), C.byref(s2)) == P.PR_OK


def test_checkpoint_argument_checks(P):
    L = P.lib()
    prm = P.admm_params(1.0, 0.1)
    rep = P.pr_admm_report()
    sz = C.c_size_t()
    assert L.pr_admm_state_bytes(None, None, C.byref(sz)) == P.PR_EINVAL
    assert L.pr_admm_state_export(None, None, 256, 256, 256, None) == P.PR_EINVAL
    assert L.pr_admm_state_import(None, None, 256, 256, 256, None) == P.PR_EINVAL
    assert L.pr_admm_resume(None, None, None, C.byref(prm), None, None, C.byref(rep), None) == P.PR_EINVAL
    assert L.pr_phi_norm(None, 10, -1.0, 256, None, None) == P.PR_EINVAL


_LAYOUT_C = r"""
#include <stddef.h>
#include <stdio.h>
#include "purimi.h"
#define F(T, f) printf(#T " " #f " %zu %zu\n", offsetof(T, f), sizeof(((T*)0)->f));
#define S(T) printf(#T " __size__ %zu 0\n", sizeof(T));
int main(void) {
  S(pr_phi_desc) F(pr_phi_desc, n) F(pr_phi_desc, oversample) F(pr_phi_desc, J) F(pr_phi_desc, D)
  F(pr_phi_desc, M) F(pr_phi_desc, prec) F(pr_phi_desc, tile) F(pr_phi_desc, interp)
  S(pr_admm_params) F(pr_admm_params, iters) F(pr_admm_params, inner_iters) F(pr_admm_params, eps)
  F(pr_admm_params, gamma) F(pr_admm_params, rho) F(pr_admm_params, varrho) F(pr_admm_params, eta)
  F(pr_admm_params, rel_tol) F(pr_admm_params, op_norm) F(pr_admm_params, gamma_factor)
  F(pr_admm_params, norm_iters)
  S(pr_admm_report) F(pr_admm_report, iters_done) F(pr_admm_report, rel_var) F(pr_admm_report, resid_norm)
  F(pr_admm_report, l1_norm) F(pr_admm_report, op_norm) F(pr_admm_report, nonfinite)
  S(pr_reweight_params) F(pr_reweight_params, rounds) F(pr_reweight_params, delta0) F(pr_reweight_params, beta)
  S(pr_fista_params) F(pr_fista_params, iters) F(pr_fista_params, inner_iters) F(pr_fista_params, gamma)
  F(pr_fista_params, lambda) F(pr_fista_params, eta) F(pr_fista_params, op_norm)
  F(pr_fista_params, gamma_factor) F(pr_fista_params, norm_iters)
  S(pr_pd_params) F(pr_pd_params, iters) F(pr_pd_params, inner_iters) F(pr_pd_params, misfit)
  F(pr_pd_params, eps) F(pr_pd_params, gamma) F(pr_pd_params, tau) F(pr_pd_params, sigma)
  F(pr_pd_params, theta) F(pr_pd_params, eta) F(pr_pd_params, op_norm) F(pr_pd_params, gamma_factor)
  F(pr_pd_params, norm_iters)
  S(pr_job_desc) F(pr_job_desc, n) F(pr_job_desc, J) F(pr_job_desc, D) F(pr_job_desc, tile)
  F(pr_job_desc, levels) F(pr_job_desc, basis_mask) F(pr_job_desc, prec) F(pr_job_desc, M) F(pr_job_desc, uv)
  F(pr_job_desc, w) F(pr_job_desc, y) F(pr_job_desc, params) F(pr_job_desc, interp)
  return 0;
}
"""


def test_ctypes_structs_match_the_c_header(P, tmp_path):
    """Every struct the binding mirrors has the header's size and field
    offsets, as laid out by the host C compiler."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    src = tmp_path / "layout.c"
    src.write_text(_LAYOUT_C)
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    rename = {"lambda": "lambda_"}
    checked = 0
    for line in out:
        if not line.strip():
            continue
        tname, field, off, size = line.split()
        T = getattr(P, tname)
        if field == "__size__":
            assert C.sizeof(T) == int(off), tname
        else:
            f = getattr(T, rename.get(field, field))
            assert (f.offset, f.size) == (int(off), int(size)), (tname, field)
        checked += 1
    assert checked >= 60
