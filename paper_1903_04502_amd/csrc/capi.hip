// The extern "C" entry points declared in include/purimi.h: argument
// validation, workspace binding and dispatch to the stage implementations.
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "ops.hpp"
#include "phi.hpp"
#include "psi.hpp"
#include "admm.hpp"

namespace pr {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
}

void clear_error() { g_err[0] = '\0'; }

}  // namespace pr

using namespace pr;

extern "C" {

const char* pr_last_error(void) { return g_err; }

int pr_version(void) { return 10000; }

// --------------------------------------------------------------------------
// measurement operator
// --------------------------------------------------------------------------
int pr_phi_plan_sizes(const pr_phi_desc* desc, size_t* persistent_bytes, size_t* scratch_bytes) {
  clear_error();
  PR_TRY(phi_validate(desc));
  PR_NONNULL(persistent_bytes);
  PR_NONNULL(scratch_bytes);
  pr_phi_plan_t tmp;
  PR_TRY(phi_prepare(&tmp, desc));
  return phi_layout(&tmp, nullptr, nullptr, persistent_bytes, scratch_bytes);
}

int pr_phi_plan_create(const pr_phi_desc* desc, const void* uv, const void* w, void* persistent_ws,
                       void* scratch_ws, void* stream, pr_phi_plan* out) {
  clear_error();
  PR_TRY(phi_validate(desc));
  PR_NONNULL(out);
  if (desc->M > 0) PR_NONNULL(uv);
  if (!persistent_ws || !scratch_ws || !aligned256(persistent_ws) || !aligned256(scratch_ws)) {
    set_error("workspaces must be non-NULL and 256-byte aligned");
    return PR_EWORKSPACE;
  }
  PR_TRY(check_sticky());
  pr_phi_plan_t* p = new (std::nothrow) pr_phi_plan_t();
  if (!p) { set_error("out of host memory"); return PR_EINVAL; }
  int rc = phi_prepare(p, desc);
  if (rc == PR_OK) rc = phi_layout(p, persistent_ws, scratch_ws, nullptr, nullptr);
  if (rc == PR_OK) rc = phi_create(p, uv, w, as_stream(stream));
  if (rc != PR_OK) { delete p; return rc; }
  *out = p;
  return PR_OK;
}

int pr_phi_plan_destroy(pr_phi_plan plan) {
  clear_error();
  delete plan;
  return PR_OK;
}

int pr_phi_plan_perm(pr_phi_plan plan, const int32_t** perm) {
  clear_error();
  PR_NONNULL(plan);
  PR_NONNULL(perm);
  *perm = plan->perm;
  return PR_OK;
}

int pr_phi_plan_perm_copy(pr_phi_plan plan, int32_t* dst, void* stream) {
  clear_error();
  PR_NONNULL(plan);
  if (plan->M == 0) return PR_OK;
  PR_NONNULL(dst);
  PR_TRY(check_sticky());
  PR_TRY_HIP(hipMemcpyAsync(dst, plan->perm, plan->M * sizeof(int32_t), hipMemcpyDeviceToDevice,
                            as_stream(stream)));
  return PR_OK;
}

int pr_phi_plan_items(pr_phi_plan plan, int64_t* items) {
  clear_error();
  PR_NONNULL(plan);
  PR_NONNULL(items);
  *items = plan->nItems;
  return PR_OK;
}

int pr_phi_fzs(pr_phi_plan plan, const void* x, void* stream) {
  clear_error();
  PR_NONNULL(plan);
  PR_NONNULL(x);
  PR_TRY(check_sticky());
  return phi_fzs(plan, x, as_stream(stream));
}

int pr_phi_gw(pr_phi_plan plan, void* y, void* stream) {
  clear_error();
  PR_NONNULL(plan);
  if (plan->M > 0) PR_NONNULL(y);
  PR_TRY(check_sticky());
  return phi_gw(plan, y, 1.0, as_stream(stream));
}

int pr_phi_gw_adjoint(pr_phi_plan plan, const void* y, void* stream) {
  clear_error();
  PR_NONNULL(plan);
  if (plan->M > 0) PR_NONNULL(y);
  PR_TRY(check_sticky());
  return phi_gw_adjoint(plan, y, 1.0, as_stream(stream));
}

int pr_phi_grid_patches(pr_phi_plan plan, const void* y, void* stream) {
  clear_error();
  PR_NONNULL(plan);
  if (plan->M > 0) PR_NONNULL(y);
  PR_TRY(check_sticky());
  return phi_gw_adjoint_parts(plan, y, 1.0, 1, as_stream(stream));
}

int pr_phi_grid_merge(pr_phi_plan plan, void* stream) {
  clear_error();
  PR_NONNULL(plan);
  PR_TRY(check_sticky());
  return phi_gw_adjoint_parts(plan, nullptr, 1.0, 2, as_stream(stream));
}

int pr_phi_fzs_adjoint(pr_phi_plan plan, void* x, void* stream) {
  clear_error();
  PR_NONNULL(plan);
  PR_NONNULL(x);
  PR_TRY(check_sticky());
  return phi_fzs_adjoint(plan, x, as_stream(stream));
}

int pr_phi_apply(pr_phi_plan plan, const void* x, void* y, void* stream) {
  clear_error();
  PR_NONNULL(plan);
  PR_NONNULL(x);
  if (plan->M > 0) PR_NONNULL(y);
  PR_TRY(check_sticky());
  PR_TRY(phi_fzs(plan, x, as_stream(stream)));
  return phi_gw(plan, y, 1.0, as_stream(stream));
}

int pr_phi_adjoint(pr_phi_plan plan, const void* y, void* x, void* stream) {
  clear_error();
  PR_NONNULL(plan);
  PR_NONNULL(x);
  if (plan->M > 0) PR_NONNULL(y);
  PR_TRY(check_sticky());
  PR_TRY(phi_gw_adjoint(plan, y, 1.0, as_stream(stream)));
  return phi_fzs_adjoint(plan, x, as_stream(stream));
}

int pr_phi_norm(pr_phi_plan plan, int32_t iters, double rtol, void* vis_ws, double* norm, void* stream) {
  clear_error();
  PR_NONNULL(plan);
  PR_NONNULL(norm);
  if (plan->M > 0) PR_NONNULL(vis_ws);
  if (iters < 1) { set_error("iters = %d must be >= 1", iters); return PR_EINVAL; }
  if (!(rtol >= 0)) { set_error("rtol must be >= 0"); return PR_EINVAL; }
  PR_TRY(check_sticky());
  return phi_norm(plan, iters, rtol, vis_ws, norm, as_stream(stream));
}

// --------------------------------------------------------------------------
// SARA dictionary
// --------------------------------------------------------------------------
int pr_psi_plan_sizes(int32_t n, int32_t levels, uint32_t basis_mask, int32_t prec, size_t* persistent_bytes,
                      size_t* scratch_bytes) {
  clear_error();
  PR_NONNULL(persistent_bytes);
  PR_NONNULL(scratch_bytes);
  PR_TRY(psi_validate(n, levels, basis_mask, prec));
  pr_psi_plan_t tmp;
  psi_prepare(&tmp, n, levels, basis_mask, prec);
  return psi_layout(&tmp, nullptr, nullptr, persistent_bytes, scratch_bytes);
}

int pr_psi_plan_create(int32_t n, int32_t levels, uint32_t basis_mask, int32_t prec, void* persistent_ws,
                       void* scratch_ws, void* stream, pr_psi_plan* out) {
  clear_error();
  PR_TRY(psi_validate(n, levels, basis_mask, prec));
  PR_NONNULL(out);
  if (!persistent_ws || !scratch_ws || !aligned256(persistent_ws) || !aligned256(scratch_ws)) {
    set_error("workspaces must be non-NULL and 256-byte aligned");
    return PR_EWORKSPACE;
  }
  PR_TRY(check_sticky());
  pr_psi_plan_t* p = new (std::nothrow) pr_psi_plan_t();
  if (!p) { set_error("out of host memory"); return PR_EINVAL; }
  psi_prepare(p, n, levels, basis_mask, prec);
  int rc = psi_layout(p, persistent_ws, scratch_ws, nullptr, nullptr);
  if (rc == PR_OK) rc = psi_create(p, as_stream(stream));
  if (rc != PR_OK) { delete p; return rc; }
  *out = p;
  return PR_OK;
}

int pr_psi_plan_destroy(pr_psi_plan plan) {
  clear_error();
  delete plan;
  return PR_OK;
}

int pr_psi_plan_bases(pr_psi_plan plan, int32_t* nb) {
  clear_error();
  PR_NONNULL(plan);
  PR_NONNULL(nb);
  *nb = plan->nb;
  return PR_OK;
}

int pr_psi_filter(pr_psi_plan plan, int32_t k, double* taps) {
  clear_error();
  PR_NONNULL(plan);
  PR_NONNULL(taps);
  if (k < 1 || k > 8) { set_error("k = %d must be in 1..8", k); return PR_EINVAL; }
  std::memcpy(taps, plan->host_filters[k], sizeof(double) * 2 * k);
  return PR_OK;
}

int pr_psi_apply(pr_psi_plan plan, const void* alpha, void* x, void* stream) {
  clear_error();
  PR_NONNULL(plan);
  PR_NONNULL(alpha);
  PR_NONNULL(x);
  PR_TRY(check_sticky());
  return psi_synthesis(plan, alpha, x, as_stream(stream));
}

int pr_psi_adjoint(pr_psi_plan plan, const void* x, void* alpha, void* stream) {
  clear_error();
  PR_NONNULL(plan);
  PR_NONNULL(x);
  PR_NONNULL(alpha);
  PR_TRY(check_sticky());
  return psi_analysis(plan, x, alpha, as_stream(stream));
}

// --------------------------------------------------------------------------
// proximal operators
// --------------------------------------------------------------------------
int pr_prox_l1(const void* in, void* out, int64_t len, int32_t is_complex, int32_t prec, double lambda,
               void* stream) {
  clear_error();
  if (len < 0) { set_error("len < 0"); return PR_EINVAL; }
  if (len > 0) { PR_NONNULL(in); PR_NONNULL(out); }
  if (prec != PR_F32 && prec != PR_F64) { set_error("prec = %d", prec); return PR_EINVAL; }
  if (!(lambda >= 0)) { set_error("lambda must be >= 0"); return PR_EINVAL; }
  PR_TRY(check_sticky());
  return soft_threshold(in, out, len, is_complex, prec, lambda, as_stream(stream));
}

size_t pr_proj_l2ball_scratch_bytes(int64_t len) {
  (void)len;
  return ball_scratch_bytes();
}

int pr_proj_l2ball(const void* in, const void* center, void* out, int64_t len, int32_t prec, double eps,
                   void* scratch, double* dist, void* stream) {
  clear_error();
  if (len < 0) { set_error("len < 0"); return PR_EINVAL; }
  if (len > 0) { PR_NONNULL(in); PR_NONNULL(center); PR_NONNULL(out); }
  if (prec != PR_F32 && prec != PR_F64) { set_error("prec = %d", prec); return PR_EINVAL; }
  if (!(eps >= 0)) { set_error("eps must be >= 0"); return PR_EINVAL; }
  if (!scratch || !aligned256(scratch)) { set_error("scratch must be non-NULL and 256-byte aligned"); return PR_EWORKSPACE; }
  PR_TRY(check_sticky());
  return proj_l2ball(in, center, out, len, prec, eps, scratch, dist, as_stream(stream));
}

// --------------------------------------------------------------------------
// ADMM
// --------------------------------------------------------------------------
int pr_admm_workspace_size(pr_phi_plan phi, pr_psi_plan psi, size_t* bytes) {
  clear_error();
  PR_NONNULL(phi);
  PR_NONNULL(psi);
  PR_NONNULL(bytes);
  PR_TRY(admm_check_plans(phi, psi));
  *bytes = admm_layout(phi, psi, nullptr, nullptr);
  return PR_OK;
}

int pr_admm_solve(pr_phi_plan phi, pr_psi_plan psi, const void* y, const pr_admm_params* params, void* x,
                  void* workspace, pr_admm_report* rep, void* stream) {
  clear_error();
  PR_NONNULL(phi);
  PR_NONNULL(psi);
  PR_NONNULL(y);
  PR_NONNULL(params);
  PR_NONNULL(x);
  if (!workspace || !aligned256(workspace)) { set_error("workspace must be non-NULL and 256-byte aligned"); return PR_EWORKSPACE; }
  PR_TRY(admm_check_plans(phi, psi));
  PR_TRY(admm_check_params(params));
  PR_TRY(check_sticky());
  return admm_solve(phi, psi, y, *params, x, workspace, rep, as_stream(stream));
}

int pr_admm_resume(pr_phi_plan phi, pr_psi_plan psi, const void* y, const pr_admm_params* params, void* x,
                   void* workspace, pr_admm_report* rep, void* stream) {
  clear_error();
  PR_NONNULL(phi);
  PR_NONNULL(psi);
  PR_NONNULL(y);
  PR_NONNULL(params);
  PR_NONNULL(x);
  if (!workspace || !aligned256(workspace)) { set_error("workspace must be non-NULL and 256-byte aligned"); return PR_EWORKSPACE; }
  PR_TRY(admm_check_plans(phi, psi));
  PR_TRY(admm_check_params(params));
  PR_TRY(check_sticky());
  return admm_resume(phi, psi, y, *params, x, workspace, rep, as_stream(stream));
}

int pr_admm_state_bytes(pr_phi_plan phi, pr_psi_plan psi, size_t* bytes) {
  clear_error();
  PR_NONNULL(phi);
  PR_NONNULL(psi);
  PR_NONNULL(bytes);
  PR_TRY(admm_check_plans(phi, psi));
  *bytes = admm_state_bytes(phi, psi);
  return PR_OK;
}

int pr_admm_state_export(pr_phi_plan phi, pr_psi_plan psi, const void* workspace, const void* x, void* state,
                         void* stream) {
  clear_error();
  PR_NONNULL(phi);
  PR_NONNULL(psi);
  PR_NONNULL(x);
  PR_NONNULL(state);
  if (!workspace || !aligned256(workspace)) { set_error("workspace must be non-NULL and 256-byte aligned"); return PR_EWORKSPACE; }
  PR_TRY(admm_check_plans(phi, psi));
  PR_TRY(check_sticky());
  return admm_state_export(phi, psi, workspace, x, state, as_stream(stream));
}

int pr_admm_state_import(pr_phi_plan phi, pr_psi_plan psi, const void* state, void* workspace, void* x,
                         void* stream) {
  clear_error();
  PR_NONNULL(phi);
  PR_NONNULL(psi);
  PR_NONNULL(state);
  PR_NONNULL(x);
  if (!workspace || !aligned256(workspace)) { set_error("workspace must be non-NULL and 256-byte aligned"); return PR_EWORKSPACE; }
  PR_TRY(admm_check_plans(phi, psi));
  PR_TRY(check_sticky());
  return admm_state_import(phi, psi, state, workspace, x, as_stream(stream));
}

}  // extern "C"
