// FISTA for the unconstrained (MAP) problem, Section "Forward-Backward
// Splitting" and Algorithm "FISTA":
//   x_{k+1} = prox_{lambda gamma g}(xh_k - lambda Re Phi^dagger (Phi xh_k - y)),
//   theta_{k+1} = (1 + sqrt(1 + 4 theta_k^2)) / 2,
//   xh_{k+1} = x_{k+1} + (theta_k - 1) / theta_{k+1} (x_{k+1} - x_k),
// with f = 1/2 ||y - Phi x||^2 for the normalised operator and
// g = ||Psi^dagger .||_1 + iota_R+, whose prox is the warm-started DualFB of
// Algorithm 1. Each iteration runs the solver's kernels: the degridding with
// the residual epilogue (t = Phi xh - y, FP64 ||t||^2), plain gridding of t,
// the adjoint FFT with the gradient-step epilogue, the DualFB launches, then
// one extrapolation pass. 1 / ||Phi|| and gamma stay on the device.
#include <cmath>

#include "admm.hpp"
#include "ops.hpp"

namespace pr {
namespace {

pr_admm_params as_admm(const pr_fista_params& f) {
  pr_admm_params p{};
  p.iters = f.iters;
  p.inner_iters = f.inner_iters;
  p.eps = INFINITY;           // no ball: the degridding epilogue only forms t = v - y
  p.gamma = f.gamma;
  p.rho = f.lambda;
  p.varrho = 1.0;
  p.eta = f.eta;
  p.rel_tol = 0.0;
  p.op_norm = f.op_norm;
  p.gamma_factor = f.gamma_factor;
  p.norm_iters = f.norm_iters;
  return p;
}

int fista_check_params(const pr_fista_params* p) {
  if (p->iters < 0) { set_error("iters < 0"); return PR_EINVAL; }
  if (p->inner_iters < 1) { set_error("inner_iters < 1"); return PR_EINVAL; }
  if (!(p->gamma > 0) && !(p->gamma_factor > 0)) {
    set_error("gamma must be > 0, or gamma <= 0 with gamma_factor > 0");
    return PR_EINVAL;
  }
  if (!(p->lambda > 0) || !(p->eta > 0)) { set_error("lambda and eta must be > 0"); return PR_EINVAL; }
  return PR_OK;
}

int fista_solve(pr_phi_plan_t* phi, pr_psi_plan_t* psi, const void* y, const pr_fista_params& fp, void* x, void* ws,
                pr_admm_report* rep, hipStream_t s) {
  AdmmJob j;
  void* xh = nullptr;
  PR_TRY(admm_job_init(&j, phi, psi, y, x, ws, as_admm(fp), s));
  accel_layout(phi, psi, ws, &j.w, &xh);
  PR_TRY(admm_device_setup(&j, s));
  const int prec = phi->prec;
  const int64_t n2 = static_cast<int64_t>(phi->n) * phi->n;
  double* sums = j.w.sums;
  // prox threshold gamma * lambda (on the device when gamma is)
  const double* thr_dev = nullptr;
  if (j.device_gamma) {
    PR_TRY(scale_scalar(sums + kSumGamma, fp.lambda, sums + kSumGammaStep, s));
    thr_dev = sums + kSumGammaStep;
  }
  PR_TRY(copy_real(xh, x, n2, prec, s));
  AdmmVis av{};
  av.y = y;
  av.s = nullptr;               // t = Phi xh - y
  av.t = j.w.t;
  av.sums = sums + kSumBall;
  av.eps = INFINITY;
  av.varrho = 1.0;
  av.scale_dev = sums + kSumScale;
  double theta = 1.0;
  for (int it = 0; it < fp.iters; ++it) {
    PR_TRY(phi_fzs(phi, xh, s));
    PR_TRY(phi_gw_admm(phi, av, 1.0, s));
    PR_TRY(phi_gw_adjoint_dev(phi, j.w.t, sums + kSumScale, s));
    PR_TRY(phi_fzs_adjoint_step(phi, xh, fp.lambda, j.w.xt, j.w.zbar, s));
    for (int k = 0; k < fp.inner_iters; ++k) {
      PR_TRY(psi_dual_update(psi, j.w.zbar, 0, j.w.d, fp.gamma * fp.lambda, fp.eta, s, thr_dev));
      const bool last = k == fp.inner_iters - 1;
      PR_TRY(psi_synthesis_step(psi, j.w.d, j.w.xt, last ? j.w.xb : j.w.zbar, last ? x : nullptr, j.w.partials,
                                sums + kSumVar, s));
    }
    const double theta_new = (1.0 + std::sqrt(1.0 + 4.0 * theta * theta)) / 2.0;
    PR_TRY(extrapolate(x, j.w.xb, xh, n2, prec, (theta - 1.0) / theta_new, s));
    theta = theta_new;
    ++j.iters_done;
  }
  if (rep) PR_TRY(admm_report(&j, rep, s));
  return PR_OK;
}

}  // namespace
}  // namespace pr

using namespace pr;

extern "C" {

int pr_fista_workspace_size(pr_phi_plan phi, pr_psi_plan psi, size_t* bytes) {
  clear_error();
  PR_NONNULL(phi);
  PR_NONNULL(psi);
  PR_NONNULL(bytes);
  PR_TRY(admm_check_plans(phi, psi));
  *bytes = accel_layout(phi, psi, nullptr, nullptr, nullptr);
  return PR_OK;
}

int pr_fista_solve(pr_phi_plan phi, pr_psi_plan psi, const void* y, const pr_fista_params* params, void* x,
                   void* workspace, pr_admm_report* rep, void* stream) {
  clear_error();
  PR_NONNULL(phi);
  PR_NONNULL(psi);
  PR_NONNULL(y);
  PR_NONNULL(params);
  PR_NONNULL(x);
  if (!workspace || !aligned256(workspace)) { set_error("workspace must be non-NULL and 256-byte aligned"); return PR_EWORKSPACE; }
  PR_TRY(admm_check_plans(phi, psi));
  PR_TRY(fista_check_params(params));
  PR_TRY(check_sticky());
  return fista_solve(phi, psi, y, *params, x, workspace, rep, as_stream(stream));
}

}  // extern "C"
