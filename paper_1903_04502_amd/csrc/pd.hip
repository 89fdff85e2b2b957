// Primal-Dual splitting, Section "Primal-Dual Splitting" and Algorithm
// "Primal-Dual Algorithm", for min f(Phi x) + gamma ||Psi^dagger x||_1 + iota_R+(x)
// with the normalised operator:
//   z_{k+1} = prox_{sigma f*}(z_k + sigma Phi xh_k),
//   x_{k+1} = prox_{tau g}(x_k - tau Phi^dagger z_{k+1}),
//   xh_{k+1} = x_{k+1} + theta (x_{k+1} - x_k).
// The dual is kept scaled, s = z / sigma. By Moreau's decomposition,
// s_{k+1} = (1 - kappa) t with t = s_k + Phi xh_k - y, where kappa =
// min(1, eps / ||t||) for f the indicator of the l2 ball of radius eps, and
// kappa = sigma / (1 + sigma) for f = 1/2 ||. - y||^2. That is the multiplier
// update of the solver's fused kernels with varrho = 1; the gridding grids
// s_{k+1} itself, and the gradient step is x_k - tau sigma Phi^dagger s_{k+1}.
// The prox of tau g is the warm-started DualFB of Algorithm 1 with threshold
// tau gamma. One extrapolation pass per iteration.
#include <cmath>

#include "admm.hpp"
#include "ops.hpp"

namespace pr {
namespace {

pr_admm_params as_admm(const pr_pd_params& f) {
  pr_admm_params p{};
  p.iters = f.iters;
  p.inner_iters = f.inner_iters;
  p.eps = f.misfit == PR_PD_BALL ? f.eps : INFINITY;
  p.gamma = f.gamma;
  p.rho = f.tau * f.sigma;
  p.varrho = 1.0;
  p.eta = f.eta;
  p.rel_tol = 0.0;
  p.op_norm = f.op_norm;
  p.gamma_factor = f.gamma_factor;
  p.norm_iters = f.norm_iters;
  return p;
}

int pd_check_params(const pr_pd_params* p) {
  if (p->iters < 0) { set_error("iters < 0"); return PR_EINVAL; }
  if (p->inner_iters < 1) { set_error("inner_iters < 1"); return PR_EINVAL; }
  if (p->misfit != PR_PD_BALL && p->misfit != PR_PD_L2) { set_error("misfit must be PR_PD_BALL or PR_PD_L2"); return PR_EINVAL; }
  if (p->misfit == PR_PD_BALL && !(p->eps >= 0)) { set_error("eps must be >= 0"); return PR_EINVAL; }
  if (!(p->gamma > 0) && !(p->gamma_factor > 0)) {
    set_error("gamma must be > 0, or gamma <= 0 with gamma_factor > 0");
    return PR_EINVAL;
  }
  if (!(p->tau > 0) || !(p->sigma > 0) || !(p->eta > 0)) { set_error("tau, sigma and eta must be > 0"); return PR_EINVAL; }
  if (!(p->theta >= 0) || !(p->theta <= 1)) { set_error("theta must be in [0, 1]"); return PR_EINVAL; }
  return PR_OK;
}

int pd_solve(pr_phi_plan_t* phi, pr_psi_plan_t* psi, const void* y, const pr_pd_params& pp, void* x, void* ws,
             pr_admm_report* rep, hipStream_t s) {
  AdmmJob j;
  void* xh = nullptr;
  PR_TRY(admm_job_init(&j, phi, psi, y, x, ws, as_admm(pp), s));
  accel_layout(phi, psi, ws, &j.w, &xh);
  PR_TRY(admm_device_setup(&j, s));
  const int prec = phi->prec;
  const int64_t n2 = static_cast<int64_t>(phi->n) * phi->n;
  double* sums = j.w.sums;
  // prox threshold tau * gamma (on the device when gamma is)
  const double* thr_dev = nullptr;
  if (j.device_gamma) {
    PR_TRY(scale_scalar(sums + kSumGamma, pp.tau, sums + kSumGammaStep, s));
    thr_dev = sums + kSumGammaStep;
  }
  PR_TRY(copy_real(xh, x, n2, prec, s));
  AdmmVis av{};
  av.y = y;
  av.s = j.w.s;                 // scaled dual, zero at the start
  av.t = j.w.t;
  av.sums = sums + kSumBall;
  av.eps = j.prm.eps;
  av.varrho = 1.0;
  av.scale_dev = sums + kSumScale;
  av.vr_coef = 0.0;             // grid s_{k+1}
  av.kappa_fixed = pp.misfit == PR_PD_L2 ? pp.sigma / (1.0 + pp.sigma) : -1.0;
  const double rho = pp.tau * pp.sigma;
  for (int it = 0; it < pp.iters; ++it) {
    PR_TRY(phi_fzs(phi, xh, s));
    PR_TRY(phi_gw_admm(phi, av, 1.0, s));
    PR_TRY(phi_gw_adjoint_admm(phi, av, 1.0, s));
    PR_TRY(phi_fzs_adjoint_step(phi, x, rho, j.w.xt, j.w.zbar, s));
    for (int k = 0; k < pp.inner_iters; ++k) {
      PR_TRY(psi_dual_update(psi, j.w.zbar, 0, j.w.d, pp.tau * pp.gamma, pp.eta, s, thr_dev));
      const bool last = k == pp.inner_iters - 1;
      PR_TRY(psi_synthesis_step(psi, j.w.d, j.w.xt, last ? j.w.xb : j.w.zbar, last ? x : nullptr, j.w.partials,
                                sums + kSumVar, s));
    }
    PR_TRY(extrapolate(x, j.w.xb, xh, n2, prec, pp.theta, s));
    ++j.iters_done;
  }
  if (rep) PR_TRY(admm_report(&j, rep, s));
  return PR_OK;
}

}  // namespace
}  // namespace pr

using namespace pr;

extern "C" {

int pr_pd_workspace_size(pr_phi_plan phi, pr_psi_plan psi, size_t* bytes) {
  clear_error();
  PR_NONNULL(phi);
  PR_NONNULL(psi);
  PR_NONNULL(bytes);
  PR_TRY(admm_check_plans(phi, psi));
  *bytes = accel_layout(phi, psi, nullptr, nullptr, nullptr);
  return PR_OK;
}

int pr_pd_solve(pr_phi_plan phi, pr_psi_plan psi, const void* y, const pr_pd_params* params, void* x,
                void* workspace, pr_admm_report* rep, void* stream) {
  clear_error();
  PR_NONNULL(phi);
  PR_NONNULL(psi);
  PR_NONNULL(y);
  PR_NONNULL(params);
  PR_NONNULL(x);
  if (!workspace || !aligned256(workspace)) { set_error("workspace must be non-NULL and 256-byte aligned"); return PR_EWORKSPACE; }
  PR_TRY(admm_check_plans(phi, psi));
  PR_TRY(pd_check_params(params));
  PR_TRY(check_sticky());
  return pd_solve(phi, psi, y, *params, x, workspace, rep, as_stream(stream));
}

}  // extern "C"
