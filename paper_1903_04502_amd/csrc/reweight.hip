// Reweighted analysis l1 around Algorithm 1 (SARA reweighting, named in
// Section "Sparse Regularization"): round 0 solves the unweighted problem;
// each further round sets w_i = delta / (delta + |[Psi^dagger x]_i|) from the
// current x, with delta = delta0 beta^(r - 1) for round r, and solves the
// problem with the weighted norm sum_i w_i |[Psi^dagger x]_i| (DualFB
// thresholds gamma w_i) from the current x with s = 0 and d = 0. 1 / ||Phi||
// and gamma are formed once and stay on the device across rounds.
#include <cmath>

#include "admm.hpp"
#include "ops.hpp"

namespace pr {
namespace {

size_t reweight_layout(const pr_phi_plan_t* phi, const pr_psi_plan_t* psi, void* ws, AdmmWs* w, void** weights) {
  const size_t base = admm_layout(phi, psi, ws, w);
  const size_t rs = phi->prec == PR_F32 ? 4 : 8;
  const size_t nw = static_cast<size_t>(psi->nb) * phi->n * phi->n;
  if (weights) *weights = ws ? static_cast<char*>(ws) + base : nullptr;
  return base + ((nw * rs + 255) & ~size_t(255));
}

}  // namespace
}  // namespace pr

using namespace pr;

extern "C" {

int pr_reweight_workspace_size(pr_phi_plan phi, pr_psi_plan psi, size_t* bytes) {
  clear_error();
  PR_NONNULL(phi);
  PR_NONNULL(psi);
  PR_NONNULL(bytes);
  PR_TRY(admm_check_plans(phi, psi));
  *bytes = reweight_layout(phi, psi, nullptr, nullptr, nullptr);
  return PR_OK;
}

int pr_admm_reweighted_solve(pr_phi_plan phi, pr_psi_plan psi, const void* y, const pr_admm_params* params,
                             const pr_reweight_params* rw, void* x, void* workspace, pr_admm_report* rep,
                             void* stream) {
  clear_error();
  PR_NONNULL(phi);
  PR_NONNULL(psi);
  PR_NONNULL(y);
  PR_NONNULL(params);
  PR_NONNULL(rw);
  PR_NONNULL(x);
  if (!workspace || !aligned256(workspace)) { set_error("workspace must be non-NULL and 256-byte aligned"); return PR_EWORKSPACE; }
  PR_TRY(admm_check_plans(phi, psi));
  PR_TRY(admm_check_params(params));
  if (params->rel_tol != 0) { set_error("rel_tol must be 0 (fixed iteration counts per round)"); return PR_EINVAL; }
  if (rw->rounds < 0) { set_error("rounds must be >= 0"); return PR_EINVAL; }
  if (!(rw->delta0 > 0) || !(rw->beta > 0) || !(rw->beta <= 1)) {
    set_error("delta0 must be > 0 and beta in (0, 1]");
    return PR_EINVAL;
  }
  PR_TRY(check_sticky());
  hipStream_t s = as_stream(stream);
  void* wts = nullptr;
  AdmmJob j;
  PR_TRY(admm_job_init(&j, phi, psi, y, x, workspace, *params, s));
  reweight_layout(phi, psi, workspace, &j.w, &wts);
  PR_TRY(admm_device_setup(&j, s));
  const int64_t nw = static_cast<int64_t>(psi->nb) * phi->n * phi->n;
  double delta = rw->delta0;
  for (int r = 0; r <= rw->rounds; ++r) {
    if (r > 0) {
      PR_TRY(psi_analysis(psi, x, j.w.alpha, s));
      PR_TRY(l1_weights(j.w.alpha, nw, phi->prec, delta, wts, s));
      j.l1_weights = wts;
      PR_TRY(admm_job_restart(&j, s));
      delta *= rw->beta;
    }
    for (int it = 0; it < params->iters; ++it) PR_TRY(admm_step(&j, s));
  }
  if (rep) PR_TRY(admm_report(&j, rep, s));
  return PR_OK;
}

}  // extern "C"
