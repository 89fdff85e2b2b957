// Tile-size autotuner for the measurement operator: builds the plan with each
// admissible tile side and times (Phi, Phi^dagger) pairs on the device.
//
// The tile side sets the work-item shape of degridding and gridding (patch of
// (T+J-1)^2 cells, moments of T^2 base cells in LDS) and thereby the balance
// between per-item fixed cost and parallelism, which depends on how the
// baselines fill the grid: the fastest side is measured rather than modelled.
#include <new>
#include <vector>

#include "ops.hpp"
#include "phi.hpp"

using namespace pr;

extern "C" {

int pr_phi_tune(const pr_phi_desc* desc, const void* uv, const void* w, void* persistent_ws, void* scratch_ws,
                void* vis_ws, int32_t reps, void* stream, int32_t* best_tile, double* best_ms) {
  clear_error();
  PR_NONNULL(desc);
  PR_NONNULL(best_tile);
  if (desc->M > 0) {
    PR_NONNULL(uv);
    PR_NONNULL(vis_ws);
  }
  if (reps < 1 || reps > 1000) { set_error("reps = %d: must be in [1, 1000]", reps); return PR_EINVAL; }
  if (!persistent_ws || !scratch_ws || !aligned256(persistent_ws) || !aligned256(scratch_ws)) {
    set_error("workspaces must be non-NULL and 256-byte aligned");
    return PR_EWORKSPACE;
  }
  PR_TRY(check_sticky());
  const hipStream_t s = as_stream(stream);
  const int cands[3] = {8, 16, 32};
  int best = 0;
  double best_t = 0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  PR_TRY_HIP(hipEventCreate(&e0));
  int rc = PR_OK;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    set_error("hipEventCreate failed");
    return PR_EHIP;
  }
  for (int T : cands) {
    pr_phi_desc d = *desc;
    d.tile = T;
    if (phi_validate(&d) != PR_OK) continue;   // tile not admissible for this J / precision
    clear_error();
    pr_phi_plan_t* p = new (std::nothrow) pr_phi_plan_t();
    if (!p) { set_error("out of host memory"); rc = PR_EINVAL; break; }
    rc = phi_prepare(p, &d);
    if (rc == PR_OK) rc = phi_layout(p, persistent_ws, scratch_ws, nullptr, nullptr);
    if (rc == PR_OK) rc = phi_create(p, uv, w, s);
    const int64_t N = static_cast<int64_t>(p->n) * p->n;
    if (rc == PR_OK) rc = fill_real(p->img_a, N, p->prec, 1.0 / p->n, s);
    // one untimed pair, then reps timed pairs
    for (int r = 0; rc == PR_OK && r <= reps; ++r) {
      if (r == 1 && hipEventRecord(e0, s) != hipSuccess) rc = PR_EHIP;
      if (rc == PR_OK) rc = phi_fzs(p, p->img_a, s);
      if (rc == PR_OK) rc = phi_gw(p, vis_ws, 1.0, s);
      if (rc == PR_OK) rc = phi_gw_adjoint(p, vis_ws, 1.0, s);
      if (rc == PR_OK) rc = phi_fzs_adjoint(p, p->img_b, s);
    }
    float ms = 0;
    if (rc == PR_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                        hipEventElapsedTime(&ms, e0, e1) != hipSuccess)) {
      set_error("event timing failed");
      rc = PR_EHIP;
    }
    delete p;
    if (rc != PR_OK) break;
    const double t = static_cast<double>(ms) / reps;
    if (best == 0 || t < best_t) {
      best = T;
      best_t = t;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != PR_OK) return rc;
  if (best == 0) {
    set_error("no admissible tile side for J = %d", desc->J);
    return PR_EUNSUPPORTED;
  }
  *best_tile = best;
  if (best_ms) *best_ms = best_t;
  return PR_OK;
}

}  // extern "C"
