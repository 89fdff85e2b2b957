// The fused form of the batched plain operator: checks, workspace layout and
// the two calls (see fused.hpp).
#include <algorithm>
#include <map>

#include "fused.hpp"

namespace pr {

namespace {

constexpr int kMaxFusedMembers = 4096;   // member field of the work items: 12 bits

int check_same(pr_phi_plan_t* const* plans, int n) {
  if (n < 1 || n > kMaxFusedMembers) {
    set_error("%d plans: fusing takes 1 to %d", n, kMaxFusedMembers);
    return PR_EINVAL;
  }
  const pr_phi_plan_t* a = plans[0];
  for (int i = 0; i < n; ++i) {
    const pr_phi_plan_t* b = plans[i];
    if (!b) { set_error("plan %d is NULL", i); return PR_EINVAL; }
    if (b->prec != a->prec || b->J != a->J || b->D != a->D || b->interp != a->interp || b->tapwords != a->tapwords ||
        b->T != a->T) {
      set_error("plan %d differs from plan 0 in precision, J, D, lookup or tile: fused launches share one kernel", i);
      return PR_EUNSUPPORTED;
    }
  }
  if (a->J > 4) {
    set_error("fused gridding uses the segment walk: J <= 4 (J = %d)", a->J);
    return PR_EUNSUPPORTED;
  }
  return PR_OK;
}

// image sizes present, ascending, with the member indices of each
std::vector<FusedStages::Cls> size_classes(pr_phi_plan_t* const* plans, int n) {
  std::map<int, std::vector<int>> by;
  for (int i = 0; i < n; ++i) by[plans[i]->n].push_back(i);
  std::vector<FusedStages::Cls> out;
  for (auto& kv : by) {
    FusedStages::Cls c;
    c.n = kv.first;
    c.idx = kv.second;
    out.push_back(c);
  }
  return out;
}

}  // namespace

int fused_bytes(pr_phi_plan_t* const* plans, int n, size_t* bytes) {
  PR_TRY(check_same(plans, n));
  int64_t items = 0;
  for (int i = 0; i < n; ++i) items += plans[i]->nItems;
  std::vector<int> counts;
  for (const auto& c : size_classes(plans, n)) counts.push_back(static_cast<int>(c.idx.size()));
  *bytes = fused_vis_bytes(n, items, plans[0]->prec) + fused_fft_bytes(counts, plans[0]->prec);
  return PR_OK;
}

int fused_build(pr_phi_plan_t* const* plans, int n, void* ws, size_t ws_bytes, FusedStages* f, hipStream_t s) {
  size_t need = 0;
  PR_TRY(fused_bytes(plans, n, &need));
  if (!ws || !aligned256(ws) || ws_bytes < need) {
    set_error("fused workspace: %zu bytes given, %zu needed (256-byte aligned)", ws_bytes, need);
    return PR_EWORKSPACE;
  }
  f->plans.assign(plans, plans + n);
  f->prec = plans[0]->prec;
  f->cls = size_classes(plans, n);
  Carver c(ws);
  PR_TRY(fused_vis_build(f, c, s));
  PR_TRY(fused_fft_build(f, c));
  return PR_OK;
}

int fused_apply(FusedStages* f, const void* const* x, void* const* y, hipStream_t s) {
  PR_TRY(fused_fzs(f, x, s));
  return fused_gw(f, y, s);
}

int fused_adjoint(FusedStages* f, const void* const* y, void* const* x, hipStream_t s) {
  PR_TRY(fused_gw_adjoint(f, y, s));
  return fused_fzs_adjoint(f, x, s);
}

}  // namespace pr
