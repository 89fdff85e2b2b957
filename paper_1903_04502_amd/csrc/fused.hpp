// The plain measurement operator and its adjoint of several plans at once,
// one launch per stage (the batched channels of the per-channel split in
// Section "Distributed Images", kept on one GPU): degridding, the gridding
// walk and the patch merge each run once over all members' work items or
// tiles, with the item's tile field tagged by its member; each FFT pass runs
// once per image size over the members of that size. Every item and every
// line is computed exactly as in a member's own launch, so the results are
// bitwise those of the plans applied one by one.
#pragma once

#include <vector>

#include "phi.hpp"

namespace pr {

struct FusedStages {
  std::vector<pr_phi_plan_t*> plans;
  int prec = PR_F32;
  // visibility stages (device tables in the caller's workspace)
  void* d_dg = nullptr;          // per-member degridding arguments
  void* d_ga = nullptr;          // per-member gridding arguments
  void* d_mg = nullptr;          // per-member merge arguments
  int4* sched_d = nullptr;
  int32_t* sched_d_off = nullptr;
  int4* sched_g = nullptr;        // the walk's items (more than kSmallItem visibilities)
  int32_t* sched_g_off = nullptr;
  int4* small = nullptr;          // the small-item kernel's items
  int64_t nSmall = 0;
  int Gd = 0, Gg = 0, tiles = 0;
  std::vector<char> h_dg, h_ga;  // host copies; each call's vector pointers patched in
  std::vector<const void*> up_dg, up_ga;   // pointers of the last upload
  // FFT passes: one class per image size
  struct Cls {
    int n = 0;
    std::vector<int> idx;        // members of this size
    void* d_fwd = nullptr;       // per-member FFT pointers, forward
    void* d_adj = nullptr;       // per-member FFT pointers, adjoint
    std::vector<char> h_fwd, h_adj;
    std::vector<const void*> up_fwd, up_adj;
  };
  std::vector<Cls> cls;
};

// Workspace bytes for fusing these plans (host only; every plan must have
// the first one's precision, J, D, lookup and tile).
int fused_bytes(pr_phi_plan_t* const* plans, int n, size_t* bytes);
// Build the schedules and member tables in ws (synchronises s once).
int fused_build(pr_phi_plan_t* const* plans, int n, void* ws, size_t ws_bytes, FusedStages* f, hipStream_t s);
// y_m = Phi_m x_m and x_m = Re Phi_m^dagger y_m for every member m (plan
// order, as the plans' own calls).
int fused_apply(FusedStages* f, const void* const* x, void* const* y, hipStream_t s);
int fused_adjoint(FusedStages* f, const void* const* y, void* const* x, hipStream_t s);

// the two halves (gridding.hip, fft.hip)
size_t fused_vis_bytes(int n, int64_t items, int prec);
int fused_vis_build(FusedStages* f, Carver& c, hipStream_t s);
int fused_gw(FusedStages* f, void* const* y, hipStream_t s);
int fused_gw_adjoint(FusedStages* f, const void* const* y, hipStream_t s);
size_t fused_fft_bytes(const std::vector<int>& class_sizes, int prec);
int fused_fft_build(FusedStages* f, Carver& c);
int fused_fzs(FusedStages* f, const void* const* x, hipStream_t s);
int fused_fzs_adjoint(FusedStages* f, void* const* x, hipStream_t s);

}  // namespace pr
