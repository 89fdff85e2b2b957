// Batched solves: many independent ADMM solves (frequency channels or
// imaging jobs of different n and M) stepped together on one GPU.
//
// A step runs one outer iteration of Algorithm 1 for every member. The members
// are spread over the batch's own streams by longest-processing-time order
// (estimated bytes moved per iteration, largest first, each to the stream with
// the least work so far), forked from and joined back to the caller's stream,
// so small channels fill the device beside large ones. With use_graph the
// step is captured once into a HIP graph and replayed until the membership
// changes: one launch per step for the whole batch. Every member has its own
// plans and workspace, so its kernels and their order are exactly those of a
// solve run alone: results are bitwise the same.
#include <algorithm>
#include <new>
#include <vector>

#include "admm.hpp"
#include "fused.hpp"
#include "ops.hpp"

struct pr_batch_t {
  struct Member {
    bool used = false;
    pr::AdmmJob job;
    double cost = 0;
  };
  int device = 0;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> join;
  hipEvent_t fork = nullptr;
  std::vector<Member> members;
  // the graph is captured and replayed on gs (the caller's stream may be the
  // legacy default stream, which cannot be captured), bridged by events
  hipStream_t gs = nullptr;
  hipEvent_t g_in = nullptr, g_out = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool dirty = true;
  // fused operator stages over the members (pr_batch_fuse); dropped when the
  // membership changes
  bool fused_ok = false;
  std::vector<int> fused_slots;     // member slot of each fused plan
  pr::FusedStages fused;
};

namespace pr {

namespace {

// Bytes one outer iteration moves, as the scheduling weight.
double member_cost(const AdmmJob& j) {
  const double rs = j.phi->prec == PR_F32 ? 4.0 : 8.0;
  const double n2 = static_cast<double>(j.phi->n) * j.phi->n;
  return (18.0 * j.phi->M + 66.0 * n2) * rs;
}

void drop_graph(pr_batch_t* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->dirty = true;
}

// Members in LPT order with their stream index.
std::vector<std::pair<int, int>> schedule(const pr_batch_t* b) {
  std::vector<int> order;
  for (int i = 0; i < static_cast<int>(b->members.size()); ++i)
    if (b->members[i].used) order.push_back(i);
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return b->members[x].cost > b->members[y].cost; });
  std::vector<double> load(b->streams.size(), 0.0);
  std::vector<std::pair<int, int>> out;
  for (int i : order) {
    const int k = static_cast<int>(std::min_element(load.begin(), load.end()) - load.begin());
    load[k] += b->members[i].cost;
    out.push_back({i, k});
  }
  return out;
}

// Fork the batch streams from s, run fn(member, stream) in LPT order, join back.
template <class F>
int fork_join(pr_batch_t* b, hipStream_t s, F fn) {
  const auto plan = schedule(b);
  if (plan.empty()) return PR_OK;
  std::vector<char> used(b->streams.size(), 0);
  for (const auto& pk : plan) used[pk.second] = 1;
  PR_TRY_HIP(hipEventRecord(b->fork, s));
  for (size_t k = 0; k < b->streams.size(); ++k)
    if (used[k]) PR_TRY_HIP(hipStreamWaitEvent(b->streams[k], b->fork, 0));
  for (const auto& pk : plan) PR_TRY(fn(b->members[pk.first], b->streams[pk.second]));
  for (size_t k = 0; k < b->streams.size(); ++k) {
    if (!used[k]) continue;
    PR_TRY_HIP(hipEventRecord(b->join[k], b->streams[k]));
    PR_TRY_HIP(hipStreamWaitEvent(s, b->join[k], 0));
  }
  return PR_OK;
}

int one_step(pr_batch_t* b, hipStream_t s) {
  return fork_join(b, s, [](pr_batch_t::Member& m, hipStream_t ms) { return admm_step(&m.job, ms); });
}

int check_slot(const pr_batch_t* b, int slot) {
  if (slot < 0 || slot >= static_cast<int>(b->members.size()) || !b->members[slot].used) {
    set_error("slot %d is not a member of the batch", slot);
    return PR_EINVAL;
  }
  return PR_OK;
}

}  // namespace

}  // namespace pr

namespace {

// The fused form applies when it is current and every member has both vectors.
template <typename X, typename Y>
bool fused_vectors(pr_batch_t* b, X* const* x, Y* const* y, std::vector<X*>& fx, std::vector<Y*>& fy) {
  if (!b->fused_ok) return false;
  fx.clear();
  fy.clear();
  for (int slot : b->fused_slots) {
    if (!x[slot] || !y[slot]) return false;
    fx.push_back(x[slot]);
    fy.push_back(y[slot]);
  }
  return true;
}

}  // namespace

using namespace pr;

extern "C" {

int pr_batch_create(int32_t max_members, int32_t nstreams, pr_batch* out) {
  clear_error();
  PR_NONNULL(out);
  if (max_members < 1 || max_members > 4096) { set_error("max_members = %d: must be in [1, 4096]", max_members); return PR_EINVAL; }
  if (nstreams < 1 || nstreams > 64) { set_error("nstreams = %d: must be in [1, 64]", nstreams); return PR_EINVAL; }
  pr_batch_t* b = new (std::nothrow) pr_batch_t();
  if (!b) { set_error("out of host memory"); return PR_EINVAL; }
  b->members.resize(max_members);
  int rc = PR_OK;
  auto fail = [&](hipError_t e) {
    set_error("pr_batch_create: %s", hipGetErrorString(e));
    rc = PR_EHIP;
  };
  hipError_t e = hipGetDevice(&b->device);
  if (e != hipSuccess) fail(e);
  for (int k = 0; rc == PR_OK && k < nstreams; ++k) {
    hipStream_t st;
    e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e != hipSuccess) { fail(e); break; }
    b->streams.push_back(st);
    hipEvent_t ev;
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) { fail(e); break; }
    b->join.push_back(ev);
  }
  if (rc == PR_OK) {
    e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->g_in, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->g_out, hipEventDisableTiming);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->gs, hipStreamNonBlocking);
    if (e != hipSuccess) fail(e);
  }
  if (rc != PR_OK) {
    pr_batch_destroy(b);
    return rc;
  }
  *out = b;
  return PR_OK;
}

int pr_batch_destroy(pr_batch b) {
  if (!b) return PR_OK;
  drop_graph(b);
  for (hipStream_t st : b->streams) (void)hipStreamSynchronize(st);
  for (hipStream_t st : b->streams) (void)hipStreamDestroy(st);
  for (hipEvent_t ev : b->join) (void)hipEventDestroy(ev);
  if (b->fork) (void)hipEventDestroy(b->fork);
  if (b->gs) {
    (void)hipStreamSynchronize(b->gs);
    (void)hipStreamDestroy(b->gs);
  }
  if (b->g_in) (void)hipEventDestroy(b->g_in);
  if (b->g_out) (void)hipEventDestroy(b->g_out);
  delete b;
  return PR_OK;
}

int pr_batch_add(pr_batch b, pr_phi_plan phi, pr_psi_plan psi, const void* y, void* x, const pr_admm_params* params,
                 void* workspace, void* stream, int32_t* slot) {
  clear_error();
  PR_NONNULL(b);
  PR_NONNULL(phi);
  PR_NONNULL(psi);
  PR_NONNULL(y);
  PR_NONNULL(x);
  PR_NONNULL(params);
  PR_NONNULL(slot);
  if (!workspace || !aligned256(workspace)) { set_error("workspace must be non-NULL and 256-byte aligned"); return PR_EWORKSPACE; }
  PR_TRY(admm_check_plans(phi, psi));
  PR_TRY(admm_check_params(params));
  int free_slot = -1;
  for (int i = 0; i < static_cast<int>(b->members.size()); ++i) {
    if (!b->members[i].used) {
      if (free_slot < 0) free_slot = i;
      continue;
    }
    const AdmmJob& o = b->members[i].job;
    if (o.phi == phi || o.psi == psi) {
      set_error("plans are already used by member %d (each member needs its own plans)", i);
      return PR_EINVAL;
    }
  }
  if (free_slot < 0) { set_error("batch is full (%zu members)", b->members.size()); return PR_EINVAL; }
  PR_TRY(check_sticky());
  pr_batch_t::Member& m = b->members[free_slot];
  const hipStream_t s = as_stream(stream);
  PR_TRY(admm_job_init(&m.job, phi, psi, y, x, workspace, *params, s));
  PR_TRY(admm_device_setup(&m.job, s));
  m.cost = member_cost(m.job);
  m.used = true;
  b->dirty = true;
  b->fused_ok = false;
  *slot = free_slot;
  return PR_OK;
}

int pr_batch_remove(pr_batch b, int32_t slot) {
  clear_error();
  PR_NONNULL(b);
  PR_TRY(check_slot(b, slot));
  b->members[slot].used = false;
  b->dirty = true;
  b->fused_ok = false;
  return PR_OK;
}

int pr_batch_step(pr_batch b, int32_t iters, int32_t use_graph, void* stream) {
  clear_error();
  PR_NONNULL(b);
  if (iters < 0) { set_error("iters = %d < 0", iters); return PR_EINVAL; }
  PR_TRY(check_sticky());
  const hipStream_t s = as_stream(stream);
  if (!use_graph) {
    for (int it = 0; it < iters; ++it) PR_TRY(one_step(b, s));
    return PR_OK;
  }
  if (iters == 0) return PR_OK;
  if (b->dirty) {
    drop_graph(b);
    // the capture records the launches without running them: keep the counters
    std::vector<int> done(b->members.size());
    for (size_t i = 0; i < b->members.size(); ++i) done[i] = b->members[i].job.iters_done;
    PR_TRY_HIP(hipStreamBeginCapture(b->gs, hipStreamCaptureModeThreadLocal));
    const int rc = one_step(b, b->gs);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->gs, &g);
    for (size_t i = 0; i < b->members.size(); ++i) b->members[i].job.iters_done = done[i];
    if (rc != PR_OK) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) {
      set_error("stream capture of the batch step failed: %s", hipGetErrorString(e));
      return PR_EHIP;
    }
    b->graph = g;
    PR_TRY_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    b->dirty = false;
  }
  PR_TRY_HIP(hipEventRecord(b->g_in, s));
  PR_TRY_HIP(hipStreamWaitEvent(b->gs, b->g_in, 0));
  for (int it = 0; it < iters; ++it) PR_TRY_HIP(hipGraphLaunch(b->exec, b->gs));
  PR_TRY_HIP(hipEventRecord(b->g_out, b->gs));
  PR_TRY_HIP(hipStreamWaitEvent(s, b->g_out, 0));
  for (auto& m : b->members)
    if (m.used) m.job.iters_done += iters;
  return PR_OK;
}

int pr_batch_fuse_bytes(pr_batch b, size_t* bytes) {
  clear_error();
  PR_NONNULL(b);
  PR_NONNULL(bytes);
  std::vector<pr_phi_plan_t*> plans;
  for (auto& m : b->members)
    if (m.used) plans.push_back(m.job.phi);
  if (plans.empty()) { set_error("the batch has no members"); return PR_EINVAL; }
  return fused_bytes(plans.data(), static_cast<int>(plans.size()), bytes);
}

int pr_batch_fuse(pr_batch b, void* workspace, size_t bytes, void* stream) {
  clear_error();
  PR_NONNULL(b);
  PR_TRY(check_sticky());
  std::vector<pr_phi_plan_t*> plans;
  std::vector<int> slots;
  for (int i = 0; i < static_cast<int>(b->members.size()); ++i) {
    if (!b->members[i].used) continue;
    plans.push_back(b->members[i].job.phi);
    slots.push_back(i);
  }
  if (plans.empty()) { set_error("the batch has no members"); return PR_EINVAL; }
  b->fused_ok = false;
  PR_TRY(fused_build(plans.data(), static_cast<int>(plans.size()), workspace, bytes, &b->fused, as_stream(stream)));
  b->fused_slots = slots;
  b->fused_ok = true;
  return PR_OK;
}

int pr_batch_phi_apply(pr_batch b, const void* const* x, void* const* y, void* stream) {
  clear_error();
  PR_NONNULL(b);
  PR_NONNULL(x);
  PR_NONNULL(y);
  PR_TRY(check_sticky());
  {
    std::vector<const void*> fx;
    std::vector<void*> fy;
    if (fused_vectors(b, x, y, fx, fy)) return fused_apply(&b->fused, fx.data(), fy.data(), as_stream(stream));
  }
  return fork_join(b, as_stream(stream), [&](pr_batch_t::Member& m, hipStream_t ms) {
    const int i = static_cast<int>(&m - b->members.data());
    if (!x[i] || !y[i]) return static_cast<int>(PR_OK);
    PR_TRY(phi_fzs(m.job.phi, x[i], ms));
    return phi_gw(m.job.phi, y[i], 1.0, ms);
  });
}

int pr_batch_phi_adjoint(pr_batch b, const void* const* y, void* const* x, void* stream) {
  clear_error();
  PR_NONNULL(b);
  PR_NONNULL(x);
  PR_NONNULL(y);
  PR_TRY(check_sticky());
  {
    std::vector<const void*> fy;
    std::vector<void*> fx;
    if (fused_vectors(b, y, x, fy, fx)) return fused_adjoint(&b->fused, fy.data(), fx.data(), as_stream(stream));
  }
  return fork_join(b, as_stream(stream), [&](pr_batch_t::Member& m, hipStream_t ms) {
    const int i = static_cast<int>(&m - b->members.data());
    if (!x[i] || !y[i]) return static_cast<int>(PR_OK);
    PR_TRY(phi_gw_adjoint(m.job.phi, y[i], 1.0, ms));
    return phi_fzs_adjoint(m.job.phi, x[i], ms);
  });
}

int pr_batch_report(pr_batch b, int32_t slot, pr_admm_report* rep, void* stream) {
  clear_error();
  PR_NONNULL(b);
  PR_NONNULL(rep);
  PR_TRY(check_slot(b, slot));
  PR_TRY(check_sticky());
  return admm_report(&b->members[slot].job, rep, as_stream(stream));
}

int pr_batch_members(pr_batch b, int32_t* count) {
  clear_error();
  PR_NONNULL(b);
  PR_NONNULL(count);
  int c = 0;
  for (const auto& m : b->members) c += m.used ? 1 : 0;
  *count = c;
  return PR_OK;
}

}  // extern "C"
