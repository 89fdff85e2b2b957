// Serving loop for imaging solves: continuous batching on one GPU.
//
// A request carries baselines, weights and visibilities already on the device
// (user order) and the solver parameters. Each call of pr_server_tick
//   1. retires running jobs whose last iteration has completed;
//   2. admits queued jobs in arrival order while the active-job limit and the
//      caller's device arena allow: the job's footprint (plans, workspace,
//      plan-ordered visibilities, image) is carved from the arena, its plans
//      are built on the admission stream, and its data are prepared on the
//      job's own stream, ending with the device-side set-up of 1 / ||Phi||
//      and gamma (nothing read back);
//   3. queues outer iterations of every running job on the job's stream,
//      keeping up to kDepth of them in flight per job.
// Jobs therefore join and leave while others run, and the work of all active
// jobs overlaps on the device. Each job runs exactly the kernels of a solve
// run alone (its own plans and workspace), so its result does not depend on
// the mix. Streams: a fixed pool, each job on the one with the least queued
// work (estimated bytes), big jobs thereby apart from small ones.
#include <algorithm>
#include <deque>
#include <map>
#include <new>
#include <vector>

#include "admm.hpp"
#include "host/arena.hpp"
#include "ops.hpp"

namespace pr {
namespace {

constexpr int kDepth = 3;   // outer iterations in flight per job

template <typename R>
__global__ void gather_cx_kernel(const cx_t<R>* __restrict__ src, const int32_t* __restrict__ perm, int64_t M,
                                 cx_t<R>* __restrict__ dst) {
  for (int64_t k = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; k < M;
       k += static_cast<int64_t>(gridDim.x) * blockDim.x)
    dst[k] = src[perm[k]];
}

template <typename R>
__global__ void zero_real_kernel(R* a, int64_t len) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < len;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    a[i] = R(0);
}

struct JobLayout {
  size_t phi_pers, phi_scr, psi_pers, psi_scr, admm, yplan, x, total;
  size_t o_phi_pers, o_phi_scr, o_psi_pers, o_psi_scr, o_admm, o_yplan, o_x;
};

pr_phi_desc phi_desc_of(const pr_job_desc& d) {
  pr_phi_desc pd{};
  pd.n = d.n;
  pd.oversample = 2;
  pd.J = d.J;
  pd.D = d.D > 0 ? d.D : 2000;
  pd.M = d.M;
  pd.prec = d.prec;
  pd.tile = d.tile;
  pd.interp = d.interp;
  return pd;
}

int job_layout(const pr_job_desc& d, JobLayout* L) {
  const pr_phi_desc pd = phi_desc_of(d);
  PR_TRY(pr_phi_plan_sizes(&pd, &L->phi_pers, &L->phi_scr));
  PR_TRY(pr_psi_plan_sizes(d.n, d.levels, d.basis_mask, d.prec, &L->psi_pers, &L->psi_scr));
  pr_phi_plan_t tphi;
  PR_TRY(phi_prepare(&tphi, &pd));
  pr_psi_plan_t tpsi;
  psi_prepare(&tpsi, d.n, d.levels, d.basis_mask, d.prec);
  L->admm = admm_layout(&tphi, &tpsi, nullptr, nullptr);
  const size_t rs = d.prec == PR_F32 ? 4 : 8;
  L->yplan = static_cast<size_t>(d.M) * 2 * rs;
  L->x = static_cast<size_t>(d.n) * d.n * rs;
  size_t o = 0;
  auto put = [&](size_t bytes, size_t* off) {
    *off = o;
    o += (bytes + 255) & ~size_t(255);
  };
  put(L->phi_pers, &L->o_phi_pers);
  put(L->phi_scr, &L->o_phi_scr);
  put(L->psi_pers, &L->o_psi_pers);
  put(L->psi_scr, &L->o_psi_scr);
  put(L->admm, &L->o_admm);
  put(L->yplan, &L->o_yplan);
  put(L->x, &L->o_x);
  L->total = o;
  return PR_OK;
}

}  // namespace
}  // namespace pr

struct pr_server_t {
  struct Job {
    int64_t id = 0;
    int state = 0;            // 0 queued, 1 running, 2 finished, 3 failed
    pr_job_desc d{};
    pr::JobLayout lay{};
    size_t off = 0;
    bool has_mem = false;
    pr_phi_plan phi = nullptr;
    pr_psi_plan psi = nullptr;
    pr::AdmmJob job;
    int stream = 0;
    int enq = 0;              // outer iterations queued
    double cost = 0;          // estimated bytes of one outer iteration
    hipEvent_t ready = nullptr;
    hipEvent_t ev[pr::kDepth] = {};
  };
  char* arena = nullptr;
  size_t arena_bytes = 0;
  pr::ArenaFreeList free_list;          // free byte ranges of the arena
  int max_active = 0;
  int active = 0;
  std::vector<hipStream_t> streams;
  std::vector<double> load;
  hipStream_t adm = nullptr;
  std::deque<int64_t> queue;
  std::map<int64_t, Job*> jobs;
  int64_t next_id = 1;
};

namespace pr {
namespace {

bool arena_alloc(pr_server_t* s, size_t bytes, size_t* off) { return s->free_list.alloc(bytes, off); }

void arena_free(pr_server_t* s, size_t off, size_t bytes) { s->free_list.release(off, bytes); }

void release(pr_server_t* s, pr_server_t::Job* j) {
  if (j->phi) pr_phi_plan_destroy(j->phi);
  if (j->psi) pr_psi_plan_destroy(j->psi);
  j->phi = nullptr;
  j->psi = nullptr;
  if (j->ready) (void)hipEventDestroy(j->ready);
  for (auto& e : j->ev)
    if (e) (void)hipEventDestroy(e);
  j->ready = nullptr;
  for (auto& e : j->ev) e = nullptr;
  if (j->has_mem) arena_free(s, j->off, j->lay.total);
  j->has_mem = false;
}

// Build the plans of an admitted job on the admission stream (plan creation
// waits for its own sort only), then its device state on the job's stream.
int setup_job(pr_server_t* s, pr_server_t::Job* j) {
  const hipStream_t js = s->streams[j->stream];
  char* base = s->arena + j->off;
  const pr_job_desc& d = j->d;
  const pr_phi_desc pd = phi_desc_of(d);
  PR_TRY(pr_phi_plan_create(&pd, d.uv, d.w, base + j->lay.o_phi_pers, base + j->lay.o_phi_scr, s->adm, &j->phi));
  PR_TRY(pr_psi_plan_create(d.n, d.levels, d.basis_mask, d.prec, base + j->lay.o_psi_pers, base + j->lay.o_psi_scr,
                            s->adm, &j->psi));
  void* yplan = base + j->lay.o_yplan;
  void* x = base + j->lay.o_x;
  const int64_t n2 = static_cast<int64_t>(d.n) * d.n;
  const int G = grid_for(d.M, 256, 8192);
  // the caller's y is read here, on the admission stream, and waited for: the
  // caller may release it once the job is running
  if (d.prec == PR_F32) {
    gather_cx_kernel<float><<<G, 256, 0, s->adm>>>(static_cast<const float2*>(d.y), j->phi->perm, d.M,
                                                   static_cast<float2*>(yplan));
    zero_real_kernel<float><<<grid_for(n2, 256, 4096), 256, 0, js>>>(static_cast<float*>(x), n2);
  } else {
    gather_cx_kernel<double><<<G, 256, 0, s->adm>>>(static_cast<const double2*>(d.y), j->phi->perm, d.M,
                                                    static_cast<double2*>(yplan));
    zero_real_kernel<double><<<grid_for(n2, 256, 4096), 256, 0, js>>>(static_cast<double*>(x), n2);
  }
  PR_TRY_LAUNCH();
  PR_TRY_HIP(hipStreamSynchronize(s->adm));
  PR_TRY(admm_job_init(&j->job, j->phi, j->psi, yplan, x, base + j->lay.o_admm, d.params, js));
  PR_TRY(admm_device_setup(&j->job, js));
  PR_TRY_HIP(hipEventCreateWithFlags(&j->ready, hipEventDisableTiming));
  for (auto& e : j->ev) PR_TRY_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  PR_TRY_HIP(hipEventRecord(j->ready, js));
  return PR_OK;
}

int check_desc(const pr_job_desc* d) {
  PR_NONNULL(d);
  if (d->M < 1) { set_error("a job needs M >= 1"); return PR_EINVAL; }
  PR_NONNULL(d->uv);
  PR_NONNULL(d->y);
  const pr_phi_desc pd = phi_desc_of(*d);
  PR_TRY(phi_validate(&pd));
  PR_TRY(psi_validate(d->n, d->levels, d->basis_mask, d->prec));
  PR_TRY(admm_check_params(&d->params));
  if (d->params.iters < 1) { set_error("a job needs params.iters >= 1"); return PR_EINVAL; }
  return PR_OK;
}

}  // namespace
}  // namespace pr

using namespace pr;

extern "C" {

int pr_server_job_bytes(const pr_job_desc* desc, size_t* bytes) {
  clear_error();
  PR_NONNULL(bytes);
  PR_TRY(check_desc(desc));
  JobLayout L;
  PR_TRY(job_layout(*desc, &L));
  *bytes = L.total;
  return PR_OK;
}

int pr_server_create(void* arena, size_t arena_bytes, int32_t max_active, int32_t nstreams, pr_server* out) {
  clear_error();
  PR_NONNULL(out);
  if (!arena || !aligned256(arena)) { set_error("arena must be non-NULL and 256-byte aligned"); return PR_EWORKSPACE; }
  if (arena_bytes < 256) { set_error("arena_bytes = %zu is too small", arena_bytes); return PR_EWORKSPACE; }
  if (max_active < 1 || max_active > 4096) { set_error("max_active = %d: must be in [1, 4096]", max_active); return PR_EINVAL; }
  if (nstreams < 1 || nstreams > 64) { set_error("nstreams = %d: must be in [1, 64]", nstreams); return PR_EINVAL; }
  pr_server_t* s = new (std::nothrow) pr_server_t();
  if (!s) { set_error("out of host memory"); return PR_EINVAL; }
  s->arena = static_cast<char*>(arena);
  s->arena_bytes = arena_bytes & ~size_t(255);
  s->free_list.reset(s->arena_bytes);
  s->max_active = max_active;
  hipError_t e = hipStreamCreateWithFlags(&s->adm, hipStreamNonBlocking);
  for (int k = 0; e == hipSuccess && k < nstreams; ++k) {
    hipStream_t st;
    e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess) s->streams.push_back(st);
  }
  if (e != hipSuccess) {
    set_error("pr_server_create: %s", hipGetErrorString(e));
    pr_server_destroy(s);
    return PR_EHIP;
  }
  s->load.assign(s->streams.size(), 0.0);
  *out = s;
  return PR_OK;
}

int pr_server_destroy(pr_server s) {
  if (!s) return PR_OK;
  for (hipStream_t st : s->streams) (void)hipStreamSynchronize(st);
  if (s->adm) (void)hipStreamSynchronize(s->adm);
  for (auto& kv : s->jobs) {
    release(s, kv.second);
    delete kv.second;
  }
  for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
  if (s->adm) (void)hipStreamDestroy(s->adm);
  delete s;
  return PR_OK;
}

int pr_server_submit(pr_server s, const pr_job_desc* desc, int64_t* job_id) {
  clear_error();
  PR_NONNULL(s);
  PR_NONNULL(job_id);
  PR_TRY(check_desc(desc));
  pr_server_t::Job* j = new (std::nothrow) pr_server_t::Job();
  if (!j) { set_error("out of host memory"); return PR_EINVAL; }
  j->d = *desc;
  int rc = job_layout(j->d, &j->lay);
  if (rc == PR_OK && j->lay.total > s->arena_bytes) {
    set_error("job needs %zu bytes, more than the whole arena (%zu)", j->lay.total, s->arena_bytes);
    rc = PR_EWORKSPACE;
  }
  if (rc != PR_OK) {
    delete j;
    return rc;
  }
  const double rs = desc->prec == PR_F32 ? 4.0 : 8.0;
  j->cost = (18.0 * desc->M + 66.0 * static_cast<double>(desc->n) * desc->n) * rs;
  j->id = s->next_id++;
  s->jobs[j->id] = j;
  s->queue.push_back(j->id);
  *job_id = j->id;
  return PR_OK;
}

int pr_server_tick(pr_server s, int32_t* queued, int32_t* running, int32_t* finished) {
  clear_error();
  PR_NONNULL(s);
  PR_TRY(check_sticky());
  // 1. retire
  for (auto& kv : s->jobs) {
    pr_server_t::Job* j = kv.second;
    if (j->state != 1 || j->enq < j->d.params.iters) continue;
    const hipError_t q = hipEventQuery(j->ev[(j->enq - 1) % kDepth]);
    if (q == hipSuccess) {
      j->state = 2;
      --s->active;
      s->load[j->stream] -= j->cost * j->d.params.iters;
    } else if (q != hipErrorNotReady) {
      set_error("job %lld: %s", static_cast<long long>(j->id), hipGetErrorString(q));
      return PR_EHIP;
    }
  }
  // 2. admit, in arrival order
  while (!s->queue.empty() && s->active < s->max_active) {
    pr_server_t::Job* j = s->jobs[s->queue.front()];
    size_t off;
    if (!arena_alloc(s, j->lay.total, &off)) break;
    s->queue.pop_front();
    j->off = off;
    j->has_mem = true;
    const int k = static_cast<int>(std::min_element(s->load.begin(), s->load.end()) - s->load.begin());
    j->stream = k;
    const int rc = setup_job(s, j);
    if (rc != PR_OK) {
      release(s, j);
      j->state = 3;
      return rc;
    }
    s->load[k] += j->cost * j->d.params.iters;
    j->state = 1;
    ++s->active;
  }
  // 3. next outer iteration of every running job, largest first
  std::vector<pr_server_t::Job*> run;
  for (auto& kv : s->jobs)
    if (kv.second->state == 1 && kv.second->enq < kv.second->d.params.iters) run.push_back(kv.second);
  std::stable_sort(run.begin(), run.end(), [](const pr_server_t::Job* a, const pr_server_t::Job* b) {
    return a->cost > b->cost;
  });
  for (pr_server_t::Job* j : run) {
    // fill the job's pipeline: up to kDepth outer iterations in flight
    while (j->enq < j->d.params.iters) {
      hipEvent_t& slot = j->ev[j->enq % kDepth];
      if (j->enq >= kDepth) {
        const hipError_t q = hipEventQuery(slot);   // iteration enq - kDepth
        if (q == hipErrorNotReady) break;
        if (q != hipSuccess) {
          set_error("job %lld: %s", static_cast<long long>(j->id), hipGetErrorString(q));
          return PR_EHIP;
        }
      }
      hipStream_t st = s->streams[j->stream];
      PR_TRY(admm_step(&j->job, st));
      PR_TRY_HIP(hipEventRecord(slot, st));
      ++j->enq;
    }
  }
  int nq = 0, nr = 0, nf = 0;
  for (auto& kv : s->jobs) {
    nq += kv.second->state == 0;
    nr += kv.second->state == 1;
    nf += kv.second->state == 2;
  }
  if (queued) *queued = nq;
  if (running) *running = nr;
  if (finished) *finished = nf;
  return PR_OK;
}

int pr_server_job_state(pr_server s, int64_t job_id, int32_t* state, int32_t* iters_done) {
  clear_error();
  PR_NONNULL(s);
  PR_NONNULL(state);
  auto it = s->jobs.find(job_id);
  if (it == s->jobs.end()) { set_error("no job %lld", static_cast<long long>(job_id)); return PR_EINVAL; }
  *state = it->second->state;
  if (iters_done) *iters_done = it->second->state == 2 ? it->second->d.params.iters : 0;
  return PR_OK;
}

int pr_server_fetch(pr_server s, int64_t job_id, void* x_out, pr_admm_report* rep, void* stream) {
  clear_error();
  PR_NONNULL(s);
  auto it = s->jobs.find(job_id);
  if (it == s->jobs.end()) { set_error("no job %lld", static_cast<long long>(job_id)); return PR_EINVAL; }
  pr_server_t::Job* j = it->second;
  if (j->state != 2) { set_error("job %lld has not finished (state %d)", static_cast<long long>(job_id), j->state); return PR_EINVAL; }
  PR_TRY(check_sticky());
  const hipStream_t st = as_stream(stream);
  const size_t bytes = static_cast<size_t>(j->d.n) * j->d.n * (j->d.prec == PR_F32 ? 4 : 8);
  if (x_out) PR_TRY_HIP(hipMemcpyAsync(x_out, j->job.x, bytes, hipMemcpyDeviceToDevice, st));
  if (rep) {
    PR_TRY(admm_report(&j->job, rep, st));
  } else {
    PR_TRY_HIP(hipStreamSynchronize(st));
  }
  release(s, j);
  delete j;
  s->jobs.erase(it);
  return PR_OK;
}

int pr_server_cancel(pr_server s, int64_t job_id) {
  clear_error();
  PR_NONNULL(s);
  auto it = s->jobs.find(job_id);
  if (it == s->jobs.end()) { set_error("no job %lld", static_cast<long long>(job_id)); return PR_EINVAL; }
  pr_server_t::Job* j = it->second;
  if (j->state == 0) {
    s->queue.erase(std::remove(s->queue.begin(), s->queue.end(), job_id), s->queue.end());
  } else if (j->state == 1) {
    // no further iterations; the ones in flight finish on the job's stream
    if (j->enq > 0) PR_TRY_HIP(hipEventSynchronize(j->ev[(j->enq - 1) % kDepth]));
    --s->active;
    s->load[j->stream] -= j->cost * j->d.params.iters;
  }
  release(s, j);
  delete j;
  s->jobs.erase(it);
  return PR_OK;
}

int pr_server_free_bytes(pr_server s, size_t* free_bytes, size_t* largest) {
  clear_error();
  PR_NONNULL(s);
  if (free_bytes) *free_bytes = s->free_list.free_bytes();
  if (largest) *largest = s->free_list.largest();
  return PR_OK;
}

}  // extern "C"
