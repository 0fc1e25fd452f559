// Continuous-batching solve server (host scheduler + per-slot HIP streams).
//
// Requests (one pressure or velocity solve each, any supported grid) are
// queued FIFO on submit and admitted as soon as (a) a worker slot is free and
// (b) an idle grid of the request's shape and footprint class exists or the
// HBM budget has room for a new one (footprint = vd_workspace_bytes, or
// vd_workspace_bytes_helmholtz for velocity solves: the Krylov basis,
// operator work fields and coefficient fields).  Each admitted request runs on its grid's
// own non-blocking stream from its own host thread, so the kernels of
// requests of different sizes overlap on the device while their Krylov state
// stays resident in HBM.  Grids are kept for reuse by later requests of the
// same shape; idle grids of other shapes are released only when the budget
// would otherwise block the head of the queue.  Results are identical to a
// solve run alone: every kernel's launch configuration and reduction order
// depend only on the request itself.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "../../include/vdsolve.h"

namespace {

using Clock = std::chrono::steady_clock;

struct GridEntry {
  vd_grid* grid = nullptr;
  hipStream_t stream = nullptr;
  vd_grid_desc desc{};
  vd_solve_opts opts{};  // options of the requests it serves (same_footprint)
  size_t bytes = 0;      // charged against the budget while the grid exists
  bool busy = false;
};

struct Job {
  unsigned long long ticket;
  vd_request req;
  double t_arrive;
  size_t bytes;
};

bool same_desc(const vd_grid_desc& a, const vd_grid_desc& b) {
  if (a.ndim != b.ndim) return false;
  for (int i = 0; i < a.ndim; ++i)
    if (a.n[i] != b.n[i] || a.basis[i] != b.basis[i] || a.length[i] != b.length[i]) return false;
  return true;
}

// A grid keeps every work buffer it has ever allocated, so a grid that ran
// requests with different options holds the union of their buffers, more
// than vd_workspace_bytes of either.  Grids are therefore reused only by
// requests whose options allocate the same buffers: same precision, solver,
// formulation and (GMRES) restart length.  A grid's charge is then exact.
bool same_footprint(const vd_solve_opts& a, const vd_solve_opts& b) {
  if (a.precision != b.precision || a.solver != b.solver || a.formulation != b.formulation) return false;
  return a.solver != VD_GMRES || a.restart == b.restart;
}

}  // namespace

struct vd_server {
  size_t budget = 0, used = 0;
  int max_slots = 1;
  bool dry = false;
  double dry_seconds = 0.0;
  Clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Job> queue;
  std::vector<GridEntry*> grids;
  struct Assign {
    bool has = false;
    Job job;
    GridEntry* ge = nullptr;
    double t_start = 0;
  };
  std::vector<Assign> slots;
  std::vector<std::thread> workers;
  std::deque<vd_result> done;
  unsigned long long next_ticket = 1;
  long long in_flight = 0;
  size_t peak_used = 0;
  int peak_busy = 0;
  bool stop = false;

  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

namespace {

int busy_slots(vd_server* S) {
  int b = 0;
  for (auto& a : S->slots) b += a.has ? 1 : 0;
  return b;
}

// Admit queued jobs in FIFO order while they fit.  Caller holds the lock.
void admit(vd_server* S) {
  while (!S->queue.empty()) {
    Job& job = S->queue.front();
    int slot = -1;
    for (int i = 0; i < S->max_slots; ++i)
      if (!S->slots[i].has) { slot = i; break; }
    if (slot < 0) return;
    GridEntry* ge = nullptr;
    for (auto* g : S->grids)
      // equal charges: the same number of Helmholtz components solved together
      if (!g->busy && same_desc(g->desc, job.req.desc) && same_footprint(g->opts, job.req.opts) &&
          g->bytes == job.bytes) {
        ge = g;
        break;
      }
    if (!ge) {
      // release idle grids of other shapes while the budget blocks the head
      while (S->used + job.bytes > S->budget) {
        GridEntry* victim = nullptr;
        for (auto* g : S->grids)
          if (!g->busy) { victim = g; break; }
        if (!victim) break;
        if (!S->dry) {
          vd_grid_destroy(victim->grid);
          hipStreamDestroy(victim->stream);
        }
        S->used -= victim->bytes;
        for (size_t i = 0; i < S->grids.size(); ++i)
          if (S->grids[i] == victim) { S->grids.erase(S->grids.begin() + i); break; }
        delete victim;
      }
      if (S->used + job.bytes > S->budget) return;  // head of line waits
      ge = new GridEntry();
      ge->desc = job.req.desc;
      ge->opts = job.req.opts;
      ge->bytes = job.bytes;
      S->used += job.bytes;
      S->peak_used = S->used > S->peak_used ? S->used : S->peak_used;
      S->grids.push_back(ge);
    }
    ge->busy = true;
    auto& a = S->slots[slot];
    a.has = true;
    a.job = job;
    a.ge = ge;
    a.t_start = S->now();
    S->queue.pop_front();
    int b = busy_slots(S);
    S->peak_busy = b > S->peak_busy ? b : S->peak_busy;
    S->cv_work.notify_all();
  }
}

vd_status run_job(vd_server* S, GridEntry* ge, const vd_request& r, vd_solve_info* info) {
  if (S->dry) {
    if (S->dry_seconds > 0) std::this_thread::sleep_for(std::chrono::duration<double>(S->dry_seconds));
    std::memset(info, 0, sizeof(*info));
    info->status = VD_ENOTSUP;  // scheduler dry run: nothing was solved
    return VD_ENOTSUP;
  }
  if (!ge->grid) {
    if (hipStreamCreateWithFlags(&ge->stream, hipStreamNonBlocking) != hipSuccess) return VD_EDEVICE;
    vd_status s = vd_grid_create(&ge->grid, &ge->desc, ge->stream);
    if (s != VD_OK) return s;
  }
  vd_status s = vd_set_density(ge->grid, r.rho);
  if (s != VD_OK) return s;
  if (r.kind == VD_OP_HELMHOLTZ)
    return vd_solve_helmholtz(ge->grid, r.dt_nu, r.ncomp > 0 ? r.ncomp : 1, r.f, r.x, &r.opts, info);
  return vd_solve_pressure(ge->grid, r.f, r.x, &r.opts, info);
}

void worker_main(vd_server* S, int slot) {
  while (true) {
    vd_server::Assign a;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_work.wait(lk, [&] { return S->stop || S->slots[slot].has; });
      if (!S->slots[slot].has && S->stop) return;
      a = S->slots[slot];
    }
    vd_solve_info info{};
    vd_status st = run_job(S, a.ge, a.job.req, &info);
    vd_result res{};
    res.ticket = a.job.ticket;
    res.user_tag = a.job.req.user_tag;
    res.status = st;
    res.iterations = info.iterations;
    res.refinements = info.refinements;
    res.rel_residual = info.rel_residual;
    res.t_arrive = a.job.t_arrive;
    res.t_start = a.t_start;
    res.slot = slot;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      res.t_done = S->now();
      if (st < 0 && a.ge->grid == nullptr && !S->dry) {
        // grid could not be created: give its budget back
        S->used -= a.ge->bytes;
        for (size_t i = 0; i < S->grids.size(); ++i)
          if (S->grids[i] == a.ge) { S->grids.erase(S->grids.begin() + i); break; }
        if (a.ge->stream) hipStreamDestroy(a.ge->stream);
        delete a.ge;
      } else {
        a.ge->busy = false;
      }
      S->slots[slot].has = false;
      S->done.push_back(res);
      S->in_flight--;
      admit(S);
    }
    S->cv_done.notify_all();
  }
}

vd_status create_impl(vd_server** out, size_t budget, int max_slots, int dry, double dry_seconds) {
  if (!out || max_slots < 1 || max_slots > 64 || budget == 0) return VD_EINVAL;
  vd_server* S = new (std::nothrow) vd_server();
  if (!S) return VD_ENOMEM;
  S->budget = budget;
  S->max_slots = max_slots;
  S->dry = dry != 0;
  S->dry_seconds = dry_seconds;
  S->t0 = Clock::now();
  S->slots.resize(max_slots);
  try {
    for (int i = 0; i < max_slots; ++i) S->workers.emplace_back(worker_main, S, i);
  } catch (...) {
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->stop = true;
    }
    S->cv_work.notify_all();
    for (auto& t : S->workers) t.join();
    delete S;
    return VD_ENOMEM;
  }
  *out = S;
  return VD_OK;
}

}  // namespace

extern "C" {

vd_status vd_server_create(vd_server** out, size_t hbm_budget, int max_slots) {
  return create_impl(out, hbm_budget, max_slots, 0, 0.0);
}

vd_status vd_server_create_dry(vd_server** out, size_t hbm_budget, int max_slots, double seconds_per_request) {
  if (!(seconds_per_request >= 0.0)) return VD_EINVAL;
  return create_impl(out, hbm_budget, max_slots, 1, seconds_per_request);
}

vd_status vd_server_submit(vd_server* S, const vd_request* r, unsigned long long* ticket) {
  if (!S || !r) return VD_EINVAL;
  if (!S->dry && (!r->rho || !r->f || !r->x)) return VD_EINVAL;
  if (r->kind != VD_OP_PRESSURE && r->kind != VD_OP_HELMHOLTZ) return VD_EINVAL;
  size_t bytes = r->kind == VD_OP_HELMHOLTZ
                     ? vd_workspace_bytes_helmholtz(&r->desc, &r->opts, r->ncomp > 0 ? r->ncomp : 1)
                     : vd_workspace_bytes(&r->desc, &r->opts);
  if (bytes == 0) return VD_EINVAL;
  if (bytes > S->budget) return VD_ETOOBIG;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    Job j;
    j.ticket = S->next_ticket++;
    j.req = *r;
    j.t_arrive = S->now();
    j.bytes = bytes;
    S->queue.push_back(j);
    S->in_flight++;
    if (ticket) *ticket = j.ticket;
    admit(S);
  }
  return VD_OK;
}

vd_status vd_server_poll(vd_server* S, vd_result* out, int cap, int* n) {
  if (!S || !n || cap < 0 || (cap > 0 && !out)) return VD_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  int k = 0;
  while (k < cap && !S->done.empty()) {
    out[k++] = S->done.front();
    S->done.pop_front();
  }
  *n = k;
  return VD_OK;
}

vd_status vd_server_wait(vd_server* S, vd_result* out, int cap, int* n, double timeout_s) {
  if (!S || !n || cap < 1 || !out) return VD_EINVAL;
  {
    std::unique_lock<std::mutex> lk(S->mu);
    S->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s > 0 ? timeout_s : 0.0),
                        [&] { return !S->done.empty() || S->in_flight == 0; });
  }
  return vd_server_poll(S, out, cap, n);
}

vd_status vd_server_stats(vd_server* S, vd_server_stats_t* st) {
  if (!S || !st) return VD_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  st->queued = (long long)S->queue.size();
  st->in_flight = S->in_flight;
  st->busy_slots = busy_slots(S);
  st->grids = (int)S->grids.size();
  st->hbm_used = S->used;
  st->hbm_peak = S->peak_used;
  st->peak_busy_slots = S->peak_busy;
  return VD_OK;
}

vd_status vd_server_destroy(vd_server* S) {
  if (!S) return VD_EINVAL;
  {
    std::unique_lock<std::mutex> lk(S->mu);
    S->cv_done.wait(lk, [&] { return S->in_flight == 0 || S->queue.size() == (size_t)S->in_flight; });
    // queued but never admitted requests are dropped
    S->in_flight -= (long long)S->queue.size();
    S->queue.clear();
    S->stop = true;
  }
  S->cv_work.notify_all();
  for (auto& t : S->workers) t.join();
  for (auto* g : S->grids) {
    if (g->grid) vd_grid_destroy(g->grid);
    if (g->stream) hipStreamDestroy(g->stream);
    delete g;
  }
  delete S;
  return VD_OK;
}

}  // extern "C"
