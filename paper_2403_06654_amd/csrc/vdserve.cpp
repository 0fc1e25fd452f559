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
constexpr int kBatchMax = 3;  // requests per shared batch (vd_solve_pressure_batch)

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
  // a slot's work: one request, or a batch of pressure requests of one
  // shape and options solved together (vd_solve_pressure_batch)
  struct Assign {
    bool has = false;
    int nj = 0;
    Job job[kBatchMax];
    GridEntry* ge[kBatchMax] = {};
    double t_start = 0;
  };
  int max_batch = kBatchMax;
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

// An idle grid that a job may use: its shape and footprint class (equal
// charges: the same number of Helmholtz components solved together), or a
// new one if the budget has room (evict: release idle grids of other shapes
// while the budget blocks, for the head of the queue only).  nullptr if none.
GridEntry* acquire_grid(vd_server* S, const Job& job, bool evict) {
  for (auto* g : S->grids)
    if (!g->busy && same_desc(g->desc, job.req.desc) && same_footprint(g->opts, job.req.opts) &&
        g->bytes == job.bytes)
      return g;
  while (evict && S->used + job.bytes > S->budget) {
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
  if (S->used + job.bytes > S->budget) return nullptr;
  GridEntry* ge = new GridEntry();
  ge->desc = job.req.desc;
  ge->opts = job.req.opts;
  ge->bytes = job.bytes;
  S->used += job.bytes;
  S->peak_used = S->used > S->peak_used ? S->used : S->peak_used;
  S->grids.push_back(ge);
  return ge;
}

// Requests that vd_solve_pressure_batch runs with shared launches: pressure,
// GMRES, direct form, a Fourier grid of two or three dimensions.
bool batchable(const vd_request& r) {
  if (r.kind != VD_OP_PRESSURE || r.opts.solver != VD_GMRES || r.opts.formulation != VD_FORM_L) return false;
  if (r.desc.ndim < 2) return false;
  for (int i = 0; i < r.desc.ndim; ++i)
    if (r.desc.basis[i] != VD_FOURIER) return false;
  return true;
}

// Requests that can share one batch: the same grid shape and the same solve
// options (no history)
bool same_batch(const vd_request& a, const vd_request& b) {
  if (!same_desc(a.desc, b.desc)) return false;
  const vd_solve_opts &x = a.opts, &y = b.opts;
  if (x.history || y.history) return false;
  return x.solver == y.solver && x.restart == y.restart && x.max_iter == y.max_iter && x.rtol == y.rtol &&
         x.precond == y.precond && x.precision == y.precision && x.inner_rtol == y.inner_rtol &&
         x.max_outer == y.max_outer && x.use_x0 == y.use_x0 && x.formulation == y.formulation &&
         (x.rho0 == y.rho0 || (x.rho0 != x.rho0 && y.rho0 != y.rho0));
}

// Admit queued jobs in FIFO order while they fit.  Caller holds the lock.
// The head of the queue is admitted first.  When more requests wait than
// slots are free and the head can share launches, up to max_batch - 1 later
// requests of the same shape and options that find a grid without evicting
// join its batch (they overtake requests of other shapes, which wait for the
// next free slot as before).  While slots are free for every waiting
// request, each gets its own: a batch finishes with its slowest member.
void admit(vd_server* S) {
  while (!S->queue.empty()) {
    Job& job = S->queue.front();
    int slot = -1;
    for (int i = 0; i < S->max_slots; ++i)
      if (!S->slots[i].has) { slot = i; break; }
    if (slot < 0) return;
    GridEntry* ge = acquire_grid(S, job, true);
    if (!ge) return;  // head of line waits
    ge->busy = true;
    auto& a = S->slots[slot];
    a.has = true;
    a.nj = 1;
    a.job[0] = job;
    a.ge[0] = ge;
    a.t_start = S->now();
    S->queue.pop_front();
    int free_slots = 0;
    for (int i = 0; i < S->max_slots; ++i) free_slots += S->slots[i].has ? 0 : 1;
    if (batchable(a.job[0].req) && S->queue.size() > (size_t)free_slots) {
      for (size_t q = 0; q < S->queue.size() && a.nj < S->max_batch;) {
        Job& cand = S->queue[q];
        if (!same_batch(cand.req, a.job[0].req)) { ++q; continue; }
        GridEntry* g2 = acquire_grid(S, cand, false);
        if (!g2) break;
        g2->busy = true;
        a.job[a.nj] = cand;
        a.ge[a.nj] = g2;
        ++a.nj;
        S->queue.erase(S->queue.begin() + (long)q);
      }
    }
    int b = busy_slots(S);
    S->peak_busy = b > S->peak_busy ? b : S->peak_busy;
    S->cv_work.notify_all();
  }
}

vd_status ensure_grid(GridEntry* ge, const vd_request& r) {
  if (!ge->grid) {
    if (hipStreamCreateWithFlags(&ge->stream, hipStreamNonBlocking) != hipSuccess) return VD_EDEVICE;
    vd_status s = vd_grid_create(&ge->grid, &ge->desc, ge->stream);
    if (s != VD_OK) return s;
  }
  return vd_set_density(ge->grid, r.rho);
}

// Run a slot's requests; st[k], info[k] per request.
void run_batch(vd_server* S, vd_server::Assign& a, vd_status* st, vd_solve_info* info) {
  for (int k = 0; k < a.nj; ++k) std::memset(&info[k], 0, sizeof(info[k]));
  if (S->dry) {
    if (S->dry_seconds > 0) std::this_thread::sleep_for(std::chrono::duration<double>(S->dry_seconds));
    for (int k = 0; k < a.nj; ++k) {  // scheduler dry run: nothing solved
      st[k] = VD_ENOTSUP;
      info[k].status = VD_ENOTSUP;
    }
    return;
  }
  // grids and densities; a request whose grid fails is reported alone
  vd_grid* grids[kBatchMax];
  const double* f[kBatchMax];
  double* x[kBatchMax];
  int idx[kBatchMax], n = 0;
  for (int k = 0; k < a.nj; ++k) {
    const vd_request& r = a.job[k].req;
    st[k] = ensure_grid(a.ge[k], r);
    if (st[k] != VD_OK) continue;
    if (r.kind == VD_OP_HELMHOLTZ) {
      st[k] = vd_solve_helmholtz(a.ge[k]->grid, r.dt_nu, r.ncomp > 0 ? r.ncomp : 1, r.f, r.x, &r.opts, &info[k]);
      continue;
    }
    grids[n] = a.ge[k]->grid;
    f[n] = r.f;
    x[n] = r.x;
    idx[n++] = k;
  }
  if (n == 1) {
    const int k = idx[0];
    st[k] = vd_solve_pressure(grids[0], f[0], x[0], &a.job[k].req.opts, &info[k]);
  } else if (n > 1) {
    vd_solve_info inf[kBatchMax] = {};
    vd_solve_pressure_batch(grids, n, f, x, &a.job[idx[0]].req.opts, inf);  // fills every info
    for (int q = 0; q < n; ++q) {
      info[idx[q]] = inf[q];
      st[idx[q]] = (vd_status)inf[q].status;
    }
  }
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
    vd_solve_info info[kBatchMax];
    vd_status st[kBatchMax];
    run_batch(S, a, st, info);
    {
      std::lock_guard<std::mutex> lk(S->mu);
      const double t_done = S->now();
      for (int k = 0; k < a.nj; ++k) {
        vd_result res{};
        res.ticket = a.job[k].ticket;
        res.user_tag = a.job[k].req.user_tag;
        res.status = st[k];
        res.iterations = info[k].iterations;
        res.refinements = info[k].refinements;
        res.rel_residual = info[k].rel_residual;
        res.t_arrive = a.job[k].t_arrive;
        res.t_start = a.t_start;
        res.t_done = t_done;
        res.slot = slot;
        GridEntry* ge = a.ge[k];
        if (st[k] < 0 && ge->grid == nullptr && !S->dry) {
          // grid could not be created: give its budget back
          S->used -= ge->bytes;
          for (size_t i = 0; i < S->grids.size(); ++i)
            if (S->grids[i] == ge) { S->grids.erase(S->grids.begin() + i); break; }
          if (ge->stream) hipStreamDestroy(ge->stream);
          delete ge;
        } else {
          ge->busy = false;
        }
        S->done.push_back(res);
        S->in_flight--;
      }
      S->slots[slot].has = false;
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
  // options the solve would reject are rejected here, before queuing
  if (!std::isnan(r->opts.rho0) && !(r->opts.rho0 > 0.0)) return VD_EINVAL;
  if (r->kind == VD_OP_HELMHOLTZ && (!(r->dt_nu >= 0.0) || !std::isfinite(r->dt_nu))) return VD_EINVAL;
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

vd_status vd_server_set_batch(vd_server* S, int max_requests) {
  if (!S || max_requests < 1 || max_requests > kBatchMax) return VD_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  S->max_batch = max_requests;
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
