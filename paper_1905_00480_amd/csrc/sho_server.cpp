// sho_server.cpp -- request server over many resident systems (C ABI).
//
// Every registered system keeps a pinned host copy of its inputs (psi and
// the coefficients w that expansion and derivative requests use).  On its
// first request, or after an eviction, it is admitted: a plan is built, its
// device buffers are allocated and the inputs are copied up on the system's
// stream.  The resident set is bounded by a byte budget; when an admission
// does not fit, the least recently used other systems are evicted (their
// last request is waited for, their device memory freed; inputs are never
// modified on the device, so nothing is copied back).
//
// Every request goes to the stream with the least outstanding work (the
// estimated cost of its requests not yet completed: support points x bands
// x a factor per job kind), so that small requests do not queue behind large
// ones; a request placed on another stream than its system's previous one
// first waits for that request (an event), so the requests of one system
// still run in submission order.  A poller thread timestamps every request
// when its completion event has fired, without taking the admission lock, so
// that latencies are not inflated by a concurrent admission.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "sho_launch.hpp"

namespace {

using Clock = std::chrono::steady_clock;

struct Sys {
  sho_grid grid{};
  int32_t natoms = 0, nbands = 0;
  std::vector<double> pos, sigma;
  std::vector<int32_t> numax;
  int64_t psi_doubles = 0, coeff_doubles = 0;
  int64_t charge = 0;        // bytes charged against the budget while resident
  int64_t table_charge = 0;  // of which the plan's tables (kept while parked)
  double *h_psi = nullptr, *h_w = nullptr;  // pinned inputs
  // resident: plan, scratch and buffers on the device; parked: only the
  // plan's tables (evicted, the host-side plan build is kept); else neither
  bool resident = false;
  bool parked = false;
  sho_plan_t plan = nullptr;
  double *d_psi = nullptr, *d_w = nullptr, *d_c = nullptr, *d_grad = nullptr,
         *d_out = nullptr;
  int stream = 0;             // stream of the latest request (or the upload)
  double units = 0.0;         // support points x bands (cost of a request)
  hipEvent_t last = nullptr;  // after the latest request (or upload) of this system
  uint64_t last_use = 0;
  std::atomic<int32_t> inflight{0};
  int64_t done_by_job[3] = {0, 0, 0};
};

struct Req {
  int64_t id = 0;
  Sys *sysp = nullptr;
  int32_t sys = 0, job = 0;
  int32_t stream = 0;
  double cost = 0.0;  // estimated work, counted on its stream until done
  sho_status status = SHO_OK;
  double t_submit = 0.0;
  std::atomic<double> t_done{-1.0};
  hipEvent_t ev = nullptr;
};

}  // namespace

struct sho_server_s {
  int64_t budget = 0;
  uint32_t flags = 0;
  bool dry = false;  // SHO_FLAG_HOST_ONLY: admission bookkeeping only
  std::vector<hipStream_t> streams;
  std::mutex wmu;                    // stream_work
  std::vector<double> stream_work;   // outstanding estimated work per stream
  // estimated costs of the latest requests (ring), for the short-request rule
  static constexpr int kRecent = 256;
  double recent[kRecent] = {};
  int64_t nrecent = 0;
  int64_t express = 0;  // requests sent to the short-request stream
  std::deque<std::unique_ptr<Sys>> systems;
  std::deque<std::unique_ptr<Req>> reqs;  // stable addresses
  int64_t resident_bytes = 0, peak_bytes = 0;
  int64_t admissions = 0, evictions = 0, rejected = 0;
  int64_t plan_reuses = 0, plan_drops = 0;
  uint64_t tick = 0;
  Clock::time_point t0 = Clock::now();
  std::mutex mu;  // systems, admission, submission

  // completion poller
  std::mutex pmu;
  std::condition_variable pcv;
  std::vector<Req *> pending;
  std::atomic<int64_t> completed{0};
  std::atomic<bool> stop{false};
  std::thread poller;

  double now() const {
    return std::chrono::duration<double>(Clock::now() - t0).count();
  }
};

namespace {

using sho::fail;
using sho::hip_fail;

void poll_loop(sho_server_s *S) {
  std::vector<Req *> mine;
  for (;;) {
    {
      // block only while nothing is outstanding; otherwise just take what
      // was submitted since the last scan
      std::unique_lock<std::mutex> lk(S->pmu);
      if (mine.empty())
        S->pcv.wait_for(lk, std::chrono::milliseconds(2),
                        [&] { return S->stop.load() || !S->pending.empty(); });
      mine.insert(mine.end(), S->pending.begin(), S->pending.end());
      S->pending.clear();
      if (S->stop.load() && mine.empty()) return;
    }
    bool any = false;
    for (Req *&r : mine) {
      const hipError_t q = hipEventQuery(r->ev);
      if (q == hipErrorNotReady) continue;
      const double t = S->now();
      if (q != hipSuccess) (void)hipGetLastError();
      (void)hipEventDestroy(r->ev);
      r->ev = nullptr;
      if (q != hipSuccess) r->status = SHO_E_DEVICE;
      r->t_done.store(t);
      {
        std::lock_guard<std::mutex> wl(S->wmu);
        S->stream_work[r->stream] -= r->cost;
      }
      r->sysp->inflight--;
      S->completed++;
      r = nullptr;
      any = true;
    }
    mine.erase(std::remove(mine.begin(), mine.end(), nullptr), mine.end());
    if (!any && !mine.empty()) std::this_thread::sleep_for(std::chrono::microseconds(20));
    if (S->stop.load() && mine.empty()) {
      std::lock_guard<std::mutex> lk(S->pmu);
      if (S->pending.empty()) return;
    }
  }
}

// Frees a system's buffers (psi, out, w, c, grad) once its queued work is done.
void free_buffers(Sys &y) {
  if (y.last) (void)hipEventSynchronize(y.last);
  for (double *q : {y.d_psi, y.d_w, y.d_c, y.d_grad, y.d_out})
    if (q) (void)hipFree(q);
  y.d_psi = y.d_w = y.d_c = y.d_grad = y.d_out = nullptr;
}

void free_plan(Sys &y) {
  if (y.plan) (void)sho_plan_destroy(y.plan);
  if (y.last) (void)hipEventDestroy(y.last);
  y.plan = nullptr;
  y.last = nullptr;
}

// Resident -> parked: the buffers and the plan's scratch go, the plan's
// tables stay (a later admission skips the host-side plan build).
void park(sho_server_s *S, Sys &y) {
  if (!S->dry) {
    free_buffers(y);
    if (y.plan) (void)sho_plan_release_scratch(y.plan);
  }
  y.resident = false;
  y.parked = true;
  S->resident_bytes -= y.charge - y.table_charge;
}

// Parked -> not on the device at all.
void drop(sho_server_s *S, Sys &y) {
  if (!S->dry) free_plan(y);
  y.parked = false;
  S->resident_bytes -= y.table_charge;
  S->plan_drops++;
}

// Makes room for `need` more bytes: parks least recently used resident
// systems other than `keep`, then, if that is not enough, drops least
// recently used parked plans.  Returns false if even that would not do.
bool make_room(sho_server_s *S, int64_t need, int32_t keep) {
  if (need > S->budget) return false;
  auto lru = [&](bool resident) {
    Sys *victim = nullptr;
    for (size_t k = 0; k < S->systems.size(); ++k) {
      Sys &y = *S->systems[k];
      if ((int32_t)k == keep || (resident ? !y.resident : !y.parked)) continue;
      if (!victim || y.last_use < victim->last_use) victim = &y;
    }
    return victim;
  };
  while (S->resident_bytes + need > S->budget) {
    Sys *victim = lru(true);
    if (!victim) break;
    park(S, *victim);
    S->evictions++;
  }
  while (S->resident_bytes + need > S->budget) {
    Sys *victim = lru(false);
    if (!victim) return false;
    drop(S, *victim);
  }
  return true;
}

// The stream with the least outstanding work among streams first..n-1.
int least_loaded(sho_server_s *S, int first = 0) {
  std::lock_guard<std::mutex> wl(S->wmu);
  const int n = (int)S->stream_work.size();
  int best = std::min(first, n - 1);
  for (int k = best + 1; k < n; ++k)
    if (S->stream_work[k] < S->stream_work[best]) best = k;
  return best;
}

// Stream of a request of estimated cost `cost`.  With two or more streams
// the first one is kept for short requests, so that they never queue behind
// a long one: a request is short when its cost is at most both the median
// and half the mean of the latest kRecent requests' costs (the current one
// included; a pool of equal requests has none).  Every other request goes to
// the remaining stream with the least outstanding work.
int choose_stream(sho_server_s *S, double cost, bool *is_short) {
  S->recent[S->nrecent % sho_server_s::kRecent] = cost;
  S->nrecent++;
  *is_short = false;
  const int n = (int)S->stream_work.size();
  if (n < 2) return 0;
  const int m = (int)std::min<int64_t>(S->nrecent, sho_server_s::kRecent);
  double v[sho_server_s::kRecent];
  double sum = 0.0;
  for (int k = 0; k < m; ++k) sum += (v[k] = S->recent[k]);
  std::nth_element(v, v + m / 2, v + m);
  if (cost <= v[m / 2] && cost <= 0.5 * sum / m) {
    *is_short = true;
    return 0;
  }
  return least_loaded(S, 1);
}

sho_status admit(sho_server_s *S, int32_t id) {
  Sys &y = *S->systems[id];
  const bool reuse = y.parked;  // the plan's tables are still on the device
  const int64_t need = reuse ? y.charge - y.table_charge : y.charge;
  if (y.charge > S->budget || !make_room(S, need, id)) {
    S->rejected++;
    return fail(SHO_E_BUDGET, "system needs " + std::to_string(y.charge) +
                                  " bytes of a budget of " + std::to_string(S->budget));
  }
  if (!S->dry) {
    // inputs are uploaded on a stream of the long requests
    const int best = least_loaded(S, S->stream_work.size() > 1 ? 1 : 0);
    y.stream = best;
    hipStream_t st = S->streams[best];
    sho_status r = SHO_OK;
    if (!reuse)
      r = sho_plan_create(&y.grid, y.natoms, y.pos.data(), y.sigma.data(), y.numax.data(),
                          nullptr, y.nbands, S->flags, &y.plan);
    hipError_t e = hipSuccess;
    const size_t pb = y.psi_doubles * sizeof(double), cb = std::max<int64_t>(y.coeff_doubles, 1) * 8;
    if (r == SHO_OK) {
      if ((e = hipMalloc((void **)&y.d_psi, pb)) == hipSuccess &&
          (e = hipMalloc((void **)&y.d_out, pb)) == hipSuccess &&
          (e = hipMalloc((void **)&y.d_w, cb)) == hipSuccess &&
          (e = hipMalloc((void **)&y.d_c, cb)) == hipSuccess &&
          (e = hipMalloc((void **)&y.d_grad, std::max(3 * y.natoms, 1) * sizeof(double))) ==
              hipSuccess &&
          (y.last || (e = hipEventCreateWithFlags(&y.last, hipEventDisableTiming)) == hipSuccess) &&
          (e = hipMemcpyAsync(y.d_psi, y.h_psi, pb, hipMemcpyHostToDevice, st)) == hipSuccess &&
          (e = hipMemcpyAsync(y.d_w, y.h_w, y.coeff_doubles * sizeof(double),
                              hipMemcpyHostToDevice, st)) == hipSuccess)
        e = hipEventRecord(y.last, st);  // requests on other streams wait for the upload
    }
    if (r != SHO_OK || e != hipSuccess) {
      const std::string why = r != SHO_OK ? std::string(sho_last_error()) : "";
      free_buffers(y);
      free_plan(y);
      if (reuse) {
        y.parked = false;
        S->resident_bytes -= y.table_charge;
      }
      if (r != SHO_OK) return fail(r, "admission: " + why);
      return e == hipErrorOutOfMemory ? fail(SHO_E_NOMEM, "admission: device allocation failed")
                                      : hip_fail(e, "admission");
    }
  }
  if (reuse) S->plan_reuses++;
  y.parked = false;
  y.resident = true;
  S->resident_bytes += need;
  S->peak_bytes = std::max(S->peak_bytes, S->resident_bytes);
  S->admissions++;
  return SHO_OK;
}

// Relative cost of a job on a system of `units` support points x bands
// (measured: an expansion and a derivative take about 1.4 and 1.3 times a
// projection).
double job_cost(double units, int32_t job) {
  static const double factor[3] = {1.0, 1.4, 1.3};
  return units * factor[job];
}

sho_status launch_job(sho_server_s *S, Sys &y, int32_t job) {
  hipStream_t st = S->streams[y.stream];
  sho_status r = SHO_OK;
  if (job == SHO_JOB_PROJECT) {
    r = sho_plan_project(y.plan, y.d_psi, y.d_c, st);
  } else if (job == SHO_JOB_EXPAND) {
    hipError_t e = sho::launch_fill(y.d_out, y.psi_doubles, 0.0, st);
    if (e != hipSuccess) return hip_fail(e, "fill");
    r = sho_plan_expand(y.plan, y.d_w, y.d_out, st);
  } else {
    r = sho_plan_force(y.plan, y.d_psi, y.d_w, y.d_grad, st);
  }
  return r;
}

}  // namespace

extern "C" {

sho_status sho_server_create(int64_t budget_bytes, int32_t nstreams, uint32_t plan_flags,
                             sho_server_t *out) {
  if (!out) return fail(SHO_E_INVALID, "out must not be NULL");
  *out = nullptr;
  if (budget_bytes <= 0) return fail(SHO_E_INVALID, "budget must be positive");
  if (nstreams < 1 || nstreams > 16) return fail(SHO_E_INVALID, "nstreams outside 1..16");
  if (plan_flags & ~(uint32_t)(SHO_FLAG_HOST_ONLY | SHO_FLAG_PER_ATOM | SHO_FLAG_STORED |
                               SHO_FLAG_ALLOW_UNDERSAMPLED))
    return fail(SHO_E_INVALID, "unknown plan flags");
  std::unique_ptr<sho_server_s> S(new (std::nothrow) sho_server_s());
  if (!S) return fail(SHO_E_NOMEM, "host allocation failed");
  S->budget = budget_bytes;
  S->flags = plan_flags;
  S->dry = (plan_flags & SHO_FLAG_HOST_ONLY) != 0;
  if (!S->dry) {
    for (int i = 0; i < nstreams; ++i) {
      hipStream_t st = nullptr;
      hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
      if (e != hipSuccess) {
        for (hipStream_t q : S->streams) (void)hipStreamDestroy(q);
        return hip_fail(e, "stream creation");
      }
      S->streams.push_back(st);
    }
    S->poller = std::thread(poll_loop, S.get());
  }
  S->stream_work.assign(nstreams, 0.0);
  *out = S.release();
  return SHO_OK;
}

sho_status sho_server_add_system(sho_server_t S, const sho_grid *grid, int32_t natoms,
                                 const double *pos, const double *sigma,
                                 const int32_t *numax, int32_t nbands,
                                 const double *psi, const double *w, int32_t *id) {
  if (!S || !id) return fail(SHO_E_INVALID, "NULL server or id");
  // validate and size with a host-only plan of the same flags
  sho_plan_t hp = nullptr;
  sho_status r = sho_plan_create(grid, natoms, pos, sigma, numax, nullptr, nbands,
                                 S->flags | SHO_FLAG_HOST_ONLY, &hp);
  if (r != SHO_OK) return r;
  sho_plan_info info;
  r = sho_plan_get_info(hp, &info);
  (void)sho_plan_destroy(hp);
  if (r != SHO_OK) return r;
  std::unique_ptr<Sys> y(new (std::nothrow) Sys());
  if (!y) return fail(SHO_E_NOMEM, "host allocation failed");
  y->grid = *grid;
  y->natoms = natoms;
  y->nbands = nbands;
  y->pos.assign(pos, pos + 3 * (size_t)natoms);
  y->sigma.assign(sigma, sigma + natoms);
  y->numax.assign(numax, numax + natoms);
  y->psi_doubles = (int64_t)grid->n[0] * grid->n[1] * grid->n[2] * nbands;
  y->coeff_doubles = info.coeff_doubles;
  // plan tables + psi + out + w + c + grad, each rounded up to 4 KiB
  auto pg = [](int64_t b) { return (b + 4095) / 4096 * 4096; };
  y->charge = pg(info.device_bytes) + 2 * pg(y->psi_doubles * 8) +
              2 * pg(std::max<int64_t>(y->coeff_doubles, 1) * 8) + pg(24 * std::max(natoms, 1));
  // the plan's tables without its scratch (the plane partials)
  y->table_charge =
      pg(info.device_bytes - std::max<int64_t>(info.expand_scratch_doubles, 1) * 8);
  y->units = (double)info.support_points * nbands;
  if (!S->dry) {
    hipError_t e = hipHostMalloc((void **)&y->h_psi, y->psi_doubles * sizeof(double));
    if (e == hipSuccess)
      e = hipHostMalloc((void **)&y->h_w, std::max<int64_t>(y->coeff_doubles, 1) * 8);
    if (e != hipSuccess) {
      if (y->h_psi) (void)hipHostFree(y->h_psi);
      return e == hipErrorOutOfMemory ? fail(SHO_E_NOMEM, "pinned host allocation failed")
                                      : hip_fail(e, "pinned host allocation");
    }
    if (psi)
      std::memcpy(y->h_psi, psi, y->psi_doubles * sizeof(double));
    else
      std::memset(y->h_psi, 0, y->psi_doubles * sizeof(double));
    if (w)
      std::memcpy(y->h_w, w, y->coeff_doubles * sizeof(double));
    else
      std::memset(y->h_w, 0, std::max<int64_t>(y->coeff_doubles, 1) * sizeof(double));
  }
  std::lock_guard<std::mutex> lk(S->mu);
  *id = (int32_t)S->systems.size();
  S->systems.push_back(std::move(y));
  return SHO_OK;
}

sho_status sho_server_submit(sho_server_t S, int32_t sys, int32_t job, int64_t *request) {
  if (!S) return fail(SHO_E_INVALID, "NULL server");
  if (job < 0 || job > 2) return fail(SHO_E_INVALID, "unknown job");
  std::lock_guard<std::mutex> lk(S->mu);
  if (sys < 0 || sys >= (int32_t)S->systems.size())
    return fail(SHO_E_INVALID, "unknown system");
  const double t_submit = S->now();
  Sys &y = *S->systems[sys];
  if (!y.resident) {
    sho_status r = admit(S, sys);
    if (r != SHO_OK) return r;
  }
  y.last_use = ++S->tick;
  std::unique_ptr<Req> q(new (std::nothrow) Req());
  if (!q) return fail(SHO_E_NOMEM, "host allocation failed");
  q->id = (int64_t)S->reqs.size();
  q->sys = sys;
  q->sysp = &y;
  q->job = job;
  q->t_submit = t_submit;
  // short requests on their own stream, the others by least outstanding
  // work; after the system's previous request if that ran (or its inputs
  // were uploaded) on another stream
  q->cost = job_cost(y.units, job);
  bool is_short = false;
  const int st_new = choose_stream(S, q->cost, &is_short);
  if (is_short) S->express++;
  if (!S->dry) {
    if (st_new != y.stream) {
      hipError_t e = hipStreamWaitEvent(S->streams[st_new], y.last, 0);
      if (e != hipSuccess) return hip_fail(e, "stream ordering");
      y.stream = st_new;
    }
    std::lock_guard<std::mutex> wl(S->wmu);
    S->stream_work[y.stream] += q->cost;
  }
  q->stream = y.stream;
  if (S->dry) {
    q->t_done.store(t_submit);
    y.done_by_job[job]++;
    S->completed++;
  } else {
    auto unclaim = [&]() {
      std::lock_guard<std::mutex> wl(S->wmu);
      S->stream_work[y.stream] -= q->cost;
    };
    sho_status r = launch_job(S, y, job);
    if (r != SHO_OK) {
      unclaim();
      return r;
    }
    hipStream_t st = S->streams[y.stream];
    hipError_t e = hipEventCreateWithFlags(&q->ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(q->ev, st);
    if (e == hipSuccess) e = hipEventRecord(y.last, st);
    if (e != hipSuccess) {
      if (q->ev) (void)hipEventDestroy(q->ev);
      unclaim();
      return hip_fail(e, "completion event");
    }
    y.inflight++;
    y.done_by_job[job]++;
  }
  if (request) *request = q->id;
  Req *raw = q.get();
  S->reqs.push_back(std::move(q));
  if (!S->dry) {
    std::lock_guard<std::mutex> pl(S->pmu);
    S->pending.push_back(raw);
    S->pcv.notify_one();
  }
  return SHO_OK;
}

sho_status sho_server_prefetch(sho_server_t S, int32_t sys) {
  if (!S) return fail(SHO_E_INVALID, "NULL server");
  std::lock_guard<std::mutex> lk(S->mu);
  if (sys < 0 || sys >= (int32_t)S->systems.size())
    return fail(SHO_E_INVALID, "unknown system");
  Sys &y = *S->systems[sys];
  if (!y.resident) {
    sho_status r = admit(S, sys);
    if (r != SHO_OK) return r;
  }
  y.last_use = ++S->tick;
  if (!S->dry) {
    hipError_t e = hipEventRecord(y.last, S->streams[y.stream]);
    if (e == hipSuccess) e = hipEventSynchronize(y.last);
    if (e != hipSuccess) return hip_fail(e, "prefetch");
  }
  return SHO_OK;
}

sho_status sho_server_drain(sho_server_t S) {
  if (!S) return fail(SHO_E_INVALID, "NULL server");
  if (S->dry) return SHO_OK;
  for (hipStream_t st : S->streams) {
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "drain");
  }
  int64_t total = 0;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    total = (int64_t)S->reqs.size();
  }
  while (S->completed.load() < total) std::this_thread::sleep_for(std::chrono::microseconds(50));
  return SHO_OK;
}

sho_status sho_server_request_info(sho_server_t S, int64_t request, int32_t *sys,
                                   int32_t *job, double *t_submit, double *t_done) {
  if (!S || !sys || !job || !t_submit || !t_done) return fail(SHO_E_INVALID, "NULL argument");
  std::lock_guard<std::mutex> lk(S->mu);
  if (request < 0 || request >= (int64_t)S->reqs.size())
    return fail(SHO_E_INVALID, "unknown request");
  const Req &q = *S->reqs[request];
  *sys = q.sys;
  *job = q.job;
  *t_submit = q.t_submit;
  *t_done = q.t_done.load();
  return q.status;
}

sho_status sho_server_read(sho_server_t S, int32_t sys, int32_t what, double *host) {
  if (!S || !host) return fail(SHO_E_INVALID, "NULL argument");
  std::lock_guard<std::mutex> lk(S->mu);
  if (sys < 0 || sys >= (int32_t)S->systems.size())
    return fail(SHO_E_INVALID, "unknown system");
  Sys &y = *S->systems[sys];
  if (S->dry || !y.resident) return fail(SHO_E_INVALID, "system is not resident");
  const double *src = nullptr;
  int64_t n = 0;
  if (what == SHO_JOB_PROJECT) {
    src = y.d_c;
    n = y.coeff_doubles;
  } else if (what == SHO_JOB_EXPAND) {
    src = y.d_out;
    n = y.psi_doubles;
  } else if (what == SHO_JOB_FORCE) {
    src = y.d_grad;
    n = 3 * (int64_t)y.natoms;
  } else {
    return fail(SHO_E_INVALID, "unknown output");
  }
  hipError_t e = hipEventSynchronize(y.last);
  if (e == hipSuccess && n) e = hipMemcpy(host, src, n * sizeof(double), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "read");
  return SHO_OK;
}

sho_status sho_server_get_stats(sho_server_t S, sho_server_stats *st) {
  if (!S || !st) return fail(SHO_E_INVALID, "NULL argument");
  std::lock_guard<std::mutex> lk(S->mu);
  st->budget_bytes = S->budget;
  st->resident_bytes = S->resident_bytes;
  st->peak_resident_bytes = S->peak_bytes;
  st->requests = (int64_t)S->reqs.size();
  st->completed = S->completed.load();
  st->admissions = S->admissions;
  st->evictions = S->evictions;
  st->rejected = S->rejected;
  int32_t res = 0;
  for (const auto &y : S->systems) res += y->resident ? 1 : 0;
  st->systems = (int32_t)S->systems.size();
  st->resident_systems = res;
  st->short_requests = S->express;
  st->plan_reuses = S->plan_reuses;
  st->plan_drops = S->plan_drops;
  return SHO_OK;
}

sho_status sho_server_system_info(sho_server_t S, int32_t sys, int64_t *charge_bytes,
                                  int32_t *resident) {
  if (!S || !charge_bytes || !resident) return fail(SHO_E_INVALID, "NULL argument");
  std::lock_guard<std::mutex> lk(S->mu);
  if (sys < 0 || sys >= (int32_t)S->systems.size())
    return fail(SHO_E_INVALID, "unknown system");
  *charge_bytes = S->systems[sys]->charge;
  *resident = S->systems[sys]->resident ? 1 : 0;
  return SHO_OK;
}

sho_status sho_server_inputs(sho_server_t S, int32_t sys, double **psi, double **w) {
  if (!S || !psi || !w) return fail(SHO_E_INVALID, "NULL argument");
  std::lock_guard<std::mutex> lk(S->mu);
  if (sys < 0 || sys >= (int32_t)S->systems.size())
    return fail(SHO_E_INVALID, "unknown system");
  *psi = S->systems[sys]->h_psi;
  *w = S->systems[sys]->h_w;
  return SHO_OK;
}

sho_status sho_server_clock(sho_server_t S, double *now) {
  if (!S || !now) return fail(SHO_E_INVALID, "NULL argument");
  *now = S->now();
  return SHO_OK;
}

sho_status sho_server_destroy(sho_server_t S) {
  if (!S) return SHO_OK;
  sho_status r = SHO_OK;
  if (!S->dry) {
    r = sho_server_drain(S);
    S->stop.store(true);
    S->pcv.notify_one();
    if (S->poller.joinable()) S->poller.join();
  }
  for (auto &y : S->systems) {
    if (y->resident) park(S, *y);
    if (y->parked) drop(S, *y);
    if (y->h_psi) (void)hipHostFree(y->h_psi);
    if (y->h_w) (void)hipHostFree(y->h_w);
  }
  for (hipStream_t st : S->streams) (void)hipStreamDestroy(st);
  delete S;
  return r;
}

}  // extern "C"
