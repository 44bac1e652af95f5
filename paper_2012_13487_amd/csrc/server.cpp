// Continuous-batching server for steady-state solves (C ABI in include/dgbgk.h).
//
// Built only on the public solver and batch calls: each admitted request is a
// dgbgk_solver initialised at rest; the running requests are advanced
// together by one dgbgk_batch, rebuilt whenever the set changes, in chunks of
// check_every RK4 steps; after each chunk the batch's residuals decide which
// requests leave.  Host-side bookkeeping only: every step of the solves runs
// in the library's kernels.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "dgbgk.h"

namespace {

struct Request {
  dgbgk_problem pb{};
  std::vector<double> ex, ey, w;  // owned copies of the velocity set
  double arrival = 0.0, admit = NAN, finish = NAN, residual = NAN, dt = 0.0;
  int status = DGBGK_REQ_WAITING;
  int prec = DGBGK_FP64;  // current precision of its solver
  int64_t steps = 0, steps64 = 0, dof = 0, K = 0, Np = 0;
  double best = INFINITY;  // lowest residual so far (mixed precision: stall detection)
  int stall = 0;
  size_t bytes = 0;
  dgbgk_solver *s = nullptr;
  std::vector<double> rho, ux, uy;
  std::string error;
};

using Clock = std::chrono::steady_clock;

}  // namespace

struct dgbgk_server {
  dgbgk_server_options opt{};
  void *stream = nullptr;
  std::vector<Request> req;
  std::vector<size_t> active;  // indices into req
  dgbgk_batch *batch = nullptr;
  bool dirty = true;
  size_t used = 0;
  double clock_s = 0.0;  // server time consumed by earlier dgbgk_server_run calls
  double wall_s = 0.0;
  double dof_updates = 0.0;
  int64_t rebuilds = 0, chunks = 0, switches = 0;
  int32_t peak_active = 0;
  size_t peak_bytes = 0;
  std::string err;
};

namespace {

int sfail(dgbgk_server *sv, int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (sv) sv->err = buf;
  return code;
}

void drop_batch(dgbgk_server *sv) {
  if (sv->batch) dgbgk_batch_destroy(sv->batch);
  sv->batch = nullptr;
  sv->dirty = true;
}

// Admits request r at server time t: a solver at rest.  On failure the request
// is marked failed (the server goes on with the others).
bool ref_form(int precision) {
  return precision == DGBGK_FP32_REF || precision == DGBGK_FP32_BF16MMA_REF;
}

bool mixed(const dgbgk_server *sv) {
  return sv->opt.precision != DGBGK_FP64 && !ref_form(sv->opt.precision) &&
         sv->opt.polish_below > 0.0;
}

void admit(dgbgk_server *sv, Request &r, double t) {
  r.admit = t;
  r.prec = sv->opt.precision;
  int rc = dgbgk_create(&r.pb, r.prec, sv->stream, &r.s);
  if (!rc) rc = dgbgk_init_equilibrium(r.s, 1.0, 0.0, 0.0);
  if (!rc) rc = dgbgk_stable_dt(r.s, sv->opt.cfl, &r.dt);
  if (rc) {
    r.error = dgbgk_last_error(r.s);
    if (r.s) dgbgk_destroy(r.s);
    r.s = nullptr;
    r.status = DGBGK_REQ_FAILED;
    r.finish = t;
    return;
  }
  int32_t np = 0;
  int32_t nfp = 0, q = 0;
  dgbgk_sizes(r.s, &r.K, &np, &nfp, &q);
  r.Np = np;
  r.dof = r.K * np * q;
  r.status = DGBGK_REQ_RUNNING;
  sv->used += r.bytes;
  sv->active.push_back((size_t)(&r - sv->req.data()));
  sv->dirty = true;
  sv->peak_active = std::max(sv->peak_active, (int32_t)sv->active.size());
  sv->peak_bytes = std::max(sv->peak_bytes, sv->used);
}

// Moves a running request from its FP32 solver to an FP64 solver with the
// same state (through host memory); false if that fails.
bool switch_to_fp64(dgbgk_server *sv, Request &r) {
  std::vector<double> f((size_t)r.dof);
  dgbgk_solver *s64 = nullptr;
  int rc = dgbgk_get_state(r.s, f.data(), f.size());
  if (!rc) rc = dgbgk_create(&r.pb, DGBGK_FP64, sv->stream, &s64);
  if (!rc) rc = dgbgk_set_state(s64, f.data(), f.size());
  if (rc) {
    r.error = dgbgk_last_error(s64 ? s64 : r.s);
    if (s64) dgbgk_destroy(s64);
    return false;
  }
  dgbgk_destroy(r.s);
  r.s = s64;
  r.prec = DGBGK_FP64;
  ++sv->switches;
  return true;
}

// Copies a finished request's moments to the host and releases its device memory.
void retire(dgbgk_server *sv, Request &r, int status, double t) {
  r.status = status;
  const size_t n = (size_t)(r.K * r.Np);
  r.rho.assign(n, 0.0);
  r.ux.assign(n, 0.0);
  r.uy.assign(n, 0.0);
  if (dgbgk_moments(r.s, r.rho.data(), r.ux.data(), r.uy.data()) != DGBGK_OK) {
    r.status = DGBGK_REQ_FAILED;
    r.error = dgbgk_last_error(r.s);
  }
  r.finish = t;
  sv->dof_updates += (double)r.dof * 4.0 * (double)r.steps;
  dgbgk_destroy(r.s);
  r.s = nullptr;
  sv->used -= r.bytes;
}

double percentile(std::vector<double> v, double p) {
  if (v.empty()) return NAN;
  std::sort(v.begin(), v.end());
  const size_t k = (size_t)std::ceil(p * (double)v.size());  // nearest rank
  return v[std::min(v.size() - 1, k > 0 ? k - 1 : 0)];
}

}  // namespace

extern "C" {

int dgbgk_server_create(const dgbgk_server_options *opt, void *hip_stream, dgbgk_server **out) {
  if (!out) return DGBGK_EINVAL;
  *out = nullptr;
  if (!opt) return DGBGK_EINVAL;
  if (opt->hbm_budget == 0 || opt->max_active < 1 || !(opt->residual_target > 0) ||
      opt->check_every < 1 || opt->max_steps < 1 || !(opt->cfl > 0) ||
      (opt->precision != DGBGK_FP64 && opt->precision != DGBGK_FP32 &&
       opt->precision != DGBGK_FP32_BF16MMA && !ref_form(opt->precision)))
    return DGBGK_EINVAL;
  dgbgk_server *sv = new (std::nothrow) dgbgk_server;
  if (!sv) return DGBGK_ENOMEM;
  sv->opt = *opt;
  sv->stream = hip_stream;
  *out = sv;
  return DGBGK_OK;
}

int dgbgk_server_submit(dgbgk_server *sv, const dgbgk_problem *pb, double arrival_s, int64_t *id) {
  if (!sv) return DGBGK_EINVAL;
  if (!pb || !std::isfinite(arrival_s) || arrival_s < 0.0)
    return sfail(sv, DGBGK_EINVAL, "need a problem and an arrival time >= 0");
  size_t bytes = 0;
  int rc = dgbgk_required_bytes(pb, sv->opt.precision, &bytes);
  if (rc) return sfail(sv, rc, "invalid problem: %s", dgbgk_last_error(nullptr));
  if (mixed(sv)) {  // reserve the FP64 size the request may move to
    size_t b64 = 0;
    if (!dgbgk_required_bytes(pb, DGBGK_FP64, &b64)) bytes = std::max(bytes, b64);
  }
  if (bytes > sv->opt.hbm_budget)
    return sfail(sv, DGBGK_EINVAL, "problem needs %zu B, more than the budget of %zu B", bytes,
                 sv->opt.hbm_budget);
  Request r;
  r.ex.assign(pb->ex, pb->ex + pb->q);
  r.ey.assign(pb->ey, pb->ey + pb->q);
  r.w.assign(pb->w, pb->w + pb->q);
  r.pb = *pb;
  r.pb.ex = nullptr;  // set when admitted (the vector storage may move until then)
  r.arrival = arrival_s;
  r.bytes = bytes;
  sv->req.push_back(std::move(r));
  if (id) *id = (int64_t)sv->req.size() - 1;
  return DGBGK_OK;
}

int dgbgk_server_run(dgbgk_server *sv, double time_limit_s) {
  if (!sv) return DGBGK_EINVAL;
  if (!(time_limit_s > 0)) return sfail(sv, DGBGK_EINVAL, "time_limit_s must be > 0");
  for (Request &r : sv->req) {  // the request vector no longer grows during the run
    r.pb.ex = r.ex.data();
    r.pb.ey = r.ey.data();
    r.pb.w = r.w.data();
  }
  std::vector<size_t> order(sv->req.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](size_t a, size_t b) { return sv->req[a].arrival < sv->req[b].arrival; });
  const Clock::time_point start = Clock::now();
  auto elapsed = [&]() { return std::chrono::duration<double>(Clock::now() - start).count(); };
  auto now_s = [&]() { return sv->clock_s + elapsed(); };
  std::vector<double> dts, res;
  int rc = DGBGK_OK;
  for (;;) {
    // admission, first come first served, at chunk boundaries
    double t = now_s();
    size_t waiting = 0;
    double next_arrival = INFINITY;
    for (size_t i : order) {
      Request &r = sv->req[i];
      if (r.status != DGBGK_REQ_WAITING) continue;
      ++waiting;
      if (r.arrival > t) {
        next_arrival = std::min(next_arrival, r.arrival);
        continue;
      }
      if ((int32_t)sv->active.size() >= sv->opt.max_active || sv->used + r.bytes > sv->opt.hbm_budget)
        break;
      drop_batch(sv);
      admit(sv, r, t);
      --waiting;
    }
    if (sv->active.empty()) {
      if (waiting == 0) break;  // every request has completed
      const double wait = std::isfinite(next_arrival) ? next_arrival - now_s() : 0.0;
      if (elapsed() + std::max(wait, 0.0) > time_limit_s) {
        rc = sfail(sv, DGBGK_ESTATE, "time limit reached with requests waiting");
        break;
      }
      if (wait > 0) std::this_thread::sleep_for(std::chrono::duration<double>(wait));
      continue;
    }
    if (elapsed() > time_limit_s) {
      rc = sfail(sv, DGBGK_ESTATE, "time limit reached with requests running");
      break;
    }
    if (sv->dirty || !sv->batch) {
      drop_batch(sv);
      std::vector<dgbgk_solver *> ss;
      for (size_t i : sv->active) ss.push_back(sv->req[i].s);
      int brc = dgbgk_batch_create(ss.data(), (int32_t)ss.size(), sv->stream, &sv->batch);
      // up to 10 RK4 steps per captured graph: fewer launches per chunk, while
      // the capture (repeated at every change of membership) stays short
      if (!brc && sv->opt.use_graph)
        brc = dgbgk_batch_set_graph(sv->batch, std::min(10, sv->opt.check_every));
      if (brc) {
        rc = sfail(sv, brc, "batch: %s", dgbgk_batch_last_error(sv->batch));
        break;
      }
      sv->dirty = false;
      ++sv->rebuilds;
    }
    dts.clear();
    for (size_t i : sv->active) dts.push_back(sv->req[i].dt);
    res.assign(sv->active.size(), NAN);
    int brc = dgbgk_batch_step(sv->batch, sv->opt.check_every, dts.data());
    if (!brc) brc = dgbgk_batch_residuals(sv->batch, res.data());
    if (brc && brc != DGBGK_ENONFINITE) {
      rc = sfail(sv, brc, "batch step: %s", dgbgk_batch_last_error(sv->batch));
      break;
    }
    ++sv->chunks;
    t = now_s();
    std::vector<size_t> keep;
    bool any_done = false;
    for (size_t k = 0; k < sv->active.size(); ++k) {
      Request &r = sv->req[sv->active[k]];
      r.steps += sv->opt.check_every;
      if (r.prec == DGBGK_FP64 && mixed(sv)) r.steps64 += sv->opt.check_every;
      r.residual = res[k];
      int status = DGBGK_REQ_RUNNING;
      if (!std::isfinite(res[k])) status = DGBGK_REQ_FAILED;
      else if (res[k] < sv->opt.residual_target) status = DGBGK_REQ_CONVERGED;
      else if (r.steps >= sv->opt.max_steps) status = DGBGK_REQ_STOPPED;
      if (status == DGBGK_REQ_RUNNING && r.prec != DGBGK_FP64 && mixed(sv)) {
        // below the polish threshold, or no longer falling: finish in FP64
        if (res[k] < 0.9 * r.best) {
          r.best = res[k];
          r.stall = 0;
        } else {
          ++r.stall;
        }
        if (res[k] < sv->opt.polish_below || r.stall >= 20) {
          if (!any_done) drop_batch(sv);
          any_done = true;
          if (!switch_to_fp64(sv, r)) status = DGBGK_REQ_FAILED;
        }
      }
      if (status == DGBGK_REQ_RUNNING && ref_form(r.prec) && dgbgk_fold(r.s) != DGBGK_OK) {
        r.error = dgbgk_last_error(r.s);
        status = DGBGK_REQ_FAILED;
      }
      if (status == DGBGK_REQ_RUNNING) {
        keep.push_back(sv->active[k]);
        continue;
      }
      if (!any_done) drop_batch(sv);  // the batch refers to the solvers about to go
      any_done = true;
      retire(sv, sv->req[sv->active[k]], status, t);
    }
    sv->active.swap(keep);
  }
  sv->clock_s += elapsed();
  sv->wall_s += elapsed();
  return rc;
}

int dgbgk_server_result(const dgbgk_server *sv, int64_t id, dgbgk_request_result *out) {
  if (!sv || !out) return DGBGK_EINVAL;
  if (id < 0 || id >= (int64_t)sv->req.size())
    return sfail(const_cast<dgbgk_server *>(sv), DGBGK_EINVAL, "no request %lld", (long long)id);
  const Request &r = sv->req[(size_t)id];
  out->status = r.status;
  out->arrival_s = r.arrival;
  out->admit_s = r.admit;
  out->finish_s = r.finish;
  out->steps = r.steps;
  out->residual = r.residual;
  out->dof = r.dof;
  out->K = r.K;
  out->Np = r.Np;
  out->steps_fp64 = r.steps64;
  return DGBGK_OK;
}

int dgbgk_server_moments(const dgbgk_server *sv, int64_t id, double *rho, double *ux, double *uy) {
  if (!sv || !rho || !ux || !uy) return DGBGK_EINVAL;
  dgbgk_server *m = const_cast<dgbgk_server *>(sv);
  if (id < 0 || id >= (int64_t)sv->req.size())
    return sfail(m, DGBGK_EINVAL, "no request %lld", (long long)id);
  const Request &r = sv->req[(size_t)id];
  if (r.rho.empty()) return sfail(m, DGBGK_ESTATE, "request %lld has no result", (long long)id);
  std::memcpy(rho, r.rho.data(), r.rho.size() * sizeof(double));
  std::memcpy(ux, r.ux.data(), r.ux.size() * sizeof(double));
  std::memcpy(uy, r.uy.data(), r.uy.size() * sizeof(double));
  return DGBGK_OK;
}

int dgbgk_server_get_stats(const dgbgk_server *sv, dgbgk_server_stats *out) {
  if (!sv || !out) return DGBGK_EINVAL;
  std::vector<double> lat;
  int64_t done = 0, admitted = 0;
  double all = 0.0;
  for (const Request &r : sv->req) {
    if (r.status >= DGBGK_REQ_CONVERGED) {
      ++done;
      lat.push_back(r.finish - r.arrival);
    }
    if (r.status != DGBGK_REQ_WAITING) ++admitted;
    all += (double)r.dof * 4.0 * (double)r.steps;
  }
  out->submitted = (int64_t)sv->req.size();
  out->completed = done;
  out->wall_s = sv->wall_s;
  out->dof_updates = sv->dof_updates;
  out->latency_p50_s = percentile(lat, 0.50);
  out->latency_p99_s = percentile(lat, 0.99);
  out->batch_rebuilds = sv->rebuilds;
  out->chunks = sv->chunks;
  out->peak_active = sv->peak_active;
  out->peak_bytes = sv->peak_bytes;
  out->precision_switches = sv->switches;
  out->dof_updates_all = all;
  out->admitted = admitted;
  return DGBGK_OK;
}

const char *dgbgk_server_last_error(const dgbgk_server *sv) {
  if (!sv) return "server is NULL";
  return sv->err.c_str();
}

void dgbgk_server_destroy(dgbgk_server *sv) {
  if (!sv) return;
  drop_batch(sv);
  for (Request &r : sv->req)
    if (r.s) dgbgk_destroy(r.s);
  delete sv;
}

}  // extern "C"
