// Continuous-batching request server.  Requests (complete problem
// descriptions) are queued on submission and admitted while the estimated
// device memory of the admitted set stays within the budget and a slot is
// free.  A preparer thread builds each admitted request's context (scattering
// matrix, contour, tables, right-hand side) on the request's own stream; the
// worker thread advances every prepared request by one solver step per tick,
// launching all of them before waiting for any, so the work of different
// requests overlaps on the device.  A request that finishes frees its slot
// and memory at once and waiting requests are admitted on the next tick.
// Every request runs with its own buffers and fixed launch shapes, so its
// result does not depend on what else is in flight.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <algorithm>
#include <vector>

#include "solve_sm.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Job {
  uint64_t ticket = 0;
  // request copy
  mpsl_request req{};
  std::vector<double> xy, rot;
  std::vector<mpsl_c128> S;
  size_t bytes = 0;
  // state
  enum State { kQueued, kPreparing, kActive, kDone } state = kQueued;
  mpsl_ctx *ctx = nullptr;
  hipStream_t stream = nullptr;
  std::unique_ptr<mpsl::SolveSM> sm;
  int status = MPSL_OK;
  std::string err;
  std::vector<mpsl_c128> beta;
  double t_submit = 0, t_admit = 0, t_start = 0, t_finish = 0;
  int iterations = 0, fp64_mv = 0, refin = 0;
  double rel_res = 0.0;
};

// Contour node count of a request (host rule of the library).
size_t request_nodes(const mpsl_request &r) {
  if (r.contour != MPSL_CONTOUR_SPAN) return static_cast<size_t>(r.n_nodes);
  const double re[3] = {r.k1.re, r.k2.re, r.k3.re};
  int ns = 0;
  if (mpsl_compute_contour_span(3, re, r.b, r.t_max, r.h_max, 0, nullptr, nullptr, &ns) != MPSL_OK) return 0;
  return static_cast<size_t>(ns);
}

size_t estimate_bytes(const mpsl_request &r) {
  const size_t n = static_cast<size_t>(r.n), P = 2 * static_cast<size_t>(r.p) + 1;
  const size_t ns = request_nodes(r);
  const int maxit = r.opts.maxiter > 0 ? r.opts.maxiter : 500;
  const size_t m = static_cast<size_t>((r.opts.restart > 0 && r.opts.restart < maxit) ? r.opts.restart : maxit);
  const size_t tb = (n + 127) / 128;
  const size_t ca = std::min(n, (2560 + tb - 1) / tb), cb = std::max<size_t>(1, std::min(ns / 8, (1024 + tb - 1) / tb));
  // far field: all-pairs tables, or the FMM (default above 8000 particles)
  // with its neighbour lists, per-particle shift rows and box expansions
  size_t b = n > 8000 ? 32768 * n + (64 << 20) : 96 * n * n;
  if (r.sommerfeld == MPSL_SOMM_INTERP)
    b += ns * 24 * 8 + 2 * ns * 16 + n * 64 * P;  // interpolation weights, node maps, tile sums
  else
    b += 2 * 2 * n * ns * 24;                  // plane-wave factors E, F, both precisions
  b += n * P * 24 + ns * P * 128;              // rotation phases, per-node tables
  b += (2 * ca + cb) * n * P * 16;             // partial local expansions (tuning headroom)
  // Krylov basis (FP32 in the mixed-precision solve) and solver vectors
  b += (m + 1) * n * P * (r.opts.precision == MPSL_FP32 ? 8 : 16) + 6 * n * P * 16 + 2 * n * P * 8;
  b += 4 * n * P * 16 + (m + 2) * 64 * 16;     // staging and reduction scratch
  if (r.precond == MPSL_PRECOND_CLUSTER && r.xy) {  // inverse cluster blocks (FP64 while built)
    const int size = r.cluster_size > 0 ? r.cluster_size : mpsl::kPcDefaultSize;
    int nc = 0, mp = 0;
    if (mpsl::cluster_shape(r.n, r.xy, size, &nc, &mp) == MPSL_OK) {
      const size_t mb = (static_cast<size_t>(mp) * P + 63) / 64 * 64;
      b += static_cast<size_t>(nc) * mb * mb * (r.opts.precision == MPSL_FP32 ? 24 : 16);
    }
  }
  return b;
}

double now_s(Clock::time_point t0) { return std::chrono::duration<double>(Clock::now() - t0).count(); }

}  // namespace

struct mpsl_server {
  int device = 0;
  size_t budget = 0;
  int max_active = 0;
  Clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv;       // work for the threads
  std::condition_variable done_cv;  // a request finished
  bool stop = false;
  uint64_t next = 1;
  size_t in_use = 0;
  std::deque<std::shared_ptr<Job>> queued, to_prepare, prepared;
  std::vector<std::shared_ptr<Job>> active;
  std::map<uint64_t, std::shared_ptr<Job>> jobs;
  std::thread worker, preparer;
  int preparing = 0;  // requests inside setup_job
  uint64_t completed = 0;
};

namespace {

int setup_job(mpsl_server *s, Job &j) {
  const mpsl_request &r = j.req;
  if (hipSetDevice(s->device) != hipSuccess) return MPSL_EHIP;
  int rc = mpsl_create(&j.ctx, s->device, 0);  // admission already charged the estimate
  if (rc) return rc;
  if (hipStreamCreateWithFlags(&j.stream, hipStreamNonBlocking) != hipSuccess) return MPSL_EHIP;
  if ((rc = mpsl_set_stream(j.ctx, j.stream)) || (rc = mpsl_set_layers(j.ctx, r.k1, r.k2, r.k3, r.d))) return rc;
  if (r.particle == MPSL_PARTICLE_DISK)
    rc = mpsl_set_particle_disk(j.ctx, r.shape[0], r.kp, r.p);
  else if (r.particle == MPSL_PARTICLE_STAR)
    rc = mpsl_set_particle_star(j.ctx, r.shape[0], r.shape[1], static_cast<int>(r.shape[2]), r.kp, r.p, r.n_bdry);
  else
    rc = mpsl_set_scattering_matrix(j.ctx, r.p, r.r_enclose, j.S.data());
  if (rc) return rc;
  if ((rc = mpsl_set_sommerfeld_method(j.ctx, r.sommerfeld)) ||
      (rc = mpsl_set_geometry(j.ctx, r.n, j.xy.data(), j.rot.empty() ? nullptr : j.rot.data())))
    return rc;
  rc = r.contour == MPSL_CONTOUR_SPAN ? mpsl_set_contour_span(j.ctx, r.b, r.t_max, r.h_max)
                                      : mpsl_set_contour(j.ctx, r.n_nodes, r.b, r.t_max);
  if (rc) return rc;
  if (r.precond == MPSL_PRECOND_CLUSTER && (rc = mpsl_set_preconditioner(j.ctx, r.precond, r.cluster_size)))
    return rc;
  if ((rc = mpsl::build_tables(j.ctx))) return rc;
  const int64_t len = r.n * static_cast<int64_t>(2 * r.p + 1);
  if ((rc = mpsl::dev_alloc(j.ctx, j.ctx->ybuf, len * sizeof(double2)))) return rc;
  if ((rc = mpsl::rhs_device(j.ctx, r.src, j.ctx->ybuf.p))) return rc;
  j.sm.reset(new mpsl::SolveSM());
  mpsl_opts o = r.opts;
  if (!(o.tol > 0.0)) o.tol = 1e-10;
  if (o.maxiter <= 0) o.maxiter = 500;
  return j.sm->init(j.ctx, o, j.ctx->ybuf.p);
}

void release_device(mpsl_server *s, Job &j) {
  (void)hipSetDevice(s->device);
  if (j.ctx) mpsl_destroy(j.ctx);
  j.ctx = nullptr;
  j.sm.reset();
  if (j.stream) (void)hipStreamDestroy(j.stream);
  j.stream = nullptr;
}

// Called with the lock held: admit queued requests in arrival order.
void admit_locked(mpsl_server *s) {
  while (!s->queued.empty()) {
    auto &j = s->queued.front();
    const int running =
        static_cast<int>(s->active.size() + s->to_prepare.size() + s->prepared.size()) + s->preparing;
    if (running >= s->max_active || s->in_use + j->bytes > s->budget) break;
    s->in_use += j->bytes;
    j->t_admit = now_s(s->t0);
    j->state = Job::kPreparing;
    s->to_prepare.push_back(j);
    s->queued.pop_front();
  }
}

void finish(mpsl_server *s, const std::shared_ptr<Job> &j, int status) {
  // result copy (the solve's stream is idle after complete())
  if (status == MPSL_OK || status == MPSL_ENOCONV) {
    const int64_t len = j->req.n * static_cast<int64_t>(2 * j->req.p + 1);
    j->beta.resize(len);
    if (hipMemcpyAsync(j->beta.data(), j->sm->x(), len * sizeof(double2), hipMemcpyDeviceToHost, j->stream) !=
            hipSuccess ||
        hipStreamSynchronize(j->stream) != hipSuccess)
      status = MPSL_EHIP;
    j->iterations = j->sm->iterations();
    j->fp64_mv = j->sm->fp64_matvecs();
    j->refin = j->sm->refinements();
    j->rel_res = j->sm->rel_residual();
  }
  if (status != MPSL_OK && j->ctx && j->err.empty()) j->err = j->ctx->err;
  release_device(s, *j);
  std::lock_guard<std::mutex> lk(s->mu);
  j->status = status;
  j->t_finish = now_s(s->t0);
  j->state = Job::kDone;
  s->in_use -= j->bytes;
  ++s->completed;
  // the finished request no longer holds a slot: drop it from the active
  // list before admitting (the worker republishes the list only later, and
  // a request submitted in between would otherwise wait for an admission
  // that no later event triggers)
  s->active.erase(std::remove(s->active.begin(), s->active.end(), j), s->active.end());
  admit_locked(s);
  s->done_cv.notify_all();
  s->cv.notify_all();
}

void preparer_loop(mpsl_server *s) {
  for (;;) {
    std::shared_ptr<Job> j;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv.wait(lk, [&] { return s->stop || !s->to_prepare.empty(); });
      if (s->to_prepare.empty()) {
        if (s->stop) return;
        continue;
      }
      j = s->to_prepare.front();
      s->to_prepare.pop_front();
      ++s->preparing;
    }
    const int rc = setup_job(s, *j);
    if (rc) {
      if (j->ctx) j->err = j->ctx->err;
      finish(s, j, rc);
      std::lock_guard<std::mutex> lk(s->mu);
      --s->preparing;
      s->cv.notify_all();
      continue;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    j->t_start = now_s(s->t0);
    s->prepared.push_back(j);
    --s->preparing;
    s->cv.notify_all();
  }
}

void worker_loop(mpsl_server *s) {
  std::vector<std::shared_ptr<Job>> act;
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(s->mu);
      const auto drained = [&] {
        return s->stop && s->queued.empty() && s->to_prepare.empty() && s->prepared.empty() && s->preparing == 0;
      };
      s->cv.wait(lk, [&] { return !s->prepared.empty() || !act.empty() || drained(); });
      while (!s->prepared.empty()) {
        auto j = s->prepared.front();
        s->prepared.pop_front();
        j->state = Job::kActive;
        act.push_back(j);
      }
      s->active = act;
      if (act.empty() && drained()) return;
    }
    // one tick: launch a step of every active request, then complete them
    std::vector<int> rc(act.size(), MPSL_OK);
    for (size_t i = 0; i < act.size(); ++i) {
      (void)hipSetDevice(s->device);
      rc[i] = act[i]->sm->launch();
    }
    for (size_t i = 0; i < act.size(); ++i)
      if (!rc[i]) rc[i] = act[i]->sm->complete();
    std::vector<std::shared_ptr<Job>> keep;
    for (size_t i = 0; i < act.size(); ++i) {
      const int st = act[i]->sm->status();
      if (rc[i]) {
        finish(s, act[i], rc[i]);
      } else if (st != mpsl::SolveSM::kRunning) {
        finish(s, act[i], st == mpsl::SolveSM::kConverged ? MPSL_OK : MPSL_ENOCONV);
      } else {
        keep.push_back(act[i]);
      }
    }
    act.swap(keep);
    std::lock_guard<std::mutex> lk(s->mu);
    s->active = act;
    admit_locked(s);
    s->cv.notify_all();
  }
}

}  // namespace

extern "C" {

int mpsl_server_create(mpsl_server **out, int device, size_t hbm_budget, int max_active) {
  if (!out || max_active <= 0 || hbm_budget == 0) return MPSL_EINVAL;
  *out = nullptr;
  int cnt = 0;
  if (hipGetDeviceCount(&cnt) != hipSuccess || device < 0 || device >= cnt) {
    (void)hipGetLastError();
    return MPSL_EHIP;
  }
  mpsl_server *s = new mpsl_server();
  s->device = device;
  s->budget = hbm_budget;
  s->max_active = max_active;
  s->t0 = Clock::now();
  s->worker = std::thread(worker_loop, s);
  s->preparer = std::thread(preparer_loop, s);
  *out = s;
  return MPSL_OK;
}

int mpsl_server_submit(mpsl_server *s, const mpsl_request *r, uint64_t *ticket) {
  if (!s || !r || !ticket || !r->xy || r->n <= 0 || r->p < mpsl::kMinP || r->p > mpsl::kMaxP)
    return MPSL_EINVAL;
  if ((r->contour != MPSL_CONTOUR_COUNT && r->contour != MPSL_CONTOUR_SPAN) ||
      (r->contour == MPSL_CONTOUR_COUNT && r->n_nodes <= 0) || (r->contour == MPSL_CONTOUR_SPAN && !(r->h_max > 0.0)) ||
      (r->sommerfeld != MPSL_SOMM_DIRECT && r->sommerfeld != MPSL_SOMM_INTERP) ||
      (r->precond != MPSL_PRECOND_NONE && r->precond != MPSL_PRECOND_CLUSTER) || r->cluster_size < 0)
    return MPSL_EINVAL;
  if (r->particle == MPSL_PARTICLE_MATRIX && !r->S) return MPSL_EINVAL;
  auto j = std::make_shared<Job>();
  j->req = *r;
  j->xy.assign(r->xy, r->xy + 2 * r->n);
  if (r->rot) j->rot.assign(r->rot, r->rot + r->n);
  if (r->particle == MPSL_PARTICLE_MATRIX) {
    const size_t PP = static_cast<size_t>(2 * r->p + 1) * (2 * r->p + 1);
    j->S.assign(r->S, r->S + PP);
  }
  j->req.xy = nullptr;
  j->req.rot = nullptr;
  j->req.S = nullptr;
  j->bytes = estimate_bytes(*r);
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return MPSL_ESTATE;
  if (j->bytes > s->budget) return MPSL_ENOMEM;
  j->ticket = s->next++;
  j->t_submit = now_s(s->t0);
  s->jobs[j->ticket] = j;
  s->queued.push_back(j);
  admit_locked(s);
  s->cv.notify_all();
  *ticket = j->ticket;
  return MPSL_OK;
}

static void fill_result(const Job &j, mpsl_result *res) {
  res->status = j.status;
  res->error = j.err.c_str();
  res->n = j.req.n;
  res->p = j.req.p;
  res->beta = j.beta.empty() ? nullptr : j.beta.data();
  res->iterations = j.iterations;
  res->fp64_matvecs = j.fp64_mv;
  res->refinements = j.refin;
  res->rel_residual = j.rel_res;
  res->t_submit = j.t_submit;
  res->t_admit = j.t_admit;
  res->t_start = j.t_start;
  res->t_finish = j.t_finish;
  res->hbm_bytes = j.bytes;
}

int mpsl_server_poll(mpsl_server *s, uint64_t ticket, mpsl_result *res) {
  if (!s || !res) return MPSL_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return MPSL_EINVAL;
  if (it->second->state != Job::kDone) return MPSL_PENDING;
  fill_result(*it->second, res);
  return MPSL_OK;
}

int mpsl_server_wait(mpsl_server *s, uint64_t ticket, double timeout_s, mpsl_result *res) {
  if (!s || !res) return MPSL_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return MPSL_EINVAL;
  auto j = it->second;
  const auto pred = [&] { return j->state == Job::kDone; };
  if (timeout_s < 0)
    s->done_cv.wait(lk, pred);
  else if (!s->done_cv.wait_for(lk, std::chrono::duration<double>(timeout_s), pred))
    return MPSL_PENDING;
  fill_result(*j, res);
  return MPSL_OK;
}

int mpsl_server_release(mpsl_server *s, uint64_t ticket) {
  if (!s) return MPSL_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end() || it->second->state != Job::kDone) return MPSL_EINVAL;
  s->jobs.erase(it);
  return MPSL_OK;
}

int mpsl_server_stats(mpsl_server *s, int *queued, int *active, uint64_t *completed, size_t *bytes_in_use) {
  if (!s) return MPSL_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  if (queued) *queued = static_cast<int>(s->queued.size());
  if (active)
    *active = static_cast<int>(s->active.size() + s->to_prepare.size() + s->prepared.size()) + s->preparing;
  if (completed) *completed = s->completed;
  if (bytes_in_use) *bytes_in_use = s->in_use;
  return MPSL_OK;
}

void mpsl_server_destroy(mpsl_server *s) {
  if (!s) return;
  {
    // requests not yet admitted are cancelled; admitted ones run to the end
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    for (auto &j : s->queued) {
      j->state = Job::kDone;
      j->status = MPSL_ESTATE;
      j->t_finish = now_s(s->t0);
    }
    s->queued.clear();
    s->cv.notify_all();
    s->done_cv.notify_all();
  }
  if (s->preparer.joinable()) s->preparer.join();
  if (s->worker.joinable()) s->worker.join();
  delete s;
}

}  // extern "C"
