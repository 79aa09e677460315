// Request server: continuous admission of independent solves onto one GPU.
//
// Each request runs the whole path (problem set-up, preconditioner of Sec. 2,
// data, GMRES of Sec. 3) through the library's own entry points, on the
// context and stream of one worker thread.  Workers take the oldest queued
// request as soon as they are free and its estimated device-memory footprint
// fits next to the requests already running; the kernels of the running
// requests overlap on the device because every worker has its own stream.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "dp_internal.hpp"

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  int64_t id = 0;
  int64_t n = 0, nrhs = 0;
  int kind = 0;
  double omega = 0, eta = 0;
  std::vector<double> xy, nrm, w, kappa, angles, f;
  dp_solve_opts opts{};
  int64_t mem = 0;
  // result
  bool done = false;
  int rc = DP_OK;
  std::string err;
  std::vector<double> q;
  dp_solve_info info{};
  dp_request_times times{};
};

int pad_cols(int64_t nrhs) {
  int r = 1;
  while (r < nrhs && r < 64) r *= 2;
  return r;
}

// Device bytes a request holds while it runs (the library's allocations for
// this shape, rounded up): geometry and tables, the near-field list, sweep
// operands and partial sums, GMRES bases (V, Z and work vectors), the
// mixed-precision refinement vectors, the preconditioner and data/solution.
int64_t estimate_bytes(const Request& r) {
  const double n = (double)r.n, nrhs = (double)r.nrhs;
  const int nd = r.kind == DP_HARD ? 2 : 1;
  int nrp = pad_cols(r.nrhs);
  const bool mixed = r.opts.precision == DP_PREC_MIXED;
  if (mixed && nrp > 4 && nrp < 32) nrp = 32;
  const double m = r.opts.restart > 0 ? r.opts.restart : 80;
  const double cplx = 16.0;
  double b = 0;
  b += n * (64 + 8 + 16);                                  // source records, Kress table, twiddles
  if ((r.kind == DP_HARD || r.kappa.empty()) && (r.n & (r.n - 1))) {
    double M = 1;
    while (M < 2 * n - 1) M *= 2;
    b += cplx * M * (2.0 + std::max(nrhs, 2.0)) + cplx * n;  // Bluestein twiddles, chirp spectrum, workspace
  }
  double L = 0;
  for (double wi : r.w) L += wi;
  const double near_per_row = 2.0 * 25.0 / (r.omega * (L / n)) + 2.0;
  b += 4.0 * n * std::min(near_per_row, n) + 4.0 * n;     // near-field CSR
  b += cplx * nd * nrp * n;                                // near-field sums
  b += cplx * nd * nrp * n;                                // packed densities
  b += cplx * nd * nrp * std::max(n, 131072.0) * 2.0;      // chunk partial sums (<= ~2048 blocks)
  b += 3.0 * cplx * n * nrhs;                              // operator work vectors
  b += cplx * n * nrhs * (2.0 * m + 4.0);                  // V, Z, W, R
  if (mixed) b += 2.0 * cplx * n * nrhs;                   // residual and correction
  b += 2.0 * cplx * n * nrhs;                              // data and solution
  if (r.opts.use_precond) b += 256.0e6 + 6.0 * cplx * n * nrhs + 64.0 * n;  // size classes, factors, vectors
  b += 64.0e6;                                             // small buffers and rounding
  return (int64_t)b;
}

}  // namespace

struct dp_server {
  int device = 0;
  int slots = 0;
  int64_t budget = 0;
  Clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<Request>> queue;
  std::map<int64_t, std::shared_ptr<Request>> all;
  int64_t next_id = 1;
  int64_t used = 0, peak = 0;
  int64_t submitted = 0, completed = 0, failed = 0, running = 0;
  bool stop = false;
  std::vector<std::thread> workers;

  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

namespace {

// One request on the worker's context (every call below is synchronous).
void run_request(dp_ctx* ctx, Request& r) {
  dp_problem* p = nullptr;
  // data and solution: stream-ordered device buffers, released without a
  // wait for the device (other slots' kernels keep running)
  dp::AllocStream alloc_guard(ctx->stream);
  dp::DevBuf fdb, qdb;
  void* fd = nullptr;
  void* qd = nullptr;
  const size_t bytes = (size_t)r.n * r.nrhs * 16;
  auto fail = [&](int rc) {
    r.rc = rc;
    r.err = dp_last_error();
  };
  int rc = dp_problem_create(ctx, r.n, r.xy.data(), r.nrm.data(), r.w.data(), r.kappa.empty() ? nullptr : r.kappa.data(), r.omega, r.eta,
                             r.kind, &p);
  if (rc != DP_OK) {
    fail(rc);
    return;
  }
  hipStream_t st = ctx->stream;
  if (r.opts.use_precond) rc = dp_precond_build(p, nullptr);
  if (rc == DP_OK && (fdb.reserve(bytes) != DP_OK || qdb.reserve(bytes) != DP_OK)) {
    dp::set_error("request %lld: device allocation of %zu bytes failed", (long long)r.id, 2 * bytes);
    rc = DP_ENOMEM;
  }
  fd = fdb.p;
  qd = qdb.p;
  if (rc == DP_OK) {
    if (!r.angles.empty()) {
      rc = dp_rhs_plane_wave(p, r.nrhs, r.angles.data(), static_cast<double*>(fd));
    } else if (hipMemcpyAsync(fd, r.f.data(), bytes, hipMemcpyHostToDevice, st) != hipSuccess ||
               hipStreamSynchronize(st) != hipSuccess) {
      dp::set_error("request %lld: data upload failed", (long long)r.id);
      rc = DP_EDEVICE;
    }
  }
  if (rc == DP_OK) {
    rc = dp_solve(p, r.nrhs, static_cast<const double*>(fd), static_cast<double*>(qd), &r.opts, &r.info, nullptr,
                  nullptr);
    if (rc >= 0) {
      r.q.resize((size_t)r.n * r.nrhs * 2);
      if (hipMemcpyAsync(r.q.data(), qd, bytes, hipMemcpyDeviceToHost, st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess) {
        dp::set_error("request %lld: result download failed", (long long)r.id);
        rc = DP_EDEVICE;
      }
    }
  }
  if (rc < 0) fail(rc);
  else r.rc = rc;
  fdb.release();
  qdb.release();
  dp_problem_destroy(p);
}

void worker_main(dp_server* s, int slot) {
  (void)hipSetDevice(s->device);
  dp_ctx* ctx = nullptr;
  const int crc = dp_ctx_create(s->device, nullptr, &ctx);
  // the admission budget counts every request's blocks: nothing stays parked
  // with the slot's context between requests
  if (crc == DP_OK) ctx->park_cap = 0;
  const std::string cerr = crc == DP_OK ? "" : dp_last_error();
  for (;;) {
    std::shared_ptr<Request> r;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_work.wait(lk, [&] {
        if (s->queue.empty()) return s->stop;
        return s->used + s->queue.front()->mem <= s->budget;
      });
      if (s->queue.empty()) break;  // stop requested and nothing left
      r = s->queue.front();
      s->queue.pop_front();
      s->used += r->mem;
      s->peak = std::max(s->peak, s->used);
      ++s->running;
      r->times.t_admit = s->now();
      r->times.slot = slot;
    }
    if (crc != DP_OK) {
      r->rc = crc;
      r->err = cerr;
    } else {
      run_request(ctx, *r);
    }
    {
      std::lock_guard<std::mutex> lk(s->mu);
      r->times.t_done = s->now();
      r->done = true;
      s->used -= r->mem;
      --s->running;
      ++s->completed;
      if (r->rc < 0) ++s->failed;
    }
    s->cv_done.notify_all();
    s->cv_work.notify_all();
  }
  if (ctx) dp_ctx_destroy(ctx);
}

}  // namespace

extern "C" {

int dp_server_create(int device, const dp_server_opts* opts, dp_server** out) {
  if (!out) {
    dp::set_error("dp_server_create: out is NULL");
    return DP_EINVAL;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    dp::set_error("dp_server_create: device %d out of range", device);
    return DP_EINVAL;
  }
  const int slots = opts && opts->slots ? opts->slots : 4;
  if (slots < 1 || slots > 64) {
    dp::set_error("dp_server_create: slots = %d must be in 1..64", slots);
    return DP_EINVAL;
  }
  int64_t budget = opts ? opts->mem_budget : 0;
  if (budget < 0) {
    dp::set_error("dp_server_create: negative memory budget");
    return DP_EINVAL;
  }
  if (budget == 0) {
    size_t fr = 0, tot = 0;
    if (hipSetDevice(device) != hipSuccess || hipMemGetInfo(&fr, &tot) != hipSuccess) {
      dp::set_error("dp_server_create: hipMemGetInfo failed");
      return DP_EDEVICE;
    }
    budget = (int64_t)(0.8 * (double)fr);
  }
  dp_server* s = new dp_server();
  s->device = device;
  s->slots = slots;
  s->budget = budget;
  s->t0 = Clock::now();
  for (int k = 0; k < slots; ++k) s->workers.emplace_back(worker_main, s, k);
  *out = s;
  return DP_OK;
}

int dp_server_submit(dp_server* s, const dp_request* rq, int64_t* id) {
  if (!s || !rq || !id) {
    dp::set_error("dp_server_submit: NULL argument");
    return DP_EINVAL;
  }
  const int64_t n = rq->n;
  // the limits of dp_problem_create (spectral derivative: at most 2^24
  // points, 2^23 unless a power of two)
  const bool fft = rq->kind == DP_HARD || !rq->kappa;
  const bool pow2 = (n & (n - 1)) == 0;
  if (!rq->xy || !rq->nrm || !rq->w || n < 16 || n % 2 || n > (1LL << 26) ||
      (fft && n > (pow2 ? (1LL << 24) : (1LL << 23))) || rq->nrhs < 1 || rq->nrhs > (1LL << 20) ||
      (rq->kind != DP_SOFT && rq->kind != DP_HARD) || (!rq->angles && !rq->f) || !(rq->omega > 0) ||
      !(rq->eta > 0)) {
    dp::set_error("dp_server_submit: invalid request (n = %lld, nrhs = %lld, kind = %d)", (long long)n,
                  (long long)rq->nrhs, rq->kind);
    return DP_EINVAL;
  }
  auto r = std::make_shared<Request>();
  r->n = n;
  r->nrhs = rq->nrhs;
  r->kind = rq->kind;
  r->omega = rq->omega;
  r->eta = rq->eta;
  r->xy.assign(rq->xy, rq->xy + 2 * n);
  r->nrm.assign(rq->nrm, rq->nrm + 2 * n);
  r->w.assign(rq->w, rq->w + n);
  if (rq->kappa) r->kappa.assign(rq->kappa, rq->kappa + n);  // empty: computed from the nodes
  if (rq->angles) r->angles.assign(rq->angles, rq->angles + rq->nrhs);
  else r->f.assign(rq->f, rq->f + 2 * n * rq->nrhs);
  r->opts = rq->solve;
  if (r->opts.tol <= 0) r->opts.tol = 1e-8;
  if (r->opts.restart <= 0) r->opts.restart = 80;
  if (r->opts.max_iters <= 0) r->opts.max_iters = 2000;
  if (r->opts.inner_tol <= 0) r->opts.inner_tol = dp::default_inner_tol(r->opts.tol);
  r->mem = estimate_bytes(*r);
  std::lock_guard<std::mutex> lk(s->mu);
  if (r->mem > s->budget) {
    dp::set_error("dp_server_submit: estimated footprint %lld bytes exceeds the budget %lld", (long long)r->mem,
                  (long long)s->budget);
    return DP_ENOMEM;
  }
  if (s->stop) {
    dp::set_error("dp_server_submit: server is shutting down");
    return DP_ESTATE;
  }
  r->id = s->next_id++;
  r->times.t_submit = s->now();
  r->times.mem_estimate = r->mem;
  r->times.slot = -1;
  s->all[r->id] = r;
  s->queue.push_back(r);
  ++s->submitted;
  *id = r->id;
  s->cv_work.notify_one();
  return DP_OK;
}

int dp_server_wait(dp_server* s, int64_t id, double* q, dp_solve_info* info, dp_request_times* times) {
  if (!s) {
    dp::set_error("dp_server_wait: NULL server");
    return DP_EINVAL;
  }
  std::shared_ptr<Request> r;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->all.find(id);
    if (it == s->all.end()) {
      dp::set_error("dp_server_wait: unknown request id %lld", (long long)id);
      return DP_EINVAL;
    }
    r = it->second;
    s->cv_done.wait(lk, [&] { return r->done; });
    s->all.erase(id);
  }
  if (q && !r->q.empty()) std::memcpy(q, r->q.data(), r->q.size() * sizeof(double));
  if (info) *info = r->info;
  if (times) *times = r->times;
  if (r->rc < 0) dp::set_error("%s", r->err.c_str());
  return r->rc;
}

int dp_server_get_stats(dp_server* s, dp_server_stats* st) {
  if (!s || !st) {
    dp::set_error("dp_server_get_stats: NULL argument");
    return DP_EINVAL;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  st->submitted = s->submitted;
  st->completed = s->completed;
  st->failed = s->failed;
  st->running = s->running;
  st->queued = (int64_t)s->queue.size();
  st->mem_in_use = s->used;
  st->mem_budget = s->budget;
  st->mem_peak = s->peak;
  return DP_OK;
}

void dp_server_destroy(dp_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  for (auto& t : s->workers) t.join();
  delete s;
}

}  // extern "C"
