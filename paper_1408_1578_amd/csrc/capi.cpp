// C-ABI of the dirprec library: argument validation, ownership and error
// reporting.  All numerical work is done by the HIP kernels in the other
// translation units.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "dense_lu.hpp"
#include "dp_internal.hpp"

namespace dp {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

static thread_local hipStream_t g_alloc_stream = nullptr;
static thread_local dp_ctx* g_alloc_ctx = nullptr;
static thread_local bool g_capturing = false;

std::shared_mutex& pool_capture_mutex() {
  static std::shared_mutex mu;
  return mu;
}

CaptureScope::CaptureScope() : lk(pool_capture_mutex()) { g_capturing = true; }
CaptureScope::~CaptureScope() { g_capturing = false; }

AllocStream::AllocStream(hipStream_t s, dp_ctx* ctx) : prev(g_alloc_stream), prev_ctx(g_alloc_ctx) {
  g_alloc_stream = s;
  g_alloc_ctx = ctx;
}
AllocStream::~AllocStream() {
  g_alloc_stream = prev;
  g_alloc_ctx = prev_ctx;
}

// The calling thread's context when it parks large blocks on its own stream.
static dp_ctx* park_ctx(size_t bytes) {
  dp_ctx* c = g_alloc_ctx;
  return c && bytes >= dp_ctx::kParkMin && c->park_cap > 0 && c->stream == g_alloc_stream ? c : nullptr;
}

// The default memory pool of each device keeps freed memory for reuse
// (release threshold: never), and reuses a block on another stream only once
// its release has completed, never by making that stream wait for the other.
static void configure_pool(int device) {
  static std::mutex mu;
  static std::vector<char> done;
  std::lock_guard<std::mutex> lk(mu);
  if ((int)done.size() <= device) done.resize(device + 1, 0);
  if (done[device]) return;
  done[device] = 1;
  hipMemPool_t pool = nullptr;
  if (hipDeviceGetDefaultMemPool(&pool, device) != hipSuccess || !pool) {
    (void)hipGetLastError();
    return;
  }
  uint64_t keep = ~0ull;
  int no = 0;
  (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
  (void)hipMemPoolSetAttribute(pool, hipMemPoolReuseAllowInternalDependencies, &no);
  (void)hipGetLastError();
}

int DevBuf::reserve(size_t want) {
  if (want <= bytes && p) return DP_OK;
  if (g_capturing) {
    set_error("device allocation of %zu bytes requested during graph capture", want);
    return DP_EDEVICE;
  }
  release();
  if (dp_ctx* c = park_ctx(want)) {  // the smallest parked block that fits, up to twice the size
    std::lock_guard<std::mutex> lk(c->park_mu);
    size_t best = c->parked.size();
    for (size_t i = 0; i < c->parked.size(); ++i)
      if (c->parked[i].second >= want && c->parked[i].second <= 2 * want &&
          (best == c->parked.size() || c->parked[i].second < c->parked[best].second))
        best = i;
    if (best < c->parked.size()) {
      p = c->parked[best].first;
      bytes = c->parked[best].second;
      s = c->stream;
      c->parked_bytes -= bytes;
      c->parked.erase(c->parked.begin() + (long)best);
      return DP_OK;
    }
  }
  if (want == 0) want = 8;
  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess) configure_pool(dev);
  std::shared_lock<std::shared_mutex> lk(pool_capture_mutex());
  const hipError_t e = hipMallocAsync(&p, want, g_alloc_stream);
  if (e != hipSuccess) {
    p = nullptr;
    bytes = 0;
    (void)hipGetLastError();
    size_t fr = 0, tot = 0;
    (void)hipMemGetInfo(&fr, &tot);
    (void)hipGetLastError();
    set_error("device allocation of %zu bytes failed (%s; %zu of %zu bytes free)", want, hipGetErrorString(e), fr,
              tot);
    return DP_ENOMEM;
  }
  s = g_alloc_stream;
  bytes = want;
  return DP_OK;
}

void DevBuf::release() {
  if (p) {
    dp_ctx* c = s == g_alloc_stream ? park_ctx(bytes) : nullptr;
    bool parked = false;
    if (c) {
      std::lock_guard<std::mutex> lk(c->park_mu);
      if (c->parked_bytes + bytes <= c->park_cap) {
        c->parked.push_back({p, bytes});
        c->parked_bytes += bytes;
        parked = true;
      }
    }
    if (!parked) {
      std::shared_lock<std::shared_mutex> lk(pool_capture_mutex());
      (void)hipFreeAsync(p, s);
    }
  }
  p = nullptr;
  bytes = 0;
  s = nullptr;
}

int pinned_borrow(dp_ctx* c, size_t bytes, void** out, size_t* got) {
  {
    std::lock_guard<std::mutex> lk(c->pin_mu);
    for (size_t i = 0; i < c->pin_free.size(); ++i) {
      if (c->pin_free[i].second >= bytes) {
        *out = c->pin_free[i].first;
        *got = c->pin_free[i].second;
        c->pin_free.erase(c->pin_free.begin() + (long)i);
        return DP_OK;
      }
    }
  }
  // grow in steps of 64 KiB so that later, slightly larger solves fit
  const size_t want = (bytes + 65535) / 65536 * 65536;
  void* h = nullptr;
  if (hipHostMalloc(&h, want, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    set_error("pinned host allocation of %zu bytes failed", want);
    return DP_ENOMEM;
  }
  *out = h;
  *got = want;
  return DP_OK;
}

void pinned_return(dp_ctx* c, void* p, size_t bytes) {
  std::lock_guard<std::mutex> lk(c->pin_mu);
  c->pin_free.emplace_back(p, bytes);
}

static bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

// A pointer documented as "device" must lie in device memory of the
// context's GPU, with `bytes` bytes inside one allocation; otherwise the call
// is refused before any kernel could touch it.
static int check_device_ptr(const dp_ctx* c, const void* ptr, size_t bytes, const char* fn, const char* name) {
  hipPointerAttribute_t a{};
  if (hipPointerGetAttributes(&a, ptr) != hipSuccess) {
    (void)hipGetLastError();
    set_error("%s: %s is not device memory of device %d", fn, name, c->device);
    return DP_EINVAL;
  }
  if ((a.type != hipMemoryTypeDevice && a.type != hipMemoryTypeManaged) || a.device != c->device) {
    set_error("%s: %s is not device memory of device %d (memory type %d, device %d)", fn, name, c->device,
              (int)a.type, a.device);
    return DP_EINVAL;
  }
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  if (hipMemGetAddressRange(&base, &size, const_cast<void*>(ptr)) == hipSuccess) {
    const char* b = static_cast<const char*>(base);
    const char* q = static_cast<const char*>(ptr);
    if (q + bytes > b + size) {
      set_error("%s: %s holds %zu bytes from its address, %zu needed", fn, name, (size_t)(b + size - q), bytes);
      return DP_EINVAL;
    }
  } else {
    (void)hipGetLastError();
  }
  return DP_OK;
}

static bool overlap(const void* a, const void* b, size_t bytes) {
  const char* x = static_cast<const char*>(a);
  const char* y = static_cast<const char*>(b);
  return x < y + bytes && y < x + bytes;
}

// Input and output of an n x nrhs complex operation: both device memory of
// the context's GPU, large enough, and disjoint.
static int check_io(const dp_problem* p, int64_t nrhs, const void* in, const void* out, const char* fn) {
  const size_t bytes = (size_t)p->n * (size_t)nrhs * 16;
  DP_TRY(check_device_ptr(p->ctx, in, bytes, fn, "input"));
  DP_TRY(check_device_ptr(p->ctx, out, bytes, fn, "output"));
  if (overlap(in, out, bytes)) {
    set_error("%s: input and output overlap", fn);
    return DP_EINVAL;
  }
  return DP_OK;
}

}  // namespace dp

using namespace dp;

#define DP_CHECK(cond, ...)        \
  do {                             \
    if (!(cond)) {                 \
      ::dp::set_error(__VA_ARGS__); \
      return DP_EINVAL;            \
    }                              \
  } while (0)

#define DP_SETDEV(ctx)                    \
  DP_HIP(hipSetDevice((ctx)->device)); \
  AllocStream alloc_stream_guard_((ctx)->stream, (ctx))

extern "C" {

const char* dp_last_error(void) { return g_err; }

int dp_ctx_create(int device, void* stream, dp_ctx** out) {
  DP_CHECK(out != nullptr, "dp_ctx_create: out is NULL");
  int ndev = 0;
  DP_HIP(hipGetDeviceCount(&ndev));
  DP_CHECK(device >= 0 && device < ndev, "dp_ctx_create: device %d out of range (%d devices)", device, ndev);
  DP_HIP(hipSetDevice(device));
  dp_ctx* c = new dp_ctx();
  c->device = device;
  if (stream) {
    c->stream = static_cast<hipStream_t>(stream);
  } else {
    if (hipStreamCreate(&c->stream) != hipSuccess) {  // blocking: orders with the null stream
      delete c;
      set_error("hipStreamCreate failed");
      return DP_EDEVICE;
    }
    c->own_stream = true;
  }
  // the scratch array of dp_precond_apply_noalloc on this device
  const int src = scratch_init(device);
  if (src != DP_OK) {
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return src;
  }
  *out = c;
  return DP_OK;
}

void dp_ctx_destroy(dp_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  for (auto& b : c->parked) (void)hipFreeAsync(b.first, c->stream);
  c->parked.clear();
  (void)hipStreamSynchronize(c->stream);
  for (auto& b : c->pin_free) (void)hipHostFree(b.first);
  if (c->own_stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

int dp_problem_create(dp_ctx* ctx, int64_t n, const double* xy, const double* nrm, const double* w,
                      const double* kappa, double omega, double eta, int kind, dp_problem** out) {
  DP_CHECK(ctx && out && xy && nrm && w, "dp_problem_create: NULL argument");
  DP_CHECK(n >= 16 && n % 2 == 0 && n <= (1LL << 26), "dp_problem_create: n = %lld must be even, >= 16",
           (long long)n);
  DP_CHECK(kind == DP_SOFT || kind == DP_HARD, "dp_problem_create: kind %d", kind);
  // the spectral derivative (sound-hard, or curvature from the nodes) runs
  // FFTs of length n (a power of two) or >= 2n - 1 (Bluestein), at most 2^24
  const bool fft = kind == DP_HARD || !kappa;
  DP_CHECK(!fft || n <= (is_pow2(n) ? (1LL << 24) : (1LL << 23)),
           "dp_problem_create: n = %lld too large for the spectral derivative (sound-hard or kappa == NULL: "
           "at most 2^24, 2^23 unless a power of two)",
           (long long)n);
  DP_CHECK(std::isfinite(omega) && omega > 0, "dp_problem_create: omega must be > 0");
  DP_CHECK(std::isfinite(eta) && eta > 0, "dp_problem_create: eta must be > 0");
  const double w0 = w[0];
  bool equi = true;
  for (int64_t i = 0; i < n; ++i) {
    const double v[6] = {xy[2 * i], xy[2 * i + 1], nrm[2 * i], nrm[2 * i + 1], w[i], kappa ? kappa[i] : 0.0};
    for (double t : v) DP_CHECK(std::isfinite(t), "dp_problem_create: non-finite input at node %lld", (long long)i);
    DP_CHECK(w[i] > 0, "dp_problem_create: weight %lld is not positive", (long long)i);
    const double nn = std::hypot(nrm[2 * i], nrm[2 * i + 1]);
    DP_CHECK(std::fabs(nn - 1.0) <= 1e-10, "dp_problem_create: normal %lld has length %.17g", (long long)i, nn);
    if (std::fabs(w[i] - w0) > 1e-12 * w0) equi = false;
  }
  DP_SETDEV(ctx);
  dp_problem* p = new dp_problem();
  p->ctx = ctx;
  p->n = n;
  p->kind = kind;
  p->omega = omega;
  p->eta = eta;
  p->equispaced = equi;
  p->hx.resize(n);
  p->hy.resize(n);
  p->hnx.resize(n);
  p->hny.resize(n);
  p->hsp.resize(n);
  p->hkap.resize(n);
  std::vector<SrcRec> rec(n);
  double L = 0;
  for (int64_t i = 0; i < n; ++i) {
    p->hx[i] = xy[2 * i];
    p->hy[i] = xy[2 * i + 1];
    p->hnx[i] = nrm[2 * i];
    p->hny[i] = nrm[2 * i + 1];
    p->hsp[i] = w[i] * (double)n / (2.0 * kPi);
    p->spmax = std::max(p->spmax, p->hsp[i]);
    p->hkap[i] = kappa ? kappa[i] : 0.0;
    L += w[i];
    rec[i] = {p->hx[i],        p->hy[i],        p->hnx[i],
              p->hny[i],       p->hsp[i],       p->hkap[i],
              (float)p->hnx[i], (float)p->hny[i], (float)(0.5 * kPi / (double)n * p->hsp[i]),
              (float)(p->hsp[i] / (4.0 * kPi))};
  }
  p->L = L;
  int rc = p->src.reserve(n * sizeof(SrcRec));
  if (rc == DP_OK && hipMemcpyAsync(p->src.p, rec.data(), n * sizeof(SrcRec), hipMemcpyHostToDevice,
                                    ctx->stream) != hipSuccess) {
    set_error("geometry upload failed");
    rc = DP_EDEVICE;
  }
  if (rc == DP_OK) rc = build_tables(p);
  if (rc == DP_OK && fft && !is_pow2(n)) rc = bluestein_init(p);
  if (rc == DP_OK && !kappa) rc = curvature_spectral(p, p->hkap.data());
  if (rc == DP_OK) rc = build_diag(p);
  if (rc == DP_OK) rc = near_build(p);
  if (rc != DP_OK) {
    dp_problem_destroy(p);
    return rc;
  }
  *out = p;
  return DP_OK;
}

void dp_problem_destroy(dp_problem* p) {
  if (!p) return;
  (void)hipSetDevice(p->ctx->device);
  AllocStream alloc_stream_guard_(p->ctx->stream, p->ctx);
  // the releases below are ordered on the stream after the problem's work:
  // no wait for the device here
  if (p->pc) precond_destroy(p->pc);
  p->clock.destroy();
  p->clock32.destroy();
  p->src.release();
  p->C.release();
  p->twiddle.release();
  p->blu_tw.release();
  p->blu_chirp.release();
  p->blu_B.release();
  p->blu_ws.release();
  p->dens.release();
  p->partial.release();
  p->dens16.release();
  p->C32.release();
  p->diag.release();
  p->srcblk.release();
  p->sc16.release();
  p->near_ptr.release();
  p->near_col.release();
  p->near_out.release();
  for (auto& b : p->near_kv) b.release();
  for (auto& b : p->near_bv) b.release();
  p->tmp1.release();
  p->tmp2.release();
  p->tmp3.release();
  krylov_graphs_destroy(p);
  for (auto& b : p->krylov_ws) b.release();
  for (auto& b : p->refine_ws) b.release();
  delete p;
}

int dp_problem_kappa(const dp_problem* p, double* kappa) {
  DP_CHECK(p && kappa, "dp_problem_kappa: NULL argument");
  std::copy(p->hkap.begin(), p->hkap.end(), kappa);
  return DP_OK;
}

int dp_rhs_plane_wave(dp_problem* p, int64_t nrhs, const double* angles, double* f) {
  DP_CHECK(p && angles && f && nrhs >= 1, "dp_rhs_plane_wave: bad argument");
  DP_SETDEV(p->ctx);
  DP_TRY(check_device_ptr(p->ctx, f, (size_t)p->n * nrhs * 16, "dp_rhs_plane_wave", "f"));
  DevBuf a;
  DP_TRY(a.reserve(nrhs * sizeof(double)));
  DP_HIP(hipMemcpyAsync(a.p, angles, nrhs * sizeof(double), hipMemcpyHostToDevice, p->ctx->stream));
  int rc = rhs_plane_wave(p, (int)nrhs, a.as<double>(), reinterpret_cast<cplx*>(f));
  DP_HIP(hipStreamSynchronize(p->ctx->stream));
  a.release();
  return rc;
}

int dp_matvec(dp_problem* p, int64_t nrhs, const double* q, double* y) {
  DP_CHECK(p && q && y && nrhs >= 1, "dp_matvec: bad argument");
  DP_SETDEV(p->ctx);
  DP_TRY(check_io(p, nrhs, q, y, "dp_matvec"));
  DP_TRY(matvec(p, (int)nrhs, reinterpret_cast<const cplx*>(q), reinterpret_cast<cplx*>(y)));
  DP_HIP(hipStreamSynchronize(p->ctx->stream));
  p->clock.collect();
  return DP_OK;
}

int dp_matvec_mixed(dp_problem* p, int64_t nrhs, const double* q, double* y) {
  DP_CHECK(p && q && y && nrhs >= 1, "dp_matvec_mixed: bad argument");
  DP_SETDEV(p->ctx);
  DP_TRY(check_io(p, nrhs, q, y, "dp_matvec_mixed"));
  DP_TRY(matvec(p, (int)nrhs, reinterpret_cast<const cplx*>(q), reinterpret_cast<cplx*>(y), 1));
  DP_HIP(hipStreamSynchronize(p->ctx->stream));
  p->clock.collect();
  p->clock32.collect();
  return DP_OK;
}

int dp_layer_apply(dp_problem* p, int op, int64_t nrhs, const double* q, double* y) {
  DP_CHECK(p && q && y && nrhs >= 1, "dp_layer_apply: bad argument");
  DP_CHECK(op == DP_OP_S || op == DP_OP_D || op == DP_OP_DP || op == DP_OP_DS, "dp_layer_apply: op %d", op);
  DP_CHECK(op != DP_OP_DS || is_pow2(p->n) || p->blu_M > 0,
           "dp_layer_apply: D_s of a sound-soft problem with given curvatures needs a power-of-two n");
  DP_SETDEV(p->ctx);
  DP_TRY(check_io(p, nrhs, q, y, "dp_layer_apply"));
  if (op == DP_OP_DS) {
    DP_TRY(spectral_derivative(p, (int)nrhs, reinterpret_cast<const cplx*>(q), reinterpret_cast<cplx*>(y)));
  } else {
    DP_TRY(sweep_apply(p, op, (int)nrhs, reinterpret_cast<const cplx*>(q), reinterpret_cast<cplx*>(y)));
  }
  DP_HIP(hipStreamSynchronize(p->ctx->stream));
  p->clock.collect();
  return DP_OK;
}

int dp_autotune(dp_problem* p, int64_t nrhs, int precision, dp_tune_info* info) {
  DP_CHECK(p != nullptr && nrhs >= 1, "dp_autotune: bad argument");
  DP_CHECK(precision == DP_PREC_FP64 || precision == DP_PREC_MIXED, "dp_autotune: precision %d", precision);
  DP_SETDEV(p->ctx);
  return autotune(p, (int)std::min<int64_t>(nrhs, 64), precision, info);
}

int dp_precond_build(dp_problem* p, const dp_precond_opts* opts) {
  DP_CHECK(p != nullptr, "dp_precond_build: NULL problem");
  DP_CHECK(p->equispaced, "dp_precond_build: nodes must be arclength-equispaced (equal weights)");
  dp_precond_opts o = {4.0, 8, 10, 3.0, 0, 1, 0};
  if (opts) o = *opts;
  DP_CHECK(o.m_ell > 0 && o.min_pts >= 2 && o.m_c >= 2 && o.m_c <= 32 && o.t_keep >= 0 && o.w_solver >= 0 &&
               o.w_solver <= 2 && (o.graphs == 0 || o.graphs == 1) && o.gj_steps >= 0,
           "dp_precond_build: bad options");
  DP_SETDEV(p->ctx);
  return precond_build(p, &o);
}

int dp_precond_apply(dp_problem* p, int64_t nrhs, const double* v, double* z) {
  DP_CHECK(p && v && z && nrhs >= 1, "dp_precond_apply: bad argument");
  if (!p->pc) {
    set_error("dp_precond_apply: call dp_precond_build first");
    return DP_ESTATE;
  }
  DP_SETDEV(p->ctx);
  DP_TRY(check_io(p, nrhs, v, z, "dp_precond_apply"));
  DP_TRY(precond_apply(p, (int)nrhs, reinterpret_cast<const cplx*>(v), reinterpret_cast<cplx*>(z)));
  DP_HIP(hipStreamSynchronize(p->ctx->stream));
  return DP_OK;
}

int dp_precond_apply_mixed(dp_problem* p, int64_t nrhs, const double* v, double* z) {
  DP_CHECK(p && v && z && nrhs >= 1, "dp_precond_apply_mixed: bad argument");
  if (!p->pc) {
    set_error("dp_precond_apply_mixed: call dp_precond_build first");
    return DP_ESTATE;
  }
  DP_SETDEV(p->ctx);
  DP_TRY(check_io(p, nrhs, v, z, "dp_precond_apply_mixed"));
  DP_TRY(precond_apply(p, (int)nrhs, reinterpret_cast<const cplx*>(v), reinterpret_cast<cplx*>(z), 1));
  DP_HIP(hipStreamSynchronize(p->ctx->stream));
  return DP_OK;
}

int dp_precond_apply_noalloc(dp_problem* p, int64_t nrhs, const double* v, double* z) {
  DP_CHECK(p && v && z && nrhs >= 1 && nrhs <= (1 << 20), "dp_precond_apply_noalloc: bad argument");
  if (!p->pc) {
    set_error("dp_precond_apply_noalloc: call dp_precond_build first");
    return DP_ESTATE;
  }
  DP_HIP(hipSetDevice(p->ctx->device));
  DP_TRY(check_io(p, nrhs, v, z, "dp_precond_apply_noalloc"));
  DP_TRY(precond_apply_noalloc(p, (int)nrhs, reinterpret_cast<const cplx*>(v), reinterpret_cast<cplx*>(z)));
  DP_HIP(hipStreamSynchronize(p->ctx->stream));
  return DP_OK;
}

int dp_precond_get_info(dp_problem* p, dp_precond_info* info) {
  DP_CHECK(p && info, "dp_precond_get_info: NULL argument");
  if (!p->pc) {
    set_error("dp_precond_get_info: no preconditioner");
    return DP_ESTATE;
  }
  return precond_info(p, info);
}

int dp_precond_export(dp_problem* p, int64_t* seg_off, int64_t* seg_len, int64_t* e_idx, double* e_val) {
  DP_CHECK(p != nullptr, "dp_precond_export: NULL problem");
  if (!p->pc) {
    set_error("dp_precond_export: no preconditioner");
    return DP_ESTATE;
  }
  return precond_export(p, seg_off, seg_len, e_idx, e_val);
}

int dp_solve(dp_problem* p, int64_t nrhs, const double* f, double* q, const dp_solve_opts* opts,
             dp_solve_info* info, int64_t* iters, double* relres) {
  DP_CHECK(p && f && q && nrhs >= 1, "dp_solve: bad argument");
  dp_solve_opts o = {1e-8, 80, 2000, 0, DP_PREC_FP64, 0.0, 0};
  if (opts) o = *opts;
  if (o.inner_tol <= 0) o.inner_tol = default_inner_tol(o.tol);
  DP_CHECK(o.tol > 0 && o.restart >= 1 && o.restart <= 1000 && o.max_iters >= 1, "dp_solve: bad options");
  DP_CHECK(o.precision == DP_PREC_FP64 || o.precision == DP_PREC_MIXED, "dp_solve: precision %d", o.precision);
  if (o.use_precond && !p->pc) {
    set_error("dp_solve: use_precond set but no preconditioner was built");
    return DP_ESTATE;
  }
  DP_SETDEV(p->ctx);
  DP_TRY(check_io(p, nrhs, f, q, "dp_solve"));
  return solve(p, (int)nrhs, reinterpret_cast<const cplx*>(f), reinterpret_cast<cplx*>(q), &o, info, iters,
               relres);
}

int dp_hankel_dev(dp_ctx* ctx, int64_t m, const double* z, double* out) {
  DP_CHECK(ctx && z && out && m >= 0, "dp_hankel_dev: bad argument");
  DP_SETDEV(ctx);
  if (m == 0) return DP_OK;
  DP_TRY(check_device_ptr(ctx, z, (size_t)m * 8, "dp_hankel_dev", "z"));
  DP_TRY(check_device_ptr(ctx, out, (size_t)m * 32, "dp_hankel_dev", "out"));
  DP_TRY(hankel_eval_dev(m, z, out, ctx->stream));
  DP_HIP(hipStreamSynchronize(ctx->stream));
  return DP_OK;
}

int dp_dense_lu_test(dp_ctx* ctx, int64_t n, const double* a, double* lu, int64_t* perm) {
  DP_CHECK(ctx && a && lu && perm && n >= 1 && n <= 8192, "dp_dense_lu_test: bad argument");
  DP_SETDEV(ctx);
  hipStream_t st = ctx->stream;
  const int nn = (int)n;
  std::vector<int> rows, cols;
  std::vector<cplx> vals;
  const cplx* ac = reinterpret_cast<const cplx*>(a);
  for (int c = 0; c < nn; ++c)
    for (int r = 0; r < nn; ++r) {
      const cplx v = ac[(size_t)c * nn + r];
      if (v.re != 0.0 || v.im != 0.0) {  // NaN entries are kept too
        rows.push_back(r);
        cols.push_back(c);
        vals.push_back(v);
      }
    }
  DenseLU d;
  int rc = d.assemble(st, nn, rows, cols, vals);
  if (rc == DP_OK) rc = d.factor(st);
  if (rc == DP_OK) {
    std::vector<int> pm(nn);
    if (hipMemcpyAsync(lu, d.a.p, (size_t)nn * nn * sizeof(cplx), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(pm.data(), d.perm.p, (size_t)nn * sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      set_error("dp_dense_lu_test: copy of the factors failed");
      rc = DP_EDEVICE;
    } else {
      for (int i = 0; i < nn; ++i) perm[i] = pm[i];
    }
  }
  (void)hipStreamSynchronize(st);
  d.release();
  return rc;
}

int dp_hankel_host(int64_t m, const double* z, double* out) {
  DP_CHECK(z && out && m >= 0, "dp_hankel_host: bad argument");
  for (int64_t k = 0; k < m; ++k) {
    DP_CHECK(z[k] > 0 && std::isfinite(z[k]), "dp_hankel_host: z must be finite and > 0");
    const H01 h = hankel01(z[k]);
    out[4 * k + 0] = h.h0.re;
    out[4 * k + 1] = h.h0.im;
    out[4 * k + 2] = h.h1.re;
    out[4 * k + 3] = h.h1.im;
  }
  return DP_OK;
}

}  // extern "C"
