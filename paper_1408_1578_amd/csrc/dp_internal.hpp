// Internal structures of the dirprec library (not part of the C-ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <shared_mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/dirprec.h"
#include "dp_math.hpp"

struct dp_ctx;

namespace dp {

void set_error(const char* fmt, ...);

#define DP_HIP(call)                                                            \
  do {                                                                          \
    hipError_t e_ = (call);                                                     \
    if (e_ != hipSuccess) {                                                     \
      ::dp::set_error("%s:%d %s: %s", __FILE__, __LINE__, #call,                \
                      hipGetErrorString(e_));                                   \
      return DP_EDEVICE;                                                        \
    }                                                                           \
  } while (0)

#define DP_TRY(call)            \
  do {                          \
    int r_ = (call);            \
    if (r_ < 0) return r_;      \
  } while (0)

// Device buffer that grows on demand, owned by the library.  Allocation and
// release are stream-ordered (hipMallocAsync / hipFreeAsync on the stream
// current in the calling thread, see AllocStream): releasing a buffer does
// not wait for the device, so one problem's set-up or teardown does not drain
// the kernels that other streams (other server slots) have queued.  The
// memory returns to the device's pool, which keeps it for later allocations.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  hipStream_t s = nullptr;  // stream of the allocation; the release is ordered on it
  int reserve(size_t want);
  void release();
  template <class T>
  T* as() const { return static_cast<T*>(p); }
};

// Stream-ordered allocation and graph capture exclude each other across
// threads: HIP refuses hipMallocAsync on any stream while another thread
// captures (even in thread-local capture mode), so DevBuf allocations and
// releases hold this lock shared and a capture holds it exclusively (begin
// to instantiate).  A capture itself never allocates.
std::shared_mutex& pool_capture_mutex();
// set while the calling thread captures a graph (DevBuf growth is refused)
struct CaptureScope {
  std::unique_lock<std::shared_mutex> lk;
  CaptureScope();
  ~CaptureScope();
};

// The stream on which DevBuf allocations of the calling thread are ordered,
// and the context whose block cache they use, for the lifetime of this
// object (each C-ABI entry sets its context's stream and the context).
struct AllocStream {
  hipStream_t prev;
  dp_ctx* prev_ctx;
  explicit AllocStream(hipStream_t s, dp_ctx* ctx = nullptr);
  ~AllocStream();
};

// One boundary node (64 bytes): position, outward normal, speed |x'(t)| and
// curvature in FP64, and for the single-precision sweep the FP32 normal,
// a quarter of the trapezoid weight, (2 pi/n) |x'(t)| / 4, and |x'(t)| / (4 pi)
// (unused by the current kernels).
struct SrcRec {
  double x, y, nx, ny, sp, kappa;
  float nxf, nyf, wf, spf;
};
static_assert(sizeof(SrcRec) == 64, "SrcRec is one 64-byte record");

enum SweepOp { OP_SOFT = 0, OP_HARD = 1, OP_S = 2, OP_D = 3, OP_DP = 4 };

struct SweepParams {
  const SrcRec* src;       // n records
  const double* C;         // n: Kress correction C_k (index (i - j) mod n)
  const float* C32;        // C_k / (pi dt) in FP32 (single-precision sweep)
  const cplx* dens;        // [j][nd][nrp] source densities (transposed layout)
  cplx* partial;           // [chunk][nd][nrp][n] partial sums
  const cplxf* dens32;     // FP32 copies (near field and the few-column FP32 sweep)
  cplxf* partial32;
  const uint4* dens16;     // split-FP16 density tiles of the many-column FP32 sweep
  const uint4* srcblk;     // per block of 32 sources: (x, y) FP64 pairs, then (nx, ny, w/4, 0) FP32
  const float* unscale16;  // [nd][nrp]: 1 / (kernel scale x density scale)
  float ksc[2];            // power-of-two scales of the FP32 kernel values, per density
  const int* guard;        // null, or guard_n flags: the launch does nothing when all are 0
  int guard_n;
  int n, nrp, nd, chunk_len, nchunks;
  double omega, eta, dt;   // dt = 2 pi / n
  double r2near;           // pairs with r^2 < r2near are left to the near-field pass
};

struct Precond;

// HIP-event timing of the pair-sweep kernel launches on one stream.
struct SweepClock {
  std::vector<hipEvent_t> ev;  // pairs (start, stop)
  size_t used = 0;             // events recorded since the last collect
  int64_t launches = 0;
  double seconds = 0.0;
  void start(hipStream_t s);
  void stop(hipStream_t s);
  void collect();  // after a stream synchronisation
  void reset() {
    collect();
    launches = 0;
    seconds = 0.0;
  }
  void destroy();
};

}  // namespace dp

struct dp_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  // pinned host staging buffers for the per-step Krylov readbacks, kept for
  // the context's lifetime and lent to one solve at a time
  std::mutex pin_mu;
  std::vector<std::pair<void*, size_t>> pin_free;
  // Device blocks of at least kParkMin bytes that the context's problems
  // release (Krylov bases, chunk partial sums) stay parked here, up to
  // park_cap bytes, for the next problem on the context (all of whose work is
  // ordered on `stream`).  Releasing such a block through the memory pool
  // took up to 8 ms of host time per problem.  park_cap = 0: no parking.
  static constexpr size_t kParkMin = (size_t)256 << 20;
  std::mutex park_mu;
  std::vector<std::pair<void*, size_t>> parked;
  size_t parked_bytes = 0;
  size_t park_cap = (size_t)16 << 30;
};

struct dp_problem {
  dp_ctx* ctx = nullptr;
  int64_t n = 0;
  int kind = 0;
  double omega = 0, eta = 0, L = 0, R0 = 0;
  bool equispaced = false;
  std::vector<double> hx, hy, hnx, hny, hsp, hkap;  // host copies
  dp::DevBuf src;       // SrcRec[n]
  dp::DevBuf C;         // double[n]
  dp::DevBuf C32;       // float[n], C_k / (pi dt) (single-precision sweep)
  dp::DevBuf diag;      // double4[n]: S_ii (re, im), D_ii
  dp::DevBuf srcblk;    // source blocks of the single-precision sweep (1 KB per 32 sources)
  dp::DevBuf twiddle;   // cplx[n]   (e^{-2 pi i l/n}), power-of-two n
  // Bluestein (chirp-z) DFT of length n for n not a power of two, through
  // power-of-two FFTs of length blu_M >= 2n - 1: chirp c_j = e^{i pi j^2/n},
  // FFT_M of the circular chirp sequence b, M twiddles, workspace M x columns
  int blu_M = 0;
  dp::DevBuf blu_tw, blu_chirp, blu_B, blu_ws;
  dp::DevBuf dens;      // sweep operands
  dp::DevBuf partial;   // sweep partial sums
  dp::DevBuf dens16;    // split-FP16 density tiles
  dp::DevBuf sc16;      // their per-column scales
  double cmax = 0;      // max |C_k| over k = 1..n-1
  double spmax = 0;     // max speed |x'(t_j)|
  // near-field pairs (i != j, r^2 < r2near = (DP_HANKEL_ZA/omega)^2), CSR by
  // target row, columns ascending; their kernel values use the small-argument
  // Hankel branch and are applied by a separate pass
  double r2near = 0;
  int64_t near_nnz = 0;
  dp::DevBuf near_ptr;  // int[n + 1]
  dp::DevBuf near_col;  // int[near_nnz]
  dp::DevBuf near_out;  // near-field sums [nd][nrp][n]
  dp::DevBuf near_kv[5];       // kernel values of the entries, per sweep operator ([q][nd])
  bool near_kv_ready[5] = {};
  // when every near pair lies within circular index distance near_band of
  // its row (a smooth curve sampled evenly: about 25/(omega h)), the same
  // values as a band [offset + near_band][d][row] (zero where a pair in the
  // band is not near), for the 64-column apply; -1: no band form
  int near_band = -1;
  dp::DevBuf near_bv[5];
  bool near_bv_ready[5] = {};
  dp::DevBuf tmp1, tmp2, tmp3;
  // GMRES workspaces (basis, preconditioned basis, w, r, partial sums, the
  // projection/norm block, the rotation state), kept between solves so that
  // repeated solves (refinement corrections, serving) do not allocate and
  // free them
  dp::DevBuf krylov_ws[7];
  // executable graphs of the Arnoldi step's orthogonalisation and rotation
  // update (basis sizes up to 16, and beyond), the workspace addresses and
  // sizes they were captured with, and whether capture works here
  hipGraphExec_t kgraph[2] = {nullptr, nullptr};
  std::vector<void*> kgraph_sig;
  bool kgraph_ok = true;
  // while set, sweeps launched for the operator skip their work when every
  // flag of sweep_guard[0 .. sweep_guard_n) is 0 (a queued Arnoldi step after
  // every column stopped)
  const int* sweep_guard = nullptr;
  int sweep_guard_n = 0;
  dp::DevBuf refine_ws[4];  // the same for the mixed-precision refinement (r, d, partial sums, flags)
  dp::Precond* pc = nullptr;
  // sweep launch configuration per (precision, operator, padded column count),
  // chosen by dp_autotune; absent keys use the default rule
  struct SweepCfg {
    int target_blocks = 2048;  // blocks of the sweep grid the source chunking aims at
    int mfma = -1;             // FP64, 5-16 columns: 0 VALU kernel, 1 matrix cores (16 columns split over the k steps), -1 default
  };
  std::map<int, SweepCfg> tuned;
  dp::SweepClock clock;    // FP64 sweep launches
  dp::SweepClock clock32;  // single-precision sweep launches
};

namespace dp {
// Pinned host memory of at least `bytes` bytes lent by the context (reused
// across solves and requests; hipHostFree, which waits for the device, only
// runs when the context is destroyed).  Returned with pinned_return.
int pinned_borrow(dp_ctx* c, size_t bytes, void** out, size_t* got);
void pinned_return(dp_ctx* c, void* p, size_t bytes);
// tables.hip
int build_tables(dp_problem* p);
// sweep.hip
// prec: 0 = FP64 sweep, 1 = mixed (FP32 kernel values and products with FP64
// geometry, phase reduction, small-argument Hankel values and diagonal terms)
int sweep_apply(dp_problem* p, int op, int nrhs, const cplx* q, cplx* y, int prec = 0);
int near_build(dp_problem* p);
int autotune(dp_problem* p, int nrhs, int prec, dp_tune_info* info);
// near.hip: near-field sums of one sweep group into p->near_out (no-op without near pairs)
int near_apply_group(dp_problem* p, int op, int nrp, const void* dens, bool dens32);
int matvec(dp_problem* p, int nrhs, const cplx* q, cplx* y, int prec = 0);
// fft.hip
int spectral_derivative(dp_problem* p, int nrhs, const cplx* in, cplx* out);
// In-place DFT of nb contiguous length-n columns (power-of-two n, twiddles
// built): dir -1 forward, +1 inverse (unnormalised).  With n = n1 n2 (n2 = 1
// up to 4096), the forward transform leaves X_k at position
// n2 (k mod n1) + k / n1 and the inverse expects that order.
void fft_inplace(dp_problem* p, cplx* d, int nb, int dir, int* n1, int* n2);
// Chirp, twiddles and chirp spectrum of the Bluestein DFT (n not a power of two).
int bluestein_init(dp_problem* p);
// Curvature from the spectral t-derivatives of the node positions (FFT
// tables built): written into the source records and into hkap (host, n).
int curvature_spectral(dp_problem* p, double* hkap);
// Per-node diagonal table (after the curvature and C_k are in place), and
// the source blocks of the single-precision sweep.
int build_diag(dp_problem* p);
// rhs
int rhs_plane_wave(dp_problem* p, int nrhs, const double* angles_dev, cplx* f);
// hankel test hook
int hankel_eval_dev(int64_t m, const double* z, double* out, hipStream_t s);
// krylov.hip
struct Gmres;
int solve(dp_problem* p, int nrhs, const cplx* f, cplx* q, const dp_solve_opts* o, dp_solve_info* info,
          int64_t* iters, double* relres);
// the executable graphs of the Arnoldi steps (problem teardown)
void krylov_graphs_destroy(dp_problem* p);
// Device-to-device copy of `bytes` (a multiple of 16) by a kernel on st
// (16-byte loads and stores, a grid-stride loop).
int dev_copy(void* dst, const void* src, size_t bytes, hipStream_t st);
// Default relative tolerance of the FP32 correction solves of a mixed solve to
// `tol`: sqrt(tol), so that two corrections share the reduction evenly (the
// second asks for 0.3 tol over the FP64 residual the first left), kept within
// [1e-5, 1e-2]: below 1e-5 a correction stops gaining in FP64 terms.
inline double default_inner_tol(double tol) {
  const double t = __builtin_sqrt(tol);
  return t < 1e-5 ? 1e-5 : (t > 1e-2 ? 1e-2 : t);
}
// precond
int precond_build(dp_problem* p, const dp_precond_opts* o);
// prec 1: single-precision tables and vectors (FP64 in and out)
int precond_apply(dp_problem* p, int nrhs, const cplx* v, cplx* z, int prec = 0);
void precond_destroy(Precond* pc);
int precond_info(dp_problem* p, dp_precond_info* info);
int precond_export(dp_problem* p, int64_t* seg_off, int64_t* seg_len, int64_t* e_idx, double* e_val);
// The device scratch array of the apply that allocates nothing: look up its
// address on `device` (that device current; once per device), its size, and
// the FP64 apply on it (DP_EINVAL beyond the size)
int scratch_init(int device);
size_t scratch_bytes();
int precond_apply_noalloc(dp_problem* p, int nrhs, const cplx* v, cplx* q);
}  // namespace dp
