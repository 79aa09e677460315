// Near-field pairs of the Nystrom matrix.
//
// The Hankel kernels are evaluated by two branches (dp_math.hpp): the
// asymptotic expansion for omega r >= DP_HANKEL_ZA and a Bessel recurrence
// below it.  The sweeps evaluate only the first (branch-free, so the
// matrix-core loop carries no divergent path and no extra live registers)
// and return 0 for pairs with r^2 < r2near = (DP_HANKEL_ZA/omega)^2.  Those
// pairs, about 2 DP_HANKEL_ZA/(omega h) per row for node spacing h (about 80
// at 10 points per wavelength), are listed here once per problem (CSR by
// target row, sources ascending), their kernel values are evaluated once per
// operator on first use, and near_apply multiplies them into the densities in
// FP64, writing sums that the sweep epilogue adds.  Both sides decide
// "near" with pair_r2, so every off-diagonal pair is applied exactly once.
#include "sweep_pair.hpp"

#include <algorithm>
#include <vector>

namespace dp {

namespace {


// Per-row count (pass 0) or fill (pass 1) of the near-field sources.  One
// thread per target row and source chunk (blockIdx.y: kScanChunks contiguous
// source ranges, so that n/64 x kScanChunks blocks fill the chip); the block
// streams its chunk's source positions through LDS in tiles of kScanTile
// (16 bytes each, read once per block instead of the 64-byte record once per
// pair), and every thread tests its row against the whole tile, so the
// entries of a (row, chunk) come out in ascending source order at the
// offset the host computed from the pass-0 counts.  The test is the sweep's
// own FP64 expression (pair_r2), so both agree on every pair.
constexpr int kScanRows = 64;     // rows (threads) per block
constexpr int kScanChunks = 8;    // source chunks per row
constexpr int kScanTile = 1024;   // sources per LDS tile (16 KB)
template <int PASS>
__global__ __launch_bounds__(kScanRows) void near_scan(const SrcRec* __restrict__ src, int n, double r2near,
                                                       int* __restrict__ cnt, const int* __restrict__ off,
                                                       int* __restrict__ col) {
  __shared__ double2 tile[kScanTile];
  const int i = blockIdx.x * kScanRows + threadIdx.x;
  const int chunk = blockIdx.y;
  const int per = (n + kScanChunks - 1) / kScanChunks;
  const int cb = min(n, chunk * per), ce = min(n, cb + per);
  const bool live = i < n;
  const double xi = live ? src[i].x : 0.0, yi = live ? src[i].y : 0.0;
  int c = 0;
  int o = (PASS == 1 && live) ? off[(size_t)chunk * n + i] : 0;
  for (int j0 = cb; j0 < ce; j0 += kScanTile) {
    const int len = min(kScanTile, ce - j0);
    __syncthreads();  // the previous tile has been read by every thread
    for (int k = threadIdx.x; k < len; k += kScanRows) tile[k] = make_double2(src[j0 + k].x, src[j0 + k].y);
    __syncthreads();
    if (!live) continue;
    int k = 0;
    for (; k + 4 <= len; k += 4) {  // four independent tests in flight
      bool hit[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double2 s = tile[k + u];
        hit[u] = (j0 + k + u != i) && pair_r2(xi, yi, s.x, s.y) < r2near;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (hit[u]) {
          if (PASS == 0) ++c;
          else col[o++] = j0 + k + u;
        }
      }
    }
    for (; k < len; ++k) {
      const double2 s = tile[k];
      if (j0 + k != i && pair_r2(xi, yi, s.x, s.y) < r2near) {
        if (PASS == 0) ++c;
        else col[o++] = j0 + k;
      }
    }
  }
  if (PASS == 0 && live) cnt[(size_t)chunk * n + i] = c;
}

struct NearParams {
  const SrcRec* src;
  const double* C;
  const int* ptr;
  const int* col;
  const cplx* kv;    // kernel values of the entries [q][nd], computed once per operator
  const void* dens;  // packed densities [j][nd][nrp] (cplx or cplxf)
  cplx* out;         // [nd][nrp][n]
  int n, nrp;
  double omega, eta, dt;
};

// Kernel values of every near-field entry (one wave per row, lanes over the
// row's entries); they depend only on the problem and the operator.
template <int OP>
__global__ __launch_bounds__(256) void near_values(NearParams p, cplx* kv) {
  constexpr int ND = Nd<OP>::v;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= p.n) return;
  const int lane = threadIdx.x & 63;
  const SrcRec tr = p.src[i];
  const Tgt t = {tr.x, tr.y, tr.nx, tr.ny};
  for (int q = p.ptr[i] + lane; q < p.ptr[i + 1]; q += 64) {
    const int j = p.col[q];
    int k = i - j;
    k += (k < 0) ? p.n : 0;
    cplx K[ND];
    pair_kernel_near<OP>(t, p.src[j], p.C[k], p.omega, p.eta, p.dt, K);
#pragma unroll
    for (int d = 0; d < ND; ++d) kv[(size_t)q * ND + d] = K[d];
  }
}

// One wave per target row (4 rows per block).  Lane l reads the kernel
// values of the row's near entry base + l; then lane (g, c), c < nrp,
// g < 64/nrp, accumulates entries l = g (mod 64/nrp) of column c, taking the
// values by cross-lane shuffles, and a butterfly over g sums the groups.
// Row blocks are spread so that each XCD (blocks b = x mod 8) works on a
// contiguous range of rows and finds the shared source densities in its L2.
template <int OP, class DT>
__global__ __launch_bounds__(256) void near_apply(NearParams p) {
  constexpr int ND = Nd<OP>::v;
  const int lane = threadIdx.x & 63;
  const int nb = gridDim.x;
  const int x = blockIdx.x & 7, q = nb >> 3, r = nb & 7;
  const int bb = x * q + min(x, r) + (blockIdx.x >> 3);
  const int i = bb * 4 + (threadIdx.x >> 6);
  if (i >= p.n) return;  // no block barriers below
  const int nrp = p.nrp;
  const int G = 64 / nrp;
  const int c = lane % nrp, g = lane / nrp;
  const DT* dens = static_cast<const DT*>(p.dens);
  cplx acc[ND];
#pragma unroll
  for (int d = 0; d < ND; ++d) acc[d] = {0.0, 0.0};
  const int e0 = p.ptr[i], e1 = p.ptr[i + 1];
  for (int base = e0; base < e1; base += 64) {
    const int cnt = min(64, e1 - base);
    int j = i;
    cplx K[ND];
#pragma unroll
    for (int d = 0; d < ND; ++d) K[d] = {0.0, 0.0};
    if (lane < cnt) {
      j = p.col[base + lane];
#pragma unroll
      for (int d = 0; d < ND; ++d) K[d] = p.kv[(size_t)(base + lane) * ND + d];
    }
    for (int l0 = 0; l0 < cnt; l0 += G) {
      const int l = l0 + g;  // < 64
      const int jl = __shfl(j, l);
#pragma unroll
      for (int d = 0; d < ND; ++d) {
        const cplx Kl = {__shfl(K[d].re, l), __shfl(K[d].im, l)};
        if (l < cnt) {
          const DT v = dens[((size_t)jl * ND + d) * nrp + c];
          cfma(acc[d], Kl, cplx{(double)v.re, (double)v.im});
        }
      }
    }
  }
  for (int off = nrp; off < 64; off <<= 1)
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      acc[d].re += __shfl_xor(acc[d].re, off);
      acc[d].im += __shfl_xor(acc[d].im, off);
    }
  if (g == 0)
#pragma unroll
    for (int d = 0; d < ND; ++d) p.out[((size_t)d * nrp + c) * p.n + i] = acc[d];
}

void launch_values(int op, const NearParams& np, cplx* kv, hipStream_t st) {
  const int grid = (np.n + 3) / 4;
  switch (op) {
    case OP_SOFT: near_values<OP_SOFT><<<grid, 256, 0, st>>>(np, kv); break;
    case OP_HARD: near_values<OP_HARD><<<grid, 256, 0, st>>>(np, kv); break;
    case OP_S: near_values<OP_S><<<grid, 256, 0, st>>>(np, kv); break;
    case OP_D: near_values<OP_D><<<grid, 256, 0, st>>>(np, kv); break;
    default: near_values<OP_DP><<<grid, 256, 0, st>>>(np, kv); break;
  }
}

constexpr int kNearGroup = 8;  // near-field entries whose density rows are gathered together

// All 64 columns: one lane per column, so a row's entries are the same for
// the whole wave (scalar loads of the column index and kernel values,
// kNearGroup entries in flight).  A block covers 16 consecutive rows, 4 per wave, and
// stages the sums in LDS (row stride padded to 17) so that each (density,
// column) is written as one 16-row run.  Row blocks are spread over the XCDs
// as in near_apply.
template <int OP, class DT>
__global__ __launch_bounds__(256) void near_apply64(NearParams p) {
  constexpr int ND = Nd<OP>::v;
  __shared__ cplx tile[ND * 64 * 17];  // [d][c][row]
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nb = gridDim.x;
  const int x = blockIdx.x & 7, q8 = nb >> 3, r8 = nb & 7;
  const int i0 = (x * q8 + min(x, r8) + (int)(blockIdx.x >> 3)) * 16;
  const DT* dens = static_cast<const DT*>(p.dens);
  for (int rr = 0; rr < 4; ++rr) {
    const int rl = wv * 4 + rr;
    const int i = i0 + rl;
    cplx acc[ND];
#pragma unroll
    for (int d = 0; d < ND; ++d) acc[d] = {0.0, 0.0};
    if (i < p.n) {
      const int e0 = p.ptr[i], e1 = p.ptr[i + 1];
      int q = e0;
      // groups of kNearGroup entries: all their density rows are requested
      // before the first product, so that enough gathers are in flight
      for (; q + kNearGroup <= e1; q += kNearGroup) {
        int j[kNearGroup];
        cplx K[kNearGroup][ND];
        DT v[kNearGroup][ND];
#pragma unroll
        for (int u = 0; u < kNearGroup; ++u) {
          j[u] = p.col[q + u];
#pragma unroll
          for (int d = 0; d < ND; ++d) K[u][d] = p.kv[(size_t)(q + u) * ND + d];
        }
#pragma unroll
        for (int u = 0; u < kNearGroup; ++u)
#pragma unroll
          for (int d = 0; d < ND; ++d) v[u][d] = dens[((size_t)j[u] * ND + d) * 64 + lane];
#pragma unroll
        for (int u = 0; u < kNearGroup; ++u)
#pragma unroll
          for (int d = 0; d < ND; ++d) cfma(acc[d], K[u][d], cplx{(double)v[u][d].re, (double)v[u][d].im});
      }
      for (; q < e1; ++q) {
        const int j = p.col[q];
#pragma unroll
        for (int d = 0; d < ND; ++d) {
          const DT v = dens[((size_t)j * ND + d) * 64 + lane];
          cfma(acc[d], p.kv[(size_t)q * ND + d], cplx{(double)v.re, (double)v.im});
        }
      }
    }
#pragma unroll
    for (int d = 0; d < ND; ++d) tile[(d * 64 + lane) * 17 + rl] = acc[d];
  }
  __syncthreads();
  for (int t = threadIdx.x; t < ND * 64 * 16; t += 256) {
    const int rl = t & 15, dc = t >> 4;  // dc = d * 64 + column
    const int i = i0 + rl;
    if (i < p.n) p.out[(size_t)dc * p.n + i] = tile[dc * 17 + rl];
  }
}

// ---- the band form of the 64-column apply
// Largest circular index distance between a row and its near sources.
__global__ __launch_bounds__(256) void near_bandwidth(const int* __restrict__ ptr, const int* __restrict__ col,
                                                      int n, int* out) {
  __shared__ int red[256];
  int m = 0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256)
    for (int q = ptr[i]; q < ptr[i + 1]; ++q) {
      int d = col[q] - i;
      d = d < 0 ? -d : d;
      d = min(d, n - d);
      m = max(m, d);
    }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = max(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(out, red[0]);
}

__global__ void zero_fill(cplx* x, size_t tot) {
  for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < tot; q += (size_t)gridDim.x * blockDim.x)
    x[q] = {0.0, 0.0};
}

// The entries' values in the band layout bv[((o nd + d) n + i)], o = the
// circular offset of the source plus B (one wave per row)
__global__ __launch_bounds__(256) void near_band_scatter(const int* __restrict__ ptr, const int* __restrict__ col,
                                                         const cplx* __restrict__ kv, cplx* bv, int n, int B, int nd) {
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  for (int q = ptr[i] + (threadIdx.x & 63); q < ptr[i + 1]; q += 64) {
    int d = col[q] - i;
    if (d > n / 2) d -= n;
    if (d < -n / 2) d += n;
    const int o = d + B;
    for (int e = 0; e < nd; ++e) bv[((size_t)o * nd + e) * n + i] = kv[(size_t)q * nd + e];
  }
}

// Near sums of 64 consecutive rows over a band of half-width B: the block
// stages the densities of its 64 + 2B source rows (mod n) in LDS, stored by
// (density, column) with the rows contiguous so that the lanes (one row each)
// read consecutive elements, and wave w accumulates CPT columns.  The values
// are stored offset by offset, [o][d][row], so that a wave reads them as 1 KB
// runs.  Every density element is loaded once per block instead of once per
// entry of every row that uses it.
constexpr int kBandRows = 64;

template <int OP, class DT, int CPT>
__global__ __launch_bounds__(512) void near_band64(NearParams p, const cplx* __restrict__ bv, int B) {
  constexpr int ND = Nd<OP>::v;
  constexpr int CB = 8 * CPT;  // columns of this block
  extern __shared__ unsigned char band_smem[];
  DT* ls = reinterpret_cast<DT*>(band_smem);  // [(d CB + c) LR + t]
  const int n = p.n;
  const int LR = kBandRows + 2 * B;
  const int lane = threadIdx.x & 63, cg = threadIdx.x >> 6;
  const int i0 = blockIdx.x * kBandRows;
  const int cb0 = blockIdx.y * CB;
  const DT* dens = static_cast<const DT*>(p.dens);
  // the tile, kTileBatch loads per thread in flight before their stores
  constexpr int kTileBatch = sizeof(DT) == sizeof(cplxf) ? 12 : 6;
  const int tot = LR * ND * CB;
  for (int e0 = threadIdx.x; e0 < tot; e0 += 512 * kTileBatch) {
    DT v[kTileBatch];
    int dst[kTileBatch];
#pragma unroll
    for (int u = 0; u < kTileBatch; ++u) {
      const int e = e0 + 512 * u;
      dst[u] = -1;
      v[u] = DT{0, 0};
      if (e < tot) {
        const int c = e % CB, rest = e / CB;
        const int d = rest % ND, t = rest / ND;
        int j = i0 - B + t;
        j += j < 0 ? n : 0;
        j -= j >= n ? n : 0;
        v[u] = dens[((size_t)j * ND + d) * 64 + cb0 + c];
        dst[u] = (d * CB + c) * LR + t;
      }
    }
#pragma unroll
    for (int u = 0; u < kTileBatch; ++u)
      if (dst[u] >= 0) ls[dst[u]] = v[u];
  }
  __syncthreads();
  const int i = i0 + lane;
  if (i >= n) return;  // no barriers below
  cplx acc[ND][CPT];
#pragma unroll
  for (int d = 0; d < ND; ++d)
#pragma unroll
    for (int u = 0; u < CPT; ++u) acc[d][u] = {0.0, 0.0};
  const DT* lrow = ls + cg * CPT * LR + lane;
  // offsets in groups of kOffBatch: the group's values are requested
  // together (the eight waves read the same ones, from the caches: staging
  // them in LDS for the block cost two barriers per group and was slower)
  constexpr int kOffBatch = 8;
  for (int o0 = 0; o0 <= 2 * B; o0 += kOffBatch) {
    cplx K[kOffBatch][ND];
#pragma unroll
    for (int t = 0; t < kOffBatch; ++t)
#pragma unroll
      for (int d = 0; d < ND; ++d)
        K[t][d] = o0 + t <= 2 * B ? bv[((size_t)(o0 + t) * ND + d) * n + i] : cplx{0.0, 0.0};
#pragma unroll
    for (int t = 0; t < kOffBatch; ++t) {
      if (o0 + t <= 2 * B) {  // source row i - B + o: tile row lane + o
        const int o = o0 + t;
#pragma unroll
        for (int d = 0; d < ND; ++d)
#pragma unroll
          for (int u = 0; u < CPT; ++u) {
            const DT v = lrow[(d * CB + u) * LR + o];
            cfma(acc[d][u], K[t][d], cplx{(double)v.re, (double)v.im});
          }
      }
    }
  }
#pragma unroll
  for (int d = 0; d < ND; ++d)
#pragma unroll
    for (int u = 0; u < CPT; ++u) p.out[((size_t)d * 64 + cb0 + cg * CPT + u) * n + i] = acc[d][u];
}

// LDS of near_band64 for one block, bytes
template <class DT>
size_t band_lds(int nd, int B) {
  const int cb = sizeof(DT) == sizeof(cplxf) ? 64 : 32;
  return (size_t)(kBandRows + 2 * B) * nd * cb * sizeof(DT);
}

constexpr size_t kBandLdsMax = 158 * 1024;  // of the 160 KB of a CU

template <int OP, class DT>
void launch_band(const NearParams& np, const cplx* bv, int B, hipStream_t st) {
  constexpr int ND = Nd<OP>::v;
  constexpr int CPT = sizeof(DT) == sizeof(cplxf) ? 8 : 4;
  const size_t lds = band_lds<DT>(ND, B);
  (void)hipFuncSetAttribute((const void*)near_band64<OP, DT, CPT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
  const dim3 grid((np.n + kBandRows - 1) / kBandRows, 64 / (8 * CPT));
  near_band64<OP, DT, CPT><<<grid, 512, lds, st>>>(np, bv, B);
}

template <class DT>
void launch_near(int op, const NearParams& np, hipStream_t st) {
  if (np.nrp == 64) {
    const int grid = (np.n + 15) / 16;
    switch (op) {
      case OP_SOFT: near_apply64<OP_SOFT, DT><<<grid, 256, 0, st>>>(np); break;
      case OP_HARD: near_apply64<OP_HARD, DT><<<grid, 256, 0, st>>>(np); break;
      case OP_S: near_apply64<OP_S, DT><<<grid, 256, 0, st>>>(np); break;
      case OP_D: near_apply64<OP_D, DT><<<grid, 256, 0, st>>>(np); break;
      default: near_apply64<OP_DP, DT><<<grid, 256, 0, st>>>(np); break;
    }
    return;
  }
  const int grid = (np.n + 3) / 4;
  switch (op) {
    case OP_SOFT: near_apply<OP_SOFT, DT><<<grid, 256, 0, st>>>(np); break;
    case OP_HARD: near_apply<OP_HARD, DT><<<grid, 256, 0, st>>>(np); break;
    case OP_S: near_apply<OP_S, DT><<<grid, 256, 0, st>>>(np); break;
    case OP_D: near_apply<OP_D, DT><<<grid, 256, 0, st>>>(np); break;
    default: near_apply<OP_DP, DT><<<grid, 256, 0, st>>>(np); break;
  }
}

}  // namespace

int near_build(dp_problem* p) {
  hipStream_t st = p->ctx->stream;
  const int n = (int)p->n;
  const double zr = DP_HANKEL_ZA / p->omega;
  p->r2near = zr * zr;
  DevBuf cnt, off;
  struct Release {
    DevBuf &a, &b;
    ~Release() {
      a.release();
      b.release();
    }
  } release{cnt, off};
  const size_t nc = (size_t)kScanChunks * n;
  DP_TRY(cnt.reserve(nc * sizeof(int)));
  const dim3 grid((n + kScanRows - 1) / kScanRows, kScanChunks);
  near_scan<0><<<grid, kScanRows, 0, st>>>(p->src.as<SrcRec>(), n, p->r2near, cnt.as<int>(), nullptr, nullptr);
  DP_HIP(hipGetLastError());
  std::vector<int> hc(nc);
  DP_HIP(hipMemcpyAsync(hc.data(), cnt.p, nc * sizeof(int), hipMemcpyDeviceToHost, st));
  DP_HIP(hipStreamSynchronize(st));
  // row pointers and, per (chunk, row), the offset of its first entry
  std::vector<int> hp(n + 1), ho(nc);
  int64_t tot = 0;
  for (int i = 0; i < n; ++i) {
    hp[i] = (int)tot;
    for (int c = 0; c < kScanChunks; ++c) {
      ho[(size_t)c * n + i] = (int)tot;
      tot += hc[(size_t)c * n + i];
    }
    if (tot > 0x7fffffff) {
      set_error("near field too large: more than 2^31 pairs have omega r < 25 (frequency too low for n)");
      return DP_EINVAL;
    }
  }
  hp[n] = (int)tot;
  p->near_nnz = tot;
  DP_TRY(p->near_ptr.reserve((size_t)(n + 1) * sizeof(int)));
  DP_TRY(p->near_col.reserve((size_t)(tot > 0 ? tot : 1) * sizeof(int)));
  DP_HIP(hipMemcpyAsync(p->near_ptr.p, hp.data(), (size_t)(n + 1) * sizeof(int), hipMemcpyHostToDevice, st));
  if (tot > 0) {
    DP_TRY(off.reserve(nc * sizeof(int)));
    DP_HIP(hipMemcpyAsync(off.p, ho.data(), nc * sizeof(int), hipMemcpyHostToDevice, st));
    near_scan<1><<<grid, kScanRows, 0, st>>>(p->src.as<SrcRec>(), n, p->r2near, nullptr, off.as<int>(),
                                             p->near_col.as<int>());
    DP_HIP(hipGetLastError());
  }
  // band form: every near source within B rows (circularly) of its target,
  // and B small against n (no source row reached by two offsets)
  p->near_band = -1;
  for (auto& b : p->near_bv_ready) b = false;
  if (tot > 0) {
    DP_HIP(hipMemsetAsync(cnt.p, 0, sizeof(int), st));
    near_bandwidth<<<std::min(1024, (n + 255) / 256), 256, 0, st>>>(p->near_ptr.as<int>(), p->near_col.as<int>(), n,
                                                                    cnt.as<int>());
    DP_HIP(hipGetLastError());
    int B = 0;
    DP_HIP(hipMemcpyAsync(&B, cnt.p, sizeof(int), hipMemcpyDeviceToHost, st));
    DP_HIP(hipStreamSynchronize(st));
    if (B >= 1 && (int64_t)4 * (kBandRows + 2 * B) <= n) p->near_band = B;
  }
  DP_HIP(hipStreamSynchronize(st));
  return DP_OK;
}

int near_apply_group(dp_problem* p, int op, int nrp, const void* dens, bool dens32) {
  if (p->near_nnz == 0) return DP_OK;
  const int nd = op == OP_HARD ? 2 : 1;
  DP_TRY(p->near_out.reserve((size_t)nd * nrp * p->n * sizeof(cplx)));
  NearParams np;
  np.src = p->src.as<SrcRec>();
  np.C = p->C.as<double>();
  np.ptr = p->near_ptr.as<int>();
  np.col = p->near_col.as<int>();
  np.dens = dens;
  np.out = p->near_out.as<cplx>();
  np.n = (int)p->n;
  np.nrp = nrp;
  np.omega = p->omega;
  np.eta = p->eta;
  np.dt = 2.0 * kPi / p->n;
  if (!p->near_kv_ready[op]) {
    DP_TRY(p->near_kv[op].reserve((size_t)p->near_nnz * nd * sizeof(cplx)));
    launch_values(op, np, p->near_kv[op].as<cplx>(), p->ctx->stream);
    DP_HIP(hipGetLastError());
    p->near_kv_ready[op] = true;
  }
  np.kv = p->near_kv[op].as<cplx>();
  const int B = p->near_band;
  const bool band = nrp == 64 && B > 0 &&
                    (dens32 ? band_lds<cplxf>(nd, B) : band_lds<cplx>(nd, B)) <= kBandLdsMax;
  if (band) {
    hipStream_t st = p->ctx->stream;
    if (!p->near_bv_ready[op]) {
      const size_t tot = (size_t)(2 * B + 1) * nd * p->n;
      DP_TRY(p->near_bv[op].reserve(tot * sizeof(cplx)));
      zero_fill<<<(int)std::min<size_t>(8192, (tot + 255) / 256), 256, 0, st>>>(p->near_bv[op].as<cplx>(), tot);
      near_band_scatter<<<(np.n + 3) / 4, 256, 0, st>>>(np.ptr, np.col, np.kv, p->near_bv[op].as<cplx>(), np.n, B,
                                                       nd);
      DP_HIP(hipGetLastError());
      p->near_bv_ready[op] = true;
    }
    const cplx* bv = p->near_bv[op].as<cplx>();
    switch (op) {
      case OP_SOFT: dens32 ? launch_band<OP_SOFT, cplxf>(np, bv, B, st) : launch_band<OP_SOFT, cplx>(np, bv, B, st); break;
      case OP_HARD: dens32 ? launch_band<OP_HARD, cplxf>(np, bv, B, st) : launch_band<OP_HARD, cplx>(np, bv, B, st); break;
      case OP_S: dens32 ? launch_band<OP_S, cplxf>(np, bv, B, st) : launch_band<OP_S, cplx>(np, bv, B, st); break;
      case OP_D: dens32 ? launch_band<OP_D, cplxf>(np, bv, B, st) : launch_band<OP_D, cplx>(np, bv, B, st); break;
      default: dens32 ? launch_band<OP_DP, cplxf>(np, bv, B, st) : launch_band<OP_DP, cplx>(np, bv, B, st); break;
    }
  } else if (dens32) {
    launch_near<cplxf>(op, np, p->ctx->stream);
  } else {
    launch_near<cplx>(op, np, p->ctx->stream);
  }
  DP_HIP(hipGetLastError());
  return DP_OK;
}

}  // namespace dp
