// Sparse LU of floor(W) = E + antidiag(T) (Sec. 2.2): the paper factors this
// extremely sparse matrix (about 1.5 - 5 non-zeros per row) with a sparse LU
// "up to possible permutations".  Here:
//   1. fill-reducing symmetric ordering Q by minimum degree on the graph of
//      W + W^t (explicit elimination graph, ties broken by index);
//   2. left-looking LU of A' = W(Q, Q) with threshold partial pivoting (the
//      diagonal is kept when |a_kk| >= 0.1 max_i |a_ik|), each column by a
//      sparse triangular solve over the reach of its pattern (depth-first
//      search in the graph of L);
//   3. row-oriented copies of L and U and their dependency levels, so that
//      the device solves process one level per step.
// When the segments couple nearly all-to-all through E the factors fill in
// (the Schur complement of the last few thousand nodes is dense); the caller
// then gets kSparseFillLimit, decided from the ordering's symbolic fill
// before any numeric work, and factors floor(W) densely on the device.
// This is setup work of O(nnz(L + U)) on the host; the per-iteration solves
// run on the GPU.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstdio>
#include <set>
#include <vector>

#include "dp_internal.hpp"
#include "sparse_lu.hpp"

namespace dp {

using zc = std::complex<double>;

// Minimum degree ordering of the symmetric pattern given by adjacency lists.
// The degree of each node when it is eliminated is the size of its column in
// the symbolic factor; their sum (times two, plus n) predicts nnz(L + U)
// without pivoting.  The ordering stops early, returning an empty order,
// once that prediction exceeds max_fill.
static std::vector<int> min_degree(int n, std::vector<std::vector<int>> adj, int64_t max_fill) {
  int64_t fill = n;
  std::vector<char> elim(n, 0);
  std::vector<int> mark(n, -1);
  std::set<std::pair<int, int>> pq;
  for (int v = 0; v < n; ++v) pq.insert({(int)adj[v].size(), v});
  std::vector<int> order;
  order.reserve(n);
  std::vector<int> nb, merged;
  int stamp = 0;
  while (!pq.empty()) {
    const int v = pq.begin()->second;
    pq.erase(pq.begin());
    elim[v] = 1;
    order.push_back(v);
    nb.clear();
    for (int a : adj[v])
      if (!elim[a]) nb.push_back(a);
    fill += 2 * (int64_t)nb.size();
    if (fill > max_fill) return {};
    for (int a : nb) {
      pq.erase({(int)adj[a].size(), a});
      ++stamp;
      merged.clear();
      for (int b : adj[a])
        if (!elim[b] && mark[b] != stamp) {
          mark[b] = stamp;
          merged.push_back(b);
        }
      for (int b : nb)
        if (b != a && mark[b] != stamp) {
          mark[b] = stamp;
          merged.push_back(b);
        }
      adj[a].swap(merged);
      pq.insert({(int)adj[a].size(), a});
    }
    adj[v].clear();
  }
  return order;
}

std::vector<int> sparse_lu_order(int n, const std::vector<int>& cp, const std::vector<int>& ri, int64_t max_fill) {
  // ordering on the symmetrised pattern
  std::vector<std::vector<int>> adj(n);
  for (int j = 0; j < n; ++j)
    for (int p = cp[j]; p < cp[j + 1]; ++p) {
      const int i = ri[p];
      if (i == j) continue;
      adj[i].push_back(j);
      adj[j].push_back(i);
    }
  for (auto& a : adj) {
    std::sort(a.begin(), a.end());
    a.erase(std::unique(a.begin(), a.end()), a.end());
  }
  return min_degree(n, adj, max_fill);
}

int sparse_lu_factor(int n, const std::vector<int>& cp, const std::vector<int>& ri, const std::vector<zc>& vx,
                     SparseLU& out, int64_t max_fill) {
  const std::vector<int> Q = sparse_lu_order(n, cp, ri, max_fill);
  if (Q.empty() && n > 0) return kSparseFillLimit;
  return sparse_lu_factor_ordered(n, cp, ri, vx, Q, out, max_fill);
}

int sparse_lu_factor_ordered(int n, const std::vector<int>& cp, const std::vector<int>& ri,
                             const std::vector<zc>& vx, const std::vector<int>& Q, SparseLU& out, int64_t max_fill) {
  std::vector<int> Qinv(n);
  for (int a = 0; a < n; ++a) Qinv[Q[a]] = a;
  // A' = W(Q, Q) in CSC: column b of A' is column Q[b] of W with rows relabelled
  std::vector<int> ap(n + 1, 0), ai;
  std::vector<zc> ax;
  ai.reserve(ri.size());
  ax.reserve(ri.size());
  for (int b = 0; b < n; ++b) {
    const int j = Q[b];
    for (int p = cp[j]; p < cp[j + 1]; ++p) {
      ai.push_back(Qinv[ri[p]]);
      ax.push_back(vx[p]);
    }
    ap[b + 1] = (int)ai.size();
  }
  // ---- left-looking LU (Gilbert-Peierls)
  std::vector<int> pinv(n, -1);
  std::vector<int> Lcp(1, 0), Lri;  // L columns: row indices in A' numbering (relabelled later)
  std::vector<zc> Lv;
  std::vector<int> Ucp(1, 0), Uri;  // U columns: row indices = pivot positions
  std::vector<zc> Uv;
  std::vector<zc> x(n, 0.0);
  std::vector<int> stack(n), pstack(n), xi(n);
  std::vector<int> visited(n, -1);
  for (int k = 0; k < n; ++k) {
    // reach of column k in the graph of L (nodes = A' rows; pivoted rows lead to their L column)
    int top = n;
    for (int p = ap[k]; p < ap[k + 1]; ++p) {
      const int r0 = ai[p];
      if (visited[r0] == k) continue;
      int head = 0;
      stack[0] = r0;
      while (head >= 0) {
        const int r = stack[head];
        const int col = pinv[r];
        if (visited[r] != k) {
          visited[r] = k;
          pstack[head] = col < 0 ? 0 : Lcp[col];
        }
        bool done = true;
        if (col >= 0) {
          const int end = Lcp[col + 1];
          for (int q = pstack[head]; q < end; ++q) {
            const int i = Lri[q];
            if (visited[i] == k) continue;
            pstack[head] = q + 1;
            stack[++head] = i;
            done = false;
            break;
          }
        }
        if (done) {
          --head;
          xi[--top] = r;
        }
      }
    }
    for (int p = ap[k]; p < ap[k + 1]; ++p) x[ai[p]] = ax[p];
    for (int t = top; t < n; ++t) {
      const int r = xi[t];
      const int col = pinv[r];
      if (col < 0) continue;
      const zc xr = x[r];
      for (int q = Lcp[col]; q < Lcp[col + 1]; ++q) x[Lri[q]] -= Lv[q] * xr;
    }
    // pivot among unpivoted rows of the reach
    int piv = -1;
    double amax = -1.0;
    for (int t = top; t < n; ++t) {
      const int r = xi[t];
      if (pinv[r] >= 0) continue;
      const double a = std::abs(x[r]);
      if (a > amax) {
        amax = a;
        piv = r;
      }
    }
    if (piv < 0 || amax == 0.0 || !std::isfinite(amax)) {
      set_error("sparse LU of floor(W): zero pivot in column %d", k);
      return DP_ESINGULAR;
    }
    if (pinv[k] < 0 && visited[k] == k && std::abs(x[k]) >= 0.1 * amax) piv = k;
    const zc pv = x[piv];
    for (int t = top; t < n; ++t) {
      const int r = xi[t];
      if (pinv[r] >= 0) {
        Uri.push_back(pinv[r]);
        Uv.push_back(x[r]);
      }
    }
    Uri.push_back(k);
    Uv.push_back(pv);
    Ucp.push_back((int)Uri.size());
    pinv[piv] = k;
    for (int t = top; t < n; ++t) {
      const int r = xi[t];
      if (pinv[r] < 0) {
        Lri.push_back(r);
        Lv.push_back(x[r] / pv);
      }
      x[r] = 0.0;
    }
    Lcp.push_back((int)Lri.size());
    // pivoting can fill more than the symbolic prediction: stop at twice it
    if (max_fill < INT64_MAX / 2 && (int64_t)(Lri.size() + Uri.size()) > 2 * max_fill) return kSparseFillLimit;
  }
  for (auto& r : Lri) r = pinv[r];
  // ---- row-oriented copies (pivot numbering)
  out.n = n;
  out.Lp.assign(n + 1, 0);
  out.Up.assign(n + 1, 0);
  out.Ud.assign(n, 0.0);
  for (int r : Lri) out.Lp[r + 1]++;
  for (int c = 0; c < n; ++c)
    for (int q = Ucp[c]; q < Ucp[c + 1]; ++q)
      if (Uri[q] != c) out.Up[Uri[q] + 1]++;
  for (int i = 0; i < n; ++i) {
    out.Lp[i + 1] += out.Lp[i];
    out.Up[i + 1] += out.Up[i];
  }
  out.Lj.assign(out.Lp[n], 0);
  out.Lx.assign(out.Lp[n], 0.0);
  out.Uj.assign(out.Up[n], 0);
  out.Ux.assign(out.Up[n], 0.0);
  std::vector<int> fl(out.Lp.begin(), out.Lp.end() - 1), fu(out.Up.begin(), out.Up.end() - 1);
  for (int c = 0; c < n; ++c) {
    for (int q = Lcp[c]; q < Lcp[c + 1]; ++q) {
      const int r = Lri[q];
      out.Lj[fl[r]] = c;
      out.Lx[fl[r]++] = Lv[q];
    }
    for (int q = Ucp[c]; q < Ucp[c + 1]; ++q) {
      const int r = Uri[q];
      if (r == c) {
        out.Ud[c] = Uv[q];
      } else {
        out.Uj[fu[r]] = c;
        out.Ux[fu[r]++] = Uv[q];
      }
    }
  }
  // ---- permutations: zp[pinv[a]] = z[Q[a]];  u[Q[b]] = u'[b]
  out.perm_in.assign(n, 0);
  out.perm_out.assign(n, 0);
  for (int a = 0; a < n; ++a) out.perm_in[pinv[a]] = Q[a];
  for (int b = 0; b < n; ++b) out.perm_out[b] = Q[b];
  // ---- levels
  auto levels = [&](const std::vector<int>& P, const std::vector<int>& J, bool lower, std::vector<int>& lptr,
                    std::vector<int>& lrows) {
    std::vector<int> lev(n, 0);
    int nl = 0;
    for (int t = 0; t < n; ++t) {
      const int i = lower ? t : n - 1 - t;
      int l = 0;
      for (int q = P[i]; q < P[i + 1]; ++q) l = std::max(l, lev[J[q]] + 1);
      lev[i] = l;
      nl = std::max(nl, l + 1);
    }
    lptr.assign(nl + 1, 0);
    for (int i = 0; i < n; ++i) lptr[lev[i] + 1]++;
    for (int l = 0; l < nl; ++l) lptr[l + 1] += lptr[l];
    lrows.assign(n, 0);
    std::vector<int> f(lptr.begin(), lptr.end() - 1);
    for (int i = 0; i < n; ++i) lrows[f[lev[i]]++] = i;
  };
  levels(out.Lp, out.Lj, true, out.lvlL_ptr, out.lvlL_rows);
  levels(out.Up, out.Uj, false, out.lvlU_ptr, out.lvlU_rows);
  return DP_OK;
}

}  // namespace dp
