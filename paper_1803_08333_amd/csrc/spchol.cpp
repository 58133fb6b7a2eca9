// Nested-dissection multifrontal Cholesky of the projector matrices (host,
// FP64).  See spchol.h for the layout of the factor.
#include "spchol.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <numeric>
#include <thread>
#include <tuple>

namespace rfcmp {
namespace {

// ------------------------------------------------------------------ ordering
// Recursive coordinate bisection.  A part of at most `leaf` nodes is a leaf
// supernode.  A larger part is split at the median of its longest axis into
// halves P and Q; the nodes of one half with a neighbour in the other half
// (the smaller such set) form the separator S.  Order: the first part, the
// second part, then S, so every separator follows both of its subtrees.
struct Dissection {
  const SpMatrix& A;
  int leaf;
  std::vector<int> order;     // elimination order (original rows)
  std::vector<int> sn_start;  // first position of each supernode
  std::vector<int> tag;       // per node: which half it lies in (unique per split)
  int next_tag = 0;

  Dissection(const SpMatrix& a, int lf) : A(a), leaf(lf), tag(a.n, -1) {}

  void emit(std::vector<int> nodes) {
    if (nodes.empty()) return;
    std::sort(nodes.begin(), nodes.end());
    sn_start.push_back((int)order.size());
    order.insert(order.end(), nodes.begin(), nodes.end());
  }

  // boundary of `from` towards the half tagged `other`
  std::vector<int> boundary(const std::vector<int>& from, int other) const {
    std::vector<int> b;
    for (int v : from)
      for (int q = A.ptr[v]; q < A.ptr[v + 1]; ++q)
        if (tag[A.idx[q]] == other) {
          b.push_back(v);
          break;
        }
    return b;
  }

  void split(std::vector<int> nodes) {
    if ((int)nodes.size() <= leaf) {
      emit(nodes);
      return;
    }
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int v : nodes)
      for (int d = 0; d < 3; ++d) {
        lo[d] = std::min(lo[d], A.xyz[3 * v + d]);
        hi[d] = std::max(hi[d], A.xyz[3 * v + d]);
      }
    int ax = 0;
    for (int d = 1; d < 3; ++d)
      if (hi[d] - lo[d] > hi[ax] - lo[ax]) ax = d;
    // median split (ties broken by index, so the order is deterministic)
    const size_t half = nodes.size() / 2;
    std::nth_element(nodes.begin(), nodes.begin() + half, nodes.end(), [&](int a, int b) {
      const double xa = A.xyz[3 * a + ax], xb = A.xyz[3 * b + ax];
      return xa < xb || (xa == xb && a < b);
    });
    std::vector<int> P(nodes.begin(), nodes.begin() + half), Q(nodes.begin() + half, nodes.end());
    const int tp = next_tag++, tq = next_tag++;
    for (int v : P) tag[v] = tp;
    for (int v : Q) tag[v] = tq;
    std::vector<int> bp = boundary(P, tq), bq = boundary(Q, tp);
    const bool from_p = bp.size() <= bq.size();
    const std::vector<int>& S = from_p ? bp : bq;
    std::vector<int>& rest = from_p ? P : Q;
    {
      const int ts = next_tag++;
      for (int v : S) tag[v] = ts;
      std::vector<int> r;
      r.reserve(rest.size() - S.size());
      for (int v : rest)
        if (tag[v] != ts) r.push_back(v);
      rest.swap(r);
    }
    std::vector<int> sep = S;
    split(std::move(P));
    split(std::move(Q));
    emit(sep);
  }
};

// y[0..n) -= f x[0..n); x and y never overlap (different front columns)
inline void axpy_neg(int n, double f, const double* __restrict x, double* __restrict y) {
  for (int i = 0; i < n; ++i) y[i] -= x[i] * f;
}

// Run f(i) for i in [0, n) on up to `threads` host threads.
template <class F>
void parallel_for(int n, int threads, F f) {
  const int t = std::min(threads, n);
  if (t <= 1) {
    for (int i = 0; i < n; ++i) f(i);
    return;
  }
  std::atomic<int> next{0};
  std::vector<std::thread> pool;
  for (int q = 0; q < t; ++q)
    pool.emplace_back([&] {
      for (int i; (i = next.fetch_add(1)) < n;) f(i);
    });
  for (auto& th : pool) th.join();
}

}  // namespace

rfcmp_status spchol_factor(const SpMatrix& A, bool grounded, int leaf, int threads, SpFactor& F) {
  const auto t0 = std::chrono::steady_clock::now();
  const int n = A.n;
  F = SpFactor{};
  F.n = n;
  F.grounded = grounded;
  if (n <= 0) {
    set_error("sparse factor of an empty matrix");
    return RFCMP_E_ARG;
  }
  // ---- order
  Dissection D(A, std::max(leaf, 1));
  {
    std::vector<int> all(n);
    std::iota(all.begin(), all.end(), 0);
    D.split(std::move(all));
  }
  const auto t1 = std::chrono::steady_clock::now();
  F.sec_order = std::chrono::duration<double>(t1 - t0).count();
  F.perm = std::move(D.order);
  std::vector<int> iperm(n);
  for (int i = 0; i < n; ++i) iperm[F.perm[i]] = i;
  const int nsn = (int)D.sn_start.size();
  F.nsn = nsn;
  F.col0 = D.sn_start;
  F.col0.push_back(n);
  std::vector<int> sn_of(n);
  for (int s = 0; s < nsn; ++s)
    for (int j = F.col0[s]; j < F.col0[s + 1]; ++j) sn_of[j] = s;

  // ---- symbolic: struct(s) = rows beyond s adjacent to its columns, and the
  // struct rows of its children beyond it
  std::vector<std::vector<int>> st(nsn), kids(nsn);
  F.parent.assign(nsn, -1);
  F.height.assign(nsn, 0);
  {
    std::vector<int> mark(n, -1);
    for (int s = 0; s < nsn; ++s) {
      const int c1 = F.col0[s + 1];
      std::vector<int>& rows = st[s];
      auto add = [&](int r) {
        if (r >= c1 && mark[r] != s) {
          mark[r] = s;
          rows.push_back(r);
        }
      };
      for (int j = F.col0[s]; j < c1; ++j) {
        const int v = F.perm[j];
        for (int q = A.ptr[v]; q < A.ptr[v + 1]; ++q) add(iperm[A.idx[q]]);
      }
      for (int c : kids[s]) {
        for (int r : st[c]) add(r);
        F.height[s] = std::max(F.height[s], F.height[c] + 1);
      }
      std::sort(rows.begin(), rows.end());
      if (!rows.empty()) {
        F.parent[s] = sn_of[rows[0]];
        kids[F.parent[s]].push_back(s);
      }
    }
  }
  F.str_off.assign(nsn + 1, 0);
  F.panel_off.assign(nsn + 1, 0);
  F.child_off.assign(nsn + 1, 0);
  for (int s = 0; s < nsn; ++s) {
    const int ncol = F.col0[s + 1] - F.col0[s];
    const int m = ncol + (int)st[s].size();
    F.str_off[s + 1] = F.str_off[s] + (int)st[s].size();
    F.panel_off[s + 1] = F.panel_off[s] + (int64_t)m * ncol;
    F.child_off[s + 1] = F.child_off[s] + (int)kids[s].size();
    F.max_front = std::max(F.max_front, m);
  }
  F.str.resize(F.str_off[nsn]);
  F.map.resize(F.str_off[nsn]);
  F.child_idx.resize(F.child_off[nsn]);
  for (int s = 0; s < nsn; ++s) {
    std::copy(st[s].begin(), st[s].end(), F.str.begin() + F.str_off[s]);
    std::copy(kids[s].begin(), kids[s].end(), F.child_idx.begin() + F.child_off[s]);
    const int p = F.parent[s];
    if (p < 0) continue;
    const int pc0 = F.col0[p], pc1 = F.col0[p + 1];
    for (size_t t = 0; t < st[s].size(); ++t) {
      const int r = st[s][t];
      int pos;
      if (r < pc1) {
        pos = r - pc0;
      } else {
        auto it = std::lower_bound(st[p].begin(), st[p].end(), r);
        pos = (pc1 - pc0) + (int)(it - st[p].begin());
      }
      F.map[F.str_off[s] + t] = pos;
    }
  }

  const auto t2 = std::chrono::steady_clock::now();
  F.sec_symbolic = std::chrono::duration<double>(t2 - t1).count();
  // ---- numeric, multifrontal, one height at a time (the supernodes of one
  // height are independent)
  F.panel.assign(F.panel_off[nsn], 0.0);
  std::vector<std::vector<double>> upd(nsn);  // update matrix of each supernode, nstr x nstr
  int H = 0;
  for (int s = 0; s < nsn; ++s) H = std::max(H, F.height[s]);
  std::vector<std::vector<int>> by_height(H + 1);
  for (int s = 0; s < nsn; ++s) by_height[F.height[s]].push_back(s);
  std::atomic<int> bad{-1};
  const int nth = std::max(1, threads);
  for (int h = 0; h <= H; ++h) {
    const std::vector<int>& level = by_height[h];
    parallel_for((int)level.size(), nth, [&](int li) {
      thread_local std::vector<double> Fr;
      thread_local std::vector<int> loc;
      if ((int)loc.size() < n) loc.assign(n, 0);
      const int s = level[li];
      const int c0 = F.col0[s], c1 = F.col0[s + 1];
      const int ncol = c1 - c0;
      const int nstr = F.str_off[s + 1] - F.str_off[s];
      const int m = ncol + nstr;
      const int* srow = &F.str[F.str_off[s]];
      Fr.assign((size_t)m * m, 0.0);
      for (int i = 0; i < ncol; ++i) loc[c0 + i] = i;
      for (int t = 0; t < nstr; ++t) loc[srow[t]] = ncol + t;
      for (int j = c0; j < c1; ++j) {
        const int v = F.perm[j];
        const size_t jj = (size_t)(j - c0) * m;
        for (int q = A.ptr[v]; q < A.ptr[v + 1]; ++q) {
          const int r = iperm[A.idx[q]];
          if (r >= j) Fr[jj + loc[r]] += A.val[q];
        }
        if (grounded && j == n - 1) Fr[jj + (j - c0)] += 1.0;
      }
      for (int q = F.child_off[s]; q < F.child_off[s + 1]; ++q) {
        const int c = F.child_idx[q];
        const int nc = F.str_off[c + 1] - F.str_off[c];
        const int* mp = &F.map[F.str_off[c]];
        const std::vector<double>& U = upd[c];
        for (int b = 0; b < nc; ++b) {
          double* col = &Fr[(size_t)mp[b] * m];
          const double* ub = &U[(size_t)b * nc];
          for (int a = b; a < nc; ++a) col[mp[a]] += ub[a];
        }
      }
      for (int q = F.child_off[s]; q < F.child_off[s + 1]; ++q) std::vector<double>().swap(upd[F.child_idx[q]]);
      // partial Cholesky of the front: the first ncol columns
      for (int j = 0; j < ncol; ++j) {
        double* cj = &Fr[(size_t)j * m];
        const double d = cj[j];
        if (!(d > 0.0) || !std::isfinite(d)) {
          bad.store(s);
          return;
        }
        const double l = std::sqrt(d), inv = 1.0 / l;
        cj[j] = l;
        for (int i = j + 1; i < m; ++i) cj[i] *= inv;
        for (int k = j + 1; k < m; ++k) {
          const double f = cj[k];
          if (f == 0.0) continue;
          axpy_neg(m - k, f, cj + k, &Fr[(size_t)k * m + k]);
        }
      }
      double* pan = &F.panel[F.panel_off[s]];
      for (int j = 0; j < ncol; ++j)
        for (int i = j; i < m; ++i) pan[(size_t)j * m + i] = Fr[(size_t)j * m + i];
      if (nstr > 0) {
        std::vector<double>& U = upd[s];
        U.assign((size_t)nstr * nstr, 0.0);
        for (int b = 0; b < nstr; ++b)
          for (int a = b; a < nstr; ++a) U[(size_t)b * nstr + a] = Fr[(size_t)(ncol + b) * m + ncol + a];
      }
    });
    if (bad.load() >= 0) {
      set_error("sparse factor: non-positive pivot in supernode %d (matrix not positive definite)", bad.load());
      return RFCMP_E_ARG;
    }
  }
  const auto t3 = std::chrono::steady_clock::now();
  F.sec_numeric = std::chrono::duration<double>(t3 - t2).count();
  F.seconds = std::chrono::duration<double>(t3 - t0).count();
  return RFCMP_OK;
}

// ------------------------------------------------------------------ matrices
namespace {
// CSR from a list of (row, col, value) with both triangles present; equal
// (row, col) entries are summed.
void to_csr(int n, std::vector<std::tuple<int, int, double>>& e, SpMatrix& A) {
  std::sort(e.begin(), e.end(), [](const auto& a, const auto& b) {
    return std::get<0>(a) < std::get<0>(b) || (std::get<0>(a) == std::get<0>(b) && std::get<1>(a) < std::get<1>(b));
  });
  A.n = n;
  A.ptr.assign(n + 1, 0);
  A.idx.clear();
  A.val.clear();
  int last_r = -1;
  for (const auto& t : e) {
    const int r = std::get<0>(t), c = std::get<1>(t);
    if (r == last_r && A.idx.back() == c) {
      A.val.back() += std::get<2>(t);
      continue;
    }
    A.idx.push_back(c);
    A.val.push_back(std::get<2>(t));
    A.ptr[r + 1]++;
    last_r = r;
  }
  for (int r = 0; r < n; ++r) A.ptr[r + 1] += A.ptr[r];
}
}  // namespace

void laplacian_matrix(const MeshHost& h, SpMatrix& A) {
  const int C = (int)h.C;
  std::vector<std::tuple<int, int, double>> e;
  e.reserve((size_t)C + 2 * h.N);
  for (int c = 0; c < C; ++c) e.emplace_back(c, c, 3.0);
  for (int64_t q = 0; q < h.N; ++q) {
    const int a = h.edge_cell[2 * q], b = h.edge_cell[2 * q + 1];
    e.emplace_back(a, b, -1.0);
    e.emplace_back(b, a, -1.0);
  }
  to_csr(C, e, A);
  A.xyz = h.centroid;
}

void gram_ll_matrix(const MeshHost& h, SpMatrix& A) {
  const int V = (int)h.V;
  std::vector<std::tuple<int, int, double>> e;
  e.reserve((size_t)9 * h.C);
  for (int64_t c = 0; c < h.C; ++c) {
    const double a = h.area[c];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) e.emplace_back(h.tri[3 * c + i], h.tri[3 * c + j], i == j ? a / 6.0 : a / 12.0);
  }
  to_csr(V, e, A);
  A.xyz = h.xyz;
}

void gram_tp_matrix(const MeshHost& h, SpMatrix& A) {
  const int C = (int)h.C;
  std::vector<std::tuple<int, int, double>> e;
  e.reserve(h.cell_nb_idx.size());
  for (int m = 0; m < C; ++m) {
    const int* tm = &h.tri[3 * m];
    for (int q = h.cell_nb_ptr[m]; q < h.cell_nb_ptr[m + 1]; ++q) {
      const int n2 = h.cell_nb_idx[q];
      const int* tn = &h.tri[3 * n2];
      double val;
      if (n2 == m) {
        val = 4.5;
        for (int i = 0; i < 3; ++i) val += 1.0 / h.noc[tm[i]];
      } else {
        int shared[3], ns = 0;
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j)
            if (tm[i] == tn[j]) shared[ns++] = tm[i];
        val = ns == 2 ? 0.5 + 1.0 / h.noc[shared[0]] + 1.0 / h.noc[shared[1]] : 1.0 / h.noc[shared[0]];
      }
      e.emplace_back(m, n2, val * (2.0 / 18.0));
    }
  }
  to_csr(C, e, A);
  A.xyz = h.centroid;
}

}  // namespace rfcmp
