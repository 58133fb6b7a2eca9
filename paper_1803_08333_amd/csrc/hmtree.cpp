// Cluster tree and block partition of the compressed EFIE blocks (host).
// See hmat.h for the rules.
#include "hmat.h"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace rfcmp {
namespace {

struct Builder {
  const MeshHost& h;
  HmTree& t;
  std::vector<int> order;          // edges in the permuted order (built in place)
  std::vector<double> mid;         // [N][3] edge midpoints
  std::vector<double> slo, shi;    // [N][3] support boxes (both cells' vertices)

  Builder(const MeshHost& hh, HmTree& tt) : h(hh), t(tt) {}

  // node over order[s, e); returns its index
  int split(int64_t s, int64_t e) {
    const int id = (int)t.nodes.size();
    t.nodes.emplace_back();
    HmNode nd;
    nd.e0 = s;
    nd.e1 = e;
    nd.t0 = (int)(s / kEdgeTile);
    nd.t1 = (int)((e + kEdgeTile - 1) / kEdgeTile);
    const int64_t n = e - s;
    if (n > kEdgeTile) {
      double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
      for (int64_t p = s; p < e; ++p)
        for (int d = 0; d < 3; ++d) {
          lo[d] = std::min(lo[d], mid[3 * order[p] + d]);
          hi[d] = std::max(hi[d], mid[3 * order[p] + d]);
        }
      int ax = 0;
      for (int d = 1; d < 3; ++d)
        if (hi[d] - lo[d] > hi[ax] - lo[ax]) ax = d;
      std::sort(order.begin() + s, order.begin() + e, [&](int a, int b) {
        const double xa = mid[3 * a + ax], xb = mid[3 * b + ax];
        return xa < xb || (xa == xb && a < b);
      });
      // the first part takes a multiple of the tile size, so that every
      // leaf but the last is a whole tile
      int64_t n1 = (int64_t)kEdgeTile * std::max<int64_t>(1, std::llround((double)n / (2.0 * kEdgeTile)));
      n1 = std::min(n1, n - 1);
      const int c0 = split(s, s + n1);
      const int c1 = split(s + n1, e);
      nd.child[0] = c0;
      nd.child[1] = c1;
    }
    t.nodes[id] = nd;
    return id;
  }
};

double box_distance(const HmNode& a, const HmNode& b) {
  double s = 0.0;
  for (int d = 0; d < 3; ++d) {
    const double g = std::max(0.0, std::max(a.lo[d] - b.hi[d], b.lo[d] - a.hi[d]));
    s += g * g;
  }
  return std::sqrt(s);
}

double diam(const HmNode& a) {
  double s = 0.0;
  for (int d = 0; d < 3; ++d) s += (a.hi[d] - a.lo[d]) * (a.hi[d] - a.lo[d]);
  return std::sqrt(s);
}

void partition(HmTree& t, int a, int b) {
  const HmNode& A = t.nodes[a];
  const HmNode& B = t.nodes[b];
  const bool la = A.child[0] < 0, lb = B.child[0] < 0;
  if (a == b) {
    if (la) {
      t.dense_I.push_back(A.t0);
      t.dense_J.push_back(A.t0);
      return;
    }
    const int c0 = A.child[0], c1 = A.child[1];
    partition(t, c0, c0);
    partition(t, c0, c1);
    partition(t, c1, c1);
    return;
  }
  const double d = box_distance(A, B);
  if (d >= t.near_dist && std::min(diam(A), diam(B)) <= kHmEta * d) {
    t.lr_a.push_back(a);
    t.lr_b.push_back(b);
    return;
  }
  if (la && lb) {
    t.dense_I.push_back(A.t0);
    t.dense_J.push_back(B.t0);
    return;
  }
  if (la) {
    for (int c : B.child) partition(t, a, c);
    return;
  }
  if (lb) {
    for (int c : A.child) partition(t, c, b);
    return;
  }
  for (int ca : A.child)
    for (int cb : B.child) partition(t, ca, cb);
}

}  // namespace

void hm_build_tree(const MeshHost& h, HmTree& t) {
  const int64_t N = h.N, C = h.C;
  t = HmTree{};
  t.N = N;
  t.C = C;
  t.ntiles = (N + kEdgeTile - 1) / kEdgeTile;
  Builder b(h, t);
  b.mid.resize(3 * N);
  b.slo.resize(3 * N);
  b.shi.resize(3 * N);
  for (int64_t e = 0; e < N; ++e) {
    const int v0 = h.edge_vtx[2 * e], v1 = h.edge_vtx[2 * e + 1];
    for (int d = 0; d < 3; ++d) {
      b.mid[3 * e + d] = 0.5 * (h.xyz[3 * v0 + d] + h.xyz[3 * v1 + d]);
      b.slo[3 * e + d] = 1e300;
      b.shi[3 * e + d] = -1e300;
    }
    for (int k = 0; k < 2; ++k) {
      const int c = h.edge_cell[2 * e + k];
      for (int i = 0; i < 3; ++i) {
        const int v = h.tri[3 * c + i];
        for (int d = 0; d < 3; ++d) {
          b.slo[3 * e + d] = std::min(b.slo[3 * e + d], h.xyz[3 * v + d]);
          b.shi[3 * e + d] = std::max(b.shi[3 * e + d], h.xyz[3 * v + d]);
        }
      }
    }
  }
  b.order.resize(N);
  std::iota(b.order.begin(), b.order.end(), 0);
  t.nodes.reserve(4 * t.ntiles + 4);
  if (N > 0) b.split(0, N);
  t.perm_e = b.order;
  t.iperm_e.assign(N, 0);
  for (int64_t p = 0; p < N; ++p) t.iperm_e[t.perm_e[p]] = (int)p;

  // home tiles and the cell order
  t.home.assign(C, 0);
  for (int64_t c = 0; c < C; ++c) {
    int p = (int)N;
    for (int i = 0; i < 3; ++i) p = std::min(p, t.iperm_e[h.cell_edge[3 * c + i]]);
    t.home[c] = p / kEdgeTile;
  }
  t.perm_c.resize(C);
  std::iota(t.perm_c.begin(), t.perm_c.end(), 0);
  std::stable_sort(t.perm_c.begin(), t.perm_c.end(), [&](int a, int c) { return t.home[a] < t.home[c]; });
  t.iperm_c.assign(C, 0);
  for (int64_t p = 0; p < C; ++p) t.iperm_c[t.perm_c[p]] = (int)p;
  t.cell_start.assign(t.ntiles + 1, 0);
  for (int64_t c = 0; c < C; ++c) ++t.cell_start[t.home[c] + 1];
  for (int64_t q = 0; q < t.ntiles; ++q) t.cell_start[q + 1] += t.cell_start[q];

  // node boxes (children first: nodes are numbered in preorder) and cell ranges
  for (int64_t q = (int64_t)t.nodes.size() - 1; q >= 0; --q) {
    HmNode& nd = t.nodes[q];
    nd.c0 = t.cell_start[nd.t0];
    nd.c1 = t.cell_start[nd.t1];
    for (int d = 0; d < 3; ++d) {
      nd.lo[d] = 1e300;
      nd.hi[d] = -1e300;
    }
    if (nd.child[0] < 0) {
      for (int64_t p = nd.e0; p < nd.e1; ++p) {
        const int e = t.perm_e[p];
        for (int d = 0; d < 3; ++d) {
          nd.lo[d] = std::min(nd.lo[d], b.slo[3 * e + d]);
          nd.hi[d] = std::max(nd.hi[d], b.shi[3 * e + d]);
        }
      }
    } else {
      for (int c : nd.child)
        for (int d = 0; d < 3; ++d) {
          nd.lo[d] = std::min(nd.lo[d], t.nodes[c].lo[d]);
          nd.hi[d] = std::max(nd.hi[d], t.nodes[c].hi[d]);
        }
    }
  }

  // the tiles as the assembly reads them
  t.et_ptr.assign(t.ntiles + 1, 0);
  t.et_cell.clear();
  t.et_rows.clear();
  t.et_cells_max = 0;
  std::vector<int> cells;
  for (int64_t q = 0; q < t.ntiles; ++q) {
    cells.clear();
    for (int64_t p = q * kEdgeTile; p < std::min<int64_t>(N, (q + 1) * kEdgeTile); ++p)
      for (int k = 0; k < 2; ++k) cells.push_back(h.edge_cell[2 * t.perm_e[p] + k]);
    std::sort(cells.begin(), cells.end());
    cells.erase(std::unique(cells.begin(), cells.end()), cells.end());
    for (int c : cells) {
      int r3 = 0;
      for (int i = 0; i < 3; ++i) {
        const int p = t.iperm_e[h.cell_edge[3 * c + i]];
        const int r = (p / kEdgeTile == q) ? p % kEdgeTile : 0xFF;
        r3 |= r << (8 * i);
      }
      t.et_cell.push_back(c);
      t.et_rows.push_back(r3);
    }
    t.et_ptr[q + 1] = (int)t.et_cell.size();
    t.et_cells_max = std::max(t.et_cells_max, (int)cells.size());
  }

  double hm = 0.0;
  for (int64_t c = 0; c < C; ++c) hm = std::max(hm, h.hmax[c]);
  t.near_dist = 2.0 * hm * (1.0 + 1e-9);
  if (N > 0) partition(t, 0, 0);
  // low-rank blocks largest first (by rows + columns, then in partition
  // order), so that the ACA of the largest blocks starts first
  std::vector<int> ord(t.lr_a.size());
  std::iota(ord.begin(), ord.end(), 0);
  auto size = [&](int b) {
    const HmNode& A = t.nodes[t.lr_a[b]];
    const HmNode& B = t.nodes[t.lr_b[b]];
    return (A.e1 - A.e0) + (B.e1 - B.e0);
  };
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return size(a) > size(b); });
  std::vector<int> la(ord.size()), lb(ord.size());
  for (size_t q = 0; q < ord.size(); ++q) {
    la[q] = t.lr_a[ord[q]];
    lb[q] = t.lr_b[ord[q]];
  }
  t.lr_a.swap(la);
  t.lr_b.swap(lb);
}

}  // namespace rfcmp
