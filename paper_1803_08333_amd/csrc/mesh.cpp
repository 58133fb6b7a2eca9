// Host topology of a closed triangle mesh: RWG edges, star/loop incidence,
// validation and the near-pair list of the quadrature spec.
//
// RWG functions (Sec. 2, eq. RWGdef) live on the interior edges; on a closed
// mesh every edge is one RWG.  Edge order, c+/c- and the signs of Sigma and
// Lambda follow the convention stated in rfcmp.h.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <system_error>
#include <thread>

#include "internal.h"

namespace rfcmp {

namespace {
thread_local std::string g_err;
}

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
}
void clear_error() { g_err.clear(); }
const char* last_error() { return g_err.c_str(); }

static rfcmp_status fail(rfcmp_status s, const char* msg, long long a = -1) {
  if (a >= 0)
    set_error("%s (index %lld)", msg, a);
  else
    set_error("%s", msg);
  return s;
}

rfcmp_status build_mesh_host(const double* xyz, int64_t nv, const int32_t* tri, int64_t nc,
                             MeshHost& h) {
  if (!xyz || !tri || nv < 4 || nc < 4) return fail(RFCMP_E_ARG, "mesh needs >= 4 vertices and cells");
  if (nc > (int64_t(1) << 30) || nv > (int64_t(1) << 30)) return fail(RFCMP_E_ARG, "mesh too large");
  for (int64_t i = 0; i < 3 * nv; ++i)
    if (!std::isfinite(xyz[i])) return fail(RFCMP_E_ARG, "non-finite vertex coordinate", i / 3);
  h = MeshHost{};
  h.V = nv;
  h.C = nc;
  h.xyz.assign(xyz, xyz + 3 * nv);
  h.tri.assign(tri, tri + 3 * nc);
  for (int64_t c = 0; c < nc; ++c) {
    const int32_t* t = &tri[3 * c];
    for (int i = 0; i < 3; ++i)
      if (t[i] < 0 || t[i] >= nv) return fail(RFCMP_E_MESH_NONMANIFOLD, "cell vertex out of range", c);
    if (t[0] == t[1] || t[1] == t[2] || t[0] == t[2])
      return fail(RFCMP_E_MESH_NONMANIFOLD, "cell with a repeated vertex", c);
  }

  // directed half-edges: local edge i of cell c runs from vertex i+1 to i+2
  struct Half {
    int64_t key;  // min*nv + max
    int32_t cell;
    int8_t local;
    int8_t forward;  // 1 if walked min -> max
  };
  std::vector<Half> he(3 * nc);
  for (int64_t c = 0; c < nc; ++c)
    for (int i = 0; i < 3; ++i) {
      int32_t a = tri[3 * c + (i + 1) % 3], b = tri[3 * c + (i + 2) % 3];
      int32_t lo = std::min(a, b), hi = std::max(a, b);
      he[3 * c + i] = Half{int64_t(lo) * nv + hi, int32_t(c), int8_t(i), int8_t(a < b)};
    }
  // order by (key, forward first): a counting sort on the lower vertex, then
  // an insertion sort inside each vertex's few half-edges (the same order
  // as a comparison sort on that key)
  {
    std::vector<int32_t> off(nv + 1, 0);
    for (int64_t c = 0; c < nc; ++c)
      for (int i = 0; i < 3; ++i) {
        const int32_t a = tri[3 * c + (i + 1) % 3], b = tri[3 * c + (i + 2) % 3];
        ++off[std::min(a, b) + 1];
      }
    for (int64_t v = 0; v < nv; ++v) off[v + 1] += off[v];
    std::vector<Half> hs(he.size());
    {
      std::vector<int32_t> fill(off.begin(), off.end() - 1);
      for (const Half& x : he) hs[fill[x.key / nv]++] = x;
    }
    auto before = [](const Half& x, const Half& y) {
      return x.key < y.key || (x.key == y.key && x.forward > y.forward);
    };
    for (int64_t v = 0; v < nv; ++v)
      for (int32_t i = off[v] + 1; i < off[v + 1]; ++i) {
        const Half x = hs[i];
        int32_t j = i - 1;
        while (j >= off[v] && before(x, hs[j])) {
          hs[j + 1] = hs[j];
          --j;
        }
        hs[j + 1] = x;
      }
    he.swap(hs);
  }
  // every undirected edge must appear exactly twice, once per direction
  std::vector<int64_t> starts;
  for (size_t i = 0; i < he.size();) {
    size_t j = i;
    while (j < he.size() && he[j].key == he[i].key) ++j;
    if (j - i == 1) return fail(RFCMP_E_MESH_OPEN, "open edge (one cell)", he[i].cell);
    if (j - i > 2) return fail(RFCMP_E_MESH_NONMANIFOLD, "edge shared by more than two cells", he[i].cell);
    if (he[i].forward != 1 || he[i + 1].forward != 0)
      return fail(RFCMP_E_MESH_ORIENT, "two cells walk an edge in the same direction", he[i].cell);
    starts.push_back(int64_t(i));
    i = j;
  }
  const int64_t N = int64_t(starts.size());
  // number the edges in the order a scan over the cells (and their local
  // edges) first meets them, so that the edges of nearby cells sit together
  std::vector<int32_t> order(N);
  {
    std::vector<int32_t> of_half(3 * nc);  // key-ordered edge of each (cell, local)
    for (int64_t k = 0; k < N; ++k)
      for (int e = 0; e < 2; ++e) {
        const Half& x = he[starts[k] + e];
        of_half[3 * int64_t(x.cell) + x.local] = int32_t(k);
      }
    std::vector<int32_t> id(N, -1);
    int32_t next = 0;
    for (int64_t hc = 0; hc < 3 * nc; ++hc)
      if (id[of_half[hc]] < 0) {
        id[of_half[hc]] = next;
        order[next++] = of_half[hc];
      }
  }
  h.N = N;
  h.edge_vtx.resize(2 * N);
  h.edge_cell.resize(2 * N);
  h.edge_local.resize(2 * N);
  h.cell_edge.assign(3 * nc, -1);
  h.cell_sign.assign(3 * nc, 0);
  for (int64_t n = 0; n < N; ++n) {
    const Half& p = he[starts[order[n]]];      // walked min -> max: c+
    const Half& q = he[starts[order[n]] + 1];  // c-
    h.edge_vtx[2 * n] = int32_t(p.key / nv);
    h.edge_vtx[2 * n + 1] = int32_t(p.key % nv);
    h.edge_cell[2 * n] = p.cell;
    h.edge_cell[2 * n + 1] = q.cell;
    h.edge_local[2 * n] = p.local;
    h.edge_local[2 * n + 1] = q.local;
    h.cell_edge[3 * p.cell + p.local] = int32_t(n);
    h.cell_sign[3 * p.cell + p.local] = 1;
    h.cell_edge[3 * q.cell + q.local] = int32_t(n);
    h.cell_sign[3 * q.cell + q.local] = -1;
  }

  // geometry
  h.area.resize(nc);
  h.centroid.resize(3 * nc);
  h.hmax.resize(nc);
  for (int64_t c = 0; c < nc; ++c) {
    const double* P[3] = {&xyz[3 * tri[3 * c]], &xyz[3 * tri[3 * c + 1]], &xyz[3 * tri[3 * c + 2]]};
    double u[3], v[3], w[3];
    for (int d = 0; d < 3; ++d) {
      u[d] = P[1][d] - P[0][d];
      v[d] = P[2][d] - P[0][d];
    }
    w[0] = u[1] * v[2] - u[2] * v[1];
    w[1] = u[2] * v[0] - u[0] * v[2];
    w[2] = u[0] * v[1] - u[1] * v[0];
    double a2 = std::sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    double hm = 0;
    for (int i = 0; i < 3; ++i) {
      const double* A = P[(i + 1) % 3];
      const double* B = P[(i + 2) % 3];
      double e2 = 0;
      for (int d = 0; d < 3; ++d) e2 += (B[d] - A[d]) * (B[d] - A[d]);
      hm = std::max(hm, std::sqrt(e2));
    }
    if (!(a2 > 1e-14 * hm * hm)) return fail(RFCMP_E_MESH_DEGENERATE, "zero-area cell", c);
    h.area[c] = 0.5 * a2;
    h.hmax[c] = hm;
    for (int d = 0; d < 3; ++d) h.centroid[3 * c + d] = (P[0][d] + P[1][d] + P[2][d]) / 3.0;
  }

  // cells at each vertex, fan check (one cycle of cells around every vertex)
  h.noc.assign(nv, 0);
  for (int64_t i = 0; i < 3 * nc; ++i) h.noc[tri[i]]++;
  for (int64_t v = 0; v < nv; ++v)
    if (h.noc[v] == 0) return fail(RFCMP_E_MESH_DISCONNECTED, "vertex used by no cell", v);
  std::vector<int32_t> vc_ptr(nv + 1, 0), vc_idx(3 * nc);
  for (int64_t v = 0; v < nv; ++v) vc_ptr[v + 1] = vc_ptr[v] + h.noc[v];
  {
    std::vector<int32_t> fill(vc_ptr.begin(), vc_ptr.end() - 1);
    for (int64_t c = 0; c < nc; ++c)
      for (int i = 0; i < 3; ++i) vc_idx[fill[tri[3 * c + i]]++] = int32_t(c);
  }
  // around vertex v, cell c with v at local position i: the next cell across
  // the edge (v, vertex i+1) is the other cell of that edge
  for (int64_t v = 0; v < nv; ++v) {
    int32_t c0 = vc_idx[vc_ptr[v]], c = c0;
    int count = 0;
    do {
      int i = 0;
      while (tri[3 * c + i] != v) ++i;
      // local edge opposite vertex i+2 joins v and vertex i+1
      int32_t e = h.cell_edge[3 * c + (i + 2) % 3];
      c = h.edge_cell[2 * e] == c ? h.edge_cell[2 * e + 1] : h.edge_cell[2 * e];
      if (++count > h.noc[v]) break;
    } while (c != c0);
    if (count != h.noc[v]) return fail(RFCMP_E_MESH_NONMANIFOLD, "vertex with more than one fan", v);
  }

  // connectivity over edges
  {
    std::vector<char> seen(nc, 0);
    std::vector<int32_t> stack{0};
    seen[0] = 1;
    int64_t reached = 1;
    while (!stack.empty()) {
      int32_t c = stack.back();
      stack.pop_back();
      for (int i = 0; i < 3; ++i) {
        int32_t e = h.cell_edge[3 * c + i];
        int32_t o = h.edge_cell[2 * e] == c ? h.edge_cell[2 * e + 1] : h.edge_cell[2 * e];
        if (!seen[o]) {
          seen[o] = 1;
          ++reached;
          stack.push_back(o);
        }
      }
    }
    if (reached != nc) return fail(RFCMP_E_MESH_DISCONNECTED, "mesh has more than one component");
  }
  const int64_t chi = nv - N + nc;
  if ((2 - chi) % 2 != 0 || chi > 2) return fail(RFCMP_E_MESH_NONMANIFOLD, "odd Euler characteristic");
  h.genus = int32_t((2 - chi) / 2);

  // Lambda^T as CSR over vertices: Lambda[n, min] = +1, Lambda[n, max] = -1
  h.vtx_edge_ptr.assign(nv + 1, 0);
  for (int64_t n = 0; n < N; ++n) {
    h.vtx_edge_ptr[h.edge_vtx[2 * n] + 1]++;
    h.vtx_edge_ptr[h.edge_vtx[2 * n + 1] + 1]++;
  }
  for (int64_t v = 0; v < nv; ++v) h.vtx_edge_ptr[v + 1] += h.vtx_edge_ptr[v];
  h.vtx_edge_idx.resize(2 * N);
  h.vtx_edge_sgn.resize(2 * N);
  {
    std::vector<int32_t> fill(h.vtx_edge_ptr.begin(), h.vtx_edge_ptr.end() - 1);
    for (int64_t n = 0; n < N; ++n) {
      int32_t a = h.edge_vtx[2 * n], b = h.edge_vtx[2 * n + 1];
      h.vtx_edge_idx[fill[a]] = int32_t(n);
      h.vtx_edge_sgn[fill[a]++] = 1;
      h.vtx_edge_idx[fill[b]] = int32_t(n);
      h.vtx_edge_sgn[fill[b]++] = -1;
    }
  }

  return RFCMP_OK;
}

// Cells sharing at least one vertex with each cell (for the mixed Gram
// matrix), built on first use.
void build_cell_nb(MeshHost& h) {
  if (!h.cell_nb_ptr.empty()) return;
  const int64_t nv = h.V, nc = h.C;
  const int32_t* tri = h.tri.data();
  std::vector<int32_t> vc_ptr(nv + 1, 0), vc_idx(3 * nc);
  for (int64_t v = 0; v < nv; ++v) vc_ptr[v + 1] = vc_ptr[v] + h.noc[v];
  {
    std::vector<int32_t> fill(vc_ptr.begin(), vc_ptr.end() - 1);
    for (int64_t c = 0; c < nc; ++c)
      for (int i = 0; i < 3; ++i) vc_idx[fill[tri[3 * c + i]]++] = int32_t(c);
  }
  h.cell_nb_ptr.assign(nc + 1, 0);
  h.cell_nb_idx.clear();
  std::vector<int32_t> nb;
  for (int64_t c = 0; c < nc; ++c) {
    nb.clear();
    for (int i = 0; i < 3; ++i) {
      int32_t v = tri[3 * c + i];
      for (int32_t k = vc_ptr[v]; k < vc_ptr[v + 1]; ++k) nb.push_back(vc_idx[k]);
    }
    std::sort(nb.begin(), nb.end());
    nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
    h.cell_nb_idx.insert(h.cell_nb_idx.end(), nb.begin(), nb.end());
    h.cell_nb_ptr[c + 1] = int32_t(h.cell_nb_idx.size());
  }
}

// Near pairs c <= c': |x_c - x_c'| < factor * max(h_c, h_c') * (1 + 1e-9),
// found through a uniform grid of bins of the largest possible threshold.
void near_pairs(const MeshHost& h, double factor, std::vector<int32_t>& out) {
  out.clear();
  const int64_t C = h.C;
  if (C == 0) return;
  double hm = 0;
  for (double x : h.hmax) hm = std::max(hm, x);
  // uniform grid of bins no smaller than the largest threshold: every near
  // pair lies in the same or an adjacent bin
  double bin = factor * hm * (1.0 + 1e-9);
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t c = 0; c < C; ++c)
    for (int d = 0; d < 3; ++d) {
      lo[d] = std::min(lo[d], h.centroid[3 * c + d]);
      hi[d] = std::max(hi[d], h.centroid[3 * c + d]);
    }
  // larger bins (never smaller ones) keep the grid within about 8 bins per cell
  int64_t nb[3];
  for (;;) {
    for (int d = 0; d < 3; ++d) nb[d] = int64_t((hi[d] - lo[d]) / bin) + 1;
    if ((double)nb[0] * (double)nb[1] * (double)nb[2] <= 8.0 * double(C) + 64.0) break;
    bin *= 1.25;
  }
  auto coord = [&](int64_t c, int d) {
    return std::min<int64_t>(int64_t((h.centroid[3 * c + d] - lo[d]) / bin), nb[d] - 1);
  };
  const int64_t nbins = nb[0] * nb[1] * nb[2];
  std::vector<int32_t> cbin(C), start(nbins + 1, 0), cells(C);
  for (int64_t c = 0; c < C; ++c) {
    cbin[c] = int32_t((coord(c, 0) * nb[1] + coord(c, 1)) * nb[2] + coord(c, 2));
    ++start[cbin[c] + 1];
  }
  for (int64_t b = 0; b < nbins; ++b) start[b + 1] += start[b];
  {
    std::vector<int32_t> fill(start.begin(), start.end() - 1);
    for (int64_t c = 0; c < C; ++c) cells[fill[cbin[c]]++] = int32_t(c);  // ascending within a bin
  }
  // cells in contiguous chunks on a few threads, each chunk's pairs in cell
  // order, concatenated in chunk order: the same list as one thread
  auto scan = [&](int64_t c0, int64_t c1, std::vector<int32_t>& res) {
    std::vector<int32_t> hit;
    for (int64_t c = c0; c < c1; ++c) {
      hit.clear();
      const int64_t b = cbin[c];
      const int64_t bx = b / (nb[1] * nb[2]), by = (b / nb[2]) % nb[1], bz = b % nb[2];
      const double* pc = &h.centroid[3 * c];
      for (int64_t x = std::max<int64_t>(bx - 1, 0); x <= std::min(bx + 1, nb[0] - 1); ++x)
        for (int64_t y = std::max<int64_t>(by - 1, 0); y <= std::min(by + 1, nb[1] - 1); ++y)
          for (int64_t z = std::max<int64_t>(bz - 1, 0); z <= std::min(bz + 1, nb[2] - 1); ++z) {
            const int64_t q = (x * nb[1] + y) * nb[2] + z;
            for (int32_t i = start[q]; i < start[q + 1]; ++i) {
              const int32_t o = cells[i];
              if (o < c) continue;
              const double* po = &h.centroid[3 * int64_t(o)];
              double d2 = 0;
              for (int d = 0; d < 3; ++d) {
                const double t = pc[d] - po[d];
                d2 += t * t;
              }
              const double thr = factor * std::max(h.hmax[c], h.hmax[o]) * (1.0 + 1e-9);
              if (std::sqrt(d2) < thr) hit.push_back(o);
            }
          }
      std::sort(hit.begin(), hit.end());
      for (int32_t o : hit) {
        res.push_back(int32_t(c));
        res.push_back(o);
      }
    }
  };
  const int64_t nthr = C >= 4096 ? std::min<int64_t>(8, std::max(1u, std::thread::hardware_concurrency())) : 1;
  std::vector<std::vector<int32_t>> part(nthr);
  std::vector<std::thread> pool;
  try {
    for (int64_t t = 1; t < nthr; ++t)
      pool.emplace_back(scan, C * t / nthr, C * (t + 1) / nthr, std::ref(part[t]));
  } catch (const std::system_error&) {
    // no threads to be had: the remaining chunks run here
    for (int64_t t = int64_t(pool.size()) + 1; t < nthr; ++t) scan(C * t / nthr, C * (t + 1) / nthr, part[t]);
  }
  scan(0, C / nthr, part[0]);
  for (auto& th : pool) th.join();
  size_t tot = 0;
  for (const auto& v : part) tot += v.size();
  out.reserve(tot);
  for (const auto& v : part) out.insert(out.end(), v.begin(), v.end());
}

}  // namespace rfcmp
