#include "mesh_prep.hpp"

#include <algorithm>
#include <cmath>
#include <utility>

#include "felbm.h"

namespace felbm {

namespace {
inline double unwrap(double dx, double period) { return period > 0 ? dx - period * std::nearbyint(dx / period) : dx; }

// Recursive coordinate bisection into blocks of `block` nodes.  Each split
// puts a multiple of `block` nodes on the left and takes whichever axis (x or
// y median split) cuts fewer mesh edges, so blocks come out compact in graph
// distance also on graded or anisotropic meshes.
struct Bisector {
  const std::vector<double>& x;
  const std::vector<double>& y;
  const std::vector<int32_t>& adj_ptr;
  const std::vector<int32_t>& adj;
  std::vector<int32_t>& ord;
  std::vector<int64_t> tag;
  int block;
  int64_t next_tag = 0;

  int64_t cut(int64_t lo, int64_t mid, int64_t hi, const std::vector<int32_t>& cand) {
    const int64_t tl = ++next_tag, tr = ++next_tag;
    for (int64_t k = lo; k < mid; ++k) tag[cand[k - lo]] = tl;
    for (int64_t k = mid; k < hi; ++k) tag[cand[k - lo]] = tr;
    int64_t c = 0;
    for (int64_t k = lo; k < mid; ++k) {
      const int32_t v = cand[k - lo];
      for (int32_t q = adj_ptr[v]; q < adj_ptr[v + 1]; ++q) c += tag[adj[q]] == tr;
    }
    return c;
  }

  // granularity of a split: multiples of `block` above one block, then of
  // block/4, block/16, ... inside it, down to leaves of four nodes
  void split(int64_t lo, int64_t hi) {
    const int64_t n = hi - lo;
    if (n <= 4) return;
    int64_t g = block;
    while (g > 4 && g >= n) g /= 4;
    int64_t nl = ((n / 2 + g / 2) / g) * g;
    nl = std::max<int64_t>(g, std::min<int64_t>(nl, ((n - 1) / g) * g));
    std::vector<int32_t> best, cand(ord.begin() + lo, ord.begin() + hi);
    int64_t best_cut = -1;
    for (int axis = 0; axis < 2; ++axis) {
      const std::vector<double>& c = axis == 0 ? x : y;
      std::nth_element(cand.begin(), cand.begin() + nl, cand.end(), [&](int32_t a, int32_t b) {
        return c[a] < c[b] || (c[a] == c[b] && a < b);
      });
      const int64_t ct = cut(lo, lo + nl, hi, cand);
      if (best_cut < 0 || ct < best_cut) {
        best_cut = ct;
        best = cand;
      }
    }
    std::copy(best.begin(), best.end(), ord.begin() + lo);
    split(lo, lo + nl);
    split(lo + nl, hi);
  }
};
}  // namespace

static int build_internal(int64_t n_nodes, const double* xy, int64_t n_tris, const int32_t* tri, int64_t n_wall,
                          const int32_t* wall_edge, double period_x, MeshPrep& m, std::string& err);

int prepare_mesh(int64_t n_nodes, const double* xy, int64_t n_tris, const int32_t* tri, int64_t n_wall,
                 const int32_t* wall_edge, double period_x, MeshPrep& m, std::string& err, bool reorder, int block) {
  // validate and build once in the caller's order (all messages use caller indices)
  MeshPrep v;
  int r = build_internal(n_nodes, xy, n_tris, tri, n_wall, wall_edge, period_x, v, err);
  if (r != FELBM_OK) return r;
  const int64_t N = n_nodes, E = n_tris;
  if (!reorder) {
    m = std::move(v);
    m.node_perm.resize(N);
    m.node_iperm.resize(N);
    m.elem_perm.resize(E);
    for (int64_t i = 0; i < N; ++i) m.node_perm[i] = m.node_iperm[i] = (int32_t)i;
    for (int64_t e = 0; e < E; ++e) m.elem_perm[e] = (int32_t)e;
    return FELBM_OK;
  }
  std::vector<int32_t> perm(N);
  for (int64_t i = 0; i < N; ++i) perm[i] = (int32_t)i;
  if (reorder && N > block) {
    // node graph = off-diagonal pattern of the mass matrix, from the validated build
    std::vector<int32_t> adj_ptr(N + 1, 0), adj;
    {
      std::vector<std::vector<int32_t>> nb(N);
      for (int64_t e = 0; e < E; ++e)
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b)
            if (a != b) nb[tri[3 * e + a]].push_back(tri[3 * e + b]);
      for (int64_t i = 0; i < N; ++i) {
        auto& l = nb[i];
        std::sort(l.begin(), l.end());
        l.erase(std::unique(l.begin(), l.end()), l.end());
        adj_ptr[i + 1] = adj_ptr[i] + (int32_t)l.size();
      }
      adj.reserve(adj_ptr[N]);
      for (auto& l : nb) adj.insert(adj.end(), l.begin(), l.end());
    }
    std::vector<double> xs(N), ys(N);
    for (int64_t i = 0; i < N; ++i) {
      xs[i] = xy[2 * i];
      ys[i] = xy[2 * i + 1];
    }
    Bisector bis{xs, ys, adj_ptr, adj, perm, std::vector<int64_t>(N, 0), block};
    bis.split(0, N);
    // Inside each block: the nodes with no neighbour outside the block first, then
    // the block's boundary nodes grouped by the neighbouring block they face (the
    // smallest one if several), each group in bisection order.  The halo that a
    // block reads from a neighbour is then a few contiguous index ranges, which
    // the gathers of the tiled kernels fetch in few cache lines.
    std::vector<int64_t> pos(N), face(N);
    for (int64_t k = 0; k < N; ++k) pos[perm[k]] = k;
    for (int64_t k = 0; k < N; ++k) {
      const int32_t v = perm[k];
      const int64_t b = k / block;
      int64_t f = -1;
      for (int32_t q = adj_ptr[v]; q < adj_ptr[v + 1]; ++q) {
        const int64_t bn = pos[adj[q]] / block;
        if (bn != b && (f < 0 || bn < f)) f = bn;
      }
      face[k] = f;
    }
    std::vector<int64_t> idx;
    std::vector<int32_t> tmp;
    for (int64_t lo = 0; lo < N; lo += block) {
      const int64_t hi = std::min<int64_t>(N, lo + block);
      idx.resize(hi - lo);
      for (int64_t i = 0; i < hi - lo; ++i) idx[i] = lo + i;
      std::stable_sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) { return face[a] < face[b]; });
      tmp.resize(hi - lo);
      for (int64_t i = 0; i < hi - lo; ++i) tmp[i] = perm[idx[i]];
      std::copy(tmp.begin(), tmp.end(), perm.begin() + lo);
    }
  }
  std::vector<int32_t> iperm(N);
  for (int64_t k = 0; k < N; ++k) iperm[perm[k]] = (int32_t)k;
  // triangles sorted by smallest internal vertex, then by caller index
  std::vector<int32_t> eperm(E);
  for (int64_t e = 0; e < E; ++e) eperm[e] = (int32_t)e;
  if (reorder) {
    std::vector<int32_t> key(E);
    for (int64_t e = 0; e < E; ++e)
      key[e] = std::min(iperm[tri[3 * e]], std::min(iperm[tri[3 * e + 1]], iperm[tri[3 * e + 2]]));
    std::stable_sort(eperm.begin(), eperm.end(), [&](int32_t a, int32_t b) { return key[a] < key[b]; });
  }
  std::vector<double> pxy(2 * N);
  for (int64_t k = 0; k < N; ++k) {
    pxy[2 * k] = xy[2 * perm[k]];
    pxy[2 * k + 1] = xy[2 * perm[k] + 1];
  }
  std::vector<int32_t> ptri(3 * E), pwall(2 * n_wall);
  for (int64_t e = 0; e < E; ++e)
    for (int t = 0; t < 3; ++t) ptri[3 * e + t] = iperm[tri[3 * eperm[e] + t]];
  for (int64_t w = 0; w < 2 * n_wall; ++w) pwall[w] = iperm[wall_edge[w]];
  r = build_internal(N, pxy.data(), E, ptri.data(), n_wall, pwall.data(), period_x, m, err);
  if (r != FELBM_OK) return r;
  uint64_t hsh = 1469598103934665603ull;  // FNV-1a over the node permutation
  for (int64_t k = 0; k < N; ++k) {
    hsh ^= (uint64_t)(uint32_t)perm[k];
    hsh *= 1099511628211ull;
  }
  m.node_perm = std::move(perm);
  m.node_iperm = std::move(iperm);
  m.elem_perm = std::move(eperm);
  m.perm_hash = hsh;
  return FELBM_OK;
}

static int build_internal(int64_t n_nodes, const double* xy, int64_t n_tris, const int32_t* tri, int64_t n_wall,
                          const int32_t* wall_edge, double period_x, MeshPrep& m, std::string& err) {
  if (n_nodes <= 0 || n_tris <= 0 || n_wall < 0 || !xy || !tri || (n_wall > 0 && !wall_edge)) {
    err = "upload_mesh: null pointer or non-positive size";
    return FELBM_EINVAL;
  }
  if (n_nodes > (int64_t(1) << 30) || n_tris > (int64_t(1) << 29)) {
    err = "upload_mesh: mesh too large for 32-bit indices";
    return FELBM_EINVAL;
  }
  if (!(period_x >= 0.0) || !std::isfinite(period_x)) {
    err = "upload_mesh: period_x must be finite and >= 0";
    return FELBM_EINVAL;
  }
  const int64_t N = n_nodes, E = n_tris;
  m.N = N;
  m.Np = (N + 63) / 64 * 64;
  m.E = E;
  m.W = n_wall;
  m.period_x = period_x;
  m.xy.assign(2 * N, 0.0);
  for (int64_t i = 0; i < N; ++i) {
    if (!std::isfinite(xy[2 * i]) || !std::isfinite(xy[2 * i + 1])) {
      err = "upload_mesh: non-finite coordinate at node " + std::to_string(i);
      return FELBM_EINVAL;
    }
    m.xy[i] = xy[2 * i];
    m.xy[N + i] = xy[2 * i + 1];
  }

  // triangles: index range, distinct vertices, positive unwrapped area, geometry
  m.tri.assign(3 * E, 0);
  m.geo.assign(7 * E, 0.0);
  for (int64_t e = 0; e < E; ++e) {
    int32_t v[3];
    for (int t = 0; t < 3; ++t) {
      v[t] = tri[3 * e + t];
      if (v[t] < 0 || v[t] >= N) {
        err = "upload_mesh: triangle " + std::to_string(e) + " has a vertex index out of range";
        return FELBM_EMESH;
      }
      m.tri[t * E + e] = v[t];
    }
    if (v[0] == v[1] || v[1] == v[2] || v[0] == v[2]) {
      err = "upload_mesh: triangle " + std::to_string(e) + " repeats a vertex";
      return FELBM_EMESH;
    }
    const double x0 = xy[2 * v[0]], y0 = xy[2 * v[0] + 1];
    const double x1 = x0 + unwrap(xy[2 * v[1]] - x0, period_x), y1 = xy[2 * v[1] + 1];
    const double x2 = x0 + unwrap(xy[2 * v[2]] - x0, period_x), y2 = xy[2 * v[2] + 1];
    const double twoA = (x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0);
    if (!(twoA > 0.0)) {
      err = "upload_mesh: triangle " + std::to_string(e) + " has non-positive area (must be counter-clockwise)";
      return FELBM_EMESH;
    }
    // gradients of the barycentric shape functions: grad N_t = perp(opposite edge) / 2A
    m.geo[e] = 0.5 * twoA;
    m.geo[1 * E + e] = (y1 - y2) / twoA;
    m.geo[2 * E + e] = (x2 - x1) / twoA;
    m.geo[3 * E + e] = (y2 - y0) / twoA;
    m.geo[4 * E + e] = (x0 - x2) / twoA;
    m.geo[5 * E + e] = (y0 - y1) / twoA;
    m.geo[6 * E + e] = (x1 - x0) / twoA;
  }

  // edges: sort (min, max, element, local vertex opposite the edge)
  struct EdgeRec {
    int64_t key;
    int32_t e;
    int32_t l;
  };
  std::vector<EdgeRec> edges(3 * E);
  for (int64_t e = 0; e < E; ++e)
    for (int l = 0; l < 3; ++l) {
      const int64_t a = m.tri[((l + 1) % 3) * E + e], b = m.tri[((l + 2) % 3) * E + e];
      edges[3 * e + l] = {std::min(a, b) * N + std::max(a, b), (int32_t)e, (int32_t)l};
    }
  std::sort(edges.begin(), edges.end(), [](const EdgeRec& p, const EdgeRec& q) {
    return p.key < q.key || (p.key == q.key && (p.e < q.e || (p.e == q.e && p.l < q.l)));
  });
  std::vector<int64_t> wkeys(n_wall);
  for (int64_t w = 0; w < n_wall; ++w) {
    const int64_t a = wall_edge[2 * w], b = wall_edge[2 * w + 1];
    if (a < 0 || a >= N || b < 0 || b >= N || a == b) {
      err = "upload_mesh: wall edge " + std::to_string(w) + " has an invalid node index";
      return FELBM_EMESH;
    }
    wkeys[w] = std::min(a, b) * N + std::max(a, b);
  }
  std::vector<int64_t> wsorted = wkeys;
  std::sort(wsorted.begin(), wsorted.end());
  if (std::adjacent_find(wsorted.begin(), wsorted.end()) != wsorted.end()) {
    err = "upload_mesh: duplicate wall edge";
    return FELBM_EMESH;
  }
  m.enbr.assign(3 * E, -1);
  int64_t boundary_edges = 0;
  for (size_t s = 0; s < edges.size();) {
    size_t t = s;
    while (t < edges.size() && edges[t].key == edges[s].key) ++t;
    const size_t cnt = t - s;
    const bool is_wall = std::binary_search(wsorted.begin(), wsorted.end(), edges[s].key);
    if (cnt > 2) {
      err = "upload_mesh: non-manifold edge shared by more than two triangles";
      return FELBM_EMESH;
    }
    if (cnt == 2) {
      if (is_wall) {
        err = "upload_mesh: a wall edge is shared by two triangles (not on the boundary)";
        return FELBM_EMESH;
      }
      m.enbr[edges[s].l * E + edges[s].e] = edges[s + 1].e;
      m.enbr[edges[s + 1].l * E + edges[s + 1].e] = edges[s].e;
    } else {
      if (!is_wall) {
        err = "upload_mesh: boundary edge that is neither a wall nor periodic";
        return FELBM_EMESH;
      }
      ++boundary_edges;
    }
    s = t;
  }
  if (boundary_edges != n_wall) {
    err = "upload_mesh: a wall edge is not an edge of any triangle";
    return FELBM_EMESH;
  }

  // node -> element gather lists (sorted by element), lumped mass
  m.n2e_ptr.assign(N + 1, 0);
  for (int64_t e = 0; e < E; ++e)
    for (int l = 0; l < 3; ++l) m.n2e_ptr[m.tri[l * E + e] + 1]++;
  for (int64_t i = 0; i < N; ++i) m.n2e_ptr[i + 1] += m.n2e_ptr[i];
  m.n2e.assign(3 * E, 0);
  {
    std::vector<int32_t> fill(m.n2e_ptr.begin(), m.n2e_ptr.end() - 1);
    for (int64_t e = 0; e < E; ++e)
      for (int l = 0; l < 3; ++l) m.n2e[fill[m.tri[l * E + e]]++] = (int32_t)(e * 4 + l);
  }
  m.mass.assign(N, 0.0);
  for (int64_t i = 0; i < N; ++i) {
    if (m.n2e_ptr[i + 1] == m.n2e_ptr[i]) {
      err = "upload_mesh: node " + std::to_string(i) + " belongs to no triangle";
      return FELBM_EMESH;
    }
    for (int q = m.n2e_ptr[i]; q < m.n2e_ptr[i + 1]; ++q) m.mass[i] += m.geo[m.n2e[q] >> 2] / 3.0;
  }

  // wall adjacency per node (at most two wall edges per node)
  m.wall_nbr.assign(2 * N, -1);
  m.wall_len.assign(2 * N, 0.0);
  m.is_wall.assign(N, 0);
  for (int64_t w = 0; w < n_wall; ++w) {
    const int32_t a = wall_edge[2 * w], b = wall_edge[2 * w + 1];
    const double dx = unwrap(xy[2 * b] - xy[2 * a], period_x), dy = xy[2 * b + 1] - xy[2 * a + 1];
    const double len = std::sqrt(dx * dx + dy * dy);
    for (int side = 0; side < 2; ++side) {
      const int32_t me = side ? b : a, other = side ? a : b;
      int slot = m.wall_nbr[me] < 0 ? 0 : (m.wall_nbr[N + me] < 0 ? 1 : -1);
      if (slot < 0) {
        err = "upload_mesh: node " + std::to_string(me) + " has more than two wall edges";
        return FELBM_EMESH;
      }
      m.wall_nbr[slot * N + me] = other;
      m.wall_len[slot * N + me] = len;
      m.is_wall[me] = 1;
    }
  }

  // consistent mass matrix rows: M11_ij = sum over shared triangles of A/12,
  // scaled by 1/m_i; the diagonal M11_ii / m_i = 1/2 is implicit
  std::vector<std::vector<std::pair<int32_t, double>>> rows(N);
  int64_t maxdeg = 0;
  for (int64_t i = 0; i < N; ++i) {
    auto& r = rows[i];
    for (int q = m.n2e_ptr[i]; q < m.n2e_ptr[i + 1]; ++q) {
      const int e = m.n2e[q] >> 2;
      for (int t = 0; t < 3; ++t) {
        const int32_t j = m.tri[t * E + e];
        if (j == i) continue;
        r.emplace_back(j, m.geo[e] / 12.0);
      }
    }
    std::sort(r.begin(), r.end(), [](auto& p, auto& q) { return p.first < q.first; });
    size_t o = 0;
    for (size_t s = 0; s < r.size(); ++s) {
      if (o > 0 && r[o - 1].first == r[s].first)
        r[o - 1].second += r[s].second;
      else
        r[o++] = r[s];
    }
    r.resize(o);
    for (auto& p : r) p.second /= m.mass[i];
    m.offdiag_nnz += (int64_t)o;
    maxdeg = std::max<int64_t>(maxdeg, (int64_t)o);
  }
  m.csr_ptr.assign(N + 1, 0);
  for (int64_t i = 0; i < N; ++i) m.csr_ptr[i + 1] = m.csr_ptr[i] + (int32_t)rows[i].size();
  m.csr_col.resize(m.csr_ptr[N]);
  m.csr_val.resize(m.csr_ptr[N]);
  for (int64_t i = 0; i < N; ++i)
    for (size_t k = 0; k < rows[i].size(); ++k) {
      m.csr_col[m.csr_ptr[i] + k] = rows[i][k].first;
      m.csr_val[m.csr_ptr[i] + k] = rows[i][k].second;
    }
  const int64_t nslices = m.Np / 64;
  m.sell_ptr.assign(nslices + 1, 0);
  for (int64_t s = 0; s < nslices; ++s) {
    int64_t w = 0;
    for (int64_t i = s * 64; i < std::min<int64_t>(N, s * 64 + 64); ++i) w = std::max<int64_t>(w, rows[i].size());
    m.sell_ptr[s + 1] = (int32_t)(m.sell_ptr[s] + w * 64);
  }
  m.sell_col.assign(m.sell_ptr[nslices], 0);
  m.sell_val.assign(m.sell_ptr[nslices], 0.0);
  for (int64_t s = 0; s < nslices; ++s) {
    const int64_t base = m.sell_ptr[s], w = (m.sell_ptr[s + 1] - base) / 64;
    for (int lane = 0; lane < 64; ++lane) {
      const int64_t i = s * 64 + lane;
      for (int64_t k = 0; k < w; ++k) {
        const int64_t idx = base + k * 64 + lane;
        if (i < N && k < (int64_t)rows[i].size()) {
          m.sell_col[idx] = rows[i][k].first;
          m.sell_val[idx] = rows[i][k].second;
        } else {
          m.sell_col[idx] = (int32_t)std::min<int64_t>(i, N - 1);  // padding: zero weight on a valid node
          m.sell_val[idx] = 0.0;
        }
      }
    }
  }
  (void)maxdeg;
  return FELBM_OK;
}

}  // namespace felbm
