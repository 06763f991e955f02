// C ABI of the 3-D FE-LBM step (declared in include/felbm3d.h): context,
// host mesh preparation for P1 tetrahedra, the per-step launch sequence and
// the read-back / timing entry points.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "felbm3d.h"
#include "kernels3d.hpp"

using felbm::DiagRecord;
using felbm::NRED;
using felbm::RBLOCK;
using namespace felbm3d;

namespace {

enum Kernel3 { K3_MOMENTS = 0, K3_REDUCE, K3_LAPC, K3_LAPMU, K3_RHS, K3_SWEEP_FIRST, K3_SWEEP_MID, K3_SWEEP_LAST,
               K3_COUNT };
const char* const kNames3[K3_COUNT] = {"moments_collide", "reduce_final", "lapC_mu_op", "lapmu_force_op",
                                       "rhs_gather", "sweep_first", "sweep_mid", "sweep_last"};

inline int grid_for(int64_t n) {
  int64_t b = (n + BLOCK - 1) / BLOCK;
  b = (b + 7) / 8 * 8;  // multiple of 8 for the XCD remap
  return (int)std::max<int64_t>(b, 8);
}

// one thread per node and population set: a block of four 64-node slices per
// set, the g blocks in the first half of the grid and the h blocks in the second
inline int grid_sets_for(int64_t n) { return 2 * grid_for(n); }

// Host-side mesh preparation (caller order kept).
struct Prep3 {
  int64_t N = 0, Np = 0, E = 0, W = 0, nnz = 0;
  std::vector<int32_t> tet, fnbr;        // [4][E]
  std::vector<double> geo;               // [13][E]
  std::vector<int32_t> n2e_ptr, n2e;     // node -> element*4 + local vertex
  std::vector<int32_t> wf_ptr, wf_list;  // node -> wall faces containing it
  std::vector<int32_t> wface;            // [3][W]
  std::vector<double> warea;             // [W]
  std::vector<uint8_t> is_wall;
  std::vector<double> mass, pvol;
  std::vector<int32_t> sell_ptr, sell_col;
  std::vector<double> sell_val;
  // right-hand side: incident elements (alpha0 = V/m_i, beta0 = V grad N_i / m_i) and patch
  // moments (G0_ij = sum V grad N_j / m_i; S0_ij = sum V grad N_i grad N_j^T / m_i as xx, yy, zz
  // and the doubled symmetric xy, xz, yz), both in sliced ELL; dt factors applied at upload
  std::vector<int32_t> inc_ptr, inc_e, pair_ptr, pair_col;
  std::vector<double> inc_w, pair_v;  // [4][inc slots], [9][pair slots]
  // field operators: patch Laplacian of C (sliced ELL over the 2-ring, weights / V_k,
  // difference form) with the wall faces of each patch (CSR: [3][L] nodes, area / V_k),
  // and the element Laplacian of mu ([4][E] vertices across the faces, [7][E] weights)
  std::vector<int32_t> lop_ptr, lop_col, wl_ptr, wl_face, eopp;
  std::vector<double> lop_w, wl_scale, ew;
  std::vector<double> dlt;  // diagonal of the FP64 composition sweeps (FP32 form)
};

struct FaceRec {
  int32_t a, b, c;
  int64_t owner;  // element * 4 + local face (= opposite vertex); -1 - index for a listed wall face
};

bool face_less(const FaceRec& x, const FaceRec& y) {
  if (x.a != y.a) return x.a < y.a;
  if (x.b != y.b) return x.b < y.b;
  if (x.c != y.c) return x.c < y.c;
  return x.owner < y.owner;
}

FaceRec sorted_face(int32_t p, int32_t q, int32_t r, int64_t owner) {
  int32_t v[3] = {p, q, r};
  std::sort(v, v + 3);
  return FaceRec{v[0], v[1], v[2], owner};
}

int prepare3(int64_t N, const double* xyz, int64_t E, const int32_t* tet, int64_t W, const int32_t* wface,
             double px, double py, Prep3& m, std::string& err) {
  if (N < 4 || E < 1 || W < 0 || !xyz || !tet || (W > 0 && !wface)) {
    err = "upload_mesh: null array or bad size";
    return FELBM_EINVAL;
  }
  if (N > (int64_t)1 << 30 || E > ((int64_t)1 << 29)) {
    err = "upload_mesh: mesh too large for 32-bit element entries";
    return FELBM_EINVAL;
  }
  if (!(px >= 0) || !(py >= 0) || !std::isfinite(px) || !std::isfinite(py)) {
    err = "upload_mesh: periods must be finite and >= 0";
    return FELBM_EINVAL;
  }
  for (int64_t i = 0; i < 3 * N; ++i)
    if (!std::isfinite(xyz[i])) {
      err = "upload_mesh: non-finite coordinate";
      return FELBM_EINVAL;
    }
  for (int64_t q = 0; q < 4 * E; ++q)
    if (tet[q] < 0 || tet[q] >= N) {
      err = "upload_mesh: tetrahedron vertex index out of range";
      return FELBM_EMESH;
    }
  for (int64_t q = 0; q < 3 * W; ++q)
    if (wface[q] < 0 || wface[q] >= N) {
      err = "upload_mesh: wall face index out of range";
      return FELBM_EMESH;
    }
  m.N = N;
  m.Np = (N + 63) / 64 * 64;
  m.E = E;
  m.W = W;
  m.tet.assign(4 * E, 0);
  m.geo.assign(13 * E, 0.0);
  const double per[2] = {px, py};
  auto unwrap = [&](int32_t n, const double* ref, double* out) {
    for (int d = 0; d < 3; ++d) out[d] = xyz[3 * n + d];
    for (int d = 0; d < 2; ++d)
      if (per[d] > 0) out[d] -= per[d] * std::nearbyint((out[d] - ref[d]) / per[d]);
  };
  for (int64_t e = 0; e < E; ++e) {
    double p[4][3];
    for (int d = 0; d < 3; ++d) p[0][d] = xyz[3 * tet[4 * e] + d];
    for (int v = 1; v < 4; ++v) unwrap(tet[4 * e + v], p[0], p[v]);
    double J[3][3];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) J[r][c] = p[c + 1][r] - p[0][r];  // columns are the edge vectors
    const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                       J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    if (!(det > 0)) {
      err = "upload_mesh: tetrahedron " + std::to_string(e) + " has non-positive volume";
      return FELBM_EMESH;
    }
    // rows of J^-1 are the gradients of the barycentric coordinates 1..3
    double inv[3][3];
    inv[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
    inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    inv[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
    inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    inv[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
    inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    m.geo[e] = det / 6.0;
    for (int r = 0; r < 3; ++r) {
      m.geo[(1 + r) * E + e] = -(inv[0][r] + inv[1][r] + inv[2][r]);
      for (int v = 1; v < 4; ++v) m.geo[(1 + 3 * v + r) * E + e] = inv[v - 1][r];
    }
    for (int v = 0; v < 4; ++v) m.tet[v * E + e] = tet[4 * e + v];
  }
  // faces: match the 4E element faces, then the listed wall faces against the unmatched ones
  std::vector<FaceRec> f;
  f.reserve(4 * E);
  for (int64_t e = 0; e < E; ++e)
    for (int l = 0; l < 4; ++l)
      f.push_back(sorted_face(tet[4 * e + ((l + 1) & 3)], tet[4 * e + ((l + 2) & 3)], tet[4 * e + ((l + 3) & 3)], 4 * e + l));
  std::sort(f.begin(), f.end(), face_less);
  m.fnbr.assign(4 * E, -1);
  std::vector<FaceRec> boundary;
  for (size_t q = 0; q < f.size();) {
    size_t r = q + 1;
    while (r < f.size() && f[r].a == f[q].a && f[r].b == f[q].b && f[r].c == f[q].c) ++r;
    if (r - q > 2) {
      err = "upload_mesh: a face is shared by more than two tetrahedra";
      return FELBM_EMESH;
    }
    if (r - q == 2) {
      const int64_t o0 = f[q].owner, o1 = f[q + 1].owner;
      m.fnbr[(o0 & 3) * E + (o0 >> 2)] = (int32_t)(o1 >> 2);
      m.fnbr[(o1 & 3) * E + (o1 >> 2)] = (int32_t)(o0 >> 2);
    } else {
      boundary.push_back(f[q]);
    }
    q = r;
  }
  std::vector<FaceRec> wl;
  wl.reserve(W);
  for (int64_t w = 0; w < W; ++w) wl.push_back(sorted_face(wface[3 * w], wface[3 * w + 1], wface[3 * w + 2], w));
  std::sort(wl.begin(), wl.end(), face_less);
  for (size_t q = 1; q < wl.size(); ++q)
    if (wl[q].a == wl[q - 1].a && wl[q].b == wl[q - 1].b && wl[q].c == wl[q - 1].c) {
      err = "upload_mesh: a wall face is listed twice";
      return FELBM_EMESH;
    }
  if (wl.size() != boundary.size()) {
    err = "upload_mesh: " + std::to_string(boundary.size()) + " boundary faces but " + std::to_string(wl.size()) +
          " wall faces listed";
    return FELBM_EMESH;
  }
  for (size_t q = 0; q < wl.size(); ++q)
    if (wl[q].a != boundary[q].a || wl[q].b != boundary[q].b || wl[q].c != boundary[q].c) {
      err = "upload_mesh: a listed wall face is not a boundary face (or a boundary face is not listed)";
      return FELBM_EMESH;
    }
  // node -> element lists, patch volumes, lumped masses
  m.n2e_ptr.assign(N + 1, 0);
  for (int64_t q = 0; q < 4 * E; ++q) m.n2e_ptr[tet[q] + 1]++;
  for (int64_t i = 0; i < N; ++i) m.n2e_ptr[i + 1] += m.n2e_ptr[i];
  m.n2e.assign(4 * E, 0);
  {
    std::vector<int32_t> fill(m.n2e_ptr.begin(), m.n2e_ptr.end() - 1);
    for (int64_t e = 0; e < E; ++e)
      for (int l = 0; l < 4; ++l) m.n2e[fill[tet[4 * e + l]]++] = (int32_t)(4 * e + l);
  }
  m.pvol.assign(N, 0.0);
  for (int64_t i = 0; i < N; ++i) {
    if (m.n2e_ptr[i + 1] == m.n2e_ptr[i]) {
      err = "upload_mesh: node " + std::to_string(i) + " belongs to no tetrahedron";
      return FELBM_EMESH;
    }
    for (int32_t q = m.n2e_ptr[i]; q < m.n2e_ptr[i + 1]; ++q) m.pvol[i] += m.geo[m.n2e[q] >> 2];
  }
  m.mass.resize(N);
  for (int64_t i = 0; i < N; ++i) m.mass[i] = 0.25 * m.pvol[i];
  // wall faces: nodes, areas (unwrapped), and the faces containing each node
  m.wface.assign(3 * W, 0);
  m.warea.assign(W, 0.0);
  m.is_wall.assign(N, 0);
  m.wf_ptr.assign(N + 1, 0);
  for (int64_t w = 0; w < W; ++w) {
    double p[3][3];
    for (int d = 0; d < 3; ++d) p[0][d] = xyz[3 * wface[3 * w] + d];
    for (int v = 1; v < 3; ++v) unwrap(wface[3 * w + v], p[0], p[v]);
    double a[3], b[3];
    for (int d = 0; d < 3; ++d) {
      a[d] = p[1][d] - p[0][d];
      b[d] = p[2][d] - p[0][d];
    }
    const double cx = a[1] * b[2] - a[2] * b[1], cy = a[2] * b[0] - a[0] * b[2], cz = a[0] * b[1] - a[1] * b[0];
    m.warea[w] = 0.5 * std::sqrt(cx * cx + cy * cy + cz * cz);
    for (int v = 0; v < 3; ++v) {
      m.wface[v * W + w] = wface[3 * w + v];
      m.is_wall[wface[3 * w + v]] = 1;
      m.wf_ptr[wface[3 * w + v] + 1]++;
    }
  }
  for (int64_t i = 0; i < N; ++i) m.wf_ptr[i + 1] += m.wf_ptr[i];
  m.wf_list.assign(3 * W, 0);
  {
    std::vector<int32_t> fill(m.wf_ptr.begin(), m.wf_ptr.end() - 1);
    for (int64_t w = 0; w < W; ++w)
      for (int v = 0; v < 3; ++v) m.wf_list[fill[wface[3 * w + v]]++] = (int32_t)w;
  }
  // patch Laplacian of C as an operator (eqn:lapl_int_mp with averaged face gradients)
  {
    auto grad = [&](int64_t e, int v, int r) { return m.geo[(1 + 3 * v + r) * E + e]; };
    std::vector<int32_t> pos(N, -1), cols;
    std::vector<double> vals;
    std::vector<int32_t> rptr_op(N + 1, 0), rcol_op;
    std::vector<double> rval_op;
    std::vector<std::array<int32_t, 3>> wl;
    m.wl_ptr.assign(N + 1, 0);
    for (int64_t k = 0; k < N; ++k) {
      cols.clear();
      vals.clear();
      auto add = [&](int32_t j, double w) {
        if (pos[j] < 0) {
          pos[j] = (int32_t)cols.size();
          cols.push_back(j);
          vals.push_back(0.0);
        }
        vals[pos[j]] += w;
      };
      const double inv_vol = 1.0 / m.pvol[k];
      for (int32_t q = m.n2e_ptr[k]; q < m.n2e_ptr[k + 1]; ++q) {
        const int64_t e = m.n2e[q] >> 2;
        const int l = m.n2e[q] & 3;
        const double V = m.geo[e];
        const int64_t nb = m.fnbr[l * E + e];
        if (nb >= 0) {
          for (int v = 0; v < 4; ++v)
            add(m.tet[v * E + e],
                -1.5 * V * (grad(e, l, 0) * grad(e, v, 0) + grad(e, l, 1) * grad(e, v, 1) + grad(e, l, 2) * grad(e, v, 2)));
          for (int w = 0; w < 4; ++w)
            add(m.tet[w * E + nb], -1.5 * V *
                                        (grad(e, l, 0) * grad(nb, w, 0) + grad(e, l, 1) * grad(nb, w, 1) +
                                         grad(e, l, 2) * grad(nb, w, 2)));
        } else {  // wall face opposite k: area 3V |grad N_l|
          const double gn = std::sqrt(grad(e, l, 0) * grad(e, l, 0) + grad(e, l, 1) * grad(e, l, 1) +
                                      grad(e, l, 2) * grad(e, l, 2));
          wl.push_back({m.tet[((l + 1) & 3) * E + e], m.tet[((l + 2) & 3) * E + e], m.tet[((l + 3) & 3) * E + e]});
          m.wl_scale.push_back(3.0 * V * gn * inv_vol);
        }
      }
      for (int32_t q = m.wf_ptr[k]; q < m.wf_ptr[k + 1]; ++q) {  // wall faces containing k
        const int32_t f = m.wf_list[q];
        wl.push_back({m.wface[f], m.wface[W + f], m.wface[2 * W + f]});
        m.wl_scale.push_back(m.warea[f] * inv_vol);
      }
      m.wl_ptr[k + 1] = (int32_t)wl.size();
      std::vector<int32_t> order(cols.size());
      for (size_t q = 0; q < order.size(); ++q) order[q] = (int32_t)q;
      std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return cols[a] < cols[b]; });
      for (int32_t q : order) {
        if (cols[q] != (int32_t)k) {  // difference form: the node's own weight drops out
          rcol_op.push_back(cols[q]);
          rval_op.push_back(vals[q] * inv_vol);
        }
        pos[cols[q]] = -1;
      }
      rptr_op[k + 1] = (int32_t)rcol_op.size();
    }
    const int64_t L = (int64_t)wl.size();
    m.wl_face.assign(3 * L, 0);
    for (int64_t q = 0; q < L; ++q)
      for (int c = 0; c < 3; ++c) m.wl_face[c * L + q] = wl[q][c];
    const int64_t ns = ((N + 63) / 64 * 64) / 64;
    m.lop_ptr.assign(ns + 1, 0);
    for (int64_t sl = 0; sl < ns; ++sl) {
      int64_t width = 0;
      for (int64_t i = sl * 64; i < std::min<int64_t>(N, (sl + 1) * 64); ++i)
        width = std::max<int64_t>(width, rptr_op[i + 1] - rptr_op[i]);
      const size_t base = m.lop_col.size();
      m.lop_col.resize(base + width * 64);
      m.lop_w.resize(base + width * 64);
      for (int64_t q = 0; q < width; ++q)
        for (int lane = 0; lane < 64; ++lane) {
          const int64_t i = sl * 64 + lane;
          const size_t idx = base + q * 64 + lane;
          const bool real_entry = i < N && q < rptr_op[i + 1] - rptr_op[i];
          m.lop_col[idx] = real_entry ? rcol_op[rptr_op[i] + q] : (int32_t)std::min<int64_t>(i, N - 1);
          m.lop_w[idx] = real_entry ? rval_op[rptr_op[i] + q] : 0.0;
        }
      m.lop_ptr[sl + 1] = (int32_t)m.lop_col.size();
    }
    // element Laplacian of mu: weights of mu_1..3 - mu_0 and of the vertices across the faces
    m.eopp.assign(4 * E, 0);
    m.ew.assign(7 * E, 0.0);
    for (int64_t e = 0; e < E; ++e) {
      double a[4] = {0, 0, 0, 0}, b[4] = {0, 0, 0, 0};
      int32_t opp[4] = {m.tet[e], m.tet[e], m.tet[e], m.tet[e]};
      for (int l = 0; l < 4; ++l) {
        const int64_t nb = m.fnbr[l * E + e];
        if (nb < 0) continue;  // zero normal flux of grad mu through a wall (eqn:bc1)
        for (int v = 0; v < 4; ++v)
          a[v] -= 1.5 * (grad(e, l, 0) * grad(e, v, 0) + grad(e, l, 1) * grad(e, v, 1) + grad(e, l, 2) * grad(e, v, 2));
        for (int w = 0; w < 4; ++w) {
          const int32_t node = m.tet[w * E + nb];
          const double wt =
              -1.5 * (grad(e, l, 0) * grad(nb, w, 0) + grad(e, l, 1) * grad(nb, w, 1) + grad(e, l, 2) * grad(nb, w, 2));
          int v = 0;
          while (v < 4 && m.tet[v * E + e] != node) ++v;
          if (v < 4) {
            a[v] += wt;
          } else {
            opp[l] = node;
            b[l] += wt;
          }
        }
      }
      for (int v = 1; v < 4; ++v) m.ew[(v - 1) * E + e] = a[v];
      for (int l = 0; l < 4; ++l) {
        m.eopp[l * E + e] = opp[l];
        m.ew[(3 + l) * E + e] = b[l];
      }
    }
  }
  // row-scaled consistent mass matrix a_ij = M11_ij / m_i (i != j), M11_ij = sum V/20
  std::vector<std::pair<int32_t, double>> row;
  std::vector<int32_t> rptr(N + 1, 0), rcol;
  std::vector<double> rval;
  for (int64_t i = 0; i < N; ++i) {
    row.clear();
    for (int32_t q = m.n2e_ptr[i]; q < m.n2e_ptr[i + 1]; ++q) {
      const int64_t e = m.n2e[q] >> 2;
      for (int v = 0; v < 4; ++v) {
        const int32_t j = tet[4 * e + v];
        if (j == (int32_t)i) continue;
        const double val = m.geo[e] / 20.0;
        bool found = false;
        for (auto& pr : row)
          if (pr.first == j) {
            pr.second += val;
            found = true;
            break;
          }
        if (!found) row.push_back({j, val});
      }
    }
    std::sort(row.begin(), row.end());
    for (auto& pr : row) {
      rcol.push_back(pr.first);
      rval.push_back(pr.second / m.mass[i]);
    }
    rptr[i + 1] = (int32_t)rcol.size();
  }
  m.nnz = (int64_t)rcol.size();
  // diagonal of the FP64 composition sweeps: with the float-rounded a_ij, sum_i m_i (A x)_i = sum_j m_j x_j
  {
    std::vector<double> colsum(N, 0.0);
    for (int64_t i = 0; i < N; ++i)
      for (int32_t q = rptr[i]; q < rptr[i + 1]; ++q) colsum[rcol[q]] += m.mass[i] * (double)(float)rval[q];
    m.dlt.resize(N);
    for (int64_t j = 0; j < N; ++j) m.dlt[j] = 1.0 - colsum[j] / m.mass[j];
  }
  const int64_t nslices = m.Np / 64;
  m.sell_ptr.assign(nslices + 1, 0);
  for (int64_t s = 0; s < nslices; ++s) {
    int64_t width = 0;
    for (int64_t i = s * 64; i < std::min<int64_t>(N, (s + 1) * 64); ++i) width = std::max<int64_t>(width, rptr[i + 1] - rptr[i]);
    const size_t base = m.sell_col.size();
    m.sell_col.resize(base + width * 64);
    m.sell_val.resize(base + width * 64);
    for (int64_t k = 0; k < width; ++k)
      for (int lane = 0; lane < 64; ++lane) {
        const int64_t i = s * 64 + lane, idx = base + k * 64 + lane;
        const bool real_entry = i < N && k < rptr[i + 1] - rptr[i];
        m.sell_col[idx] = real_entry ? rcol[rptr[i] + k] : (int32_t)std::min<int64_t>(i, N - 1);
        m.sell_val[idx] = real_entry ? rval[rptr[i] + k] : 0.0;
      }
    m.sell_ptr[s + 1] = (int32_t)m.sell_col.size();
  }
  // incident-element weights in sliced ELL (padding: element -1)
  m.inc_ptr.assign(nslices + 1, 0);
  {
    std::vector<int32_t> ie;
    std::vector<double> iw[4];
    for (int64_t s = 0; s < nslices; ++s) {
      int64_t width = 0;
      for (int64_t i = s * 64; i < std::min<int64_t>(N, (s + 1) * 64); ++i)
        width = std::max<int64_t>(width, m.n2e_ptr[i + 1] - m.n2e_ptr[i]);
      const size_t base = ie.size();
      ie.resize(base + width * 64, -1);
      for (auto& v : iw) v.resize(base + width * 64, 0.0);
      for (int64_t i = s * 64; i < std::min<int64_t>(N, (s + 1) * 64); ++i)
        for (int32_t q = m.n2e_ptr[i]; q < m.n2e_ptr[i + 1]; ++q) {
          const int64_t e = m.n2e[q] >> 2, l = m.n2e[q] & 3;
          const size_t idx = base + (size_t)(q - m.n2e_ptr[i]) * 64 + (size_t)(i - s * 64);
          ie[idx] = (int32_t)(4 * e + l);
          iw[0][idx] = m.geo[e] / m.mass[i];
          for (int r = 0; r < 3; ++r) iw[1 + r][idx] = m.geo[e] * m.geo[(1 + 3 * l + r) * E + e] / m.mass[i];
        }
      m.inc_ptr[s + 1] = (int32_t)ie.size();
    }
    m.inc_e = std::move(ie);
    m.inc_w.resize(4 * m.inc_e.size());
    for (int c = 0; c < 4; ++c) std::copy(iw[c].begin(), iw[c].end(), m.inc_w.begin() + c * m.inc_e.size());
  }
  // patch moments: the row of node i holds i and every node sharing an element with it
  {
    std::vector<int32_t> pos(N, -1), cols;
    std::vector<std::array<double, 9>> vals;
    std::vector<int32_t> pptr(N + 1, 0), pcol;
    std::vector<std::array<double, 9>> pval;
    for (int64_t i = 0; i < N; ++i) {
      cols.clear();
      vals.clear();
      for (int32_t q = m.n2e_ptr[i]; q < m.n2e_ptr[i + 1]; ++q) {
        const int64_t e = m.n2e[q] >> 2, l = m.n2e[q] & 3;
        const double V = m.geo[e];
        const double gi[3] = {m.geo[(1 + 3 * l) * E + e], m.geo[(2 + 3 * l) * E + e], m.geo[(3 + 3 * l) * E + e]};
        for (int v = 0; v < 4; ++v) {
          const int32_t j = tet[4 * e + v];
          if (pos[j] < 0) {
            pos[j] = (int32_t)cols.size();
            cols.push_back(j);
            vals.push_back(std::array<double, 9>{});
          }
          std::array<double, 9>& a = vals[pos[j]];
          const double gj[3] = {m.geo[(1 + 3 * v) * E + e], m.geo[(2 + 3 * v) * E + e], m.geo[(3 + 3 * v) * E + e]};
          for (int r = 0; r < 3; ++r) {
            a[r] += V * gj[r];
            a[3 + r] += V * gi[r] * gj[r];
          }
          a[6] += V * (gi[0] * gj[1] + gi[1] * gj[0]);
          a[7] += V * (gi[0] * gj[2] + gi[2] * gj[0]);
          a[8] += V * (gi[1] * gj[2] + gi[2] * gj[1]);
        }
      }
      std::vector<int32_t> order(cols.size());
      for (size_t k = 0; k < order.size(); ++k) order[k] = (int32_t)k;
      std::sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return cols[x] < cols[y]; });
      for (int32_t k : order) {
        pcol.push_back(cols[k]);
        std::array<double, 9> a = vals[k];
        for (double& v : a) v /= m.mass[i];
        pval.push_back(a);
        pos[cols[k]] = -1;
      }
      pptr[i + 1] = (int32_t)pcol.size();
    }
    m.pair_ptr.assign(nslices + 1, 0);
    std::vector<double> pv[9];
    for (int64_t s = 0; s < nslices; ++s) {
      int64_t width = 0;
      for (int64_t i = s * 64; i < std::min<int64_t>(N, (s + 1) * 64); ++i)
        width = std::max<int64_t>(width, pptr[i + 1] - pptr[i]);
      const size_t base = m.pair_col.size();
      m.pair_col.resize(base + width * 64);
      for (auto& v : pv) v.resize(base + width * 64, 0.0);
      for (int64_t k = 0; k < width; ++k)
        for (int lane = 0; lane < 64; ++lane) {
          const int64_t i = s * 64 + lane;
          const size_t idx = base + k * 64 + lane;
          const bool real_entry = i < N && k < pptr[i + 1] - pptr[i];
          m.pair_col[idx] = real_entry ? pcol[pptr[i] + k] : (int32_t)std::min<int64_t>(i, N - 1);
          if (real_entry)
            for (int c = 0; c < 9; ++c) pv[c][idx] = pval[pptr[i] + k][c];
        }
      m.pair_ptr[s + 1] = (int32_t)m.pair_col.size();
    }
    m.pair_v.resize(9 * m.pair_col.size());
    for (int c = 0; c < 9; ++c) std::copy(pv[c].begin(), pv[c].end(), m.pair_v.begin() + c * m.pair_col.size());
  }
  return FELBM_OK;
}

struct PendingTiming3 {
  int kid;
  hipEvent_t start, stop;
};

}  // namespace

struct felbm3d_ctx {
  felbm_params prm{};
  StepParams sp{};
  std::string err;
  int device = 0;
  hipStream_t own_stream = nullptr, stream = nullptr;
  bool has_mesh = false, has_state = false;
  int64_t N = 0, Np = 0, E = 0, W = 0, nnz = 0, step = 0;
  size_t rs = 8;
  std::vector<double> cheb_w;
  int32_t* tet = nullptr;
  int32_t *sell_ptr = nullptr, *sell_col = nullptr, *first_bad = nullptr;
  int32_t *inc_ptr = nullptr, *inc_e = nullptr, *pair_ptr = nullptr, *pair_col = nullptr;
  int64_t inc_slots = 0, pair_slots = 0;
  void *inc_w = nullptr, *pair_v = nullptr, *fpar = nullptr;
  double *bc = nullptr, *mass = nullptr;
  // FP32 composition transport (null in FP64)
  double *rC = nullptr, *jp = nullptr, *em = nullptr, *geo64 = nullptr, *fC = nullptr, *xCa = nullptr, *xCb = nullptr,
         *dlt = nullptr;
  double* grad = nullptr;  // [9][E] grad N_1 .. grad N_3 (FP64 steps)
  uint8_t* is_wall = nullptr;
  void *sell_val = nullptr, *pop = nullptr, *f = nullptr, *xa = nullptr, *xb = nullptr, *pn = nullptr, *un = nullptr;
  int32_t *lop_ptr = nullptr, *lop_col = nullptr, *wl_ptr = nullptr, *wl_face = nullptr, *eopp = nullptr;
  double* wl_scale = nullptr;
  void* lop_w = nullptr;
  double* ew = nullptr;
  int64_t n_wall_entries = 0;
  double *Cn = nullptr, *mu = nullptr, *lapC = nullptr, *lapmu = nullptr, *partials = nullptr;
  DiagRecord *hist = nullptr, *diag_now = nullptr;
  bool timing = false;
  int64_t launches[K3_COUNT] = {};
  double total_ms[K3_COUNT] = {}, bytes[K3_COUNT] = {};
  std::vector<PendingTiming3> pending;
  std::vector<hipEvent_t> event_pool;
  std::vector<void*> allocations;
};

namespace {

thread_local std::string g_create_error3;

int fail(felbm3d_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define HIP_OK3(c, call)                                                                          \
  do {                                                                                            \
    hipError_t e_ = (call);                                                                       \
    if (e_ != hipSuccess)                                                                         \
      return fail((c), FELBM_EDEVICE, std::string(#call) + " failed: " + hipGetErrorString(e_));  \
  } while (0)

#define TRY3(x)                    \
  do {                             \
    int r_ = (x);                  \
    if (r_ != FELBM_OK) return r_; \
  } while (0)

template <typename T>
int dalloc(felbm3d_ctx* c, T** p, size_t count) {
  void* q = nullptr;
  if (hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess)
    return fail(c, FELBM_ENOMEM, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed");
  c->allocations.push_back(q);
  *p = reinterpret_cast<T*>(q);
  return FELBM_OK;
}

int dalloc_bytes(felbm3d_ctx* c, void** p, size_t bytes) {
  if (hipMalloc(p, std::max<size_t>(bytes, 1)) != hipSuccess)
    return fail(c, FELBM_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  c->allocations.push_back(*p);
  return FELBM_OK;
}

template <typename T>
int upload(felbm3d_ctx* c, T* dst, const std::vector<T>& src) {
  if (src.empty()) return FELBM_OK;
  HIP_OK3(c, hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, c->stream));
  return FELBM_OK;
}

template <typename F, typename... Args>
int launch3(felbm3d_ctx* c, int kid, F kernel, int grid, int block, Args... args) {
  if (c->timing) {
    hipEvent_t s = nullptr, t = nullptr;
    if (!c->event_pool.empty()) {
      s = c->event_pool.back();
      c->event_pool.pop_back();
    } else if (hipEventCreate(&s) != hipSuccess) {
      return fail(c, FELBM_EDEVICE, "hipEventCreate failed");
    }
    if (!c->event_pool.empty()) {
      t = c->event_pool.back();
      c->event_pool.pop_back();
    } else if (hipEventCreate(&t) != hipSuccess) {
      return fail(c, FELBM_EDEVICE, "hipEventCreate failed");
    }
    hipExtLaunchKernelGGL(kernel, dim3(grid), dim3(block), 0, c->stream, s, t, 0, args...);
    c->pending.push_back({kid, s, t});
  } else {
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), 0, c->stream, args...);
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, FELBM_EDEVICE, std::string("kernel launch failed: ") + hipGetErrorString(e));
  return FELBM_OK;
}

int harvest(felbm3d_ctx* c) {
  for (auto& p : c->pending) {
    float ms = 0.f;
    HIP_OK3(c, hipEventSynchronize(p.stop));
    HIP_OK3(c, hipEventElapsedTime(&ms, p.start, p.stop));
    c->launches[p.kid] += 1;
    c->total_ms[p.kid] += ms;
    c->event_pool.push_back(p.start);
    c->event_pool.push_back(p.stop);
  }
  c->pending.clear();
  return FELBM_OK;
}

std::vector<double> chebyshev_steps(int K, double lo, double hi) {
  std::vector<double> lam(K), out;
  for (int i = 0; i < K; ++i) lam[i] = 0.5 * (hi + lo) + 0.5 * (hi - lo) * std::cos((2.0 * i + 1.0) * M_PI / (2.0 * K));
  int i = 0, j = K - 1;
  while (i <= j) {  // alternately from the top and the bottom of the spectrum
    out.push_back(1.0 / lam[i]);
    if (i != j) out.push_back(1.0 / lam[j]);
    ++i;
    --j;
  }
  return out;
}

// FP32 composition transport arguments (all null in FP64); em only in a step
Cons3 cons3(felbm3d_ctx* c, bool step, double w = 0.0, const double* xCin = nullptr, double* xCout = nullptr) {
  if (c->prm.precision != FELBM_FP32) return Cons3{};
  return Cons3{c->rC, c->jp, step ? c->em : nullptr, c->geo64, c->fC, xCin, xCout, c->dlt, c->Cn, w};
}

template <typename real>
int enqueue_fields(felbm3d_ctx* c, bool collide, DiagRecord* rec) {
  const int gN = grid_for(c->N), gE = grid_for(c->E);
  const int N = (int)c->N, Np = (int)c->Np, E = (int)c->E;
  real* pop = (real*)c->pop;
  const Cons3 cs = cons3(c, collide);
  if (collide)
    TRY3(launch3(c, K3_MOMENTS, k3_moments<real, true>, gN, BLOCK, pop, N, Np, c->sp, c->Cn, (real*)c->pn, (real*)c->un,
                 (const double*)c->mass, c->partials, cs));
  else
    TRY3(launch3(c, K3_MOMENTS, k3_moments<real, false>, gN, BLOCK, pop, N, Np, c->sp, c->Cn, (real*)c->pn,
                 (real*)c->un, (const double*)c->mass, c->partials, cs));
  if (rec)
    TRY3(launch3(c, K3_REDUCE, felbm::k_reduce_final<>, 1, RBLOCK, (const double*)c->partials, gN, N, (int64_t)c->step,
                 rec, c->first_bad));
  TRY3(launch3(c, K3_LAPC, k3_lapC_mu_op<real>, gN, BLOCK, N, (const int*)c->lop_ptr, (const int*)c->lop_col,
               (const real*)c->lop_w, (const int*)c->wl_ptr, (const int*)c->wl_face, (const double*)c->wl_scale,
               (int)c->n_wall_entries, (const double*)c->Cn, (const double*)c->bc, c->sp, c->lapC, c->mu));
  return launch3(c, K3_LAPMU, k3_lapmu_force_op<real, double>, gE, BLOCK, E, Np, (const int*)c->tet,
                 (const int*)c->eopp, (const double*)c->ew, (const double*)c->grad, (const double*)c->Cn,
                 (const double*)c->mu, (const real*)c->pn, (const real*)c->un, c->sp, c->lapmu, (real*)c->fpar, cs);
}

template <typename real, int MODE>
int sweep3(felbm3d_ctx* c, int kid, const real* xin, real* xout, int j, const double* xCin, double* xCout) {
  const double w = MODE == 4 ? 0.0 : c->cheb_w[j];
  return launch3(c, kid, k3_sweep<real, MODE>, grid_sets_for(c->N), BLOCK, (int)c->N, (int)c->Np, (const int*)c->sell_ptr,
                 (const int*)c->sell_col, (const real*)c->sell_val, (const real*)c->f, xin, xout, (real*)c->pop,
                 (const uint8_t*)c->is_wall, (real)w, cons3(c, true, w, xCin, xCout));
}

template <typename real>
int enqueue_step(felbm3d_ctx* c) {
  TRY3(enqueue_fields<real>(c, true, c->hist + (c->step & 1)));
  TRY3(launch3(c, K3_RHS, k3_rhs<real>, grid_sets_for(c->N), BLOCK, (int)c->N, (int)c->Np, (int)c->E,
               (const int*)c->inc_ptr, (const int*)c->inc_e, (const real*)c->inc_w, (int)c->inc_slots,
               (const real*)c->fpar, (const int*)c->pair_ptr, (const int*)c->pair_col, (const real*)c->pair_v,
               (int)c->pair_slots, (const real*)c->pop, (real*)c->f, (const double*)c->mass, cons3(c, true)));
  const int K = c->prm.solver_sweeps;
  real *xa = (real*)c->xa, *xb = (real*)c->xb;
  double *ca = c->xCa, *cb = c->xCb;
  if (K == 0) {
    TRY3((sweep3<real, 4>(c, K3_SWEEP_LAST, nullptr, nullptr, 0, nullptr, nullptr)));
  } else if (K == 1) {
    TRY3((sweep3<real, 3>(c, K3_SWEEP_LAST, nullptr, nullptr, 0, nullptr, nullptr)));
  } else {
    TRY3((sweep3<real, 0>(c, K3_SWEEP_FIRST, nullptr, xa, 0, nullptr, ca)));
    real *xin = xa, *xout = xb;
    double *cin = ca, *cout = cb;
    for (int j = 1; j < K - 1; ++j) {
      TRY3((sweep3<real, 1>(c, K3_SWEEP_MID, xin, xout, j, cin, cout)));
      std::swap(xin, xout);
      std::swap(cin, cout);
    }
    TRY3((sweep3<real, 2>(c, K3_SWEEP_LAST, xin, nullptr, K - 1, cin, nullptr)));
  }
  c->step += 1;
  return FELBM_OK;
}

int enqueue_steps(felbm3d_ctx* c, int64_t n) {
  for (int64_t s = 0; s < n; ++s)
    TRY3(c->prm.precision == FELBM_FP64 ? enqueue_step<double>(c) : enqueue_step<float>(c));
  return FELBM_OK;
}

// copy n device values in the working precision (or double) to a host double array
int copy_out(felbm3d_ctx* c, const void* src, bool is_real, int64_t n, std::vector<double>& host) {
  host.resize(n);
  if (!is_real || c->prm.precision == FELBM_FP64) {
    HIP_OK3(c, hipMemcpyAsync(host.data(), src, n * 8, hipMemcpyDeviceToHost, c->stream));
  } else {
    std::vector<float> tmp(n);
    HIP_OK3(c, hipMemcpyAsync(tmp.data(), src, n * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_OK3(c, hipStreamSynchronize(c->stream));
    for (int64_t i = 0; i < n; ++i) host[i] = tmp[i];
  }
  HIP_OK3(c, hipStreamSynchronize(c->stream));
  return FELBM_OK;
}

}  // namespace

extern "C" {

const char* felbm3d_last_error(const felbm3d_ctx* c) { return c ? c->err.c_str() : g_create_error3.c_str(); }

int felbm3d_create(const felbm_params* p, felbm3d_ctx** out) {
  g_create_error3.clear();
  if (!p || !out) {
    g_create_error3 = "create: null argument";
    return FELBM_EINVAL;
  }
  *out = nullptr;
  auto bad = [](double v) { return !std::isfinite(v); };
  if (bad(p->sigma) || bad(p->xi) || bad(p->mobility) || bad(p->rho_l) || bad(p->rho_v) || bad(p->nu_l) ||
      bad(p->nu_v) || bad(p->dt) || p->xi <= 0 || p->sigma < 0 || p->mobility < 0 || p->rho_l <= 0 || p->rho_v <= 0 ||
      p->nu_l <= 0 || p->nu_v <= 0 || p->dt <= 0) {
    g_create_error3 = "create: parameters must be finite with xi, densities, viscosities, dt > 0 and sigma, mobility >= 0";
    return FELBM_EINVAL;
  }
  if (p->precision != FELBM_FP64 && p->precision != FELBM_FP32) {
    g_create_error3 = "create: precision must be FELBM_FP64 or FELBM_FP32";
    return FELBM_EINVAL;
  }
  if (p->kernels != 0 || p->force_scheme != 0) {
    g_create_error3 = "create: the 3-D step has one kernel family and the mixed force scheme (kernels, force_scheme = 0)";
    return FELBM_EINVAL;
  }
  if (p->solver_sweeps < 0 || p->solver_sweeps > 256) {
    g_create_error3 = "create: solver_sweeps must be in [0, 256]";
    return FELBM_EINVAL;
  }
  double lo = p->lambda_min, hi = p->lambda_max;
  if (lo == 0.0 && hi == 0.0) {
    lo = 0.2;  // spectrum of diag(m)^-1 M11 for every P1 tetrahedral mesh
    hi = 1.0;
  }
  if (!(lo > 0.0 && hi > lo) || bad(lo) || bad(hi)) {
    g_create_error3 = "create: need 0 < lambda_min < lambda_max";
    return FELBM_EINVAL;
  }
  felbm3d_ctx* c = new (std::nothrow) felbm3d_ctx();
  if (!c) {
    g_create_error3 = "create: out of host memory";
    return FELBM_ENOMEM;
  }
  c->prm = *p;
  c->prm.lambda_min = lo;
  c->prm.lambda_max = hi;
  c->rs = p->precision == FELBM_FP64 ? 8 : 4;
  const double kappa = 1.5 * p->sigma * p->xi, beta = 12.0 * p->sigma / p->xi;
  c->sp = StepParams{kappa, beta, p->mobility, p->rho_l, p->rho_v, CS2 * p->dt / p->nu_l, CS2 * p->dt / p->nu_v, p->dt};
  c->cheb_w = chebyshev_steps(p->solver_sweeps, lo, hi);
  if (hipGetDevice(&c->device) != hipSuccess || hipStreamCreateWithFlags(&c->own_stream, hipStreamNonBlocking) != hipSuccess) {
    g_create_error3 = "create: no usable HIP device";
    delete c;
    return FELBM_EDEVICE;
  }
  c->stream = c->own_stream;
  *out = c;
  return FELBM_OK;
}

int felbm3d_upload_mesh(felbm3d_ctx* c, int64_t n_nodes, const double* xyz, int64_t n_tets, const int32_t* tet,
                        int64_t n_wall, const int32_t* wall_face, double px, double py) {
  if (!c) return FELBM_EINVAL;
  if (c->has_mesh) return fail(c, FELBM_ESTATE, "upload_mesh: a mesh was already uploaded to this context");
  Prep3 m;
  TRY3(prepare3(n_nodes, xyz, n_tets, tet, n_wall, wall_face, px, py, m, c->err));
  c->N = m.N;
  c->Np = m.Np;
  c->E = m.E;
  c->W = m.W;
  c->nnz = m.nnz;
  HIP_OK3(c, hipSetDevice(c->device));
  const int64_t N = m.N, Np = m.Np, E = m.E;
  const size_t rs = c->rs;
  TRY3(dalloc(c, &c->tet, 4 * E));
  TRY3(dalloc(c, &c->is_wall, N));
  TRY3(dalloc(c, &c->bc, N));
  TRY3(dalloc(c, &c->mass, N));
  TRY3(dalloc(c, &c->sell_ptr, m.sell_ptr.size()));
  TRY3(dalloc(c, &c->sell_col, m.sell_col.size()));
  TRY3(dalloc_bytes(c, &c->sell_val, m.sell_val.size() * rs));
  c->inc_slots = (int64_t)m.inc_e.size();
  c->pair_slots = (int64_t)m.pair_col.size();
  TRY3(dalloc(c, &c->inc_ptr, m.inc_ptr.size()));
  TRY3(dalloc(c, &c->inc_e, m.inc_e.size()));
  TRY3(dalloc(c, &c->pair_ptr, m.pair_ptr.size()));
  TRY3(dalloc(c, &c->pair_col, m.pair_col.size()));
  TRY3(dalloc_bytes(c, &c->inc_w, m.inc_w.size() * rs));
  TRY3(dalloc_bytes(c, &c->pair_v, m.pair_v.size() * rs));
  TRY3(dalloc_bytes(c, &c->fpar, 13 * E * rs));
  c->n_wall_entries = (int64_t)m.wl_scale.size();
  TRY3(dalloc(c, &c->lop_ptr, m.lop_ptr.size()));
  TRY3(dalloc(c, &c->lop_col, m.lop_col.size()));
  TRY3(dalloc_bytes(c, &c->lop_w, m.lop_w.size() * rs));
  TRY3(dalloc(c, &c->wl_ptr, m.wl_ptr.size()));
  TRY3(dalloc(c, &c->wl_face, m.wl_face.size()));
  TRY3(dalloc(c, &c->wl_scale, m.wl_scale.size()));
  TRY3(dalloc(c, &c->eopp, m.eopp.size()));
  TRY3(dalloc(c, &c->ew, m.ew.size()));  // double in both precisions: conserves mass in the FP32 form
  if (c->prm.precision == FELBM_FP32) {
    TRY3(dalloc(c, &c->rC, N));
    TRY3(dalloc(c, &c->jp, 9 * Np));
    TRY3(dalloc(c, &c->em, 4 * E));
    TRY3(dalloc(c, &c->geo64, 10 * E));  // V, grad N_1 .. grad N_3
    TRY3(dalloc(c, &c->fC, Np));
    TRY3(dalloc(c, &c->xCa, Np));
    TRY3(dalloc(c, &c->xCb, Np));
    TRY3(dalloc(c, &c->dlt, N));
  }
  if (c->prm.precision == FELBM_FP64) TRY3(dalloc(c, &c->grad, 9 * E));  // grad N_1 .. grad N_3
  TRY3(dalloc_bytes(c, &c->pop, 2 * QS * Np * rs));  // [2][5][Np][4]
  TRY3(dalloc_bytes(c, &c->f, 2 * QS * Np * rs));  // solve vectors: [2][5][Np][4]
  TRY3(dalloc_bytes(c, &c->xa, 2 * QS * Np * rs));
  TRY3(dalloc_bytes(c, &c->xb, 2 * QS * Np * rs));
  TRY3(dalloc_bytes(c, &c->pn, Np * rs));
  TRY3(dalloc_bytes(c, &c->un, 3 * Np * rs));
  TRY3(dalloc(c, &c->Cn, N));
  TRY3(dalloc(c, &c->mu, N));
  TRY3(dalloc(c, &c->lapC, N));
  TRY3(dalloc(c, &c->lapmu, E));
  TRY3(dalloc(c, &c->partials, (size_t)NRED * grid_for(N)));
  TRY3(dalloc(c, &c->hist, 2));
  TRY3(dalloc(c, &c->diag_now, 1));
  TRY3(dalloc(c, &c->first_bad, 1));
  TRY3(upload(c, c->tet, m.tet));
  TRY3(upload(c, c->is_wall, m.is_wall));
  TRY3(upload(c, c->mass, m.mass));
  TRY3(upload(c, c->sell_ptr, m.sell_ptr));
  TRY3(upload(c, c->sell_col, m.sell_col));
  TRY3(upload(c, c->lop_ptr, m.lop_ptr));
  TRY3(upload(c, c->lop_col, m.lop_col));
  TRY3(upload(c, c->wl_ptr, m.wl_ptr));
  TRY3(upload(c, c->wl_face, m.wl_face));
  TRY3(upload(c, c->wl_scale, m.wl_scale));
  TRY3(upload(c, c->eopp, m.eopp));
  TRY3(upload(c, c->ew, m.ew));
  TRY3(upload(c, c->inc_ptr, m.inc_ptr));
  TRY3(upload(c, c->inc_e, m.inc_e));
  TRY3(upload(c, c->pair_ptr, m.pair_ptr));
  TRY3(upload(c, c->pair_col, m.pair_col));
  // dt factors of the right-hand side: dt/4 on alpha and G, dt^2/2 on beta and S
  const double c1 = c->prm.dt / 4.0, c2 = 0.5 * c->prm.dt * c->prm.dt;
  for (size_t q = 0; q < m.inc_w.size(); ++q) m.inc_w[q] *= (q < m.inc_e.size()) ? c1 : c2;
  for (size_t q = 0; q < m.pair_v.size(); ++q) m.pair_v[q] *= (q < 3 * m.pair_col.size()) ? c1 : c2;
  if (c->prm.precision == FELBM_FP64) {
    TRY3(upload(c, (double*)c->sell_val, m.sell_val));
    TRY3(upload(c, (double*)c->inc_w, m.inc_w));
    TRY3(upload(c, (double*)c->pair_v, m.pair_v));
    TRY3(upload(c, (double*)c->lop_w, m.lop_w));
    std::vector<double> g64(m.geo.begin() + 4 * E, m.geo.end());
    TRY3(upload(c, (double*)c->grad, g64));
    HIP_OK3(c, hipStreamSynchronize(c->stream));
  } else {
    std::vector<float> v32(m.sell_val.begin(), m.sell_val.end()), w32(m.inc_w.begin(), m.inc_w.end()),
        p32(m.pair_v.begin(), m.pair_v.end());
    TRY3(upload(c, (float*)c->sell_val, v32));
    TRY3(upload(c, (float*)c->inc_w, w32));
    TRY3(upload(c, (float*)c->pair_v, p32));
    std::vector<float> l32(m.lop_w.begin(), m.lop_w.end());
    TRY3(upload(c, (float*)c->lop_w, l32));
    std::vector<double> geo(10 * E);  // V, then the rows of grad N_1 .. grad N_3
    std::copy(m.geo.begin(), m.geo.begin() + E, geo.begin());
    std::copy(m.geo.begin() + 4 * E, m.geo.end(), geo.begin() + E);
    TRY3(upload(c, c->geo64, geo));
    TRY3(upload(c, c->dlt, m.dlt));
    HIP_OK3(c, hipStreamSynchronize(c->stream));
  }
  std::vector<double> zeros(N, 0.0);
  TRY3(upload(c, c->bc, zeros));
  HIP_OK3(c, hipMemsetAsync(c->pop, 0, 2 * QS * Np * rs, c->stream));
  HIP_OK3(c, hipMemsetAsync(c->f, 0, 2 * QS * Np * rs, c->stream));
  HIP_OK3(c, hipMemsetAsync(c->xa, 0, 2 * QS * Np * rs, c->stream));
  HIP_OK3(c, hipMemsetAsync(c->xb, 0, 2 * QS * Np * rs, c->stream));
  HIP_OK3(c, hipMemsetAsync(c->un, 0, 3 * Np * rs, c->stream));
  HIP_OK3(c, hipStreamSynchronize(c->stream));
  // algorithmic bytes per launch (perfect reuse of gathered data)
  const double Nd = (double)N, Ed = (double)E, s = (double)rs, nnz = (double)m.nnz;
  const double pops = 38.0 * Nd * s, mat = nnz * (4.0 + s) + (double)(Np / 64 + 1) * 4.0;
  c->bytes[K3_MOMENTS] = 2 * pops + Nd * (8 + 4 * s + 8);
  c->bytes[K3_LAPC] = (double)m.lop_col.size() * (4 + s) + Nd * (8 + 8 + 8 + 4) + (double)m.wl_scale.size() * (12 + 8);
  const double cons = c->prm.precision == FELBM_FP32 ? 1.0 : 0.0;
  c->bytes[K3_MOMENTS] += cons * Nd * (8 + 72);
  c->bytes[K3_LAPMU] = Ed * (16 + 16 + 7 * 8 + 12 * s + 8 + 13 * s) + Nd * (8 + 8 + s + 3 * s) +
                       cons * (Ed * (96 + 32) + Nd * 72);
  c->bytes[K3_RHS] = 2 * pops + (double)m.inc_e.size() * (4 + 4 * s) + (double)m.pair_col.size() * (4 + 9 * s) +
                     Ed * 13 * s + cons * (Ed * 32 + Nd * 16);
  c->bytes[K3_SWEEP_FIRST] = 2 * pops + mat + cons * Nd * 24;
  c->bytes[K3_SWEEP_MID] = 3 * pops + mat + cons * Nd * 32;
  c->bytes[K3_SWEEP_LAST] = 4 * pops + mat + Nd + cons * Nd * 40;
  c->has_mesh = true;
  return FELBM_OK;
}

int felbm3d_set_wetting(felbm3d_ctx* c, const double* omega_c) {
  if (!c) return FELBM_EINVAL;
  if (!c->has_mesh) return fail(c, FELBM_ESTATE, "set_wetting: no mesh");
  if (!omega_c) return fail(c, FELBM_EINVAL, "set_wetting: null omega_c");
  std::vector<uint8_t> wall(c->N);
  HIP_OK3(c, hipMemcpy(wall.data(), c->is_wall, c->N, hipMemcpyDeviceToHost));
  std::vector<double> bc(c->N, 0.0);
  const double kappa = c->sp.kappa, beta = c->sp.beta;
  for (int64_t i = 0; i < c->N; ++i) {
    if (!std::isfinite(omega_c[i])) return fail(c, FELBM_EINVAL, "set_wetting: non-finite value");
    if (!wall[i] || omega_c[i] == 0.0) continue;
    if (kappa <= 0.0) return fail(c, FELBM_EINVAL, "set_wetting: a nonzero wetting potential needs kappa > 0");
    bc[i] = omega_c[i] * std::sqrt(2.0 * kappa * beta) / kappa;  // phi_c / kappa (Young)
  }
  TRY3(upload(c, c->bc, bc));
  HIP_OK3(c, hipStreamSynchronize(c->stream));
  return FELBM_OK;
}

int felbm3d_init(felbm3d_ctx* c, const double* C, const double* u, const double* p) {
  if (!c) return FELBM_EINVAL;
  if (!c->has_mesh) return fail(c, FELBM_ESTATE, "init: no mesh");
  if (!C) return fail(c, FELBM_EINVAL, "init: null C");
  const int64_t N = c->N;
  std::vector<double> hC(C, C + N), hU(3 * N, 0.0), hP(N, 0.0);
  if (u) std::copy(u, u + 3 * N, hU.begin());
  if (p) std::copy(p, p + N, hP.begin());
  for (int64_t i = 0; i < N; ++i)
    if (!std::isfinite(hC[i]) || !std::isfinite(hP[i]) || !std::isfinite(hU[3 * i]) || !std::isfinite(hU[3 * i + 1]) ||
        !std::isfinite(hU[3 * i + 2]))
      return fail(c, FELBM_EINVAL, "init: non-finite input at node " + std::to_string(i));
  double *dC = nullptr, *dU = nullptr, *dP = nullptr;
  TRY3(dalloc(c, &dC, N));
  TRY3(dalloc(c, &dU, 3 * N));
  TRY3(dalloc(c, &dP, N));
  // these three are freed right away (not kept in the allocation list)
  c->allocations.resize(c->allocations.size() - 3);
  int r = FELBM_OK;
  hipError_t e = hipMemcpyAsync(dC, hC.data(), N * 8, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(dU, hU.data(), 3 * N * 8, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(dP, hP.data(), N * 8, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) {
    const int g = (int)((N + BLOCK - 1) / BLOCK);
    if (c->prm.precision == FELBM_FP64)
      hipLaunchKernelGGL(k3_init<double>, dim3(g), dim3(BLOCK), 0, c->stream, (int)N, (int)c->Np, c->sp,
                         (const double*)dC, (const double*)dU, (const double*)dP, (const uint8_t*)c->is_wall,
                         (double*)c->pop, (double*)nullptr);
    else
      hipLaunchKernelGGL(k3_init<float>, dim3(g), dim3(BLOCK), 0, c->stream, (int)N, (int)c->Np, c->sp,
                         (const double*)dC, (const double*)dU, (const double*)dP, (const uint8_t*)c->is_wall,
                         (float*)c->pop, c->rC);
    e = hipGetLastError();
  }
  const int32_t minus1 = -1;
  if (e == hipSuccess) e = hipMemcpyAsync(c->first_bad, &minus1, sizeof(int32_t), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) r = fail(c, FELBM_EDEVICE, std::string("init: ") + hipGetErrorString(e));
  (void)hipFree(dC);
  (void)hipFree(dU);
  (void)hipFree(dP);
  if (r != FELBM_OK) return r;
  c->step = 0;
  c->has_state = true;
  return FELBM_OK;
}

int felbm3d_step_async(felbm3d_ctx* c, int64_t n) {
  if (!c) return FELBM_EINVAL;
  if (!c->has_state) return fail(c, FELBM_ESTATE, "step: not initialised");
  if (n < 0) return fail(c, FELBM_EINVAL, "step: negative step count");
  return enqueue_steps(c, n);
}

int felbm3d_step(felbm3d_ctx* c, int64_t n) {
  TRY3(felbm3d_step_async(c, n));
  HIP_OK3(c, hipStreamSynchronize(c->stream));
  if (c->timing) TRY3(harvest(c));
  int32_t bad = -1;
  HIP_OK3(c, hipMemcpy(&bad, c->first_bad, sizeof(int32_t), hipMemcpyDeviceToHost));
  if (bad >= 0) return fail(c, FELBM_ENONFINITE, "step: non-finite state entering step " + std::to_string(bad));
  return FELBM_OK;
}

int felbm3d_read(felbm3d_ctx* c, int32_t field, double* out) {
  if (!c) return FELBM_EINVAL;
  if (!c->has_state) return fail(c, FELBM_ESTATE, "read: not initialised");
  if (!out) return fail(c, FELBM_EINVAL, "read: null output");
  if (field < FELBM_FIELD_C || field > FELBM_FIELD_UZ) return fail(c, FELBM_EINVAL, "read: unknown field");
  TRY3(c->prm.precision == FELBM_FP64 ? enqueue_fields<double>(c, false, nullptr) : enqueue_fields<float>(c, false, nullptr));
  std::vector<double> host;
  const int64_t N = c->N, Np = c->Np;
  switch (field) {
    case FELBM_FIELD_C:
    case FELBM_FIELD_RHO: TRY3(copy_out(c, c->Cn, false, N, host)); break;
    case FELBM_FIELD_P: TRY3(copy_out(c, c->pn, true, N, host)); break;
    case FELBM_FIELD_MU: TRY3(copy_out(c, c->mu, false, N, host)); break;
    case FELBM_FIELD_LAPC: TRY3(copy_out(c, c->lapC, false, N, host)); break;
    case FELBM_FIELD_LAPMU: TRY3(copy_out(c, c->lapmu, false, c->E, host)); break;
    default: {
      const int comp = field == FELBM_FIELD_UX ? 0 : (field == FELBM_FIELD_UY ? 1 : 2);
      const char* base = static_cast<const char*>(c->un) + (size_t)comp * Np * c->rs;
      TRY3(copy_out(c, base, true, N, host));
    }
  }
  if (c->timing) TRY3(harvest(c));
  std::copy(host.begin(), host.end(), out);
  if (field == FELBM_FIELD_RHO)
    for (int64_t i = 0; i < N; ++i) out[i] = out[i] * c->prm.rho_l + (1.0 - out[i]) * c->prm.rho_v;
  return FELBM_OK;
}

int felbm3d_read_populations(felbm3d_ctx* c, double* out) {
  if (!c) return FELBM_EINVAL;
  if (!c->has_state) return fail(c, FELBM_ESTATE, "read_populations: not initialised");
  if (!out) return fail(c, FELBM_EINVAL, "read_populations: null output");
  std::vector<double> host;
  TRY3(copy_out(c, c->pop, true, 2 * QS * c->Np, host));
  // device [set][a / 4][Np][a % 4] -> caller [set * 19 + a][N]
  const int64_t Np = c->Np, N = c->N;
  for (int64_t set = 0; set < 2; ++set)
    for (int64_t a = 0; a < Q; ++a) {
      const double* src = host.data() + set * QS * Np + (a >> 2) * 4 * Np + (a & 3);
      double* dst = out + (set * Q + a) * N;
      for (int64_t j = 0; j < N; ++j) dst[j] = src[4 * j];
    }
  return FELBM_OK;
}

int felbm3d_diagnostics(felbm3d_ctx* c, felbm_diag* out) {
  if (!c) return FELBM_EINVAL;
  if (!c->has_state) return fail(c, FELBM_ESTATE, "diagnostics: not initialised");
  if (!out) return fail(c, FELBM_EINVAL, "diagnostics: null output");
  const int gN = grid_for(c->N);
  const int N = (int)c->N, Np = (int)c->Np;
  if (c->prm.precision == FELBM_FP64)
    TRY3(launch3(c, K3_MOMENTS, k3_moments<double, false>, gN, BLOCK, (double*)c->pop, N, Np, c->sp, c->Cn,
                 (double*)c->pn, (double*)c->un, (const double*)c->mass, c->partials, cons3(c, false)));
  else
    TRY3(launch3(c, K3_MOMENTS, k3_moments<float, false>, gN, BLOCK, (float*)c->pop, N, Np, c->sp, c->Cn,
                 (float*)c->pn, (float*)c->un, (const double*)c->mass, c->partials, cons3(c, false)));
  // the final pass writes its non-finite flag only where it is negative: a zeroed
  // scratch flag keeps the step's own first-bad-step record untouched
  int32_t* scratch = nullptr;
  TRY3(dalloc(c, &scratch, 1));
  c->allocations.pop_back();
  const int32_t zero = 0;
  hipError_t e = hipMemcpyAsync(scratch, &zero, sizeof(int32_t), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(felbm::k_reduce_final<>, dim3(1), dim3(RBLOCK), 0, c->stream, (const double*)c->partials, gN, N,
                       (int64_t)c->step, c->diag_now, scratch);
    e = hipGetLastError();
  }
  DiagRecord rec{};
  if (e == hipSuccess) e = hipMemcpyAsync(&rec, c->diag_now, sizeof(DiagRecord), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  (void)hipFree(scratch);
  if (e != hipSuccess) return fail(c, FELBM_EDEVICE, std::string("diagnostics: ") + hipGetErrorString(e));
  if (c->timing) TRY3(harvest(c));
  std::memset(out, 0, sizeof(*out));
  out->step = rec.step;
  out->mass = rec.mass;
  out->mean_ke = rec.mean_ke;
  out->max_u = rec.max_u;
  out->nonfinite = rec.nonfinite;
  out->solver_sweeps = c->prm.solver_sweeps;
  out->solver_residual = -1.0;
  out->residual_step = -1;
  return FELBM_OK;
}

int felbm3d_bind_stream(felbm3d_ctx* c, void* s) {
  if (!c) return FELBM_EINVAL;
  HIP_OK3(c, hipStreamSynchronize(c->stream));
  c->stream = s ? (hipStream_t)s : c->own_stream;
  return FELBM_OK;
}

int felbm3d_kernel_timing(felbm3d_ctx* c, int32_t enable) {
  if (!c) return FELBM_EINVAL;
  HIP_OK3(c, hipStreamSynchronize(c->stream));
  TRY3(harvest(c));
  c->timing = enable != 0;
  for (int k = 0; k < K3_COUNT; ++k) {
    c->launches[k] = 0;
    c->total_ms[k] = 0.0;
  }
  return FELBM_OK;
}

int felbm3d_kernel_stats(felbm3d_ctx* c, felbm_kstat* out, int32_t max_entries, int32_t* n_out) {
  if (!c) return FELBM_EINVAL;
  if (!out || !n_out || max_entries < 0) return fail(c, FELBM_EINVAL, "kernel_stats: bad arguments");
  HIP_OK3(c, hipStreamSynchronize(c->stream));
  TRY3(harvest(c));
  const int n = std::min<int>(K3_COUNT, max_entries);
  for (int k = 0; k < n; ++k) {
    std::memset(&out[k], 0, sizeof(felbm_kstat));
    std::snprintf(out[k].name, sizeof(out[k].name), "%s", kNames3[k]);
    out[k].launches = c->launches[k];
    out[k].total_ms = c->total_ms[k];
    out[k].bytes_per_launch = c->bytes[k];
  }
  *n_out = n;
  return FELBM_OK;
}

int felbm3d_mesh_info(const felbm3d_ctx* c, int64_t* n_nodes, int64_t* n_tets, int64_t* n_wall, int64_t* nnz) {
  if (!c || !c->has_mesh) return FELBM_ESTATE;
  if (n_nodes) *n_nodes = c->N;
  if (n_tets) *n_tets = c->E;
  if (n_wall) *n_wall = c->W;
  if (nnz) *nnz = c->nnz;
  return FELBM_OK;
}

void felbm3d_destroy(felbm3d_ctx* c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (auto& p : c->pending) {
    (void)hipEventDestroy(p.start);
    (void)hipEventDestroy(p.stop);
  }
  for (auto e : c->event_pool) (void)hipEventDestroy(e);
  for (void* p : c->allocations) (void)hipFree(p);
  if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
  delete c;
}

}  // extern "C"
