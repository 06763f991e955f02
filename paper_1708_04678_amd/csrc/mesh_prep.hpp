// Host-side mesh preprocessing for the FE-LBM step: validation, element
// geometry in FP64, element adjacency across edges, node->element gather
// lists, wall adjacency per node and the row-scaled consistent mass matrix
// diag(m)^-1 M11 in sliced-ELL form (Sec. II.C: P1 elements, lumped mass).
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

namespace felbm {

struct MeshPrep {
  int64_t N = 0, Np = 0, E = 0, W = 0;
  std::vector<int32_t> tri;        // [3][E]
  std::vector<int32_t> enbr;       // [3][E] element across the edge opposite local vertex l, -1 = wall
  std::vector<double> geo;         // [7][E] A, dN0/dx, dN0/dy, dN1/dx, dN1/dy, dN2/dx, dN2/dy
  std::vector<int32_t> n2e_ptr;    // [N+1]
  std::vector<int32_t> n2e;        // packed element*4 + local vertex, sorted by element
  std::vector<int32_t> wall_nbr;   // [2][N] other end of the wall edges incident to the node, -1 = none
  std::vector<double> wall_len;    // [2][N]
  std::vector<uint8_t> is_wall;    // [N]
  std::vector<double> mass;        // [N] lumped mass m_i = sum_T A_T / 3
  std::vector<double> xy;          // [2][N]
  // sliced ELL (slice height 64) of a_ij = M11_ij / m_i, i != j
  std::vector<int32_t> sell_ptr;   // [Np/64 + 1] entry offset of each slice
  std::vector<int32_t> sell_col;
  std::vector<double> sell_val;
  // the same rows in CSR form: row i holds (j, a_ij) for its mesh neighbours j, sorted by j
  std::vector<int32_t> csr_ptr, csr_col;
  std::vector<double> csr_val;
  int64_t offdiag_nnz = 0;         // true (unpadded) off-diagonal count
  double period_x = 0.0;
  // internal orderings: node_perm[internal] = caller node, node_iperm[caller] = internal,
  // elem_perm[internal] = caller triangle
  std::vector<int32_t> node_perm, node_iperm, elem_perm;
  uint64_t perm_hash = 0;
};

// Returns 0 on success or a negative FELBM_E* code with a message in err.
// Arrays in `out` are in the internal order: nodes are renumbered by recursive
// bisection into compact blocks of `block` consecutive nodes (the workgroup
// tile of the gather kernels), triangles sorted by their smallest internal
// vertex.  reorder = false keeps the caller's order.
int prepare_mesh(int64_t n_nodes, const double* xy, int64_t n_tris, const int32_t* tri, int64_t n_wall,
                 const int32_t* wall_edge, double period_x, MeshPrep& out, std::string& err,
                 bool reorder = true, int block = 256);

}  // namespace felbm
