// Host-side set-up of the constant PD factor (Section 3.1 of the paper).
//
// The free DOFs are split into x1 (collision-free, n1 vertices) and x2
// (collision-aware, n2 vertices), Eq. (6).  Because vec(F) row r depends only
// on coordinate r of the vertices, H = H_s (x) I_3 with a scalar H_s, so every
// factor here is scalar and is applied to 3 right-hand sides at once.
//
// x1 is ordered by geometric nested dissection; every dissection-tree node
// (a leaf sub-domain or a separator) is one dense supernode J with columns
// [c0, c0 + s) and an off-diagonal row set R(J) of r later indices.  A
// multifrontal sweep factors H11 = L1 L1^T and, treating x2 as the root front,
// also produces the rows L21 = H21 L1^-T and the Schur complement
// Sigma_s = H22 - H21 H11^-1 H12 of Eq. (8).  Extended indices: [0, n1) are x1
// in dissection order, [n1, n1 + n2) are x2 in caller order.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace pdipc {

struct FactorNode {
  int32_t c0, s, r, parent, level;
  int64_t rows_off, panel_off, dinv_off;
};

struct HostFactor {
  int32_t n1 = 0, n2 = 0, nlevels = 0;
  std::vector<int32_t> perm;          // dissection position -> x1 input index
  std::vector<FactorNode> nodes;      // post-order (children first)
  std::vector<int32_t> rows;          // concatenated R(J), extended indices
  std::vector<double> panel;          // per node r x s row-major: L[R(J), cols(J)]
  std::vector<double> dinv;           // per node s x s row-major inverse of L[J,J]
  std::vector<int64_t> fwd_ptr;       // n1 + n2 + 1: CSR by row of all panel entries
  std::vector<int32_t> fwd_col;       // column (x1 dissection index)
  std::vector<double> fwd_val;
  std::vector<double> sigma;          // n2 x n2 row-major Schur complement Sigma_s
  int64_t factor_nnz = 0;             // lower entries of the supernodal L1 and L21
};

// Scalar symmetric matrix over the free vertices in extended *input* order:
// indices [0, n1) are x1 (input order), [n1, n1 + n2) are x2.  Full pattern
// (both triangles) in CSR.  coords1: n1 x 3 positions used for dissection.
struct ScalarCSR {
  int32_t n = 0;
  std::vector<int64_t> ptr;
  std::vector<int32_t> col;
  std::vector<double> val;
};

// Returns 0 on success; -3 if a pivot is not positive (matrix not SPD).
int build_host_factor(int32_t n1, int32_t n2, const double* coords1, const ScalarCSR& H,
                      int32_t leaf_size, HostFactor& out, std::string& err);

}  // namespace pdipc
