// Host side of the geometric h-multigrid on the Q_1 space (the h-coarse solver below
// p = 1, Sec. 5.1): CSR matrices, their products, and the hierarchy of nested
// Cartesian meshes with trilinear interpolation and Galerkin operators.
#pragma once
#include <cstdint>
#include <vector>

namespace rz {

struct HostCsr {
  int n = 0, m = 0;  // rows, columns
  std::vector<int> ptr{0}, col;
  std::vector<double> val;
};

// C = A B, columns of each row in ascending order (the sums run in the order of A's
// row entries, then of B's: deterministic)
HostCsr csr_product(const HostCsr &A, const HostCsr &B);
HostCsr csr_transpose(const HostCsr &A);

// The free vertices of a Q_1 lattice of n[a] cells per axis form the box lo..hi per
// axis (vertex 0 and n[a] constrained where the Dirichlet bit 2a resp. 2a+1 of dir is
// set), numbered x fastest.
struct FreeBox {
  int n[3], lo[3], hi[3];
  int ext(int a) const { return hi[a] - lo[a] + 1; }
  int64_t size() const { return (int64_t)ext(0) * ext(1) * ext(2); }
};
FreeBox free_box(const int n[3], unsigned dir);

// Trilinear interpolation from the mesh with half the cells (every count even) to the
// fine one, on the free vertices: weight 1 where a fine vertex is a coarse one, 1/2
// per axis where it lies midway between two coarse vertices.
HostCsr trilinear_interpolation(const FreeBox &fine, const FreeBox &coarse);

// Levels 0..L of the hierarchy from the operator A0 on the free vertices of the mesh
// with n cells per axis: while every cell count is even and the level holds more than
// min_free DoFs, the next level halves the cells, with P_l the interpolation, R_l =
// P_l^T and A_{l+1} = R_l A_l P_l.  A[l] for l = 0..L, P and R for l < L.
void hmg_hierarchy(HostCsr A0, const int n[3], unsigned dir, int64_t min_free, std::vector<HostCsr> &A,
                   std::vector<HostCsr> &P, std::vector<HostCsr> &R);

}  // namespace rz
