// Host-side cell algebra of the statically condensed Pavarino-Hiptmair relaxation
// for H(curl) (NCE_p) and H(div) (NCF_p) on axis-aligned cells with
// cellwise-constant coefficients (Sec. 4.3-4.5): the cell operator from its six
// weights, the exact block factorisation of its interior block (blocks of at most
// 3 x 3, remark of Sec. 4.4), the interface Schur complement, and the layout and
// Cholesky factors of the edge-star patches (Sec. 4.5).
#pragma once
#include <array>
#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "tables1d.hpp"

namespace rz {

// Local numbering of one cell of NCE_p (space 1) or NCF_p (space 2): the three
// components one after the other, each tile x fastest (the order of the apply's
// per-cell buffer).
struct VecLocal {
  int space = 0, p = 0, nloc = 0;
  int ext[3][3];              // tile extents of component m along axis a
  int off[4];                 // first local index of each component
  std::vector<int> comp;      // per local DoF: component
  std::vector<int> crd;       // per local DoF: 3 tile coordinates
  std::vector<char> interior; // every continuous coordinate strictly inside the cell
};
void vec_local_layout(int space, int p, VecLocal &L);
// continuous (P) kind of component m along axis a
inline bool vec_is_P(int space, int m, int a) { return space == 1 ? a != m : a == m; }

// Sparse rows (column, value), columns ascending.
using SpRow = std::vector<std::pair<int, double>>;
using SpRows = std::vector<SpRow>;

// The cell operator is sum_k w_k K_k over six basis matrices: k = 0..2 the
// stiffness terms (curl component k for NCE; k = 0 the divergence for NCF, k = 1, 2
// empty), k = 3..5 the mass of component k - 3.  Reference FDM tables of degree p.
void vec_basis_matrices(const Tables1D &t, const VecLocal &L, SpRows basis[6]);

// Static condensation of one cell operator (weights w[6]).
struct CellCondensed {
  std::vector<int> I, G;                  // local indices of the interior / interface DoFs
  std::vector<int> gpos;                  // nloc: position in G (or -1)
  std::vector<std::array<int, 3>> blocks; // interior blocks: positions in I, -1 padded
  std::vector<double> linv;               // 9 per block: L^{-1} (row-major, lower) of P_II = L L^T
  std::vector<int> gi_ptr, gi_col;        // P_GI: rows = G positions, columns = I positions
  std::vector<double> gi_val;
  std::vector<int> ig_ptr, ig_col;        // P_IG: rows = I positions, columns = G positions
  std::vector<double> ig_val;
  std::vector<double> S;                  // dense nG x nG interface Schur complement (if asked)
};
// Returns false with a message if a block of P_II exceeds 3 x 3 or is not positive
// definite.  The sparsity of P_GI / P_IG is the structural one of the basis matrices
// (the same for every set of positive weights).
bool vec_condense(const VecLocal &L, const SpRows basis[6], const double w[6], bool want_S, CellCondensed &out,
                  std::string &err);

// Edge-star patches of NCE_p (Sec. 4.5).  The patch of an edge along axis m holds
// the free interface DoFs of the edge and of the (up to four) faces through it.  In
// the FDM basis on Cartesian cells its Schur-complement matrix splits into p blocks,
// one per mode i along the edge (block 0: 4p-3 rows, blocks 1..p-1: 8p-3 rows); every
// patch keeps this fixed slot layout, absent DoFs (outside the mesh or on a
// Dirichlet face) being identity rows that are never gathered.
struct EdgeLayout {
  int p = 0, nslot = 0;
  std::vector<int> blk_n, blk_slot, blk_fac;  // per block: rows, first slot, first factor value
  int fac_stride = 0;                         // factor values of one patch type
};
void edge_layout(int p, EdgeLayout &E);

struct EdgePatches {
  EdgeLayout lay;
  std::vector<int64_t> edge_id;   // non-empty patches: edge ids (axis-major, lattice order)
  std::vector<int> idx;           // npatch * nslot: global DoF of each slot, -1 absent
  std::vector<int> type;          // npatch: factor set
  std::vector<double> fac;        // ntypes * fac_stride: per mode block W = L^{-1} of the
                                  // FP64 Cholesky factor L of the patch matrix, packed by
                                  // columns and again by rows (n(n+1) values)
  // sum back to the interface: for every free interface DoF (in the order of `rows`)
  // the slots holding it (positions patch * nslot + slot, ascending patch)
  std::vector<int> rows, ptr, pos;
};
// nx, ny, nz: cells; dir: Dirichlet face bits; ext/off: NCE lattice extents and
// component offsets; cell_key: key of every cell; conds: the condensation of every
// key (with S).  Returns false with a message on a non-positive pivot.
bool edge_patches_build(int p, const int n[3], unsigned dir, const int ext[3][3], const int64_t off[4],
                        const VecLocal &L, const std::vector<int> &cell_key, const std::vector<CellCondensed> &conds,
                        EdgePatches &out, std::string &err);

}  // namespace rz
