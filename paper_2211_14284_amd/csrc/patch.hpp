// Symbolic data of the vertex-star interface patch of degree p (host).
#pragma once
#include <cstdint>
#include <vector>

namespace rz {

struct PatchSymbolic {
  int p = 0;
  int nrows = 0;
  int nnz = 0;                     // lower triangle including the diagonal
  std::vector<int> off;            // 3*nrows offsets (dx, dy, dz)
  // lower CSR, columns ascending, the diagonal is the last entry of each row
  std::vector<int> rowptr, col;
  // column access of the lower factor: for row i, the entries L_ji (j > i):
  // (row j, position of L_ji in the CSR value array), j ascending
  std::vector<int> uptr, urow, upos;
  // level schedules of the forward and backward triangular solves
  std::vector<int> flev_ptr, flev_rows, blev_ptr, blev_rows;
  // Storage order of a slot's factor values: the nrows diagonal entries (row
  // order), then the off-diagonal entries sorted by (forward level of the row,
  // row, column).  perm[k] = storage position of CSR entry k.
  int nlev = 0, noff = 0;
  std::vector<int> level;          // forward level of every row
  std::vector<int> perm;           // nnz
  std::vector<int> rc;             // noff packed entries: row | col << 10 | level(row) << 20
  // gather form of the two sweeps, in storage numbering of the off-diagonals:
  // row i's entries (L_ij, j < i) are fptr[2i] .. fptr[2i+1]-1 with columns fcol;
  // column i's entries (L_ji, j > i) are listed in blist[bptr[i] .. bptr[i+1]-1]
  // as (storage index | j << 16), j ascending
  std::vector<int> fptr, fcol, bptr, blist;
};

// Build the layout and the static-condensation pattern of a full (untruncated)
// interior vertex patch on a Cartesian mesh.
void build_patch_symbolic(int p, PatchSymbolic &ps);

}  // namespace rz
