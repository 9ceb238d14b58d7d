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
  // for the IC factorisation: rows grouped by forward level (same as flev)
};

// Build the layout and the static-condensation pattern of a full (untruncated)
// interior vertex patch on a Cartesian mesh.
void build_patch_symbolic(int p, PatchSymbolic &ps);

}  // namespace rz
