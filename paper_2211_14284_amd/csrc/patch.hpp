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
  int nlev = 0, noff = 0;          // forward levels, off-diagonal entries
  std::vector<int> level;          // forward level of every row

  // Wavefront schedule of the two sweeps (one 64-lane wavefront per patch).  A
  // pass works on up to 64/G rows of one forward level, G lanes each; lane j*G+q
  // takes entries q, q+G, ... of its row (from a rotation of its column list), so
  // step s of the pass has index table position base + 64 s + lane (ecol) and
  // value position ell0 + ell_pos(base, K, s, lane).  A slot's factor values are
  // [diagonal (nrows)] [pad to even] [ELL (ef)], padding zero.  The forward sweep runs the passes in order, each row gathering
  // its entries (L z = r); the backward sweep runs the same passes in reverse, each
  // row first finishing x_j = w_j / L_jj and then pushing L_ji x_j to its columns
  // (L^T x = z), so the off-diagonals are stored and streamed once per sweep.
  static constexpr int kLanes = 64, kMaxSteps = 8;
  int npass = 0, nfpass = 0, ef = 0, eb = 0, stride = 0;  // eb = 0, npass = nfpass
  int ell0 = 0;  // offset of the ELL values in a slot (nrows rounded up to even)
  std::vector<int> pass_g, pass_k, pass_base;  // per pass: lanes per row, steps, ELL offset
  std::vector<int> ecol;   // ef: index of the x entry read at each ELL position (padding 0)
  std::vector<int> erow;   // npass*64: row solved by the lane's group (-1: none)
  std::vector<int> pos1;   // nnz: CSR entry -> value position in the slot (diagonal or ELL)
  std::vector<int> pos2;   // nnz: all -1 (no second copy of the off-diagonals)
};

// Value position (relative to ell0) of step s of lane `lane` in a pass with ELL
// offset base and K steps: steps 2g and 2g + 1 of a lane are adjacent, so that one
// 16-byte (FP64) or 8-byte (FP32) load per lane fetches both (fully coalesced
// across the wavefront); an odd last step stands alone.
inline int ell_pos(int base, int K, int s, int lane) {
  return s < (K & ~1) ? base + 128 * (s >> 1) + 2 * lane + (s & 1) : base + 64 * s + lane;
}
// Build the layout and the static-condensation pattern of a full (untruncated)
// interior vertex patch on a Cartesian mesh.
void build_patch_symbolic(int p, PatchSymbolic &ps);
// The wavefront schedule (called by build_patch_symbolic).
void build_wave_schedule(PatchSymbolic &ps);

}  // namespace rz
