// Symbolic static-condensation pattern of a vertex-star interface patch
// (Sec. 4.4 Remark: the Schur complement of the auxiliary operator keeps the
// Cartesian sparsity; Sec. 4.5: incomplete Cholesky restricted to that pattern).
// An entry (r, c) is in the pattern iff some cell of the star contains both DoFs
// and they are coupled in that cell's Schur complement (lattice.hpp).
#include "patch.hpp"

#include <algorithm>
#include <array>

#include "lattice.hpp"

namespace rz {

void build_patch_symbolic(int p, PatchSymbolic &ps) {
  ps.p = p;
  const int n = patch_nrows(p);
  ps.nrows = n;
  ps.off.assign(3 * n, 0);
  for (int k = 0; k < n; ++k) patch_offsets(p, k, ps.off[3 * k], ps.off[3 * k + 1], ps.off[3 * k + 2]);
  std::vector<std::vector<int>> rows(n);
  for (int r = 0; r < n; ++r) {
    for (int c = 0; c <= r; ++c) {
      bool coupled = (r == c);
      for (int cell = 0; cell < 8 && !coupled; ++cell) {
        int o[3] = {(cell & 1) ? 0 : -p, (cell & 2) ? 0 : -p, (cell & 4) ? 0 : -p};
        int u[3], w[3];
        bool in = true;
        for (int a = 0; a < 3; ++a) {
          u[a] = ps.off[3 * r + a] - o[a];
          w[a] = ps.off[3 * c + a] - o[a];
          if (u[a] < 0 || u[a] > p || w[a] < 0 || w[a] > p) in = false;
        }
        if (in && cell_schur_coupled(p, u, w)) coupled = true;
      }
      if (coupled) rows[r].push_back(c);
    }
  }
  ps.rowptr.assign(n + 1, 0);
  ps.col.clear();
  for (int r = 0; r < n; ++r) {
    ps.col.insert(ps.col.end(), rows[r].begin(), rows[r].end());
    ps.rowptr[r + 1] = (int)ps.col.size();
  }
  ps.nnz = (int)ps.col.size();
  // column access (transpose of the strictly lower part)
  std::vector<std::vector<std::pair<int, int>>> cols(n);
  for (int r = 0; r < n; ++r)
    for (int k = ps.rowptr[r]; k < ps.rowptr[r + 1] - 1; ++k) cols[ps.col[k]].push_back({r, k});
  ps.uptr.assign(n + 1, 0);
  ps.urow.clear();
  ps.upos.clear();
  for (int i = 0; i < n; ++i) {
    for (auto &e : cols[i]) {
      ps.urow.push_back(e.first);
      ps.upos.push_back(e.second);
    }
    ps.uptr[i + 1] = (int)ps.urow.size();
  }
  // level schedules
  std::vector<int> flev(n, 0), blev(n, 0);
  int fmax = 0, bmax = 0;
  for (int r = 0; r < n; ++r) {
    int l = 0;
    for (int k = ps.rowptr[r]; k < ps.rowptr[r + 1] - 1; ++k) l = std::max(l, flev[ps.col[k]] + 1);
    flev[r] = l;
    fmax = std::max(fmax, l);
  }
  for (int r = n - 1; r >= 0; --r) {
    int l = 0;
    for (int k = ps.uptr[r]; k < ps.uptr[r + 1]; ++k) l = std::max(l, blev[ps.urow[k]] + 1);
    blev[r] = l;
    bmax = std::max(bmax, l);
  }
  auto group = [n](const std::vector<int> &lev, int lmax, std::vector<int> &ptr, std::vector<int> &rws) {
    ptr.assign(lmax + 2, 0);
    rws.clear();
    for (int l = 0; l <= lmax; ++l) {
      for (int r = 0; r < n; ++r)
        if (lev[r] == l) rws.push_back(r);
      ptr[l + 1] = (int)rws.size();
    }
  };
  group(flev, fmax, ps.flev_ptr, ps.flev_rows);
  group(blev, bmax, ps.blev_ptr, ps.blev_rows);
  // storage order for the level-parallel solve
  ps.nlev = fmax + 1;
  ps.level = flev;
  ps.noff = ps.nnz - n;
  ps.perm.assign(ps.nnz, -1);
  // off-diagonal entries sorted by (level of the row, row, column)
  std::vector<std::array<int, 4>> offd;  // level, row, col, csr position
  for (int r = 0; r < n; ++r)
    for (int k = ps.rowptr[r]; k < ps.rowptr[r + 1]; ++k) {
      int c = ps.col[k];
      if (c == r) ps.perm[k] = r;
      else offd.push_back({flev[r], r, c, k});
    }
  std::sort(offd.begin(), offd.end());
  ps.rc.resize(offd.size());
  ps.fcol.resize(offd.size());
  ps.fptr.assign(n + 1, 0);
  std::vector<std::vector<std::pair<int, int>>> colent(n);  // (j, storage index)
  for (size_t e = 0; e < offd.size(); ++e) {
    int r = offd[e][1], c = offd[e][2], k = offd[e][3];
    ps.perm[k] = n + (int)e;
    ps.rc[e] = r | (c << 10) | (flev[r] << 20);
    ps.fcol[e] = c;
    ps.fptr[r + 1]++;
    colent[c].push_back({r, (int)e});
  }
  // rows of one level are contiguous and ordered, so the counts turn into offsets
  // in level order; fptr is indexed by row
  {
    std::vector<int> start(n, 0);
    for (size_t e = 0; e < offd.size(); ++e) {
      int r = offd[e][1];
      if (e == 0 || offd[e - 1][1] != r) start[r] = (int)e;
    }
    std::vector<int> cnt(ps.fptr.begin() + 1, ps.fptr.end());
    ps.fptr.assign(2 * n, 0);  // (start, end) per row
    for (int r = 0; r < n; ++r) {
      ps.fptr[2 * r] = cnt[r] ? start[r] : 0;
      ps.fptr[2 * r + 1] = ps.fptr[2 * r] + cnt[r];
    }
  }
  ps.bptr.assign(n + 1, 0);
  ps.blist.clear();
  for (int i = 0; i < n; ++i) {
    std::sort(colent[i].begin(), colent[i].end());
    for (auto &pr : colent[i]) ps.blist.push_back(pr.second | (pr.first << 16));
    ps.bptr[i + 1] = (int)ps.blist.size();
  }
}

}  // namespace rz
