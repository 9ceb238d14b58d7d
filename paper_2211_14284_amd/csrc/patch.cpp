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
  ps.nlev = fmax + 1;
  ps.level = flev;
  ps.noff = ps.nnz - n;
  build_wave_schedule(ps);
}

// Lay out one level's rows in passes.  items: (row, list of (CSR entry, x index)).
// G is the power of two that minimises the padded size with at most kMaxSteps
// steps per pass (ties: the smaller G).
static void schedule_level(PatchSymbolic &ps, std::vector<std::pair<int, std::vector<std::pair<int, int>>>> items) {
  const int W = PatchSymbolic::kLanes, KM = PatchSymbolic::kMaxSteps;
  std::stable_sort(items.begin(), items.end(),
                   [](const auto &a, const auto &b) { return a.second.size() > b.second.size(); });
  const int n = (int)items.size();
  if (n == 0) return;
  int bestG = -1;
  long best = 0;
  for (int G = 1; G <= W; G *= 2) {
    const int R = W / G;
    long tot = 0;
    bool ok = true;
    for (int t = 0; t < n; t += R) {
      const int K = ((int)items[t].second.size() + G - 1) / G;
      if (K > KM) ok = false;
      tot += (long)W * K;
    }
    if (ok && (bestG < 0 || tot < best)) {
      bestG = G;
      best = tot;
    }
  }
  const int G = bestG, R = W / G;
  for (int t = 0; t < n; t += R) {
    const int K = ((int)items[t].second.size() + G - 1) / G;
    const int base = (int)ps.ecol.size();
    ps.pass_g.push_back(G);
    ps.pass_k.push_back(K);
    ps.pass_base.push_back(base);
    ps.ecol.resize(base + (size_t)W * K, 0);
    const size_t r0 = ps.erow.size();
    ps.erow.resize(r0 + W, -1);
    // Row j's entries start at a rotation of j G: the rows of a level share many
    // columns, and the rotation spreads a column over different steps, so that the
    // backward sweep's pushes of one step hit fewer equal addresses.
    for (int j = 0; j < R && t + j < n; ++j) {
      const auto &it = items[t + j];
      const int len = (int)it.second.size();
      for (int q = 0; q < G; ++q) ps.erow[r0 + j * G + q] = it.first;
      for (int m = 0; m < len; ++m) {
        const auto &e = it.second[(m + j * G) % len];
        const int s = m / G, lane = j * G + (m % G);
        ps.ecol[base + s * W + lane] = e.second;
        ps.pos1[e.first] = ps.ell0 + ell_pos(base, K, s, lane);
      }
    }
  }
}

void build_wave_schedule(PatchSymbolic &ps) {
  const int n = ps.nrows;
  ps.pos1.assign(ps.nnz, -1);
  ps.pos2.assign(ps.nnz, -1);
  ps.pass_g.clear();
  ps.pass_k.clear();
  ps.pass_base.clear();
  ps.ecol.clear();
  ps.erow.clear();
  ps.ell0 = (n + 1) & ~1;
  for (int r = 0; r < n; ++r) ps.pos1[ps.rowptr[r + 1] - 1] = r;  // diagonal
  // forward: row i gathers L_ij x_j, j < i
  for (int l = 0; l < ps.nlev; ++l) {
    std::vector<std::pair<int, std::vector<std::pair<int, int>>>> items;
    for (int r = 0; r < n; ++r)
      if (ps.level[r] == l) {
        std::vector<std::pair<int, int>> e;
        for (int k = ps.rowptr[r]; k < ps.rowptr[r + 1] - 1; ++k) e.push_back({k, ps.col[k]});
        items.push_back({r, e});
      }
    schedule_level(ps, items);
  }
  ps.nfpass = (int)ps.pass_g.size();
  ps.ef = (int)ps.ecol.size();
  // the backward sweep reuses these passes in reverse (push form): no second copy
  ps.npass = ps.nfpass;
  ps.eb = 0;
  ps.stride = ps.ell0 + ps.ef;
}

}  // namespace rz
