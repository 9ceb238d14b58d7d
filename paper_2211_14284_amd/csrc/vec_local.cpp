// Host-side cell algebra of the H(curl) / H(div) relaxation (see vec_local.hpp).
#include "vec_local.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>

namespace rz {

void vec_local_layout(int space, int p, VecLocal &L) {
  L.space = space;
  L.p = p;
  int o = 0;
  for (int m = 0; m < 3; ++m) {
    L.off[m] = o;
    int s = 1;
    for (int a = 0; a < 3; ++a) {
      L.ext[m][a] = vec_is_P(space, m, a) ? p + 1 : p;
      s *= L.ext[m][a];
    }
    o += s;
  }
  L.off[3] = o;
  L.nloc = o;
  L.comp.resize(o);
  L.crd.resize(3 * (size_t)o);
  L.interior.resize(o);
  for (int m = 0; m < 3; ++m)
    for (int k = L.off[m]; k < L.off[m + 1]; ++k) {
      const int r = k - L.off[m];
      const int c[3] = {r % L.ext[m][0], (r / L.ext[m][0]) % L.ext[m][1], r / (L.ext[m][0] * L.ext[m][1])};
      L.comp[k] = m;
      bool in = true;
      for (int a = 0; a < 3; ++a) {
        L.crd[3 * k + a] = c[a];
        if (vec_is_P(space, m, a) && (c[a] == 0 || c[a] == p)) in = false;
      }
      L.interior[k] = in;
    }
}

namespace {

// One factor of a 1-D pairing along an axis of a target field.  An operand along the
// axis is a continuous function (kind 0), the derivative of a continuous function
// (kind 1, which lies in the broken space through D) or a broken function (kind 2).
// A continuous target pairs two continuous values with the mass B; a broken target
// pairs the broken coefficients (orthonormal r basis: identity).
struct Pair1D {
  const Tables1D &t;
  int p;
  double operator()(bool tgtP, int ku, int a, int kv, int b) const {
    const int n1 = p + 1;
    if (tgtP) return (ku == 0 && kv == 0) ? t.B[a * n1 + b] : 0.0;
    if (ku == 2 && kv == 2) return a == b ? 1.0 : 0.0;
    if (ku == 1 && kv == 2) return t.D[b * n1 + a];
    if (ku == 2 && kv == 1) return t.D[a * n1 + b];
    if (ku == 1 && kv == 1) {
      double s = 0.0;
      for (int j = 0; j < p; ++j) s += t.D[j * n1 + a] * t.D[j * n1 + b];
      return s;
    }
    return 0.0;
  }
};

// a term sgn * d_{deriv} u_{comp} of a derived field (deriv < 0: the value itself)
struct Term {
  int sgn, comp, deriv;
};

}  // namespace

void vec_basis_matrices(const Tables1D &t, const VecLocal &L, SpRows basis[6]) {
  const int p = L.p, space = L.space;
  const Pair1D pair{t, p};
  for (int k = 0; k < 6; ++k) basis[k].assign(L.nloc, SpRow());
  // target field kinds along each axis and the terms that produce it from u
  struct Field {
    bool tgtP[3];
    std::vector<Term> terms;
  };
  std::vector<std::pair<int, Field>> fields;  // (basis index, field)
  for (int m = 0; m < 3; ++m) {               // mass of component m
    Field f;
    for (int a = 0; a < 3; ++a) f.tgtP[a] = vec_is_P(space, m, a);
    f.terms.push_back({1, m, -1});
    fields.push_back({3 + m, f});
  }
  if (space == 1) {
    for (int n = 0; n < 3; ++n) {  // curl component n = d_{a1} u_{a2} - d_{a2} u_{a1}
      const int a1 = (n + 1) % 3, a2 = (n + 2) % 3;
      Field f;
      for (int a = 0; a < 3; ++a) f.tgtP[a] = a == n;  // NCF component n
      f.terms.push_back({1, a2, a1});
      f.terms.push_back({-1, a1, a2});
      fields.push_back({n, f});
    }
  } else {
    Field f;  // divergence = sum_m d_m u_m, broken along every axis
    for (int a = 0; a < 3; ++a) f.tgtP[a] = false;
    for (int m = 0; m < 3; ++m) f.terms.push_back({1, m, m});
    fields.push_back({0, f});
  }
  auto kind = [&](const Term &tm, int a) {
    if (a == tm.deriv) return 1;
    return vec_is_P(space, tm.comp, a) ? 0 : 2;
  };
  for (auto &bf : fields) {
    const Field &f = bf.second;
    SpRows &M = basis[bf.first];
    for (const Term &tu : f.terms)
      for (const Term &tv : f.terms) {
        const int cu = tu.comp, cv = tv.comp;
        for (int u = L.off[cu]; u < L.off[cu + 1]; ++u)
          for (int v = L.off[cv]; v < L.off[cv + 1]; ++v) {
            double val = tu.sgn * tv.sgn;
            for (int a = 0; a < 3 && val != 0.0; ++a)
              val *= pair(f.tgtP[a], kind(tu, a), L.crd[3 * u + a], kind(tv, a), L.crd[3 * v + a]);
            if (val != 0.0) M[u].push_back({v, val});
          }
      }
    for (SpRow &row : M) {  // merge duplicate columns (several term pairs)
      std::sort(row.begin(), row.end(), [](const std::pair<int, double> &x, const std::pair<int, double> &y) {
        return x.first < y.first;
      });
      SpRow out;
      for (auto &e : row) {
        if (!out.empty() && out.back().first == e.first) out.back().second += e.second;
        else out.push_back(e);
      }
      row.swap(out);
    }
  }
}

bool vec_condense(const VecLocal &L, const SpRows basis[6], const double w[6], bool want_S, CellCondensed &out,
                  std::string &err) {
  const int n = L.nloc;
  // A = sum_k w_k K_k on the union of the basis patterns
  SpRows A(n);
  std::vector<double> acc(n, 0.0);
  std::vector<char> mark(n, 0);
  std::vector<int> cols;
  for (int r = 0; r < n; ++r) {
    cols.clear();
    for (int k = 0; k < 6; ++k)
      for (auto &e : basis[k][r]) {
        if (!mark[e.first]) {
          mark[e.first] = 1;
          cols.push_back(e.first);
        }
        acc[e.first] += w[k] * e.second;
      }
    std::sort(cols.begin(), cols.end());
    for (int c : cols) {
      A[r].push_back({c, acc[c]});
      acc[c] = 0.0;
      mark[c] = 0;
    }
  }
  out.I.clear();
  out.G.clear();
  out.gpos.assign(n, -1);
  std::vector<int> ipos(n, -1);
  for (int k = 0; k < n; ++k) {
    if (L.interior[k]) {
      ipos[k] = (int)out.I.size();
      out.I.push_back(k);
    } else {
      out.gpos[k] = (int)out.G.size();
      out.G.push_back(k);
    }
  }
  const int nI = (int)out.I.size(), nG = (int)out.G.size();
  // blocks of P_II: connected components of its pattern (union-find)
  std::vector<int> par(nI);
  for (int i = 0; i < nI; ++i) par[i] = i;
  auto find = [&](int x) {
    while (par[x] != x) x = par[x] = par[par[x]];
    return x;
  };
  for (int i = 0; i < nI; ++i)
    for (auto &e : A[out.I[i]])
      if (ipos[e.first] >= 0) {
        int a = find(i), b = find(ipos[e.first]);
        if (a != b) par[std::max(a, b)] = std::min(a, b);
      }
  std::map<int, std::vector<int>> comps;
  for (int i = 0; i < nI; ++i) comps[find(i)].push_back(i);
  out.blocks.clear();
  out.linv.clear();
  for (auto &cmp : comps) {
    const std::vector<int> &rows = cmp.second;  // ascending I positions
    const int b = (int)rows.size();
    if (b > 3) {
      err = "the interior block of a cell operator exceeds 3 x 3";
      return false;
    }
    double M[3][3] = {{0}}, Lf[3][3] = {{0}}, Li[3][3] = {{0}};
    for (int r = 0; r < b; ++r)
      for (auto &e : A[out.I[rows[r]]])
        for (int c = 0; c < b; ++c)
          if (ipos[e.first] == rows[c]) M[r][c] = e.second;
    for (int j = 0; j < b; ++j) {  // Cholesky
      double d = M[j][j];
      for (int k = 0; k < j; ++k) d -= Lf[j][k] * Lf[j][k];
      if (!(d > 0.0)) {
        err = "an interior block of a cell operator is not positive definite";
        return false;
      }
      Lf[j][j] = std::sqrt(d);
      for (int i = j + 1; i < b; ++i) {
        double s = M[i][j];
        for (int k = 0; k < j; ++k) s -= Lf[i][k] * Lf[j][k];
        Lf[i][j] = s / Lf[j][j];
      }
    }
    for (int j = 0; j < b; ++j) {  // L^{-1} column by column (forward substitution)
      for (int i = 0; i < b; ++i) {
        double s = i == j ? 1.0 : 0.0;
        for (int k = j; k < i; ++k) s -= Lf[i][k] * Li[k][j];
        Li[i][j] = i < j ? 0.0 : s / Lf[i][i];
      }
    }
    std::array<int, 3> blk = {-1, -1, -1};
    for (int r = 0; r < b; ++r) blk[r] = rows[r];
    out.blocks.push_back(blk);
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) out.linv.push_back(r < b && c < b ? Li[r][c] : 0.0);
  }
  // P_GI and P_IG with the structural pattern
  out.gi_ptr.assign(1, 0);
  out.gi_col.clear();
  out.gi_val.clear();
  for (int g = 0; g < nG; ++g) {
    for (auto &e : A[out.G[g]])
      if (ipos[e.first] >= 0) {
        out.gi_col.push_back(ipos[e.first]);
        out.gi_val.push_back(e.second);
      }
    out.gi_ptr.push_back((int)out.gi_col.size());
  }
  out.ig_ptr.assign(1, 0);
  out.ig_col.clear();
  out.ig_val.clear();
  for (int i = 0; i < nI; ++i) {
    for (auto &e : A[out.I[i]])
      if (out.gpos[e.first] >= 0) {
        out.ig_col.push_back(out.gpos[e.first]);
        out.ig_val.push_back(e.second);
      }
    out.ig_ptr.push_back((int)out.ig_col.size());
  }
  if (!want_S) return true;
  // S = P_GG - W^T W with W = L^{-1} P_IG, block by block
  out.S.assign((size_t)nG * nG, 0.0);
  for (int g = 0; g < nG; ++g)
    for (auto &e : A[out.G[g]])
      if (out.gpos[e.first] >= 0) out.S[(size_t)g * nG + out.gpos[e.first]] = e.second;
  std::vector<double> wrow(nG, 0.0);
  std::vector<int> wcols;
  std::vector<char> wmark(nG, 0);
  for (size_t bi = 0; bi < out.blocks.size(); ++bi) {
    const std::array<int, 3> &blk = out.blocks[bi];
    const double *Li = &out.linv[9 * bi];
    for (int r = 0; r < 3 && blk[r] >= 0; ++r) {
      wcols.clear();
      for (int c = 0; c <= r; ++c) {
        const int i = blk[c];
        for (int k = out.ig_ptr[i]; k < out.ig_ptr[i + 1]; ++k) {
          const int g = out.ig_col[k];
          if (!wmark[g]) {
            wmark[g] = 1;
            wcols.push_back(g);
          }
          wrow[g] += Li[3 * r + c] * out.ig_val[k];
        }
      }
      for (int g1 : wcols)
        for (int g2 : wcols) out.S[(size_t)g1 * nG + g2] -= wrow[g1] * wrow[g2];
      for (int g : wcols) {
        wrow[g] = 0.0;
        wmark[g] = 0;
      }
    }
  }
  return true;
}

void edge_layout(int p, EdgeLayout &E) {
  E.p = p;
  E.blk_n.resize(p);
  E.blk_slot.resize(p);
  E.blk_fac.resize(p);
  int s = 0, f = 0;
  for (int i = 0; i < p; ++i) {
    const int nb = i == 0 ? 4 * p - 3 : 8 * p - 3;
    E.blk_n[i] = nb;
    E.blk_slot[i] = s;
    E.blk_fac[i] = f;
    s += nb;
    f += nb * (nb + 1);
  }
  E.nslot = s;
  E.fac_stride = f;
}

namespace {

// Dirichlet test of an NCE_p lattice DoF (tangential trace on a Dirichlet face).
bool nce_dirichlet(unsigned dir, const int ext[3][3], int m, const int X[3]) {
  for (int a = 0; a < 3; ++a) {
    if (a == m) continue;
    if ((dir & (1u << (2 * a))) && X[a] == 0) return true;
    if ((dir & (1u << (2 * a + 1))) && X[a] == ext[m][a] - 1) return true;
  }
  return false;
}

}  // namespace

bool edge_patches_build(int p, const int n[3], unsigned dir, const int ext[3][3], const int64_t off[4],
                        const VecLocal &L, const std::vector<int> &cell_key, const std::vector<CellCondensed> &conds,
                        EdgePatches &out, std::string &err) {
  EdgeLayout &E = out.lay;
  edge_layout(p, E);
  const int ns = E.nslot;
  out.edge_id.clear();
  out.idx.clear();
  out.type.clear();
  out.fac.clear();
  std::map<std::vector<int>, int> types;
  // per slot: component and lattice coordinates
  std::vector<int> sc(ns), sX(3 * (size_t)ns);
  std::vector<char> sok(ns);
  const int64_t ndofs = off[3];
  std::vector<int> cnt(ndofs, 0);
  int64_t eoff = 0;
  for (int m = 0; m < 3; ++m) {
    const int a = m == 0 ? 1 : 0, b = m == 2 ? 1 : 2;  // the two other axes, ascending
    int ee[3];
    for (int d = 0; d < 3; ++d) ee[d] = d == m ? n[d] : n[d] + 1;
    for (int e2 = 0; e2 < ee[2]; ++e2)
      for (int e1 = 0; e1 < ee[1]; ++e1)
        for (int e0 = 0; e0 < ee[0]; ++e0) {
          const int ec[3] = {e0, e1, e2};
          const int cm = ec[m], va = ec[a], vb = ec[b];
          // slots
          int s = 0;
          auto put = [&](int comp, int Xm, int Xa, int Xb, bool exists) {
            int X[3];
            X[m] = Xm;
            X[a] = Xa;
            X[b] = Xb;
            sc[s] = comp;
            for (int d = 0; d < 3; ++d) sX[3 * s + d] = X[d];
            sok[s] = exists && !nce_dirichlet(dir, ext, comp, X);
            ++s;
          };
          for (int i = 0; i < p; ++i) {
            put(m, cm * p + i, va * p, vb * p, true);
            for (int sb = 0; sb < 2; ++sb) {
              const int cb = vb - 1 + sb;
              const bool ex = cb >= 0 && cb < n[b];
              for (int j = 1; j < p; ++j) put(m, cm * p + i, va * p, cb * p + j, ex);
              if (i >= 1)
                for (int j = 0; j < p; ++j) put(b, cm * p + i, va * p, cb * p + j, ex);
            }
            for (int sa = 0; sa < 2; ++sa) {
              const int ca = va - 1 + sa;
              const bool ex = ca >= 0 && ca < n[a];
              for (int j = 1; j < p; ++j) put(m, cm * p + i, ca * p + j, vb * p, ex);
              if (i >= 1)
                for (int j = 0; j < p; ++j) put(a, cm * p + i, ca * p + j, vb * p, ex);
            }
          }
          bool any = false;
          for (int k = 0; k < ns; ++k) any = any || sok[k];
          if (!any) continue;
          // the four cells of the star (quadrant q = sa + 2 sb) and their keys
          int qcell[4];
          std::vector<int> key = {m};
          for (int q = 0; q < 4; ++q) {
            int c[3];
            c[m] = cm;
            c[a] = va - 1 + (q & 1);
            c[b] = vb - 1 + (q >> 1);
            const bool in = c[a] >= 0 && c[a] < n[a] && c[b] >= 0 && c[b] < n[b];
            qcell[q] = in ? c[0] + n[0] * (c[1] + n[1] * c[2]) : -1;
            key.push_back(in ? cell_key[qcell[q]] : -1);
          }
          for (int k = 0; k < ns; ++k) key.push_back(sok[k]);
          const int pid = (int)out.edge_id.size();
          out.edge_id.push_back(eoff + ec[0] + (int64_t)ee[0] * (ec[1] + (int64_t)ee[1] * ec[2]));
          for (int k = 0; k < ns; ++k) {
            int g = -1;
            if (sok[k]) {
              const int c = sc[k];
              g = (int)(off[c] + sX[3 * k] + (int64_t)ext[c][0] * (sX[3 * k + 1] + (int64_t)ext[c][1] * sX[3 * k + 2]));
              cnt[g] += 1;
            }
            out.idx.push_back(g);
          }
          (void)pid;
          auto it = types.find(key);
          if (it != types.end()) {
            out.type.push_back(it->second);
            continue;
          }
          const int tid = (int)types.size();
          types[key] = tid;
          out.type.push_back(tid);
          // local interface position of every slot in every star cell (-1: not held)
          std::vector<int> lg(4 * (size_t)ns, -1);
          for (int q = 0; q < 4; ++q) {
            if (qcell[q] < 0) continue;
            int c[3];
            c[m] = cm;
            c[a] = va - 1 + (q & 1);
            c[b] = vb - 1 + (q >> 1);
            const CellCondensed &cc = conds[cell_key[qcell[q]]];
            for (int k = 0; k < ns; ++k) {
              if (!sok[k]) continue;
              const int comp = sc[k];
              int l[3];
              bool in = true;
              for (int d = 0; d < 3; ++d) {
                l[d] = sX[3 * k + d] - c[d] * p;
                in = in && l[d] >= 0 && l[d] < L.ext[comp][d];
              }
              if (!in) continue;
              const int loc = L.off[comp] + l[0] + L.ext[comp][0] * (l[1] + L.ext[comp][1] * l[2]);
              lg[(size_t)q * ns + k] = cc.gpos[loc];
            }
          }
          const size_t fo = out.fac.size();
          out.fac.resize(fo + E.fac_stride, 0.0);
          for (int i = 0; i < p; ++i) {
            const int nb = E.blk_n[i], s0 = E.blk_slot[i];
            std::vector<double> M((size_t)nb * nb, 0.0);
            for (int r = 0; r < nb; ++r) {
              if (!sok[s0 + r]) {
                M[(size_t)r * nb + r] = 1.0;
                continue;
              }
              for (int q = 0; q < 4; ++q) {
                const int gr = lg[(size_t)q * ns + s0 + r];
                if (gr < 0) continue;
                const CellCondensed &cc = conds[cell_key[qcell[q]]];
                const int nG = (int)cc.G.size();
                for (int c = 0; c < nb; ++c) {
                  const int gc = lg[(size_t)q * ns + s0 + c];
                  if (gc >= 0) M[(size_t)r * nb + c] += cc.S[(size_t)gr * nG + gc];
                }
              }
            }
            // Cholesky, stored by column: 1/L_jj then L_{j+1..nb-1, j}
            for (int j = 0; j < nb; ++j) {
              double d = M[(size_t)j * nb + j];
              for (int k = 0; k < j; ++k) d -= M[(size_t)j * nb + k] * M[(size_t)j * nb + k];
              if (!(d > 0.0)) {
                char msg[128];
                std::snprintf(msg, sizeof msg, "edge-star patch %lld: Cholesky pivot %d of block %d is not positive",
                              (long long)out.edge_id.back(), j, i);
                err = msg;
                return false;
              }
              const double ljj = std::sqrt(d);
              M[(size_t)j * nb + j] = ljj;
              for (int r = j + 1; r < nb; ++r) {
                double s2 = M[(size_t)r * nb + j];
                for (int k = 0; k < j; ++k) s2 -= M[(size_t)r * nb + k] * M[(size_t)j * nb + k];
                M[(size_t)r * nb + j] = s2 / ljj;
              }
            }
            // W = L^{-1} of the block's Cholesky factor (forward substitution, column
            // by column); the solve applies it twice, S^{-1} b = W^T (W b), which is as
            // accurate as the two triangular sweeps (the full inverse S^{-1} is not, for
            // the nearly singular curl-curl blocks).  Stored packed twice: by columns
            // (column c: rows c..n-1) for W b, by rows (row c: columns 0..c) for W^T y.
            std::vector<double> W((size_t)nb * nb, 0.0);
            for (int c = 0; c < nb; ++c)
              for (int r = c; r < nb; ++r) {
                double s2 = r == c ? 1.0 : 0.0;
                for (int k = c; k < r; ++k) s2 -= M[(size_t)r * nb + k] * W[(size_t)k * nb + c];
                W[(size_t)r * nb + c] = s2 / M[(size_t)r * nb + r];
              }
            double *dst = &out.fac[fo + E.blk_fac[i]];
            size_t o = 0;
            for (int c = 0; c < nb; ++c)
              for (int r = c; r < nb; ++r) dst[o++] = W[(size_t)r * nb + c];
            for (int r = 0; r < nb; ++r)
              for (int c = 0; c <= r; ++c) dst[o++] = W[(size_t)r * nb + c];
          }
        }
    eoff += (int64_t)ee[0] * ee[1] * ee[2];
  }
  // sum back: free interface DoFs in ascending order, their slots by ascending patch
  out.rows.clear();
  out.ptr.assign(1, 0);
  std::vector<int> start(ndofs, -1);
  for (int64_t g = 0; g < ndofs; ++g)
    if (cnt[g] > 0) {
      start[g] = out.ptr.back();
      out.rows.push_back((int)g);
      out.ptr.push_back(out.ptr.back() + cnt[g]);
    }
  out.pos.assign(out.ptr.back(), 0);
  std::vector<int> fill(ndofs, 0);
  const int npatch = (int)out.edge_id.size();
  for (int pid = 0; pid < npatch; ++pid)
    for (int k = 0; k < ns; ++k) {
      const int g = out.idx[(size_t)pid * ns + k];
      if (g >= 0) out.pos[start[g] + fill[g]++] = pid * ns + k;
    }
  return true;
}

}  // namespace rz
