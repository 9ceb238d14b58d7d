// 1-D FDM element on [-1,1] (Sec. 2.2: eqs. fdmbasis, fdmdualbasis, unisolvence,
// eigs; Sec. 2.3: DP_{p-1} basis and differentiation matrix; Sec. 3.2: broken
// basis).  Host FP64, computed once per degree at setup.
//
// Conventions fixed here (the paper leaves them open): eigenvalues ascending,
// eigenvector sign with s_j'(-1) > 0, broken interface pair
// s_pm = (s_0 +- s_p)/sqrt(2 (B_00 +- B_0p)) at broken indices 0 and p.
// Entries that the definitions fix exactly are set exactly: B_II = I, B_IG = 0,
// A_II = diag(lambda), D_II = diag(sqrt(lambda)), D row 0 = (-1/sqrt2, 0.., 1/sqrt2).
#include "tables1d.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace rz {

namespace {

// Legendre P_n and P_n' at x by the three-term recurrence.
void legendre(int n, double x, double &P, double &dP) {
  double p0 = 1.0, p1 = x;
  if (n == 0) { P = 1.0; dP = 0.0; return; }
  for (int k = 2; k <= n; ++k) {
    double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  P = p1;
  // (1-x^2) P_n' = n (P_{n-1} - x P_n)
  dP = n * (p0 - x * p1) / (1.0 - x * x);
}

// Lagrange polynomials on `nodes`: value and derivative of l_i at x.
void lagrange(const std::vector<double> &nodes, double x, std::vector<double> &l,
              std::vector<double> &dl) {
  const int n = (int)nodes.size();
  l.assign(n, 0.0);
  dl.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double v = 1.0;
    for (int k = 0; k < n; ++k)
      if (k != i) v *= (x - nodes[k]) / (nodes[i] - nodes[k]);
    l[i] = v;
    double d = 0.0;
    for (int m = 0; m < n; ++m) {
      if (m == i) continue;
      double t = 1.0 / (nodes[i] - nodes[m]);
      for (int k = 0; k < n; ++k)
        if (k != i && k != m) t *= (x - nodes[k]) / (nodes[i] - nodes[k]);
      d += t;
    }
    dl[i] = d;
  }
}

// Cyclic Jacobi eigenvalue iteration for a symmetric n x n matrix (row-major).
// On exit a holds the eigenvalues on its diagonal and v the eigenvectors (columns).
void jacobi_eigen(int n, std::vector<double> &a, std::vector<double> &v) {
  v.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) v[i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j)
        (i == j ? diag : off) += a[i * n + j] * a[i * n + j];
    if (off <= 1e-34 * diag) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = a[p * n + q];
        if (apq == 0.0) continue;
        double theta = (a[q * n + q] - a[p * n + p]) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {  // columns p, q
          double akp = a[k * n + p], akq = a[k * n + q];
          a[k * n + p] = c * akp - s * akq;
          a[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          double apk = a[p * n + k], aqk = a[q * n + k];
          a[p * n + k] = c * apk - s * aqk;
          a[q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          double vkp = v[k * n + p], vkq = v[k * n + q];
          v[k * n + p] = c * vkp - s * vkq;
          v[k * n + q] = s * vkp + c * vkq;
        }
      }
  }
}

}  // namespace

void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre(n, z, P, dP);
      double dz = P / dP;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double P, dP;
    legendre(n, z, P, dP);
    x[n - 1 - i] = z;
    w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dP * dP);
  }
}

static void gll_nodes(int p, std::vector<double> &xi) {
  xi.assign(p + 1, 0.0);
  xi[0] = -1.0;
  xi[p] = 1.0;
  for (int i = 1; i < p; ++i) {
    // interior roots of P_p': Newton on f = P_p' with f' from the Legendre ODE
    double z = -std::cos(M_PI * i / p);
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre(p, z, P, dP);
      double d2P = (2.0 * z * dP - p * (p + 1.0) * P) / (1.0 - z * z);
      double dz = dP / d2P;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    xi[i] = z;
  }
  std::sort(xi.begin(), xi.end());
}

void gll_rule(int q, std::vector<double> &x, std::vector<double> &w) {
  gll_nodes(q - 1, x);
  w.assign(q, 0.0);
  for (int i = 0; i < q; ++i) {
    double P, dP;
    legendre(q - 1, x[i], P, dP);
    w[i] = 2.0 / (q * (q - 1.0) * P * P);
  }
}

bool build_tables1d(int p, Tables1D &t) {
  if (p < 1 || p > 16) return false;
  const int n = p + 1;
  t.p = p;
  gll_nodes(p, t.gll);
  // exact GLL mass and stiffness with p+2 Gauss-Legendre points
  std::vector<double> xq, wq;
  gauss_legendre(p + 2, xq, wq);
  std::vector<double> Bg(n * n, 0.0), Ag(n * n, 0.0), l, dl;
  std::vector<std::vector<double>> Lq, dLq;
  for (size_t q = 0; q < xq.size(); ++q) {
    lagrange(t.gll, xq[q], l, dl);
    Lq.push_back(l);
    dLq.push_back(dl);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        Bg[i * n + j] += wq[q] * l[i] * l[j];
        Ag[i * n + j] += wq[q] * dl[i] * dl[j];
      }
  }
  // generalised eigenproblem on the interior block (eq. eigs):
  // B_II = L L^T, C = L^{-1} A_II L^{-T}, C y = lam y, s = L^{-T} y
  const int m = p - 1;
  std::vector<double> S(n * n, 0.0);
  S[0] = 1.0;
  S[p * n + p] = 1.0;
  t.lam.assign(m, 0.0);
  if (m > 0) {
    std::vector<double> Lc(m * m, 0.0);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j <= i; ++j) {
        double s = Bg[(i + 1) * n + (j + 1)];
        for (int k = 0; k < j; ++k) s -= Lc[i * m + k] * Lc[j * m + k];
        if (i == j) {
          if (s <= 0) return false;
          Lc[i * m + i] = std::sqrt(s);
        } else {
          Lc[i * m + j] = s / Lc[j * m + j];
        }
      }
    // X = L^{-1} A_II (forward substitution per column), C = X L^{-T}
    std::vector<double> X(m * m), C(m * m);
    for (int c = 0; c < m; ++c)
      for (int i = 0; i < m; ++i) {
        double s = Ag[(i + 1) * n + (c + 1)];
        for (int k = 0; k < i; ++k) s -= Lc[i * m + k] * X[k * m + c];
        X[i * m + c] = s / Lc[i * m + i];
      }
    for (int r = 0; r < m; ++r)
      for (int i = 0; i < m; ++i) {
        double s = X[r * m + i];
        for (int k = 0; k < i; ++k) s -= Lc[i * m + k] * C[r * m + k];
        C[r * m + i] = s / Lc[i * m + i];
      }
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < i; ++j) C[i * m + j] = C[j * m + i] = 0.5 * (C[i * m + j] + C[j * m + i]);
    std::vector<double> V;
    jacobi_eigen(m, C, V);
    std::vector<int> order(m);
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(), [&](int a, int b) { return C[a * m + a] < C[b * m + b]; });
    // derivative of the Lagrange basis at -1 for the sign rule
    lagrange(t.gll, -1.0, l, dl);
    for (int jj = 0; jj < m; ++jj) {
      int src = order[jj];
      t.lam[jj] = C[src * m + src];
      std::vector<double> y(m), s(m);
      for (int i = 0; i < m; ++i) y[i] = V[i * m + src];
      for (int i = m - 1; i >= 0; --i) {  // s = L^{-T} y
        double v = y[i];
        for (int k = i + 1; k < m; ++k) v -= Lc[k * m + i] * s[k];
        s[i] = v / Lc[i * m + i];
      }
      double slope = 0.0;
      for (int i = 0; i < m; ++i) slope += dl[i + 1] * s[i];
      double sg = slope > 0 ? 1.0 : -1.0;
      for (int i = 0; i < m; ++i) S[(i + 1) * n + (jj + 1)] = sg * s[i];
    }
    // S_IG = -S_II S_II^T B_IG
    for (int g = 0; g < 2; ++g) {
      int col = g == 0 ? 0 : p;
      std::vector<double> tmp(m, 0.0);  // S_II^T B_I,col
      for (int j = 0; j < m; ++j)
        for (int i = 0; i < m; ++i) tmp[j] += S[(i + 1) * n + (j + 1)] * Bg[(i + 1) * n + col];
      for (int i = 0; i < m; ++i) {
        double v = 0.0;
        for (int j = 0; j < m; ++j) v += S[(i + 1) * n + (j + 1)] * tmp[j];
        S[(i + 1) * n + col] = -v;
      }
    }
  }
  t.S = S;
  // B = S^T Bg S, A = S^T Ag S
  auto congruence = [&](const std::vector<double> &M) {
    std::vector<double> T(n * n, 0.0), R(n * n, 0.0);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j)
        for (int k = 0; k < n; ++k) T[i * n + j] += M[i * n + k] * S[k * n + j];
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j)
        for (int k = 0; k < n; ++k) R[i * n + j] += S[k * n + i] * T[k * n + j];
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < i; ++j) R[i * n + j] = R[j * n + i] = 0.5 * (R[i * n + j] + R[j * n + i]);
    return R;
  };
  t.B = congruence(Bg);
  t.A = congruence(Ag);
  // D[i][j] = (r_i, s_j') by quadrature, r_0 = 2^{-1/2}, r_i = lam_i^{-1/2} s_i'
  t.D.assign(p * n, 0.0);
  for (size_t q = 0; q < xq.size(); ++q) {
    std::vector<double> ds(n, 0.0);
    for (int j = 0; j < n; ++j)
      for (int k = 0; k < n; ++k) ds[j] += dLq[q][k] * S[k * n + j];
    for (int i = 0; i < p; ++i) {
      double ri = i == 0 ? std::sqrt(0.5) : ds[i] / std::sqrt(t.lam[i - 1]);
      for (int j = 0; j < n; ++j) t.D[i * n + j] += wq[q] * ri * ds[j];
    }
  }
  // exact entries fixed by the definitions
  for (int i = 1; i < p; ++i) {
    for (int j = 1; j < p; ++j) {
      t.B[i * n + j] = i == j ? 1.0 : 0.0;
      t.A[i * n + j] = i == j ? t.lam[i - 1] : 0.0;
      t.D[i * n + j] = i == j ? std::sqrt(t.lam[i - 1]) : 0.0;
    }
    t.B[i * n + 0] = t.B[0 * n + i] = 0.0;
    t.B[i * n + p] = t.B[p * n + i] = 0.0;
  }
  for (int j = 0; j < n; ++j) t.D[j] = 0.0;
  t.D[0] = -std::sqrt(0.5);
  t.D[p] = std::sqrt(0.5);
  // embedding of the linear hats: rows 0, p identity; interior rows (s_i, hat_j)
  t.E.assign(n * 2, 0.0);
  t.E[0 * 2 + 0] = 1.0;
  t.E[p * 2 + 1] = 1.0;
  {
    std::vector<double> x2, w2;
    gauss_legendre(p + 3, x2, w2);
    for (size_t q = 0; q < x2.size(); ++q) {
      lagrange(t.gll, x2[q], l, dl);
      for (int i = 1; i < p; ++i) {
        double si = 0.0;
        for (int k = 0; k < n; ++k) si += l[k] * S[k * n + i];
        t.E[i * 2 + 0] += w2[q] * si * 0.5 * (1.0 - x2[q]);
        t.E[i * 2 + 1] += w2[q] * si * 0.5 * (1.0 + x2[q]);
      }
    }
  }
  // broken basis transformation
  double np_ = std::sqrt(2.0 * (t.B[0] + t.B[p])), nm_ = std::sqrt(2.0 * (t.B[0] - t.B[p]));
  t.G.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i) t.G[i * n + i] = 1.0;
  t.G[0] = t.G[p] = 0.5 * np_;
  t.G[p * n + 0] = 0.5 * nm_;
  t.G[p * n + p] = -0.5 * nm_;
  return true;
}

void fdm_eval(const Tables1D &t, const std::vector<double> &x, std::vector<double> &val,
              std::vector<double> &der) {
  const int n = t.p + 1;
  val.assign(x.size() * n, 0.0);
  der.assign(x.size() * n, 0.0);
  std::vector<double> l, dl;
  for (size_t q = 0; q < x.size(); ++q) {
    lagrange(t.gll, x[q], l, dl);
    for (int j = 0; j < n; ++j)
      for (int k = 0; k < n; ++k) {
        val[q * n + j] += l[k] * t.S[k * n + j];
        der[q * n + j] += dl[k] * t.S[k * n + j];
      }
  }
}

}  // namespace rz
