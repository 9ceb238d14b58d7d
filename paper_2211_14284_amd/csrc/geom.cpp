// Host geometry of trilinear cells (see geom.hpp).
#include "geom.hpp"

#include <cmath>

namespace rz {

void build_quad_tables(const Tables1D &t, int q, QuadTables &Q) {
  Q.p = t.p;
  Q.q = q;
  gll_rule(q, Q.xq, Q.wq);
  fdm_eval(t, Q.xq, Q.Bq, Q.Dq);
  Q.Lq.assign(3 * q, 0.0);
  for (int i = 0; i < q; ++i) {
    const double x = Q.xq[i];
    Q.Lq[3 * i] = 0.5 * x * (x - 1.0);
    Q.Lq[3 * i + 1] = 1.0 - x * x;
    Q.Lq[3 * i + 2] = 0.5 * x * (x + 1.0);
  }
}

double trilinear_jacobian(const double *c, const double xi[3], double J[9]) {
  for (int e = 0; e < 9; ++e) J[e] = 0.0;
  for (int k = 0; k < 8; ++k) {
    double sg[3], f[3];
    for (int a = 0; a < 3; ++a) {
      sg[a] = ((k >> a) & 1) ? 1.0 : -1.0;
      f[a] = 0.5 * (1.0 + sg[a] * xi[a]);
    }
    const double dN[3] = {0.5 * sg[0] * f[1] * f[2], 0.5 * sg[1] * f[0] * f[2], 0.5 * sg[2] * f[0] * f[1]};
    for (int r = 0; r < 3; ++r)
      for (int s = 0; s < 3; ++s) J[3 * r + s] += dN[s] * c[3 * k + r];
  }
  return J[0] * (J[4] * J[8] - J[5] * J[7]) - J[1] * (J[3] * J[8] - J[5] * J[6]) + J[2] * (J[3] * J[7] - J[4] * J[6]);
}

static void inverse3(const double J[9], double det, double Ji[9]) {
  Ji[0] = (J[4] * J[8] - J[5] * J[7]) / det;
  Ji[1] = (J[2] * J[7] - J[1] * J[8]) / det;
  Ji[2] = (J[1] * J[5] - J[2] * J[4]) / det;
  Ji[3] = (J[5] * J[6] - J[3] * J[8]) / det;
  Ji[4] = (J[0] * J[8] - J[2] * J[6]) / det;
  Ji[5] = (J[2] * J[3] - J[0] * J[5]) / det;
  Ji[6] = (J[3] * J[7] - J[4] * J[6]) / det;
  Ji[7] = (J[1] * J[6] - J[0] * J[7]) / det;
  Ji[8] = (J[0] * J[4] - J[1] * J[3]) / det;
}

static double interp27(const double *s, const QuadTables &Q, int i, int j, int k) {
  double v = 0.0;
  for (int c = 0; c < 3; ++c)
    for (int b = 0; b < 3; ++b)
      for (int a = 0; a < 3; ++a) v += s[a + 3 * b + 9 * c] * Q.Lq[3 * i + a] * Q.Lq[3 * j + b] * Q.Lq[3 * k + c];
  return v;
}

bool averaged_weights(const double *corners, const double *as, const double *bs, const QuadTables &Q,
                      double out[6]) {
  const int q = Q.q;
  double sig[3] = {0, 0, 0}, mu = 0;
  for (int k = 0; k < q; ++k)
    for (int j = 0; j < q; ++j)
      for (int i = 0; i < q; ++i) {
        const double xi[3] = {Q.xq[i], Q.xq[j], Q.xq[k]};
        double J[9], Ji[9];
        const double det = trilinear_jacobian(corners, xi, J);
        if (!(det > 0)) return false;
        inverse3(J, det, Ji);
        const double al = interp27(as, Q, i, j, k), be = interp27(bs, Q, i, j, k);
        if (!(al > 0) || !(be > 0)) return false;
        const double w = Q.wq[i] * Q.wq[j] * Q.wq[k] * det;
        for (int s = 0; s < 3; ++s)
          sig[s] += w * al * (Ji[3 * s] * Ji[3 * s] + Ji[3 * s + 1] * Ji[3 * s + 1] + Ji[3 * s + 2] * Ji[3 * s + 2]);
        mu += w * be;
      }
  for (int s = 0; s < 3; ++s) out[s] = 0.125 * sig[s];
  for (int s = 0; s < 3; ++s) out[3 + s] = 0.125 * mu;
  return true;
}

bool q1_cell_matrix(const double *corners, const double *as, const double *bs, const QuadTables &Q,
                    double K[64]) {
  const int q = Q.q;
  for (int e = 0; e < 64; ++e) K[e] = 0.0;
  for (int k = 0; k < q; ++k)
    for (int j = 0; j < q; ++j)
      for (int i = 0; i < q; ++i) {
        const double xi[3] = {Q.xq[i], Q.xq[j], Q.xq[k]};
        double J[9], Ji[9];
        const double det = trilinear_jacobian(corners, xi, J);
        if (!(det > 0)) return false;
        inverse3(J, det, Ji);
        const double al = interp27(as, Q, i, j, k), be = interp27(bs, Q, i, j, k);
        const double w = Q.wq[i] * Q.wq[j] * Q.wq[k] * det;
        double N[8], gx[8][3];
        for (int n = 0; n < 8; ++n) {
          double sg[3], f[3];
          for (int a = 0; a < 3; ++a) {
            sg[a] = ((n >> a) & 1) ? 1.0 : -1.0;
            f[a] = 0.5 * (1.0 + sg[a] * xi[a]);
          }
          N[n] = f[0] * f[1] * f[2];
          const double g[3] = {0.5 * sg[0] * f[1] * f[2], 0.5 * sg[1] * f[0] * f[2], 0.5 * sg[2] * f[0] * f[1]};
          // physical gradient J^-T g: component r = sum_s Ji[s][r] g_s
          for (int r = 0; r < 3; ++r) gx[n][r] = Ji[r] * g[0] + Ji[3 + r] * g[1] + Ji[6 + r] * g[2];
        }
        for (int a = 0; a < 8; ++a)
          for (int b = 0; b < 8; ++b)
            K[8 * a + b] += w * (al * (gx[a][0] * gx[b][0] + gx[a][1] * gx[b][1] + gx[a][2] * gx[b][2]) +
                                 be * N[a] * N[b]);
      }
  return true;
}

// inverse of the broken transformation G (Gauss-Jordan with partial pivoting)
static std::vector<double> broken_inverse(const Tables1D &t) {
  const int n = t.p + 1;
  std::vector<double> G(t.G), Gi(n * n, 0.0);
  for (int i = 0; i < n; ++i) Gi[i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(G[r * n + c]) > std::fabs(G[piv * n + c])) piv = r;
    for (int k = 0; k < n; ++k) {
      std::swap(G[c * n + k], G[piv * n + k]);
      std::swap(Gi[c * n + k], Gi[piv * n + k]);
    }
    const double d = G[c * n + c];
    for (int k = 0; k < n; ++k) {
      G[c * n + k] /= d;
      Gi[c * n + k] /= d;
    }
    for (int r = 0; r < n; ++r)
      if (r != c) {
        const double f = G[r * n + c];
        for (int k = 0; k < n; ++k) {
          G[r * n + k] -= f * G[c * n + k];
          Gi[r * n + k] -= f * Gi[c * n + k];
        }
      }
  }
  return Gi;
}

// squares of the broken degree-p functions (fP, q x (p+1): s(x) G^-1) and of the
// degree-(p-1) L2 basis (fD, q x p: r_0 = 2^-1/2, r_k = lambda_k^-1/2 s_k') at Q.xq
static void broken_squares(const Tables1D &t, const QuadTables &Q, std::vector<double> &fP, std::vector<double> &fD) {
  const int p = t.p, n = p + 1, q = Q.q;
  const std::vector<double> Gi = broken_inverse(t);
  fP.assign((size_t)q * n, 0.0);
  fD.assign((size_t)q * p, 0.0);
  for (int i = 0; i < q; ++i) {
    for (int k = 0; k < n; ++k) {
      double v = 0.0;
      for (int j = 0; j < n; ++j) v += Q.Bq[i * n + j] * Gi[j * n + k];
      fP[(size_t)i * n + k] = v * v;
    }
    fD[(size_t)i * p] = 0.5;
    for (int k = 1; k < p; ++k) {
      const double r = Q.Dq[i * n + k] / std::sqrt(t.lam[k - 1]);
      fD[(size_t)i * p + k] = r * r;
    }
  }
}

void christoffel(const Tables1D &t, const QuadTables &Q, std::vector<double> &kP, std::vector<double> &kD) {
  const int p = t.p, n = p + 1, q = Q.q;
  const std::vector<double> Gi = broken_inverse(t);
  kP.assign(q, 0.0);
  kD.assign(q, 0.0);
  for (int i = 0; i < q; ++i) {
    // broken functions: values s(x) G^-1
    for (int k = 0; k < n; ++k) {
      double v = 0.0;
      for (int j = 0; j < n; ++j) v += Q.Bq[i * n + j] * Gi[j * n + k];
      kP[i] += v * v;
    }
    kP[i] /= n;
    // L2 basis of degree p-1: r_0 = 2^-1/2, r_k = lambda_k^-1/2 s_k'
    double s = 0.5;
    for (int k = 1; k < p; ++k) {
      const double r = Q.Dq[i * n + k] / std::sqrt(t.lam[k - 1]);
      s += r * r;
    }
    kD[i] = s / p;
  }
}

bool fit_targets(const double *corners, const double *as, const double *bs, const QuadTables &Q,
                 const std::vector<double> &kP, const std::vector<double> &kD, double out[6]) {
  const int q = Q.q;
  double sig[3] = {0, 0, 0}, mu = 0;
  for (int k = 0; k < q; ++k)
    for (int j = 0; j < q; ++j)
      for (int i = 0; i < q; ++i) {
        const double xi[3] = {Q.xq[i], Q.xq[j], Q.xq[k]};
        double J[9], Ji[9];
        const double det = trilinear_jacobian(corners, xi, J);
        if (!(det > 0)) return false;
        inverse3(J, det, Ji);
        const double al = interp27(as, Q, i, j, k), be = interp27(bs, Q, i, j, k);
        const double w = Q.wq[i] * Q.wq[j] * Q.wq[k] * det;
        const double kp[3] = {kP[i], kP[j], kP[k]}, kd[3] = {kD[i], kD[j], kD[k]};
        for (int s = 0; s < 3; ++s) {
          double kw = kd[s];
          for (int a = 0; a < 3; ++a)
            if (a != s) kw *= kp[a];
          sig[s] += w * al * kw *
                    (Ji[3 * s] * Ji[3 * s] + Ji[3 * s + 1] * Ji[3 * s + 1] + Ji[3 * s + 2] * Ji[3 * s + 2]);
        }
        mu += w * be * kp[0] * kp[1] * kp[2];
      }
  for (int s = 0; s < 3; ++s) out[s] = sig[s];
  for (int s = 0; s < 3; ++s) out[3 + s] = mu;
  return true;
}

PaperDiagTables::PaperDiagTables(const Tables1D &t, const QuadTables &Q) : p(t.p), q(Q.q) {
  broken_squares(t, Q, fP, fD);
}

// d[l][j][i] = sum_{z,y,x} W[z][y][x] f2[z][l] f1[y][j] f0[x][i] (sum factorised: x,
// then y, then z), f_a with n_a columns; d x fastest
static void diag_contract(const std::vector<double> &W, int q, const double *f0, int n0, const double *f1, int n1,
                          const double *f2, int n2, double *d) {
  std::vector<double> t1((size_t)q * q * n0), t2((size_t)q * n1 * n0);
  for (int z = 0; z < q; ++z)
    for (int y = 0; y < q; ++y)
      for (int i = 0; i < n0; ++i) {
        double s = 0.0;
        for (int x = 0; x < q; ++x) s += W[((size_t)z * q + y) * q + x] * f0[x * n0 + i];
        t1[((size_t)z * q + y) * n0 + i] = s;
      }
  for (int z = 0; z < q; ++z)
    for (int j = 0; j < n1; ++j)
      for (int i = 0; i < n0; ++i) {
        double s = 0.0;
        for (int y = 0; y < q; ++y) s += t1[((size_t)z * q + y) * n0 + i] * f1[y * n1 + j];
        t2[((size_t)z * n1 + j) * n0 + i] = s;
      }
  for (int l = 0; l < n2; ++l)
    for (int j = 0; j < n1; ++j)
      for (int i = 0; i < n0; ++i) {
        double s = 0.0;
        for (int z = 0; z < q; ++z) s += t2[((size_t)z * n1 + j) * n0 + i] * f2[z * n2 + l];
        d[((size_t)l * n1 + j) * n0 + i] = s;
      }
}

bool paper_diagonals(const double *corners, const double *as, const double *bs, const QuadTables &Q,
                     const PaperDiagTables &T, double *dm, double *da) {
  const int q = Q.q, p = T.p, n = p + 1;
  const size_t nq = (size_t)q * q * q;
  std::vector<double> wb(nq), wa[3] = {std::vector<double>(nq), std::vector<double>(nq), std::vector<double>(nq)};
  for (int k = 0; k < q; ++k)
    for (int j = 0; j < q; ++j)
      for (int i = 0; i < q; ++i) {
        const double xi[3] = {Q.xq[i], Q.xq[j], Q.xq[k]};
        double J[9], Ji[9];
        const double det = trilinear_jacobian(corners, xi, J);
        if (!(det > 0)) return false;
        inverse3(J, det, Ji);
        const double al = interp27(as, Q, i, j, k), be = interp27(bs, Q, i, j, k);
        if (!(al > 0) || !(be > 0)) return false;
        const double w = Q.wq[i] * Q.wq[j] * Q.wq[k] * det;
        const size_t o = ((size_t)k * q + j) * q + i;
        wb[o] = w * be;
        for (int m = 0; m < 3; ++m)
          wa[m][o] = w * al * (Ji[3 * m] * Ji[3 * m] + Ji[3 * m + 1] * Ji[3 * m + 1] + Ji[3 * m + 2] * Ji[3 * m + 2]);
      }
  const double *fP = T.fP.data(), *fD = T.fD.data();
  diag_contract(wb, q, fP, n, fP, n, fP, n, dm);
  const size_t nc = (size_t)p * n * n;
  diag_contract(wa[0], q, fD, p, fP, n, fP, n, da);
  diag_contract(wa[1], q, fP, n, fD, p, fP, n, da + nc);
  diag_contract(wa[2], q, fP, n, fP, n, fD, p, da + 2 * nc);
  return true;
}

void cell_features(const double *corners, const double *as, double out[51]) {
  double cen[3] = {0, 0, 0};
  for (int k = 0; k < 8; ++k)
    for (int r = 0; r < 3; ++r) cen[r] += corners[3 * k + r] / 8.0;
  static const int E[12][2] = {{0, 1}, {2, 3}, {4, 5}, {6, 7}, {0, 2}, {1, 3},
                               {4, 6}, {5, 7}, {0, 4}, {1, 5}, {2, 6}, {3, 7}};
  double h = 0;
  for (auto &e : E) {
    double d2 = 0;
    for (int r = 0; r < 3; ++r) {
      const double d = corners[3 * e[1] + r] - corners[3 * e[0] + r];
      d2 += d * d;
    }
    h += std::sqrt(d2) / 12.0;
  }
  for (int k = 0; k < 8; ++k)
    for (int r = 0; r < 3; ++r)
      out[3 * k + r] = (corners[3 * k + r] - cen[r]) / h - (((k >> r) & 1) ? 0.5 : -0.5);
  double m = 0;
  for (int k = 0; k < 27; ++k) m += std::log(as[k]) / 27.0;
  for (int k = 0; k < 27; ++k) out[24 + k] = std::log(as[k]) - m;
}

}  // namespace rz
