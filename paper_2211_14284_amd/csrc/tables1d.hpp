// 1-D FDM element tables (host, FP64), Sec. 2.2-2.3 and 3.2 of the paper.
#pragma once
#include <vector>

namespace rz {

struct Tables1D {
  int p = 0;
  std::vector<double> gll;      // p+1 GLL nodes
  std::vector<double> lam;      // p-1 eigenvalues (ascending), eq. eigs
  std::vector<double> S;        // (p+1)x(p+1) row-major: S[i*(p+1)+j] = s_j(gll_i)
  std::vector<double> B, A;     // (p+1)x(p+1) FDM mass / stiffness, row-major
  std::vector<double> D;        // p x (p+1) differentiation matrix (r_i, s_j')
  std::vector<double> E;        // (p+1) x 2 embedding of the linear hats
  std::vector<double> G;        // (p+1)x(p+1) broken-basis transformation
};

// Build all tables of degree p (1 <= p <= 16).  Returns false on failure.
bool build_tables1d(int p, Tables1D &t);

// Gauss-Legendre rule with n points on [-1,1].
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w);

// Gauss-Lobatto-Legendre rule with q >= 2 points on [-1,1] (exact to degree 2q-3).
void gll_rule(int q, std::vector<double> &x, std::vector<double> &w);

// Values and derivatives of the FDM basis s_0..s_p at points x (n points):
// val[k*(p+1)+j] = s_j(x_k), der likewise.
void fdm_eval(const Tables1D &t, const std::vector<double> &x, std::vector<double> &val,
              std::vector<double> &der);

}  // namespace rz
