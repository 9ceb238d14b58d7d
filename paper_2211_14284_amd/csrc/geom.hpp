// Host geometry of trilinear cells and the quadrature tables of the
// variable-coefficient path (Sec. 3.1 pullbacks, Sec. 5 quadrature rule).
#pragma once
#include <vector>

#include "tables1d.hpp"

namespace rz {

// Tensor quadrature on [-1,1]^3 from a q-point 1-D Gauss-Lobatto-Legendre rule, and
// the 1-D tabulations it needs: Bq[i*(p+1)+a] = s_a(x_i), Dq = s_a'(x_i) (FDM
// basis of degree p), Lq[i*3+c] = quadratic Lagrange basis on {-1,0,1} at x_i.
struct QuadTables {
  int p = 0, q = 0;
  std::vector<double> xq, wq, Bq, Dq, Lq;
};

// ceil(3(p+1)/2), the number of points per axis of the paper's rule.
inline int default_quad_points(int p) { return (3 * (p + 1) + 1) / 2; }

void build_quad_tables(const Tables1D &t, int q, QuadTables &Q);

// Trilinear map of a cell with corners c[8][3] (corner k = kx + 2 ky + 4 kz) at the
// reference point xi: J[3*r + s] = d x_r / d xi_s.  Returns det J.
double trilinear_jacobian(const double *c, const double xi[3], double J[9]);

// Separable auxiliary weights of one cell (sigma_1..3, mu, mu, mu):
// sigma_s = 1/8 sum w det(J) alpha (J^-1 J^-T)_ss, mu = 1/8 sum w det(J) beta, with
// alpha, beta the triquadratic interpolants of the 27 samples.  Returns false if
// det J or an interpolated coefficient is not positive at a quadrature point.
bool averaged_weights(const double *corners, const double *as, const double *bs, const QuadTables &Q,
                      double out[6]);

// 8x8 cell matrix of the p=1 form (standard trilinear hats) by quadrature.
bool q1_cell_matrix(const double *corners, const double *as, const double *bs, const QuadTables &Q,
                    double K[64]);

// Christoffel functions of the 1-D bases at the points Q.xq: kP = mean over the
// broken degree-p basis of its squares, kD = the same for the degree-(p-1) L2 basis.
void christoffel(const Tables1D &t, const QuadTables &Q, std::vector<double> &kP, std::vector<double> &kD);

// Least-squares separable fit to the broken diagonals of the auxiliary operator
// (the mean of each diagonal), Christoffel-factorised: out = (sigma_1..3, mu x3).
bool fit_targets(const double *corners, const double *as, const double *bs, const QuadTables &Q,
                 const std::vector<double> &kP, const std::vector<double> &kD, double out[6]);

// The paper's auxiliary operator on a trilinear cell (Sec. 3.2, eqs.
// mass_in_broken_basis and sum-factorization_approx): the diagonals of the weighted
// mass matrices in the broken bases, by the quadrature Q.  PaperDiagTables holds the
// squares of the broken 1-D functions at the points (per degree).
struct PaperDiagTables {
  int p = 0, q = 0;
  std::vector<double> fP, fD;  // q x (p+1) broken P_p squares, q x p DP_{p-1} squares
  PaperDiagTables() = default;
  PaperDiagTables(const Tables1D &t, const QuadTables &Q);
};
// dm: (p+1)^3 values, diag of the beta-mass in the broken Q_p basis; da: three blocks
// of p (p+1)^2, diag of the alpha-mass weighted by (J^-1 J^-T)_mm in the broken basis
// of NCE_p component m (its DP index along axis m); x-fastest local order.  Returns
// false if det J or an interpolated coefficient is not positive at a point.
bool paper_diagonals(const double *corners, const double *as, const double *bs, const QuadTables &Q,
                     const PaperDiagTables &T, double *dm, double *da);

// 51 dimensionless features of a cell: corner offsets from the centroid over the
// mean edge length minus those of a cube (24), log alpha samples minus their mean (27).
void cell_features(const double *corners, const double *as, double out[51]);

}  // namespace rz
