"""Quadrature rules, sampled coefficients and cell-averaged separable weights
(oracle; test infrastructure).

* The paper integrates with a Gauss-Lobatto rule of about 3(p+1)/2 points per axis
  on non-affine cells (Sec. 5); read here as q = ceil(3(p+1)/2) Gauss-Lobatto-
  Legendre points (exact to degree 2q-3).
* Variable coefficients enter as 27 samples per cell at the reference points
  {-1, 0, 1}^3 (x fastest) and are interpolated triquadratically on the reference
  cell.
* Separable auxiliary weights from cell averages (the fallback auxiliary of the
  learned variant): sigma_d = (1/8) int alpha det(J) (J^-1 J^-T)_dd dxi and
  mu = (1/8) int beta det(J) dxi over the reference cube; on an axis-aligned box
  with constant coefficients they are the exact weights alpha V/(2 h_d^2), beta V/8.
"""
import numpy as np
from numpy.polynomial import legendre as npleg

from .tables1d import gll_nodes, gauss_legendre
from .assemble import trilinear_jacobian


def default_points(p: int) -> int:
    return (3 * (p + 1) + 1) // 2


def gll_rule(q: int):
    """q-point Gauss-Lobatto-Legendre rule: nodes -1, roots of P_{q-1}', +1;
    weights 2 / (q (q-1) P_{q-1}(x)^2)."""
    if q < 2:
        raise ValueError("q >= 2")
    x = gll_nodes(q - 1)
    c = np.zeros(q)
    c[q - 1] = 1.0
    P = npleg.legval(x, c)
    return x, 2.0 / (q * (q - 1) * P ** 2)


def rule(q: int, kind: str = "gll"):
    return gll_rule(q) if kind == "gll" else gauss_legendre(q)


def quadratic_lagrange(t):
    """(len(t), 3) values of the quadratic Lagrange basis on the nodes -1, 0, 1."""
    t = np.asarray(t, dtype=np.float64)
    return np.stack([0.5 * t * (t - 1.0), 1.0 - t * t, 0.5 * t * (t + 1.0)], 1)


def sampled_values(samples, xq):
    """Values of the triquadratic interpolants of per-cell samples (ncells, 27) at
    the tensor points of the 1-D points xq: (ncells, q^3), x fastest."""
    s = np.asarray(samples, dtype=np.float64).reshape(-1, 3, 3, 3)   # (cell, c, b, a)
    L = quadratic_lagrange(xq)                                        # (q, 3)
    v = np.einsum("ncba,ia,jb,kc->nkji", s, L, L, L)
    return v.reshape(s.shape[0], -1)


def averaged_coefficients(mesh, alpha_samples, beta_samples, q, kind="gll"):
    """(ncells, 6) separable weights (sigma_1..3, mu, mu, mu) of H(grad) from cell
    averages of the coefficient-weighted metric."""
    xq, wq = rule(q, kind)
    W = np.einsum("z,y,x->zyx", wq, wq, wq).ravel()
    cv = mesh.cell_vertices()
    a = sampled_values(alpha_samples, xq)
    b = sampled_values(beta_samples, xq)
    out = np.zeros((mesh.ncells, 6))
    for k in range(mesh.ncells):
        _, J = trilinear_jacobian(cv[k], xq)
        det = np.linalg.det(J)
        Ji = np.linalg.inv(J)
        G = np.einsum("qsr,qsr->qs", Ji, Ji)      # (J^-1 J^-T)_ss = sum_r (J^-1)_sr^2
        for s in range(3):
            out[k, s] = 0.125 * np.sum(W * det * a[k] * G[:, s])
        out[k, 3:] = 0.125 * np.sum(W * det * b[k])
    return out


def sample_function(mesh, f):
    """Samples (ncells, 27) of a function f of physical points (n, 3) at the images
    of the reference points {-1, 0, 1}^3 under each cell's trilinear map."""
    cv = mesh.cell_vertices()
    t = np.array([-1.0, 0.0, 1.0])
    out = np.zeros((mesh.ncells, 27))
    for k in range(mesh.ncells):
        X, _ = trilinear_jacobian(cv[k], t)
        out[k] = f(X)
    return out
