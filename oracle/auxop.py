"""Auxiliary sparse operator P^k (oracle; test infrastructure).

``paper_cell_matrix`` follows eq. sum-factorization_approx (Sec. 3.2):
    P_K = Gb^T diag(Mb_beta) Gb + Db^T diag(Mb_alpha) Db,   Db = Gb D,
where Gb maps FDM coefficients to coefficients in the broken basis whose 1-D
factor along every P-direction is the orthonormalised interface pair plus the
interior eigenfunctions, and diag(Mb) is the diagonal of the weighted mass matrix
in that broken basis (pulled back with the k- or (k+1)-form Piola map).  The
diagonal entries are computed by Gauss-Legendre quadrature on the (trilinear)
cell.

``separable_cell_matrix`` is the per-cell separable form used when the
coefficients of the auxiliary operator are given as six numbers per cell
(sigma_1..3, mu_1..3): the 1-D Kronecker structure of the Cartesian case with
per-cell weights.  On an axis-aligned box with constant alpha, beta and
``cartesian_coefficients`` it equals A_K (Sec. 3.2: P = A in the Cartesian,
constant-coefficient case).
"""
import numpy as np

from .tables1d import Element1D, gauss_legendre
from .lattice import Lattice, component_kinds
from .assemble import (kron3, ref_grad, ref_curl, ref_div, trilinear_jacobian, assemble,
                       _blockdiag, cell_sizes, _cell_coef)


def _broken_1d(el):
    """Broken-basis tabulations: values of the broken P functions at xq are
    s(xq) @ inv(G) (FDM coefficients c, broken coefficients G c)."""
    return np.linalg.inv(el.G)


def _gbar(el, kinds):
    """Broken transformation for one component: G along P axes, identity along DP."""
    p = el.p
    mats = [el.G if k == "P" else np.eye(p) for k in kinds]
    return kron3(mats[0], mats[1], mats[2])


def _diag_mass(el, kinds, weight, xq):
    """Diagonal of the mass matrix weighted by ``weight`` (q,q,q array indexed
    [z, y, x], already including quadrature weights and the Piola factor) in the
    broken tensor basis of one component; returned in x-fastest local order."""
    Ginv = _broken_1d(el)
    sb = el.s(xq) @ Ginv
    r = el.r(xq)
    f = [sb if k == "P" else r for k in kinds]
    d = np.einsum("zyx,zl,yj,xi->lji", weight, f[2] ** 2, f[1] ** 2, f[0] ** 2, optimize=True)
    return d.ravel()


def paper_cell_matrix(el: Element1D, space, corners, alpha, beta, q, kind="gl"):
    """P_K of eq. sum-factorization_approx on one trilinear cell, the broken mass
    diagonals by q-point Gauss-Legendre (kind="gl") or Gauss-Lobatto-Legendre
    (kind="gll") quadrature per axis.  alpha, beta: scalars, callables of physical
    points, or 27 reference samples of the cell (triquadratic interpolation)."""
    if kind == "gl":
        xq, wq = gauss_legendre(q)
    else:
        from .quadrature import rule
        xq, wq = rule(q, kind)
    W = np.einsum("z,y,x->zyx", wq, wq, wq).ravel()
    X, J = trilinear_jacobian(corners, xq)
    det = np.linalg.det(J)
    Jinv = np.linalg.inv(J)
    a = _cell_coef(alpha, X, xq)
    b = _cell_coef(beta, X, xq)
    G_ = np.einsum("qrs,qts->qrt", Jinv, Jinv)            # J^{-1} J^{-T}
    H_ = np.einsum("qsr,qst->qrt", J, J) / (det ** 2)[:, None, None]   # J^T J / det^2
    p = el.p
    sh = (q, q, q)
    if space == "grad":
        kV = component_kinds("grad", p)
        Gv = _gbar(el, kV[0])
        dm = _diag_mass(el, kV[0], (W * det * b).reshape(sh), xq)
        kE = component_kinds("curl", p)
        Gd = _blockdiag([_gbar(el, kE[m]) for m in range(3)])
        da = np.concatenate([_diag_mass(el, kE[m], (W * det * a * G_[:, m, m]).reshape(sh), xq)
                             for m in range(3)])
        Dref = ref_grad(el)
    elif space == "curl":
        kE = component_kinds("curl", p)
        Gv = _blockdiag([_gbar(el, kE[m]) for m in range(3)])
        dm = np.concatenate([_diag_mass(el, kE[m], (W * det * b * G_[:, m, m]).reshape(sh), xq)
                             for m in range(3)])
        kF = component_kinds("div", p)
        Gd = _blockdiag([_gbar(el, kF[m]) for m in range(3)])
        da = np.concatenate([_diag_mass(el, kF[m], (W * det * a * H_[:, m, m]).reshape(sh), xq)
                             for m in range(3)])
        Dref = ref_curl(el)
    elif space == "div":
        kF = component_kinds("div", p)
        Gv = _blockdiag([_gbar(el, kF[m]) for m in range(3)])
        dm = np.concatenate([_diag_mass(el, kF[m], (W * det * b * H_[:, m, m]).reshape(sh), xq)
                             for m in range(3)])
        kQ = ("D", "D", "D")
        Gd = np.eye(p ** 3)
        da = _diag_mass(el, kQ, (W * a / det).reshape(sh), xq)
        Dref = ref_div(el)
    else:
        raise ValueError(space)
    Db = Gd @ Dref
    return Gv.T @ (dm[:, None] * Gv) + Db.T @ (da[:, None] * Db)


def cartesian_coefficients(space, h, alpha, beta):
    """Six per-cell weights (sigma_1..3, mu_1..3) that make the separable form equal
    to the exact cell matrix on a box with sides h and constant alpha, beta."""
    h1, h2, h3 = h
    V = h1 * h2 * h3
    hs = np.array([h1, h2, h3])
    if space == "grad":
        return np.concatenate([alpha * V / (2 * hs ** 2), np.full(3, beta * V / 8.0)])
    if space == "curl":
        return np.concatenate([alpha * 2 * hs ** 2 / V, beta * V / (2 * hs ** 2)])
    if space == "div":
        return np.concatenate([np.full(3, alpha * 8.0 / V), beta * 2 * hs ** 2 / V])
    raise ValueError(space)


def separable_cell_matrix(el: Element1D, space, c):
    """Separable auxiliary cell matrix from six weights c = (sigma_1..3, mu_1..3).
      grad: sum_d sigma_d (A along d, B elsewhere) + mu_1 B x B x B
      curl: blockdiag_m mu_m (I along m, B elsewhere)
            + C^T blockdiag_n sigma_n (B along n, I elsewhere) C
      div : blockdiag_m mu_m (B along m, I elsewhere) + sigma_1 Div^T Div
    """
    p = el.p
    A, B, J = el.A, el.B, np.eye(p)
    s1, s2, s3, m1, m2, m3 = [float(v) for v in c]
    if space == "grad":
        return s1 * kron3(A, B, B) + s2 * kron3(B, A, B) + s3 * kron3(B, B, A) + m1 * kron3(B, B, B)
    if space == "curl":
        ME = _blockdiag([m1 * kron3(J, B, B), m2 * kron3(B, J, B), m3 * kron3(B, B, J)])
        MF = _blockdiag([s1 * kron3(B, J, J), s2 * kron3(J, B, J), s3 * kron3(J, J, B)])
        C = ref_curl(el)
        return ME + C.T @ MF @ C
    if space == "div":
        MF = _blockdiag([m1 * kron3(B, J, J), m2 * kron3(J, B, J), m3 * kron3(J, J, B)])
        Dv = ref_div(el)
        return MF + s1 * Dv.T @ Dv
    raise ValueError(space)


def paper_operator(lat: Lattice, alpha, beta, q=None, kind="gl"):
    """Global auxiliary operator with the paper's broken-diagonal construction.
    alpha, beta: scalar, callable, per-cell array (ncells,) or per-cell samples
    (ncells, 27)."""
    mesh = lat.mesh
    el = Element1D(lat.p)
    q = q or (lat.p + 2)
    cv = mesh.cell_vertices()

    def pick(c, k):
        if callable(c) or np.isscalar(c):
            return c
        c = np.asarray(c)
        return c[k] if c.ndim == 2 else float(c[k])

    mats = []
    for k in range(mesh.ncells):
        mats.append(paper_cell_matrix(el, lat.space, cv[k], pick(alpha, k), pick(beta, k), q, kind))
    return assemble(lat, mats)


def paper_diagonals_grad(el: Element1D, corners, alpha, beta, q, kind="gll"):
    """The two broken diagonals of one H(grad) cell: diag of the beta-mass in the
    broken Q_p basis ((p+1)^3 values) and, per NCE component m, diag of the
    alpha-mass with the metric entry (J^-1 J^-T)_mm in the broken NCE_p basis
    (p (p+1)^2 values each); x-fastest local order, component m with its DP index
    along axis m."""
    if kind == "gl":
        xq, wq = gauss_legendre(q)
    else:
        from .quadrature import rule
        xq, wq = rule(q, kind)
    W = np.einsum("z,y,x->zyx", wq, wq, wq).ravel()
    X, J = trilinear_jacobian(corners, xq)
    det = np.linalg.det(J)
    Jinv = np.linalg.inv(J)
    a = _cell_coef(alpha, X, xq)
    b = _cell_coef(beta, X, xq)
    G_ = np.einsum("qrs,qts->qrt", Jinv, Jinv)
    sh = (q, q, q)
    p = el.p
    dm = _diag_mass(el, component_kinds("grad", p)[0], (W * det * b).reshape(sh), xq)
    kE = component_kinds("curl", p)
    da = [_diag_mass(el, kE[m], (W * det * a * G_[:, m, m]).reshape(sh), xq) for m in range(3)]
    return dm, da


def separable_operator(lat: Lattice, coefs):
    """Global auxiliary operator from per-cell six-weight arrays (ncells, 6)."""
    el = Element1D(lat.p)
    mats = [separable_cell_matrix(el, lat.space, coefs[k]) for k in range(coefs.shape[0])]
    return assemble(lat, mats)


def cartesian_coefficient_array(lat: Lattice, alpha, beta):
    """(ncells, 6) separable weights reproducing A on a Cartesian mesh."""
    mesh = lat.mesh
    hs = cell_sizes(mesh)
    al = np.broadcast_to(np.asarray(alpha, dtype=np.float64), (mesh.ncells,))
    be = np.broadcast_to(np.asarray(beta, dtype=np.float64), (mesh.ncells,))
    return np.array([cartesian_coefficients(lat.space, hs[k], al[k], be[k]) for k in range(mesh.ncells)])
