"""Assembled global operators of a^k(v,u) = (v, beta u) + (d^k v, alpha d^k u)
(oracle; test infrastructure).

Two independent routes to the cell matrices:
  * ``cartesian_cell_matrix``: closed form on an axis-aligned box with constant
    alpha, beta.  With the pullbacks of Sec. 3.1 (identity, J^{-T}, J/detJ,
    1/detJ) and the 1-D FDM mass B, stiffness A and differentiation matrix D,
    eq. sum-factorization A_K = M_beta + D^T M_alpha D becomes a sum of Kronecker
    products of 1-D matrices;
  * ``quadrature_cell_matrix``: dense tabulation of every basis function and its
    reference derivative at Gauss-Legendre points of a trilinear cell, pulled
    back explicitly (Sec. 3.1, eq. form-reference-values).
Local ordering of a cell's degrees of freedom: component-major, x-local fastest.
"""
import numpy as np
import scipy.sparse as sp

from .tables1d import Element1D, gauss_legendre
from .lattice import Lattice, component_kinds


def kron3(Mx, My, Mz):
    """Matrix acting on a tile stored x-fastest: kron(Mz, kron(My, Mx))."""
    return np.kron(Mz, np.kron(My, Mx))


# ----------------------------------------------------------------------------------
# reference discrete exterior derivatives between FDM bases (cell-local)
# ----------------------------------------------------------------------------------
def ref_grad(el: Element1D):
    """Q_p -> NCE_p on the reference cell (eq. gradbasis generalised): component m
    of grad(s_i s_j s_l) replaces s along axis m by s' = sum_a D[a, .] r_a."""
    p = el.p
    I = np.eye(p + 1)
    D = el.D
    return np.vstack([kron3(D, I, I), kron3(I, D, I), kron3(I, I, D)])


def ref_curl(el: Element1D):
    """NCE_p -> NCF_p on the reference cell (eq. curlbasis generalised)."""
    p = el.p
    I, J, D = np.eye(p + 1), np.eye(p), el.D
    # NCE components: 0 = (D,P,P), 1 = (P,D,P), 2 = (P,P,D) ; NCF: 0 = (P,D,D), 1 = (D,P,D), 2 = (D,D,P)
    n_e = [p * (p + 1) ** 2] * 3
    n_f = [(p + 1) * p * p] * 3
    C = np.zeros((sum(n_f), sum(n_e)))
    oe = np.cumsum([0] + n_e)
    of = np.cumsum([0] + n_f)
    # curl_x = d_y u_z - d_z u_y ; curl_y = d_z u_x - d_x u_z ; curl_z = d_x u_y - d_y u_x
    # d_y of u_z (P,P,D) along y -> (P,D,D) = NCF 0
    C[of[0]:of[1], oe[2]:oe[3]] += kron3(I, D, J)
    C[of[0]:of[1], oe[1]:oe[2]] -= kron3(I, J, D)
    C[of[1]:of[2], oe[0]:oe[1]] += kron3(J, I, D)
    C[of[1]:of[2], oe[2]:oe[3]] -= kron3(D, I, J)
    C[of[2]:of[3], oe[1]:oe[2]] += kron3(D, J, I)
    C[of[2]:of[3], oe[0]:oe[1]] -= kron3(J, D, I)
    return C


def ref_div(el: Element1D):
    """NCF_p -> DQ_{p-1} on the reference cell (eq. divbasis generalised)."""
    p = el.p
    J, D = np.eye(p), el.D
    return np.hstack([kron3(D, J, J), kron3(J, D, J), kron3(J, J, D)])


# ----------------------------------------------------------------------------------
# closed form on Cartesian cells
# ----------------------------------------------------------------------------------
def cartesian_cell_matrix(el: Element1D, space: str, h, alpha: float, beta: float):
    """Cell matrix on a box with sides h = (h1, h2, h3), constant alpha, beta."""
    h1, h2, h3 = h
    V = h1 * h2 * h3
    B, A = el.B, el.A
    p = el.p
    J = np.eye(p)
    if space == "grad":
        K = (V / (2 * h1 ** 2)) * kron3(A, B, B) + (V / (2 * h2 ** 2)) * kron3(B, A, B) \
            + (V / (2 * h3 ** 2)) * kron3(B, B, A)
        return alpha * K + beta * (V / 8.0) * kron3(B, B, B)
    if space == "curl":
        # NCE mass: component m weight V/(2 h_m^2) (J^{-T} pullback), identity along m
        ME = [V / (2 * h1 ** 2) * kron3(J, B, B), V / (2 * h2 ** 2) * kron3(B, J, B),
              V / (2 * h3 ** 2) * kron3(B, B, J)]
        # NCF mass: component m weight 2 h_m^2 / V (J/detJ pullback), B along m
        MF = [2 * h1 ** 2 / V * kron3(B, J, J), 2 * h2 ** 2 / V * kron3(J, B, J),
              2 * h3 ** 2 / V * kron3(J, J, B)]
        C = ref_curl(el)
        return beta * _blockdiag(ME) + alpha * C.T @ _blockdiag(MF) @ C
    if space == "div":
        MF = [2 * h1 ** 2 / V * kron3(B, J, J), 2 * h2 ** 2 / V * kron3(J, B, J),
              2 * h3 ** 2 / V * kron3(J, J, B)]
        Dv = ref_div(el)
        return beta * _blockdiag(MF) + alpha * (8.0 / V) * Dv.T @ Dv
    raise ValueError(space)


def _blockdiag(blocks):
    n = sum(b.shape[0] for b in blocks)
    out = np.zeros((n, n))
    o = 0
    for b in blocks:
        k = b.shape[0]
        out[o:o + k, o:o + k] = b
        o += k
    return out


# ----------------------------------------------------------------------------------
# quadrature on trilinear cells
# ----------------------------------------------------------------------------------
def trilinear_jacobian(corners, xq):
    """Physical points and Jacobians of the trilinear map of one cell at the tensor
    quadrature points built from 1-D points xq (x fastest).
    Returns X (nq, 3) and J (nq, 3, 3) with J[:, r, s] = d x_r / d xi_s."""
    n = xq.size
    Z, Y, Xg = np.meshgrid(xq, xq, xq, indexing="ij")
    xi = np.stack([Xg.ravel(), Y.ravel(), Z.ravel()], 1)
    X = np.zeros((xi.shape[0], 3))
    J = np.zeros((xi.shape[0], 3, 3))
    for k in range(8):
        sgn = np.array([2 * ((k >> a) & 1) - 1 for a in range(3)], dtype=np.float64)
        f = 0.5 * (1 + sgn[None, :] * xi)          # per-axis linear factors
        N = f[:, 0] * f[:, 1] * f[:, 2]
        X += N[:, None] * corners[k][None, :]
        for s in range(3):
            dN = 0.5 * sgn[s] * np.prod([f[:, a] for a in range(3) if a != s], axis=0)
            J[:, :, s] += dN[:, None] * corners[k][None, :]
    return X, J


def _tab(el, xq, kinds, deriv_axis=None):
    """Tabulate tensor basis of one component at tensor points (nq, nloc)."""
    s, ds, r = el.s(xq), el.ds(xq), el.r(xq)
    mats = []
    for a in range(3):
        if kinds[a] == "P":
            mats.append(ds if deriv_axis == a else s)
        else:
            assert deriv_axis != a
            mats.append(r)
    # point index (qz, qy, qx), dof index (l, j, i)
    T = np.einsum("zl,yj,xi->zyxlji", mats[2], mats[1], mats[0])
    nq = xq.size ** 3
    return T.reshape(nq, -1)


def reference_values(el, space, xq):
    """Reference values of every local basis function (vector-valued for k=1,2)
    and of their reference exterior derivative, at tensor points.
    Returns (val, dval) with shapes (nq, ncomp_val, nloc), (nq, ncomp_d, nloc)."""
    p = el.p
    kinds = component_kinds(space, p)
    if space == "grad":
        val = _tab(el, xq, kinds[0])[:, None, :]
        dval = np.stack([_tab(el, xq, kinds[0], deriv_axis=a) for a in range(3)], 1)
        return val, dval
    nloc = [int(np.prod([p + 1 if k == "P" else p for k in kinds[m]])) for m in range(3)]
    off = np.cumsum([0] + nloc)
    nq = xq.size ** 3
    val = np.zeros((nq, 3, off[-1]))
    for m in range(3):
        val[:, m, off[m]:off[m + 1]] = _tab(el, xq, kinds[m])
    if space == "curl":
        dval = np.zeros((nq, 3, off[-1]))
        for m in range(3):
            sl = slice(off[m], off[m + 1])
            for a in range(3):
                if a == m:
                    continue
                d = _tab(el, xq, kinds[m], deriv_axis=a)
                # curl_n = eps_{n a m} d_a u_m
                n = 3 - a - m
                eps = 1.0 if (n, a, m) in ((0, 1, 2), (1, 2, 0), (2, 0, 1)) else -1.0
                dval[:, n, sl] += eps * d
        return val, dval
    if space == "div":
        dval = np.zeros((nq, 1, off[-1]))
        for m in range(3):
            dval[:, 0, off[m]:off[m + 1]] = _tab(el, xq, kinds[m], deriv_axis=m)
        return val, dval
    raise ValueError(space)


def _cell_coef(c, X, xq):
    """Coefficient values at the tensor points: scalar, callable of physical points,
    or 27 reference samples of the cell (triquadratic interpolation)."""
    if callable(c):
        return c(X)
    c = np.asarray(c, dtype=np.float64)
    if c.size == 27:
        from .quadrature import sampled_values
        return sampled_values(c[None, :], xq)[0]
    return np.full(X.shape[0], float(c))


def quadrature_cell_matrix(el, space, corners, alpha, beta, q, kind="gl"):
    """Dense cell matrix on a trilinear cell with q points per axis (Gauss-Legendre,
    or Gauss-Lobatto-Legendre for kind="gll").  alpha, beta: scalars, callables of
    physical points (nq, 3), or 27 reference samples."""
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
    val, dval = reference_values(el, space, xq)
    if space == "grad":
        phys_v = val                                              # identity
        phys_d = np.einsum("qsr,qsn->qrn", Jinv, dval)           # J^{-T} grad
    elif space == "curl":
        phys_v = np.einsum("qsr,qsn->qrn", Jinv, val)            # J^{-T} u
        phys_d = np.einsum("qrs,qsn->qrn", J, dval) / det[:, None, None]   # J curl / det
    else:
        phys_v = np.einsum("qrs,qsn->qrn", J, val) / det[:, None, None]    # J u / det
        phys_d = dval / det[:, None, None]                                 # div / det
    wb = W * det * b
    wa = W * det * a
    M = np.einsum("q,qrn,qrm->nm", wb, phys_v, phys_v)
    K = np.einsum("q,qrn,qrm->nm", wa, phys_d, phys_d)
    return M + K


# ----------------------------------------------------------------------------------
# global assembly
# ----------------------------------------------------------------------------------
def assemble(lat: Lattice, cellmats):
    """Sum cell matrices into a global CSR matrix on all lattice DoFs."""
    cd = lat.cell_dofs()
    nl = cd.shape[1]
    rows = np.repeat(cd, nl, axis=1).ravel()
    cols = np.tile(cd, (1, nl)).ravel()
    vals = np.asarray(cellmats).reshape(cd.shape[0], nl * nl).ravel()
    return sp.csr_matrix(sp.coo_matrix((vals, (rows, cols)), shape=(lat.ndofs, lat.ndofs)))


def with_dirichlet(lat: Lattice, A):
    """Replace constrained rows and columns by the identity."""
    mask = lat.dirichlet_mask()
    keep = sp.diags((~mask).astype(np.float64))
    return sp.csr_matrix(keep @ A @ keep + sp.diags(mask.astype(np.float64)))


def cell_sizes(mesh):
    """(ncells, 3) box side lengths of a Cartesian mesh."""
    cv = mesh.cell_vertices()
    return np.stack([cv[:, 1, 0] - cv[:, 0, 0], cv[:, 2, 1] - cv[:, 0, 1], cv[:, 4, 2] - cv[:, 0, 2]], 1)


def cartesian_operator(lat: Lattice, alpha, beta):
    """Global matrix on a Cartesian mesh with cellwise-constant alpha, beta (arrays
    of length ncells or scalars), via the closed-form cell matrices."""
    mesh = lat.mesh
    el = Element1D(lat.p)
    hs = cell_sizes(mesh)
    al = np.broadcast_to(np.asarray(alpha, dtype=np.float64), (mesh.ncells,))
    be = np.broadcast_to(np.asarray(beta, dtype=np.float64), (mesh.ncells,))
    mats = [cartesian_cell_matrix(el, lat.space, hs[k], al[k], be[k]) for k in range(mesh.ncells)]
    return assemble(lat, mats)


def quadrature_operator(lat: Lattice, alpha, beta, q=None, kind="gl"):
    """Global matrix by per-cell quadrature (any trilinear mesh).  alpha, beta:
    scalar, per-cell array (ncells,), per-cell samples (ncells, 27), or callable of
    physical points."""
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
        mats.append(quadrature_cell_matrix(el, lat.space, cv[k], pick(alpha, k), pick(beta, k), q, kind))
    return assemble(lat, mats)
