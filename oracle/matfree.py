"""Matrix-free sum-factorised operator application (oracle; test infrastructure).

Evaluates y = A x cell by cell as in eq. form-reference-values / eq.
sum-factorization of Sec. 3.2: interpolate the cell coefficients to tensor
quadrature points one axis at a time with 1-D tabulations, apply the pulled-back
coefficients (Sec. 3.1) pointwise, and contract back.  This is a separate code
path from ``assemble``; it is checked against it on small meshes.

Dirichlet rows act as the identity (y_D = x_D); Dirichlet entries of x are
treated as zero in the free rows.
"""
import numpy as np

from .tables1d import Element1D, gauss_legendre
from .lattice import Lattice, component_kinds
from .assemble import trilinear_jacobian


def _axis_tables(el, xq):
    s, ds, r = el.s(xq), el.ds(xq), el.r(xq)
    return {"P": s, "dP": ds, "D": r}


def _interp(T, tile):
    """tile[K, l, j, i] -> values[K, qz, qy, qx] with per-axis tables T = (Tx, Ty, Tz)."""
    return np.einsum("zl,yj,xi,Klji->Kzyx", T[2], T[1], T[0], tile, optimize=True)


def _interp_t(T, vals):
    return np.einsum("zl,yj,xi,Kzyx->Klji", T[2], T[1], T[0], vals, optimize=True)


def cell_geometry(mesh, xq, cells):
    """J (nc, nq, 3, 3) and physical points (nc, nq, 3) of the selected cells."""
    cv = mesh.cell_vertices()[cells]
    Js, Xs = [], []
    for k in range(cv.shape[0]):
        X, J = trilinear_jacobian(cv[k], xq)
        Js.append(J)
        Xs.append(X)
    return np.array(Js), np.array(Xs)


def apply(lat: Lattice, x, alpha, beta, q=None, chunk=2048, kind="gl"):
    """y = A x by sum factorisation.  alpha, beta: scalar, per-cell array (ncells,),
    per-cell reference samples (ncells, 27), or callable of physical points (n, 3).
    q points per axis, Gauss-Legendre (kind "gl") or Gauss-Lobatto-Legendre ("gll")."""
    mesh, p, space = lat.mesh, lat.p, lat.space
    el = Element1D(p)
    q = q or (p + 2)
    if kind == "gl":
        xq, wq = gauss_legendre(q)
    else:
        from .quadrature import rule
        xq, wq = rule(q, kind)
    W = np.einsum("z,y,x->zyx", wq, wq, wq)
    tabs = _axis_tables(el, xq)
    kinds = component_kinds(space, p)
    ncomp = len(kinds)
    mask = lat.dirichlet_mask()
    xf = np.where(mask, 0.0, x)
    cd = lat.cell_dofs()
    y = np.zeros(lat.ndofs)
    nloc = [int(np.prod(lat.local_shape(m))) for m in range(ncomp)]
    off = np.cumsum([0] + nloc)
    for c0 in range(0, mesh.ncells, chunk):
        cells = np.arange(c0, min(mesh.ncells, c0 + chunk))
        nc = cells.size
        J, X = cell_geometry(mesh, xq, cells)
        det = np.linalg.det(J)
        Jinv = np.linalg.inv(J)
        Xf = X.reshape(-1, 3)
        a = _coef(alpha, cells, Xf, q, xq)
        b = _coef(beta, cells, Xf, q, xq)
        wdet = (W.ravel()[None, :] * det)
        tiles = [xf[cd[cells, off[m]:off[m + 1]]].reshape((nc,) + lat.local_shape(m)[::-1])
                 for m in range(ncomp)]
        # reference values and reference exterior derivative at quadrature points
        val = np.zeros((nc, q ** 3, 3 if space != "grad" else 1))
        dval = np.zeros((nc, q ** 3, 1 if space == "div" else 3))
        for m in range(ncomp):
            k = kinds[m]
            T = tuple(tabs[k[ax]] for ax in range(3))
            val[:, :, m if space != "grad" else 0] = _interp(T, tiles[m]).reshape(nc, -1)
            for ax in range(3):
                if k[ax] != "P":
                    continue
                if space == "div" and ax != m:
                    continue
                Td = tuple(tabs["dP"] if a_ == ax else tabs[k[a_]] for a_ in range(3))
                d = _interp(Td, tiles[m]).reshape(nc, -1)
                if space == "grad":
                    dval[:, :, ax] += d
                elif space == "curl":
                    n = 3 - ax - m
                    eps = 1.0 if (n, ax, m) in ((0, 1, 2), (1, 2, 0), (2, 0, 1)) else -1.0
                    dval[:, :, n] += eps * d
                else:
                    dval[:, :, 0] += d
        # pullbacks and coefficients
        if space == "grad":
            Gm = np.einsum("cqrs,cqts->cqrt", Jinv, Jinv)          # J^{-1} J^{-T}
            fv = (wdet * b)[:, :, None] * val
            fd = (wdet * a)[:, :, None] * np.einsum("cqrt,cqt->cqr", Gm, dval)
        elif space == "curl":
            Gm = np.einsum("cqrs,cqts->cqrt", Jinv, Jinv)
            Hm = np.einsum("cqsr,cqst->cqrt", J, J) / (det ** 2)[:, :, None, None]  # J^T J / det^2
            fv = (wdet * b)[:, :, None] * np.einsum("cqrt,cqt->cqr", Gm, val)
            fd = (wdet * a)[:, :, None] * np.einsum("cqrt,cqt->cqr", Hm, dval)
        else:
            Hm = np.einsum("cqsr,cqst->cqrt", J, J) / (det ** 2)[:, :, None, None]
            fv = (wdet * b)[:, :, None] * np.einsum("cqrt,cqt->cqr", Hm, val)
            fd = (wdet * a / det ** 2)[:, :, None] * dval
        # transposed contractions
        for m in range(ncomp):
            k = kinds[m]
            T = tuple(tabs[k[ax]] for ax in range(3))
            out = _interp_t(T, fv[:, :, m if space != "grad" else 0].reshape(nc, q, q, q))
            for ax in range(3):
                if k[ax] != "P":
                    continue
                if space == "div" and ax != m:
                    continue
                Td = tuple(tabs["dP"] if a_ == ax else tabs[k[a_]] for a_ in range(3))
                if space == "grad":
                    comp, eps = ax, 1.0
                elif space == "curl":
                    comp = 3 - ax - m
                    eps = 1.0 if (comp, ax, m) in ((0, 1, 2), (1, 2, 0), (2, 0, 1)) else -1.0
                else:
                    comp, eps = 0, 1.0
                out = out + eps * _interp_t(Td, fd[:, :, comp].reshape(nc, q, q, q))
            np.add.at(y, cd[cells, off[m]:off[m + 1]], out.reshape(nc, -1))
    y[mask] = x[mask]
    return y


def _coef(c, cells, Xf, q, xq):
    n = cells.size
    if callable(c):
        return c(Xf).reshape(n, q ** 3)
    c = np.asarray(c, dtype=np.float64)
    if c.ndim == 0:
        return np.full((n, q ** 3), float(c))
    if c.ndim == 2:
        from .quadrature import sampled_values
        return sampled_values(c[cells], xq)
    return np.repeat(c[cells][:, None], q ** 3, axis=1)
