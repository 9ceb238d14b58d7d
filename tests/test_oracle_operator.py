"""Pins of the oracle's operators: two independent assembly routes, the
matrix-free route, symmetry / definiteness, exact reproduction of manufactured
solutions that lie in the discrete space, and the de Rham identities of Sec. 2.4
(eqs. gradbasis, curlbasis, divbasis)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle.tables1d import Element1D, gauss_legendre
from oracle.lattice import Mesh, Lattice
from oracle import assemble as asm, matfree, auxop


def distorted_mesh(n=2, shift=0.07):
    m = Mesh(n, n, n)
    v = m.vertices.copy()
    for k in range(v.shape[0]):
        vx, vy, vz = k % (n + 1), (k // (n + 1)) % (n + 1), k // (n + 1) ** 2
        if 0 < vx < n and 0 < vy < n and 0 < vz < n:
            v[k] += shift * np.array([1.0, -0.5, 0.3])
    return Mesh(n, n, n, v)


@pytest.mark.parametrize("space", ["grad", "curl", "div"])
def test_closed_form_equals_quadrature(space):
    m = Mesh(2, 3, 2)
    m.vertices[:, 0] *= 1.7           # anisotropic boxes
    lat = Lattice(m, space, 3)
    A1 = asm.cartesian_operator(lat, 2.0, 0.5)
    A2 = asm.quadrature_operator(lat, 2.0, 0.5)
    assert abs(A1 - A2).max() < 1e-12 * abs(A1).max()


@pytest.mark.parametrize("space", ["grad", "curl", "div"])
def test_matfree_equals_assembled(space):
    m = distorted_mesh()
    lat = Lattice(m, space, 3)
    al = lambda X: 1 + X[:, 0] * X[:, 1]
    A = asm.with_dirichlet(lat, asm.quadrature_operator(lat, al, 0.3, q=6))
    x = np.random.default_rng(1).standard_normal(lat.ndofs)
    y1 = A @ x
    y2 = matfree.apply(lat, x, al, 0.3, q=6)
    assert np.abs(y1 - y2).max() < 1e-13 * np.abs(y1).max()


@pytest.mark.parametrize("space", ["grad", "curl", "div"])
def test_symmetric_positive_definite(space):
    lat = Lattice(distorted_mesh(), space, 2)
    A = asm.with_dirichlet(lat, asm.quadrature_operator(lat, lambda X: 1 + X[:, 2], 1e-3)).toarray()
    assert np.abs(A - A.T).max() < 1e-13 * np.abs(A).max()
    assert np.linalg.eigvalsh(A).min() > 0


def test_derham_reference_identities():
    for p in (1, 3, 5):
        el = Element1D(p)
        G, C, Dv = asm.ref_grad(el), asm.ref_curl(el), asm.ref_div(el)
        assert np.abs(C @ G).max() < 1e-13
        assert np.abs(Dv @ C).max() < 1e-12


def _eval_ref(el, space, coef, pts):
    """Evaluate a reference function (vector-valued for curl/div) and its reference
    exterior derivative at points pts (n, 3) by direct tabulation."""
    xq = pts
    s = [el.s(pts[:, a]) for a in range(3)]
    ds = [el.ds(pts[:, a]) for a in range(3)]
    r = [el.r(pts[:, a]) for a in range(3)]
    p = el.p
    def tens(f0, f1, f2):
        return np.einsum("ni,nj,nl->nlji", f0, f1, f2).reshape(pts.shape[0], -1)
    if space == "grad":
        v = tens(s[0], s[1], s[2]) @ coef
        g = np.stack([tens(ds[0], s[1], s[2]) @ coef, tens(s[0], ds[1], s[2]) @ coef,
                      tens(s[0], s[1], ds[2]) @ coef], 1)
        return v, g
    if space == "curl":
        n1 = p * (p + 1) ** 2
        c = [coef[k * n1:(k + 1) * n1] for k in range(3)]
        u = np.stack([tens(r[0], s[1], s[2]) @ c[0], tens(s[0], r[1], s[2]) @ c[1],
                      tens(s[0], s[1], r[2]) @ c[2]], 1)
        return u, None
    n1 = (p + 1) * p * p
    c = [coef[k * n1:(k + 1) * n1] for k in range(3)]
    u = np.stack([tens(s[0], r[1], r[2]) @ c[0], tens(r[0], s[1], r[2]) @ c[1],
                  tens(r[0], r[1], s[2]) @ c[2]], 1)
    return u, None


def test_grad_of_Qp_lies_in_NCEp():
    p = 4
    el = Element1D(p)
    rng = np.random.default_rng(3)
    c = rng.standard_normal((p + 1) ** 3)
    pts = rng.uniform(-1, 1, (50, 3))
    _, g = _eval_ref(el, "grad", c, pts)
    u, _ = _eval_ref(el, "curl", asm.ref_grad(el) @ c, pts)
    assert np.abs(g - u).max() < 1e-11 * np.abs(g).max()


def test_curl_of_NCEp_lies_in_NCFp():
    p = 3
    el = Element1D(p)
    rng = np.random.default_rng(4)
    c = rng.standard_normal(3 * p * (p + 1) ** 2)
    pts = rng.uniform(-1, 1, (40, 3))
    # curl by finite differences of the tabulated field (polynomial: use a tight
    # centred difference and compare at 1e-6 relative)
    h = 1e-5
    def U(P):
        return _eval_ref(el, "curl", c, P)[0]
    J = np.zeros((pts.shape[0], 3, 3))
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        J[:, :, a] = (U(pts + e) - U(pts - e)) / (2 * h)
    curl = np.stack([J[:, 2, 1] - J[:, 1, 2], J[:, 0, 2] - J[:, 2, 0], J[:, 1, 0] - J[:, 0, 1]], 1)
    w, _ = _eval_ref(el, "div", asm.ref_curl(el) @ c, pts)
    assert np.abs(curl - w).max() < 1e-6 * np.abs(curl).max()


# ---------------------------------------------------------------------------------
# manufactured solutions inside the discrete space are reproduced exactly
# ---------------------------------------------------------------------------------
def _cell_dof_values(lat, funcs):
    """FDM coefficients of a field given per component as a sum of separable
    terms [(fx, fy, fz), ...] of physical coordinates, pulled back to each cell."""
    mesh, p = lat.mesh, lat.p
    el = Element1D(p)
    cv = mesh.cell_vertices()
    cd = lat.cell_dofs()
    c = np.zeros(lat.ndofs)
    for k in range(mesh.ncells):
        lo, hi = cv[k, 0], cv[k, 7]
        h = hi - lo
        loc = []
        for m, kind in enumerate(lat.kinds):
            scale = _piola_scale(lat.space, m, h)
            acc = 0.0
            for term in funcs[m]:
                fac = []
                for a in range(3):
                    f = (lambda xi, a=a, f=term[a]: f(lo[a] + 0.5 * (xi + 1) * h[a]))
                    fac.append(el.dof_functionals(f) if kind[a] == "P" else el.r_functionals(f))
                acc = acc + np.einsum("k,j,i->kji", fac[2], fac[1], fac[0]).ravel()
            loc.append(scale * acc)
        c[cd[k]] = np.concatenate(loc)
    return c


def _piola_scale(space, m, h):
    if space == "grad":
        return 1.0
    if space == "curl":
        return 0.5 * h[m]                          # u_ref = J^T u
    return np.prod(h) / 8.0 / (0.5 * h[m])          # u_ref = det J^{-1} u


def _load(lat, u, du, alpha, beta, q=9):
    """F(v) = (v, beta u) + (d v, alpha d u) by quadrature with analytic u, du."""
    mesh, p = lat.mesh, lat.p
    el = Element1D(p)
    xq, wq = gauss_legendre(q)
    W = np.einsum("z,y,x->zyx", wq, wq, wq).ravel()
    cv = mesh.cell_vertices()
    cd = lat.cell_dofs()
    val, dval = asm.reference_values(el, lat.space, xq)
    Z, Y, X = np.meshgrid(xq, xq, xq, indexing="ij")
    xi = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
    F = np.zeros(lat.ndofs)
    for k in range(mesh.ncells):
        lo, hi = cv[k, 0], cv[k, 7]
        h = hi - lo
        P = lo + 0.5 * (xi + 1) * h
        det = np.prod(h) / 8.0
        J = np.diag(h / 2)
        Ji = np.diag(2 / h)
        if lat.space == "grad":
            pv = val[:, 0, :]
            pd = np.einsum("rs,qsn->qrn", Ji, dval)
            Fk = W * det * beta * u(P) @ pv + np.einsum("q,qr,qrn->n", W * det * alpha, du(P), pd)
        elif lat.space == "curl":
            pv = np.einsum("rs,qsn->qrn", Ji, val)
            pd = np.einsum("rs,qsn->qrn", J, dval) / det
            Fk = np.einsum("q,qr,qrn->n", W * det * beta, u(P), pv) + \
                np.einsum("q,qr,qrn->n", W * det * alpha, du(P), pd)
        else:
            pv = np.einsum("rs,qsn->qrn", J, val) / det
            pd = dval[:, 0, :] / det
            Fk = np.einsum("q,qr,qrn->n", W * det * beta, u(P), pv) + (W * det * alpha * du(P)) @ pd
        np.add.at(F, cd[k], Fk)
    return F


def _solve(lat, F, alpha, beta):
    A = asm.with_dirichlet(lat, asm.quadrature_operator(lat, alpha, beta))
    mask = lat.dirichlet_mask()
    return spla.spsolve(A.tocsc(), np.where(mask, 0.0, F))


def test_manufactured_hgrad():
    m = Mesh(2, 2, 2)
    lat = Lattice(m, "grad", 4)
    b = lambda t: t * (1 - t)
    db = lambda t: 1 - 2 * t
    # u = x(1-x) y(1-y) z(1-z) (1 + x + y^2 z): degree <= 4 per axis
    terms = [((b), (b), (b)), ((lambda t: t * b(t)), (b), (b)), ((b), (lambda t: t * t * b(t)), (lambda t: t * b(t)))]
    u = lambda P: sum(t[0](P[:, 0]) * t[1](P[:, 1]) * t[2](P[:, 2]) for t in terms)
    def du(P):
        x, y, z = P[:, 0], P[:, 1], P[:, 2]
        f = 1 + x + y * y * z
        g = b(x) * b(y) * b(z)
        gx = db(x) * b(y) * b(z) * f + g
        gy = b(x) * db(y) * b(z) * f + g * 2 * y * z
        gz = b(x) * b(y) * db(z) * f + g * y * y
        return np.stack([gx, gy, gz], 1)
    cu = _cell_dof_values(lat, [terms])
    c = _solve(lat, _load(lat, u, du, 1.3, 0.7), 1.3, 0.7)
    assert np.abs(c - cu).max() < 1e-11 * np.abs(cu).max()


def test_manufactured_hcurl():
    m = Mesh(2, 2, 2)
    lat = Lattice(m, "curl", 3)
    b = lambda t: t * (1 - t)
    one = lambda t: np.ones_like(t)
    idt = lambda t: t
    # u = (b(y)b(z)(1+x), b(x)b(z) y, b(x)b(y)): tangential trace zero on the cube
    funcs = [[(one, b, b), (idt, b, b)], [(b, idt, b)], [(b, b, one)]]
    def u(P):
        x, y, z = P[:, 0], P[:, 1], P[:, 2]
        return np.stack([b(y) * b(z) * (1 + x), b(x) * b(z) * y, b(x) * b(y)], 1)
    def curl(P):
        x, y, z = P[:, 0], P[:, 1], P[:, 2]
        db = lambda t: 1 - 2 * t
        uy_z = b(x) * db(z) * y
        uz_y = b(x) * db(y)
        ux_z = b(y) * db(z) * (1 + x)
        uz_x = db(x) * b(y)
        uy_x = db(x) * b(z) * y
        ux_y = db(y) * b(z) * (1 + x)
        return np.stack([uz_y - uy_z, ux_z - uz_x, uy_x - ux_y], 1)
    cu = _cell_dof_values(lat, funcs)
    c = _solve(lat, _load(lat, u, curl, 0.8, 1.9), 0.8, 1.9)
    assert np.abs(c - cu).max() < 1e-11 * np.abs(cu).max()


def test_manufactured_hdiv():
    m = Mesh(2, 2, 2)
    lat = Lattice(m, "div", 3)
    b = lambda t: t * (1 - t)
    one = lambda t: np.ones_like(t)
    idt = lambda t: t
    # u = (b(x) y, b(y) (1+z), b(z) x): normal trace zero on the cube
    funcs = [[(b, idt, one)], [(one, b, one), (one, b, idt)], [(idt, one, b)]]
    def u(P):
        x, y, z = P[:, 0], P[:, 1], P[:, 2]
        return np.stack([b(x) * y, b(y) * (1 + z), b(z) * x], 1)
    def div(P):
        x, y, z = P[:, 0], P[:, 1], P[:, 2]
        db = lambda t: 1 - 2 * t
        return db(x) * y + db(y) * (1 + z) + db(z) * x
    cu = _cell_dof_values(lat, funcs)
    c = _solve(lat, _load(lat, u, div, 2.1, 0.4), 2.1, 0.4)
    assert np.abs(c - cu).max() < 1e-11 * np.abs(cu).max()


@pytest.mark.parametrize("space", ["grad", "curl", "div"])
def test_auxiliary_equals_operator_on_cartesian(space):
    # Sec. 3.2: P = A on Cartesian cells with constant coefficients
    m = Mesh(2, 2, 1)
    m.vertices[:, 1] *= 0.6
    lat = Lattice(m, space, 3)
    A = asm.quadrature_operator(lat, 2.0, 0.3)
    P = auxop.paper_operator(lat, 2.0, 0.3)
    S = auxop.separable_operator(lat, auxop.cartesian_coefficient_array(lat, 2.0, 0.3))
    assert abs(A - P).max() < 1e-13 * abs(A).max()
    assert abs(A - S).max() < 1e-13 * abs(A).max()


@pytest.mark.parametrize("space", ["grad", "curl", "div"])
def test_auxiliary_spd_on_distorted(space):
    lat = Lattice(distorted_mesh(), space, 3)
    P = asm.with_dirichlet(lat, auxop.paper_operator(lat, lambda X: 1 + X[:, 0], 0.5)).toarray()
    assert np.abs(P - P.T).max() < 1e-13 * np.abs(P).max()
    assert np.linalg.eigvalsh(P).min() > 0


def test_auxiliary_sampled_gll_equals_operator_on_cartesian():
    # Sec. 3.2: P = A on Cartesian cells with constant coefficients, also when the
    # coefficients come as 27 reference samples and the diagonals use the GLL rule
    m = Mesh(2, 2, 1)
    m.vertices[:, 1] *= 0.6
    lat = Lattice(m, "grad", 3)
    A = asm.quadrature_operator(lat, 2.0, 0.3)
    P = auxop.paper_operator(lat, np.full((m.ncells, 27), 2.0), np.full((m.ncells, 27), 0.3), q=6, kind="gll")
    assert abs(A - P).max() < 1e-13 * abs(A).max()


@pytest.mark.parametrize("p", [2, 5])
def test_paper_diagonals_closed_form_on_boxes(p):
    # the broken bases are L2-orthonormal on the reference cell, so on a box with
    # constant coefficients the weighted mass matrices are multiples of the
    # identity: beta det J for the Q_p part and alpha det J (J^-1 J^-T)_mm =
    # alpha V / (2 h_m^2) for NCE component m
    from oracle.tables1d import Element1D
    el = Element1D(p)
    h = np.array([0.5, 0.3, 0.8])
    corners = np.array([[(k & 1) * h[0], ((k >> 1) & 1) * h[1], (k >> 2) * h[2]] for k in range(8)])
    V = h.prod()
    dm, da = auxop.paper_diagonals_grad(el, corners, 1.7, 0.4, p + 2, kind="gll")
    assert dm.size == (p + 1) ** 3 and np.allclose(dm, 0.4 * V / 8, rtol=1e-12)
    for m_ in range(3):
        assert da[m_].size == p * (p + 1) ** 2
        assert np.allclose(da[m_], 1.7 * V / (2 * h[m_] ** 2), rtol=1e-12)


def test_paper_auxiliary_interior_block_diagonal_on_distorted():
    # the remark of Sec. 4.4 for k = 0: P_II stays diagonal for the broken-diagonal
    # auxiliary on any cell (the interior FDM functions are unchanged by the broken
    # transformation and D has a single entry in each interior column); its entries
    # are dm + sum_m lambda_{i_m} da_m
    from oracle.tables1d import Element1D
    from oracle.quadrature import sample_function
    from oracle.schwarz import interior_mask
    m = distorted_mesh()
    lat = Lattice(m, "grad", 4)
    a = sample_function(m, lambda X: 1 + X[:, 0] ** 2)
    P = auxop.paper_operator(lat, a, 0.7, q=8, kind="gll").tocsr()
    I = np.where(interior_mask(lat))[0]
    PII = P[I][:, I].toarray()
    assert np.abs(PII - np.diag(np.diag(PII))).max() == 0.0
    el = Element1D(4)
    dm, da = auxop.paper_diagonals_grad(el, m.cell_vertices()[0], a[0], 0.7, 8, kind="gll")
    n1, p = 5, 4
    g = lat.cell_dofs()[0]
    for (ia, ib, ic) in [(1, 1, 1), (2, 3, 1), (3, 2, 2)]:
        k = ia + n1 * (ib + n1 * ic)
        want = dm[k] + el.lam[ia - 1] * da[0][ia + p * (ib + n1 * ic)] \
            + el.lam[ib - 1] * da[1][ia + n1 * (ib + p * ic)] + el.lam[ic - 1] * da[2][ia + n1 * (ib + n1 * ic)]
        # cell 0's interior DoF is owned by cell 0 alone
        assert abs(P[g[k], g[k]] - want) < 1e-12 * abs(want)
