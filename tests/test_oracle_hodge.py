"""Pins of the Hodge-Laplacian oracle (Sec. 5.3): Chebyshev against its closed-form
error polynomial, MINRES against the brute-force minimiser over the Krylov space,
the exterior derivatives against the assembled stiffness matrices and the complex
property d d = 0, and the exactly preconditioned k = 3 spectrum against its closed
form."""
import numpy as np
import numpy.polynomial.chebyshev as npcheb
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle.lattice import Mesh, Lattice
from oracle import hodge, assemble as asm
from oracle.hiptmair import exterior_derivative


def graded_mesh(nx, ny, nz):
    """Cartesian mesh with unequal cell sizes along every axis."""
    ax = [np.cumsum(np.r_[0.0, 1.0 + 0.3 * np.arange(n)]) for n in (nx, ny, nz)]
    ax = [a / a[-1] for a in ax]
    Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    return Mesh(nx, ny, nz, vertices=np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1), dirichlet=0)


def test_chebyshev_closed_form():
    # diagonal A, B = I: the m-step error is T_m((b+a-2 lam)/(b-a)) / T_m((b+a)/(b-a)) times x*
    lam = np.linspace(0.2, 1.3, 23)
    f = np.cos(np.arange(23.0))
    a, b = 0.3, 1.2
    for m in (1, 2, 4, 7):
        x = hodge.chebyshev(sp.diags(lam), lambda r: r.copy(), a, b, m)(f)
        cm = np.zeros(m + 1)
        cm[m] = 1.0
        pm = npcheb.chebval((b + a - 2 * lam) / (b - a), cm) / npcheb.chebval((b + a) / (b - a), cm)
        xs = f / lam
        np.testing.assert_allclose(xs - x, pm * xs, rtol=0, atol=1e-13)


def test_minres_minimises_natural_residual():
    rng = np.random.default_rng(3)
    n = 30
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = np.r_[-np.linspace(0.5, 3.0, 12), np.linspace(0.2, 4.0, 18)]
    K = Q @ np.diag(ev) @ Q.T
    dP = rng.uniform(0.5, 2.0, n)
    Pinv = lambda r: r / dP
    b = rng.standard_normal(n)
    Wm = np.diag(1.0 / dP)          # the P^{-1} inner product
    for j in range(1, 9):
        x, it, hist = hodge.minres(K, b, Pinv, rtol=0.0, maxit=j)
        assert it == j
        # Krylov space span{(P^{-1} K)^i P^{-1} b}, i < j; minimise ||b - K y||_{P^{-1}}
        basis = [Pinv(b)]
        for _ in range(j - 1):
            basis.append(Pinv(K @ basis[-1]))
        Vb = np.linalg.qr(np.column_stack(basis))[0]
        L = np.linalg.cholesky(Wm)
        c = np.linalg.lstsq(L.T @ (K @ Vb), L.T @ b, rcond=None)[0]
        y = Vb @ c
        assert np.linalg.norm(x - y) <= 1e-9 * np.linalg.norm(y)
        res = b - K @ x
        assert abs(np.sqrt(res @ (res / dP)) - hist[-1]) <= 1e-10 * hist[0]


def test_exterior_derivatives_against_assembled_stiffness():
    m = graded_mesh(2, 3, 2)
    p = 3
    lg, lc, ld = Lattice(m, "grad", p), Lattice(m, "curl", p), Lattice(m, "div", p)
    G, C, Dv = exterior_derivative(lg, lc), exterior_derivative(lc, ld), hodge.divergence(ld)
    # the complex: curl grad = 0, div curl = 0
    assert abs(C @ G).max() < 1e-12 * abs(C).max() * abs(G).max()
    assert abs(Dv @ C).max() < 1e-12 * abs(Dv).max() * abs(C).max()
    # the stiffness of each space is d^T M d with the mass of the next one
    Mg, Mc, Md = (asm.cartesian_operator(l, 0.0, 1.0) for l in (lg, lc, ld))
    M3 = sp.diags(hodge.l2_mass_diagonal(m, p))
    for D, Mn, lat in ((G, Mc, lg), (C, Md, lc), (Dv, M3, ld)):
        S = asm.cartesian_operator(lat, 1.0, 0.0)
        E = (D.T @ Mn @ D - S).toarray()
        assert abs(E).max() < 1e-11 * abs(S).max()


def test_k3_exact_preconditioner_spectrum():
    # with exact Riesz inverses, K z = lam P z has lam = -1 or lam = mu / (1 + mu) for the
    # eigenvalues mu > 0 of S_2 sigma = mu M_2 sigma (S_2 = div-div, P = diag(M_2 + S_2, M_3))
    m = graded_mesh(1, 2, 1)
    s = hodge.HodgeSystem(m, 3, 2)
    K = s.K.toarray()
    P = sla.block_diag(s.A_lo.toarray(), s.M_hi.toarray())
    lam = sla.eigh(K, P, eigvals_only=True)
    S2 = (s.D.T @ s.M_hi @ s.D).toarray()
    mu = sla.eigh(S2, s.M_lo.toarray(), eigvals_only=True)
    allowed = np.r_[-1.0, (mu / (1 + mu))[mu > 1e-9]]
    dist = np.min(np.abs(lam[:, None] - allowed[None, :]), axis=1)
    assert dist.max() < 1e-9
    # the number of -1 eigenvalues: the divergence-free sigma plus one per DQ value
    nneg = int(np.sum(np.abs(lam + 1.0) < 1e-9))
    assert nneg == s.n_lo - int(np.sum(mu > 1e-9)) + s.n_hi


def test_minres_hodge_reaches_direct_solution():
    m = Mesh(2, 2, 2, dirichlet=0)
    for k in (1, 2, 3):
        sysm, P, b, x, it, hist = hodge.hodge_solve(m, k, 2)
        xs = spla.spsolve(sysm.K.tocsc(), b)
        assert hist[-1] <= 1e-8 * hist[0]
        assert np.linalg.norm(x - xs) <= 1e-6 * np.linalg.norm(xs)
        assert 4 <= it <= 16
        # the preconditioner is a fixed symmetric operator
        rng = np.random.default_rng(k)
        u, v = rng.standard_normal(b.size), rng.standard_normal(b.size)
        assert abs(u @ P(v) - v @ P(u)) <= 1e-10 * np.linalg.norm(u) * np.linalg.norm(P(v))
