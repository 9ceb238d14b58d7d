"""Pins of the oracle's geometric h-multigrid coarse solver on the p = 1 space
(Sec. 5.1): the 1-D interpolation reproduces linear functions, the Galerkin operator
of nested Q_1 spaces equals the discretisation on the coarser mesh, and the V(1,1)
cycle is a symmetric positive definite approximate inverse that contracts the error."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle.lattice import Mesh, Lattice
from oracle import assemble as asm, pmg


def test_interp_1d_is_piecewise_linear_interpolation():
    # the coarse piecewise-linear function (zero at Dirichlet ends) evaluated at the
    # fine vertices x = f / 2 in coarse units
    rng = np.random.default_rng(5)
    v = np.concatenate([[0.0], rng.standard_normal(3), [0.0]])
    P = pmg.interp_1d(9, 1, 7, 1, 3)
    assert np.allclose(P @ v[1:4], np.interp(np.arange(1, 8) / 2, np.arange(5), v), atol=1e-15)
    w = rng.standard_normal(5)          # no Dirichlet ends: all vertices free
    Pn = pmg.interp_1d(9, 0, 8, 0, 4)
    assert np.allclose(Pn @ w, np.interp(np.arange(9) / 2, np.arange(5), w), atol=1e-15)
    assert np.allclose(Pn @ (1.5 + 0.5 * np.arange(5)), 1.5 + 0.25 * np.arange(9), atol=1e-15)


def test_hmg_galerkin_equals_coarse_discretisation():
    # nested Q_1 spaces with constant coefficients: P^T A_h P is the Q_1 operator of
    # the mesh with half the cells (free DoFs), to rounding
    m, mc = Mesh(8, 4, 6), Mesh(4, 2, 3)
    lat, latc = Lattice(m, "grad", 1), Lattice(mc, "grad", 1)
    A = asm.with_dirichlet(lat, asm.cartesian_operator(lat, 1.3, 0.7))
    Ac = asm.with_dirichlet(latc, asm.cartesian_operator(latc, 1.3, 0.7))
    H = pmg.HMGCoarse(lat, A, min_free=1)
    fc = np.where(~latc.dirichlet_mask())[0]
    ref = sp.csr_matrix(Ac)[fc][:, fc].toarray()
    assert np.abs(H.A[1].toarray() - ref).max() < 1e-13 * np.abs(ref).max()


def test_hmg_cycle_spd_and_contracts():
    m = Mesh(8, 8, 8)
    lat = Lattice(m, "grad", 1)
    A = asm.with_dirichlet(lat, asm.cartesian_operator(lat, 1.0, 1e-3))
    H = pmg.HMGCoarse(lat, A, min_free=10)
    assert len(H.A) == 3
    free = H.free
    Af = sp.csr_matrix(A)[free][:, free].toarray()
    B = np.zeros_like(Af)
    for k in range(free.size):
        e = np.zeros(lat.ndofs)
        e[free[k]] = 1.0
        B[:, k] = H.solve(e)[free]
    assert np.abs(B - B.T).max() < 1e-12 * np.abs(B).max()
    ev = np.linalg.eigvals(np.eye(free.size) - B @ Af)
    assert np.abs(ev).max() < 0.5          # the V-cycle's error contraction
    assert np.linalg.eigvalsh(0.5 * (B + B.T)).min() > 0


def test_halve_1d_broken_axis():
    # a coarse cell's r_0 on its two halves: weight 1/2 each, nothing across cells
    P = pmg.halve_1d(6, 3, False).toarray()
    assert np.array_equal(P, 0.5 * np.kron(np.eye(3), np.ones((2, 1))))


def _interp(lat_f, lat_c):
    # per-component Kronecker interpolation between nested lowest-order spaces, on
    # the free DoFs
    nf = [lat_f.mesh.nx, lat_f.mesh.ny, lat_f.mesh.nz]
    nc = [lat_c.mesh.nx, lat_c.mesh.ny, lat_c.mesh.nz]
    blocks = [sp.kron(*[pmg.halve_1d(nf[a], nc[a], kind[a] == "P") for a in (2,)],
                      sp.kron(pmg.halve_1d(nf[1], nc[1], kind[1] == "P"), pmg.halve_1d(nf[0], nc[0], kind[0] == "P")))
              for kind in lat_f.kinds]
    ff = np.where(~lat_f.dirichlet_mask())[0]
    fc = np.where(~lat_c.dirichlet_mask())[0]
    return sp.csr_matrix(sp.block_diag(blocks, format="csr")[ff][:, fc])


@pytest.mark.parametrize("space", ["curl", "div"])
def test_hiptmair_galerkin_equals_coarse_discretisation(space):
    # nested lowest-order spaces with constant coefficients: P^T A_h P is the
    # operator of the mesh with half the cells (free DoFs), to rounding
    m, mc = Mesh(4, 6, 4), Mesh(2, 3, 2)
    lat, latc = Lattice(m, space, 1), Lattice(mc, space, 1)
    A = asm.with_dirichlet(lat, asm.cartesian_operator(lat, 1.3, 0.7))
    Ac = asm.with_dirichlet(latc, asm.cartesian_operator(latc, 1.3, 0.7))
    H = pmg.HiptmairHMG(lat, A, min_free=1)
    assert len(H.A) == 2
    fc = np.where(~latc.dirichlet_mask())[0]
    ref = sp.csr_matrix(Ac)[fc][:, fc].toarray()
    assert np.abs(H.A[1].toarray() - ref).max() < 1e-13 * np.abs(ref).max()
    # the interpolations commute with the exterior derivative: P G_c = G_f P_pot,
    # P_pot the interpolation of the potential space (trilinear for Q_1, the same
    # Kronecker rule for NCE_1)
    pot = {"curl": "grad", "div": "curl"}[space]
    Ppot = _interp(Lattice(m, pot, 1), Lattice(mc, pot, 1))
    lhs = (H.P[0] @ H.G[1]).toarray()
    rhs = (H.G[0] @ Ppot).toarray()
    assert np.abs(lhs).max() > 0.1 and np.abs(lhs - rhs).max() < 1e-14


@pytest.mark.parametrize("space", ["curl", "div"])
def test_hiptmair_cycle_spd_and_contracts(space):
    n = (8, 8, 8)
    lat = Lattice(Mesh(*n), space, 1)
    nc = int(np.prod(n))
    rng = np.random.default_rng(3)
    al, be = 10.0 ** rng.uniform(-1, 1, nc), 10.0 ** rng.uniform(-1, 1, nc)
    A = asm.with_dirichlet(lat, asm.cartesian_operator(lat, al, be))
    H = pmg.HiptmairHMG(lat, A, min_free=100)   # levels 8^3, 4^3, 2^3
    assert len(H.A) == 3
    free = H.free
    Af = sp.csr_matrix(A)[free][:, free].toarray()
    B = np.zeros_like(Af)
    for k in range(free.size):
        e = np.zeros(lat.ndofs)
        e[free[k]] = 1.0
        B[:, k] = H.solve(e)[free]
    assert np.abs(B - B.T).max() < 1e-12 * np.abs(B).max()
    assert np.linalg.eigvalsh(0.5 * (B + B.T)).min() > 0
    rho = np.abs(np.linalg.eigvals(np.eye(free.size) - B @ Af)).max()
    print(space, "rho", rho)
    assert rho < 0.97, rho
    # the potential relaxation is needed: without it the near-kernel of the curl
    # (or divergence) part converges far more slowly at small beta
    Ab = asm.with_dirichlet(lat, asm.cartesian_operator(lat, 1.0, 1e-6))
    Hs = pmg.HiptmairHMG(lat, Ab, min_free=100)
    Abf = sp.csr_matrix(Ab)[free][:, free].toarray()
    I = np.eye(lat.ndofs)
    Bh = np.column_stack([Hs.solve(I[free[k]])[free] for k in range(free.size)])
    rho_h = np.abs(np.linalg.eigvals(np.eye(free.size) - Bh @ Abf)).max()
    Hs.wp = [0.0] * len(Hs.wp)
    Bs = np.column_stack([Hs.solve(I[free[k]])[free] for k in range(free.size)])
    rho_s = np.abs(np.linalg.eigvals(np.eye(free.size) - Bs @ Abf)).max()
    print(space, "rho with / without potential relaxation", rho_h, rho_s)
    assert rho_h < 0.7 and rho_s > 0.99, (rho_h, rho_s)


def test_jacobi_weight_bounds_the_spectrum_on_anisotropic_cells():
    # 1:20 cells: the weighted Jacobi spectrum stays in (0, 1.5] (the Gershgorin
    # bound), where a fixed weight of 2/3 would exceed 2 and make the cycle indefinite
    m0 = Mesh(6, 6, 6)
    m = Mesh(6, 6, 6, vertices=m0.vertices * np.array([0.05, 1.0, 1.0])[None, :])
    for space in ("grad", "curl", "div"):
        lat = Lattice(m, space, 1)
        free = np.where(~lat.dirichlet_mask())[0]
        Af = sp.csr_matrix(asm.cartesian_operator(lat, 1.0, 1.0))[free][:, free]
        w = pmg.jacobi_weight(Af)
        d = Af.diagonal()
        S = (sp.diags(1 / np.sqrt(d)) @ Af @ sp.diags(1 / np.sqrt(d))).toarray()
        lam = np.linalg.eigvalsh(S)
        assert lam.min() > 0 and w * lam.max() <= pmg.JACOBI_C + 1e-12
        if space == "grad":
            assert (2.0 / 3.0) * lam.max() > 2.0


def test_pcg_reports_breakdown_of_an_indefinite_preconditioner():
    # r^T M r < 0 is a CG breakdown, never a converged natural norm
    A = sp.diags(np.arange(1.0, 11.0)).tocsr()
    b = np.ones(10)
    for norm in ("natural", "l2"):
        _, it, _ = pmg.pcg(A, b, lambda r: -r, norm=norm)
        assert it == -1
    _, it, _ = pmg.pcg(A, b, lambda r: r / A.diagonal(), norm="natural")
    assert it >= 1
