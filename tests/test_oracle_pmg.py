"""Pins of the oracle's geometric h-multigrid coarse solver on the p = 1 space
(Sec. 5.1): the 1-D interpolation reproduces linear functions, the Galerkin operator
of nested Q_1 spaces equals the discretisation on the coarser mesh, and the V(1,1)
cycle is a symmetric positive definite approximate inverse that contracts the error."""
import numpy as np
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
