"""Pins of the oracle's static condensation, patches, incomplete Cholesky,
relaxation, p-transfer and PCG (Sec. 4.3-4.5, Sec. 5)."""
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import synth
from oracle.tables1d import Element1D, p1_embedding
from oracle.lattice import Mesh, Lattice
from oracle import assemble as asm, auxop, schwarz, pmg

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_patch_counts_c1():
    lat = Lattice(Mesh(4, 4, 4), "grad", 4)
    pl = schwarz.vertex_patches_grad(lat)
    assert len(pl) == 125 - 8               # the 8 corner stars hold no free DoF
    sizes = [len(d) for _, d in pl]
    assert sizes.count(1 + 6 * 3 + 12 * 9) == 27   # full interior stars
    assert max(sizes) == 127


def test_pattern_counts_fixture():
    rows = [l.split() for l in open(os.path.join(GOLD, "vertex_patch_pattern_counts.txt")) if l[0] != "#"]
    for row in rows:
        p, nrow, nnz, mx = (int(v) for v in row)
        lat = Lattice(Mesh(2, 2, 2), "grad", p)
        pat = schwarz.symbolic_schur_pattern_grad(lat)
        vid, dofs = [x for x in schwarz.vertex_patches_grad(lat) if x[0] == 13][0]
        pv = pat[dofs][:, dofs].toarray().astype(bool)
        assert len(dofs) == nrow == 1 + 6 * (p - 1) + 12 * (p - 1) ** 2
        assert np.tril(pv).sum() == nnz
        assert pv.sum(1).max() == mx == 6 * p - 5


@pytest.mark.parametrize("p", [2, 3, 4])
def test_symbolic_pattern_equals_numeric(p):
    # generic separable coefficients: numerical nonzeros of S = symbolic pattern
    m = Mesh(3, 3, 3)
    lat = Lattice(m, "grad", p)
    rng = np.random.default_rng(p)
    co = rng.uniform(0.5, 2.0, (m.ncells, 6))
    P = auxop.separable_operator(lat, co)
    R = schwarz.SCRelaxGrad(lat, P)
    pat = schwarz.symbolic_schur_pattern_grad(lat)
    S = R.S.toarray()
    numeric = np.abs(S) > 1e-12 * np.abs(S).max()
    sym = pat[R.G][:, R.G].toarray().astype(bool)
    assert (numeric == sym).all()


def test_symbolic_pattern_contains_distorted():
    # the auxiliary operator keeps the Cartesian pattern on any geometry (Remark in Sec. 4.4)
    m = Mesh(2, 2, 2)
    m.vertices[13] += [0.05, -0.03, 0.02]
    lat = Lattice(m, "grad", 3)
    P = auxop.paper_operator(lat, lambda X: 1 + X[:, 0] ** 2, 0.4)
    R = schwarz.SCRelaxGrad(lat, P)
    pat = schwarz.symbolic_schur_pattern_grad(lat)[R.G][:, R.G].toarray().astype(bool)
    S = R.S.toarray()
    assert (np.abs(S[~pat]) < 1e-13 * np.abs(S).max()).all()


def test_ic_full_pattern_is_cholesky():
    rng = np.random.default_rng(0)
    M = rng.standard_normal((30, 30))
    S = M @ M.T + 30 * np.eye(30)
    L = schwarz.ic_on_pattern(S, np.ones((30, 30), dtype=bool))
    assert np.allclose(L, np.linalg.cholesky(S), atol=1e-12)


def test_ic_drops_fill_outside_pattern():
    # tridiagonal pattern on a matrix with an off-band entry: L stays banded
    S = np.array([[4.0, 1, 1], [1, 4, 1], [1, 1, 4]])
    pat = np.array([[1, 1, 0], [1, 1, 1], [0, 1, 1]], dtype=bool)
    L = schwarz.ic_on_pattern(S, pat)
    assert L[2, 0] == 0.0
    assert np.isclose(L[1, 0], 0.5) and np.isclose(L[1, 1], np.sqrt(4 - 0.25))
    assert np.isclose(L[2, 1], 1 / np.sqrt(3.75))


def test_ic_breakdown_detected():
    S = np.array([[1.0, 2.0], [2.0, 1.0]])
    with pytest.raises(schwarz.ICBreakdown):
        schwarz.ic_on_pattern(S, np.ones((2, 2), dtype=bool))


def test_single_patch_exact_inverse():
    # one interior vertex (n=2), Cholesky patch, P = A: the SC relaxation is A^{-1}
    m = Mesh(2, 2, 2)
    lat = Lattice(m, "grad", 3)
    A = asm.with_dirichlet(lat, asm.cartesian_operator(lat, 1.7, 0.2))
    P = auxop.separable_operator(lat, auxop.cartesian_coefficient_array(lat, 1.7, 0.2))
    R = schwarz.SCRelaxGrad(lat, P, factor="chol")
    # only the interior vertex patch covers the full interface: drop the others
    keep = [i for i, (v, _) in enumerate(R.patches) if v == 13]
    R.patches = [R.patches[i] for i in keep]
    R.factors = [R.factors[i] for i in keep]
    b = np.where(lat.dirichlet_mask(), 0.0, np.random.default_rng(2).standard_normal(lat.ndofs))
    x = spla.spsolve(A.tocsc(), b)
    assert np.abs(R.apply(b) - x).max() < 1e-11 * np.abs(x).max()


def test_relax_symmetric_positive_definite():
    m = Mesh(3, 3, 3)
    lat = Lattice(m, "grad", 3)
    co = np.random.default_rng(5).uniform(0.3, 3.0, (m.ncells, 6))
    R = schwarz.SCRelaxGrad(lat, auxop.separable_operator(lat, co))
    free = np.where(~lat.dirichlet_mask())[0]
    Mi = np.zeros((free.size, free.size))
    for k, g in enumerate(free):
        e = np.zeros(lat.ndofs)
        e[g] = 1.0
        Mi[:, k] = R.apply(e)[free]
    assert np.abs(Mi - Mi.T).max() < 1e-12 * np.abs(Mi).max()
    assert np.linalg.eigvalsh(0.5 * (Mi + Mi.T)).min() > 0


def test_prolongation_reproduces_trilinear():
    m = Mesh(2, 3, 2)
    p = 4
    latf, latc = Lattice(m, "grad", p), Lattice(m, "grad", 1)
    Pr = pmg.prolongation(latf, latc)
    # coarse vertex values of a function vanishing on the boundary (only interior vertices)
    co_c = latc.coords()
    uc = np.where(latc.dirichlet_mask(), 0.0, 1.0 + co_c[:, 1] + 2 * co_c[:, 2] - co_c[:, 3])
    uf = Pr @ uc
    # fine FDM coefficients of the same piecewise-trilinear function, per cell
    el = Element1D(p)
    E = p1_embedding(el)
    cdf, cdc = latf.cell_dofs(), latc.cell_dofs()
    for k in range(m.ncells):
        assert np.allclose(uf[cdf[k]], np.kron(E, np.kron(E, E)) @ uc[cdc[k]], atol=1e-13)


def _solver(n, p, al, be, factor="ic"):
    m = Mesh(n, n, n)
    lat, latc = Lattice(m, "grad", p), Lattice(m, "grad", 1)
    A = asm.with_dirichlet(lat, asm.cartesian_operator(lat, al, be))
    R = schwarz.SCRelaxGrad(lat, auxop.separable_operator(lat, auxop.cartesian_coefficient_array(lat, al, be)), factor)
    Pr = pmg.prolongation(lat, latc)
    cs = pmg.CoarseSolver(latc, asm.with_dirichlet(latc, asm.cartesian_operator(latc, al, be)))
    return lat, A, R, Pr, cs


def test_lanczos_estimate_below_exact():
    lat, A, R, Pr, cs = _solver(2, 3, 1.0, 1.0)
    mask = lat.dirichlet_mask()
    free = np.where(~mask)[0]
    Mi = np.zeros((free.size, free.size))
    for k, g in enumerate(free):
        e = np.zeros(lat.ndofs)
        e[g] = 1.0
        Mi[:, k] = R.apply(e)[free]
    lam_exact = np.linalg.eigvals(Mi @ A.toarray()[np.ix_(free, free)]).real.max()
    v0 = np.where(mask, 0.0, synth.uniform_pm1(7, lat.ndofs))
    lam = pmg.lanczos_lambda_max(A, lambda r: np.where(mask, 0.0, R.apply(r)), v0)
    assert lam <= lam_exact * (1 + 1e-10)
    assert lam >= 0.9 * lam_exact


@pytest.mark.parametrize("n,p", [(4, 4), (3, 5)])
def test_pcg_reaches_direct_solution(n, p):
    al = synth.cell_coefficients(n ** 3, 1)
    be = synth.cell_coefficients(n ** 3, 2)
    lat, A, R, Pr, cs = _solver(n, p, al, be)
    mask = lat.dirichlet_mask()
    v0 = np.where(mask, 0.0, synth.uniform_pm1(99, lat.ndofs))
    lam = pmg.lanczos_lambda_max(A, lambda r: np.where(mask, 0.0, R.apply(r)), v0)
    V = pmg.VCycle(lat, A, R, Pr, cs, pmg.omega_from_lambda(lam))
    b = np.where(mask, 0.0, synth.rhs_values(lat.ndofs, 0))
    x, it, hist = pmg.pcg(A, b, V, rtol=1e-8)
    xs = spla.spsolve(A.tocsc(), b)
    assert np.linalg.norm(b - A @ x) <= 1e-8 * np.linalg.norm(b)
    eA = np.sqrt((x - xs) @ (A @ (x - xs)) / (xs @ (A @ xs)))
    assert eA < 1e-7
    # iteration count inside the band of Table hgrad-iter (SC-ICC, Cartesian: 10-11)
    assert 8 <= it <= 16


def test_vcycle_symmetric_positive_definite():
    """With the same symmetric smoother before and after an exact coarse correction,
    the V(1,1) cycle's error propagation (I - S A)(I - P A0^{-1} P^T A)(I - S A) is
    self-adjoint in the A inner product, so the cycle is a symmetric operator on the
    free DoFs, and positive for a damping below 2 / lambda_max(S A).  A residual taken
    against the wrong iterate, a coarse correction that skips the transpose, or an
    unequal pre- and post-smoothing breaks the symmetry."""
    n, p = 3, 3
    al = synth.cell_coefficients(n ** 3, 3)
    be = synth.cell_coefficients(n ** 3, 4)
    lat, A, R, Pr, cs = _solver(n, p, al, be)
    mask = lat.dirichlet_mask()
    v0 = np.where(mask, 0.0, synth.uniform_pm1(5, lat.ndofs))
    lam = pmg.lanczos_lambda_max(A, lambda r: np.where(mask, 0.0, R.apply(r)), v0)
    V = pmg.VCycle(lat, A, R, Pr, cs, pmg.omega_from_lambda(lam))
    us = [np.where(mask, 0.0, synth.uniform_pm1(20 + k, lat.ndofs)) for k in range(3)]
    Vu = [V(u) for u in us]
    for i in range(3):
        assert us[i] @ Vu[i] > 0
        for j in range(i + 1, 3):
            a, b = us[i] @ Vu[j], us[j] @ Vu[i]
            assert abs(a - b) <= 1e-12 * np.sqrt((us[i] @ Vu[i]) * (us[j] @ Vu[j])), (i, j, a, b)
    # the same check fails for a cycle whose post-smoothing uses the first residual
    class Skewed(pmg.VCycle):
        def __call__(self, r):
            r = np.where(self.dmask, 0.0, r)
            z = self.omega * np.where(self.dmask, 0.0, self.relax.apply(r))
            r1 = r - self.A @ z
            r1[self.dmask] = 0.0
            z = z + self.Pr @ self.coarse.solve(self.Pr.T @ r1)
            return z + self.omega * np.where(self.dmask, 0.0, self.relax.apply(r1))
    S = Skewed(lat, A, R, Pr, cs, pmg.omega_from_lambda(lam))
    a, b = us[0] @ S(us[1]), us[1] @ S(us[0])
    assert abs(a - b) > 1e-8 * abs(a)


def test_full_star_single_patch_exact_inverse():
    # n = 2, all faces Dirichlet: the centre vertex's full star holds every free DoF,
    # so with exact factors its solve alone is A^{-1} (P = A on Cartesian cells)
    m = Mesh(2, 2, 2)
    lat = Lattice(m, "grad", 3)
    A = asm.with_dirichlet(lat, asm.cartesian_operator(lat, 0.6, 2.5))
    P = auxop.separable_operator(lat, auxop.cartesian_coefficient_array(lat, 0.6, 2.5))
    R = schwarz.PAFWRelaxGrad(lat, P, factor="chol")
    free = np.where(~lat.dirichlet_mask())[0]
    keep = [i for i, (v, d) in enumerate(R.patches) if v == 13]
    assert len(keep) == 1 and np.array_equal(np.sort(R.patches[keep[0]][1]), free)
    R.patches = [R.patches[keep[0]]]
    R.factors = [R.factors[keep[0]]]
    b = np.where(lat.dirichlet_mask(), 0.0, np.random.default_rng(4).standard_normal(lat.ndofs))
    x = spla.spsolve(A.tocsc(), b)
    assert np.abs(R.apply(b) - x).max() < 1e-11 * np.abs(x).max()


def test_full_star_sizes_and_order():
    # an interior vertex's full star is the (2p-1)^3 box around it, x fastest
    m = Mesh(3, 3, 3)
    p = 2
    lat = Lattice(m, "grad", p)
    pts = dict(schwarz.full_star_patches_grad(lat))
    v = 1 + 4 * (1 + 4 * 1)
    co = lat.coords()
    d = co[pts[v], 1:] - np.array([p, p, p])
    assert len(pts[v]) == (2 * p - 1) ** 3
    assert d[:3].tolist() == [[-1, -1, -1], [0, -1, -1], [1, -1, -1]]
    assert d[3].tolist() == [-1, 0, -1]
    # a corner vertex with Dirichlet faces: only the free points of its one cell
    assert len(pts[0]) == (p - 1) ** 3


def test_full_star_relax_spd_and_ic_differs():
    m = Mesh(2, 2, 2)
    lat = Lattice(m, "grad", 3)
    co = np.random.default_rng(8).uniform(0.3, 3.0, (m.ncells, 6))
    P = auxop.separable_operator(lat, co)
    Rc = schwarz.PAFWRelaxGrad(lat, P, factor="chol")
    Ri = schwarz.PAFWRelaxGrad(lat, P, factor="ic")
    free = np.where(~lat.dirichlet_mask())[0]
    for R in (Rc, Ri):
        Mi = np.zeros((free.size, free.size))
        for k, g in enumerate(free):
            e = np.zeros(lat.ndofs)
            e[g] = 1.0
            Mi[:, k] = R.apply(e)[free]
        assert np.abs(Mi - Mi.T).max() < 1e-12 * np.abs(Mi).max()
        assert np.linalg.eigvalsh(0.5 * (Mi + Mi.T)).min() > 0
    r = np.where(lat.dirichlet_mask(), 0.0, np.random.default_rng(9).standard_normal(lat.ndofs))
    assert np.linalg.norm(Rc.apply(r) - Ri.apply(r)) > 1e-6 * np.linalg.norm(Rc.apply(r))
