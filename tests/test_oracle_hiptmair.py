"""Pins of the oracle's SC-PH relaxation for H(curl) and H(div) (Sec. 4.3-4.5), its
exterior derivatives, patches and p-transfers.

What pins what:
  * cell-interior blocks: the FDM bases make the interior coupling of NCE_p/NCF_p
    block diagonal with blocks of at most 3 x 3 (remark of Sec. 4.4).  The block
    counts below are derived by hand from the 1-D orthogonality relations (mass
    and stiffness diagonal on interior modes, D interior-diagonal): for NCE_p per
    cell (p-1)^3 blocks of 3 (one per interior mode triple) and 3(p-1)^2 blocks of
    1 (a zero DP index); for NCF_p (p-1)^3 of 3, 3(p-1)^2 of 2, 3(p-1) of 1.
  * edge stars (H(curl)): the patch matrix splits into p independent blocks, one
    per mode along the edge (Sec. 4.5 and Fig. spy_feec(e)); sizes 4p-3 (mode 0)
    and 8p-3 (modes 1..p-1) by the same counting.
  * face stars (H(div)): no coupling between face DoFs (Sec. 4.5).
  * exterior derivatives: curl grad = 0 and div curl = 0 on the global lattices;
    grad of a constant is zero.
  * transfers: the p=1 operator is the Galerkin product P^T A_p P (the coarse space
    is a subspace and the same form is used, Sec. 4.3), for all three spaces.
  * relaxation: symmetric positive definite (dense on tiny meshes).
  * whole solver: CG iteration counts in the paper's band for alpha = 1,
    beta = 1e-8 with its natural-norm criterion (Tables hcurl-iter, hdiv-iter,
    Cartesian, p = 3: 14-16 and 11-13); dropping the potential term (a plausible
    slip) costs at least 5 more iterations at beta = 1e-4, and at beta = 1e-8 it
    lets the natural-norm criterion stop on a wrong solution (H(curl)).
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from scipy.sparse.csgraph import connected_components

import synth
from oracle.tables1d import Element1D
from oracle.lattice import Mesh, Lattice
from oracle import assemble as asm, hiptmair as hp, pmg


def _relax(space, n, p, al=1.0, be=1.0, dirichlet=0x3F, potential=True):
    m = Mesh(*((n,) * 3 if np.isscalar(n) else n), dirichlet=dirichlet)
    lat = Lattice(m, space, p)
    Araw = asm.cartesian_operator(lat, al, be)
    return lat, Araw, hp.SCRelaxPH(lat, Araw, be, potential=potential)


@pytest.mark.parametrize("space,p", [("curl", 2), ("curl", 3), ("curl", 4), ("div", 2), ("div", 3), ("div", 4)])
def test_interior_block_counts(space, p):
    m = Mesh(2, 2, 2, dirichlet=0)           # no Dirichlet: every cell interior DoF counts
    lat = Lattice(m, space, p)
    al = synth.cell_coefficients(m.ncells, 1)
    be = synth.cell_coefficients(m.ncells, 2)
    c = hp.Condensed(lat, asm.cartesian_operator(lat, al, be))
    hist = np.bincount(c.block_sizes, minlength=4)
    q = p - 1
    if space == "curl":
        expected = [0, 3 * q * q, 0, q ** 3]
    else:
        expected = [0, 3 * q, 3 * q * q, q ** 3]
    assert list(hist[:4]) == [e * m.ncells for e in expected]


@pytest.mark.parametrize("p", [2, 3, 4])
def test_edge_star_splits_into_p_blocks(p):
    lat, Araw, R = _relax("curl", 3, p)
    sizes = [len(d) for _, d in R.patches]
    assert max(sizes) == p + 8 * p * (p - 1)          # an interior edge: the edge and its 4 faces
    for (e, dofs) in R.patches:
        if len(dofs) != max(sizes):
            continue
        loc = R.cond.pos[dofs]
        S = R.cond.S[loc][:, loc].toarray()
        nc, lab = connected_components(np.abs(S) > 1e-13 * np.abs(S).max(), directed=False)
        assert nc == p
        assert sorted(np.bincount(lab)) == sorted([4 * p - 3] + [8 * p - 3] * (p - 1))


@pytest.mark.parametrize("p", [2, 3, 5])
def test_face_star_is_diagonal(p):
    m = Mesh(3, 2, 2)
    lat = Lattice(m, "div", p)
    al = synth.cell_coefficients(m.ncells, 1)
    be = synth.cell_coefficients(m.ncells, 2)
    c = hp.Condensed(lat, asm.cartesian_operator(lat, al, be))
    for f, dofs in hp.face_patches(lat):
        loc = c.pos[dofs]
        S = c.S[loc][:, loc].toarray()
        off = S - np.diag(np.diag(S))
        assert np.abs(off).max() <= 1e-13 * np.abs(S).max()
        assert len(dofs) in (p * p,)


def test_patch_counts_and_membership():
    # 3^3 mesh, Dirichlet everywhere: NCE tangential traces vanish on the boundary,
    # so boundary edges keep only the interior faces through them
    lat, _, R = _relax("curl", 3, 2)
    p = 2
    patches = dict(R.patches)
    # every free interface DoF is in 1 (edge DoF) or 4 (face DoF) patches
    count = np.zeros(lat.ndofs, dtype=int)
    for _, d in R.patches:
        count[d] += 1
    G = R.cond.G
    assert set(np.unique(count[G])) <= {1, 2, 3, 4}
    co = lat.coords()
    for g in G:
        m = co[g, 0]
        on = [co[g, 1 + a] % p == 0 for a in range(3) if a != m]
        if all(on):
            assert count[g] == 1
    # H(div): one patch per face DoF
    latf, _, Rf = _relax("div", 3, 2)
    cnt = np.zeros(latf.ndofs, dtype=int)
    for _, d in Rf.patches:
        cnt[d] += 1
    assert (cnt[Rf.cond.G] == 1).all()


def test_exterior_derivatives_compose_to_zero():
    m = Mesh(3, 2, 2)
    m.vertices[:, 0] *= 1.7
    for p in (1, 2, 4):
        lq, le, lf = Lattice(m, "grad", p), Lattice(m, "curl", p), Lattice(m, "div", p)
        G = hp.exterior_derivative(lq, le)
        C = hp.exterior_derivative(le, lf)
        x = synth.uniform_pm1(3, lq.ndofs)
        y = synth.uniform_pm1(4, le.ndofs)
        assert np.abs(C @ (G @ x)).max() <= 1e-12 * np.abs(G @ x).max()
        assert np.abs(G @ x).max() > 0.1
        # div of the curl, on the reference cell (NCF -> DQ), then summed globally
        el = Element1D(p)
        Dv = asm.ref_div(el)
        cd = lf.cell_dofs()
        w = C @ y
        assert np.abs(np.einsum("ij,kj->ki", Dv, w[cd])).max() <= 1e-12 * np.abs(w).max()
        # the constant function: per axis the FDM coefficients of 1 are 1 at the
        # vertices and (s_i, 1) on interior modes; its gradient is zero
        one = el.dof_functionals(lambda t: np.ones_like(t))
        Ex, Ey, _ = lq.extents[0]
        g = np.arange(lq.ndofs)
        co = [g % Ex, (g // Ex) % Ey, g // (Ex * Ey)]
        c1 = np.prod([np.where(c % p != 0, one[c % p], 1.0) for c in co], axis=0)
        assert np.abs(G @ c1).max() <= 1e-12


@pytest.mark.parametrize("space", ["grad", "curl", "div"])
def test_coarse_operator_is_galerkin_product(space):
    m = Mesh(3, 2, 2)
    m.vertices[:, 2] *= 0.6
    al = synth.cell_coefficients(m.ncells, 1)
    be = synth.cell_coefficients(m.ncells, 2)
    for p in (2, 3, 5):
        lat, latc = Lattice(m, space, p), Lattice(m, space, 1)
        Pr = pmg.prolongation(lat, latc)
        Ap = asm.cartesian_operator(lat, al, be)
        A1 = asm.cartesian_operator(latc, al, be)
        keep = sp.diags((~latc.dirichlet_mask()).astype(float))
        ref = (keep @ A1 @ keep).toarray()
        gal = (Pr.T @ Ap @ Pr).toarray()
        assert np.abs(gal - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("space,p", [("curl", 2), ("curl", 3), ("div", 2), ("div", 3)])
def test_relaxation_symmetric_positive(space, p):
    lat, Araw, R = _relax(space, 2, p, synth.cell_coefficients(8, 1), synth.cell_coefficients(8, 2))
    free = np.where(~lat.dirichlet_mask())[0]
    M = np.zeros((free.size, free.size))
    for j, g in enumerate(free):
        e = np.zeros(lat.ndofs)
        e[g] = 1.0
        M[:, j] = R.apply(e)[free]
    assert np.abs(M - M.T).max() <= 1e-11 * np.abs(M).max()
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > 0


def test_edge_star_solve_equals_dense_inverse():
    lat, _, R = _relax("curl", 2, 3, synth.cell_coefficients(8, 1), synth.cell_coefficients(8, 2))
    rt = synth.uniform_pm1(8, R.cond.G.size)
    ref = np.zeros_like(rt)
    for _, dofs in R.patches:
        loc = R.cond.pos[dofs]
        ref[loc] += np.linalg.inv(R.cond.S[loc][:, loc].toarray()) @ rt[loc]
    assert np.linalg.norm(R.local(rt) - ref) <= 1e-10 * np.linalg.norm(ref)


def _solve(space, n, p, al, be, potential=True, norm="natural"):
    m = Mesh(n, n, n)
    lat, latc = Lattice(m, space, p), Lattice(m, space, 1)
    Araw = asm.cartesian_operator(lat, al, be)
    A = asm.with_dirichlet(lat, Araw)
    R = hp.SCRelaxPH(lat, Araw, be, potential=potential)
    Pr = pmg.prolongation(lat, latc)
    cs = pmg.CoarseSolver(latc, asm.with_dirichlet(latc, asm.cartesian_operator(latc, al, be)))
    mask = lat.dirichlet_mask()
    v0 = np.where(mask, 0.0, synth.uniform_pm1(99, lat.ndofs))
    lam = pmg.lanczos_lambda_max(A, lambda r: np.where(mask, 0.0, R.apply(r)), v0)
    V = pmg.VCycle(lat, A, R, Pr, cs, pmg.omega_from_lambda(lam))
    b = np.where(mask, 0.0, synth.rhs_values(lat.ndofs, 0))
    x, it, _ = pmg.pcg(A, b, V, maxit=120, norm=norm)
    xs = spla.spsolve(A.tocsc(), b)
    e = x - xs
    return it, np.sqrt(e @ (A @ e) / (xs @ (A @ xs)))


@pytest.mark.parametrize("space,band", [("curl", (12, 18)), ("div", (10, 15))])
def test_iterations_in_paper_band(space, band):
    it, err = _solve(space, 3, 3, 1.0, 1e-8)
    assert band[0] <= it <= band[1]
    assert err < 1e-4


def test_potential_term_matters():
    for space in ("curl", "div"):
        it_full, _ = _solve(space, 3, 3, 1.0, 1e-4)
        it_drop, _ = _solve(space, 3, 3, 1.0, 1e-4, potential=False)
        assert it_drop >= it_full + 5
    _, err_full = _solve("curl", 3, 3, 1.0, 1e-8)
    _, err_drop = _solve("curl", 3, 3, 1.0, 1e-8, potential=False)
    assert err_full < 1e-4 < 1e-3 < err_drop


def test_pafw_vec_star_membership_brute_force():
    # a free DoF is in the star of v iff every cell whose local DoFs include it is one
    # of the cells around v (checked from the cell-to-DoF map)
    from oracle import hiptmair as hp2
    for space in ("curl", "div"):
        m = Mesh(3, 2, 2, dirichlet=0x15)
        lat = Lattice(m, space, 2)
        cd = lat.cell_dofs()
        nx, ny, nz = m.nx, m.ny, m.nz
        support = [set() for _ in range(lat.ndofs)]
        for c in range(m.ncells):
            for g in cd[c]:
                support[g].add(c)
        free = ~lat.dirichlet_mask()
        got = dict(hp2.vertex_star_patches_vec(lat))
        for vz in range(nz + 1):
            for vy in range(ny + 1):
                for vx in range(nx + 1):
                    cells = {cx + nx * (cy + ny * cz) for cx in (vx - 1, vx) for cy in (vy - 1, vy)
                             for cz in (vz - 1, vz) if 0 <= cx < nx and 0 <= cy < ny and 0 <= cz < nz}
                    want = [g for g in range(lat.ndofs) if free[g] and support[g] <= cells]
                    vid = vx + (nx + 1) * (vy + (ny + 1) * vz)
                    assert list(got.get(vid, [])) == want, (space, vid)


@pytest.mark.parametrize("space", ["curl", "div"])
def test_pafw_vec_single_star_exact_and_spd(space):
    from oracle import hiptmair as hp2
    lat = Lattice(Mesh(2, 2, 2), space, 2)
    A = asm.with_dirichlet(lat, asm.cartesian_operator(lat, 1.3, 0.4))
    R = hp2.PAFWRelaxVec(lat, A)
    free = np.where(~lat.dirichlet_mask())[0]
    Mi = np.zeros((free.size, free.size))
    for k, g in enumerate(free):
        e = np.zeros(lat.ndofs)
        e[g] = 1.0
        Mi[:, k] = R.apply(e)[free]
    assert np.abs(Mi - Mi.T).max() < 1e-12 * np.abs(Mi).max()
    assert np.linalg.eigvalsh(0.5 * (Mi + Mi.T)).min() > 0
    keep = [i for i, (v, d) in enumerate(R.patches) if v == 13]
    R.patches, R.factors = [R.patches[keep[0]]], [R.factors[keep[0]]]
    b = np.where(lat.dirichlet_mask(), 0.0, np.random.default_rng(6).standard_normal(lat.ndofs))
    x = spla.spsolve(A.tocsc(), b)
    assert np.abs(R.apply(b) - x).max() < 1e-11 * np.abs(x).max()


@pytest.mark.parametrize("space", ["curl", "div"])
def test_sc_pafw_one_cell_is_eight_exact_solves(space):
    # one cell, no Dirichlet face: each of the 8 vertex stars holds every interface
    # DoF, so the interface part of SC-PAFW is 8 S^{-1} rt, i.e. 8 times the
    # interface values of the exact solve A^{-1} r (a dense solve)
    lat = Lattice(Mesh(1, 1, 1, dirichlet=0), space, 3)
    A = asm.cartesian_operator(lat, 1.7, 0.6)
    R = hp.SCPAFWRelaxVec(lat, A)
    assert len(R.patches) == 8
    r = synth.uniform_pm1(7, lat.ndofs)
    z = R.apply(r)
    x = np.linalg.solve(A.toarray(), r)
    G = R.cond.G
    assert np.abs(z[G] - 8.0 * x[G]).max() < 1e-10 * np.abs(x[G]).max()
    # the interior follows from the interface by the exact back-substitution
    I = R.cond.I
    zI = np.linalg.solve(A.toarray()[np.ix_(I, I)], r[I] - A.toarray()[np.ix_(I, G)] @ z[G])
    assert np.abs(z[I] - zI).max() < 1e-10 * np.abs(zI).max()


@pytest.mark.parametrize("space", ["curl", "div"])
def test_sc_pafw_spd_and_stars_on_the_interface(space):
    lat = Lattice(Mesh(2, 2, 2), space, 2)
    nc = 8
    al, be = synth.cell_coefficients(nc, 1), synth.cell_coefficients(nc, 2)
    A = asm.with_dirichlet(lat, asm.cartesian_operator(lat, al, be))
    R = hp.SCPAFWRelaxVec(lat, asm.cartesian_operator(lat, al, be))
    inner = hp.interior_mask(lat)
    for _, d in R.patches:
        assert not inner[d].any()
    free = np.where(~lat.dirichlet_mask())[0]
    M = np.column_stack([R.apply(np.eye(lat.ndofs)[k])[free] for k in free])
    assert np.abs(M - M.T).max() < 1e-10 * np.abs(M).max()
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > 0


@pytest.mark.parametrize("space,count", [("curl", 12), ("div", 6)])
def test_ph_one_cell_stars_are_exact_solves(space, count):
    # one cell, no Dirichlet face: each of the cell's 12 edges (6 faces) has the whole
    # cell as its star, so without the potential term PH is count times A^{-1}
    lat = Lattice(Mesh(1, 1, 1, dirichlet=0), space, 2)
    A = asm.cartesian_operator(lat, 1.7, 0.6)
    R = hp.PHRelaxVec(lat, A, 0.6)
    assert len(R.patches) == count and all(d.size == lat.ndofs for _, d in R.patches)
    r = synth.uniform_pm1(9, lat.ndofs)
    x = np.linalg.solve(A.toarray(), r)
    assert np.abs(R.apply(r, potential=False) - count * x).max() < 1e-10 * np.abs(x).max()


@pytest.mark.parametrize("space,dim", [("curl", 1), ("div", 2), ("curl", 2)])
def test_entity_stars_by_brute_force(space, dim):
    # a DoF lies in the star of an entity exactly when every cell whose closure holds
    # the DoF's support point contains the entity (checked cell by cell)
    lat = Lattice(Mesh(3, 2, 2), space, 2)
    pl = hp.entity_star_patches(lat, dim)
    co = lat.coords()
    cd = lat.cell_dofs()
    holders = [set() for _ in range(lat.ndofs)]
    for c in range(cd.shape[0]):
        for g in cd[c]:
            holders[g].add(c)
    n = (3, 2, 2)

    def cells_of(eid):
        base = 0
        for m in range(3):
            cell_axes = [m] if dim == 1 else [a for a in range(3) if a != m]
            ext = [n[a] if a in cell_axes else n[a] + 1 for a in range(3)]
            cnt = ext[0] * ext[1] * ext[2]
            if eid < base + cnt:
                k = eid - base
                c = (k % ext[0], (k // ext[0]) % ext[1], k // (ext[0] * ext[1]))
                out = set()
                for cz in range(n[2]):
                    for cy in range(n[1]):
                        for cx in range(n[0]):
                            cc = (cx, cy, cz)
                            if all((cc[a] == c[a]) if a in cell_axes else (cc[a] in (c[a] - 1, c[a]))
                                   for a in range(3)):
                                out.add(cx + n[0] * (cy + n[1] * cz))
                return out
            base += cnt
    free = ~lat.dirichlet_mask()
    for eid, d in pl:
        cells = cells_of(eid)
        want = [g for g in range(lat.ndofs) if free[g] and holders[g] <= cells]
        assert sorted(want) == list(d)
