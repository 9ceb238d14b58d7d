"""Statically condensed Pavarino-Hiptmair relaxation for H(curl) and H(div)
(oracle; test infrastructure).

Sec. 4.3, eq. ph (the space decomposition) and eq. asm-hiptmair; Sec. 4.4, eqs.
sc-ph and sc-asm-hiptmair with eq. schur for the cell interiors; Sec. 4.5 (edge
stars solved by a Cholesky factorisation, the vertex-star potential problem by
incomplete Cholesky on the static-condensation pattern, face stars exactly); the
remark of Sec. 4.3 on the singular H(div) potential problem.

  z_I  = P_II^{-1} r_I
  rt   = r_G - P_GI z_I
  z_G  = sum_i R_i^T S_i^{-1} R_i rt  +  Dt (sum_j R_j^T Bt_j^{-1} R_j) Dt^T rt
  z_I -= P_II^{-1} P_IG z_G

Readings of the paper (it fixes none of these):
  * patches: every mesh entity of dimension k (edges for H(curl), faces for H(div))
    has a star; its patch holds the free interface DoFs of the entities whose
    closure contains that entity and that lie in the star: for an edge, the edge
    itself and the (up to four) faces through it; for a face, the face.  Empty
    patches are dropped; patch ids run over the axis of the entity, then lattice
    order.  The local solves are exact (Cholesky), so the order inside a patch
    does not change the result (lattice order here).
  * potential spaces and their operators: k = 1: Q_p on the same mesh and
    Dirichlet faces, B = (grad phi, beta grad psi), vertex-star patches of its
    interface Schur complement factored by incomplete Cholesky on the symbolic
    static-condensation pattern (as for H(grad)); k = 2: NCE_p on the same mesh
    and Dirichlet faces, B = (curl phi, beta curl psi) + eps (phi, beta psi)
    (eps = 1e-3: the small multiple of the mass matrix of the remark), edge-star
    patches of its interface Schur complement, exact Cholesky.
  * Dt = D_GG: the rows of the free interface DoFs of V^k and the columns of the
    free interface DoFs of V^{k-1} of the global matrix of d^{k-1} written in FDM
    coefficients.
  * P = A (Cartesian cells, cellwise-constant coefficients); P_II is block diagonal
    with blocks of at most 3 x 3 (remark of Sec. 4.4) and is inverted exactly, block
    by block.
  * Dirichlet rows: z_D = r_D.
"""
import numpy as np
import scipy.linalg
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

from .tables1d import Element1D
from .lattice import Lattice
from .assemble import ref_grad, ref_curl, cartesian_operator
from .auxop import separable_operator, cartesian_coefficient_array
from .schwarz import interior_mask, SCRelaxGrad, full_star_patches_grad

EPS_HDIV = 1e-3


# ----------------------------------------------------------------------------------
# the exterior derivative between global FDM spaces
# ----------------------------------------------------------------------------------
def exterior_derivative(lat_from: Lattice, lat_to: Lattice):
    """Sparse (ndofs_to x ndofs_from) matrix of d^{k-1} in FDM coefficients: grad
    Q_p -> NCE_p or curl NCE_p -> NCF_p.  On a cell the reference derivative maps
    reference coefficients to reference coefficients (the Piola maps of Sec. 3.1
    make them the physical ones), and the FDM bases are conforming, so each global
    row is the row of any one cell holding that DoF."""
    el = Element1D(lat_from.p)
    pair = (lat_from.space, lat_to.space)
    if pair == ("grad", "curl"):
        R = ref_grad(el)
    elif pair == ("curl", "div"):
        R = ref_curl(el)
    else:
        raise ValueError(pair)
    cdf, cdt = lat_from.cell_dofs(), lat_to.cell_dofs()
    owner = -np.ones(lat_to.ndofs, dtype=np.int64)
    for k in range(cdt.shape[0]):
        new = owner[cdt[k]] < 0
        owner[cdt[k][new]] = k
    r_, c_ = np.nonzero(R)
    rows, cols, vals = [], [], []
    for k in range(cdt.shape[0]):
        g = cdt[k, r_]
        sel = owner[g] == k
        rows.append(g[sel])
        cols.append(cdf[k, c_[sel]])
        vals.append(R[r_[sel], c_[sel]])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(lat_to.ndofs, lat_from.ndofs))


# ----------------------------------------------------------------------------------
# patches of entities of dimension k
# ----------------------------------------------------------------------------------
def _axes(m):
    return [a for a in range(3) if a != m]


def edge_patches(lat: Lattice):
    """NCE_p: list of (edge id, free interface DoFs) over all edges with a non-empty
    patch, edge ids by axis then lattice order (x fastest)."""
    assert lat.space == "curl"
    p, n = lat.p, lat.mesh.n
    free = ~lat.dirichlet_mask() & ~interior_mask(lat)
    co = lat.coords()
    # edge along m: (cell index along m, vertex index along the other two axes)
    ext = []
    for m in range(3):
        e = [n[a] if a == m else n[a] + 1 for a in range(3)]
        ext.append(e)
    off = np.cumsum([0] + [int(np.prod(e)) for e in ext])

    def eid(m, c):
        e = ext[m]
        return off[m] + c[0] + e[0] * (c[1] + e[1] * c[2])

    members = {}
    for g in np.where(free)[0]:
        m = int(co[g, 0])
        X = co[g, 1:]
        a, b = _axes(m)
        on_a, on_b = X[a] % p == 0, X[b] % p == 0
        cm = X[m] // p
        edges = []
        if on_a and on_b:                       # an edge DoF
            c = [0, 0, 0]
            c[m], c[a], c[b] = cm, X[a] // p, X[b] // p
            edges.append(eid(m, c))
        else:                                   # a face DoF: the face's four edges
            fa, fb = (a, b) if on_a else (b, a)  # fa: normal of the face, fb: its other axis
            va, cb = X[fa] // p, X[fb] // p
            for vb in (cb, cb + 1):             # the two edges along m
                c = [0, 0, 0]
                c[m], c[fa], c[fb] = cm, va, vb
                edges.append(eid(m, c))
            for vm in (cm, cm + 1):             # the two edges along fb
                c = [0, 0, 0]
                c[fb], c[fa], c[m] = cb, va, vm
                edges.append(eid(fb, c))
        for e in edges:
            members.setdefault(int(e), []).append(g)
    return [(e, np.array(sorted(members[e]), dtype=np.int64)) for e in sorted(members)]


def face_patches(lat: Lattice):
    """NCF_p: list of (face id, free interface DoFs) over faces with a non-empty
    patch, face ids by normal axis then lattice order (x fastest)."""
    assert lat.space == "div"
    p, n = lat.p, lat.mesh.n
    free = ~lat.dirichlet_mask() & ~interior_mask(lat)
    co = lat.coords()
    ext = []
    for m in range(3):
        ext.append([n[a] + 1 if a == m else n[a] for a in range(3)])
    off = np.cumsum([0] + [int(np.prod(e)) for e in ext])
    members = {}
    for g in np.where(free)[0]:
        m = int(co[g, 0])
        X = co[g, 1:]
        c = [X[a] // p for a in range(3)]       # vertex plane along m, cells along the others
        e = ext[m]
        f = int(off[m] + c[0] + e[0] * (c[1] + e[1] * c[2]))
        members.setdefault(f, []).append(g)
    return [(f, np.array(sorted(members[f]), dtype=np.int64)) for f in sorted(members)]


# ----------------------------------------------------------------------------------
# static condensation of one operator
# ----------------------------------------------------------------------------------
class Condensed:
    """Interior/interface split of the free DoFs of P, the exact block factorisation
    of P_II (blocks of at most 3 x 3, P_II = L L^T block by block) and the interface
    Schur complement (eqs. LDU, schur) in the symmetric form
    S = P_GG - W^T W with W = L^{-1} P_IG (for tiny beta the blocks of P_II are
    nearly singular along discrete gradients; this form keeps S symmetric positive
    definite in floating point)."""

    def __init__(self, lat: Lattice, P):
        P = sp.csr_matrix(P)
        mask = lat.dirichlet_mask()
        inner = interior_mask(lat)
        self.I = np.where(inner & ~mask)[0]
        self.G = np.where(~inner & ~mask)[0]
        PII = P[self.I][:, self.I].tocsr()
        ncomp, lab = connected_components(PII != 0, directed=False)
        sizes = np.bincount(lab, minlength=ncomp)
        if sizes.size and sizes.max() > 3:
            raise ValueError("P_II has a block larger than 3 x 3")
        self.block_sizes = sizes
        rows, cols, vals = [], [], []
        order = np.argsort(lab, kind="stable")
        starts = np.concatenate([[0], np.cumsum(sizes)])
        for b in range(ncomp):
            idx = np.sort(order[starts[b]:starts[b + 1]])
            blk = PII[idx][:, idx].toarray()
            Linv = scipy.linalg.solve_triangular(np.linalg.cholesky(blk), np.eye(idx.size), lower=True)
            rr, cc = np.meshgrid(idx, idx, indexing="ij")
            rows.append(rr.ravel())
            cols.append(cc.ravel())
            vals.append(Linv.ravel())
        n = self.I.size
        if n:
            self.Linv = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                                      shape=(n, n))
        else:                       # p = 1: no cell-interior DoF
            self.Linv = sp.csr_matrix((0, 0))
        self.PGI = P[self.G][:, self.I].tocsr()
        self.PIG = P[self.I][:, self.G].tocsr()
        W = self.Linv @ self.PIG
        self.S = sp.csr_matrix(P[self.G][:, self.G] - W.T @ W)
        pos = -np.ones(lat.ndofs, dtype=np.int64)
        pos[self.G] = np.arange(self.G.size)
        self.pos = pos
        self.mask = mask

    def solve_II(self, v):
        """P_II^{-1} v, block by block through the Cholesky factors."""
        return self.Linv.T @ (self.Linv @ v)


class PatchSolves:
    """sum_i R_i^T S_i^{-1} R_i with S_i = S[patch, patch] factored by Cholesky."""

    def __init__(self, cond: Condensed, patches):
        self.patches = patches
        self.loc = [cond.pos[d] for _, d in patches]
        self.factors = []
        for loc in self.loc:
            Si = cond.S[loc][:, loc].toarray()
            self.factors.append(scipy.linalg.cho_factor(Si, lower=True))
        self.n = cond.G.size

    def __call__(self, rt):
        z = np.zeros(self.n)
        for loc, f in zip(self.loc, self.factors):
            z[loc] += scipy.linalg.cho_solve(f, rt[loc])
        return z


# ----------------------------------------------------------------------------------
# the relaxation
# ----------------------------------------------------------------------------------
class SCRelaxPH:
    """z = M^{-1} r for SC-PH (H(curl) or H(div)) on the operator P of the Riesz map
    with cellwise coefficients beta (the potential problem's weight) on a Cartesian
    mesh."""

    def __init__(self, lat: Lattice, P, beta, eps=EPS_HDIV, potential=True):
        self.lat = lat
        self.cond = cond = Condensed(lat, P)
        self.potential = potential
        mesh, p = lat.mesh, lat.p
        if lat.space == "curl":
            self.patches = edge_patches(lat)
            self.local = PatchSolves(cond, self.patches)
            latQ = Lattice(mesh, "grad", p)
            B = separable_operator(latQ, cartesian_coefficient_array(latQ, beta, 0.0))
            self.pot = SCRelaxGrad(latQ, B)
            self.pot_lat = latQ
            potG, self.pot_sum = self.pot.G, self.pot.patch_sum
            D = exterior_derivative(latQ, lat)
        elif lat.space == "div":
            self.patches = face_patches(lat)
            self.local = PatchSolves(cond, self.patches)
            latE = Lattice(mesh, "curl", p)
            be = np.broadcast_to(np.asarray(beta, dtype=np.float64), (mesh.ncells,))
            B = cartesian_operator(latE, be, eps * be)
            self.pot = Condensed(latE, B)
            self.pot_lat = latE
            self.pot_patches = edge_patches(latE)
            potG, self.pot_sum = self.pot.G, PatchSolves(self.pot, self.pot_patches)
            D = exterior_derivative(latE, lat)
        else:
            raise ValueError(lat.space)
        self.Dt = sp.csr_matrix(D[cond.G][:, potG])

    def interface_solve(self, rt):
        """The interface part of eq. sc-asm-hiptmair (without the coarse term)."""
        z = self.local(rt)
        if self.potential:
            z = z + self.Dt @ self.pot_sum(self.Dt.T @ rt)
        return z

    def apply(self, r):
        c = self.cond
        r = np.asarray(r, dtype=np.float64)
        z = np.zeros_like(r)
        zI = c.solve_II(r[c.I])
        rt = r[c.G] - c.PGI @ zI
        zG = self.interface_solve(rt)
        zI = zI - c.solve_II(c.PIG @ zG)
        z[c.I] = zI
        z[c.G] = zG
        z[c.mask] = r[c.mask]
        return z


# ----------------------------------------------------------------------------------
# PAFW without static condensation for H(curl) / H(div) (Sec. 4.3, eq. pafw): the
# vertex stars of the k-forms, every DoF whose support lies in the cells around a
# vertex, with exact patch solves (the PAFW column of Tables hcurl-iter / hdiv-iter).
# ----------------------------------------------------------------------------------
def vertex_star_patches_vec(lat: Lattice):
    """List of (vertex_id, dof array, ascending) of the non-empty vertex stars: a free
    DoF belongs to the star of vertex v when every cell holding it (along each axis:
    the cell of a DP coordinate, the one or two existing cells of a continuous
    coordinate, two on an interior vertex plane) is among the cells v_a - 1, v_a."""
    mesh, p = lat.mesh, lat.p
    nc = (mesh.nx, mesh.ny, mesh.nz)
    co = lat.coords()
    free = ~lat.dirichlet_mask()
    comp = co[:, 0]
    lo = np.zeros((lat.ndofs, 3), dtype=np.int64)
    hi = np.zeros((lat.ndofs, 3), dtype=np.int64)
    for a in range(3):
        C = co[:, 1 + a]
        cont = np.array([lat.kinds[m][a] == "P" for m in range(len(lat.kinds))])[comp]
        c = C // p
        on = cont & (C % p == 0)
        lo[:, a] = np.where(on, np.maximum(c - 1, 0), np.minimum(c, nc[a] - 1))
        hi[:, a] = np.where(on, np.minimum(c, nc[a] - 1), np.minimum(c, nc[a] - 1))
    out = []
    nvx, nvy, nvz = nc[0] + 1, nc[1] + 1, nc[2] + 1
    for vz in range(nvz):
        for vy in range(nvy):
            for vx in range(nvx):
                v = np.array([vx, vy, vz])
                inside = np.all((lo >= v - 1) & (hi <= v), axis=1) & free
                sel = np.where(inside)[0]
                if sel.size:
                    out.append((vx + nvx * (vy + nvy * vz), sel))
    return out


class PAFWRelaxVec:
    """z = M^{-1} r for PAFW on H(curl) / H(div) without static condensation:
    z = sum_v R_v^T P_v^{-1} R_v r over the vertex stars (exact Cholesky of each
    P_v = R_v P R_v^T); Dirichlet rows copy r."""

    def __init__(self, lat: Lattice, P):
        P = sp.csr_matrix(P)
        self.dmask = lat.dirichlet_mask()
        self.patches = vertex_star_patches_vec(lat)
        self.factors = [np.linalg.cholesky(P[d][:, d].toarray()) for _, d in self.patches]

    def apply(self, r):
        r = np.asarray(r, dtype=np.float64)
        z = np.zeros_like(r)
        for (vid, dofs), L in zip(self.patches, self.factors):
            y = scipy.linalg.solve_triangular(L, r[dofs], lower=True)
            z[dofs] += scipy.linalg.solve_triangular(L.T, y, lower=False)
        z[self.dmask] = r[self.dmask]
        return z


# ----------------------------------------------------------------------------------
# SC-PAFW for H(curl) / H(div) (Sec. 4.4, eq. sc-asm-afw on the k-forms): the vertex
# stars of the non-condensed PAFW restricted to the free interface DoFs, each solved
# exactly on the interface Schur complement; no potential term (the vertex stars
# already hold the kernel of the derivative).  The SC-PAFW column of Tables
# hcurl-iter / hdiv-iter.
# ----------------------------------------------------------------------------------
class SCPAFWRelaxVec(SCRelaxPH):
    """z = M^{-1} r for SC-PAFW: P_II solved exactly per cell, the interface by
    sum_v R_v^T S_v^{-1} R_v over the vertex stars of the interface DoFs, then the
    interior back-substitution; Dirichlet rows copy r."""

    def __init__(self, lat: Lattice, P):
        self.lat = lat
        self.cond = cond = Condensed(lat, P)
        self.potential = False
        inner = interior_mask(lat)
        self.patches = [(vid, d[~inner[d]]) for vid, d in vertex_star_patches_vec(lat) if (~inner[d]).any()]
        self.local = PatchSolves(cond, self.patches)


# ----------------------------------------------------------------------------------
# PH without static condensation for H(curl) / H(div) (Sec. 4.3, eq. ph with eq.
# asm-hiptmair): the stars of the k-dimensional entities (edges for H(curl), faces for
# H(div)) holding every free DoF whose cells all contain the entity, solved exactly,
# plus the potential term through the full stars of the potential space (vertex stars
# of Q_p, resp. edge stars of NCE_p) and the full exterior derivative.  The PH column
# of Tables hcurl-iter / hdiv-iter.
# ----------------------------------------------------------------------------------
def _holding_cells(lat: Lattice):
    """Per free DoF and axis, the range lo..hi of the cells holding it (as in
    vertex_star_patches_vec)."""
    mesh, p = lat.mesh, lat.p
    nc = (mesh.nx, mesh.ny, mesh.nz)
    co = lat.coords()
    comp = co[:, 0]
    lo = np.zeros((lat.ndofs, 3), dtype=np.int64)
    hi = np.zeros((lat.ndofs, 3), dtype=np.int64)
    for a in range(3):
        C = co[:, 1 + a]
        cont = np.array([lat.kinds[m][a] == "P" for m in range(len(lat.kinds))])[comp]
        c = C // p
        on = cont & (C % p == 0)
        lo[:, a] = np.where(on, np.maximum(c - 1, 0), np.minimum(c, nc[a] - 1))
        hi[:, a] = np.minimum(c, nc[a] - 1)
    return lo, hi


def entity_star_patches(lat: Lattice, dim):
    """List of (entity id, dof array, ascending) of the non-empty stars of the entities
    of dimension dim (1: edges, 2: faces) without static condensation.  The cells
    containing an edge along m are its cell along m and the (up to) two cells on
    either side of each of its vertex coordinates; those containing a face normal to
    m are the (up to) two cells on either side of its vertex plane.  A free DoF belongs
    to the star when every cell holding it is among them.  Entity ids run over the
    axis (of the edge, of the face normal), then lattice order, x fastest."""
    mesh = lat.mesh
    n = (mesh.nx, mesh.ny, mesh.nz)
    lo, hi = _holding_cells(lat)
    free = ~lat.dirichlet_mask()
    out, base = [], 0
    for m in range(3):
        # entity coordinates: a cell index along the entity's own axes, a vertex index
        # along the others (edge along m: cell along m; face normal to m: vertex along m)
        cell_axes = [m] if dim == 1 else [a for a in range(3) if a != m]
        ext = [n[a] if a in cell_axes else n[a] + 1 for a in range(3)]
        for k2 in range(ext[2]):
            for k1 in range(ext[1]):
                for k0 in range(ext[0]):
                    c = (k0, k1, k2)
                    inside = free.copy()
                    for a in range(3):
                        blo, bhi = (c[a], c[a]) if a in cell_axes else (c[a] - 1, c[a])
                        inside &= (lo[:, a] >= blo) & (hi[:, a] <= bhi)
                    sel = np.where(inside)[0]
                    if sel.size:
                        out.append((base + k0 + ext[0] * (k1 + ext[1] * k2), sel))
        base += ext[0] * ext[1] * ext[2]
    return out


class PHRelaxVec:
    """z = M^{-1} r for PH without static condensation on H(curl) / H(div):
    z = sum_E R_E^T P_E^{-1} R_E r + D (sum_j R_j^T B_j^{-1} R_j) D^T r, the first sum
    over the edge (H(curl)) or face (H(div)) stars with exact Cholesky of
    P_E = R_E P R_E^T, the second over the full stars of the potential problem B
    (H(curl): Q_p with (grad phi, beta grad psi), vertex stars; H(div): NCE_p with
    (curl phi, beta curl psi) + eps (phi, beta psi), edge stars), exact, and D the
    exterior derivative between the free DoFs; Dirichlet rows copy r."""

    def __init__(self, lat: Lattice, P, beta, eps=EPS_HDIV):
        P = sp.csr_matrix(P)
        mesh, p = lat.mesh, lat.p
        self.dmask = lat.dirichlet_mask()
        dim = 1 if lat.space == "curl" else 2
        self.patches = entity_star_patches(lat, dim)
        self.factors = [np.linalg.cholesky(P[d][:, d].toarray()) for _, d in self.patches]
        be = np.broadcast_to(np.asarray(beta, dtype=np.float64), (mesh.ncells,))
        if lat.space == "curl":
            latp = Lattice(mesh, "grad", p)
            B = separable_operator(latp, cartesian_coefficient_array(latp, be, 0.0))
            self.pot_patches = full_star_patches_grad(latp)
        else:
            latp = Lattice(mesh, "curl", p)
            B = cartesian_operator(latp, be, eps * be)
            self.pot_patches = entity_star_patches(latp, 1)
        B = sp.csr_matrix(B)
        self.pot_factors = [np.linalg.cholesky(B[d][:, d].toarray()) for _, d in self.pot_patches]
        keep = sp.diags((~self.dmask).astype(np.float64))
        keepp = sp.diags((~latp.dirichlet_mask()).astype(np.float64))
        self.D = sp.csr_matrix(keep @ exterior_derivative(latp, lat) @ keepp)
        self.npot = latp.ndofs

    @staticmethod
    def _stars(patches, factors, r, n):
        z = np.zeros(n)
        for (_, d), L in zip(patches, factors):
            y = scipy.linalg.solve_triangular(L, r[d], lower=True)
            z[d] += scipy.linalg.solve_triangular(L.T, y, lower=False)
        return z

    def apply(self, r, potential=True):
        r = np.asarray(r, dtype=np.float64)
        z = self._stars(self.patches, self.factors, r, r.size)
        if potential:
            z = z + self.D @ self._stars(self.pot_patches, self.pot_factors, self.D.T @ r, self.npot)
        z[self.dmask] = r[self.dmask]
        return z
