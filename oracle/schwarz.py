"""Statically condensed additive Schwarz relaxation (oracle; test infrastructure).

H(grad) (k = 0): SC-PAFW of Sec. 4.4, eqs. LDU, schur and sc-asm-afw, with the
vertex-star interface patch matrices S_v = R_v S R_v^T factored by incomplete
Cholesky restricted to the symbolic static-condensation pattern (Sec. 4.5).

Readings of the paper (it fixes none of these):
  * symbolic pattern: the structural pattern of S computed from the Cartesian
    Kronecker structure of the auxiliary operator -- 1-D mass pattern = diagonal
    plus (0,p); 1-D stiffness pattern = diagonal plus full rows/columns 0 and p;
    cell pattern = union of (stiffness along one axis, mass along the others) and
    mass^3; S pattern = pattern(P_GG) union the cliques of the interface
    neighbours of every interior DoF.  Never thresholded.
  * order inside a vertex patch: the 12 faces (normal axis x, y, z; then the
    side -/+ along the lower remaining axis, then along the higher one; lattice
    order inside a face), then the 6 edges (axis x, y, z; side -/+ along the edge
    axis; lattice order), then the vertex.  Dirichlet DoFs removed; empty patches
    dropped; patches in lattice vertex order.
  * incomplete Cholesky is unmodified: fill outside the pattern is discarded; a
    pivot <= 0 is a breakdown.
  * Dirichlet rows: z_D = r_D.
"""
import numpy as np
import scipy.linalg
import scipy.sparse as sp

from .lattice import Lattice


class ICBreakdown(RuntimeError):
    pass


# ----------------------------------------------------------------------------------
# interior / interface split
# ----------------------------------------------------------------------------------
def interior_mask(lat: Lattice):
    """DoFs in the interior of a cell: every P-direction coordinate is not a
    multiple of p."""
    co = lat.coords()
    p = lat.p
    mask = np.ones(lat.ndofs, dtype=bool)
    for m, kind in enumerate(lat.kinds):
        sel = co[:, 0] == m
        for a in range(3):
            if kind[a] == "P":
                mask[sel & (co[:, 1 + a] % p == 0)] = False
    return mask


# ----------------------------------------------------------------------------------
# symbolic static-condensation pattern (H(grad))
# ----------------------------------------------------------------------------------
def _pat_mass(p):
    P = np.eye(p + 1, dtype=bool)
    P[0, p] = P[p, 0] = True
    return P


def _pat_stiff(p):
    P = np.eye(p + 1, dtype=bool)
    P[0, :] = P[p, :] = P[:, 0] = P[:, p] = True
    return P


def _bkron3(a, b, c):
    return np.kron(c, np.kron(b, a)).astype(bool)


def symbolic_schur_pattern_grad(lat: Lattice):
    """Boolean sparse pattern of the global interface Schur complement (all DoFs
    indexed; only interface rows/columns are populated)."""
    p = lat.p
    Bm, As = _pat_mass(p), _pat_stiff(p)
    Pc = _bkron3(As, Bm, Bm) | _bkron3(Bm, As, Bm) | _bkron3(Bm, Bm, As) | _bkron3(Bm, Bm, Bm)
    n1 = p + 1
    loc = np.arange(n1 ** 3)
    i, j, l = loc % n1, (loc // n1) % n1, loc // (n1 * n1)
    inter = (i % p != 0) & (j % p != 0) & (l % p != 0)
    Gi, Ii = np.where(~inter)[0], np.where(inter)[0]
    SK = np.zeros((n1 ** 3, n1 ** 3), dtype=bool)
    SK[np.ix_(Gi, Gi)] = Pc[np.ix_(Gi, Gi)]
    PGI = Pc[np.ix_(Gi, Ii)].astype(np.int64)
    SK[np.ix_(Gi, Gi)] |= (PGI @ PGI.T) > 0
    cd = lat.cell_dofs()
    r, c = np.nonzero(SK)
    rows = cd[:, r].ravel()
    cols = cd[:, c].ravel()
    M = sp.coo_matrix((np.ones(rows.size, dtype=np.int8), (rows, cols)), shape=(lat.ndofs, lat.ndofs))
    M = sp.csr_matrix(M)
    M.data[:] = 1
    return M


# ----------------------------------------------------------------------------------
# vertex-star interface patches (H(grad))
# ----------------------------------------------------------------------------------
def vertex_patches_grad(lat: Lattice):
    """List of (vertex_id, dof array) for every non-empty vertex-star interface
    patch, in lattice vertex order, DoFs in the patch order documented above."""
    mesh, p = lat.mesh, lat.p
    co = lat.coords()
    free = ~lat.dirichlet_mask()
    X, Y, Z = co[:, 1], co[:, 2], co[:, 3]
    out = []
    nvx, nvy, nvz = mesh.nx + 1, mesh.ny + 1, mesh.nz + 1
    for vz in range(nvz):
        for vy in range(nvy):
            for vx in range(nvx):
                Xv, Yv, Zv = vx * p, vy * p, vz * p
                dX, dY, dZ = X - Xv, Y - Yv, Z - Zv
                inbox = (np.abs(dX) < p) & (np.abs(dY) < p) & (np.abs(dZ) < p)
                onplane = (dX == 0) | (dY == 0) | (dZ == 0)
                sel = np.where(inbox & onplane & free)[0]
                if sel.size == 0:
                    continue
                d = np.stack([dX[sel], dY[sel], dZ[sel]], 1)
                keys = [_patch_key(d[k], sel[k]) for k in range(sel.size)]
                order = sorted(range(sel.size), key=lambda k: keys[k])
                out.append((vx + nvx * (vy + nvy * vz), sel[order]))
    return out


def _patch_key(d, g):
    zero = [a for a in range(3) if d[a] == 0]
    side = lambda a: 0 if d[a] < 0 else 1
    if len(zero) == 1:                       # face with normal axis zero[0]
        a = zero[0]
        rest = [b for b in range(3) if b != a]
        return (0, a, side(rest[0]), side(rest[1]), g)
    if len(zero) == 2:                       # edge along the non-zero axis
        a = [b for b in range(3) if d[b] != 0][0]
        return (1, a, side(a), 0, g)
    return (2, 0, 0, 0, g)                   # the vertex


# ----------------------------------------------------------------------------------
# incomplete Cholesky on a given pattern
# ----------------------------------------------------------------------------------
def ic_on_pattern(S, pattern):
    """Lower factor L (dense array) with L L^T ~ S, L restricted to the lower
    triangle of ``pattern`` (boolean, symmetric).  Row-oriented: for each row i,
    entries j < i in ascending order, then the pivot."""
    n = S.shape[0]
    L = np.zeros((n, n))
    low = np.tril(pattern, -1)
    for i in range(n):
        cols = np.nonzero(low[i])[0]
        for j in cols:
            s = S[i, j] - np.dot(L[i, :j], L[j, :j])
            L[i, j] = s / L[j, j]
        d = S[i, i] - np.dot(L[i, :i], L[i, :i])
        if not d > 0.0:
            raise ICBreakdown(f"pivot {d} at row {i}")
        L[i, i] = np.sqrt(d)
    return L


# ----------------------------------------------------------------------------------
# the relaxation
# ----------------------------------------------------------------------------------
class SCRelaxGrad:
    """z = M^{-1} r for SC-PAFW (H(grad)) on the auxiliary operator P.

    Steps (eq. schur with S^{-1} replaced by the additive vertex-patch sum):
      z_I  = P_II^{-1} r_I
      rt   = r_G - P_GI z_I
      z_G  = sum_v R_v^T (L_v L_v^T)^{-1} R_v rt
      z_I -= P_II^{-1} P_IG z_G
    """

    def __init__(self, lat: Lattice, P, factor="ic"):
        self.lat = lat
        P = sp.csr_matrix(P)
        mask = lat.dirichlet_mask()
        self.dmask = mask
        inter = interior_mask(lat) & ~mask
        iface = ~interior_mask(lat) & ~mask
        self.I = np.where(inter)[0]
        self.G = np.where(iface)[0]
        PII = P[self.I][:, self.I]
        off = PII - sp.diags(PII.diagonal())
        if off.count_nonzero() and np.abs(off.data).max() > 0:
            raise ValueError("P_II is not diagonal")
        self.dII = PII.diagonal()
        self.PIG = P[self.I][:, self.G]
        self.PGI = P[self.G][:, self.I]
        PGG = P[self.G][:, self.G]
        S = PGG - self.PGI @ sp.diags(1.0 / self.dII) @ self.PIG
        self.S = sp.csr_matrix(S)
        pos = -np.ones(lat.ndofs, dtype=np.int64)
        pos[self.G] = np.arange(self.G.size)
        self.pos = pos
        self.patches = vertex_patches_grad(lat)
        pat = symbolic_schur_pattern_grad(lat)
        self.factors = []
        self.patterns = []
        for vid, dofs in self.patches:
            loc = pos[dofs]
            Sv = self.S[loc][:, loc].toarray()
            pv = pat[dofs][:, dofs].toarray().astype(bool)
            if factor == "ic":
                L = ic_on_pattern(Sv, pv)
            else:
                L = np.linalg.cholesky(Sv)
            self.factors.append(L)
            self.patterns.append(pv)

    def patch_sum(self, rt):
        """sum_v R_v^T (L_v L_v^T)^{-1} R_v rt for a vector rt on the interface set G."""
        zG = np.zeros(self.G.size)
        for (vid, dofs), L in zip(self.patches, self.factors):
            loc = self.pos[dofs]
            y = scipy.linalg.solve_triangular(L, rt[loc], lower=True)
            zG[loc] += scipy.linalg.solve_triangular(L.T, y, lower=False)
        return zG

    def apply(self, r):
        r = np.asarray(r, dtype=np.float64)
        z = np.zeros_like(r)
        zI = r[self.I] / self.dII
        rt = r[self.G] - self.PGI @ zI
        zG = self.patch_sum(rt)
        zI = zI - (self.PIG @ zG) / self.dII
        z[self.I] = zI
        z[self.G] = zG
        z[self.dmask] = r[self.dmask]
        return z



def full_star_patches_grad(lat: Lattice):
    """List of (vertex_id, dof array) of the vertex stars without static
    condensation (Sec. 4.3, eq. pafw): every free DoF strictly inside the cells around
    the vertex (|X - vx p| < p on every axis), ordered lexicographically by its offset
    from the vertex with x fastest (a reading: the paper does not fix an order; it
    matters for the incomplete factorisation only)."""
    mesh, p = lat.mesh, lat.p
    co = lat.coords()
    free = ~lat.dirichlet_mask()
    X, Y, Z = co[:, 1], co[:, 2], co[:, 3]
    out = []
    nvx, nvy, nvz = mesh.nx + 1, mesh.ny + 1, mesh.nz + 1
    for vz in range(nvz):
        for vy in range(nvy):
            for vx in range(nvx):
                dX, dY, dZ = X - vx * p, Y - vy * p, Z - vz * p
                sel = np.where((np.abs(dX) < p) & (np.abs(dY) < p) & (np.abs(dZ) < p) & free)[0]
                if sel.size == 0:
                    continue
                order = np.lexsort((dX[sel], dY[sel], dZ[sel]))
                out.append((vx + nvx * (vy + nvy * vz), sel[order]))
    return out


class PAFWRelaxGrad:
    """z = M^{-1} r for PAFW without static condensation (H(grad); Sec. 4.3 eq. pafw,
    the additive fine part of eq. asm-afw): z = sum_v R_v^T P_v^{-1} R_v r over the full
    vertex stars, P_v = R_v P R_v^T, factored exactly (factor="chol") or by incomplete
    Cholesky on the pattern of P_v (factor="ic"); Dirichlet rows copy r."""

    def __init__(self, lat: Lattice, P, factor="chol"):
        self.lat = lat
        P = sp.csr_matrix(P)
        self.dmask = lat.dirichlet_mask()
        self.patches = full_star_patches_grad(lat)
        self.factors = []
        for vid, dofs in self.patches:
            Pv = P[dofs][:, dofs].toarray()
            if factor == "ic":
                self.factors.append(ic_on_pattern(Pv, Pv != 0))
            else:
                self.factors.append(np.linalg.cholesky(Pv))

    def apply(self, r):
        r = np.asarray(r, dtype=np.float64)
        z = np.zeros_like(r)
        for (vid, dofs), L in zip(self.patches, self.factors):
            y = scipy.linalg.solve_triangular(L, r[dofs], lower=True)
            z[dofs] += scipy.linalg.solve_triangular(L.T, y, lower=False)
        z[self.dmask] = r[self.dmask]
        return z
