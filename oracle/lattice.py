"""Degree-of-freedom numbering on structured hexahedral meshes (oracle; test
infrastructure).

Spaces (Sec. 2.4): Q_p = P x P x P, NCE_p component m is DP along axis m and P
along the others, NCF_p component m is P along axis m and DP along the others.
On a structured mesh whose cells all share one orientation, each global space is
a tensor product of 1-D continuous (P, extent n*p+1) and broken (DP, extent n*p)
spaces, so degrees of freedom sit on a lattice:

  * a P-direction coordinate X = c*p + a, a in 0..p  (a=0 and a=p are shared
    with the neighbouring cell);
  * a DP-direction coordinate X = c*p + a, a in 0..p-1;
  * global index  offset_m + X + E_x*(Y + E_y*Z)  (x fastest), components of
    NCE/NCF stored one after the other (x, y, z).

Dirichlet rows (Sec. 2.1, traces): a degree of freedom is constrained iff along
some P-direction axis its coordinate is 0 (or the last) and that face belongs to
Gamma_D.  Face bits: 1=x0, 2=x1, 4=y0, 8=y1, 16=z0, 32=z1.
"""
import numpy as np

SPACES = ("grad", "curl", "div")


class Mesh:
    """Structured nx*ny*nz hexahedral mesh with arbitrary vertex positions."""

    def __init__(self, nx, ny, nz, vertices=None, dirichlet=0x3F):
        self.nx, self.ny, self.nz = nx, ny, nz
        if vertices is None:
            x = np.linspace(0, 1, nx + 1)
            y = np.linspace(0, 1, ny + 1)
            z = np.linspace(0, 1, nz + 1)
            Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
            vertices = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
        self.vertices = np.asarray(vertices, dtype=np.float64).reshape(-1, 3)
        assert self.vertices.shape[0] == (nx + 1) * (ny + 1) * (nz + 1)
        self.dirichlet = dirichlet
        self.n = (nx, ny, nz)

    @property
    def ncells(self):
        return self.nx * self.ny * self.nz

    def cell_index(self):
        """(ncells, 3) integer cell coordinates, cells in lattice order."""
        c = np.arange(self.ncells)
        return np.stack([c % self.nx, (c // self.nx) % self.ny, c // (self.nx * self.ny)], 1)

    def cell_vertices(self):
        """(ncells, 8, 3) corner coordinates; corner k = kx + 2 ky + 4 kz."""
        ci = self.cell_index()
        out = np.zeros((self.ncells, 8, 3))
        for k in range(8):
            kx, ky, kz = k & 1, (k >> 1) & 1, (k >> 2) & 1
            vid = (ci[:, 0] + kx) + (self.nx + 1) * ((ci[:, 1] + ky) + (self.ny + 1) * (ci[:, 2] + kz))
            out[:, k] = self.vertices[vid]
        return out

    def is_cartesian(self, tol=1e-14):
        """True if every cell is an axis-aligned box."""
        cv = self.cell_vertices()
        for k in range(8):
            for a in range(3):
                bit = (k >> a) & 1
                ref = cv[:, bit << a, a]
                if np.abs(cv[:, k, a] - ref).max() > tol:
                    return False
        return True


def component_kinds(space, p):
    """For each component, the per-axis kind: 'P' (continuous) or 'D' (broken)."""
    if space == "grad":
        return [("P", "P", "P")]
    if space == "curl":
        return [tuple("D" if a == m else "P" for a in range(3)) for m in range(3)]
    if space == "div":
        return [tuple("P" if a == m else "D" for a in range(3)) for m in range(3)]
    raise ValueError(space)


class Lattice:
    """Numbering of one space on one mesh."""

    def __init__(self, mesh: Mesh, space: str, p: int):
        self.mesh, self.space, self.p = mesh, space, p
        self.kinds = component_kinds(space, p)
        self.extents = []
        self.offsets = []
        off = 0
        for kind in self.kinds:
            ext = tuple(mesh.n[a] * p + (1 if kind[a] == "P" else 0) for a in range(3))
            self.extents.append(ext)
            self.offsets.append(off)
            off += ext[0] * ext[1] * ext[2]
        self.ndofs = off

    def local_shape(self, m):
        """Per-cell (x, y, z) extents of component m."""
        return tuple(self.p + 1 if k == "P" else self.p for k in self.kinds[m])

    def ncell_dofs(self):
        return sum(int(np.prod(self.local_shape(m))) for m in range(len(self.kinds)))

    def cell_dofs(self):
        """(ncells, ncell_dofs) global indices; local order = component-major, then
        x-local fastest, then y, then z."""
        ci = self.mesh.cell_index()
        cols = []
        p = self.p
        for m in range(len(self.kinds)):
            lx, ly, lz = self.local_shape(m)
            Ex, Ey, _ = self.extents[m]
            for c in range(lz):
                for b in range(ly):
                    for a in range(lx):
                        X = ci[:, 0] * p + a
                        Y = ci[:, 1] * p + b
                        Z = ci[:, 2] * p + c
                        cols.append(self.offsets[m] + X + Ex * (Y + Ey * Z))
        return np.stack(cols, 1)

    def coords(self):
        """(ndofs, 4) array (component, X, Y, Z) for every global index."""
        out = np.zeros((self.ndofs, 4), dtype=np.int64)
        for m in range(len(self.kinds)):
            Ex, Ey, Ez = self.extents[m]
            g = np.arange(Ex * Ey * Ez)
            sl = slice(self.offsets[m], self.offsets[m] + g.size)
            out[sl, 0] = m
            out[sl, 1] = g % Ex
            out[sl, 2] = (g // Ex) % Ey
            out[sl, 3] = g // (Ex * Ey)
        return out

    def dirichlet_mask(self):
        """Boolean (ndofs,) mask of constrained rows."""
        co = self.coords()
        mask = np.zeros(self.ndofs, dtype=bool)
        bits = self.mesh.dirichlet
        for m in range(len(self.kinds)):
            sel = co[:, 0] == m
            for a in range(3):
                if self.kinds[m][a] != "P":
                    continue
                E = self.extents[m][a]
                if bits & (1 << (2 * a)):
                    mask[sel & (co[:, 1 + a] == 0)] = True
                if bits & (1 << (2 * a + 1)):
                    mask[sel & (co[:, 1 + a] == E - 1)] = True
        return mask
