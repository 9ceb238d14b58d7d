"""Synthetic workloads: structured hexahedral meshes of the unit cube, per-cell
coefficients and right-hand sides, all drawn from SplitMix64 streams.

Conventions (shared by every consumer):
  * vertices are numbered ``vx + (nx+1)*(vy + (ny+1)*vz)`` and stored as an
    array of shape ``(n_vertices, 3)`` (x, y, z);
  * cells are numbered ``cx + nx*(cy + ny*cz)``;
  * a right-hand side is one U[-1, 1) draw per lattice degree of freedom, in the
    order of the lattice numbering; entries on Dirichlet rows are ignored by
    both the oracle and the library (they are treated as zero).
Seeds: ``s`` for the right-hand side, ``s+1`` for alpha, ``s+2`` for beta and
``s+3`` for the vertex perturbation.
"""
import numpy as np

from .splitmix import uniform01, uniform_pm1, log_uniform


def unit_cube_vertices(nx: int, ny: int, nz: int) -> np.ndarray:
    """Vertices of the uniform nx*ny*nz hexahedral mesh of (0,1)^3."""
    x = np.linspace(0.0, 1.0, nx + 1)
    y = np.linspace(0.0, 1.0, ny + 1)
    z = np.linspace(0.0, 1.0, nz + 1)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1).copy()


def perturbed_vertices(n: int, seed: int, amplitude: float = 0.15) -> np.ndarray:
    """Uniform n^3 mesh with interior vertices moved by amplitude*h*U[-1,1) per coordinate.

    Draws 3 numbers per vertex (vertex-major, x/y/z minor) from stream ``seed``;
    the draws of boundary vertices are discarded so that the mapping from a
    vertex to its draws does not depend on which vertices are interior.
    """
    v = unit_cube_vertices(n, n, n)
    h = 1.0 / n
    d = uniform_pm1(seed, 3 * v.shape[0]).reshape(-1, 3)
    idx = np.arange(v.shape[0])
    vx = idx % (n + 1)
    vy = (idx // (n + 1)) % (n + 1)
    vz = idx // ((n + 1) * (n + 1))
    interior = (vx > 0) & (vx < n) & (vy > 0) & (vy < n) & (vz > 0) & (vz < n)
    v[interior] += amplitude * h * d[interior]
    return v


def cell_coefficients(n_cells: int, seed: int, lo: float = 1e-2, hi: float = 1e2) -> np.ndarray:
    """One log-uniform value in [lo, hi) per cell, cells in lattice order."""
    return log_uniform(seed, n_cells, lo, hi)


def c5_alpha(X: np.ndarray, amplitude: float = 0.5) -> np.ndarray:
    """The smooth coefficient exp(a sin(2 pi x) sin(2 pi y) sin(2 pi z)) at points X (n, 3)."""
    return np.exp(amplitude * np.sin(2 * np.pi * X[:, 0]) * np.sin(2 * np.pi * X[:, 1]) *
                  np.sin(2 * np.pi * X[:, 2]))


def reference_sample_points(vertices: np.ndarray, nx: int, ny: int, nz: int) -> np.ndarray:
    """Physical images (ncells, 27, 3) of the reference points {-1,0,1}^3 (x fastest)
    under each cell's trilinear map (corner k = kx + 2 ky + 4 kz)."""
    v = np.asarray(vertices, dtype=np.float64).reshape(-1, 3)
    c = np.arange(nx * ny * nz)
    cx, cy, cz = c % nx, (c // nx) % ny, c // (nx * ny)
    corners = np.zeros((c.size, 8, 3))
    for k in range(8):
        vid = (cx + (k & 1)) + (nx + 1) * ((cy + ((k >> 1) & 1)) + (ny + 1) * (cz + (k >> 2)))
        corners[:, k] = v[vid]
    t = np.array([-1.0, 0.0, 1.0])
    out = np.zeros((c.size, 27, 3))
    for m in range(27):
        xi = (t[m % 3], t[(m // 3) % 3], t[m // 9])
        for k in range(8):
            w = 1.0
            for a in range(3):
                w *= 0.5 * (1.0 + (1.0 if (k >> a) & 1 else -1.0) * xi[a])
            out[:, m] += w * corners[:, k]
    return out


def c5_coefficient_samples(vertices: np.ndarray, n: int, amplitude: float = 0.5) -> np.ndarray:
    """(n^3, 27) samples of c5_alpha at each cell's reference points."""
    X = reference_sample_points(vertices, n, n, n)
    return c5_alpha(X.reshape(-1, 3), amplitude).reshape(-1, 27)


def batch_spec(i: int):
    """Problem i of the batched workload: (space, n, p) from stream 1000 + i with
    space uniform in (grad, curl, div), n uniform in 4..16 cells per axis, p uniform
    in 3..9; its right-hand sides use seeds 4i .. 4i+3."""
    u = uniform01(1000 + i, 3)
    space = ("grad", "curl", "div")[min(2, int(3 * u[0]))]
    return space, 4 + min(12, int(13 * u[1])), 3 + min(6, int(7 * u[2]))


def rhs_values(n_dofs: int, seed: int) -> np.ndarray:
    """One U[-1,1) right-hand side of length n_dofs from stream ``seed``."""
    return uniform_pm1(seed, n_dofs)


def multi_rhs(n_dofs: int, seeds) -> np.ndarray:
    """Stack of right-hand sides, one per seed, shape (len(seeds), n_dofs)."""
    return np.stack([uniform_pm1(s, n_dofs) for s in seeds])


# The five benchmark configurations, by their sizes and seeds.
WORKLOADS = {
    "C1": dict(space="grad", n=4, p=4, coef="const", alpha=1.0, beta=1.0, seed=0,
               note="H(grad) Q_4 on 4^3, alpha=beta=1"),
    "C2": dict(space="grad", n=32, p=7, coef="cell_loguniform", seed=0,
               note="H(grad) Q_7 on 32^3, cellwise alpha,beta log-uniform in [1e-2,1e2)"),
    "C3": dict(space="curl", n=16, p=6, coef="const", alpha=1.0, beta=1.0, seed=0,
               note="H(curl) NCE_6 on 16^3, alpha=beta=1"),
    "C5": dict(space="grad", n=24, p=8, coef="func", alpha_amp=0.5, beta=1.0, seed=0,
               perturb=0.15, note="H(grad) Q_8 on perturbed 24^3, alpha(x)=exp(0.5 sin sin sin)"),
}
