"""p-multigrid V(1,1) cycle and preconditioned CG (oracle; test infrastructure).

Sec. 4.3 (eq. asm-afw: coarse space V_{h,1}, A_0 the form rediscretised at p=1,
R_0 the restriction), Sec. 5 (hybrid multigrid/Schwarz: additive within a level,
multiplicative across levels in a V(1,1) cycle; CG from a zero guess).

Readings of the paper (it fixes none of these):
  * prolongation: the natural embedding V_{h,1} in V_{h,p} written in FDM DoFs
    (per P-axis the (p+1)x2 matrix of the linear hats; per DP-axis r_0 -> r_0);
    restriction is its transpose;
  * smoothing: one damped step z += omega M^{-1} (r - A z) before and after the
    coarse correction, omega = 2 / (0.1 lam + 1.1 lam) with lam an estimate of
    the largest eigenvalue of M^{-1} A (first-degree Chebyshev on [0.1, 1.1] lam);
  * stop when the 2-norm of the residual drops by the relative tolerance (1e-8),
    the true residual b - A x being checked at exit;
  * Dirichlet rows act as the identity.
"""
import numpy as np
import scipy.linalg
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .tables1d import Element1D, p1_embedding
from .lattice import Lattice


def prolongation(lat_f: Lattice, lat_c: Lattice):
    """Sparse (ndofs_f x ndofs_c) embedding of the p=1 space in the degree-p space;
    rows and columns of Dirichlet DoFs are zero."""
    assert lat_c.p == 1 and lat_f.space == lat_c.space
    el = Element1D(lat_f.p)
    E = p1_embedding(el)
    ED = np.zeros((lat_f.p, 1))
    ED[0, 0] = 1.0
    cdf = lat_f.cell_dofs()
    cdc = lat_c.cell_dofs()
    owner = -np.ones(lat_f.ndofs, dtype=np.int64)
    for k in range(cdf.shape[0]):
        new = owner[cdf[k]] < 0
        owner[cdf[k][new]] = k
    rows, cols, vals = [], [], []
    nloc_f = [int(np.prod(lat_f.local_shape(m))) for m in range(len(lat_f.kinds))]
    nloc_c = [int(np.prod(lat_c.local_shape(m))) for m in range(len(lat_c.kinds))]
    of = np.cumsum([0] + nloc_f)
    oc = np.cumsum([0] + nloc_c)
    for m, kind in enumerate(lat_f.kinds):
        mats = [E if k == "P" else ED for k in kind]
        Pm = np.kron(mats[2], np.kron(mats[1], mats[0]))       # local fine x local coarse
        r_, c_ = np.nonzero(np.abs(Pm) > 0)
        for k in range(cdf.shape[0]):
            gf = cdf[k, of[m] + r_]
            sel = owner[gf] == k
            rows.append(gf[sel])
            cols.append(cdc[k, oc[m] + c_[sel]])
            vals.append(Pm[r_[sel], c_[sel]])
    Pr = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                       shape=(lat_f.ndofs, lat_c.ndofs))
    kf = sp.diags((~lat_f.dirichlet_mask()).astype(np.float64))
    kc = sp.diags((~lat_c.dirichlet_mask()).astype(np.float64))
    return sp.csr_matrix(kf @ Pr @ kc)


class CoarseSolver:
    """A_0^{-1} on the free coarse DoFs by Cholesky (dense or sparse LU)."""

    def __init__(self, lat_c: Lattice, A0):
        self.free = np.where(~lat_c.dirichlet_mask())[0]
        A0f = sp.csr_matrix(A0)[self.free][:, self.free]
        self.n = lat_c.ndofs
        if self.free.size <= 4000:
            self.chol = scipy.linalg.cho_factor(A0f.toarray(), lower=True)
            self.lu = None
        else:
            self.chol = None
            self.lu = spla.splu(sp.csc_matrix(A0f))

    def solve(self, r):
        out = np.zeros(self.n)
        rf = r[self.free]
        out[self.free] = scipy.linalg.cho_solve(self.chol, rf) if self.chol is not None else self.lu.solve(rf)
        return out


JACOBI_C = 1.5


def jacobi_weight(M):
    """Damping of point Jacobi on the SPD matrix M: JACOBI_C over the largest row sum
    of |D^{-1/2} M D^{-1/2}| (Gershgorin), an upper bound of the spectrum of D^{-1} M,
    so that the weighted spectrum stays in (0, JACOBI_C] and the relaxation contracts
    on any mesh (anisotropic cells included) and for any positive coefficients."""
    M = sp.csr_matrix(M)
    d = M.diagonal()
    S = sp.diags(1.0 / np.sqrt(d)) @ abs(M) @ sp.diags(1.0 / np.sqrt(d))
    return JACOBI_C / np.asarray(S.sum(axis=1)).max()


def interp_1d(nf, lo_f, hi_f, lo_c, hi_c):
    """Linear interpolation on one axis from the coarse vertices c (at fine vertex 2c)
    to the fine vertices f: 1 where f = 2c, 1/2 where |f - 2c| = 1; rows the free
    fine range lo_f..hi_f, columns the free coarse range lo_c..hi_c."""
    rows, cols, vals = [], [], []
    for f in range(lo_f, hi_f + 1):
        for c in range(lo_c, hi_c + 1):
            d = abs(f - 2 * c)
            if d <= 1:
                rows.append(f - lo_f)
                cols.append(c - lo_c)
                vals.append(1.0 if d == 0 else 0.5)
    return sp.csr_matrix((vals, (rows, cols)), shape=(hi_f - lo_f + 1, hi_c - lo_c + 1))


class HMGCoarse:
    """Geometric h-multigrid on the p = 1 space as the coarse solver (the h-hierarchy
    below p = 1 of Sec. 5.1): the free Q_1 DoFs form a box; while every cell count is
    even and the level holds more than min_free DoFs, the next level is the mesh with
    half the cells per axis, with trilinear interpolation P (the Kronecker product of
    the 1-D linear interpolations on the free coordinates) and the Galerkin operator
    P^T A P; the coarsest level is solved exactly.  solve(r) is one V(1,1) cycle from a
    zero guess with damped point Jacobi (the level's jacobi_weight) before and after the
    coarse correction (a symmetric positive definite approximation of A_0^{-1})."""

    def __init__(self, lat_c: Lattice, A0, min_free=1000):
        mesh = lat_c.mesh
        mask = lat_c.dirichlet_mask()
        self.free = np.where(~mask)[0]
        self.n = lat_c.ndofs
        n = [mesh.nx, mesh.ny, mesh.nz]
        d = mesh.dirichlet
        lo = [1 if d & (1 << (2 * a)) else 0 for a in range(3)]
        hi = [n[a] - 1 if d & (1 << (2 * a + 1)) else n[a] for a in range(3)]
        A = sp.csr_matrix(A0)[self.free][:, self.free]
        self.A, self.P, self.dinv = [A], [], [1.0 / A.diagonal()]
        while all(k % 2 == 0 for k in n) and A.shape[0] > min_free:
            nc = [k // 2 for k in n]
            loc = [1 if d & (1 << (2 * a)) else 0 for a in range(3)]
            hic = [nc[a] - 1 if d & (1 << (2 * a + 1)) else nc[a] for a in range(3)]
            Ps = [interp_1d(n[a] + 1, lo[a], hi[a], loc[a], hic[a]) for a in range(3)]
            P = sp.csr_matrix(sp.kron(Ps[2], sp.kron(Ps[1], Ps[0])))
            A = sp.csr_matrix(P.T @ A @ P)
            self.P.append(P)
            self.A.append(A)
            self.dinv.append(1.0 / A.diagonal())
            n, lo, hi = nc, loc, hic
        self.w = [jacobi_weight(M) for M in self.A]
        self.chol = scipy.linalg.cho_factor(self.A[-1].toarray(), lower=True)

    def cycle(self, level, b):
        if level == len(self.A) - 1:
            return scipy.linalg.cho_solve(self.chol, b)
        A, w, dinv = self.A[level], self.w[level], self.dinv[level]
        x = w * dinv * b
        xc = self.cycle(level + 1, self.P[level].T @ (b - A @ x))
        x = x + self.P[level] @ xc
        return x + w * dinv * (b - A @ x)

    def solve(self, r):
        out = np.zeros(self.n)
        out[self.free] = self.cycle(0, r[self.free])
        return out


def halve_1d(nf, nc, continuous):
    """One axis of the interpolation between nested lowest-order spaces on meshes of
    nf = 2 nc and nc cells (all vertices or cells, before Dirichlet rows are taken
    out).  Continuous axis: the hats, linear interpolation (interp_1d).  Broken axis:
    a coarse cell's constant r_0 is, in the reference coefficients of the Piola-mapped
    fine functions, one half of r_0 on each of its two halves (the Piola factor of
    that axis scales with the cell size)."""
    if continuous:
        return interp_1d(nf + 1, 0, nf, 0, nc)
    return sp.csr_matrix((np.full(nf, 0.5), (np.arange(nf), np.arange(nf) // 2)), shape=(nf, nc))


class HiptmairHMG:
    """Geometric h-multigrid on the lowest-order space NCE_1 (H(curl)) or NCF_1
    (H(div)) as the p-coarse solver, with Hiptmair-Jacobi relaxation (the h-hierarchy
    of Sec. 5.1 in the solver diagram of Fig. hcurl_solver_diagram).

    Levels: the mesh with half the cells per axis while every count is even and the
    level holds more than min_free free DoFs; P the per-component Kronecker product
    of halve_1d on the free DoFs, A_{l+1} = P^T A_l P.  Potential space of each level:
    Q_1 (H(curl)) or NCE_1 (H(div)) on that level's mesh with the same Dirichlet faces,
    G the exterior derivative between the two lowest-order spaces on the free DoFs
    (exterior_derivative), its operator G^T A_l G.  Relaxation: damped Jacobi on A_l
    and damped Jacobi on G^T A_l G (each with its jacobi_weight), pre-smoothing in that
    order and post-smoothing in the reverse order, so one V(1,1) cycle from a zero
    guess is symmetric; the coarsest level is solved exactly."""

    def __init__(self, lat_c: Lattice, A0, min_free=512):
        from .lattice import Mesh
        from .hiptmair import exterior_derivative
        space = lat_c.space
        pot = {"curl": "grad", "div": "curl"}[space]
        mesh = lat_c.mesh
        d = mesh.dirichlet
        n = [mesh.nx, mesh.ny, mesh.nz]
        lat = lat_c
        self.free = np.where(~lat.dirichlet_mask())[0]
        self.n = lat.ndofs
        A = sp.csr_matrix(A0)[self.free][:, self.free]
        self.A, self.P, self.G, self.dinv, self.dpinv, self.w, self.wp = [], [], [], [], [], [], []

        def add_level(lat, A):
            f = np.where(~lat.dirichlet_mask())[0]
            latp = Lattice(lat.mesh, pot, 1)
            fp = np.where(~latp.dirichlet_mask())[0]
            G = sp.csr_matrix(exterior_derivative(latp, lat))[f][:, fp]
            Ap = sp.csr_matrix(G.T @ A @ G)
            self.A.append(A)
            self.G.append(G)
            self.dinv.append(1.0 / A.diagonal())
            self.dpinv.append(1.0 / Ap.diagonal())
            self.w.append(jacobi_weight(A))
            self.wp.append(jacobi_weight(Ap))
            return f

        f = add_level(lat, A)
        while all(k % 2 == 0 for k in n) and A.shape[0] > min_free:
            nc = [k // 2 for k in n]
            latn = Lattice(Mesh(*nc, dirichlet=d), space, 1)
            blocks = []
            for m, kind in enumerate(lat.kinds):
                Ps = [halve_1d(n[a], nc[a], kind[a] == "P") for a in range(3)]
                blocks.append(sp.kron(Ps[2], sp.kron(Ps[1], Ps[0])))
            fn = np.where(~latn.dirichlet_mask())[0]
            P = sp.csr_matrix(sp.block_diag(blocks, format="csr")[f][:, fn])
            A = sp.csr_matrix(P.T @ A @ P)
            self.P.append(P)
            lat, n = latn, nc
            f = add_level(lat, A)
        self.chol = scipy.linalg.cho_factor(self.A[-1].toarray(), lower=True)

    def _space_jacobi(self, l, b, x):
        return x + self.w[l] * self.dinv[l] * (b - self.A[l] @ x)

    def _pot_jacobi(self, l, b, x, wp=None):
        G = self.G[l]
        wp = self.wp[l] if wp is None else wp
        return x + G @ (wp * self.dpinv[l] * (G.T @ (b - self.A[l] @ x)))

    def cycle(self, level, b):
        if level == len(self.A) - 1:
            return scipy.linalg.cho_solve(self.chol, b)
        x = self._space_jacobi(level, b, np.zeros_like(b))
        x = self._pot_jacobi(level, b, x)
        x = x + self.P[level] @ self.cycle(level + 1, self.P[level].T @ (b - self.A[level] @ x))
        x = self._pot_jacobi(level, b, x)
        return self._space_jacobi(level, b, x)

    def solve(self, r):
        out = np.zeros(self.n)
        out[self.free] = self.cycle(0, r[self.free])
        return out


class VCycle:
    """Hybrid V(1,1): z = w M r; z += P A0^{-1} P^T (r - A z); z += w M (r - A z)."""

    def __init__(self, lat: Lattice, A, relax, Pr, coarse, omega):
        self.A = sp.csr_matrix(A)
        self.relax = relax
        self.Pr = Pr
        self.coarse = coarse
        self.omega = omega
        self.dmask = lat.dirichlet_mask()

    def __call__(self, r):
        r = np.where(self.dmask, 0.0, r)
        w = self.omega
        z = w * np.where(self.dmask, 0.0, self.relax.apply(r))
        r1 = r - self.A @ z
        r1[self.dmask] = 0.0
        z = z + self.Pr @ self.coarse.solve(self.Pr.T @ r1)
        r2 = r - self.A @ z
        r2[self.dmask] = 0.0
        z = z + w * np.where(self.dmask, 0.0, self.relax.apply(r2))
        return z


def lanczos_lambda_max(A, Minv, v0, steps=10):
    """Largest eigenvalue of M^{-1} A estimated from ``steps`` preconditioned CG
    iterations on A x = v0 (Lanczos tridiagonal from the CG coefficients)."""
    x = np.zeros_like(v0)
    r = v0.copy()
    z = Minv(r)
    p = z.copy()
    rz = r @ z
    alphas, betas = [], []
    for _ in range(steps):
        Ap = A @ p
        a = rz / (p @ Ap)
        x += a * p
        r -= a * Ap
        z = Minv(r)
        rz_new = r @ z
        b = rz_new / rz
        alphas.append(a)
        betas.append(b)
        rz = rz_new
        p = z + b * p
    k = len(alphas)
    T = np.zeros((k, k))
    for j in range(k):
        T[j, j] = 1.0 / alphas[j] + (betas[j - 1] / alphas[j - 1] if j > 0 else 0.0)
        if j + 1 < k:
            T[j, j + 1] = T[j + 1, j] = np.sqrt(betas[j]) / alphas[j]
    return float(np.linalg.eigvalsh(T).max())


def omega_from_lambda(lam):
    return 2.0 / (0.1 * lam + 1.1 * lam)


def pcg(A, b, M, rtol=1e-8, maxit=500, norm="l2"):
    """Preconditioned CG from x0 = 0.  Returns x, iterations, residual 2-norm history.

    norm="l2": stop when the 2-norm of the residual has dropped by rtol (the true
    residual is checked at exit); norm="natural": stop when the natural norm
    (r^T M^{-1} r)^{1/2} has dropped by rtol, the criterion of the paper's
    experiments (Sec. 5.1).  CG needs a positive definite preconditioner: a negative
    r^T M^{-1} r is a breakdown, reported as iterations = -1."""
    if norm == "natural":
        return _pcg_natural(A, b, M, rtol, maxit)
    A = sp.csr_matrix(A)
    x = np.zeros_like(b)
    r = b.copy()
    nb = np.linalg.norm(b)
    hist = [np.linalg.norm(r)]
    if nb == 0:
        return x, 0, hist
    z = M(r)
    p = z.copy()
    rz = r @ z
    it = 0
    while it < maxit:
        Ap = A @ p
        a = rz / (p @ Ap)
        x += a * p
        r -= a * Ap
        it += 1
        hist.append(np.linalg.norm(r))
        if hist[-1] <= rtol * nb:
            rtrue = b - A @ x
            if np.linalg.norm(rtrue) <= rtol * nb:
                break
            r = rtrue
        z = M(r)
        rz_new = r @ z
        if rz_new < 0:          # breakdown: M is not positive definite
            return x, -1, hist
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, it, hist


def _pcg_natural(A, b, M, rtol, maxit):
    A = sp.csr_matrix(A)
    x = np.zeros_like(b)
    r = b.copy()
    hist = [np.linalg.norm(r)]
    z = M(r)
    rz = r @ z
    if rz < 0:
        return x, -1, hist
    if not rz > 0:
        return x, 0, hist
    tol = rtol * np.sqrt(rz)
    p = z.copy()
    it = 0
    while it < maxit:
        Ap = A @ p
        a = rz / (p @ Ap)
        x += a * p
        r -= a * Ap
        it += 1
        hist.append(np.linalg.norm(r))
        z = M(r)
        rz_new = r @ z
        if rz_new < 0:          # breakdown: M is not positive definite
            return x, -1, hist
        if np.sqrt(rz_new) <= tol:
            break
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, it, hist
