"""Mixed Hodge-Laplacian problems preconditioned by the Riesz maps (oracle; test
infrastructure).

Sec. 5.3: with no essential boundary (Gamma_D empty) find (sigma, u) in
V^{k-1} x V^k such that -(tau, sigma) + (d tau, u) = 0 for all tau and
(v, d sigma) + (d v, d u) = F(v) for all v.  In FDM coefficients the system is

    K = [ -M_{k-1}    D^T M_k ]      D   = d^{k-1} between the FDM spaces (exact:
        [  M_k D      S_k     ]            grad Q_p in NCE_p, curl NCE_p in NCF_p,
                                           div NCF_p in DQ_{p-1})
                                     M_j = mass matrix of V^j (beta = 1, alpha = 0)
                                     S_k = (d v, d u) (alpha = 1, beta = 0; 0 for k = 3)

with F(v) = (v, w) + (d v, d w) for a seeded w in V^k (eq. random_rhs), i.e. the
right-hand side [0; A_k w] with A_k the Riesz map alpha = beta = 1.

Preconditioner (the operator-preconditioning framework the section follows): the
block diagonal of the two Riesz maps alpha = beta = 1, each applied inexactly by a
fixed number of Chebyshev steps (4 in the paper) preconditioned by the p-multigrid
V-cycle of that space (SC-PAFW relaxation for Q_p, SC-PH for NCE_p / NCF_p, the
exact p = 1 coarse solve); for V^3 = DQ_{p-1}, Chebyshev steps preconditioned by
point Jacobi of the L^2 mass in the FDM basis.  Outer solver: preconditioned
MINRES (Paige & Saunders 1975) from a zero guess, stopped once the natural
P^{-1}-norm of the residual has dropped by rtol (1e-8 in the paper).

Readings of the paper (it fixes none of these):
  * Chebyshev interval [0.9 lambda_min, 1.1 lambda_max], the extreme eigenvalues of
    the Lanczos tridiagonal of 10 preconditioned CG steps on B A from the SplitMix64
    start vector of seed 99 (Ritz values lie inside the spectrum, hence the
    widening); for the L^2 block B A = I on Cartesian cells (the mass is diagonal in
    the broken FDM basis), so the interval is [0.9, 1.1].  (The interval
    [lambda_max / 10, 1.1 lambda_max] gives 19, 18 and 13 MINRES iterations for
    k = 1, 2, 3 at 3^3 cells, p = 3, against 10, 10 and 10 with this one and the
    paper's 9, 8 and 8 at 6^3);
  * each V-cycle takes its space's default damping (omega from 10 Lanczos steps of
    the relaxation, start vector seed 99);
  * the DQ_{p-1} numbering: one block of p^3 values per cell, x-local fastest,
    global index X + (n_x p) (Y + (n_y p) Z) as for the broken axes of NCE/NCF.
"""
import numpy as np
import scipy.sparse as sp

from synth.splitmix import uniform_pm1

from .tables1d import Element1D
from .lattice import Mesh, Lattice
from .assemble import ref_div, cartesian_operator, cell_sizes
from .auxop import separable_operator, cartesian_coefficient_array
from .schwarz import SCRelaxGrad
from .hiptmair import SCRelaxPH, exterior_derivative
from . import pmg

SPACES = ["grad", "curl", "div", "l2"]


# ----------------------------------------------------------------------------------
# V^3 = DQ_{p-1}
# ----------------------------------------------------------------------------------
def l2_cell_dofs(mesh: Mesh, p: int):
    """(ncells, p^3) global indices of DQ_{p-1}; local order x fastest."""
    ci = mesh.cell_index()
    Ex, Ey = mesh.nx * p, mesh.ny * p
    cols = []
    for c in range(p):
        for b in range(p):
            for a in range(p):
                cols.append((ci[:, 0] * p + a) + Ex * ((ci[:, 1] * p + b) + Ey * (ci[:, 2] * p + c)))
    return np.stack(cols, 1)


def l2_mass_diagonal(mesh: Mesh, p: int):
    """Diagonal of the DQ_{p-1} mass: the 3-form Piola map u = u_hat / det J makes it
    (8 / V) times the identity of the reference broken basis, which is L^2-orthonormal
    on [-1, 1] (Sec. 2.3, 3.1)."""
    hs = cell_sizes(mesh)
    cd = l2_cell_dofs(mesh, p)
    d = np.zeros(mesh.ncells * p ** 3)
    for k in range(mesh.ncells):
        d[cd[k]] = 8.0 / np.prod(hs[k])
    return d


def divergence(lat_div: Lattice):
    """Sparse (ndofs(DQ_{p-1}) x ndofs(NCF_p)) matrix of div in FDM coefficients: the
    reference divergence of each cell (every DQ value belongs to one cell)."""
    mesh, p = lat_div.mesh, lat_div.p
    R = ref_div(Element1D(p))
    cdf, cdq = lat_div.cell_dofs(), l2_cell_dofs(mesh, p)
    r_, c_ = np.nonzero(R)
    rows = np.concatenate([cdq[k, r_] for k in range(mesh.ncells)])
    cols = np.concatenate([cdf[k, c_] for k in range(mesh.ncells)])
    vals = np.tile(R[r_, c_], mesh.ncells)
    return sp.csr_matrix((vals, (rows, cols)), shape=(mesh.ncells * p ** 3, lat_div.ndofs))


# ----------------------------------------------------------------------------------
# the block system
# ----------------------------------------------------------------------------------
class HodgeSystem:
    """Blocks of the mixed Hodge Laplacian for k in {1, 2, 3} on a Cartesian mesh with
    no essential boundary."""

    def __init__(self, mesh: Mesh, k: int, p: int):
        assert k in (1, 2, 3) and mesh.dirichlet == 0
        self.mesh, self.k, self.p = mesh, k, p
        lo, hi = SPACES[k - 1], SPACES[k]
        self.lat_lo = Lattice(mesh, lo, p)
        self.M_lo = cartesian_operator(self.lat_lo, 0.0, 1.0)
        if k < 3:
            self.lat_hi = Lattice(mesh, hi, p)
            self.n_hi = self.lat_hi.ndofs
            self.M_hi = cartesian_operator(self.lat_hi, 0.0, 1.0)
            self.S_hi = cartesian_operator(self.lat_hi, 1.0, 0.0)
            self.D = exterior_derivative(self.lat_lo, self.lat_hi)
        else:
            self.lat_hi = None
            self.n_hi = mesh.ncells * p ** 3
            self.M_hi = sp.diags(l2_mass_diagonal(mesh, p))
            self.S_hi = sp.csr_matrix((self.n_hi, self.n_hi))
            self.D = divergence(self.lat_lo)
        self.n_lo = self.lat_lo.ndofs
        B = (self.M_hi @ self.D).tocsr()
        self.K = sp.bmat([[-self.M_lo, B.T], [B, self.S_hi]]).tocsr()
        # Riesz maps alpha = beta = 1 of the two spaces
        self.A_lo = cartesian_operator(self.lat_lo, 1.0, 1.0)
        self.A_hi = (self.M_hi + self.S_hi).tocsr()

    def rhs(self, seed=7):
        """[0; A_k w] with w seeded uniform in [-1, 1) (eq. random_rhs)."""
        w = uniform_pm1(seed, self.n_hi)
        return np.concatenate([np.zeros(self.n_lo), self.A_hi @ w])


# ----------------------------------------------------------------------------------
# Chebyshev and MINRES
# ----------------------------------------------------------------------------------
def chebyshev(A, Binv, lmin, lmax, steps):
    """Callable f -> x: ``steps`` Chebyshev iterations on A x = f from x = 0,
    preconditioned by Binv, for the spectrum of Binv A in [lmin, lmax] (the
    three-term recurrence of the Chebyshev semi-iterative method; Saad, Iterative
    Methods for Sparse Linear Systems, Sec. 12.3).  The result is q(Binv A) Binv f
    with x* - x = p(Binv A) x*, p the scaled Chebyshev polynomial of degree steps."""
    theta, delta = 0.5 * (lmax + lmin), 0.5 * (lmax - lmin)
    sigma = theta / delta

    def apply(f):
        rho = 1.0 / sigma
        x = np.zeros_like(f)
        r = f.copy()
        d = Binv(r) / theta
        for j in range(steps):
            x = x + d
            if j + 1 == steps:
                break
            r = r - A @ d
            rho_next = 1.0 / (2.0 * sigma - rho)
            d = (rho_next * rho) * d + (2.0 * rho_next / delta) * Binv(r)
            rho = rho_next
        return x

    return apply


def minres(K, b, Pinv, rtol=1e-8, maxit=500):
    """Preconditioned MINRES (Paige & Saunders) on the symmetric K from x = 0 with the
    SPD preconditioner Pinv.  The Lanczos process in the P-inner product builds
    v_j (unnormalised, (v_j, Pinv v_j) = gamma_j^2) and z_j = Pinv v_j / gamma_j;
    Givens rotations (c, s) reduce the tridiagonal to upper triangular form, the
    search directions w_j follow from the three-term recurrence, and |eta| is the
    P^{-1}-norm of the current residual.  Returns (x, iterations, [|eta_0|, ...])."""
    n = b.size
    x = np.zeros(n)
    v_prev, v = np.zeros(n), b.copy()
    z = Pinv(v)
    gamma = np.sqrt(v @ z)
    gamma_prev = 1.0
    eta = gamma
    c_prev = c = 1.0
    s_prev = s = 0.0
    w_prev, w = np.zeros(n), np.zeros(n)
    hist = [abs(eta)]
    it = 0
    while it < maxit and abs(eta) > rtol * hist[0]:
        it += 1
        z = z / gamma
        Kz = K @ z
        delta = Kz @ z
        v_next = Kz - (delta / gamma) * v - (gamma / gamma_prev) * v_prev
        z_next = Pinv(v_next)
        gamma_next = np.sqrt(v_next @ z_next)
        a0 = c * delta - c_prev * s * gamma
        a1 = np.hypot(a0, gamma_next)
        a2 = s * delta + c_prev * c * gamma
        a3 = s_prev * gamma
        c_prev, c = c, a0 / a1
        s_prev, s = s, gamma_next / a1
        w_next = (z - a3 * w_prev - a2 * w) / a1
        x = x + (c * eta) * w_next
        eta = -s * eta
        v_prev, v = v, v_next
        w_prev, w = w, w_next
        gamma_prev, gamma = gamma, gamma_next
        z = z_next
        hist.append(abs(eta))
    return x, it, hist


# ----------------------------------------------------------------------------------
# the block preconditioner
# ----------------------------------------------------------------------------------
def riesz_vcycle(lat: Lattice, A, lanczos_seed=99):
    """p-MG V(1,1) cycle of the Riesz map alpha = beta = 1 on lat (no Dirichlet rows),
    damping from the relaxation's Lanczos estimate."""
    mesh = lat.mesh
    latc = Lattice(mesh, lat.space, 1)
    if lat.space == "grad":
        R = SCRelaxGrad(lat, separable_operator(lat, cartesian_coefficient_array(lat, 1.0, 1.0)))
    else:
        R = SCRelaxPH(lat, A, 1.0)
    v0 = uniform_pm1(lanczos_seed, lat.ndofs)
    om = pmg.omega_from_lambda(pmg.lanczos_lambda_max(A, R.apply, v0))
    cs = pmg.CoarseSolver(latc, cartesian_operator(latc, 1.0, 1.0))
    return pmg.VCycle(lat, A, R, pmg.prolongation(lat, latc), cs, om)


def lanczos_extremes(A, Binv, v0, steps=10):
    """(smallest, largest) eigenvalue of the Lanczos tridiagonal built from ``steps``
    preconditioned CG iterations on A x = v0 (coefficients a_j, b_j: diagonal
    1/a_j + b_{j-1}/a_{j-1}, off-diagonal sqrt(b_j)/a_j)."""
    r = v0.copy()
    z = Binv(r)
    d = z.copy()
    rz = r @ z
    diag, off = [], []
    a_prev = b_prev = None
    for _ in range(steps):
        Ad = A @ d
        a = rz / (d @ Ad)
        r = r - a * Ad
        z = Binv(r)
        rz_new = r @ z
        b = rz_new / rz
        diag.append(1.0 / a + (b_prev / a_prev if a_prev is not None else 0.0))
        off.append(np.sqrt(b) / a)
        a_prev, b_prev, rz = a, b, rz_new
        d = z + b * d
    T = np.diag(diag) + np.diag(off[:-1], 1) + np.diag(off[:-1], -1)
    ev = np.linalg.eigvalsh(T)
    return float(ev[0]), float(ev[-1])


class HodgePreconditioner:
    """blockdiag(Cheb_m(A_{k-1}, V_{k-1}), Cheb_m(A_k, V_k or Jacobi))."""

    def __init__(self, sysm: HodgeSystem, steps=4, lanczos_seed=99):
        self.sysm, self.steps = sysm, steps
        self.V_lo = riesz_vcycle(sysm.lat_lo, sysm.A_lo, lanczos_seed)
        self.eig_lo = lanczos_extremes(sysm.A_lo, self.V_lo, uniform_pm1(lanczos_seed, sysm.n_lo))
        self.C_lo = chebyshev(sysm.A_lo, self.V_lo, 0.9 * self.eig_lo[0], 1.1 * self.eig_lo[1], steps)
        if sysm.k < 3:
            self.V_hi = riesz_vcycle(sysm.lat_hi, sysm.A_hi, lanczos_seed)
            self.eig_hi = lanczos_extremes(sysm.A_hi, self.V_hi, uniform_pm1(lanczos_seed, sysm.n_hi))
        else:
            dinv = 1.0 / sysm.M_hi.diagonal()
            self.V_hi = lambda r: dinv * r
            self.eig_hi = (1.0, 1.0)
        self.C_hi = chebyshev(sysm.A_hi, self.V_hi, 0.9 * self.eig_hi[0], 1.1 * self.eig_hi[1], steps)

    def __call__(self, r):
        n = self.sysm.n_lo
        return np.concatenate([self.C_lo(r[:n]), self.C_hi(r[n:])])


def hodge_solve(mesh: Mesh, k: int, p: int, steps=4, rtol=1e-8, seed=7, maxit=500):
    """MINRES on the Hodge Laplacian with the Riesz-map block preconditioner."""
    sysm = HodgeSystem(mesh, k, p)
    P = HodgePreconditioner(sysm, steps)
    b = sysm.rhs(seed)
    x, it, hist = minres(sysm.K, b, P, rtol, maxit)
    return sysm, P, b, x, it, hist
