"""1-D FDM element on the reference interval [-1, 1] (oracle; test infrastructure).

Follows Sec. 2.2 (eqs. fdmbasis, fdmdualbasis, unisolvence, eigs), Sec. 2.3
(DP_{p-1} basis r_j and the differentiation matrix D) and Sec. 3.2 (broken basis
of P_p with orthonormalised interface pair).

Readings (where the paper fixes nothing):
  * eigenvalues in ascending order; eigenvector sign such that s_j'(-1) > 0;
  * broken basis: s_pm = (s_0 +- s_p) / sqrt(2 (B_00 +- B_0p)), ordered so that
    broken index 0 is s_+, index p is s_-, interior indices are unchanged.
"""
import numpy as np
import scipy.linalg
from numpy.polynomial import legendre as npleg


def gll_nodes(p: int) -> np.ndarray:
    """Gauss-Lobatto-Legendre nodes: -1, the roots of P_p', +1 (ascending)."""
    if p < 1:
        raise ValueError("p >= 1")
    if p == 1:
        return np.array([-1.0, 1.0])
    c = np.zeros(p + 1)
    c[p] = 1.0
    dc = npleg.legder(c)
    r = np.sort(npleg.legroots(dc).real)
    # Newton polish on P_p'(x) = 0
    ddc = npleg.legder(dc)
    for _ in range(4):
        r = r - npleg.legval(r, dc) / npleg.legval(r, ddc)
    return np.concatenate([[-1.0], r, [1.0]])


def gauss_legendre(n: int):
    """n-point Gauss-Legendre rule on [-1, 1] (exact for degree 2n-1)."""
    x, w = npleg.leggauss(n)
    return x, w


def lagrange_eval(nodes: np.ndarray, x: np.ndarray):
    """Values V[k, i] = l_i(x_k) and derivatives dV[k, i] = l_i'(x_k) of the
    Lagrange polynomials on ``nodes`` (direct product formulas)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = nodes.size
    V = np.ones((x.size, n))
    dV = np.zeros((x.size, n))
    for i in range(n):
        others = [k for k in range(n) if k != i]
        for k in others:
            V[:, i] *= (x - nodes[k]) / (nodes[i] - nodes[k])
        for m in others:
            term = np.full(x.size, 1.0 / (nodes[i] - nodes[m]))
            for k in others:
                if k != m:
                    term *= (x - nodes[k]) / (nodes[i] - nodes[k])
            dV[:, i] += term
    return V, dV


class Element1D:
    """All 1-D tables of the FDM element of degree p.

    Attributes
      xi      GLL nodes (p+1)
      Bgll    GLL-basis mass  (l_i, l_j)          (p+1)x(p+1)
      Agll    GLL-basis stiffness (l_i', l_j')    (p+1)x(p+1)
      lam     eigenvalues lambda_1..lambda_{p-1} (ascending)
      S       tabulation S[i, j] = s_j(xi_i)      (p+1)x(p+1)
      B, A    FDM mass and stiffness  (s_i, s_j), (s_i', s_j')
      D       differentiation matrix D[i, j] = (r_i, s_j')   p x (p+1)
      G       broken-basis transformation (p+1)x(p+1): broken coeffs = G @ FDM coeffs
    """

    def __init__(self, p: int):
        self.p = p
        xi = gll_nodes(p)
        self.xi = xi
        xq, wq = gauss_legendre(p + 2)          # exact for degree 2p+3
        V, dV = lagrange_eval(xi, xq)
        self.Bgll = V.T @ (wq[:, None] * V)
        self.Agll = dV.T @ (wq[:, None] * dV)
        I = np.arange(1, p)
        Gm = np.array([0, p])
        S = np.zeros((p + 1, p + 1))
        S[0, 0] = 1.0
        S[p, p] = 1.0
        if p >= 2:
            lam, SII = scipy.linalg.eigh(self.Agll[np.ix_(I, I)], self.Bgll[np.ix_(I, I)])
            # sign rule: s_j'(-1) > 0
            _, dVm1 = lagrange_eval(xi, np.array([-1.0]))
            slope = dVm1[0, I] @ SII
            SII = SII * np.sign(slope)[None, :]
            S[np.ix_(I, I)] = SII
            S[np.ix_(I, Gm)] = -SII @ SII.T @ self.Bgll[np.ix_(I, Gm)]
            self.lam = lam
        else:
            self.lam = np.zeros(0)
        self.S = S
        self.B_raw = S.T @ self.Bgll @ S
        self.A_raw = S.T @ self.Agll @ S
        # DP_{p-1} basis and D by quadrature: r_0 = 2^{-1/2}, r_j = lam_j^{-1/2} s_j'
        dS = dV @ S                              # s_j'(xq)
        R = np.zeros((xq.size, p))
        R[:, 0] = 2.0 ** -0.5
        for j in range(1, p):
            R[:, j] = dS[:, j] / np.sqrt(self.lam[j - 1])
        self.D_raw = R.T @ (wq[:, None] * dS)
        # Tables with the entries that eqs. fdmbasis / unisolvence fix exactly:
        # (s_i, s_j) = delta_ij and (s_i', s_j') = lam_i delta_ij for interior i, j,
        # (s_i, s_0) = (s_i, s_p) = 0 (duality), r_0 = 2^{-1/2} so that row 0 of D is
        # 2^{-1/2} (s_j(1) - s_j(-1)), and (r_i, s_j') = lam_i^{1/2} delta_ij.
        B = 0.5 * (self.B_raw + self.B_raw.T)
        A = 0.5 * (self.A_raw + self.A_raw.T)
        D = self.D_raw.copy()
        if p >= 2:
            B[np.ix_(I, I)] = np.eye(p - 1)
            B[np.ix_(I, Gm)] = 0.0
            B[np.ix_(Gm, I)] = 0.0
            A[np.ix_(I, I)] = np.diag(self.lam)
            D[np.ix_(I, I)] = np.diag(np.sqrt(self.lam))
        D[0, :] = 0.0
        D[0, 0], D[0, p] = -2.0 ** -0.5, 2.0 ** -0.5
        self.B, self.A, self.D = B, A, D
        # broken basis (Sec. 3.2): orthonormalise the interface pair
        npl = np.sqrt(2.0 * (self.B[0, 0] + self.B[0, p]))
        nmi = np.sqrt(2.0 * (self.B[0, 0] - self.B[0, p]))
        G = np.eye(p + 1)
        G[0, 0] = G[0, p] = 0.5 * npl
        G[p, 0] = 0.5 * nmi
        G[p, p] = -0.5 * nmi
        self.G = G

    # --- evaluation of the bases at arbitrary points -----------------------------
    def s(self, x):
        """Values of s_0..s_p at points x: shape (len(x), p+1)."""
        V, _ = lagrange_eval(self.xi, x)
        return V @ self.S

    def ds(self, x):
        """Derivatives s_j'(x): shape (len(x), p+1)."""
        _, dV = lagrange_eval(self.xi, x)
        return dV @ self.S

    def r(self, x):
        """Values of the DP_{p-1} basis r_0..r_{p-1} at x: shape (len(x), p)."""
        x = np.atleast_1d(x)
        out = np.zeros((x.size, self.p))
        out[:, 0] = 2.0 ** -0.5
        d = self.ds(x)
        for j in range(1, self.p):
            out[:, j] = d[:, j] / np.sqrt(self.lam[j - 1])
        return out

    def dof_functionals(self, f, nq: int = 40):
        """Apply the FDM dual DoFs (eq. fdmdualbasis) to a callable f on [-1,1]:
        f(-1), (s_i, f) for interior i, f(1)."""
        xq, wq = gauss_legendre(nq)
        out = np.zeros(self.p + 1)
        out[0] = f(np.array([-1.0]))[0]
        out[self.p] = f(np.array([1.0]))[0]
        if self.p >= 2:
            sv = self.s(xq)
            fv = f(xq)
            out[1:self.p] = (wq * fv) @ sv[:, 1:self.p]
        return out

    def r_functionals(self, f, nq: int = 40):
        """L2 projection coefficients (r_j, f) of f onto DP_{p-1} (r is orthonormal)."""
        xq, wq = gauss_legendre(nq)
        return (wq * f(xq)) @ self.r(xq)


def p1_embedding(el: Element1D) -> np.ndarray:
    """(p+1)x2 matrix of the linear hats (1-x)/2, (1+x)/2 written in the FDM DoFs
    of degree p: rows 0 and p are the identity, interior rows are (s_i, hat_j)."""
    E = np.zeros((el.p + 1, 2))
    E[:, 0] = el.dof_functionals(lambda x: 0.5 * (1.0 - x))
    E[:, 1] = el.dof_functionals(lambda x: 0.5 * (1.0 + x))
    return E
