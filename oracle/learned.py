"""Learned separable auxiliary coefficients (oracle; test infrastructure).

The method's own auxiliary operator (eq. sum-factorization_approx) keeps, per
cell, the diagonals of the beta-mass in the broken H(grad) basis and of the
alpha-weighted mass of the gradient components in the broken NCE basis.  The
separable surrogate replaces them by one weight per gradient component and one
for the mass: c = (sigma_1..3, mu, mu, mu).  Its least-squares fit to the
diagonals is their mean (readings: a constant fitted to a vector in the 2-norm is
its mean; the mass weight is shared by the three axes).

Because the broken bases are tensor products, the mean over a tensor basis of
the squared functions factors per axis into Christoffel functions
kappa_P(t) = mean_k sbar_k(t)^2 (degree-p broken basis) and
kappa_D(t) = mean_k r_k(t)^2 (degree-(p-1) L2 basis), so
  mu      = sum_q w det(J) beta kappa_P(x) kappa_P(y) kappa_P(z),
  sigma_m = sum_q w det(J) alpha (J^-1 J^-T)_mm kappa_D(xi_m) prod_{a != m} kappa_P(xi_a).

A small MLP predicts log(c / c_avg) (c_avg: the cell-averaged weights) from
dimensionless per-cell features: the 24 corner offsets from the cell's centroid
divided by its mean edge length, minus those of a cube, and the 27 log-alpha
samples minus their mean.  Network: 51 -> H (tanh) -> H (tanh) -> 6, loss = mean
over samples and outputs of the squared error; Adam.
"""
import numpy as np

from .tables1d import Element1D
from .assemble import trilinear_jacobian
from .quadrature import rule, sampled_values, default_points
from .auxop import _diag_mass


def christoffel(el: Element1D, x):
    """kappa_P(x) and kappa_D(x) at points x."""
    sb = el.s(x) @ np.linalg.inv(el.G)       # broken P basis values (n, p+1)
    r = el.r(x)                              # DP basis values (n, p)
    return (sb ** 2).mean(1), (r ** 2).mean(1)


def diagonal_targets(mesh, alpha_samples, beta_samples, p, q=None):
    """(ncells, 6) least-squares separable fit to the broken diagonals, factorised form."""
    el = Element1D(p)
    q = q or default_points(p)
    xq, wq = rule(q, "gll")
    kP, kD = christoffel(el, xq)
    W = np.einsum("z,y,x->zyx", wq, wq, wq).ravel()
    KP = np.einsum("z,y,x->zyx", kP, kP, kP).ravel()
    KD = [np.einsum("z,y,x->zyx", kP, kP, kD).ravel(), np.einsum("z,y,x->zyx", kP, kD, kP).ravel(),
          np.einsum("z,y,x->zyx", kD, kP, kP).ravel()]
    a = sampled_values(alpha_samples, xq)
    b = sampled_values(beta_samples, xq)
    cv = mesh.cell_vertices()
    out = np.zeros((mesh.ncells, 6))
    for k in range(mesh.ncells):
        _, J = trilinear_jacobian(cv[k], xq)
        det = np.linalg.det(J)
        Ji = np.linalg.inv(J)
        G = np.einsum("qsr,qsr->qs", Ji, Ji)
        for m in range(3):
            out[k, m] = np.sum(W * det * a[k] * G[:, m] * KD[m])
        out[k, 3:] = np.sum(W * det * b[k] * KP)
    return out


def diagonal_targets_direct(mesh, alpha_samples, beta_samples, p, q=None):
    """Same fit computed from the full broken diagonals (no factorisation)."""
    el = Element1D(p)
    q = q or default_points(p)
    xq, wq = rule(q, "gll")
    W = np.einsum("z,y,x->zyx", wq, wq, wq).ravel()
    a = sampled_values(alpha_samples, xq)
    b = sampled_values(beta_samples, xq)
    cv = mesh.cell_vertices()
    sh = (q, q, q)
    kinds_e = [("D", "P", "P"), ("P", "D", "P"), ("P", "P", "D")]
    out = np.zeros((mesh.ncells, 6))
    for k in range(mesh.ncells):
        _, J = trilinear_jacobian(cv[k], xq)
        det = np.linalg.det(J)
        Ji = np.linalg.inv(J)
        G = np.einsum("qsr,qsr->qs", Ji, Ji)
        dm = _diag_mass(el, ("P", "P", "P"), (W * det * b[k]).reshape(sh), xq)
        for m in range(3):
            out[k, m] = _diag_mass(el, kinds_e[m], (W * det * a[k] * G[:, m]).reshape(sh), xq).mean()
        out[k, 3:] = dm.mean()
    return out


def features(mesh, alpha_samples):
    """(ncells, 51) dimensionless per-cell features."""
    cv = mesh.cell_vertices()                                  # (nc, 8, 3)
    cen = cv.mean(1, keepdims=True)
    # mean edge length over the 12 edges
    edges = [(0, 1), (2, 3), (4, 5), (6, 7), (0, 2), (1, 3), (4, 6), (5, 7), (0, 4), (1, 5), (2, 6), (3, 7)]
    h = np.mean([np.linalg.norm(cv[:, j] - cv[:, i], axis=1) for i, j in edges], axis=0)
    ref = np.array([[(-0.5 if not (k >> a) & 1 else 0.5) for a in range(3)] for k in range(8)])
    geo = ((cv - cen) / h[:, None, None] - ref[None]).reshape(-1, 24)
    la = np.log(np.asarray(alpha_samples, dtype=np.float64))
    la = la - la.mean(1, keepdims=True)
    return np.concatenate([geo, la], 1)


# ---------------------------------------------------------------------------------
# the network (plain NumPy, FP64 or FP32)
# ---------------------------------------------------------------------------------
def init_params(nin, nhid, nout, seed):
    """Glorot-uniform weights from SplitMix64 stream `seed` (W1, W2, W3 drawn in this
    order, row-major, out x in), zero biases."""
    from synth import uniform_pm1
    sizes = [(nhid, nin), (nhid, nhid), (nout, nhid)]
    u = uniform_pm1(seed, sum(a * b for a, b in sizes))
    params, o = [], 0
    for (fo, fi) in sizes:
        lim = np.sqrt(6.0 / (fi + fo))
        params.append(lim * u[o:o + fo * fi].reshape(fo, fi))
        params.append(np.zeros(fo))
        o += fo * fi
    return params


def forward(params, X):
    W1, b1, W2, b2, W3, b3 = params
    z1 = X @ W1.T + b1
    a1 = np.tanh(z1)
    z2 = a1 @ W2.T + b2
    a2 = np.tanh(z2)
    y = a2 @ W3.T + b3
    return y, (X, a1, a2)


def loss_and_grads(params, X, Y):
    """Mean squared error over all outputs and its gradient (hand-written backward)."""
    W1, b1, W2, b2, W3, b3 = params
    y, (X, a1, a2) = forward(params, X)
    n = X.shape[0] * Y.shape[1]
    d = y - Y
    loss = np.sum(d * d) / n
    gy = 2.0 * d / n
    gW3 = gy.T @ a2
    gb3 = gy.sum(0)
    g2 = (gy @ W3) * (1.0 - a2 * a2)
    gW2 = g2.T @ a1
    gb2 = g2.sum(0)
    g1 = (g2 @ W2) * (1.0 - a1 * a1)
    gW1 = g1.T @ X
    gb1 = g1.sum(0)
    return loss, [gW1, gb1, gW2, gb2, gW3, gb3]


def adam_step(params, grads, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t counts from 1), in place."""
    for k in range(len(params)):
        m[k] = b1 * m[k] + (1 - b1) * grads[k]
        v[k] = b2 * v[k] + (1 - b2) * grads[k] * grads[k]
        mh = m[k] / (1 - b1 ** t)
        vh = v[k] / (1 - b2 ** t)
        params[k] = params[k] - lr * mh / (np.sqrt(vh) + eps)
    return params
